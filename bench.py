#!/usr/bin/env python
"""Throughput benchmark of the diffuse-scattering hot path on one MI355X.

Workload (displacive disorder): fcc-type basis with 4 sites per cell and
scattering lengths {1.0, 0.7, 0.7, 0.7}, a 32^3 supercell (131072 atoms),
Gaussian displacements of sigma = 0.05 a smoothed by a periodic Gaussian of
width 1.5 cells, Taylor order 8, every supercell Bragg point G with
|h|,|k|,|l| <= 8 (513^3 voxels).  Synthetic, seeded inputs.

One step is one pass of the whole hot path over the resident inputs:
  set_sites (device copy) -> float64 lattice sums -> field generation + 3D FFTs
  -> recombination on the box grown by the Lanczos window -> float64 Bragg
  points -> Lanczos filter (m = 2) into the 513^3 output.
value = output voxels x configurations per second.

Besides the JSON line fields of the contract it reports:
  roofline      the dominant kernel (recombination) measured with HIP events on
                its own stream over the timed region, against its algorithmic
                flops and bytes per launch;
  cpu_baseline  the FP64 oracle (direct sum, OpenMP) on a bounded seeded voxel
                sample of the same workload, scaled to voxels/s;
  parity        relative L2 of the GPU I(G) against the oracle on that sample.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "diffuse-intensity voxels/s at ≤1e-5 rel L2 vs FP64; p50/p99 request latency"
PROFILES = os.path.join(ROOT, "profiles")
# rocprofv3 summaries per workload: (title, kernel-name fragment of the dominant kernel)
WORKLOADS = {
    "displacive32_order8": ("displacive 32^3 fcc, Taylor order 8, 513^3 box, Lanczos m = 2 (the filtered step)",
                            "k_recombine"),
    "magnetic24": ("magnetic pyrochlore 24^3, 16 sites, 289^3 box (set_sites_async + compute_intensity)",
                   "k_recombine_magnetic"),
    "ensemble8x8": ("batched ensemble, 8 models x 8 configurations, one graph replay per step", "k_recombine"),
    "ensemble8x8_merged": ("batched ensemble, 8 models x 8 configurations, merged graph forced, one replay per step",
                           "k_recombine"),
    "compositional1024": ("1024 compositional models (12^3, 48^3 voxels each) in one batch, one graph replay "
                          "per step", "k_recombine"),
}
BATCH_MODES = {"auto": 0, "per_model": 1, "merged": 2}


def ktrace_md(name):
    return os.path.join(PROFILES, f"kernels_{name}.md")


def traffic_md(name):
    return os.path.join(PROFILES, f"traffic_{name}.md")
COPY_PROBE_BYTES = 256 << 20     # plain device copy of known size, read + write


def kernel_source_hash():
    """Hash of the kernel sources: stored traces and traffic are only used while it matches."""
    h = hashlib.sha256()
    for src in ("recombine.hip", "recombine_o0.hip", "recombine_o5.hip", "recombine_o7.hip", "recombine_o9.hip",
                "fft.hip", "lanczos.hip"):
        with open(os.path.join(ROOT, "paper_1809_07088_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _after_probe(rows):
    """The dispatches issued after the copy probe's fill kernel: the timed steps and
    their warmup, not the plan tuning that comes before the probe."""
    marks = [int(r["Dispatch_Id"]) for r in rows if "FillFunctor" in r["Kernel_Name"]]
    first = max(marks) if marks else -1
    return [r for r in rows if int(r["Dispatch_Id"]) > first]


def summarize_pmc(fetch_dir, write_dir, name, command):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) into the
    traffic summary of a workload: per kernel, the HBM bytes per launch, each counter
    scaled by the ratio of the known size of the plain copy probe to what the same
    counter reads for it; the dominant kernel's record is kept as JSON for the bench."""
    title, dominant = WORKLOADS[name]

    def per_kernel(d, counter):
        vals = {}
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
            for r in _after_probe(rows):
                vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return vals
    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")

    def probe(vals):
        cands = [max(v) for k, v in vals.items() if "copyBuffer" in k]
        return max(cands) if cands else None
    pf, pw = probe(fetch), probe(write)
    if not pf or not pw:
        raise SystemExit("summarize: copy probe missing in the counter files")
    sf, sw = COPY_PROBE_BYTES / pf, COPY_PROBE_BYTES / pw
    kernels = [k for k in fetch if "dsx::" in k and k in write]
    kernels.sort(key=lambda k: -sum(fetch[k]) / len(fetch[k]) - sum(write[k]) / len(write[k]))
    dom = [k for k in kernels if dominant in k]
    if not dom:
        raise SystemExit("summarize: dominant kernel missing in the counter files")
    dk = max(dom, key=lambda k: len(fetch[k]))
    f_avg = sum(fetch[dk]) / len(fetch[dk]) * sf
    w_avg = sum(write[dk]) / len(write[dk]) * sw
    rec = {"kernel": dominant, "kernel_name": dk, "source_hash": kernel_source_hash(),
           "fetch_bytes": f_avg, "write_bytes": w_avg, "traffic_bytes": f_avg + w_avg,
           "copy_probe_bytes": COPY_PROBE_BYTES, "fetch_scale": sf, "write_scale": sw}
    with open(traffic_md(name), "w") as f:
        f.write("# HBM traffic per kernel launch, %s\n\n" % title)
        f.write("Two rocprofv3 PMC runs of the benchmark (`FETCH_SIZE`, then `WRITE_SIZE`, KiB per "
                "dispatch), each scaled by copy-probe bytes / counter reading of the plain device "
                "copy of %d MiB issued by the benchmark after its warm-up (fetch scale %.4f, write scale %.4f).  "
                "Only the dispatches after the probe count.  Kernel sources: %s.\n\n"
                % (COPY_PROBE_BYTES >> 20, sf, sw, kernel_source_hash()))
        f.write("Command (run from /tmp with TMPDIR=/tmp, R = repository root):\n\n```\n%s\n```\n\n" % command)
        f.write("| kernel | launches | FETCH raw (MB) | WRITE raw (MB) | fetch scaled (MB) | write scaled (MB) |\n"
                "|---|---|---|---|---|---|\n")
        for k in kernels:
            fr, wr = sum(fetch[k]) / len(fetch[k]), sum(write[k]) / len(write[k])
            f.write("| `%s` | %d | %.2f | %.2f | %.2f | %.2f |\n" % (
                k, len(fetch[k]), fr / 1e6, wr / 1e6, fr * sf / 1e6, wr * sw / 1e6))
        f.write("\nDominant kernel record:\n\n```json\n%s\n```\n" % json.dumps(rec))
    return rec


def summarize_ktrace(trace_dir, name, command):
    """Kernel-time summary of a workload from a rocprofv3 --kernel-trace folder: per
    kernel, calls and average / min / max duration of the dispatches after the copy probe
    (the timed steps and their warm-up; the dominant kernel's average is compared with
    the benchmark's HIP-event launch time)."""
    title, _ = WORKLOADS[name]
    paths = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not paths:
        raise SystemExit("summarize: no kernel_trace.csv under " + trace_dir)
    rows = [r for r in _after_probe(list(csv.DictReader(open(paths[0])))) if "dsx::" in r["Kernel_Name"]]
    per = {}
    for r in rows:
        per.setdefault(r["Kernel_Name"], []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    total = sum(sum(v) for v in per.values())
    order = sorted(per, key=lambda k: -sum(per[k]))
    with open(ktrace_md(name), "w") as f:
        f.write("# Kernel time, %s\n\n" % title)
        f.write("rocprofv3 kernel trace of the benchmark: the library's dispatches after the plain device "
                "copy issued after the warm-up (the same probe the PMC runs use).  MI355X, one GPU.\n\n"
                "Command (run from /tmp with TMPDIR=/tmp, R = repository root):\n\n```\n%s\n```\n\n" % command)
        f.write("Kernel sources: %s.\n\n" % kernel_source_hash())
        f.write("| kernel | calls | average (us) | min (us) | max (us) | share of GPU time |\n"
                "|---|---|---|---|---|---|\n")
        for k in order:
            v = per[k]
            f.write("| `%s` | %d | %.1f | %.1f | %.1f | %.2f %% |\n" % (
                k, len(v), sum(v) / len(v) / 1e3, min(v) / 1e3, max(v) / 1e3, 100.0 * sum(v) / total))
    return len(order)


def stored_trace_avg(name, kernel_substr):
    """Average launch time (s) of a kernel in the committed kernel-trace summary of a
    workload, while the kernel sources it was taken with are unchanged."""
    try:
        txt = open(ktrace_md(name)).read()
    except OSError:
        return None
    if ("Kernel sources: %s." % kernel_source_hash()) not in txt:
        return None
    for line in txt.splitlines():
        if line.startswith("| `") and kernel_substr in line:
            return float(line.split("|")[3]) * 1e-6
    return None


def stored_traffic(name):
    """The dominant kernel's HBM bytes per launch from the committed traffic summary of a
    workload, while the kernel sources are unchanged."""
    try:
        txt = open(traffic_md(name)).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", txt, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    return rec if rec.get("source_hash") == kernel_source_hash() else None


HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PUBLISHED_TFLOPS = 157.3  # MI355X published FP32 vector peak: counts packed FP32 (two per lane)
# The reachable FP32 vector peak of this build, which compiles without packed FP32:
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.
FP32_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def roofline(flops, bytes_, t_launch, kernel, trace_avg_s=None):
    """The roofline object of one kernel: the binding roof is whichever of the reachable
    FP32 vector rate and HBM takes longer for the algorithmic flops and bytes; achieved
    = algorithmic work per launch / the launch's HIP-event time (and, when given, the
    rocprofv3 trace's average launch time)."""
    tflops, gbs = flops / t_launch / 1e12, bytes_ / t_launch / 1e9
    alu = flops / (FP32_VALU_TFLOPS * 1e12) > bytes_ / (HBM_PEAK_GBS * 1e9)
    if alu:
        roof = {"bound": "alu", "achieved": round(tflops, 3), "peak": round(FP32_VALU_TFLOPS, 1),
                "unit": "TFLOP/s", "frac": round(tflops / FP32_VALU_TFLOPS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4)}
    roof["traffic"] = None
    roof.update({"kernel": kernel, "launch_ms": round(t_launch * 1e3, 4),
                 "algorithmic_flops_per_launch": int(flops), "algorithmic_bytes_per_launch": int(bytes_),
                 "achieved_TFLOPs": round(tflops, 3), "achieved_hbm_GBs": round(gbs, 1),
                 "frac_fp32_valu": round(tflops / FP32_VALU_TFLOPS, 4),
                 "frac_fp32_published": round(tflops / FP32_PUBLISHED_TFLOPS, 4),
                 "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)})
    if trace_avg_s:
        rate = (flops / trace_avg_s / 1e12 / FP32_VALU_TFLOPS) if alu else (bytes_ / trace_avg_s / 1e9 / HBM_PEAK_GBS)
        roof["trace_launch_ms"] = round(trace_avg_s * 1e3, 4)
        roof["frac_from_trace"] = round(rate, 4)
    return roof


def c15_report(G, gpu, ref, n):
    """Error of the GPU result against the FP64 oracle at the points G: relative L2,
    max |dI| / max |I_ref|, relative L2 per |g| shell (g = G/n, reciprocal-lattice
    units, shells 2 wide) and the worst voxel."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    d = gpu - ref
    gn = np.linalg.norm(np.asarray(G, np.float64) / np.asarray(n, np.float64), axis=1)
    shells = {}
    for lo in range(0, int(np.ceil(gn.max())) + 2, 2):
        sel = (gn >= lo) & (gn < lo + 2)
        if sel.any() and np.linalg.norm(ref[sel]) > 0:
            shells[f"{lo}-{lo + 2}"] = float(np.linalg.norm(d[sel]) / np.linalg.norm(ref[sel]))
    w = int(np.argmax(np.abs(d)))
    return {"rel_l2": float(np.linalg.norm(d) / np.linalg.norm(ref)),
            "max_abs_err_over_max_ref": float(np.max(np.abs(d)) / np.max(np.abs(ref))),
            "rel_l2_by_g_shell": shells,
            "worst_voxel": {"G": [int(v) for v in G[w]], "gpu": float(gpu[w]), "oracle": float(ref[w])},
            "voxels": int(len(G))}


def oracle_filtered_points(O, model, Q, m, order):
    """The oracle's filtered intensity at integer output points Q: I(G) by direct sum
    on each point's (2m)^3 window, then the oracle's windowed sum."""
    Q = np.asarray(Q, np.int64)
    off = np.stack(np.meshgrid(*[np.arange(2 * m)] * 3, indexing="ij"), -1).reshape(-1, 3)
    e0 = Q - m + 1
    allG = (e0[:, None, :] + off[None]).reshape(-1, 3)
    Gu, inv = np.unique(allG, axis=0, return_inverse=True)
    win = O.intensity(model, Gu.astype(np.int32), order)[inv.ravel()].reshape(len(Q), 2 * m, 2 * m, 2 * m)
    return np.array([O.lanczos_points(win[i], e0[i].astype(np.int32), m, Q[i:i + 1].astype(np.float64))[0]
                     for i in range(len(Q))])


def hcount(k, n, g0, cnt):
    """Number of H with g0 <= k + n H < g0 + cnt."""
    lo = -((k - g0) // n)
    hi = (g0 + cnt - 1 - k) // n
    return max(0, hi - lo + 1)


def recombine_work(n, S, nclass3, N, M, g0, cnt, nh, F, friedel=False):
    """Algorithmic flops and bytes of one recombination launch over the box (g0, cnt).

    flops: the sum-factorised evaluation --
      level C  per voxel and r3 class: Horner (4N) + class phase (8); |F|^2 (4)
      level B  per (G1, G2, k3) and site: 4 QR (q sums) + 10 (N+1) + 6
      level A  per (G1, k2) column, site and k3: 10 flops per Taylor term
    bytes: float32 output written once + every half spectrum read once.
    On a box symmetric about G = 0 only half of the voxels are evaluated (the
    other half is I(-G) = I(G)), so the flops are halved."""
    QR = (N + 1) * (N + 2) // 2
    T = (N + 1) * (N + 2) * (N + 3) // 6
    V = int(np.prod(cnt))
    rows12 = cnt[0] * cnt[1]
    items = sum(1 for k3 in range(n[2]) if hcount(k3, n[2], g0[2], cnt[2]) > 0) * rows12
    cols = cnt[0] * sum(1 for k2 in range(n[1]) if hcount(k2, n[1], g0[1], cnt[1]) > 0)
    fl_c = V * (nclass3 * (4 * N + 8) + 4)
    fl_b = items * S * (4 * QR + 10 * (N + 1) + 6)
    fl_a = cols * S * n[2] * 10 * T
    flops = M * (fl_a + fl_b + fl_c) * (0.5 if friedel else 1.0)
    bytes_ = 4 * V + M * n[0] * n[1] * S * F * nh * 8
    return flops, bytes_


def copy_probe(torch, dev):
    """One plain device copy of known size: the reference the PMC byte counters are
    scaled by, and the mark after which profiled dispatches count."""
    src = torch.empty(COPY_PROBE_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def magnetic_work(n, S, nclass3, M, g0, cnt, nh, friedel):
    """Algorithmic flops and bytes of one magnetic recombination launch (spin spectra, one
    form factor for every site):
      level C  per voxel and r3 class: 3 complex multiply-adds (24); per voxel Q, its
               direction, the perpendicular projection, |F_perp|^2 and f(|Q|)^2 (40)
      level B  per (G1, G2, k3) and site: phase product (6) + 3 complex multiply-adds (24)
      level A  per (G1, k2) column, site, component and k3: b e^{2 pi i g1 r1} times X (6)
    bytes: float32 output written once + every half spin spectrum read once; halved
    flops on a box symmetric about G = 0."""
    V = int(np.prod(cnt))
    items = sum(1 for k3 in range(n[2]) if hcount(k3, n[2], g0[2], cnt[2]) > 0) * cnt[0] * cnt[1]
    cols = cnt[0] * sum(1 for k2 in range(n[1]) if hcount(k2, n[1], g0[1], cnt[1]) > 0)
    flops = M * (V * (24 * nclass3 + 40) + items * S * 30 + cols * S * 3 * n[2] * 6) * (0.5 if friedel else 1.0)
    bytes_ = 4 * V + M * n[0] * n[1] * S * 3 * nh * 8
    return flops, bytes_


def bench_magnetic(dsx, torch, dev, steps, warmup, O=None, probe=False):
    """The magnetic workload: pyrochlore, 16 sites, 24^3 supercell, unit spins with a
    nearest-neighbour correlated component, magnetic form factor, perpendicular
    projection, |h|,|k|,|l| <= 6 (289^3 voxels).  One step = set_sites_async (device copy)
    + compute_intensity; the recombination is timed with HIP events on its stream."""
    import synth
    m = synth.magnetic(n=24, M=1, hmax=6)
    count = tuple(m.count)
    spin = torch.from_numpy(m.spin[0]).to(dev)
    h = dsx.Model(cell=m.cell, n=m.n, frac=m.frac, b=m.b, kind=dsx.MAGNETIC, ff=m.ff, n_configs=1)
    h.set_grid(m.g0, count)
    h.set_sites_async(0, None, None, spin)
    h.autotune(0)
    out = torch.empty(count, dtype=torch.float32, device=dev)

    def step():
        h.set_sites_async(0, None, None, spin)
        h.compute_intensity(out)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if probe:
        copy_probe(torch, dev)
    dsx.profile_reset()
    dsx.profile_select("recombine")
    dsx.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    dsx.profile_enable(False)
    ks = dsx.profile_read()
    dsx.profile_reset()
    dsx.profile_select(None)
    launches, tot = ks.get("recombine", (0, float("nan")))
    t_launch = tot / max(launches, 1) / 1e3
    nclass3 = len(np.unique(m.frac[:, 2]))
    flops, bytes_ = magnetic_work(m.n, m.n_sites, nclass3, 1, m.g0, count, m.n[2] // 2 + 1, friedel=True)
    vox = int(np.prod(count))
    res = {"workload": "magnetic pyrochlore 16 sites/cell, 24^3 supercell, unit spins (nearest-neighbour "
                       "correlated), form factor (0.4,20,0.5,7,0.1,2,0), |h|,|k|,|l|<=6 (289^3 voxels)",
           "voxels_per_step": vox, "ms_per_step": round(sec * 1e3, 4), "voxels_per_s": round(vox / sec, 1),
           "roofline": roofline(flops, bytes_, t_launch, "recombine_magnetic",
                                stored_trace_avg("magnetic24", "k_recombine_magnetic"))}
    tr = stored_traffic("magnetic24")
    if tr is not None:
        res["roofline"]["traffic"] = int(tr["traffic_bytes"])
    if O is not None:
        rng = np.random.default_rng([3, 0, 777])
        G = np.stack([rng.integers(m.g0[a], m.g0[a] + count[a], 512) for a in range(3)], -1)
        H = np.stack(np.meshgrid(*[np.arange(-6, 7, 3)] * 3, indexing="ij"), -1).reshape(-1, 3) * 24
        G = np.concatenate([G, H]).astype(np.int32)
        t = torch.as_tensor(G - np.asarray(m.g0), device=dev)
        g = out[t[:, 0], t[:, 1], t[:, 2]].cpu().numpy()
        res["parity"] = c15_report(G, g, O.intensity(m, G), m.n)
    h.close()
    return res


def bench_compositional(dsx, torch, dev, steps, O=None, seeds=1024, probe=False, batch_mode="auto"):
    """The compositional workload: simple cubic, one site, 12^3 supercell, Bernoulli(0.5)
    occupancies, 48^3 voxels (|h|,|k|,|l| < 2).  Single-instance latency of one
    synchronous set_sites_async + compute_intensity, and throughput over `seeds`
    configurations: (a) one model holding them as its ensemble (one FFT batch, one
    recombination over configurations), (b) `seeds` independent models in one batch."""
    import synth
    base = synth.compositional(n=12, M=1, hmax=2)
    count = tuple(base.count)
    vox = int(np.prod(count))
    occs = [torch.from_numpy((synth.rng_for(1, 0, s).random((1, 12, 12, 12)) < 0.5).astype(np.float32)).to(dev)
            for s in range(seeds)]
    desc = dict(cell=base.cell, n=base.n, frac=base.frac, b=base.b, taylor_order=0, has_occ=True)
    # single instance
    h = dsx.Model(**desc, n_configs=1)
    h.set_grid(base.g0, count)
    h.set_sites(0, occs[0])
    out = torch.empty(count, dtype=torch.float32, device=dev)
    lat = []
    for i in range(steps + 10):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.set_sites_async(0, occs[i % seeds])
        h.compute_intensity(out)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    lat = np.sort(np.array(lat[10:]))
    res = {"workload": "compositional simple cubic, 12^3 supercell, Bernoulli(0.5), 48^3 voxels",
           "voxels": vox,
           "single_instance": {"p50_ms": round(float(np.median(lat)) * 1e3, 4),
                               "p99_ms": round(float(lat[int(0.99 * (len(lat) - 1))]) * 1e3, 4),
                               "voxels_per_s": round(vox / float(np.median(lat)), 1)}}
    if O is not None:
        m0 = synth.compositional(n=12, M=1, hmax=2)
        m0.occ = occs[(steps + 9) % seeds].cpu().numpy()[None]
        res["single_instance"]["parity"] = c15_report(O.grid_points(m0.g0, m0.count), out.cpu().numpy().ravel(),
                                                      O.intensity(m0), m0.n)
    h.close()
    # (a) the seeds as one model's ensemble
    he = dsx.Model(**desc, n_configs=seeds)
    he.set_grid(base.g0, count)
    for c in range(seeds):
        he.set_sites(c, occs[c])
    he.autotune(0)

    def ens_step():
        for c in range(seeds):
            he.set_sites_async(c, occs[c])
        he.compute_intensity(out)

    ens_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(3, steps // 4)):
        ens_step()
    torch.cuda.synchronize()
    te = (time.perf_counter() - t0) / max(3, steps // 4)
    he.close()
    res["ensemble_one_model"] = {"configurations": seeds, "ms_per_step": round(te * 1e3, 3),
                                 "config_voxels_per_s": round(seeds * vox / te, 1),
                                 "note": "step includes the stream-ordered upload of every configuration"}
    # (b) independent models in one batch
    hs, outs = [], []
    for c in range(seeds):
        hm = dsx.Model(**desc, n_configs=1)
        hm.set_grid(base.g0, count)
        hm.set_sites(0, occs[c])
        hm.tune_set(0, 0, 12)
        hs.append(hm)
        outs.append(torch.empty(count, dtype=torch.float32, device=dev))
    c0 = time.perf_counter()
    batch = dsx.Batch(hs, outs, mode=BATCH_MODES[batch_mode])
    t_create = time.perf_counter() - c0
    batch.run()
    torch.cuda.synchronize()
    if probe:
        copy_probe(torch, dev)
    t0 = time.perf_counter()
    for _ in range(max(3, steps // 4)):
        batch.run()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / max(3, steps // 4)
    res["batch_of_models"] = {"models": seeds, "ms_per_step": round(tb * 1e3, 3),
                              "voxels_per_s": round(seeds * vox / tb, 1), "create_s": round(t_create, 2),
                              "graph": batch_graph_report(dsx, batch.info())}
    if O is not None:
        m1 = synth.compositional(n=12, M=1, hmax=2)
        m1.occ = occs[seeds - 1].cpu().numpy()[None]
        res["batch_of_models"]["parity_last_model"] = c15_report(
            O.grid_points(m1.g0, m1.count), outs[-1].cpu().numpy().ravel(), O.intensity(m1), m1.n)
    batch.close()
    for hm in hs:
        hm.close()
    return res


def bench_ensemble(dsx, torch, dev, steps, warmup, lm=2, probe=False, batched_only=False, batch_mode="auto"):
    """Batched ensemble (8 models x 8 configurations, edges from {16,20,24,32,40}, 1-4
    sites, Taylor order 6, |h|,|k|,|l| <= 4, Lanczos filter): one graph replay against the
    plain path that calls noise_filter model by model.  Both steps first upload every
    configuration again (stream-ordered device copies), so both recompute all spectra."""
    import synth
    models = synth.ensemble()
    hs, outs, sites = [], [], []
    for m in models:
        h = dsx.Model(cell=m.cell, n=m.n, frac=m.frac, b=m.b, taylor_order=m.order,
                      n_configs=m.n_configs, has_occ=m.occ is not None)
        h.set_grid(m.g0, m.count)
        st = []
        for c in range(m.n_configs):
            occ = None if m.occ is None else torch.from_numpy(m.occ[c]).to(dev)
            disp = None if m.disp is None else torch.from_numpy(m.disp[c]).to(dev)
            st.append((occ, disp))
            h.set_sites(c, occ, disp)
        hs.append(h)
        sites.append(st)
        outs.append(torch.empty(tuple(m.count), dtype=torch.float32, device=dev))
    voxels = sum(int(np.prod(m.count)) * m.n_configs for m in models)
    for h in hs:              # the plain path and the batch run the same tuned plans
        h.autotune(lm)

    def upload():
        for h, st in zip(hs, sites):
            for c, (occ, disp) in enumerate(st):
                h.set_sites_async(c, occ, disp)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def plain():
        upload()
        for h, o in zip(hs, outs):
            h.noise_filter(lm, 1, o)

    t_upload = timed(upload)
    t_plain = timed(plain)
    ref = [o.clone() for o in outs]
    c0 = time.perf_counter()
    batch = dsx.Batch(hs, outs, lanczos_m=lm, mode=BATCH_MODES[batch_mode])
    t_create = time.perf_counter() - c0

    def batched():
        upload()
        batch.run()

    if probe:
        for _ in range(warmup):
            batched()
        copy_probe(torch, dev)
    t_batch = timed(batched)
    same = all(torch.equal(a, b) for a, b in zip(ref, outs))
    graph = batch.info()
    batch.close()
    for h in hs:
        h.close()
    return {"workload": "8 models x 8 configurations, edges {16,20,24,32,40}, 1-4 fcc-prefix sites, "
                        "displacive (Taylor order 6) or compositional, |h|,|k|,|l|<=4, Lanczos m=2",
            "voxels_per_step": voxels,
            "batched_voxels_per_s": round(voxels / t_batch, 1),
            "plain_voxels_per_s": round(voxels / t_plain, 1),
            "batched_ms": round(t_batch * 1e3, 3), "plain_ms": round(t_plain * 1e3, 3),
            "upload_ms": round(t_upload * 1e3, 3),
            "batched_compute_ms": round((t_batch - t_upload) * 1e3, 3),
            "plain_compute_ms": round((t_plain - t_upload) * 1e3, 3),
            "create_and_tune_s": round(t_create, 2),
            "batched_equals_plain": bool(same),
            "graph": batch_graph_report(dsx, graph)}


def batch_graph_report(dsx, info):
    """The batch's graph: the form it runs (chosen by timing both at creation), kernel
    launches of the models against dispatches of the graph, and both forms' replay times."""
    return {"form": "merged" if info["mode"] == dsx.BATCH_MERGED else "per_model",
            "model_launches": info["launches"], "graph_dispatches": info["dispatches"],
            "merged_dispatches": info["merged_nodes"], "kept_apart_for_spills": info["unmerged_spill"],
            "merged_form_dispatches": info["merged_form_dispatches"] if info["merged_form_dispatches"] >= 0 else None,
            "per_model_replay_ms": round(info["per_model_ms"], 4) if info["per_model_ms"] > 0 else None,
            "merged_replay_ms": round(info["merged_ms"], 4) if info["merged_ms"] > 0 else None}


def serving_pool(n_models=64, variants=4, frac=0.01):
    """Resident models of the serving workload and, per model, device-ready site variants:
    the model's own sites, and refinement moves that each change 1 % of its sites (an
    occupancy flipped, a displacement or a spin drawn anew)."""
    import synth
    pool = [synth.serving_request_model(workload=5, model=i) for i in range(n_models)]
    sites = []
    for i, m in enumerate(pool):
        base = (None if m.occ is None else m.occ[0], None if m.disp is None else m.disp[0],
                None if m.spin is None else m.spin[0])
        vs = [base]
        r = np.random.default_rng([5, i, 40_000])
        S, nn = m.n_sites, tuple(m.n)
        for _ in range(variants - 1):
            occ, disp, spin = (None if a is None else a.copy() for a in base)
            nsite = S * int(np.prod(nn))
            pick = r.choice(nsite, max(1, int(round(frac * nsite))), replace=False)
            if occ is not None:
                flat = occ.reshape(-1)
                flat[pick] = 1.0 - flat[pick]
            elif disp is not None:
                flat = disp.reshape(-1, 3)
                flat[pick] = r.normal(0.0, 0.004, (len(pick), 3)).astype(np.float32)
            else:
                flat = spin.reshape(-1, 3)
                v = r.normal(size=(len(pick), 3))
                flat[pick] = (v / np.linalg.norm(v, axis=-1, keepdims=True)).astype(np.float32)
            vs.append((occ, disp, spin))
        sites.append(vs)
    return pool, sites


def bench_serving(dsx, torch, dev, seconds, slots=4):
    """Open-loop Poisson requests (200/s) over 64 resident models of the serving workload
    (edge 8..64, 1-16 random sites, compositional / displacive order 6 / magnetic,
    |h|,|k|,|l| <= 2), each request a refinement move of 1 % of its model's sites: the server (continuous batching over `slots` streams, arena
    admission) against the plain path serving the same trace first come first served
    with one synchronous call at a time.  A burst of every request at once gives the
    saturated throughput of both."""
    import synth
    pool, sites = serving_pool()
    arrivals = synth.poisson_arrivals(rate=200.0, duration=seconds)
    pick = np.random.default_rng([5, 0, 50_000])
    reqs = [(int(pick.integers(0, len(pool))), int(pick.integers(0, len(sites[0])))) for _ in arrivals]
    dsites = [[tuple(None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in v)
               for v in vs] for vs in sites]
    outs = [torch.empty(tuple(m.count), dtype=torch.float32, device=dev) for m in pool]
    vox = [int(np.prod(m.count)) for m in pool]

    def desc(m):
        return dict(cell=m.cell, n=m.n, frac=m.frac, b=m.b, kind=m.kind,
                    taylor_order=m.order if m.kind == 0 else 0, n_configs=1,
                    has_occ=m.occ is not None, ff=m.ff)

    # ---- server
    srv = dsx.Server(slots=slots, queue_capacity=4096, arena_bytes=24 << 30)
    hs = []
    for m, v in zip(pool, dsites):
        h = srv.add_model(**desc(m))
        h.set_grid(m.g0, m.count)
        h.set_sites(0, *v[0])
        hs.append(h)
    for i in range(len(pool)):          # warm: tables, first launches
        srv.wait(srv.submit(hs[i], outs[i], 0, *dsites[i][0]))
    srv.stats(reset=True)
    lag = 0.0
    t0 = time.perf_counter()
    tickets = []
    for ta, (i, v) in zip(arrivals, reqs):
        while True:
            dt = t0 + ta - time.perf_counter()
            if dt <= 0:
                break
            time.sleep(dt if dt > 2e-3 else 0)
        lag = max(lag, time.perf_counter() - (t0 + ta))
        tickets.append(srv.submit(hs[i], outs[i], 0, *dsites[i][v]))
    for t in tickets:
        srv.wait(t)
    open_srv = srv.stats(reset=True)
    tb = time.perf_counter()
    tickets = [srv.submit(hs[i], outs[i], 0, *dsites[i][v]) for (i, v) in reqs]
    for t in tickets:
        srv.wait(t)
    burst_srv = time.perf_counter() - tb
    burst_stats = srv.stats(reset=True)
    srv.close()
    # the same burst on a server without merged rounds (one request per slot)
    srv1 = dsx.Server(slots=slots, queue_capacity=4096, arena_bytes=24 << 30, max_round=1)
    hs1 = []
    for m, v in zip(pool, dsites):
        h = srv1.add_model(**desc(m))
        h.set_grid(m.g0, m.count)
        h.set_sites(0, *v[0])
        hs1.append(h)
    for i in range(len(pool)):
        srv1.wait(srv1.submit(hs1[i], outs[i], 0, *dsites[i][0]))
    tb = time.perf_counter()
    tickets = [srv1.submit(hs1[i], outs[i], 0, *dsites[i][v]) for (i, v) in reqs]
    for t in tickets:
        srv1.wait(t)
    burst_srv1 = time.perf_counter() - tb
    srv1.close()

    # ---- plain path: one synchronous call at a time, same trace
    plain = []
    for m, v in zip(pool, dsites):
        h = dsx.Model(**desc(m))
        h.set_grid(m.g0, m.count)
        h.set_sites(0, *v[0])
        h.compute_intensity(outs[len(plain)])
        plain.append(h)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for ta, (i, v) in zip(arrivals, reqs):
        while time.perf_counter() < t0 + ta:
            dt = t0 + ta - time.perf_counter()
            time.sleep(dt if dt > 2e-3 else 0)
        plain[i].set_sites(0, *dsites[i][v])
        plain[i].compute_intensity(outs[i])
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - (t0 + ta)) * 1e3)
    span_plain = time.perf_counter() - t0
    tb = time.perf_counter()
    for (i, v) in reqs:
        plain[i].set_sites(0, *dsites[i][v])
        plain[i].compute_intensity(outs[i])
    torch.cuda.synchronize()
    burst_plain = time.perf_counter() - tb
    for h in plain:
        h.close()
    total_vox = sum(vox[i] for (i, _) in reqs)
    lat = np.sort(np.array(lat))
    pct = lambda p: float(lat[max(0, int(np.ceil(p * len(lat))) - 1)])
    return {"workload": f"Poisson 200 req/s for {seconds:g} s ({len(reqs)} requests) over {len(pool)} resident "
                        "models: edge U{8..64}, 1-16 sites, compositional / displacive (order 6) / "
                        "magnetic, |h|,|k|,|l|<=2, each request a refinement move of 1 % of its model's sites",
            "server": {"slots": slots, "voxels_per_s": round(open_srv["voxels"] / max(open_srv["span_s"], 1e-9), 1),
                       "p50_ms": round(open_srv["p50_ms"], 3), "p99_ms": round(open_srv["p99_ms"], 3),
                       "max_ms": round(open_srv["max_ms"], 3), "completed": open_srv["completed"],
                       "peak_in_flight": open_srv["peak_in_flight"],
                       "arena_peak_GB": round(open_srv["arena_peak_bytes"] / 1e9, 3),
                       "max_submit_lag_ms": round(lag * 1e3, 3),
                       "mean_round": round(open_srv["round_requests"] / max(open_srv["rounds"], 1), 2),
                       "saturated_voxels_per_s": round(total_vox / burst_srv, 1),
                       "saturated_p99_ms": round(burst_stats["p99_ms"], 3),
                       "saturated_mean_round": round(burst_stats["round_requests"] / max(burst_stats["rounds"], 1), 2),
                       "saturated_voxels_per_s_one_request_per_slot": round(total_vox / burst_srv1, 1)},
            "plain": {"voxels_per_s": round(total_vox / span_plain, 1), "p50_ms": round(pct(0.5), 3),
                      "p99_ms": round(pct(0.99), 3), "max_ms": round(float(lat[-1]), 3),
                      "saturated_voxels_per_s": round(total_vox / burst_plain, 1)},
            "offered_voxels_per_s": round(total_vox / seconds, 1)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--order", type=int, default=8)
    ap.add_argument("--lanczos-m", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", action="store_true", help="also time compute_intensity for orders 1..8")
    ap.add_argument("--copy-probe", action="store_true",
                    help="issue one plain device copy of known size (reference for PMC byte counters)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the traffic summary from two rocprofv3 --pmc output folders and exit")
    ap.add_argument("--pmc-command", default="", help="command line recorded in the summary")
    ap.add_argument("--summarize-ktrace", metavar="TRACE_DIR",
                    help="write the kernel-time summary from a rocprofv3 --kernel-trace --stats folder and exit")
    ap.add_argument("--profile-name", default="displacive32_order8", choices=sorted(WORKLOADS),
                    help="workload the summary covers (names the file under profiles/)")
    ap.add_argument("--only-steps", action="store_true",
                    help="time the filtered steps only (no unfiltered pass, sweep, ensemble, serving or "
                         "CPU baseline): the run the profiles are taken from")
    ap.add_argument("--no-tune", action="store_true", help="run with the default plan instead of tuning it")
    ap.add_argument("--plan", metavar="FORM,FFT,FILTER",
                    help="run this plan instead of tuning (recombination form, FFT fields per plane block, "
                         "filter planes per block, as the line's plan object reports them)")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble comparison")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="time only the batched ensemble (for kernel traces of the graph path)")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the Poisson request trace of the serving comparison (0: skip)")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving comparison")
    ap.add_argument("--magnetic-only", action="store_true",
                    help="time only the magnetic workload (for kernel traces of its recombination)")
    ap.add_argument("--compositional-only", action="store_true", help="time only the compositional workload")
    ap.add_argument("--batch-mode", default="auto", choices=sorted(BATCH_MODES),
                    help="graph form of the batched legs (auto: the faster of the two, timed at creation)")
    args = ap.parse_args()
    if args.summarize_ktrace:
        print(summarize_ktrace(args.summarize_ktrace, args.profile_name, args.pmc_command))
        return
    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.profile_name,
                                       args.pmc_command)))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs the hot path on one GPU; --gpus must be 1 "
              "(the multi-GPU sharding is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1809_07088_amd as dsx
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.ensemble_only:
        print(json.dumps({"ensemble": bench_ensemble(dsx, torch, dev, args.steps, args.warmup,
                                                     probe=args.copy_probe, batch_mode=args.batch_mode)}))
        return
    if args.serving_only:
        print(json.dumps({"serving": bench_serving(dsx, torch, dev, args.serve_seconds)}))
        return
    if args.magnetic_only:
        print(json.dumps({"magnetic": bench_magnetic(dsx, torch, dev, args.steps, args.warmup,
                                                     probe=args.copy_probe)}))
        return
    if args.compositional_only:
        print(json.dumps({"compositional": bench_compositional(dsx, torch, dev, args.steps, probe=args.copy_probe,
                                                               batch_mode=args.batch_mode)}))
        return
    N, lm = args.order, args.lanczos_m
    model = synth.displacive(n=32, M=1, order=N, hmax=8)
    n, S, M = model.n, model.n_sites, model.n_configs
    count = tuple(model.count)
    voxels = int(np.prod(count)) * M
    disp_dev = torch.from_numpy(model.disp[0]).to(dev)
    h = dsx.Model(cell=model.cell, n=n, frac=model.frac, b=model.b, taylor_order=N, n_configs=M)
    h.set_grid(model.g0, count)
    out = torch.empty(count, dtype=torch.float32, device=dev)
    info = dsx.plan_query(cell=model.cell, n=n, frac=model.frac, b=model.b, taylor_order=N, n_configs=M)

    def step():
        h.set_sites_async(0, None, disp_dev)     # stream-ordered device copy of the sites
        h.noise_filter(lm, 1, out)

    # plan tuning happens once per model, before any timed step
    h.set_sites_async(0, None, disp_dev)
    if args.plan:
        h.tune_set(*[int(v) for v in args.plan.split(",")])
    elif not args.no_tune:
        h.autotune(lm)
    plan = h.tune_query()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # the probe also marks where profiled dispatches start counting: after the tuning
    # and the warm-up (the recombination needs some 20 steps to reach its steady time)
    if args.copy_probe:
        copy_probe(torch, dev)
    # HIP events bracket only the dominant kernel inside the timed region (events
    # around every launch add about 30 us to a step)
    dsx.profile_reset()
    dsx.profile_select("recombine")
    dsx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dsx.profile_enable(False)
    kstats = dsx.profile_read()
    # per-kernel breakdown from untimed steps with every launch bracketed
    dsx.profile_reset()
    dsx.profile_select(None)
    dsx.profile_enable(True)
    for _ in range(min(args.steps, 20)):
        step()
    torch.cuda.synchronize()
    dsx.profile_enable(False)
    kall = dsx.profile_read()
    dsx.profile_reset()
    # sampled filtered outputs for the parity check (faces, mirror plane, tile edges)
    rs = np.random.default_rng([2, 0, 778])
    edges = [np.array(sorted({0, 1, 255, 256, 257, 511, 512} | {b + d for b in range(0, c, 32) for d in (-1, 0)}))
             for c in count]
    fidx = np.stack([np.where(rs.random(64) < 0.75, e[rs.integers(0, len(e), 64)], rs.integers(0, c, 64))
                     for e, c in zip(edges, count)], -1).clip(0, np.asarray(count) - 1)
    tidx = torch.as_tensor(fidx, device=dev)
    F_gpu = out[tidx[:, 0], tidx[:, 1], tidx[:, 2]].cpu().numpy()
    sec = (t1 - t0) / args.steps
    value = voxels / sec

    # dominant kernel: recombination on the grown box
    ext_g0 = tuple(g - lm for g in model.g0)
    ext_cnt = tuple(c + 2 * lm for c in count)
    nclass3 = len(np.unique(model.frac[:, 2]))
    sym = all(c % 2 == 1 and g == -(c - 1) // 2 for g, c in zip(ext_g0, ext_cnt))
    flops, bytes_ = recombine_work(n, S, nclass3, N, M, ext_g0, ext_cnt, n[2] // 2 + 1,
                                   info.fields_per_site, friedel=sym)
    launches, tot_ms = kstats.get("recombine", (0, float("nan")))
    t_launch = tot_ms / max(launches, 1) / 1e3
    roof = roofline(flops, bytes_, t_launch, "recombine", stored_trace_avg("displacive32_order8", "k_recombine"))
    tr = stored_traffic("displacive32_order8")
    if tr is not None:
        roof["traffic"] = int(tr["traffic_bytes"])
    kernels = {k: {"launches": v[0], "avg_ms": round(v[1] / max(v[0], 1), 4)} for k, v in kall.items()}

    if args.only_steps:
        args.no_cpu_baseline, args.sweep, args.no_ensemble, args.serve_seconds = True, False, True, 0.0
    # unfiltered path (compute_intensity) for context
    unfiltered = None
    for _ in range(0 if args.only_steps else 2):
        h.set_sites_async(0, None, disp_dev)
        h.compute_intensity(out)
    torch.cuda.synchronize()
    if not args.only_steps:
        u0 = time.perf_counter()
        for _ in range(args.steps):
            h.set_sites_async(0, None, disp_dev)
            h.compute_intensity(out)
        torch.cuda.synchronize()
        unfiltered = voxels / ((time.perf_counter() - u0) / args.steps)
        I_gpu = out.cpu().numpy()

    # the widened filter: the m' cutoff modification on the same box, and an off-axis
    # (h h l) plane of 401 x 401 points over |h|, |l| <= 8 (the paper's plane format)
    widened = None
    if not args.only_steps:
        widened = {}
        out2 = torch.empty(count, dtype=torch.float32, device=dev)
        for _ in range(2):
            h.set_sites_async(0, None, disp_dev)
            h.noise_filter_cutoff(lm, 4, 1, out2)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        reps = max(3, args.steps // 2)
        for _ in range(reps):
            h.set_sites_async(0, None, disp_dev)
            h.noise_filter_cutoff(lm, 4, 1, out2)
        torch.cuda.synchronize()
        tc = (time.perf_counter() - c0) / reps
        widened["cutoff_mprime4"] = {"ms_per_step": round(tc * 1e3, 4), "voxels_per_s": round(voxels / tc, 1),
                                     "lanczos_m": lm, "mprime": 4}
        hh, ll = np.meshgrid(np.linspace(-8, 8, 401), np.linspace(-8, 8, 401), indexing="ij")
        Qp = np.stack([hh, hh, ll], -1).reshape(-1, 3) * np.asarray(n, dtype=np.float64)
        pts = torch.empty(len(Qp), dtype=torch.float32, device=dev)
        h.set_sites_async(0, None, disp_dev)
        h.filter_points(lm, Qp, pts)
        c0 = time.perf_counter()
        for _ in range(3):
            h.set_sites_async(0, None, disp_dev)
            h.filter_points(lm, Qp, pts)
        tp = (time.perf_counter() - c0) / 3
        widened["hhl_plane_401x401"] = {"ms_per_call": round(tp * 1e3, 3), "points": int(len(Qp)),
                                        "points_per_s": round(len(Qp) / tp, 1), "lanczos_m": lm,
                                        "note": "I(G) on the 513^3 box holding every window, then "
                                                "the windowed sum per point; host point list, "
                                                "synchronous call"}
        del out2, pts
        # the spherical cutoff (non-separable (2m)^3 stencil) on the same box
        out4 = torch.empty(count, dtype=torch.float32, device=dev)
        for _ in range(2):
            h.set_sites_async(0, None, disp_dev)
            h.noise_filter_spherical(lm, 1, out4)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        for _ in range(reps):
            h.set_sites_async(0, None, disp_dev)
            h.noise_filter_spherical(lm, 1, out4)
        torch.cuda.synchronize()
        tsph = (time.perf_counter() - c0) / reps
        widened["spherical_cutoff"] = {"ms_per_step": round(tsph * 1e3, 4), "voxels_per_s": round(voxels / tsph, 1),
                                       "lanczos_m": lm}
        del out4
        # split sites: the fcc model with 4 discrete displacements per site (16 split
        # sites, compositional path, exact exponential), filtered on the same box
        rs = np.random.default_rng(1234)
        vals = rs.uniform(-0.02, 0.02, (S, 4, 3)).astype(np.float32)
        pick = rs.integers(0, 4, (1, S) + tuple(n))
        dd = np.ascontiguousarray(vals[np.arange(S)[None, :, None, None, None], pick])
        c0 = time.perf_counter()
        fr2, b2, par2, occ2 = dsx.split_sites(n, model.frac, model.b, dd)
        t_map = time.perf_counter() - c0
        hs = dsx.Model(cell=model.cell, n=n, frac=fr2, b=b2, taylor_order=0, n_configs=1, has_occ=True,
                       pos_id=par2, norm_N=float(np.prod(n)) * S)
        hs.set_grid(model.g0, count)
        occ_dev = torch.from_numpy(np.ascontiguousarray(occ2[0])).to(dev)
        out3 = torch.empty(count, dtype=torch.float32, device=dev)
        hs.set_sites_async(0, occ_dev, None)
        hs.autotune(lm)
        for _ in range(2):
            hs.set_sites_async(0, occ_dev, None)
            hs.noise_filter(lm, 1, out3)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        for _ in range(reps):
            hs.set_sites_async(0, occ_dev, None)
            hs.noise_filter(lm, 1, out3)
        torch.cuda.synchronize()
        ts = (time.perf_counter() - c0) / reps
        widened["split_sites_fcc32_K4"] = {"ms_per_step": round(ts * 1e3, 4), "voxels_per_s": round(voxels / ts, 1),
                                           "split_sites": int(len(b2)), "host_mapping_ms": round(t_map * 1e3, 1),
                                           "lanczos_m": lm}
        hs.close()
        del out3, occ_dev

    # one GPU's share of Q-zone sharding over eight GPUs at its real shape: the centred
    # slab |G1| <= 32 of the same box (65 x 513 x 513, Friedel-symmetric like the whole
    # box), with its own tuned plan; the per-voxel rate against the whole box's rate
    # says how far one shard's kernels keep the full-box efficiency
    shard = None
    if not args.only_steps:
        hq = dsx.Model(cell=model.cell, n=n, frac=model.frac, b=model.b, taylor_order=N, n_configs=M)
        g0q = (-32, model.g0[1], model.g0[2])
        cntq = (65, count[1], count[2])
        hq.set_grid(g0q, cntq)
        outq = torch.empty(cntq, dtype=torch.float32, device=dev)
        hq.set_sites_async(0, None, disp_dev)
        hq.autotune(lm)
        for _ in range(3):
            hq.set_sites_async(0, None, disp_dev)
            hq.noise_filter(lm, 1, outq)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        for _ in range(args.steps):
            hq.set_sites_async(0, None, disp_dev)
            hq.noise_filter(lm, 1, outq)
        torch.cuda.synchronize()
        tq = (time.perf_counter() - c0) / args.steps
        vq = int(np.prod(cntq)) * M
        shard = {"slab": "G1 in [-32, 32] (1 of 8 Q zones), G2 and G3 as the whole box",
                 "voxels_per_step": vq, "ms_per_step": round(tq * 1e3, 4),
                 "voxels_per_s": round(vq / tq, 1), "rate_vs_whole_box": round(vq / tq / value, 3),
                 "plan": hq.tune_query(), "lanczos_m": lm}
        hq.close()
        del outq

    sweep = None
    if args.sweep:
        sweep = {}
        for NN in range(1, 9):
            hm = dsx.Model(cell=model.cell, n=n, frac=model.frac, b=model.b, taylor_order=NN, n_configs=M)
            hm.set_grid(model.g0, count)
            hm.set_sites(0, None, disp_dev)
            for _ in range(2):
                hm.set_sites_async(0, None, disp_dev)
                hm.compute_intensity(out)
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            for _ in range(args.steps):
                hm.set_sites_async(0, None, disp_dev)
                hm.compute_intensity(out)
            torch.cuda.synchronize()
            sweep[str(NN)] = round(voxels / ((time.perf_counter() - s0) / args.steps), 1)
            hm.close()

    cpu = None
    parity = None
    order_rule = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        rng = np.random.default_rng([2, 0, 777])
        G_all = lambda k: np.stack([rng.integers(model.g0[a], model.g0[a] + count[a], k)
                                    for a in range(3)], -1).astype(np.int32)
        threads = O.max_threads()
        Gs = G_all(64)
        c0 = time.perf_counter()
        O.intensity(model, Gs, N)
        dt = time.perf_counter() - c0
        k = int(min(65536, max(64, 64 * args.cpu_seconds / max(dt, 1e-3))))
        Gs = G_all(k)
        c0 = time.perf_counter()
        I_or = O.intensity(model, Gs, N)
        dt = time.perf_counter() - c0
        # the same direct sum on one thread: the per-core rate
        per_g_1thread = dt / len(Gs) * threads          # seconds per voxel on one core, about
        G1 = Gs[:int(min(512, max(16, 2.0 / max(per_g_1thread, 1e-6))))]
        O.set_threads(1)
        c1 = time.perf_counter()
        O.intensity(model, G1, N)
        dt1 = time.perf_counter() - c1
        O.set_threads(threads)
        cpu = {"value": round(len(Gs) / dt, 2), "unit": "voxels/s", "cores": threads, "kind": "oracle",
               "sample": f"{len(Gs)} seeded random G of the 513^3 box, FP64 direct sum over all "
                         f"131072 atoms, Taylor order {N}, {dt:.1f} s",
               "per_core_value": round(len(G1) / dt1, 2),
               "per_core_sample": f"{len(G1)} of those G on 1 thread, {dt1:.2f} s"}
        idx = tuple((Gs[:, a] - model.g0[a]) for a in range(3))
        g = I_gpu[idx].astype(np.float64)
        parity = {"unfiltered_vs_fp64_order_N": c15_report(Gs, g, I_or, n)}
        I_ex = O.intensity(model, Gs[:256], -1)
        parity["unfiltered_vs_fp64_exact_256"] = c15_report(Gs[:256], g[:256], I_ex, n)
        Qf = fidx + np.asarray(model.g0)
        F_or = oracle_filtered_points(O, model, Qf, lm, N)
        parity["filtered_vs_fp64_order_N"] = c15_report(Qf, F_gpu, F_or, n)
        # the order rule: the GPU at each Taylor order N against the exact exponential
        order_rule = {"voxels": 256, "rel_l2_vs_exact": {}, "rel_l2_vs_same_order_oracle": {}}
        for NN in range(1, 9):
            hm = dsx.Model(cell=model.cell, n=n, frac=model.frac, b=model.b, taylor_order=NN, n_configs=M)
            hm.set_grid(model.g0, count)
            hm.set_sites(0, None, disp_dev)
            hm.compute_intensity(out)
            torch.cuda.synchronize()
            gN = out[tuple(torch.as_tensor(v, device=dev) for v in idx)][:256].cpu().numpy().astype(np.float64)
            order_rule["rel_l2_vs_exact"][str(NN)] = float(np.linalg.norm(gN - I_ex) / np.linalg.norm(I_ex))
            IN = O.intensity(model, Gs[:256], NN)
            order_rule["rel_l2_vs_same_order_oracle"][str(NN)] = float(np.linalg.norm(gN - IN) / np.linalg.norm(IN))
            hm.close()
    h.close()

    Ocheck = None
    if not args.no_cpu_baseline:
        from oracle import oracle as Ocheck
    magnetic = None if args.only_steps else bench_magnetic(dsx, torch, dev, args.steps, args.warmup, Ocheck)
    compositional = None if args.only_steps else bench_compositional(dsx, torch, dev, args.steps, Ocheck)
    ensemble = None if args.no_ensemble else bench_ensemble(dsx, torch, dev, max(3, args.steps // 4), 2)
    serving = bench_serving(dsx, torch, dev, args.serve_seconds) if args.serve_seconds > 0 else None

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "voxels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"displacive fcc 4 sites/cell, 32^3 supercell, Taylor order {N}, "
                               f"|h|,|k|,|l|<=8 step 1/32 ({count[0]}^3 voxels), Lanczos m={lm}",
                   "voxels_per_step": voxels, "taylor_order": N, "lanczos_m": lm,
                   "fft_fields": info.total_fields},
        "plan": plan,
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": parity,
        "order_rule": order_rule,
        "unfiltered_voxels_per_s": None if unfiltered is None else round(unfiltered, 1),
        "kernels": kernels,
    }
    if sweep is not None:
        line["compute_intensity_voxels_per_s_by_order"] = sweep
    if widened is not None:
        line["widened_filter"] = widened
    if shard is not None:
        line["q_zone_shard"] = shard
    if magnetic is not None:
        line["magnetic"] = magnetic
    if compositional is not None:
        line["compositional"] = compositional
    if ensemble is not None:
        line["ensemble"] = ensemble
    if serving is not None:
        line["serving"] = serving
    print(json.dumps(line))


if __name__ == "__main__":
    main()
