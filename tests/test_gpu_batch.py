"""GPU tests of batched execution (one hipGraph over several models) and the
autotuner: a batch must reproduce, bit for bit, what each model computes alone,
and match the FP64 oracle."""
import sys

import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests.helpers import assert_parity, max_rel, MAXTOL, rel_l2, to_dsx

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(msg):
    print(f"[gpu case] {msg}", flush=True)
    sys.stdout.flush()


def small_ensemble():
    # uneven sizes, both disorder types, several configurations each
    ms = [synth.displacive(workload=40, model=0, n=8, M=3, order=6, hmax=2, n_sites=3),
          synth.compositional(workload=40, model=1, n=10, M=4, hmax=2, closed=True,
                              frac=synth.FCC_BASIS[:2], b=synth.FCC_B[:2]),
          synth.displacive(workload=40, model=2, n=12, M=2, order=4, hmax=1, n_sites=1),
          synth.random_model(41, n=(6, 5, 7), S=2, M=2, order=3)]
    ms[3].g0, ms[3].count = (-6, -5, -7), (13, 11, 15)
    return ms


MODES = {"auto": 0, "per_model": 1, "merged": 2}


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("lm", [0, 2])
def test_batch_equals_individual_and_oracle(lm, mode):
    import torch
    import paper_1809_07088_amd as dsx
    models = small_ensemble()
    say(f"batch of {len(models)} models, lanczos_m={lm}, mode {mode}")
    hs = [to_dsx(m) for m in models]
    outs = [torch.full(tuple(m.count), -1.0, device="cuda") for m in models]
    batch = dsx.Batch(hs, outs, lanczos_m=lm, mode=MODES[mode])
    info = batch.info()
    print("batch info", info)
    if mode == "merged":
        # uneven n, orders and kinds: launches of one kernel and LDS class are shared (the
        # lattice-sum reduction at least), so the graph has fewer dispatches than launches
        assert info["mode"] == dsx.BATCH_MERGED and info["merged_nodes"] >= 1
        assert info["dispatches"] < info["launches"]
    elif mode == "per_model":
        assert info["mode"] == dsx.BATCH_PER_MODEL and info["merged_nodes"] == 0
        assert info["dispatches"] == info["launches"]
    else:
        assert info["merged_ms"] > 0 and info["per_model_ms"] > 0
        assert info["mode"] == (dsx.BATCH_MERGED if info["merged_ms"] <= info["per_model_ms"] else dsx.BATCH_PER_MODEL)
    batch.run()
    torch.cuda.synchronize()
    got = [o.cpu().numpy() for o in outs]
    for m, h, g in zip(models, hs, got):
        alone = torch.empty(tuple(m.count), device="cuda")
        if lm:
            h.noise_filter(lm, 1, alone)
        else:
            h.compute_intensity(alone)
        torch.cuda.synchronize()
        assert np.array_equal(alone.cpu().numpy(), g)
        ref = O.filtered_intensity(m, lm, 1) if lm else O.intensity(m).reshape(m.count)
        assert_parity(g, ref)
    # replay after new sites: the graph recomputes the spectra
    m0, h0 = models[0], hs[0]
    new = synth.displacive(workload=40, model=9, n=8, M=3, order=6, hmax=2, n_sites=3)
    for c in range(m0.n_configs):
        h0.set_sites(c, None, torch.from_numpy(new.disp[c]).cuda())
    batch.run()
    torch.cuda.synchronize()
    ref = O.filtered_intensity(new, lm, 1) if lm else O.intensity(new).reshape(new.count)
    assert_parity(outs[0].cpu().numpy(), ref)
    # the batch holds its models' recorded buffers
    with pytest.raises(dsx.DsxError) as e:
        h0.set_grid(m0.g0, m0.count)
    assert e.value.status == dsx.ERR_BUSY
    with pytest.raises(dsx.DsxError) as e:
        dsx.destroy_model(h0.handle)
    assert e.value.status == dsx.ERR_BUSY
    batch.close()
    h0.set_grid(m0.g0, m0.count)
    for h in hs:
        h.close()


def test_merged_batch_of_many_small_models():
    """64 compositional models of one shape and 16 of another: one dispatch per step for
    each shape; every output equals the model computed alone, bit for bit, and the oracle."""
    import torch
    import paper_1809_07088_amd as dsx
    models = [synth.compositional(workload=46, model=i, n=6 if i < 64 else 5, M=1, hmax=1)
              for i in range(80)]
    say("merged batch of 80 small models (two shapes)")
    hs = [to_dsx(m) for m in models]
    for h in hs:
        h.tune_set(0, 0, 12)
    outs = [torch.full(tuple(m.count), -1.0, device="cuda") for m in models]
    batch = dsx.Batch(hs, outs, mode=dsx.BATCH_MERGED)
    info = batch.info()
    print("batch info", info)
    # about six launches a model (sums, their reduction, two FFT passes, recombination,
    # Bragg points); the two shapes share a node wherever they run the same kernel with
    # the same block size, so a step has at most two nodes
    assert info["launches"] >= 5 * len(models)
    assert info["dispatches"] <= 16 and info["merged_nodes"] >= 5
    batch.run()
    torch.cuda.synchronize()
    for k in (0, 1, 37, 63, 64, 79):
        alone = torch.empty(tuple(models[k].count), device="cuda")
        hs[k].compute_intensity(alone)
        torch.cuda.synchronize()
        assert torch.equal(alone, outs[k]), k
        assert_parity(outs[k].cpu().numpy(), O.intensity(models[k]).reshape(models[k].count))
    # a second replay after new sites on some models
    for k in (3, 70):
        new = synth.compositional(workload=47, model=k, n=models[k].n[0], M=1, hmax=1)
        hs[k].set_sites(0, torch.from_numpy(new.occ[0]).cuda())
        models[k] = new
    batch.run()
    torch.cuda.synchronize()
    for k in (3, 70):
        assert_parity(outs[k].cpu().numpy(), O.intensity(models[k]).reshape(models[k].count))
    batch.close()
    for h in hs:
        h.close()


def test_merged_and_per_model_batches_agree_bitwise():
    import torch
    import paper_1809_07088_amd as dsx
    models = small_ensemble()
    say("merged vs per-model batch, bitwise")
    hs = [to_dsx(m) for m in models]
    res = {}
    for mode in (dsx.BATCH_PER_MODEL, dsx.BATCH_MERGED):
        outs = [torch.full(tuple(m.count), -1.0, device="cuda") for m in models]
        b = dsx.Batch(hs, outs, lanczos_m=2, mode=mode)
        for _ in range(3):      # replays with the program's own work between them
            b.run()
            torch.cuda.synchronize()
            res.setdefault(mode, []).append([o.clone() for o in outs])
        b.close()
    for r in res[dsx.BATCH_PER_MODEL] + res[dsx.BATCH_MERGED]:
        for a, b in zip(res[dsx.BATCH_PER_MODEL][0], r):
            assert torch.equal(a, b)
    for h in hs:
        h.close()


def test_autotune_cache_is_deterministic(tmp_path, monkeypatch):
    import torch
    import paper_1809_07088_amd as dsx
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("DSX_TUNE_CACHE", str(cache))
    m = synth.displacive(workload=42, n=8, M=1, order=5, hmax=2)
    say("autotune with a cache file")
    h = to_dsx(m)
    h.autotune(2)
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and "\t" in lines[0]
    h2 = to_dsx(m)
    assert not h2.tune_query()["tuned"]
    h2.autotune(2)                        # read back, no second entry
    assert cache.read_text().strip().splitlines() == lines
    q, q2 = h.tune_query(), h2.tune_query()
    assert q == q2 and q["tuned"]
    # the cache line holds the choices in the order form, FFT fields per block, filter
    # planes, axis-1 column tile, then the radix sequence of each axis
    f = lines[0].split("\t")[1].split()
    assert len(f) == 7
    v, fc, t1, tc = (int(x) for x in f[:4])
    assert (q["recombine_form"], q["fft_fields_per_block"], q["filter_planes_per_block"]) == (v, fc, t1)
    qf = h.tune_query_fft()
    assert qf == h2.tune_query_fft() and qf["col_tile"] == tc
    for a in range(3):
        assert "x".join(str(r) for r in qf["radices"][a]) == f[4 + a]
        assert int(np.prod(qf["radices"][a])) == m.n[a]
    assert v in (0, 2, 3, 4) and fc in (0, 1, 2, 4) and t1 in (4, 6, 8, 12, 16, 20, 26, 32, 52, 64)
    a = torch.empty(tuple(m.count), device="cuda")
    b = torch.empty(tuple(m.count), device="cuda")
    h.compute_intensity(a)
    h2.compute_intensity(b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert_parity(a.cpu().numpy(), O.intensity(m).reshape(m.count))
    h.close()
    h2.close()


def test_batch_rejects_bad_arguments():
    import torch
    import paper_1809_07088_amd as dsx
    m = synth.random_model(43, n=(4, 4, 4), S=1, M=1, order=1)
    say("batch argument errors")
    h = to_dsx(m)
    out = torch.empty(tuple(m.count), device="cuda")
    with pytest.raises(dsx.DsxError) as e:
        dsx.Batch([h, h], [out, out])
    assert e.value.status == dsx.ERR_ARG
    with pytest.raises(dsx.DsxError) as e:
        dsx.Batch([h], [out], lanczos_m=1)
    assert e.value.status == dsx.ERR_ARG
    # outputs: the binding checks size, dtype, layout and device before the call
    with pytest.raises(ValueError):
        dsx.Batch([h], [torch.empty(out.numel() - 1, device="cuda")])
    with pytest.raises(ValueError):
        dsx.Batch([h], [out.double()])
    with pytest.raises(ValueError):
        dsx.Batch([h], [out.cpu()])
    with pytest.raises(ValueError):
        dsx.Batch([h], [out], lanczos_m=2, oversample=2)     # s = 2 needs 8 times the voxels
    h.close()


def test_profile_select_times_one_kernel_kind():
    import torch
    import paper_1809_07088_amd as dsx
    m = synth.random_model(44, n=(6, 5, 7), S=2, M=2, order=3)
    say("profile_select")
    h = to_dsx(m)
    out = torch.empty(tuple(m.count), device="cuda")
    h.compute_intensity(out)
    ref = out.clone()
    try:
        dsx.profile_reset()
        dsx.profile_select("recombine")
        dsx.profile_enable(True)
        for _ in range(3):
            h.compute_intensity(out)
        torch.cuda.synchronize()
        dsx.profile_enable(False)
        only = dsx.profile_read()
        dsx.profile_reset()
        dsx.profile_select(None)
        dsx.profile_enable(True)
        h.compute_intensity(out)
        torch.cuda.synchronize()
        dsx.profile_enable(False)
        every = dsx.profile_read()
    finally:
        dsx.profile_enable(False)
        dsx.profile_select(None)
        dsx.profile_reset()
    assert set(only) == {"recombine"}
    assert only["recombine"][0] == 3 and only["recombine"][1] > 0
    # unchanged sites keep their spectra: a repeated call runs recombination and Bragg points
    assert {"recombine", "bragg"} <= set(every)
    assert torch.equal(out, ref)
    h.close()


def test_tune_set_plan_and_errors():
    import torch
    import paper_1809_07088_amd as dsx
    m = synth.random_model(45, n=(6, 5, 7), S=2, M=2, order=3)
    say("tune_set")
    h = to_dsx(m)
    out = torch.empty(tuple(m.count), device="cuda")
    ref = O.intensity(m).reshape(m.count)
    for plan in [(0, 0, 12), (0, 2, 8), (2, 1, 4), (3, 4, 64), (4, 2, 1)]:
        h.tune_set(*plan)
        q = h.tune_query()
        assert (q["recombine_form"], q["fft_fields_per_block"], q["filter_planes_per_block"]) == plan
        assert q["tuned"]
        h.compute_intensity(out)
        torch.cuda.synchronize()
        assert_parity(out.cpu().numpy(), ref)
    for bad in [(1, 0, 12), (5, 0, 12), (0, 3, 12), (0, 0, 0), (0, 0, 65)]:
        with pytest.raises(dsx.DsxError) as e:
            h.tune_set(*bad)
        assert e.value.status == dsx.ERR_ARG
    h.close()


def test_fft_radix_orders_and_column_tiles():
    """Every radix order the tuner may pick computes the same intensities (to rounding):
    forced sequences on edges 12, 20 and 18 (radices 2, 3, 4, 5 and the odd 9), and the
    axis-1 column tiles."""
    import torch
    import paper_1809_07088_amd as dsx
    m = synth.random_model(48, n=(12, 20, 18), S=2, M=2, order=4)
    m.g0, m.count = (-13, -21, -19), (27, 43, 39)
    say("forced FFT radix orders and column tiles")
    h = to_dsx(m)
    ref = O.intensity(m).reshape(m.count)
    out = torch.empty(tuple(m.count), device="cuda")
    plans = [None, ([3, 4], [5, 4], [2, 9]), ([4, 3], [4, 5], [9, 2]), ([2, 2, 3], [2, 5, 2], [3, 2, 3]),
             ([3, 2, 2], [2, 2, 5], [3, 3, 2])]
    for plan in plans:
        for tile in (0, 16, 32, 64):
            h.tune_set_fft(plan, tile)
            q = h.tune_query_fft()
            assert q["col_tile"] == tile
            if plan is not None:
                assert q["radices"] == [list(r) for r in plan]
            h.compute_intensity(out)
            torch.cuda.synchronize()
            assert_parity(out.cpu().numpy(), ref, what=f"{plan} tile {tile}")
    for bad in [([4, 4], [5, 4], [2, 9]), ([3, 4], [5, 4], [6, 3]), ([3, 4], [5, 4], [1, 18])]:
        with pytest.raises(dsx.DsxError) as e:
            h.tune_set_fft(bad, 0)
        assert e.value.status == dsx.ERR_ARG
    with pytest.raises(dsx.DsxError) as e:
        h.tune_set_fft(None, 48)
    assert e.value.status == dsx.ERR_ARG
    h.close()


def test_autotune_picks_valid_fft_plans():
    import torch
    import paper_1809_07088_amd as dsx
    m = synth.random_model(49, n=(24, 20, 14), S=2, M=1, order=3)
    m.g0, m.count = (-25, -21, -15), (51, 43, 31)
    say("autotune over FFT radix orders")
    h = to_dsx(m)
    h.autotune(0)
    q = h.tune_query_fft()
    for a in range(3):
        assert int(np.prod(q["radices"][a])) == m.n[a]
        assert all(r in (2, 4) or (r % 2 == 1 and r >= 3) for r in q["radices"][a])
    assert q["col_tile"] in (0, 16, 32, 64)
    out = torch.empty(tuple(m.count), device="cuda")
    h.compute_intensity(out)
    torch.cuda.synchronize()
    assert_parity(out.cpu().numpy(), O.intensity(m).reshape(m.count))
    h.close()


def test_merged_magnetic_batch_bitwise():
    """Magnetic models (row-staged recombination, FP64 Bragg points) merged and per model:
    the same bits, and the oracle."""
    import torch
    import paper_1809_07088_amd as dsx
    models = [synth.serving_request_model(workload=50, model=i, n=8, S=S, typ=2) for i, S in enumerate((4, 2, 3))]
    say("magnetic batch, merged against per-model")
    hs = [to_dsx(m) for m in models]
    got = {}
    for mode in (dsx.BATCH_PER_MODEL, dsx.BATCH_MERGED):
        outs = [torch.full(tuple(m.count), -1.0, device="cuda") for m in models]
        b = dsx.Batch(hs, outs, mode=mode)
        b.run()
        torch.cuda.synchronize()
        got[mode] = [o.cpu() for o in outs]
        if mode == dsx.BATCH_MERGED:
            assert b.info()["merged_nodes"] >= 3
        b.close()
    for k, m in enumerate(models):
        assert torch.equal(got[dsx.BATCH_PER_MODEL][k], got[dsx.BATCH_MERGED][k]), k
        assert_parity(got[dsx.BATCH_MERGED][k].numpy(), O.intensity(m).reshape(m.count))
    for h in hs:
        h.close()
