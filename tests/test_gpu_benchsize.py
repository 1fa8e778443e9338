"""GPU parity of the benchmarked outputs at their full size, in the launch
configuration the benchmark times: the filtered 513^3 box of the displacive 32^3 fcc
model at Taylor order 8 (plain filter with the plans the tuner picks from, the m' = 4
cutoff, the spherical cutoff) and points of the 401 x 401 (h h l) plane, each sampled
where the filter's tiles, segments, mirror plane and box faces meet and compared with
the FP64 oracle's windowed sum over I(G) summed directly on each sample's window.
Also the largest serving edges (59, 61, 64) against the oracle on sampled voxels."""
import sys

import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests.helpers import assert_parity, edge_sample_indices, oracle_filtered_at, to_dsx

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def headline():
    """The benchmark's model on the device, its output box, and a torch output."""
    import torch
    m = synth.displacive(n=32, M=1, order=8, hmax=8)
    h = to_dsx(m)
    out = torch.empty(tuple(m.count), dtype=torch.float32, device="cuda")
    yield m, h, out
    h.close()


_oracle_cache = {}


def _cached_oracle(key, fn):
    if key not in _oracle_cache:
        _oracle_cache[key] = fn()
    return _oracle_cache[key]


def _at(out, idx):
    import torch
    t = torch.as_tensor(idx, device=out.device)
    return out[t[:, 0], t[:, 1], t[:, 2]].cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("plan", [None, (0, 0, 8), (0, 0, 12), (0, 1, 16)])
def test_filtered_headline_box(headline, plan):
    import torch
    m, h, out = headline
    if plan is None:
        h.autotune(2)
    else:
        h.tune_set(*plan)
    say(f"filtered 513^3 box, plan {h.tune_query()}")
    out.fill_(float("nan"))
    h.noise_filter(2, 1, out)
    torch.cuda.synchronize()
    assert not torch.isnan(out).any()
    idx = edge_sample_indices(m.count, 192, 11)
    ref = _cached_oracle("plain", lambda: oracle_filtered_at(m, idx + np.asarray(m.g0), 2))
    got = _at(out, idx)
    print("sampled filtered 513^3: rel L2", np.linalg.norm(got - ref) / np.linalg.norm(ref))
    assert_parity(got, ref, what="filtered 513^3")
    # the mirrored half is the computed half written again (I(-Q) = I(Q)): bit for bit
    # off the plane G1 = 0, whose two halves are computed separately
    mid = m.count[0] // 2
    flip = torch.flip(out, dims=(0, 1, 2))
    assert torch.equal(out[:mid], flip[:mid]) and torch.equal(out[mid + 1:], flip[mid + 1:])
    assert_parity(out[mid].cpu().numpy(), flip[mid].cpu().numpy(), what="plane G1 = 0 vs its mirror")


def test_cutoff_mprime4_headline_box(headline):
    import torch
    m, h, out = headline
    say("m' = 4 cutoff filter on the 513^3 box")
    h.noise_filter_cutoff(2, 4, 1, out)
    torch.cuda.synchronize()
    idx = edge_sample_indices(m.count, 32, 12)
    ref = oracle_filtered_at(m, idx + np.asarray(m.g0), 2, mprime=4)
    assert_parity(_at(out, idx), ref, what="m'=4 513^3")


def test_spherical_cutoff_headline_box(headline):
    import torch
    m, h, out = headline
    say("spherical cutoff filter on the 513^3 box")
    h.noise_filter_spherical(2, 1, out)
    torch.cuda.synchronize()
    idx = edge_sample_indices(m.count, 64, 13)
    ref = oracle_filtered_at(m, idx + np.asarray(m.g0), 2, spherical=True)
    assert_parity(_at(out, idx), ref, what="spherical 513^3")


def test_hhl_plane_401(headline):
    import torch
    m, h, _ = headline
    say("(h h l) plane, 401 x 401 points, |h|,|l| <= 8")
    hh, ll = np.meshgrid(np.linspace(-8, 8, 401), np.linspace(-8, 8, 401), indexing="ij")
    Q = np.stack([hh, hh, ll], -1).reshape(-1, 3) * np.asarray(m.n, dtype=np.float64)
    pts = torch.empty(len(Q), dtype=torch.float32, device="cuda")
    h.filter_points(2, Q, pts)
    rng = np.random.default_rng(14)
    corners = [0, 400, 400 * 401, 401 * 401 - 1, 200 * 401 + 200]
    sel = np.concatenate([corners, rng.choice(len(Q), 59, replace=False)])
    ref = oracle_filtered_at(m, Q[sel], 2)
    assert_parity(pts.cpu().numpy()[sel], ref, what="hhl plane")


@pytest.mark.parametrize("kind,n,order", [(synth.NUCLEAR, (59, 61, 64), 6),
                                          (synth.MAGNETIC, (64, 59, 61), 0),
                                          (synth.MAGNETIC, (61, 64, 59), 2)])
def test_largest_serving_edges(kind, n, order):
    """Edges 59 and 61 (prime: direct DFT passes) and 64 on every axis, sampled voxels
    and unit-cell Bragg points of a |h|,|k|,|l| <= 1 box against the oracle."""
    import torch
    m = synth.random_model(3000 + n[0], n=n, S=1 if kind == synth.NUCLEAR else 2, M=1, order=order,
                           kind=kind, mag_order=order, sigma=0.02, with_occ=kind == synth.NUCLEAR)
    m.g0, m.count = synth.box_from_rlu(n, 1, True)
    say(f"largest serving edges kind={kind} n={n} order={order}")
    h = to_dsx(m)
    out = torch.empty(tuple(m.count), dtype=torch.float32, device="cuda")
    h.compute_intensity(out)
    torch.cuda.synchronize()
    idx = edge_sample_indices(m.count, 384, 15)
    H = np.array([[a, b, c] for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]) * np.asarray(n)
    idx = np.concatenate([idx, H - np.asarray(m.g0)])
    ref = O.intensity(m, (idx + np.asarray(m.g0)).astype(np.int32))
    assert_parity(_at(out, idx), ref, what=f"edges {n}")
    h.close()
