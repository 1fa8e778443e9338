"""GPU parity at the workloads' full sizes, in the launch configuration the benchmark
times: sampled voxels against the FP64 oracle (one by one), plus properties that
hold on the whole grid (Friedel symmetry, zero diffuse intensity at the unit-cell
Bragg points of a single configuration)."""
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


def sample_points(model, k, seed):
    rng = np.random.default_rng(seed)
    G = np.stack([rng.integers(model.g0[a], model.g0[a] + model.count[a], k) for a in range(3)], -1)
    n = np.asarray(model.n)
    H = np.stack([rng.integers(-(-model.g0[a] // n[a]), (model.g0[a] + model.count[a] - 1) // n[a] + 1, 64)
                  for a in range(3)], -1) * n
    line = np.stack([np.arange(model.g0[2], model.g0[2] + model.count[2], 7)] * 3, -1)
    line[:, 0] = 0
    line[:, 1] = model.g0[1] + model.count[1] // 3
    return np.concatenate([G, H, line]).astype(np.int32)


def run_full(model):
    import torch
    h = to_dsx(model)
    out = torch.empty(tuple(model.count), dtype=torch.float32, device="cuda")
    h.compute_intensity(out)
    torch.cuda.synchronize()
    I = out.cpu().numpy()
    h.close()
    return I


def at(I, model, G):
    return I[tuple(G[:, a] - model.g0[a] for a in range(3))].astype(np.float64)


@pytest.mark.parametrize("order", [1, 4, 8])
def test_displacive_fcc_32_full_box(order):
    m = synth.displacive(n=32, M=1, order=order, hmax=8)
    say(f"displacive 32^3 order {order}, box {m.count}")
    I = run_full(m)
    assert np.all(np.isfinite(I))
    G = sample_points(m, 768, order)
    ref = O.intensity(m, G, order)
    print("sampled rel L2 vs same-order oracle", rel_l2(at(I, m, G), ref), "worst voxel", max_rel(at(I, m, G), ref))
    assert_parity(at(I, m, G), ref)
    # Friedel symmetry over the whole (symmetric) box
    assert_parity(I, I[::-1, ::-1, ::-1])
    # one configuration: no diffuse intensity at G = 0 (mod n)
    assert np.max(np.abs(I[::32, ::32, ::32])) <= 1e-6 * np.max(I)
    if order == 8:   # truncation below float32 resolution: matches the exact exponential too
        ex = O.intensity(m, G[:256], -1)
        assert_parity(at(I, m, G[:256]), ex)


def test_magnetic_pyrochlore_24_full_box():
    m = synth.magnetic(n=24, M=1, hmax=6)
    say(f"magnetic pyrochlore 24^3, box {m.count}")
    I = run_full(m)
    assert np.all(np.isfinite(I)) and np.all(I >= -1e-6 * I.max())
    G = sample_points(m, 512, 3)
    ref = O.intensity(m, G)
    print("sampled rel L2", rel_l2(at(I, m, G), ref), "worst voxel", max_rel(at(I, m, G), ref))
    assert_parity(at(I, m, G), ref)
    assert_parity(I, I[::-1, ::-1, ::-1])


@pytest.mark.parametrize("mi", [0, 1, 2, 3])
def test_ensemble_members(mi):
    models = synth.ensemble(n_models=8)
    m = models[mi]
    say(f"ensemble member {mi}: {m.name}, box {m.count}")
    I = run_full(m)
    G = sample_points(m, 256, 40 + mi)
    ref = O.intensity(m, G)
    assert_parity(at(I, m, G), ref)


def test_compositional_filter_full_box():
    import torch
    m = synth.compositional(n=12, M=4, hmax=2)
    say("compositional 12^3 M=4, Lanczos m=2 on the full box")
    h = to_dsx(m)
    out = torch.empty(tuple(m.count), dtype=torch.float32, device="cuda")
    h.noise_filter(2, 1, out)
    torch.cuda.synchronize()
    ref = O.filtered_intensity(m, 2, 1)
    assert_parity(out.cpu().numpy(), ref)
    h.close()
