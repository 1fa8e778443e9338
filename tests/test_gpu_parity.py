"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Tolerance: relative L2 <= 1e-5 over every compared voxel (float32 FFT and
recombination, float64 Bragg points), the bar the path is built to.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests.helpers import assert_parity, max_rel, MAXTOL, desc_kwargs, gpu_filtered, gpu_intensity, rel_l2, to_dsx

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(msg):
    print(f"[gpu case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1809_07088_amd as dsx
    dsx.lib()
    yield


# ------------------------------------------------------------------ compositional, full grid

@pytest.mark.parametrize("M", [1, 4])
def test_compositional_simple_cubic_full_grid(M):
    m = synth.compositional(n=12, M=M, hmax=2)
    say(f"compositional n=12 M={M} box={m.count}")
    I = gpu_intensity(m)
    ref = O.intensity(m).reshape(m.count)
    print("rel L2", rel_l2(I, ref), "worst voxel", max_rel(I, ref))
    assert_parity(I, ref)
    if M == 1:   # Parseval on the GPU output: mean = c (1 - c)
        c = float(m.occ.astype(np.float64).mean())
        assert abs(I.astype(np.float64).mean() - c * (1 - c)) < 1e-6


@pytest.mark.parametrize("S,M", [(3, 2), (16, 3), (17, 2), (24, 1)])
def test_occupancy_bragg_points_across_site_counts(S, M):
    """Order-0 (occupancy) models: up to 16 sites take the lane-per-H form of the float64
    Bragg points, more sites the (site, monomial) form; both against the oracle on the whole
    box and at its Bragg points G = n H (the variance over configurations; 0 for M = 1)."""
    m = synth.random_model(440 + S, n=(3, 4, 3), S=S, M=M, order=0, with_disp=False)
    m.g0, m.count = (-6, -8, -7), (13, 17, 15)
    say(f"occupancy Bragg points S={S} M={M}")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count), 0).reshape(m.count)
    assert_parity(I, ref)
    G = O.grid_points(m.g0, m.count).reshape(m.count + (3,))
    at_h = np.all(G % np.asarray(m.n) == 0, axis=-1)
    assert at_h.sum() == 5 * 5 * 5
    scale = np.abs(ref).max()
    assert np.allclose(I[at_h], ref[at_h], rtol=1e-5, atol=1e-7 * scale)
    if M == 1:
        assert np.all(I[at_h] == 0.0)


# ------------------------------------------------------------------ displacive, every order

@pytest.mark.parametrize("order", list(range(0, 9)))
def test_random_model_every_order_full_box(order):
    m = synth.random_model(100 + order, n=(6, 5, 8), S=3, M=2, order=order)
    m.g0, m.count = (-7, -9, -10), (15, 13, 21)       # several zones, ragged on every axis
    say(f"random model order={order} n={m.n} box={m.count}")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count), order).reshape(m.count)
    print("rel L2", rel_l2(I, ref), "worst voxel", max_rel(I, ref))
    assert_parity(I, ref)


@pytest.mark.parametrize("n,order", [((256, 2, 3), 3), ((3, 256, 2), 3), ((2, 3, 256), 3),
                                     ((2, 256, 256), 0), ((3, 144, 250), 2)])
def test_edges_up_to_256(n, order):
    """Supercell edges up to 256 on every axis; planes of 256 x 256 and 144 x 250 exceed
    the LDS and take the row route (axis 3 per row pair, then axis 2 in place)."""
    m = synth.random_model(400 + sum(n), n=n, S=1 if order == 0 else 2, M=1, order=order,
                           with_disp=order > 0, sigma=0.03)
    m.g0 = tuple(-min(v + 1, 20) for v in n)
    m.count = tuple(min(2 * v + 3, 41) for v in n)
    say(f"edges n={n} order={order} box={m.count}")
    I = gpu_intensity(m)
    G = O.grid_points(m.g0, m.count)
    if len(G) > 6000:
        sel = np.random.default_rng(1).choice(len(G), 6000, replace=False)
        G = G[sel]
        got = I[tuple((G - np.asarray(m.g0)).T)]
    else:
        got = I.reshape(-1)
    assert_parity(got, O.intensity(m, G, order if order > 0 else None))


@pytest.mark.parametrize("order", [9, 12, 16])
def test_high_taylor_orders_tiny_cell(order):
    """Orders above 8 (class form, runs of at most 8 H3 per thread) up to the largest
    supported, 16, on a tiny cell with occupancies and two configurations."""
    m = synth.random_model(150 + order, n=(3, 4, 5), S=2, M=2, order=order, sigma=0.03)
    m.g0, m.count = (-4, -5, -6), (9, 11, 13)
    say(f"order {order} on n={m.n}")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count), order).reshape(m.count)
    assert_parity(I, ref)


def test_high_order_magnetic_debye_waller():
    m = synth.random_model(170, n=(3, 4, 3), S=2, M=1, kind=synth.MAGNETIC, mag_order=12, sigma=0.03,
                           cell=[5.0, 6.0, 7.0, 90.0, 97.0, 90.0])
    say("magnetic Debye-Waller at order 12")
    I = gpu_intensity(m)
    assert_parity(I, O.intensity(m, O.grid_points(m.g0, m.count)).reshape(m.count))


@pytest.mark.parametrize("n", [(7, 11, 9), (1, 4, 3), (5, 3, 1), (16, 2, 10),
                               (13, 26, 7), (49, 2, 7), (53, 1, 3), (2, 58, 3)])
def test_odd_prime_and_degenerate_edges(n):
    m = synth.random_model(200 + sum(n), n=n, S=2, M=1, order=3)
    m.g0 = tuple(-v - 1 for v in n)
    m.count = tuple(2 * v + 3 for v in n)
    say(f"edge n={n} box={m.count}")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count), 3).reshape(m.count)
    assert_parity(I, ref)


def test_box_smaller_than_supercell_without_bragg_points():
    m = synth.random_model(300, n=(8, 8, 8), S=2, M=2, order=2)
    m.g0, m.count = (3, 1, 2), (3, 4, 5)
    say("small box, no k = 0 point")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count), 2).reshape(m.count)
    assert_parity(I, ref)


def test_fcc_no_occupancy_shares_r3_classes():
    m = synth.displacive(n=8, M=3, order=6, hmax=2)
    say("fcc n=8 order 6 M=3")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count), 6).reshape(m.count)
    assert_parity(I, ref)
    assert np.allclose(I, I[::-1, ::-1, ::-1], rtol=1e-4, atol=1e-6 * np.abs(I).max())


# ------------------------------------------------------------------ magnetic

def test_magnetic_random_noncubic_full_box():
    m = synth.random_model(400, n=(4, 5, 6), S=3, M=2, kind=synth.MAGNETIC,
                           cell=[7.0, 8.0, 9.0, 80.0, 95.0, 100.0])
    m.g0, m.count = (-5, -6, -8), (11, 12, 17)
    say("magnetic random non-cubic")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count)).reshape(m.count)
    assert_parity(I, ref)


@pytest.mark.parametrize("r3s,M", [((0.0,), 1), ((0.0, 0.5), 2), ((0.0, 1 / 3, 2 / 3), 1), ((0.0, 0.25, 0.5, 0.75), 2),
                                   ((0.0, 1 / 6, 1 / 3, 0.5, 2 / 3, 5 / 6), 1)])
def test_magnetic_class_residue_sums(r3s, M):
    """Sites whose r3 lie on a 1/q grid: the row-staged magnetic form sums the r3 classes per
    residue of H3 mod q (unrolled up to four classes; six classes take level C per class)."""
    S = 2 * len(r3s)
    m = synth.random_model(410 + len(r3s), n=(6, 5, 6), S=S, M=M, kind=synth.MAGNETIC,
                           cell=[6.0, 6.5, 7.0, 90.0, 90.0, 90.0])
    m.frac[:, 2] = np.repeat(np.asarray(r3s), 2)      # two sites per class
    m.g0, m.count = (-7, -6, -13), (15, 13, 27)
    say(f"magnetic residue sums: {len(r3s)} classes, M={M}")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count)).reshape(m.count)
    assert_parity(I, ref)


ORTHO = [6.0, 6.5, 7.0, 90.0, 90.0, 90.0]
TRIC = [6.0, 6.5, 7.0, 84.0, 97.0, 103.0]


@pytest.mark.parametrize("r2s,M,cell,q1", [((0.0,), 1, ORTHO, 1), ((0.0, 0.5), 2, ORTHO, 2),
                                           ((0.0, 0.25, 0.5, 0.75), 1, ORTHO, 2), ((0.0, 1 / 3, 2 / 3), 2, TRIC, 0),
                                           ((0.0, 0.25, 0.5, 0.75), 1, TRIC, 4)])
def test_magnetic_row_residues(r2s, M, cell, q1):
    """Sites whose r2 lie on a 1/q grid: rows of a block whose H2 agree mod q have the same
    site phases, so the row-staged magnetic form stages q rows and maps the others onto
    them (nine rows per column here).  With r1 on a 1/q1 grid and one configuration a block
    serves up to four G1 planes of one H1 residue (q1 = 0: random r1, one plane a block).
    On the orthogonal cell b* is orthogonal to a* and c* and the form factor is split into
    a per-column and a per-row part."""
    S = 2 * len(r2s)
    m = synth.random_model(420 + 3 * len(r2s) + M, n=(2, 3, 5), S=S, M=M, kind=synth.MAGNETIC, cell=cell)
    m.frac[:, 1] = np.repeat(np.asarray(r2s), 2)      # two sites per r2 value
    if q1:
        m.frac[:, 0] = (np.arange(S) % q1) / q1
    m.g0, m.count = (-10, -13, -8), (21, 27, 17)
    say(f"magnetic row residues: q2={len(r2s)}, q1={q1}, M={M}, cell angles {cell[3:]}")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count)).reshape(m.count)
    assert_parity(I, ref)


def test_magnetic_per_site_form_factors():
    m = synth.random_model(401, n=(4, 4, 5), S=3, M=1, kind=synth.MAGNETIC,
                           cell=[6.0, 6.0, 6.0, 90.0, 90.0, 90.0])
    m.ff = np.array([[0.4, 20, 0.5, 7, 0.1, 2, 0.0], [0.3, 10, 0.6, 3, 0.1, 1, 0.0],
                     [1.0, 5, 0, 0, 0, 0, 0.0]])
    m.g0, m.count = (-6, -5, -7), (13, 11, 15)
    say("magnetic per-site form factors")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count)).reshape(m.count)
    assert_parity(I, ref)


# ------------------------------------------------------------------ Lanczos filter

@pytest.mark.parametrize("lm,s", [(2, 1), (4, 1), (2, 2), (3, 3)])
def test_lanczos_filter_matches_direct_window(lm, s):
    m = synth.random_model(500 + lm, n=(5, 6, 4), S=2, M=2, order=2)
    m.g0, m.count = (-4, -5, -3), (9, 11, 8)
    say(f"lanczos m={lm} s={s}")
    out = gpu_filtered(m, lm, s)
    ref = O.filtered_intensity(m, lm, s, order=2)
    assert out.shape == ref.shape
    assert_parity(out, ref)


# ------------------------------------------------------------------ ABI behaviour on the GPU

def test_host_and_device_outputs_identical_and_deterministic():
    m = synth.random_model(600, n=(6, 6, 6), S=2, M=2, order=4)
    say("host vs device output, determinism")
    a = gpu_intensity(m, device=True)
    b = gpu_intensity(m, device=False)
    c = gpu_intensity(m, device=True)
    assert np.array_equal(a, c)
    assert np.array_equal(a, b)


def test_state_errors():
    import torch
    import paper_1809_07088_amd as dsx
    m = synth.random_model(601, n=(4, 4, 4), S=1, M=2, order=1)
    say("state errors")
    h = dsx.Model(**desc_kwargs(m))
    out = torch.empty(tuple(m.count), device="cuda")
    with pytest.raises(dsx.DsxError) as e:
        h.compute_intensity(out)
    assert e.value.status == dsx.ERR_STATE
    h.set_sites(0, torch.from_numpy(m.occ[0]).cuda(), torch.from_numpy(m.disp[0]).cuda())
    with pytest.raises(dsx.DsxError) as e:
        h.set_sites(2, torch.from_numpy(m.occ[0]).cuda(), torch.from_numpy(m.disp[0]).cuda())
    assert e.value.status == dsx.ERR_ARG
    with pytest.raises(dsx.DsxError) as e:
        h.set_sites(1, torch.from_numpy(m.occ[1]).cuda(), None)
    assert e.value.status == dsx.ERR_ARG
    h.set_sites(1, torch.from_numpy(m.occ[1]).cuda(), torch.from_numpy(m.disp[1]).cuda())
    with pytest.raises(dsx.DsxError) as e:
        h.compute_intensity(out)          # no grid yet
    assert e.value.status == dsx.ERR_STATE
    h.set_grid(m.g0, m.count)
    with pytest.raises(dsx.DsxError) as e:
        h.noise_filter(1, 1, out)
    assert e.value.status == dsx.ERR_ARG
    h.compute_intensity(out)
    torch.cuda.synchronize()
    ref = O.intensity(m).reshape(m.count)
    assert_parity(out.cpu().numpy(), ref)
    h.close()


def test_set_sites_marks_spectra_stale():
    import torch
    m = synth.random_model(602, n=(5, 4, 6), S=2, M=1, order=2)
    m2 = synth.random_model(603, n=(5, 4, 6), S=2, M=1, order=2)
    m2.frac, m2.b = m.frac, m.b
    say("set_sites invalidates spectra")
    h = to_dsx(m)
    out = torch.empty(tuple(m.count), device="cuda")
    h.compute_intensity(out)
    h.set_sites(0, torch.from_numpy(m2.occ[0]).cuda(), torch.from_numpy(m2.disp[0]).cuda())
    h.compute_intensity(out)
    torch.cuda.synchronize()
    assert_parity(out.cpu().numpy(), O.intensity(m2).reshape(m.count))
    h.close()


# ------------------------------------------------------------------ recombination forms

def _half_r2_model(seed, order, M, parity):
    """Four sites whose r2 are multiples of 1/2 and which share two r3 classes (the
    folded form applies); r3 are halves too when `parity`."""
    m = synth.random_model(seed, n=(6, 4, 6), S=4, M=M, order=order)
    r3 = (0.0, 0.5) if parity else (0.13, 0.71)
    m.frac = np.array([[0.0, 0.0, r3[0]], [0.31, 0.5, r3[0]], [0.5, 0.0, r3[1]], [0.77, 1.5, r3[1]]])
    m.g0, m.count = (-7, -5, -6), (15, 11, 13)
    return m


@pytest.mark.parametrize("variant", ["0", "1", "2", "3"])
@pytest.mark.parametrize("order,M,parity", [(8, 1, True), (5, 2, True), (3, 1, False), (6, 2, False),
                                            (0, 2, True)])
def test_every_recombination_form(monkeypatch, variant, order, M, parity):
    """Variant 0: the default (folded where it applies), 1: the multi-configuration form,
    2: the class form, 3: unfolded."""
    monkeypatch.setenv("DSX_RECOMBINE_VARIANT", variant)
    m = _half_r2_model(700 + order, order, M, parity)
    say(f"recombination form variant={variant} order={order} M={M} parity={parity}")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count), order).reshape(m.count)
    assert_parity(I, ref)


def _half_r2_long_k3(seed, n3, order, M, parity):
    m = _half_r2_model(seed, order, M, parity)
    small = synth.random_model(seed, n=(4, 4, n3), S=4, M=M, order=order)
    small.frac = m.frac
    return small


@pytest.mark.parametrize("variant", ["0", "1", "2", "4"])
@pytest.mark.parametrize("n3,order,M,parity", [(16, 8, 1, True), (17, 5, 2, True), (20, 3, 1, False),
                                               (33, 4, 2, False)])
def test_folded_k3_slices(monkeypatch, variant, n3, order, M, parity):
    """Supercells with n3 >= 16 cut the folded blocks into two k3 slices (odd n3: of
    unequal length); variant 4 keeps whole blocks.  The box is ragged at both ends."""
    monkeypatch.setenv("DSX_RECOMBINE_VARIANT", variant)
    m = _half_r2_long_k3(1000 + n3, n3, order, M, parity)
    m.g0, m.count = (-5, -4, -(n3 + 3)), (9, 9, 2 * n3 + 7)
    say(f"folded k3 slices variant={variant} n3={n3} order={order} M={M} parity={parity}")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count), order).reshape(m.count)
    assert_parity(I, ref)


@pytest.mark.parametrize("lm", [0, 2])
def test_folded_k3_slices_symmetric_box(lm):
    """Sliced folded blocks on a box symmetric about G = 0 (Friedel mirror writes) and,
    through the filter, on its half-stored grown box."""
    m = _half_r2_long_k3(1100 + lm, 16, 4, 2, True)
    m.g0, m.count = (-9, -8, -21), (19, 17, 43)
    say(f"folded k3 slices symmetric box lanczos m={lm}")
    if lm == 0:
        out = gpu_intensity(m)
        ref = O.intensity(m, O.grid_points(m.g0, m.count), 4).reshape(m.count)
    else:
        out = gpu_filtered(m, lm, 1)
        ref = O.filtered_intensity(m, lm, 1, order=4)
    assert_parity(out, ref)


@pytest.mark.parametrize("n,kind,order", [((16, 8, 32), synth.NUCLEAR, 3), ((8, 32, 16), synth.NUCLEAR, 0),
                                          ((8, 16, 8), synth.MAGNETIC, 0), ((32, 32, 8), synth.NUCLEAR, 5),
                                          ((32, 16, 32), synth.NUCLEAR, 1), ((16, 32, 16), synth.MAGNETIC, 0),
                                          ((8, 32, 32), synth.NUCLEAR, 0)])
def test_power_of_two_edges_register_transforms(n, kind, order):
    """Edges 8, 16, 32 take the register-resident transforms (occupancy, Taylor
    p-runs and spin components all pass through them)."""
    m = synth.random_model(800 + sum(n), n=n, S=2, M=2, order=order, kind=kind,
                           cell=None if kind == synth.NUCLEAR else [6.0, 7.0, 8.0, 90.0, 90.0, 90.0])
    m.g0 = tuple(-(v // 2) - 1 for v in n)      # every residue k, ragged at both ends
    m.count = tuple(v + 3 for v in n)
    say(f"register transforms n={n} kind={kind} order={order}")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count), order if kind == synth.NUCLEAR else None).reshape(m.count)
    assert_parity(I, ref)


def test_set_sites_async_matches_set_sites():
    import torch
    m = synth.random_model(900, n=(6, 8, 5), S=3, M=2, order=4)
    m2 = synth.random_model(901, n=(6, 8, 5), S=3, M=2, order=4)
    say("set_sites_async")
    h = to_dsx(m)
    out = torch.empty(tuple(m.count), device="cuda")
    h.compute_intensity(out)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for c in range(m.n_configs):
            h.set_sites_async(c, torch.from_numpy(m2.occ[c]).cuda(), torch.from_numpy(m2.disp[c]).cuda(), stream=s)
    h.compute_intensity(out)                       # the default stream: ordered after the copies
    torch.cuda.synchronize()
    m2.frac, m2.b = m.frac, m.b
    ref = gpu_intensity(m2)
    assert np.array_equal(out.cpu().numpy(), ref)
    h.close()


@pytest.mark.parametrize("lm,s", [(2, 1), (3, 1), (4, 1), (2, 2)])
def test_lanczos_symmetric_box_half_storage(lm, s):
    """On a box symmetric about G = 0 the grown box is stored as its half G1 <= 0 and
    (s = 1) the filter computes half the planes and writes their mirrors."""
    m = synth.random_model(950 + lm + s, n=(6, 4, 8), S=3, M=2, order=3)
    m.g0, m.count = (-7, -6, -9), (15, 13, 19)
    say(f"lanczos symmetric box m={lm} s={s}")
    out = gpu_filtered(m, lm, s)
    ref = O.filtered_intensity(m, lm, s, order=3)
    assert_parity(out, ref)


# ------------------------------------------------------------------ cutoff variant, arbitrary Q

@pytest.mark.parametrize("m,mp,s", [(2, 4, 1), (2, 3, 1), (3, 4, 1), (2, 4, 2), (4, 3, 1)])
def test_noise_filter_cutoff_variant(m, mp, s):
    """The m' cutoff modification (r_cut = (1 - 1/m)/m', window m m'/2): w = 3, 4 take
    the register-ring filter, w = 6 and s > 1 the general one."""
    model = synth.random_model(1200 + 10 * m + mp + s, n=(5, 6, 4), S=2, M=2, order=2)
    say(f"noise_filter_cutoff m={m} m'={mp} s={s}")
    out = gpu_filtered(model, m, s, mprime=mp)
    ref = O.filtered_intensity(model, m, s, order=2, mprime=mp)
    assert_parity(out, ref)


def test_noise_filter_cutoff_symmetric_box():
    model = synth.random_model(1250, n=(6, 4, 8), S=3, M=2, order=3)
    model.g0, model.count = (-7, -6, -9), (15, 13, 19)
    say("noise_filter_cutoff symmetric box m=2 m'=4")
    out = gpu_filtered(model, 2, 1, mprime=4)
    ref = O.filtered_intensity(model, 2, 1, order=3, mprime=4)
    assert_parity(out, ref)


def _hhl_points(n, hmax, npts):
    """Q of an (h h l) plane in units of the supercell Bragg grid (G_a = n_a h_a)."""
    h, l = np.meshgrid(np.linspace(-hmax, hmax, npts), np.linspace(-hmax, hmax, npts), indexing="ij")
    hkl = np.stack([h, h, l], -1).reshape(-1, 3)
    return hkl * np.asarray(n, dtype=np.float64)


@pytest.mark.parametrize("m,mp", [(2, 2), (2, 4), (3, 2)])
def test_filter_points_on_an_hhl_plane(m, mp):
    import torch
    import paper_1809_07088_amd as dsx
    model = synth.random_model(1300 + 10 * m + mp, n=(5, 5, 4), S=2, M=2, order=3)
    Q = _hhl_points(model.n, 1.3, 23)
    say(f"filter_points (h h l) m={m} m'={mp}")
    h = to_dsx(model)
    dev = torch.empty(len(Q), dtype=torch.float32, device="cuda")
    h.filter_points(m, Q, dev, mprime=mp)
    host = np.empty(len(Q), dtype=np.float32)
    h.filter_points(m, Q, host, mprime=mp)
    assert np.array_equal(dev.cpu().numpy(), host)
    ref = O.filtered_points(model, m, Q, order=3, mprime=mp)
    assert_parity(host, ref)
    # grid points agree with the box filter of the same window
    if mp == 2:
        box = np.empty(tuple(model.count), dtype=np.float32)
        h.noise_filter(m, 1, box)
        G = O.grid_points(model.g0, model.count).astype(np.float64)
        at = np.empty(len(G), dtype=np.float32)
        h.filter_points(m, G, at)
        assert_parity(at, box.reshape(-1))
    with pytest.raises(dsx.DsxError) as e:
        h.filter_points(m, np.array([[0.5, np.nan, 1.0]]), host[:1])
    assert e.value.status == dsx.ERR_ARG
    with pytest.raises(dsx.DsxError) as e:
        h.filter_points(3, Q, host, mprime=3)       # m m' odd
    assert e.value.status == dsx.ERR_ARG
    h.close()


# ------------------------------------------------------------------ split sites

@pytest.mark.parametrize("seed,K,occ", [(40, 2, True), (41, 3, False), (42, 4, True)])
def test_split_sites_on_the_compositional_path(seed, K, occ):
    """Discrete displacements mapped to split sites (dsx_split_sites) and evaluated by
    the compositional kernels equal the exact-exponential displacive intensity."""
    from tests.helpers import discrete_displacement_model, split_model
    m = discrete_displacement_model(seed, n=(4, 6, 5), S=2, M=2, K=K, with_occ=occ)
    if not occ:
        m.occ = None
    s = split_model(m)
    say(f"split sites seed={seed} K={K} occ={occ} -> {s.n_sites} sites")
    I = gpu_intensity(s)
    ref = O.intensity(m, O.grid_points(m.g0, m.count), -1).reshape(m.count)
    assert_parity(I, ref)


# ------------------------------------------------------------------ spherical cutoff

@pytest.mark.parametrize("m,s", [(2, 1), (3, 1), (2, 2), (4, 1)])
def test_noise_filter_spherical_cutoff(m, s):
    """The spherically symmetric cutoff W_r (non-separable: the (2m)^3 stencil), on a
    non-cubic cell so that the metric enters."""
    model = synth.random_model(1400 + 10 * m + s, n=(5, 6, 4), S=2, M=2, order=2,
                               cell=[4.1, 5.3, 6.2, 84.0, 97.0, 101.0])
    say(f"noise_filter_spherical m={m} s={s}")
    h = to_dsx(model)
    out = np.empty(tuple(s * c for c in model.count), dtype=np.float32)
    h.noise_filter_spherical(m, s, out)
    h.close()
    ref = O.filtered_intensity_spherical(model, m, s, order=2)
    assert_parity(out, ref)


def test_noise_filter_spherical_symmetric_box():
    model = synth.random_model(1450, n=(6, 4, 8), S=3, M=2, order=3)
    model.g0, model.count = (-7, -6, -9), (15, 13, 19)
    say("noise_filter_spherical symmetric box (half-stored grown box)")
    h = to_dsx(model)
    import torch
    out = torch.empty(tuple(model.count), dtype=torch.float32, device="cuda")
    h.noise_filter_spherical(2, 1, out)
    torch.cuda.synchronize()
    h.close()
    ref = O.filtered_intensity_spherical(model, 2, 1, order=3)
    assert_parity(out.cpu().numpy(), ref)


# ------------------------------------------------------------------ magnetic Debye-Waller

@pytest.mark.parametrize("order,M,share_r3,occ", [(1, 2, False, True), (3, 1, True, True), (6, 2, True, False)])
def test_magnetic_debye_waller_factor_eq_dw(order, M, share_r3, occ):
    """T_mu(G) of Eq. dw from the model's own displacements (the order-N mean of
    e^{i G.u} over each site's occupied atoms and configurations) in Eq. mag_sf, through
    the recombination (each site at level C on its own) and the FP64 Bragg points."""
    m = synth.random_model(1500 + order, n=(4, 5, 6), S=3, M=M, kind=synth.MAGNETIC, mag_order=order,
                           with_occ=occ, sigma=0.04, cell=[5.0, 6.0, 7.0, 88.0, 94.0, 101.0])
    if share_r3:
        m.frac[:, 2] = [0.25, 0.25, 0.6]
    say(f"magnetic Debye-Waller order={order} M={M} share_r3={share_r3} occ={occ}")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count)).reshape(m.count)
    assert_parity(I, ref)
    assert max_rel(I, ref) <= MAXTOL


def test_magnetic_pyrochlore_with_displacements():
    """The pyrochlore spin workload at n = 6 with correlated displacements, order 4."""
    m = synth.magnetic(n=6, hmax=2)
    m.disp = synth.correlated_displacements(synth.rng_for(3, 0, 7), 1, m.n_sites, m.n, sigma=0.05, width=1.0)
    m.order = 4
    say("magnetic pyrochlore n=6 order-4 Debye-Waller")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count)).reshape(m.count)
    assert_parity(I, ref)
    assert max_rel(I, ref) <= MAXTOL


# ------------------------------------------------------------------ X-ray scattering factors

@pytest.mark.parametrize("order,M,share_r3", [(3, 2, False), (0, 2, True), (5, 1, True)])
def test_nuclear_q_dependent_scattering_factors(order, M, share_r3):
    """Nuclear sites with |Q|-dependent scattering factors (X-ray f_j(|Q|)): the class
    form with the class's factor at level C, and the FP64 Bragg points; sites sharing
    r3 but not f stay in different classes."""
    m = synth.random_model(1600 + order, n=(4, 5, 6), S=3, M=M, order=order, with_disp=order > 0,
                           cell=[4.3, 5.2, 6.1, 88.0, 93.0, 99.0])
    if share_r3:
        m.frac[:, 2] = [0.3, 0.3, 0.75]
    m.ff = np.array([[2.1, 3.0, 1.2, 0.7, 0.4, 9.0, 0.3],
                     [1.5, 1.1, 0.9, 4.0, 0.2, 0.5, 0.8],
                     [0.6, 2.5, 1.8, 0.3, 0.9, 6.0, 0.1]])
    say(f"nuclear scattering factors order={order} M={M} share_r3={share_r3}")
    I = gpu_intensity(m)
    ref = O.intensity(m, O.grid_points(m.g0, m.count), order if order > 0 else None).reshape(m.count)
    assert_parity(I, ref)


def test_filter_variant_argument_errors():
    import paper_1809_07088_amd as dsx
    model = synth.random_model(1700, n=(4, 4, 4), S=1, M=1, order=1)
    say("filter variant argument errors")
    h = to_dsx(model)
    out = np.empty(tuple(model.count), dtype=np.float32)
    for call, status in [(lambda: h.noise_filter_cutoff(3, 3, 1, out), dsx.ERR_ARG),        # m m' odd
                         (lambda: h.noise_filter_cutoff(2, 1, 1, out), dsx.ERR_ARG),        # m' < 2
                         (lambda: h.noise_filter_cutoff(8, 6, 1, out), dsx.ERR_UNSUPPORTED),  # w = 24
                         (lambda: h.noise_filter_spherical(5, 1, out), dsx.ERR_UNSUPPORTED),
                         (lambda: h.noise_filter_spherical(1, 1, out), dsx.ERR_ARG),
                         (lambda: h.filter_points(2, np.zeros((1, 3)), out[:1, 0, 0].copy(), mprime=20),
                          dsx.ERR_UNSUPPORTED)]:                                          # w = 20 > 8
        with pytest.raises(dsx.DsxError) as e:
            call()
        assert e.value.status == status
    h.close()
