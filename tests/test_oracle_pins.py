"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: printed values,
closed forms, exact invariances, the Taylor remainder bound, an independent
brute-force formula (pair double sum), or an independent algorithm (the paper's
FFT route against the direct sum).  All run on the CPU.
"""
import itertools
import math
import os

import numpy as np
import pytest

import synth
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def golden():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                key, val = line.split()[:2]
                vals[key] = float(val)
    return vals


# --------------------------------------------------------------------------- printed values

def test_printed_constants_and_counts():
    g = golden()
    assert O.MAG_CONSTANT_BARN == g["mag_constant_barn"]
    for n in (0, 1, 2, 5):
        assert sum(1 for t in O.monomials(n) if sum(t) == n) == g[f"ffts_per_order_{n}"]
    # fully occupied sites: the constant monomial needs no transform
    assert len(O.monomials(5)) - 1 == g["ffts_fifth_order_total"]


def test_multiset_regrouping_of_ordered_tuples():
    # Eq. gu_expansion sums over ordered tuples; the oracle's FFT route sums over
    # multisets with multinomial weights. Same value for any g, u.
    assert O.ordered_tuple_weight_check(6, np.array([0.7, -1.3, 2.1])) < 1e-12


# --------------------------------------------------------------------------- P1 zero disorder

@pytest.mark.parametrize("n", [4, 32])
def test_zero_disorder_only_bragg_closed_form(n):
    m = synth.displacive(n=n, order=0, hmax=1)
    m.disp = None
    H = np.array([[0, 0, 0], [1, 1, 1], [1, 0, 0], [0, 2, 0], [1, 1, 0], [2, -1, 1]])
    off = np.array([[1, 0, 0], [3, 5, 7], [n - 1, 1, 2], [-5, 2, n + 3]])
    G = np.concatenate([H * n, off])
    F = O.structure_factor(m, G, order=-1)[0]
    Itot = np.abs(F) ** 2 / O.norm_N(m)
    # Eq. total_sf with u = 0, delta = 1: F(nH) = n^3 sum_mu b_mu e^{2 pi i H.r_mu}, 0 elsewhere
    S = np.array([np.sum(m.b * np.exp(2j * np.pi * (m.frac @ h))) for h in H])
    expect = (n ** 3 / m.n_sites) * np.abs(S) ** 2
    assert np.allclose(Itot[:len(H)], expect, rtol=1e-10, atol=1e-9)
    assert np.max(Itot[len(H):]) < 1e-18 * n ** 3
    if n == 32:   # unmixed / mixed hkl of the fcc basis with b = 1, .7, .7, .7 (closed form)
        assert abs(Itot[1] - 78725.12) < 1e-5 and abs(Itot[2] - 737.28) < 1e-6
    Id = O.intensity(m, G, order=-1)
    assert np.max(np.abs(Id)) < 1e-9


# --------------------------------------------------------------------------- P2 Parseval

def test_parseval_compositional_full_grid():
    m = synth.compositional(n=12, M=1, hmax=2)
    I = O.intensity(m).reshape(m.count)
    cbar = float(m.occ.astype(np.float64).mean())
    assert abs(I.mean() - cbar * (1 - cbar)) < 1e-12
    # every 12^3 zone is identical (one site at the origin, no displacements)
    z = I.reshape(4, 12, 4, 12, 4, 12)
    assert np.allclose(z, z[:1, :, :1, :, :1, :], rtol=1e-10, atol=1e-12)


# --------------------------------------------------------------------------- P3 Friedel

@pytest.mark.parametrize("order", [-1, 0, 3, 6])
def test_friedel_nuclear(order):
    m = synth.random_model(3, n=(3, 4, 5), S=3, M=2, order=max(order, 0))
    G = O.grid_points(m.g0, m.count)
    sel = np.random.default_rng(0).choice(len(G), 300, replace=False)
    I1 = O.intensity(m, G[sel], order)
    I2 = O.intensity(m, -G[sel], order)
    assert np.allclose(I1, I2, rtol=1e-10, atol=1e-12)


def test_friedel_magnetic():
    m = synth.random_model(4, n=(3, 3, 4), S=3, M=2, kind=synth.MAGNETIC,
                           cell=[7.0, 8.0, 9.0, 80.0, 95.0, 100.0])
    G = O.grid_points(m.g0, m.count)[::7]
    assert np.allclose(O.intensity(m, G), O.intensity(m, -G), rtol=1e-10, atol=1e-14)


# --------------------------------------------------------------------------- P4 invariances

def test_invariance_shift_roll_permutation():
    m = synth.random_model(5, n=(4, 3, 5), S=3, M=2, order=4)
    G = O.grid_points(m.g0, m.count)[::5]
    I0 = O.intensity(m, G)
    # global shift of every average site position
    m2 = synth.random_model(5, n=(4, 3, 5), S=3, M=2, order=4)
    m2.frac = m2.frac + np.array([0.123, -0.31, 0.77])
    assert np.allclose(O.intensity(m2, G), I0, rtol=1e-10, atol=1e-12)
    # cyclic shift of lattice points in one configuration
    m3 = synth.random_model(5, n=(4, 3, 5), S=3, M=2, order=4)
    m3.occ[1] = np.roll(m3.occ[1], (1, 2, 3), axis=(1, 2, 3))
    m3.disp[1] = np.roll(m3.disp[1], (1, 2, 3), axis=(1, 2, 3))
    assert np.allclose(O.intensity(m3, G), I0, rtol=1e-10, atol=1e-12)
    # permutation of the site order
    m4 = synth.random_model(5, n=(4, 3, 5), S=3, M=2, order=4)
    p = [2, 0, 1]
    m4.frac, m4.b = m4.frac[p], m4.b[p]
    m4.occ, m4.disp = m4.occ[:, p], m4.disp[:, p]
    assert np.allclose(O.intensity(m4, G), I0, rtol=1e-10, atol=1e-12)


def test_tiling_doubles_lattice():
    m = synth.random_model(6, n=(2, 3, 2), S=2, M=2, order=3)
    big = synth.random_model(6, n=(4, 6, 4), S=2, M=2, order=3)
    big.frac, big.b = m.frac, m.b
    big.occ = np.tile(m.occ, (1, 1, 2, 2, 2))
    big.disp = np.tile(m.disp, (1, 1, 2, 2, 2, 1))
    G = O.grid_points((-3, -4, -3), (7, 9, 7))
    assert np.allclose(O.intensity(big, 2 * G), 8 * O.intensity(m, G), rtol=1e-10, atol=1e-12)
    odd = 2 * G + np.array([1, 0, 0])
    assert np.max(np.abs(O.intensity(big, odd[::3]))) < 1e-12


# --------------------------------------------------------------------------- P5 Taylor

def test_taylor_remainder_bound_and_convergence():
    m = synth.random_model(7, n=(3, 3, 3), S=2, M=2, order=8, sigma=0.02)
    G = O.grid_points(m.g0, m.count)[::3]
    Fx = O.structure_factor(m, G, order=-1)
    g = G / np.array(m.n)
    # per-atom |2 pi g.u| and weights |b delta|
    x = 2 * np.pi * np.einsum("ga,msijka->msijkg", g, m.disp.astype(np.float64))
    w = np.abs(m.b[None, :, None, None, None] * m.occ.astype(np.float64))
    errs = []
    for N in range(0, 9):
        FN = O.structure_factor(m, G, order=N)
        bound = np.einsum("msijk,msijkg->mg", w, np.abs(x) ** (N + 1)) / math.factorial(N + 1)
        assert np.all(np.abs(FN - Fx) <= bound * (1 + 1e-9) + 1e-12)
        errs.append(np.max(np.abs(FN - Fx)))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))
    assert errs[-1] < 1e-4 * errs[0] and errs[-1] < 1e-5 * np.max(np.abs(Fx)) * 10


# --------------------------------------------------------------------------- P7 magnetic

def test_magnetic_form_factor_and_projection():
    assert abs(O.magnetic_form_factor(synth.MAG_FF, 0.0) - 1.0) < 1e-15
    m = synth.random_model(8, n=(3, 3, 3), S=2, M=1, kind=synth.MAGNETIC,
                           cell=[5.0, 6.0, 7.0, 90.0, 100.0, 90.0])
    G = O.grid_points(m.g0, m.count)[::4]
    Fs = O.structure_factor_magnetic_sites(m, G)
    Fp = O.magnetic_perp(m, G, Fs)
    q = np.linalg.norm(O.q_cartesian(m, G), axis=-1)
    f = np.stack([O.magnetic_form_factor(m.ff[mu], q / (4 * np.pi)) for mu in range(m.n_sites)], -1)
    F = np.einsum("gs,mgsc->mgc", f, Fs)
    assert np.all(np.sum(np.abs(Fp) ** 2, -1) <= np.sum(np.abs(F) ** 2, -1) * (1 + 1e-12) + 1e-15)
    # F_perp is orthogonal to Q
    Q = O.q_cartesian(m, G)
    assert np.max(np.abs(np.einsum("gc,mgc->mg", Q, Fp))) < 1e-9


def test_magnetic_ising_along_x_matches_scalar_route():
    # moments +-x: |F_perp|^2 = (1 - Ghat_x^2) |F_x|^2, F_x the scalar sum with weights +-1
    m = synth.random_model(9, n=(3, 4, 3), S=2, M=2, kind=synth.MAGNETIC,
                           cell=[4.0, 4.5, 5.0, 90.0, 90.0, 90.0])
    sgn = np.where(np.random.default_rng(3).random(m.spin.shape[:-1]) < 0.5, -1.0, 1.0)
    m.occ = None
    m.spin = np.zeros_like(m.spin)
    m.spin[..., 0] = sgn
    m.ff = np.tile(np.array([0, 0, 0, 0, 0, 0, 1.0]), (m.n_sites, 1))   # f = 1
    G = O.grid_points(m.g0, m.count)[::3]
    Imag = O.intensity(m, G)
    nuc = synth.Model(cell=m.cell, n=m.n, frac=m.frac, b=m.b, occ=sgn.astype(np.float32))
    Fx = O.structure_factor(nuc, G, order=-1)
    Q = O.q_cartesian(m, G)
    qn = np.linalg.norm(Q, axis=-1)
    with np.errstate(invalid="ignore", divide="ignore"):
        gx2 = np.where(qn > 0, (Q[:, 0] / qn) ** 2, 1.0)
    Fperp = np.sqrt(1 - gx2)[None] * Fx
    expect = O.MAG_CONSTANT_BARN * O.bragg_diffuse(Fperp, G, m.n, O.norm_N(m))
    assert np.allclose(Imag, expect, rtol=1e-10, atol=1e-14)


def test_magnetic_collinear_z_zero_on_00l():
    m = synth.random_model(10, n=(3, 3, 4), S=2, M=1, kind=synth.MAGNETIC)
    m.spin = np.zeros_like(m.spin)
    m.spin[..., 2] = np.where(np.random.default_rng(1).random(m.spin.shape[:-1]) < .5, -1, 1)
    G = np.array([[0, 0, l] for l in range(-9, 10)])
    assert np.max(np.abs(O.intensity(m, G))) < 1e-14


# --------------------------------------------------------------------------- P8 Lanczos

def _sep_lanczos(I_ext, e0, m, s, q0, qcount):
    """Independent separable evaluation: three 1D normalised passes (Sec. V.B)."""
    rcut = 0.5 * (1 - 1 / m)

    def w(d):
        d = np.asarray(d, float)
        out = 2 * rcut * np.sinc(2 * rcut * d) * np.sinc(d / m)   # np.sinc(x) = sin(pi x)/(pi x)
        return np.where(np.abs(d) < m, out, 0.0)

    X = np.asarray(I_ext, float)
    for ax in range(3):
        Q = q0[ax] + np.arange(qcount[ax]) / s
        fl = np.floor(Q).astype(int)
        rows = []
        for qi, Qv in enumerate(Q):
            Gs = np.arange(fl[qi] - m + 1, fl[qi] + m + 1)
            ww = w(Qv - Gs)
            idx = Gs - e0[ax]
            rows.append(np.tensordot(ww / ww.sum(), np.take(X, idx, axis=ax), axes=([0], [ax])))
        X = np.moveaxis(np.stack(rows), 0, ax)
    return X


@pytest.mark.parametrize("m,s", [(2, 1), (4, 1), (2, 3), (3, 2)])
def test_lanczos_direct_equals_separable_and_keeps_constants(m, s):
    rng = np.random.default_rng(m * 10 + s)
    e0 = np.array([-7, -5, -6])
    I_ext = rng.random((17, 14, 15))
    q0 = e0 + m
    qc = [(17 - 2 * m) * s - s + 1, (14 - 2 * m) * s - s + 1, (15 - 2 * m) * s - s + 1]
    qc = [max(1, (e - 2 * m - 1) * s) for e in (17, 14, 15)]
    d = O.lanczos(I_ext, e0, m, s, q0, qc)
    sep = _sep_lanczos(I_ext, e0, m, s, q0, qc)
    assert np.allclose(d, sep, rtol=1e-12, atol=1e-13)
    c = O.lanczos(np.full_like(I_ext, 3.25), e0, m, s, q0, qc)
    assert np.allclose(c, 3.25, rtol=1e-13)


def test_lanczos_m2_weights_closed_form():
    # impulse response on the G grid: neighbours weighted by (2/pi)^2 per axis, normalised
    e0 = np.array([-3, -3, -3])
    I = np.zeros((7, 7, 7))
    I[3, 3, 3] = 1.0
    out = O.lanczos(I, e0, 2, 1, [-1, -1, -1], [3, 3, 3])
    w1 = (2 / np.pi) ** 2
    line = np.array([w1, 1.0, w1]) / (1 + 2 * w1)
    assert np.allclose(out, np.einsum("i,j,k->ijk", line[::-1], line[::-1], line[::-1]), atol=1e-15)
    assert abs(w1 - 0.405285) < 1e-6


# ------------------------------------------------- P8' cutoff modification, arbitrary Q

def _cosine_response(m, mp, dr):
    """Filter I(G) = 1 + cos(2 pi G1 dr) (one real-space separation dr along axis 1)
    and read the attenuation of the cosine at Q = 0."""
    w = O.window_halfwidth(m, mp)
    e0 = np.array([-w - 2, -w - 2, -w - 2])
    cnt = 2 * w + 5
    G1 = e0[0] + np.arange(cnt)
    I = np.broadcast_to((1.0 + np.cos(2 * np.pi * G1 * dr))[:, None, None], (cnt, cnt, cnt))
    out = O.lanczos(I, e0, m, 1, [0, 0, 0], [1, 1, 1], mp)
    return float(out[0, 0, 0]) - 1.0


@pytest.mark.parametrize("m,mp", [(2, 4), (3, 4), (2, 3), (4, 3)])
def test_cutoff_variant_reaches_zero_at_one_over_mprime(m, mp):
    """The m' modification (Sec. V.B): the real-space cutoff of the filter reaches 0
    at |dr| = 1/m' instead of 1/2, and stays near 1 at short range."""
    assert _cosine_response(m, mp, 0.02) > 0.95
    for dr in (1 / mp + 0.06, 1 / mp + 0.12, 0.5):
        assert abs(_cosine_response(m, mp, dr)) < 0.03
    # the plain filter (m' = 2) still passes a large part of a separation 1/m' + 0.06
    assert _cosine_response(m, 2, 1 / mp + 0.06) > 0.1


def test_cutoff_variant_m2_is_close_to_the_triangle():
    # m = 2: the idealized cutoff is the triangle 1 - m'|dr| for |dr| < 1/m'
    for mp in (3, 4):
        half = _cosine_response(2, mp, 0.5 / mp)
        assert 0.4 < half < 0.7


def test_points_match_the_grid_filter_and_are_mirror_symmetric():
    rng = np.random.default_rng(5)
    e0 = np.array([-9, -9, -9])
    A = rng.random((19, 19, 19))
    I = A + A[::-1, ::-1, ::-1]                 # I(G) = I(-G) on the box symmetric about 0
    for m, mp, s in [(2, 2, 2), (2, 4, 1), (3, 2, 3)]:
        w = O.window_halfwidth(m, mp)
        q0 = [-9 + w, -9 + w, -9 + w]
        qc = [max(1, (19 - 2 * w - 1) * s)] * 3
        box = O.lanczos(I, e0, m, s, q0, qc, mp)
        idx = np.stack(np.meshgrid(*[np.arange(c) for c in qc], indexing="ij"), -1).reshape(-1, 3)
        Q = np.asarray(q0) + idx / s
        assert np.allclose(O.lanczos_points(I, e0, m, Q, mp), box.reshape(-1), rtol=1e-13, atol=1e-14)
    # off-axis points of an (h h l) plane, away from the grid: I(Q) = I(-Q), constants kept
    h, l = np.meshgrid(np.linspace(-2.37, 2.41, 9), np.linspace(-1.93, 2.07, 7), indexing="ij")
    Q = np.stack([h, h, l], -1).reshape(-1, 3)
    for m, mp in [(2, 2), (2, 4)]:
        a = O.lanczos_points(I, e0, m, Q, mp)
        b = O.lanczos_points(I, e0, m, -Q, mp)
        assert np.allclose(a, b, rtol=1e-12)
        assert np.allclose(O.lanczos_points(np.full_like(I, 2.5), e0, m, Q, mp), 2.5, rtol=1e-13)


# --------------------------------------------------------------------------- P9 brute force

@pytest.mark.parametrize("seed", [11, 12])
def test_pair_double_sum_equals_single_sum(seed):
    m = synth.random_model(seed, n=(2, 3, 3), S=3, M=1, order=0, sigma=0.1)
    G = O.grid_points(m.g0, m.count)[::11]
    P = O.pair_sum(m, 0, G)
    F = O.structure_factor(m, G, order=-1)[0]
    assert np.allclose(P.real, np.abs(F) ** 2 / O.norm_N(m), rtol=1e-11, atol=1e-12)
    assert np.max(np.abs(P.imag)) < 1e-11


# --------------------------------------------------------------------------- P10 FFT route

@pytest.mark.parametrize("seed,order", [(13, 0), (14, 2), (15, 5)])
def test_fft_route_equals_direct_sum(seed, order):
    m = synth.random_model(seed, n=(3, 4, 5), S=2, M=3, order=order)
    G = O.grid_points(m.g0, m.count)
    Id = O.intensity(m, G, order)
    If = O.fft_route_intensity(m, G, order)
    assert np.linalg.norm(Id - If) <= 1e-12 * np.linalg.norm(Id)


def test_fft_route_compositional_equals_direct():
    m = synth.compositional(n=(4, 5, 6), M=2, hmax=1, frac=synth.FCC_BASIS[:3], b=synth.FCC_B[:3])
    G = O.grid_points(m.g0, m.count)
    assert np.allclose(O.intensity(m, G), O.fft_route_intensity(m, G), rtol=1e-11, atol=1e-13)


# ----------------------------------------------------------- P8'' spherical cutoff W_r

@pytest.mark.parametrize("x", [1e-5, 4e-3, 0.3, 2.0, 7.5, 20.0])
def test_ball_transform_against_quadrature(x):
    """The bracket of W_r is the Fourier transform of a unit ball over 4 pi:
    int_0^1 r^2 sin(x r)/(x r) dr, by quadrature."""
    from scipy.integrate import quad
    v, _ = quad(lambda r: r * r * np.sinc(x * r / np.pi), 0.0, 1.0, epsabs=1e-14, epsrel=1e-12, limit=200)
    assert abs(O.ball_ft(x) - v) <= 1e-10 * max(1.0, abs(v))


def test_inscribed_sphere_radius_from_real_space():
    """r_max = half the smallest distance between opposite faces of the supercell,
    computed from the cell vectors (volume over face area)."""
    for cell, n in [([3.1, 4.7, 5.2, 90, 90, 90], (4, 3, 2)), ([4.0, 4.0, 6.5, 90, 90, 120], (5, 5, 3)),
                    ([3.3, 4.1, 4.9, 81, 97, 104], (3, 4, 3))]:
        A = O.cell_vectors(cell) * np.asarray(n, float)[:, None]
        V = abs(np.dot(A[0], np.cross(A[1], A[2])))
        gaps = [V / np.linalg.norm(np.cross(A[(a + 1) % 3], A[(a + 2) % 3])) for a in range(3)]
        for m in (2, 3):
            assert abs(O.spherical_rc(cell, n, m) - (1 - 1 / m) * min(gaps) / 2) < 1e-12


@pytest.mark.parametrize("m,s", [(2, 1), (2, 2), (3, 1)])
def test_spherical_cutoff_is_isotropic_and_keeps_constants(m, s):
    """On a cubic cell with n1 = n2 = n3 the weight depends on |Q - G| and the window,
    both symmetric under exchanging axes: filtering commutes with transposing I(G)."""
    rng = np.random.default_rng(50 + m + s)
    e0 = np.array([-6, -6, -6])
    I = rng.random((13, 13, 13))
    cell, n = [4.0, 4.0, 4.0, 90, 90, 90], (5, 5, 5)
    q0 = [-6 + m] * 3
    qc = [max(1, (13 - 2 * m - 1) * s)] * 3
    a = O.lanczos_spherical(I, e0, m, s, q0, qc, cell, n)
    b = O.lanczos_spherical(I.transpose(2, 0, 1), e0, m, s, q0, qc, cell, n)
    assert np.allclose(b, a.transpose(2, 0, 1), rtol=1e-12)
    c = O.lanczos_spherical(np.full_like(I, 1.75), e0, m, s, q0, qc, cell, n)
    assert np.allclose(c, 1.75, rtol=1e-13)


# ------------------------------------------------- magnetic Debye-Waller factor T_mu(G)

def _mag_with_disp(seed, order=4, M=2, S=3, sigma=0.03, cell=(4.2, 5.1, 6.3, 86.0, 95.0, 104.0), occ=True):
    return synth.random_model(seed, n=(3, 4, 3), S=S, M=M, kind=synth.MAGNETIC, cell=list(cell),
                              mag_order=order, sigma=sigma, with_occ=occ)


def test_debye_waller_of_a_rigid_displacement_is_a_site_shift():
    """Eq. dw with the same displacement u0 on every atom of a site: T = e^{i G.u0}, so the
    magnetic intensity is that of the model whose site sits at r_mu + u0 (Eq. mag_sf)."""
    m = _mag_with_disp(62, order=0)
    m.order = -1
    u0 = np.array([[0.071, -0.043, 0.118], [0.0, 0.0, 0.0], [-0.09, 0.033, 0.02]])
    m.disp = np.broadcast_to(u0[None, :, None, None, None, :],
                             (m.n_configs, m.n_sites) + tuple(m.n) + (3,)).astype(np.float32).copy()
    G = O.grid_points(m.g0, m.count)[::3]
    shifted = _mag_with_disp(62, order=0)
    shifted.frac = m.frac + m.disp[0, :, 0, 0, 0].astype(np.float64)
    assert np.allclose(O.intensity(m, G, order=-1), O.intensity(shifted, G), rtol=1e-10, atol=1e-14)
    T = O.debye_waller(m, G, order=-1)
    g = G / np.asarray(m.n, float)
    assert np.allclose(T, np.exp(2j * np.pi * g @ m.disp[0, :, 0, 0, 0].astype(np.float64).T), atol=1e-12)


def test_debye_waller_averages_over_occupied_atoms_only():
    """1 + a = delta / c: displacements on vacant cells carry no weight, and a site's T is
    the plain mean over its occupied atoms of every configuration."""
    m = _mag_with_disp(63)
    G = O.grid_points(m.g0, m.count)[::5]
    I0 = O.intensity(m, G, order=-1)
    m2 = _mag_with_disp(63)
    rng = np.random.default_rng(5)
    vac = m2.occ == 0
    m2.disp[vac] = rng.normal(0, 0.2, (int(vac.sum()), 3)).astype(np.float32)
    assert np.allclose(O.intensity(m2, G, order=-1), I0, rtol=1e-12, atol=1e-15)
    # a site mean by brute force over (configuration, cell)
    g = G[7] / np.asarray(m.n, float)
    for mu in range(m.n_sites):
        sel = m.occ[:, mu] > 0
        u = m.disp[:, mu][sel].astype(np.float64)
        expect = np.mean(np.exp(2j * np.pi * (u @ g)))
        assert abs(O.debye_waller(m, G[7:8], order=-1)[0, mu] - expect) < 1e-13


def test_debye_waller_of_symmetric_displacements_is_real_and_at_most_one():
    """Displacements that come in +-u pairs: <e^{iG.u}> = <cos G.u>, real and <= 1."""
    m = _mag_with_disp(64, occ=False)
    m.disp[1] = -m.disp[0]
    G = O.grid_points(m.g0, m.count)[::2]
    T = O.debye_waller(m, G, order=-1)
    assert np.max(np.abs(T.imag)) < 1e-14
    assert np.all(T.real <= 1 + 1e-15)
    assert np.allclose(T[np.all(G == 0, axis=1)], 1.0)


@pytest.mark.parametrize("N", [1, 3, 6])
def test_debye_waller_taylor_remainder(N):
    """Order-N T stays within the mean Taylor remainder |x|^{N+1}/(N+1)! of the exact one."""
    m = _mag_with_disp(65, order=N, sigma=0.05)
    G = O.grid_points(m.g0, m.count)[::4]
    Tn = O.debye_waller(m, G)
    Tx = O.debye_waller(m, G, order=-1)
    g = G / np.asarray(m.n, float)
    for mu in range(m.n_sites):
        sel = m.occ[:, mu] > 0
        x = 2 * np.pi * (m.disp[:, mu][sel].astype(np.float64) @ g.T)
        bound = np.mean(np.abs(x) ** (N + 1), axis=0) / math.factorial(N + 1)
        assert np.all(np.abs(Tn[:, mu] - Tx[:, mu]) <= bound * (1 + 1e-9) + 1e-14)


def test_magnetic_with_displacements_keeps_friedel_symmetry():
    m = _mag_with_disp(66, order=5)
    G = O.grid_points(m.g0, m.count)[::7]
    assert np.allclose(O.intensity(m, G), O.intensity(m, -G), rtol=1e-10, atol=1e-14)


def test_nuclear_form_factor_scales_a_single_site_by_f_squared():
    """A |Q|-dependent scattering factor (X-ray f(|Q|)) on one site: I scales by f(s)^2,
    s = |Q|/(4 pi) from the real-space metric."""
    m = synth.random_model(61, n=(3, 4, 3), S=1, M=2, order=3, cell=[4.2, 5.1, 6.3, 86.0, 95.0, 104.0])
    G = O.grid_points(m.g0, m.count)[::5]
    I0 = O.intensity(m, G)
    ff = np.array([2.1, 3.0, 1.2, 0.7, 0.4, 9.0, 0.3])
    m.ff = ff[None, :]
    I1 = O.intensity(m, G)
    A = O.cell_vectors(m.cell)
    Gi = np.linalg.inv(A @ A.T)
    g = G / np.asarray(m.n, float)
    s2 = np.einsum("gi,ij,gj->g", g, Gi, g) / 4
    f = ff[0] * np.exp(-ff[1] * s2) + ff[2] * np.exp(-ff[3] * s2) + ff[4] * np.exp(-ff[5] * s2) + ff[6]
    assert np.allclose(I1, I0 * f * f, rtol=1e-11, atol=1e-14)


# ------------------------------------------------- the ensemble mean and the Bragg rule

def test_identical_configurations_give_the_single_configuration_intensity():
    """M copies of one configuration: (1/M) sum |F|^2 = |F|^2 and |<F>|^2 = |F|^2, so the
    intensity equals the M = 1 intensity at every G, the unit-cell Bragg points included
    (where it is 0).  A 1/M^2 in place of 1/M, or the subtraction applied off H, fails."""
    base = synth.random_model(70, n=(3, 4, 3), S=2, M=1, order=3)
    G = np.concatenate([O.grid_points(base.g0, base.count)[::5], np.array([[0, 0, 0], [3, -4, 6]])])
    I1 = O.intensity(base, G)
    for M in (2, 5):
        rep = synth.random_model(70, n=(3, 4, 3), S=2, M=1, order=3)
        rep.occ = np.repeat(base.occ, M, axis=0)
        rep.disp = np.repeat(base.disp, M, axis=0)
        IM = O.intensity(rep, G)
        assert np.allclose(IM, I1, rtol=1e-12, atol=1e-13)
    assert np.all(np.abs(I1[O.is_unit_cell_bragg(G, base.n)]) < 1e-10)
    mag = synth.random_model(71, n=(3, 3, 4), S=2, M=1, kind=synth.MAGNETIC, mag_order=2)
    magM = synth.random_model(71, n=(3, 3, 4), S=2, M=1, kind=synth.MAGNETIC, mag_order=2)
    magM.spin, magM.occ, magM.disp = (np.repeat(a, 3, axis=0) for a in (mag.spin, mag.occ, mag.disp))
    Gm = O.grid_points(mag.g0, mag.count)[::9]
    assert np.allclose(O.intensity(magM, Gm), O.intensity(mag, Gm), rtol=1e-12, atol=1e-15)


def test_bragg_points_carry_the_population_variance():
    """At H (G = 0 mod n) the diffuse intensity is (1/N) times the population variance
    (1/M) sum_m |F_m - mean F|^2, computed two-pass; elsewhere it is (1/N) mean |F_m|^2."""
    m = synth.random_model(72, n=(3, 2, 4), S=3, M=6, order=2)
    H = np.array([[0, 0, 0], [3, 2, 4], [-6, 2, 8], [3, -4, -4]])
    off = np.array([[1, 0, 0], [2, 1, 3], [-4, 1, 5]])
    G = np.concatenate([H, off])
    F = O.structure_factor(m, G)
    N = O.norm_N(m)
    I = O.intensity(m, G)
    mean = F.mean(axis=0)
    var = np.mean(np.abs(F - mean[None]) ** 2, axis=0)
    assert np.allclose(I[:len(H)], var[:len(H)] / N, rtol=1e-10, atol=1e-12)
    assert np.allclose(I[len(H):], np.mean(np.abs(F[:, len(H):]) ** 2, axis=0) / N, rtol=1e-12)
    # and the variance is not zero: the configurations differ
    assert np.all(var[:len(H)] > 1e-6)


# ------------------------------------------------- the windowed-sinc weights and support

def test_lanczos_m4_weights_closed_form():
    """Impulse response of the m = 4 filter on the G grid: the weights of Eq. lanczos with
    r_cut = 0.375, sinc(2 pi r_cut d) sinc(pi d / 4) at d = 0, 1, 2, 3 (and 0 at |d| = 4),
    normalised per axis."""
    w = np.array([0.030021, -0.135095, 0.270190, 1.0, 0.270190, -0.135095, 0.030021])
    e0 = np.array([-7, -7, -7])
    I = np.zeros((15, 15, 15))
    I[7, 7, 7] = 1.0
    out = O.lanczos(I, e0, 4, 1, [-3, -3, -3], [7, 7, 7])
    line = w / w.sum()
    assert np.allclose(out, np.einsum("i,j,k->ijk", line, line, line), atol=3e-6 * line.max() ** 3)
    # the weights themselves, to the 6 digits given
    assert np.allclose(out[3, 3, :] / out[3, 3, 3], w, atol=5e-7)


@pytest.mark.parametrize("m", [2, 4])
def test_lanczos_support_and_nominal_cutoff_are_the_printed_ones(m):
    """The sum at an off-grid Q reads exactly (2m)^3 supercell Bragg points (64 for m = 2,
    512 for m = 4), and the weight of Eq. weight_sinc vanishes where 2 r_cut d is a
    nonzero integer, r_cut = 0.5 (1 - 1/m) (0.25 and 0.375)."""
    g = golden()
    rng = np.random.default_rng(80 + m)
    e0 = np.array([-8, -8, -8])
    base = rng.random((17, 17, 17))
    Q = np.array([[0.37, -0.81, 1.23]])
    ref = O.lanczos_points(base, e0, m, Q)[0]
    touched = 0
    for idx in itertools.product(range(17), repeat=3):
        if max(abs(idx[a] + e0[a] - Q[0, a]) for a in range(3)) > m + 1:
            continue
        pert = base.copy()
        pert[idx] += 1.0
        if O.lanczos_points(pert, e0, m, Q)[0] != ref:
            touched += 1
    assert touched == g[f"lanczos_support_m{m}"]
    rcut = g[f"lanczos_rcut_m{m}"]
    # impulse at G = 0 read at Q = (d, 0, 0): proportional to the axis weight at d
    imp = np.zeros((17, 17, 17))
    imp[8, 8, 8] = 1.0
    for k in range(1, 4):
        d = k / (2 * rcut)
        if d < m:
            v = O.lanczos_points(imp, e0, m, np.array([[d, 0.0, 0.0]]))[0]
            assert abs(v) < 1e-15
    v = O.lanczos_points(imp, e0, m, np.array([[0.5 / (2 * rcut), 0.0, 0.0]]))[0]
    assert v > 1e-3


def _cosine_response_mean(m, dr, s=8):
    """The plain filter applied to I(G) = 1 + cos(2 pi G1 dr), averaged over s output
    points Q1 = i/s in [0, 1): the cutoff function at the separation dr."""
    w = O.window_halfwidth(m)
    e0 = np.array([-w - 2, -w - 2, -w - 2])
    cnt = 2 * w + 6
    G1 = e0[0] + np.arange(cnt)
    I = np.broadcast_to((1.0 + np.cos(2 * np.pi * G1 * dr))[:, None, None], (cnt, cnt, cnt))
    return float(np.mean(O.lanczos(I, e0, m, s, [0, 0, 0], [s, 1, 1])[:, 0, 0])) - 1.0


@pytest.mark.parametrize("m", [2, 3, 4])
def test_plain_filter_cutoff_is_half_at_the_nominal_cutoff(m):
    """Sec. V.B: the idealized cutoff function equals 0.5 at the nominal cutoff
    r_cut = 0.5 (1 - 1/m) (0.25 at m = 2, 0.375 at m = 4), is flat near 0, and ends at
    the periodic limit r_cut = 0.5 of Sec. II; the actual (finite-sum) cutoff read on
    the G grid follows it."""
    g = golden()
    rc = g.get(f"lanczos_rcut_m{m}", 0.5 * (1 - 1 / m))
    assert abs(_cosine_response(m, 2, rc) - 0.5) < 0.06
    assert _cosine_response(m, 2, 0.05) > 0.95
    assert abs(_cosine_response_mean(m, g["periodic_rcut"])) < 0.02
    assert _cosine_response_mean(m, 0.5 * g["periodic_rcut"] * (1 - 2 / m)) > 0.6


@pytest.mark.parametrize("m", [4, 6])
def test_spherical_cutoff_radius_in_real_space(m):
    """The spherical cutoff W_r(|Q - G|) with r_c = (1 - 1/m) r_max, r_max the radius of
    the sphere inscribed in the supercell (Sec. V.B), read in real space on a non-cubic
    cell along directions off the axes: I(G) = 1 + cos(Q(G).dr) with Q(G) Cartesian
    (inverse Angstrom) and dr Cartesian (Angstrom); the response at Q = 0 is I(0) - 1.
    A ball of radius r_c, blurred by the window, keeps half of a separation at |dr| = r_c,
    all of a short one and none of one well beyond r_c: any slip in the argument
    |Q - G| r_c (a lost 2 pi, n or unit) moves the half-way point."""
    cell, n = [4.0, 4.6, 5.3, 84.0, 97.0, 101.0], (6, 6, 6)
    R = O.reciprocal_basis(cell)
    rc = O.spherical_rc(cell, n, m)
    e0 = np.array([-m - 1] * 3)
    cnt = 2 * m + 3
    Qc = (O.grid_points(e0, (cnt, cnt, cnt)) / np.asarray(n, float)) @ R

    def response(dr):
        I = (1.0 + np.cos(Qc @ dr)).reshape(cnt, cnt, cnt)
        return float(O.lanczos_spherical(I, e0, m, 1, [0, 0, 0], [1, 1, 1], cell, n)[0, 0, 0]) - 1.0

    for direction in ([1.0, 0.4, -0.3], [-0.2, 1.0, 0.7], [0.5, -0.5, 1.0]):
        u = np.asarray(direction) / np.linalg.norm(direction)
        assert response(0.3 * rc * u) > 0.9
        assert abs(response(rc * u) - 0.5) < 0.15
        assert abs(response(1.4 * rc * u)) < 0.06


def test_sampled_windows_match_the_box_filter():
    """The sampled check used at full size (I(G) on each output's own window, then the
    windowed sum at that output) equals the oracle's filter of the whole box."""
    from tests.helpers import edge_sample_indices, oracle_filtered_at
    m = synth.random_model(5, n=(3, 4, 3), S=2, M=2, order=3)
    m.g0, m.count = (-4, -5, -4), (9, 11, 9)
    for mp, sph in [(2, False), (4, False), (2, True)]:
        ref = O.filtered_intensity_spherical(m, 2) if sph else O.filtered_intensity(m, 2, 1, mprime=mp)
        idx = edge_sample_indices(m.count, 40, 1)
        got = oracle_filtered_at(m, idx + np.asarray(m.g0), 2, mp, sph)
        assert np.allclose(got, ref[tuple(idx.T)], rtol=1e-13, atol=1e-15)


# ------------------------------------------------- the method of sub-boxes (Sec. V.A)

def _autocorrelation(occ):
    """A(k) = mean over configurations of (1/N) sum_R delta(R) delta(R + k), periodic,
    by brute force over every shift k."""
    M, n = occ.shape[0], occ.shape[1:]
    A = np.zeros(n)
    for k in itertools.product(*[range(v) for v in n]):
        A[k] = np.mean([np.mean(occ[m] * np.roll(occ[m], [-v for v in k], axis=(0, 1, 2))) for m in range(M)])
    return A


def test_subbox_applies_the_triangular_cutoff():
    """Sec. V.A: with every lattice point a sub-box origin, the number of pairs at a
    separation of k cells inside a box of nsb cells is nsb - |k| per axis, so
    <|F_sb(Q)|^2> = b^2 sum_k prod_a (nsb_a - |k_a|) A(k) e^{2 pi i Q.k} -- the periodic
    pair correlations under a triangular cutoff that reaches 0 at |k_a| = nsb_a -- and
    <F_sb(Q)> = b c sum_d e^{2 pi i Q.(d + r)} with c the mean occupancy."""
    n, nsb = (6, 5, 4), (3, 2, 3)
    m = synth.compositional(n=n, M=2, hmax=1, frac=np.array([[0.13, 0.29, 0.41]]), b=np.array([0.8]))
    Q = np.random.default_rng(9).uniform(-1.3, 1.7, (12, 3))
    sq, mean = O.subbox_moments(m, Q, nsb)
    A = _autocorrelation(m.occ[:, 0].astype(np.float64))
    ks = list(itertools.product(*[range(-(v - 1), v) for v in nsb]))
    tri = np.array([np.prod([nsb[a] - abs(k[a]) for a in range(3)]) for k in ks])
    Ak = np.array([A[tuple(k[a] % n[a] for a in range(3))] for k in ks])
    ph = np.exp(2j * np.pi * Q @ np.array(ks).T)
    expect = 0.8 ** 2 * (ph * (tri * Ak)[None]).sum(axis=1)
    assert np.allclose(sq, expect.real, rtol=1e-11, atol=1e-11) and np.max(np.abs(expect.imag)) < 1e-9
    c = float(m.occ.astype(np.float64).mean())
    d = np.array(list(itertools.product(*[range(v) for v in nsb])))
    fm = 0.8 * c * np.exp(2j * np.pi * Q @ (d + m.frac[0]).T).sum(axis=1)
    assert np.allclose(mean, fm, rtol=1e-11, atol=1e-12)


def test_subbox_rigid_shift_moves_the_site():
    """Exact mode: one displacement u0 for every atom of a site is the site at r + u0."""
    m = synth.random_model(74, n=(3, 4, 3), S=2, M=2, order=0, with_disp=False)
    m.disp = np.zeros((2, 2, 3, 4, 3, 3), np.float32)
    m.disp[:, 1] = np.array([0.07, -0.11, 0.05], np.float32)
    Q = np.random.default_rng(2).uniform(-1, 1, (9, 3))
    a = O.subbox_intensity(m, Q, (2, 3, 2), order=-1)
    s = synth.random_model(74, n=(3, 4, 3), S=2, M=2, order=0, with_disp=False)
    s.frac = m.frac + np.array([[0, 0, 0], m.disp[0, 1, 0, 0, 0].astype(np.float64)])
    assert np.allclose(a, O.subbox_intensity(s, Q, (2, 3, 2)), rtol=1e-11, atol=1e-13)


def test_lanczos_m2_cutoff_is_close_to_the_subbox_triangle():
    """Sec. V.B: the m = 2 filter's effective cutoff resembles a smoothed triangle -- the
    sub-box cutoff 1 - |dr| n/nsb with nsb = n/2, i.e. 1 - 2|dr| -- and its intensities
    resemble the sub-box ones far more than the unfiltered supercell Bragg points do."""
    for dr in np.linspace(0.0, 0.5, 11):
        assert abs(_cosine_response_mean(2, dr) - (1 - 2 * dr)) < 0.16
    n = (12, 12, 12)
    rng = np.random.default_rng(3)
    occ = np.stack([(synth._periodic_gaussian_smooth(rng.normal(size=n), 1.0) > 0) for _ in range(2)])
    mdl = synth.Model(cell=np.array([1.0, 1, 1, 90, 90, 90]), n=n, frac=np.zeros((1, 3)), b=np.ones(1),
                      occ=occ[:, None].astype(np.float32))
    h = np.linspace(0.05, 1.95, 39)
    Q = np.stack([h, 0.5 * h, np.full_like(h, 0.3)], -1)
    sb = O.subbox_intensity(mdl, Q, (6, 6, 6))
    lz = O.filtered_points(mdl, 2, Q * np.asarray(n))
    near = O.intensity(mdl, np.round(Q * np.asarray(n)).astype(np.int32))
    rel = lambda a: np.linalg.norm(a - sb) / np.linalg.norm(sb)
    assert rel(lz) < 0.3 and rel(lz) < 0.5 * rel(near)
