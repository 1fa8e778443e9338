"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: printed values,
closed forms, exact invariances, the Taylor remainder bound, an independent
brute-force formula (pair double sum), or an independent algorithm (the paper's
FFT route against the direct sum).  All run on the CPU.
"""
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

def test_debye_waller_scales_a_single_site_by_exp_minus_2Bs2():
    """One magnetic site: T = exp(-B s^2) multiplies F, so I scales by exp(-2 B s^2),
    with s = |Q|/(4 pi) taken here from the real-space metric (|Q|^2 = 4 pi^2 g.Gi.g)."""
    m = synth.random_model(60, n=(3, 4, 3), S=1, M=2, kind=synth.MAGNETIC,
                           cell=[4.2, 5.1, 6.3, 86.0, 95.0, 104.0])
    G = O.grid_points(m.g0, m.count)[::5]
    I0 = O.intensity(m, G)
    m.dw_b = np.array([0.8])
    I1 = O.intensity(m, G)
    A = O.cell_vectors(m.cell)
    Gi = np.linalg.inv(A @ A.T)                          # inverse real-space metric
    g = G / np.asarray(m.n, float)
    s2 = np.einsum("gi,ij,gj->g", g, Gi, g) * 4 * np.pi ** 2 / (16 * np.pi ** 2)
    assert np.allclose(I1, I0 * np.exp(-2 * 0.8 * s2), rtol=1e-12, atol=1e-15)


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
