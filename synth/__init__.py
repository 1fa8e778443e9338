"""Seeded synthetic inputs for the diffuse-scattering hot path.

This module only *draws* atomistic models: unit cells, site lists, and the
per-configuration occupancy, displacement and spin arrays, with the shapes,
sizes and value distributions of the paper's workloads.  It holds none of the
method's arithmetic (no Fourier sums, no structure factors, no filters), so
both the FP64 oracle and the GPU library consume the very same arrays.

Data model (Sec. II, Eq. r_vec): an atom sits at R + r_mu + u_{R,mu}, with R a
lattice point of an n1 x n2 x n3 supercell, r_mu the average fractional site
position and u a displacement in fractional unit-cell coordinates.  Each site
carries an occupancy delta (1 = occupied) and, for magnetic models, a moment M
in Cartesian components (Sec. III.D).

Array layouts (C order, float32):
  occ  [M][S][n1][n2][n3]        occupancy delta, or None when every site is occupied
  disp [M][S][n1][n2][n3][3]     fractional displacement components, or None
  spin [M][S][n1][n2][n3][3]     Cartesian moment components, or None

Every draw uses ``numpy.random.default_rng([workload, model, member])`` and
fills arrays in C order, so a model is reproducible from its integers alone.

The paper's own supercells (Monte Carlo ice-rule models, Sec. IV) are not
available; these generators stand in for them with the same array structure.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import List, Optional

import numpy as np

NUCLEAR = 0
MAGNETIC = 1

# fcc-type four-site basis and scattering lengths used by the displacive workload.
FCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])
FCC_B = np.array([1.0, 0.7, 0.7, 0.7])

# Magnetic form-factor parameters (A, a, B, b, C, c, D) of the magnetic workload.
MAG_FF = np.array([0.4, 20.0, 0.5, 7.0, 0.1, 2.0, 0.0])


@dataclasses.dataclass
class Model:
    """One atomistic model: a unit cell, its sites, a supercell and an ensemble."""
    cell: np.ndarray              # (6,) a, b, c [Angstrom]; alpha, beta, gamma [deg]
    n: tuple                      # supercell (n1, n2, n3)
    frac: np.ndarray              # (S, 3) average fractional site positions r_mu
    b: np.ndarray                 # (S,) scattering length (nuclear) or moment scale (magnetic)
    kind: int = NUCLEAR
    order: int = 0                # Taylor order of exp(i G.u); 0 when there are no displacements
    ff: Optional[np.ndarray] = None   # (S, 7) magnetic form factor parameters
    pos_id: Optional[np.ndarray] = None  # (S,) position index for the normalisation
    norm_N: float = 0.0           # 0 => n1 n2 n3 x number of distinct positions
    occ: Optional[np.ndarray] = None
    disp: Optional[np.ndarray] = None
    spin: Optional[np.ndarray] = None
    g0: tuple = (0, 0, 0)         # output box origin, supercell Bragg indices G
    count: tuple = (1, 1, 1)      # output box extent
    name: str = ""

    @property
    def n_sites(self) -> int:
        return int(self.frac.shape[0])

    @property
    def n_configs(self) -> int:
        for a in (self.occ, self.disp, self.spin):
            if a is not None:
                return int(a.shape[0])
        return 1

    @property
    def n_voxels(self) -> int:
        return int(np.prod(self.count))


def rng_for(workload: int, model: int = 0, member: int = 0) -> np.random.Generator:
    return np.random.default_rng([workload, model, member])


def box_from_rlu(n, hmax, closed=True):
    """Supercell box G_alpha in [-hmax n_alpha, hmax n_alpha] (closed) or [.., ..) (half-open)."""
    g0 = tuple(-hmax * int(v) for v in n)
    count = tuple(2 * hmax * int(v) + (1 if closed else 0) for v in n)
    return g0, count


def _periodic_gaussian_smooth(field: np.ndarray, width: float) -> np.ndarray:
    """Periodic convolution of a 3D array with a unit-sum Gaussian (std = width cells)."""
    shp = field.shape
    ax = [np.minimum(np.arange(s), s - np.arange(s)).astype(np.float64) for s in shp]
    d2 = ax[0][:, None, None] ** 2 + ax[1][None, :, None] ** 2 + ax[2][None, None, :] ** 2
    ker = np.exp(-d2 / (2.0 * width * width))
    ker /= ker.sum()
    return np.fft.irfftn(np.fft.rfftn(field) * np.fft.rfftn(ker), s=shp, axes=(0, 1, 2))


def correlated_displacements(rng, M, S, n, sigma=0.05, width=1.5, renormalise=False):
    """iid N(0, sigma^2) per (config, site, cell, component), smoothed per sublattice
    and component by a periodic unit-sum Gaussian of std `width` cells.
    renormalise=True rescales each configuration to a marginal rms of sigma."""
    raw = rng.normal(0.0, sigma, size=(M, S) + tuple(n) + (3,))
    out = np.empty_like(raw)
    for m in range(M):
        for s in range(S):
            for c in range(3):
                out[m, s, ..., c] = _periodic_gaussian_smooth(raw[m, s, ..., c], width)
        if renormalise:
            out[m] *= sigma / np.sqrt(np.mean(out[m] ** 2))
    return out.astype(np.float32)


def compositional(workload=1, model=0, n=12, M=1, hmax=2, closed=False, p=0.5,
                  frac=None, b=None) -> Model:
    """Occupational disorder on a simple-cubic lattice (a = 1, one site at the origin by
    default); Bernoulli(p) occupancies drawn per configuration."""
    frac = np.zeros((1, 3)) if frac is None else np.asarray(frac, dtype=np.float64)
    b = np.ones(frac.shape[0]) if b is None else np.asarray(b, dtype=np.float64)
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    occ = np.empty((M, frac.shape[0]) + nn, dtype=np.float32)
    for m in range(M):
        occ[m] = (rng_for(workload, model, m).random((frac.shape[0],) + nn) < p)
    g0, count = box_from_rlu(nn, hmax, closed)
    return Model(cell=np.array([1.0, 1.0, 1.0, 90.0, 90.0, 90.0]), n=nn, frac=frac, b=b,
                 kind=NUCLEAR, order=0, occ=occ, g0=g0, count=count,
                 name=f"compositional n={nn} S={frac.shape[0]} M={M}")


def displacive(workload=2, model=0, n=32, M=1, order=8, hmax=8, n_sites=4,
               sigma=0.05, width=1.5, renormalise=False, with_occ=False) -> Model:
    """Displacive disorder on the fcc-type basis (prefix of `n_sites` sites), fractional
    displacements drawn by `correlated_displacements` (delta == 1 unless with_occ)."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    frac = FCC_BASIS[:n_sites].copy()
    b = FCC_B[:n_sites].copy()
    disp = np.concatenate([correlated_displacements(rng_for(workload, model, m), 1, n_sites, nn,
                                                    sigma, width, renormalise) for m in range(M)])
    occ = None
    if with_occ:
        occ = np.stack([(rng_for(workload, model, 1000 + m).random((n_sites,) + nn) < 0.7)
                        for m in range(M)]).astype(np.float32)
    g0, count = box_from_rlu(nn, hmax, True)
    return Model(cell=np.array([1.0, 1.0, 1.0, 90.0, 90.0, 90.0]), n=nn, frac=frac, b=b,
                 kind=NUCLEAR, order=order, occ=occ, disp=disp, g0=g0, count=count,
                 name=f"displacive n={nn} S={n_sites} M={M} N={order}")


def pyrochlore_sites() -> np.ndarray:
    """16 pyrochlore sites of the conventional cubic cell: fcc translations of a
    regular tetrahedron with vertices 0, (1/4,1/4,0), (1/4,0,1/4), (0,1/4,1/4)."""
    tet = np.array([[0, 0, 0], [0.25, 0.25, 0], [0.25, 0, 0.25], [0, 0.25, 0.25]])
    return np.array([(t + v) % 1.0 for t in FCC_BASIS for v in tet])


def pyrochlore_neighbours(frac: np.ndarray, n) -> List[List[tuple]]:
    """For each site mu, the list of (dR1, dR2, dR3, nu) nearest neighbours at the
    minimum distance sqrt(2)/4 (cubic cell, a = 1)."""
    S = frac.shape[0]
    nbrs = []
    target = np.sqrt(2.0) / 4.0
    for mu in range(S):
        lst = []
        for nu in range(S):
            for d in itertools.product((-1, 0, 1), repeat=3):
                v = np.array(d) + frac[nu] - frac[mu]
                if abs(np.linalg.norm(v) - target) < 1e-9:
                    lst.append((d[0], d[1], d[2], nu))
        nbrs.append(lst)
    return nbrs


def magnetic(workload=3, model=0, n=24, M=1, hmax=6, a=10.0) -> Model:
    """Pyrochlore spins: v iid N(0, I3) per spin; each spin is the normalised sum of its
    own v and the v of its six nearest neighbours (minimum image)."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    frac = pyrochlore_sites()
    S = frac.shape[0]
    nb = pyrochlore_neighbours(frac, nn)
    spin = np.empty((M, S) + nn + (3,), dtype=np.float32)
    for m in range(M):
        v = rng_for(workload, model, m).normal(size=(S,) + nn + (3,))
        acc = v.copy()
        for mu in range(S):
            for (d1, d2, d3, nu) in nb[mu]:
                acc[mu] += np.roll(v[nu], shift=(-d1, -d2, -d3), axis=(0, 1, 2))
        acc /= np.linalg.norm(acc, axis=-1, keepdims=True)
        spin[m] = acc
    g0, count = box_from_rlu(nn, hmax, True)
    return Model(cell=np.array([a, a, a, 90.0, 90.0, 90.0]), n=nn, frac=frac, b=np.ones(S),
                 kind=MAGNETIC, order=0, ff=np.tile(MAG_FF, (S, 1)), spin=spin,
                 g0=g0, count=count, name=f"magnetic pyrochlore n={nn} M={M}")


ENSEMBLE_SIZES = (16, 20, 24, 32, 40)


def ensemble(workload=4, n_models=8, configs_per_model=8, order=6, hmax=4,
             sizes=ENSEMBLE_SIZES) -> List[Model]:
    """Batched ensemble: each model draws (type, n, number of sites) from its own seed;
    sites are a prefix of the fcc-type basis."""
    models = []
    for mi in range(n_models):
        r = rng_for(workload, mi, 10_000)
        typ = int(r.integers(0, 2))            # 0 displacive, 1 compositional
        n = int(sizes[int(r.integers(0, len(sizes)))])
        S = int(r.integers(1, 5))
        if typ == 0:
            mdl = displacive(workload, mi, n=n, M=configs_per_model, order=order,
                             hmax=hmax, n_sites=S)
        else:
            mdl = compositional(workload, mi, n=n, M=configs_per_model, hmax=hmax,
                                closed=True, frac=FCC_BASIS[:S], b=FCC_B[:S])
        models.append(mdl)
    return models


def serving_request_model(workload=5, model=0, n=None, S=None, typ=None, order=6, hmax=2):
    """A model of the serving workload: edge n ~ U{8..64}, 1-16 sites at uniform random
    positions, b ~ U(0.5, 1.5), disorder type uniform over {compositional, displacive,
    magnetic}, one configuration, box |h|,|k|,|l| <= hmax (closed)."""
    r = rng_for(workload, model, 20_000)
    n = int(r.integers(8, 65)) if n is None else int(n)
    S = int(r.integers(1, 17)) if S is None else int(S)
    typ = int(r.integers(0, 3)) if typ is None else int(typ)
    frac = r.random((S, 3))
    b = r.uniform(0.5, 1.5, S)
    nn = (n, n, n)
    g0, count = box_from_rlu(nn, hmax, True)
    r2 = rng_for(workload, model, 0)
    cell = np.array([1.0, 1.0, 1.0, 90.0, 90.0, 90.0])
    if typ == 0:
        occ = (r2.random((1, S) + nn) < 0.5).astype(np.float32)
        return Model(cell=cell, n=nn, frac=frac, b=b, kind=NUCLEAR, order=0, occ=occ,
                     g0=g0, count=count, name=f"serve comp n={n} S={S}")
    if typ == 1:
        disp = correlated_displacements(r2, 1, S, nn)
        return Model(cell=cell, n=nn, frac=frac, b=b, kind=NUCLEAR, order=order, disp=disp,
                     g0=g0, count=count, name=f"serve disp n={n} S={S}")
    v = r2.normal(size=(1, S) + nn + (3,))
    spin = (v / np.linalg.norm(v, axis=-1, keepdims=True)).astype(np.float32)
    return Model(cell=np.array([10.0, 10.0, 10.0, 90.0, 90.0, 90.0]), n=nn, frac=frac, b=b,
                 kind=MAGNETIC, order=0, ff=np.tile(MAG_FF, (S, 1)), spin=spin,
                 g0=g0, count=count, name=f"serve mag n={n} S={S}")


def poisson_arrivals(workload=5, rate=200.0, duration=30.0):
    """Open-loop Poisson arrival times (seconds) of the serving workload."""
    r = rng_for(workload, 0, 30_000)
    t, out = 0.0, []
    while True:
        t += r.exponential(1.0 / rate)
        if t >= duration:
            return np.array(out)
        out.append(t)


def random_model(seed, n=(3, 4, 5), S=2, M=2, order=3, kind=NUCLEAR, with_occ=True,
                 with_disp=True, sigma=0.05, cell=None, mag_order=0):
    """Small general test model: non-centrosymmetric random site positions, random b,
    optional occupancies and uncorrelated displacements, non-cubic cells allowed.
    Magnetic models carry displacements (for the Debye-Waller factor) only when
    mag_order > 0, which is then their Taylor order."""
    r = np.random.default_rng([99, seed])
    nn = tuple(int(v) for v in n)
    frac = r.random((S, 3))
    b = r.uniform(0.3, 1.5, S)
    occ = (r.random((M, S) + nn) < 0.6).astype(np.float32) if with_occ else None
    disp = (r.normal(0.0, sigma, (M, S) + nn + (3,))).astype(np.float32) if with_disp else None
    cell = np.array([1.0, 1.0, 1.0, 90.0, 90.0, 90.0]) if cell is None else np.asarray(cell, float)
    spin = None
    ff = None
    if kind == MAGNETIC:
        v = r.normal(size=(M, S) + nn + (3,))
        spin = (v / np.linalg.norm(v, axis=-1, keepdims=True)).astype(np.float32)
        order = int(mag_order)
        if order == 0:
            disp = None
        ff = np.tile(MAG_FF, (S, 1))
    g0 = tuple(-2 * v - 1 for v in nn)
    count = tuple(4 * v + 3 for v in nn)
    return Model(cell=cell, n=nn, frac=frac, b=b, kind=kind,
                 order=order if disp is not None else 0, ff=ff, occ=occ, disp=disp, spin=spin,
                 g0=g0, count=count, name=f"random seed={seed}")
