"""Test glue: hand a synthetic model to the HIP library through the C-ABI binding."""
import numpy as np

import paper_1809_07088_amd as dsx


def desc_kwargs(model):
    return dict(cell=model.cell, n=model.n, frac=model.frac, b=model.b, kind=model.kind,
                taylor_order=model.order,
                n_configs=model.n_configs, has_occ=model.occ is not None, ff=model.ff,
                pos_id=model.pos_id, norm_N=model.norm_N)


def to_dsx(model, device=True):
    """Create a dsx model and upload every configuration (torch device tensors or host)."""
    import torch
    h = dsx.Model(**desc_kwargs(model))
    for m in range(model.n_configs):
        arrs = []
        for a in (model.occ, model.disp, model.spin):
            if a is None:
                arrs.append(None)
            elif device:
                arrs.append(torch.from_numpy(np.ascontiguousarray(a[m])).cuda())
            else:
                arrs.append(np.ascontiguousarray(a[m]))
        h.set_sites(m, *arrs)
    h.set_grid(model.g0, model.count)
    return h


def gpu_intensity(model, device=True):
    import torch
    h = to_dsx(model, device)
    if device:
        out = torch.empty(tuple(model.count), dtype=torch.float32, device="cuda")
        h.compute_intensity(out)
        torch.cuda.synchronize()
        res = out.cpu().numpy()
    else:
        res = np.empty(tuple(model.count), dtype=np.float32)
        h.compute_intensity(res)
    h.close()
    return res


def gpu_filtered(model, m, s=1, mprime=2):
    import torch
    h = to_dsx(model)
    out = torch.empty(tuple(s * c for c in model.count), dtype=torch.float32, device="cuda")
    if mprime == 2:
        h.noise_filter(m, s, out)
    else:
        h.noise_filter_cutoff(m, mprime, s, out)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    h.close()
    return res


def rel_l2(a, ref):
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def max_rel(a, ref):
    """Worst voxel: max |a - ref| / max |ref|."""
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


# The parity bar: relative L2 over every compared voxel <= 1e-5 (float32 FFTs and
# recombination against the float64 oracle), and the worst voxel within 1e-5 of the
# largest reference value.
TOL = 1e-5
MAXTOL = 1e-5


def assert_parity(a, ref, tol=TOL, maxtol=MAXTOL, what=""):
    e, w = rel_l2(a, ref), max_rel(a, ref)
    assert e <= tol and w <= maxtol, f"{what} rel L2 {e:.3e} (<= {tol:.0e}), worst voxel {w:.3e} (<= {maxtol:.0e})"


def discrete_displacement_model(seed, n=(4, 3, 5), S=2, M=2, K=3, amp=0.03, with_occ=True):
    """A nuclear model whose displacements take K values per site (a split-site case)."""
    import synth
    m = synth.random_model(seed, n=n, S=S, M=M, order=8, with_occ=with_occ)
    r = np.random.default_rng([7, seed])
    vals = r.uniform(-amp, amp, (S, K, 3)).astype(np.float32)
    pick = r.integers(0, K, (M, S) + tuple(n))
    m.disp = np.ascontiguousarray(vals[np.arange(S)[None, :, None, None, None], pick]).astype(np.float32)
    return m


def split_model(model, tol=0.0):
    """The split-site form of `model` (dsx_split_sites), N kept from the original."""
    import copy
    from oracle import oracle as O
    fr, b, parent, occ = dsx.split_sites(model.n, model.frac, model.b, model.disp, model.occ, tol)
    s = copy.copy(model)
    s.frac, s.b, s.occ, s.disp, s.order = fr, b, occ, None, 0
    s.pos_id = (parent if model.pos_id is None else np.asarray(model.pos_id)[parent]).astype(np.int32)
    s.norm_N = O.norm_N(model)
    return s


# ----------------------------------------------------------------- sampled filtered outputs

def edge_sample_indices(count, k, seed, edges=None):
    """k output indices (i1, i2, i3) of a box of `count` voxels, drawn so that most
    coordinates sit on the places a tiled, half-stored filter treats specially: the
    box faces, both sides of the mirror plane, and both sides of tile and segment
    boundaries (multiples of 4, 8, 12, 16, 32, 64 and their mirrors), the rest uniform."""
    rng = np.random.default_rng(seed)
    out = np.empty((k, 3), dtype=np.int64)
    for a in range(3):
        c = int(count[a])
        cand = {0, 1, c - 2, c - 1, c // 2 - 1, c // 2, c // 2 + 1}
        for t in (4, 8, 12, 16, 32, 64):
            for b in range(t, c, t):
                cand.update({b - 1, b, c - 1 - b, c - b})
        if edges:
            cand.update(edges[a])
        cand = np.array(sorted(v for v in cand if 0 <= v < c))
        pick = rng.random(k) < 0.75
        out[:, a] = np.where(pick, cand[rng.integers(0, len(cand), k)], rng.integers(0, c, k))
    return out


def oracle_windows(model, Q, w, order=None):
    """I(G) by the oracle's direct sum on the (2w)^3 window [floor(Q_a) - w + 1,
    floor(Q_a) + w] of every point Q [k][3]: (windows [k][2w][2w][2w], their origins
    [k][3]).  Every G shared by several windows is summed once."""
    from oracle import oracle as O
    Q = np.asarray(Q, dtype=np.float64).reshape(-1, 3)
    e0 = np.floor(Q).astype(np.int64) - w + 1
    off = np.stack(np.meshgrid(*[np.arange(2 * w)] * 3, indexing="ij"), -1).reshape(-1, 3)
    allG = (e0[:, None, :] + off[None, :, :]).reshape(-1, 3)
    Gu, inv = np.unique(allG, axis=0, return_inverse=True)
    Iu = O.intensity(model, Gu.astype(np.int32), order)
    return Iu[inv.ravel()].reshape(len(Q), 2 * w, 2 * w, 2 * w), e0.astype(np.int32)


def oracle_filtered_at(model, Q, m, mprime=2, spherical=False, order=None):
    """The oracle's filtered intensity at the points Q [k][3] (units of the supercell
    Bragg grid): I(G) on each window by direct sum, then the oracle's windowed sum
    (Sec. V.B) -- the separable weights with the m' cutoff, or the spherical W_r."""
    from oracle import oracle as O
    Q = np.asarray(Q, dtype=np.float64).reshape(-1, 3)
    w = m if spherical else O.window_halfwidth(m, mprime)
    win, e0 = oracle_windows(model, Q, w, order)
    out = np.empty(len(Q))
    for i in range(len(Q)):
        if spherical:
            q0 = np.floor(Q[i]).astype(np.int32)
            assert np.all(q0 == Q[i]), "the spherical filter is sampled on the G grid"
            out[i] = O.lanczos_spherical(win[i], e0[i], m, 1, q0, (1, 1, 1), model.cell, model.n)[0, 0, 0]
        else:
            out[i] = O.lanczos_points(win[i], e0[i], m, Q[i:i + 1], mprime)[0]
    return out
