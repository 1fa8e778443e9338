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
