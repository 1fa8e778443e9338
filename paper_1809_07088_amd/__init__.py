"""Python binding of the dsx C-ABI (include/dsx.h): argument marshalling only.

Every step of the hot path runs in the gfx950 HIP library libdsx.so built in this
package directory (``paper_1809_07088_amd.build.build()``).  There is no Python or
CPU fallback: if the library is missing, loading it raises.

Device memory and streams come from PyTorch: pass CUDA (HIP) tensors for
device arrays and ``torch.cuda.current_stream()`` (the default) or any other
stream; NumPy arrays are passed as host memory.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsx.so")

NUCLEAR, MAGNETIC = 0, 1
NOALLOC_SCRATCH_BYTES = 96 * 1024 * 1024
HOST, DEVICE = 0, 1
OK, ERR_ARG, ERR_STATE, ERR_NOMEM, ERR_DEVICE, ERR_UNSUPPORTED, ERR_BUSY = 0, -1, -2, -3, -4, -5, -6
MAX_N, MAX_SITES, MAX_ORDER = 256, 64, 16


class DsxError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"dsx status {status}: {message}")
        self.status = status


class ModelDesc(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_double * 6), ("n", ctypes.c_int32 * 3), ("n_sites", ctypes.c_int32),
                ("frac", ctypes.c_void_p), ("pos_id", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("ff", ctypes.c_void_p), ("kind", ctypes.c_int32), ("has_occ", ctypes.c_int32),
                ("taylor_order", ctypes.c_int32), ("n_configs", ctypes.c_int32), ("norm_N", ctypes.c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("fields_per_site", ctypes.c_int32), ("total_fields", ctypes.c_int32),
                ("n_classes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("spectrum_bytes", ctypes.c_int64), ("device_bytes", ctypes.c_int64)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


EXPORTS = ("dsx_plan_query", "dsx_create_model", "dsx_set_sites", "dsx_set_sites_async", "dsx_set_grid",
           "dsx_compute_intensity", "dsx_compute_intensity_noalloc", "dsx_noise_filter", "dsx_destroy_model", "dsx_last_error",
           "dsx_version", "dsx_profile_enable", "dsx_profile_select", "dsx_profile_read", "dsx_profile_reset",
           "dsx_noise_filter_cutoff", "dsx_filter_points", "dsx_split_sites", "dsx_noise_filter_spherical",
           "dsx_batch_create", "dsx_batch_create_mode", "dsx_batch_query", "dsx_batch_run", "dsx_batch_destroy",
           "dsx_autotune", "dsx_tune_query", "dsx_tune_set_fft", "dsx_tune_query_fft",
           "dsx_tune_set", "dsx_server_create", "dsx_server_add_model", "dsx_server_submit", "dsx_server_wait",
           "dsx_server_stats_read", "dsx_server_destroy")

class BatchInfo(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("launches", ctypes.c_int32), ("dispatches", ctypes.c_int32),
                ("merged_nodes", ctypes.c_int32), ("unmerged_spill", ctypes.c_int32),
                ("merged_form_dispatches", ctypes.c_int32),
                ("per_model_ms", ctypes.c_float), ("merged_ms", ctypes.c_float)]


BATCH_AUTO, BATCH_PER_MODEL, BATCH_MERGED = 0, 1, 2


class ServerConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("queue_capacity", ctypes.c_int32), ("arena_bytes", ctypes.c_int64),
                ("max_round", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("model", ctypes.c_void_p), ("config", ctypes.c_int32), ("occ", ctypes.c_void_p),
                ("disp", ctypes.c_void_p), ("spin", ctypes.c_void_p), ("where", ctypes.c_int32),
                ("lanczos_m", ctypes.c_int32), ("oversample", ctypes.c_int32), ("out", ctypes.c_void_p)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("voxels", ctypes.c_int64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("span_s", ctypes.c_double), ("arena_bytes", ctypes.c_int64),
                ("arena_peak_bytes", ctypes.c_int64), ("slots", ctypes.c_int32),
                ("peak_in_flight", ctypes.c_int32), ("rounds", ctypes.c_int64),
                ("round_requests", ctypes.c_int64)]


_lib = None


def lib():
    """Load libdsx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1809_07088_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32 = ctypes.c_void_p, ctypes.c_int32
        L.dsx_plan_query.argtypes = [ctypes.POINTER(ModelDesc), ctypes.POINTER(PlanInfo)]
        L.dsx_create_model.argtypes = [ctypes.POINTER(ModelDesc), ctypes.POINTER(P)]
        L.dsx_set_sites.argtypes = [P, i32, P, P, P, i32]
        L.dsx_set_sites_async.argtypes = [P, i32, P, P, P, P]
        L.dsx_set_sites_async.restype = i32
        L.dsx_set_grid.argtypes = [P, P, P]
        L.dsx_compute_intensity.argtypes = [P, P, i32, P]
        L.dsx_compute_intensity_noalloc.argtypes = [P, P, P]
        L.dsx_compute_intensity_noalloc.restype = i32
        L.dsx_noise_filter.argtypes = [P, i32, i32, P, i32, P]
        L.dsx_noise_filter_cutoff.argtypes = [P, i32, i32, i32, P, i32, P]
        L.dsx_noise_filter_cutoff.restype = i32
        L.dsx_noise_filter_spherical.argtypes = [P, i32, i32, P, i32, P]
        L.dsx_noise_filter_spherical.restype = i32
        L.dsx_filter_points.argtypes = [P, i32, i32, ctypes.c_int64, P, P, i32, P]
        L.dsx_filter_points.restype = i32
        L.dsx_split_sites.argtypes = [P, i32, P, P, i32, P, P, ctypes.c_double, i32, ctypes.POINTER(i32),
                                      P, P, P, P]
        L.dsx_split_sites.restype = i32
        L.dsx_destroy_model.argtypes = [P]
        L.dsx_last_error.argtypes = []
        L.dsx_last_error.restype = ctypes.c_char_p
        L.dsx_version.restype = i32
        L.dsx_profile_enable.argtypes = [i32]
        L.dsx_profile_enable.restype = i32
        L.dsx_profile_select.argtypes = [ctypes.c_char_p]
        L.dsx_profile_select.restype = i32
        L.dsx_profile_read.argtypes = [P, i32]
        L.dsx_profile_read.restype = i32
        L.dsx_profile_reset.argtypes = []
        L.dsx_profile_reset.restype = i32
        L.dsx_batch_create.argtypes = [P, i32, i32, i32, P, ctypes.POINTER(P)]
        L.dsx_batch_create_mode.argtypes = [P, i32, i32, i32, P, i32, ctypes.POINTER(P)]
        L.dsx_batch_query.argtypes = [P, ctypes.POINTER(BatchInfo)]
        L.dsx_batch_run.argtypes = [P, P]
        L.dsx_batch_destroy.argtypes = [P]
        L.dsx_autotune.argtypes = [P, i32, P]
        L.dsx_tune_query.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.dsx_tune_set.argtypes = [P, ctypes.POINTER(i32)]
        L.dsx_tune_set_fft.argtypes = [P, P, i32]
        L.dsx_tune_set_fft.restype = i32
        L.dsx_tune_query_fft.argtypes = [P, P, ctypes.POINTER(i32)]
        L.dsx_tune_query_fft.restype = i32
        L.dsx_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(P)]
        L.dsx_server_add_model.argtypes = [P, ctypes.POINTER(ModelDesc), ctypes.POINTER(P)]
        L.dsx_server_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_int64)]
        L.dsx_server_wait.argtypes = [P, ctypes.c_int64, i32, ctypes.POINTER(i32)]
        L.dsx_server_stats_read.argtypes = [P, i32, ctypes.POINTER(ServerStats)]
        L.dsx_server_destroy.argtypes = [P]
        for f in ("dsx_batch_create", "dsx_batch_create_mode", "dsx_batch_query", "dsx_batch_run",
                  "dsx_batch_destroy", "dsx_autotune", "dsx_tune_query",
                  "dsx_tune_set", "dsx_server_create", "dsx_server_add_model", "dsx_server_submit", "dsx_server_wait",
                  "dsx_server_stats_read", "dsx_server_destroy"):
            getattr(L, f).restype = i32
        for f in ("dsx_plan_query", "dsx_create_model", "dsx_set_sites", "dsx_set_grid",
                  "dsx_compute_intensity", "dsx_compute_intensity_noalloc", "dsx_noise_filter", "dsx_destroy_model"):
            getattr(L, f).restype = i32
        _lib = L
    return _lib


def last_error() -> str:
    return lib().dsx_last_error().decode()


def _check(status):
    if status != OK:
        raise DsxError(status, last_error())


def _ptr_where(a, nelem=None):
    """(pointer, where, keepalive) of an input array: a numpy array (host memory,
    converted to contiguous float32 if needed) or a contiguous float32 torch tensor.
    nelem, when given, is the element count the library will read."""
    if a is None:
        return None, None, None
    if isinstance(a, np.ndarray):
        a = np.ascontiguousarray(a, dtype=np.float32)
        ptr, where, size = a.ctypes.data, HOST, a.size
    else:
        import torch
        if not isinstance(a, torch.Tensor):
            raise TypeError(f"unsupported array type {type(a)}")
        if a.dtype != torch.float32 or not a.is_contiguous():
            raise ValueError("device arrays must be contiguous float32 tensors")
        ptr, where, size = a.data_ptr(), (DEVICE if a.is_cuda else HOST), a.numel()
    if nelem is not None and size != nelem:
        raise ValueError(f"input array has {size} elements, the model reads {nelem}")
    return ptr, where, a


def _ptr_out(a, nelem=None):
    """(pointer, where) of an output array, written in place and never copied: a
    writable C-contiguous float32 numpy array (host) or a contiguous float32 torch
    tensor.  nelem, when given, is the element count the library will write."""
    if isinstance(a, np.ndarray):
        if a.dtype != np.float32 or not a.flags.c_contiguous or not a.flags.writeable:
            raise ValueError("host outputs must be writable C-contiguous float32 numpy arrays")
        ptr, where, size = a.ctypes.data, HOST, a.size
    else:
        import torch
        if not isinstance(a, torch.Tensor):
            raise TypeError(f"unsupported output type {type(a)}")
        if a.dtype != torch.float32 or not a.is_contiguous():
            raise ValueError("outputs must be contiguous float32 tensors")
        ptr, where, size = a.data_ptr(), (DEVICE if a.is_cuda else HOST), a.numel()
    if nelem is not None and size != nelem:
        raise ValueError(f"output array has {size} elements, the call writes {nelem}")
    return ptr, where


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def make_desc(cell, n, frac, b, kind=NUCLEAR, taylor_order=0, n_configs=1, has_occ=False,
              ff=None, pos_id=None, norm_N=0.0):
    """A dsx_model_desc plus the arrays it points to (kept alive by the caller)."""
    frac = np.ascontiguousarray(frac, dtype=np.float64).reshape(-1, 3)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    ffa = None if ff is None else np.ascontiguousarray(ff, dtype=np.float64).reshape(-1, 7)
    pid = None if pos_id is None else np.ascontiguousarray(pos_id, dtype=np.int32)
    d = ModelDesc()
    d.cell[:] = [float(v) for v in cell]
    d.n[:] = [int(v) for v in n]
    d.n_sites = frac.shape[0]
    d.frac = frac.ctypes.data
    d.b = b.ctypes.data
    d.ff = None if ffa is None else ffa.ctypes.data
    d.pos_id = None if pid is None else pid.ctypes.data
    d.kind, d.has_occ, d.taylor_order = int(kind), int(bool(has_occ)), int(taylor_order)
    d.n_configs, d.norm_N = int(n_configs), float(norm_N)
    return d, (frac, b, ffa, pid)


def plan_query(**kw) -> PlanInfo:
    d, keep = make_desc(**kw)
    info = PlanInfo()
    _check(lib().dsx_plan_query(ctypes.byref(d), ctypes.byref(info)))
    return info


def create_model(**kw) -> int:
    d, keep = make_desc(**kw)
    h = ctypes.c_void_p()
    _check(lib().dsx_create_model(ctypes.byref(d), ctypes.byref(h)))
    return h.value


def set_sites(model, config, occ=None, disp=None, spin=None, sizes=(None, None, None)):
    ptrs = [_ptr_where(a, z) for a, z in zip((occ, disp, spin), sizes)]
    wheres = {w for (_, w, _) in ptrs if w is not None}
    if len(wheres) > 1:
        raise ValueError("occ, disp and spin must all be host or all device arrays")
    where = wheres.pop() if wheres else HOST
    _check(lib().dsx_set_sites(model, int(config), ptrs[0][0], ptrs[1][0], ptrs[2][0], where))


def set_sites_async(model, config, occ=None, disp=None, spin=None, stream=None, sizes=(None, None, None)):
    """Stream-ordered site upload from device tensors (kept unchanged until it has run)."""
    ptrs = [_ptr_where(a, z) for a, z in zip((occ, disp, spin), sizes)]
    if any(w == HOST for (_, w, _) in ptrs):
        raise ValueError("set_sites_async takes device tensors")
    _check(lib().dsx_set_sites_async(model, int(config), ptrs[0][0], ptrs[1][0], ptrs[2][0],
                                     _stream_handle(stream)))


def set_grid(model, g0, count):
    g = np.ascontiguousarray(g0, dtype=np.int32)
    c = np.ascontiguousarray(count, dtype=np.int32)
    _check(lib().dsx_set_grid(model, g.ctypes.data, c.ctypes.data))


def compute_intensity(model, out, stream=None, nelem=None):
    p, where = _ptr_out(out, nelem)
    st = _stream_handle(stream) if where == DEVICE else None
    _check(lib().dsx_compute_intensity(model, p, where, st))
    return out


def compute_intensity_noalloc(model, out, stream=None, nelem=None):
    """dsx_compute_intensity_noalloc: the same I(G) into a device tensor, allocating
    nothing (device scratch shared by every such call on the device)."""
    p, where = _ptr_out(out, nelem)
    if where != DEVICE:
        raise ValueError("compute_intensity_noalloc writes device memory only")
    _check(lib().dsx_compute_intensity_noalloc(model, p, _stream_handle(stream)))
    return out


def noise_filter(model, lanczos_m, oversample, out, stream=None, nelem=None):
    p, where = _ptr_out(out, nelem)
    st = _stream_handle(stream) if where == DEVICE else None
    _check(lib().dsx_noise_filter(model, int(lanczos_m), int(oversample), p, where, st))
    return out


def noise_filter_cutoff(model, lanczos_m, mprime, oversample, out, stream=None, nelem=None):
    """dsx_noise_filter_cutoff: the filter with the m' cutoff modification."""
    p, where = _ptr_out(out, nelem)
    st = _stream_handle(stream) if where == DEVICE else None
    _check(lib().dsx_noise_filter_cutoff(model, int(lanczos_m), int(mprime), int(oversample), p, where, st))
    return out


def noise_filter_spherical(model, lanczos_m, oversample, out, stream=None, nelem=None):
    """dsx_noise_filter_spherical: the filter with the spherical cutoff W_r."""
    p, where = _ptr_out(out, nelem)
    st = _stream_handle(stream) if where == DEVICE else None
    _check(lib().dsx_noise_filter_spherical(model, int(lanczos_m), int(oversample), p, where, st))
    return out


def filter_points(model, lanczos_m, q, out, mprime=2, stream=None):
    """dsx_filter_points: the filter at arbitrary points q [npts][3] (float64 host
    array, units of the supercell Bragg grid) into out [npts]."""
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
    p, where = _ptr_out(out, q.shape[0])
    st = _stream_handle(stream) if where == DEVICE else None
    _check(lib().dsx_filter_points(model, int(lanczos_m), int(mprime), q.shape[0],
                                   q.ctypes.data_as(ctypes.c_void_p), p, where, st))
    return out


def split_sites(n, frac, b, disp, occ=None, tol=0.0, max_sites=64):
    """dsx_split_sites (host only): the split-site form of a model whose displacements
    take few values.  disp [M][S][n1][n2][n3][3], occ [M][S][n1][n2][n3] or None.
    Returns (frac [S'][3], b [S'], parent [S'], occ [M][S'][n1][n2][n3])."""
    n = np.ascontiguousarray(n, dtype=np.int32)
    frac = np.ascontiguousarray(frac, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    disp = np.ascontiguousarray(disp, dtype=np.float32)
    M, S = disp.shape[0], disp.shape[1]
    occ_in = None if occ is None else np.ascontiguousarray(occ, dtype=np.float32)
    fo = np.zeros((max_sites, 3)); bo = np.zeros(max_sites)
    po = np.zeros(max_sites, dtype=np.int32)
    oo = np.zeros((M, max_sites) + tuple(int(v) for v in n), dtype=np.float32)
    ns = ctypes.c_int32(0)
    vp = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    _check(lib().dsx_split_sites(vp(n), S, vp(frac), vp(b), M, vp(occ_in), vp(disp), float(tol), int(max_sites),
                                 ctypes.byref(ns), vp(fo), vp(bo), vp(po), vp(oo)))
    k = ns.value
    return fo[:k].copy(), bo[:k].copy(), po[:k].copy(), np.ascontiguousarray(oo[:, :k])


def destroy_model(model):
    _check(lib().dsx_destroy_model(model))


def version() -> int:
    return int(lib().dsx_version())


def profile_enable(on=True):
    _check(lib().dsx_profile_enable(1 if on else 0))


def profile_select(kernel=None):
    """Time only `kernel` (a name as profile_read reports it), or every kernel for None."""
    _check(lib().dsx_profile_select(None if kernel is None else kernel.encode()))


def profile_reset():
    _check(lib().dsx_profile_reset())


def profile_read() -> dict:
    """{kernel name: (launches, total ms)} accumulated since the last reset."""
    n = lib().dsx_profile_read(None, 0)
    arr = (KernelStat * max(n, 1))()
    n = lib().dsx_profile_read(ctypes.cast(arr, ctypes.c_void_p), n)
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n)}


def autotune(model, lanczos_m=0, stream=None):
    _check(lib().dsx_autotune(model, int(lanczos_m), _stream_handle(stream)))


def tune_query(model):
    """The plan choices of a model (dsx_tune_query): recombination form, FFT fields
    per plane block, filter planes per block, and whether they were tuned."""
    c = (ctypes.c_int32 * 3)()
    t = ctypes.c_int32(0)
    _check(lib().dsx_tune_query(model, c, ctypes.byref(t)))
    return {"recombine_form": int(c[0]), "fft_fields_per_block": int(c[1]),
            "filter_planes_per_block": int(c[2]), "tuned": bool(t.value)}


def tune_query_fft(model):
    """The FFT knobs of a model (dsx_tune_query_fft): per axis the radix sequence of its
    passes, and the axis-1 column tile (0 = by edge)."""
    r = (ctypes.c_int32 * 48)()
    t = ctypes.c_int32(0)
    _check(lib().dsx_tune_query_fft(model, r, ctypes.byref(t)))
    return {"radices": [[int(x) for x in r[16 * a:16 * a + 16] if x] for a in range(3)],
            "col_tile": int(t.value)}


def tune_set_fft(model, radices=None, col_tile=0):
    """Set the FFT knobs without timing (dsx_tune_set_fft): radices is None or three
    sequences (each product = the axis's edge)."""
    arr = None
    if radices is not None:
        if len(radices) != 3 or any(len(r) > 16 for r in radices):
            raise ValueError("three radix sequences of at most 16 radices")
        arr = (ctypes.c_int32 * 48)()
        for a, rs in enumerate(radices):
            for i, v in enumerate(rs):
                arr[16 * a + i] = int(v)
    _check(lib().dsx_tune_set_fft(model, arr, int(col_tile)))


def tune_set(model, recombine_form, fft_fields_per_block, filter_planes_per_block):
    """Set the plan choices without timing (dsx_tune_set); the model counts as tuned."""
    c = (ctypes.c_int32 * 3)(int(recombine_form), int(fft_fields_per_block), int(filter_planes_per_block))
    _check(lib().dsx_tune_set(model, c))


class Batch:
    """A recorded launch sequence over several models (dsx_batch_*): run() replays it.
    mode: BATCH_AUTO (time both forms, keep the faster), BATCH_PER_MODEL or BATCH_MERGED."""

    def __init__(self, models, outs, lanczos_m=0, oversample=1, mode=BATCH_AUTO):
        handles = [m.handle if isinstance(m, Model) else m for m in models]
        if len(handles) != len(outs) or not handles:
            raise ValueError("one output per model, at least one model")
        self._keep = (list(models), list(outs))
        # device outputs: contiguous float32 tensors, large enough for their model's box
        # (checked where the model is a Model, whose grid the binding knows)
        sv = int(oversample) if lanczos_m else 1
        ptrs = []
        for mdl, o in zip(models, outs):
            nelem = mdl._box_voxels(sv) if isinstance(mdl, Model) else None
            p, w = _ptr_out(o, nelem)
            if w != DEVICE:
                raise ValueError("batch outputs must be device tensors")
            ptrs.append(p)
        arr_m = (ctypes.c_void_p * len(handles))(*handles)
        arr_o = (ctypes.c_void_p * len(outs))(*ptrs)
        h = ctypes.c_void_p()
        _check(lib().dsx_batch_create_mode(ctypes.cast(arr_m, ctypes.c_void_p), len(handles), int(lanczos_m),
                                           int(oversample), ctypes.cast(arr_o, ctypes.c_void_p), int(mode),
                                           ctypes.byref(h)))
        self.handle = h.value

    def info(self):
        """The form the batch runs and its graph: dict of dsx_batch_info."""
        i = BatchInfo()
        _check(lib().dsx_batch_query(self.handle, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in BatchInfo._fields_}

    def run(self, stream=None):
        _check(lib().dsx_batch_run(self.handle, _stream_handle(stream)))

    def close(self):
        if self.handle:
            _check(lib().dsx_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Model:
    """Convenience owner of one dsx model handle; checks array sizes against the model
    before every call that reads or writes caller memory."""

    def __init__(self, **kw):
        self.desc_kw = dict(kw)
        self.handle = create_model(**kw)
        self.g0 = self.count = None

    def _site_sizes(self):
        kw = self.desc_kw
        n = [int(v) for v in kw["n"]]
        S = np.asarray(kw["frac"]).reshape(-1, 3).shape[0]
        per = S * n[0] * n[1] * n[2]
        return (per, 3 * per, 3 * per)

    def _box_voxels(self, s=1):
        if self.count is None:
            return None          # the library reports the missing grid
        return int(np.prod([s * int(c) for c in self.count]))

    def set_sites(self, config, occ=None, disp=None, spin=None):
        set_sites(self.handle, config, occ, disp, spin, sizes=self._site_sizes())

    def set_sites_async(self, config, occ=None, disp=None, spin=None, stream=None):
        set_sites_async(self.handle, config, occ, disp, spin, stream, sizes=self._site_sizes())

    def set_grid(self, g0, count):
        set_grid(self.handle, g0, count)
        self.g0, self.count = tuple(int(v) for v in g0), tuple(int(v) for v in count)

    def compute_intensity(self, out, stream=None):
        return compute_intensity(self.handle, out, stream, nelem=self._box_voxels())

    def compute_intensity_noalloc(self, out, stream=None):
        return compute_intensity_noalloc(self.handle, out, stream, nelem=self._box_voxels())

    def noise_filter(self, lanczos_m, oversample, out, stream=None):
        return noise_filter(self.handle, lanczos_m, oversample, out, stream,
                            nelem=self._box_voxels(int(oversample)))

    def noise_filter_cutoff(self, lanczos_m, mprime, oversample, out, stream=None):
        return noise_filter_cutoff(self.handle, lanczos_m, mprime, oversample, out, stream,
                                   nelem=self._box_voxels(int(oversample)))

    def noise_filter_spherical(self, lanczos_m, oversample, out, stream=None):
        return noise_filter_spherical(self.handle, lanczos_m, oversample, out, stream,
                                      nelem=self._box_voxels(int(oversample)))

    def filter_points(self, lanczos_m, q, out, mprime=2, stream=None):
        return filter_points(self.handle, lanczos_m, q, out, mprime, stream)

    def autotune(self, lanczos_m=0, stream=None):
        autotune(self.handle, lanczos_m, stream)

    def tune_query(self):
        return tune_query(self.handle)

    def tune_set(self, recombine_form, fft_fields_per_block, filter_planes_per_block):
        tune_set(self.handle, recombine_form, fft_fields_per_block, filter_planes_per_block)

    def tune_query_fft(self):
        return tune_query_fft(self.handle)

    def tune_set_fft(self, radices=None, col_tile=0):
        tune_set_fft(self.handle, radices, col_tile)

    def close(self):
        if self.handle:
            destroy_model(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ServedModel(Model):
    """A resident model owned by a Server (released with it)."""

    def __init__(self, server, **kw):
        self.desc_kw = dict(kw)
        d, keep = make_desc(**kw)
        h = ctypes.c_void_p()
        _check(lib().dsx_server_add_model(server.handle, ctypes.byref(d), ctypes.byref(h)))
        self.handle = h.value
        self.server = server
        self.g0 = self.count = None

    def close(self):
        self.handle = None


class Server:
    """Continuous-batching request server over resident models (dsx_server_*).
    max_round: requests merged into one round (0 = 16, 1 = one request per slot)."""

    def __init__(self, slots=4, queue_capacity=1024, arena_bytes=8 << 30, max_round=0):
        c = ServerConfig(int(slots), int(queue_capacity), int(arena_bytes), int(max_round))
        h = ctypes.c_void_p()
        _check(lib().dsx_server_create(ctypes.byref(c), ctypes.byref(h)))
        self.handle = h.value
        self._keep = {}

    def add_model(self, **kw) -> ServedModel:
        return ServedModel(self, **kw)

    def submit(self, model, out, config=-1, occ=None, disp=None, spin=None, lanczos_m=0, oversample=1):
        """Queue a request; returns its ticket (DsxError ERR_BUSY when the queue is full)."""
        ptrs = [_ptr_where(a, z) for a, z in zip((occ, disp, spin), model._site_sizes())]
        wheres = {w for (_, w, _) in ptrs if w is not None}
        if len(wheres) > 1:
            raise ValueError("occ, disp and spin must all be host or all device arrays")
        nelem = model._box_voxels(int(oversample) if lanczos_m else 1)
        p_out, w_out = _ptr_out(out, nelem)
        if w_out != DEVICE:
            raise ValueError("out must be a device tensor")
        r = Request(model.handle, int(config), ptrs[0][0], ptrs[1][0], ptrs[2][0],
                    wheres.pop() if wheres else DEVICE, int(lanczos_m), int(oversample), p_out)
        t = ctypes.c_int64()
        _check(lib().dsx_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = (out, [k for (_, _, k) in ptrs])
        return t.value

    def wait(self, ticket, timeout_ms=-1):
        """True once the request finished (raises DsxError if it failed); False on timeout."""
        res = ctypes.c_int32()
        st = lib().dsx_server_wait(self.handle, int(ticket), int(timeout_ms), ctypes.byref(res))
        if st == ERR_BUSY:
            return False
        _check(st)
        self._keep.pop(ticket, None)
        if res.value != OK:
            raise DsxError(res.value, last_error())
        return True

    def stats(self, reset=False) -> dict:
        z = ServerStats()
        _check(lib().dsx_server_stats_read(self.handle, 1 if reset else 0, ctypes.byref(z)))
        return {f: getattr(z, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self.handle:
            _check(lib().dsx_server_destroy(self.handle))
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
