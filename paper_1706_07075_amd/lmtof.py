"""Thin ctypes binding of liblmtof.so (argument marshalling only).

Every function keeps the name of the C entry point it wraps (include/lmtof.h)
and raises LmtofError on a non-zero return code.  Arrays may be NumPy arrays
(host memory) or torch tensors on the GPU (device memory, passed by pointer);
all arithmetic runs inside the library's HIP kernels.  There is no fallback:
if the shared library is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Any, Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblmtof.so")

LMTOF_OK = 0
LMTOF_EINVAL = -1
LMTOF_ESTATE = -2
LMTOF_ENOMEM = -3
LMTOF_EHIP = -4
LMTOF_EUNSUPPORTED = -5
LMTOF_EAGAIN = -6

LMTOF_FMT_F32X7 = 0
LMTOF_FMT_PACKED16 = 1
LMTOF_MEM_HOST = 0
LMTOF_MEM_DEVICE = 1

LMTOF_OPT_STORAGE = 1
LMTOF_OPT_SORT = 2
LMTOF_OPT_SENS_NPHI = 3
LMTOF_OPT_EVENTS_PER_THREAD = 5
LMTOF_OPT_SORT_CELL_MM = 6
LMTOF_OPT_MEDIAN_SIEVE = 8
LMTOF_OPT_FORWARD = 9
LMTOF_FORWARD_BRICKS = 0
LMTOF_FORWARD_EVENTS = 1
LMTOF_REQ_BACKGROUND = 1
LMTOF_OPT_BRICK_CHUNKS = 10
LMTOF_TUNE_MAX_CANDIDATES = 16

ERROR_NAMES = {0: "OK", -1: "EINVAL", -2: "ESTATE", -3: "ENOMEM", -4: "EHIP", -5: "EUNSUPPORTED", -6: "EAGAIN"}


class LmtofError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lmtof {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code
        self.msg = msg


class lmtof_geometry(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("reserved0", C.c_int32),
                ("vx", C.c_double), ("vy", C.c_double), ("vz", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
                ("scanner_radius", C.c_double), ("scanner_half_length", C.c_double),
                ("max_axial_angle_deg", C.c_double), ("tof_fwhm_ps", C.c_double),
                ("tof_trunc_sigmas", C.c_double), ("c_mm_per_ps", C.c_double)]


class lmtof_iter_stats(C.Structure):
    _fields_ = [("iter", C.c_int32), ("reserved0", C.c_int32), ("n_eff", C.c_int64), ("sum_sx", C.c_double),
                ("loglik", C.c_double), ("ms", C.c_float), ("project_ms", C.c_float),
                ("forward_ms", C.c_float), ("back_ms", C.c_float), ("back_kernel_ms", C.c_float),
                ("update_ms", C.c_float), ("forward_kernel_ms", C.c_float)]


class lmtof_tune_candidate(C.Structure):
    _fields_ = [("forward", C.c_int32), ("events_per_thread", C.c_int32), ("brick_chunks", C.c_int32),
                ("reserved0", C.c_int32), ("pass_ms", C.c_float), ("build_ms", C.c_float)]


class lmtof_tune_result(C.Structure):
    _fields_ = [("forward", C.c_int32), ("events_per_thread", C.c_int32), ("brick_chunks", C.c_int32),
                ("n_candidates", C.c_int32), ("cached", C.c_int32), ("reserved0", C.c_int32),
                ("cand", lmtof_tune_candidate * LMTOF_TUNE_MAX_CANDIDATES)]


class lmtof_request(C.Structure):
    _fields_ = [("geometry", lmtof_geometry), ("events", C.c_void_p), ("n_events", C.c_int64),
                ("format", C.c_int32), ("mem", C.c_int32), ("n_iter", C.c_int32), ("storage", C.c_int32),
                ("flags", C.c_int32), ("reserved0", C.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")

# PyTorch wheels bundle their own HIP runtime under the SONAME libamdhip64.so.7.
# Loading torch first lets the dynamic linker resolve this library's HIP
# dependency to that same runtime, so one HIP runtime serves the process and
# device pointers move freely between torch tensors and the library.  If
# this library loaded first, torch would bring a second runtime that cannot
# see the GPU.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_lib = C.CDLL(LIB_PATH)
_P = C.c_void_p
_i64 = C.c_int64
_sig = {
    "lmtof_create": ([C.POINTER(_P), C.c_int, _P], C.c_int),
    "lmtof_destroy": ([_P], C.c_int),
    "lmtof_last_error": ([_P], C.c_char_p),
    "lmtof_check_geometry": ([C.POINTER(lmtof_geometry), C.c_char_p, C.c_int64], C.c_int),
    "lmtof_set_option": ([_P, C.c_int, _i64], C.c_int),
    "lmtof_get_option": ([_P, C.c_int, C.POINTER(_i64)], C.c_int),
    "lmtof_set_geometry": ([_P, C.POINTER(lmtof_geometry)], C.c_int),
    "lmtof_load_events": ([_P, _P, _i64, C.c_int, C.c_int], C.c_int),
    "lmtof_num_events": ([_P, C.POINTER(_i64)], C.c_int),
    "lmtof_read_packed_events": ([_P, _P, _i64, C.c_int], C.c_int),
    "lmtof_compute_sensitivity": ([_P], C.c_int),
    "lmtof_read_sensitivity": ([_P, _P, _i64, C.c_int], C.c_int),
    "lmtof_set_sensitivity": ([_P, _P, _i64, C.c_int], C.c_int),
    "lmtof_set_image": ([_P, _P, _i64, C.c_int], C.c_int),
    "lmtof_read_image": ([_P, _P, _i64, C.c_int], C.c_int),
    "lmtof_iterate": ([_P, C.c_int, C.POINTER(lmtof_iter_stats)], C.c_int),
    "lmtof_forward_project": ([_P, _P, _i64, _P, _i64, C.c_int], C.c_int),
    "lmtof_back_project": ([_P, _P, _i64, _P, _i64, C.c_int], C.c_int),
    "lmtof_median_filter": ([_P, _P, _i64, _P, _i64, C.c_int], C.c_int),
    "lmtof_tof_keep": ([_P, _P, _i64, _P, _i64, C.c_int], C.c_int),
    "lmtof_attenuation_factors": ([_P, _P, _i64, _P, _i64, C.c_int], C.c_int),
    "lmtof_set_event_weights": ([_P, _P, _i64, C.c_int], C.c_int),
    "lmtof_sampled_forward_project": ([_P, _P, _i64, _P, _i64, C.c_int], C.c_int),
    "lmtof_sampled_back_project": ([_P, _P, _i64, _P, _i64, C.c_int], C.c_int),
    "lmtof_sampled_forward_project_noalloc": ([_P, _P, _i64, _P, _i64], C.c_int),
    "lmtof_count_segments": ([_P, C.POINTER(_i64), C.POINTER(_i64)], C.c_int),
    "lmtof_autotune": ([_P, C.c_int, C.POINTER(lmtof_tune_result)], C.c_int),
    "lmtof_set_regions": ([_P, C.POINTER(C.c_int32), C.c_int, C.c_int], C.c_int),
    "lmtof_region_info": ([_P, C.c_int, C.POINTER(C.c_int32), C.POINTER(_i64)], C.c_int),
    "lmtof_read_region_image": ([_P, C.c_int, _P, _i64, C.c_int], C.c_int),
    "lmtof_clear_regions": ([_P], C.c_int),
    "lmtof_event_regions": ([_P, _P, _i64, C.c_int], C.c_int),
    "lmtof_pool_create": ([C.POINTER(_P), C.c_int, _P, _i64], C.c_int),
    "lmtof_pool_destroy": ([_P], C.c_int),
    "lmtof_pool_last_error": ([_P], C.c_char_p),
    "lmtof_pool_request_bytes": ([C.POINTER(lmtof_request), C.POINTER(_i64)], C.c_int),
    "lmtof_pool_submit": ([_P, C.POINTER(lmtof_request), C.POINTER(_i64)], C.c_int),
    "lmtof_pool_step": ([_P, C.POINTER(C.c_int)], C.c_int),
    "lmtof_pool_poll": ([_P, _i64, C.POINTER(C.c_int), _P, _i64, C.c_int], C.c_int),
    "lmtof_pool_info": ([_P, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def lmtof_last_error(ctx) -> str:
    m = _lib.lmtof_last_error(ctx)
    return m.decode() if m else ""


def _check(rc: int, ctx) -> None:
    if rc != LMTOF_OK:
        raise LmtofError(rc, lmtof_last_error(ctx))


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _in(a, dtype):
    """(pointer, mem kind, keep-alive) for an input array."""
    if a is None:
        return None, LMTOF_MEM_HOST, None
    if _is_torch(a):
        import torch
        if a.is_cuda:
            if not a.is_contiguous():
                raise ValueError("device tensors must be contiguous")
            torch.cuda.current_stream(a.device).synchronize()
            return C.c_void_p(a.data_ptr()), LMTOF_MEM_DEVICE, a
        a = a.numpy()
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data_as(C.c_void_p), LMTOF_MEM_HOST, arr


def _out(out, n, dtype):
    if out is None:
        out = np.empty(n, dtype=dtype)
    if _is_torch(out):
        if not out.is_cuda:
            raise ValueError("torch outputs must be on the GPU")
        return out, C.c_void_p(out.data_ptr()), LMTOF_MEM_DEVICE
    if not (isinstance(out, np.ndarray) and out.dtype == dtype and out.flags.c_contiguous and out.size == n):
        raise ValueError(f"output must be a contiguous {dtype} array of {n} elements")
    return out, out.ctypes.data_as(C.c_void_p), LMTOF_MEM_HOST


def geometry_struct(g: Dict[str, Any]) -> lmtof_geometry:
    s = lmtof_geometry()
    for k in ("nx", "ny", "nz"):
        setattr(s, k, int(g[k]))
    for k in ("vx", "vy", "vz", "x0", "y0", "z0", "scanner_radius", "scanner_half_length"):
        setattr(s, k, float(g[k]))
    s.max_axial_angle_deg = float(g.get("max_axial_angle_deg", 0.0))
    s.tof_fwhm_ps = float(g.get("tof_fwhm_ps", 0.0))
    s.tof_trunc_sigmas = float(g.get("tof_trunc_sigmas", 0.0))
    s.c_mm_per_ps = float(g.get("c_mm_per_ps", 0.0))
    return s


# ---------------------------------------------------------------- wrappers
def lmtof_create(hip_device: int = 0, hip_stream: Optional[int] = None):
    h = C.c_void_p()
    rc = _lib.lmtof_create(C.byref(h), hip_device, C.c_void_p(hip_stream) if hip_stream else None)
    _check(rc, None)
    return h


def lmtof_destroy(ctx) -> None:
    _check(_lib.lmtof_destroy(ctx), None)


def lmtof_check_geometry(g) -> str:
    """Host-only validation; returns '' if valid, else the reason."""
    buf = C.create_string_buffer(512)
    gs = g if isinstance(g, lmtof_geometry) else geometry_struct(g)
    rc = _lib.lmtof_check_geometry(C.byref(gs), buf, len(buf))
    return "" if rc == LMTOF_OK else buf.value.decode()


def lmtof_set_option(ctx, key: int, value: int) -> None:
    _check(_lib.lmtof_set_option(ctx, key, value), ctx)


def lmtof_get_option(ctx, key: int) -> int:
    v = C.c_int64()
    _check(_lib.lmtof_get_option(ctx, key, C.byref(v)), ctx)
    return v.value


def lmtof_set_geometry(ctx, g) -> None:
    gs = g if isinstance(g, lmtof_geometry) else geometry_struct(g)
    _check(_lib.lmtof_set_geometry(ctx, C.byref(gs)), ctx)


def lmtof_load_events(ctx, ev, fmt: Optional[int] = None) -> None:
    """ev: float32 (n, 7) or packed int16 (n, 8); NumPy or a GPU tensor."""
    if fmt is None:
        dt = str(ev.dtype)
        fmt = LMTOF_FMT_PACKED16 if "int16" in dt else LMTOF_FMT_F32X7
    per = 7 if fmt == LMTOF_FMT_F32X7 else 8
    n = int(np.prod(ev.shape)) // per
    p, mem, keep = _in(ev, np.float32 if fmt == LMTOF_FMT_F32X7 else np.int16)
    _check(_lib.lmtof_load_events(ctx, p, n, fmt, mem), ctx)


def lmtof_num_events(ctx) -> int:
    v = C.c_int64()
    _check(_lib.lmtof_num_events(ctx, C.byref(v)), ctx)
    return v.value


def lmtof_read_packed_events(ctx, out=None):
    n = lmtof_num_events(ctx)
    o, p, mem = _out(out, n * 8, np.int16)
    _check(_lib.lmtof_read_packed_events(ctx, p, n, mem), ctx)
    return o.reshape(n, 8) if isinstance(o, np.ndarray) else o


def lmtof_compute_sensitivity(ctx) -> None:
    _check(_lib.lmtof_compute_sensitivity(ctx), ctx)


def lmtof_read_sensitivity(ctx, n: int, out=None):
    o, p, mem = _out(out, n, np.float32)
    _check(_lib.lmtof_read_sensitivity(ctx, p, n, mem), ctx)
    return o


def lmtof_set_sensitivity(ctx, s) -> None:
    p, mem, keep = _in(s, np.float32)
    _check(_lib.lmtof_set_sensitivity(ctx, p, int(np.prod(s.shape)), mem), ctx)


def lmtof_set_image(ctx, x0=None) -> None:
    if x0 is None:
        _check(_lib.lmtof_set_image(ctx, None, 0, LMTOF_MEM_HOST), ctx)
        return
    p, mem, keep = _in(x0, np.float32)
    _check(_lib.lmtof_set_image(ctx, p, int(np.prod(x0.shape)), mem), ctx)


def lmtof_read_image(ctx, n: int, out=None):
    o, p, mem = _out(out, n, np.float32)
    _check(_lib.lmtof_read_image(ctx, p, n, mem), ctx)
    return o


def lmtof_iterate(ctx, n_iter: int):
    st = (lmtof_iter_stats * n_iter)()
    _check(_lib.lmtof_iterate(ctx, n_iter, st), ctx)
    return [dict(iter=s.iter, n_eff=s.n_eff, sum_sx=s.sum_sx, loglik=s.loglik, ms=s.ms, project_ms=s.project_ms,
                 forward_ms=s.forward_ms, forward_kernel_ms=s.forward_kernel_ms, back_ms=s.back_ms,
                 back_kernel_ms=s.back_kernel_ms, update_ms=s.update_ms) for s in st]


def lmtof_forward_project(ctx, x, n_events: int, out=None):
    p, mem, keep = _in(x, np.float32)
    if mem == LMTOF_MEM_DEVICE and out is None:
        import torch
        out = torch.empty(n_events, dtype=torch.float32, device=x.device)
    o, po, memo = _out(out, n_events, np.float32)
    if memo != mem:
        raise ValueError("x and f must both be host or both be device arrays")
    _check(_lib.lmtof_forward_project(ctx, p, int(np.prod(x.shape)), po, n_events, mem), ctx)
    return o


def lmtof_back_project(ctx, w, n_voxels: int, out=None):
    p, mem, keep = _in(w, np.float32)
    if mem == LMTOF_MEM_DEVICE and out is None:
        import torch
        out = torch.empty(n_voxels, dtype=torch.float32, device=w.device)
    o, po, memo = _out(out, n_voxels, np.float32)
    if memo != mem:
        raise ValueError("w and b must both be host or both be device arrays")
    _check(_lib.lmtof_back_project(ctx, p, int(np.prod(w.shape)), po, n_voxels, mem), ctx)
    return o


def lmtof_median_filter(ctx, x, n_voxels: int, out=None):
    p, mem, keep = _in(x, np.float32)
    if mem == LMTOF_MEM_DEVICE and out is None:
        import torch
        out = torch.empty(n_voxels, dtype=torch.float32, device=x.device)
    o, po, memo = _out(out, n_voxels, np.float32)
    if memo != mem:
        raise ValueError("x and y must both be host or both be device arrays")
    _check(_lib.lmtof_median_filter(ctx, p, int(np.prod(x.shape)), po, n_voxels, mem), ctx)
    return o


def lmtof_tof_keep(ctx, mask, n_events: int, out=None):
    """uint8 keep flag per loaded event (caller order) of the TOF scatter rejection."""
    p, mem, keep_alive = _in(mask, np.uint8)
    if mem == LMTOF_MEM_DEVICE and out is None:
        import torch
        out = torch.empty(n_events, dtype=torch.uint8, device=mask.device)
    o, po, memo = _out(out, n_events, np.uint8)
    if memo != mem:
        raise ValueError("mask and keep must both be host or both be device arrays")
    _check(_lib.lmtof_tof_keep(ctx, p, int(np.prod(mask.shape)), po, n_events, mem), ctx)
    return o


def lmtof_attenuation_factors(ctx, mu, n_events: int, out=None):
    p, mem, keep_alive = _in(mu, np.float32)
    if mem == LMTOF_MEM_DEVICE and out is None:
        import torch
        out = torch.empty(n_events, dtype=torch.float32, device=mu.device)
    o, po, memo = _out(out, n_events, np.float32)
    if memo != mem:
        raise ValueError("mu and acf must both be host or both be device arrays")
    _check(_lib.lmtof_attenuation_factors(ctx, p, int(np.prod(mu.shape)), po, n_events, mem), ctx)
    return o


def lmtof_set_event_weights(ctx, w) -> None:
    if w is None:
        _check(_lib.lmtof_set_event_weights(ctx, None, 0, LMTOF_MEM_HOST), ctx)
        return
    p, mem, keep_alive = _in(w, np.float32)
    _check(_lib.lmtof_set_event_weights(ctx, p, int(np.prod(w.shape)), mem), ctx)


def _project_call(fn, ctx, a, n_out):
    p, mem, keep_alive = _in(a, np.float32)
    out = None
    if mem == LMTOF_MEM_DEVICE:
        import torch
        out = torch.empty(n_out, dtype=torch.float32, device=a.device)
    o, po, memo = _out(out, n_out, np.float32)
    _check(fn(ctx, p, int(np.prod(a.shape)), po, n_out, mem), ctx)
    return o


def lmtof_sampled_forward_project(ctx, x, n_events: int):
    return _project_call(_lib.lmtof_sampled_forward_project, ctx, x, n_events)


def lmtof_sampled_forward_project_noalloc(ctx, x, f):
    """x and f: contiguous float32 tensors on the context's GPU (f holds
    the loaded event count); f is filled in place, nothing is allocated."""
    for a in (x, f):
        if not (_is_torch(a) and a.is_cuda and a.is_contiguous() and str(a.dtype) == "torch.float32"):
            raise ValueError("x and f must be contiguous float32 tensors on the GPU")
    import torch
    torch.cuda.current_stream(x.device).synchronize()
    _check(_lib.lmtof_sampled_forward_project_noalloc(ctx, C.c_void_p(x.data_ptr()), x.numel(),
                                                      C.c_void_p(f.data_ptr()), f.numel()), ctx)
    return f


def lmtof_sampled_back_project(ctx, r, n_voxels: int):
    return _project_call(_lib.lmtof_sampled_back_project, ctx, r, n_voxels)


def lmtof_count_segments(ctx):
    """(pieces visited, pieces with non-zero weight) over all loaded events."""
    a, b = C.c_int64(), C.c_int64()
    _check(_lib.lmtof_count_segments(ctx, C.byref(a), C.byref(b)), ctx)
    return a.value, b.value


def lmtof_autotune(ctx, use_cache: bool = False):
    """Chosen configuration (now set) and the timed candidates."""
    r = lmtof_tune_result()
    _check(_lib.lmtof_autotune(ctx, 1 if use_cache else 0, C.byref(r)), ctx)
    names = ("forward", "events_per_thread", "brick_chunks")
    return dict({k: getattr(r, k) for k in names}, cached=bool(r.cached),
                candidates=[dict({k: getattr(q, k) for k in names}, pass_ms=q.pass_ms, build_ms=q.build_ms)
                            for q in r.cand[:r.n_candidates]])


def lmtof_set_regions(ctx, z_bounds, margin_slices: int = -1) -> None:
    zb = np.ascontiguousarray(z_bounds, dtype=np.int32)
    _check(_lib.lmtof_set_regions(ctx, zb.ctypes.data_as(C.POINTER(C.c_int32)), len(zb) - 1, margin_slices), ctx)


def lmtof_region_info(ctx, k: int):
    o = (C.c_int32 * 4)()
    n = C.c_int64()
    _check(_lib.lmtof_region_info(ctx, k, o, C.byref(n)), ctx)
    return dict(z_lo=o[0], nz=o[1], core_lo=o[2], core_hi=o[3], n_events=n.value)


def lmtof_read_region_image(ctx, k: int, n: int, out=None):
    o, p, mem = _out(out, n, np.float32)
    _check(_lib.lmtof_read_region_image(ctx, k, p, n, mem), ctx)
    return o


def lmtof_event_regions(ctx, n: int, out=None):
    o, p, mem = _out(out, n, np.int32)
    _check(_lib.lmtof_event_regions(ctx, p, n, mem), ctx)
    return o


def lmtof_clear_regions(ctx) -> None:
    _check(_lib.lmtof_clear_regions(ctx), ctx)


# ---------------------------------------------------------------- serving
def lmtof_pool_last_error(pool) -> str:
    m = _lib.lmtof_pool_last_error(pool)
    return m.decode() if m else ""


def _pcheck(rc: int, pool) -> None:
    if rc != LMTOF_OK:
        raise LmtofError(rc, lmtof_pool_last_error(pool))


def lmtof_pool_create(hbm_budget_bytes: int, hip_device: int = 0, hip_stream: Optional[int] = None):
    h = C.c_void_p()
    rc = _lib.lmtof_pool_create(C.byref(h), hip_device, C.c_void_p(hip_stream) if hip_stream else None,
                                int(hbm_budget_bytes))
    _pcheck(rc, None)
    return h


def lmtof_pool_destroy(pool) -> None:
    _pcheck(_lib.lmtof_pool_destroy(pool), None)


def make_request(geometry, ev, n_iter: int, storage: int = 0, fmt: Optional[int] = None,
                 background: bool = False):
    """(lmtof_request, keep-alive) for events ev (NumPy or GPU tensor).  With
    background=True the pool prepares it on its own thread and stream: keep
    the keep-alive object until the request is polled done."""
    if fmt is None:
        fmt = LMTOF_FMT_PACKED16 if "int16" in str(ev.dtype) else LMTOF_FMT_F32X7
    per = 7 if fmt == LMTOF_FMT_F32X7 else 8
    p, mem, keep = _in(ev, np.float32 if fmt == LMTOF_FMT_F32X7 else np.int16)
    q = lmtof_request()
    q.geometry = geometry if isinstance(geometry, lmtof_geometry) else geometry_struct(geometry)
    q.events = p
    q.n_events = int(np.prod(ev.shape)) // per
    q.format = fmt
    q.mem = mem
    q.n_iter = int(n_iter)
    q.storage = int(storage)
    q.flags = LMTOF_REQ_BACKGROUND if background else 0
    return q, keep


def lmtof_pool_request_bytes(req) -> int:
    v = C.c_int64()
    _pcheck(_lib.lmtof_pool_request_bytes(C.byref(req), C.byref(v)), None)
    return v.value


def lmtof_pool_submit(pool, req) -> int:
    """Request id; raises LmtofError (code LMTOF_EAGAIN when it does not fit now)."""
    v = C.c_int64()
    _pcheck(_lib.lmtof_pool_submit(pool, C.byref(req), C.byref(v)), pool)
    return v.value


def lmtof_pool_step(pool) -> int:
    n = C.c_int()
    _pcheck(_lib.lmtof_pool_step(pool, C.byref(n)), pool)
    return n.value


def lmtof_pool_poll(pool, rid: int, n_voxels: int, out=None):
    """Image (and release) if request rid finished, else None."""
    o, p, mem = _out(out, n_voxels, np.float32)
    done = C.c_int()
    _pcheck(_lib.lmtof_pool_poll(pool, rid, C.byref(done), p, n_voxels, mem), pool)
    return o if done.value else None


def lmtof_pool_info(pool):
    used, budget = C.c_int64(), C.c_int64()
    na, nf = C.c_int(), C.c_int()
    _pcheck(_lib.lmtof_pool_info(pool, C.byref(used), C.byref(budget), C.byref(na), C.byref(nf)), pool)
    return dict(used=used.value, budget=budget.value, active=na.value, finished=nf.value)


def exported_symbols():
    """Names the binding resolved from the shared library."""
    return sorted(_sig)


class Reconstruction:
    """Owns one context; each method calls the entry point of the same name."""

    def __init__(self, geometry: Dict[str, Any], device: int = 0, **options):
        self.ctx = lmtof_create(device)
        self.geometry = dict(geometry)
        self.V = int(geometry["nx"]) * int(geometry["ny"]) * int(geometry["nz"])
        try:
            for k, v in options.items():
                lmtof_set_option(self.ctx, globals()["LMTOF_OPT_" + k.upper()], int(v))
            lmtof_set_geometry(self.ctx, geometry)
        except Exception:
            self.close()
            raise

    def close(self):
        if getattr(self, "ctx", None):
            lmtof_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_option(self, key: str, value: int):
        lmtof_set_option(self.ctx, globals()["LMTOF_OPT_" + key.upper()], int(value))

    def load_events(self, ev, fmt=None):
        lmtof_load_events(self.ctx, ev, fmt)

    @property
    def n_events(self) -> int:
        return lmtof_num_events(self.ctx)

    def compute_sensitivity(self):
        lmtof_compute_sensitivity(self.ctx)

    def read_sensitivity(self, out=None):
        return lmtof_read_sensitivity(self.ctx, self.V, out)

    def set_sensitivity(self, s):
        lmtof_set_sensitivity(self.ctx, s)

    def set_image(self, x0=None):
        lmtof_set_image(self.ctx, x0)

    def read_image(self, out=None):
        return lmtof_read_image(self.ctx, self.V, out)

    def iterate(self, n_iter: int):
        return lmtof_iterate(self.ctx, n_iter)

    def forward_project(self, x, out=None):
        return lmtof_forward_project(self.ctx, x, self.n_events, out)

    def back_project(self, w, out=None):
        return lmtof_back_project(self.ctx, w, self.V, out)

    def median_filter(self, x, out=None):
        return lmtof_median_filter(self.ctx, x, self.V, out)

    def tof_keep(self, mask, out=None):
        return lmtof_tof_keep(self.ctx, mask, lmtof_num_events(self.ctx), out)

    def attenuation_factors(self, mu, out=None):
        return lmtof_attenuation_factors(self.ctx, mu, lmtof_num_events(self.ctx), out)

    def set_event_weights(self, w):
        lmtof_set_event_weights(self.ctx, w)

    def sampled_forward_project(self, x):
        return lmtof_sampled_forward_project(self.ctx, x, lmtof_num_events(self.ctx))

    def sampled_forward_project_noalloc(self, x, f):
        return lmtof_sampled_forward_project_noalloc(self.ctx, x, f)

    def sampled_back_project(self, r):
        return lmtof_sampled_back_project(self.ctx, r, self.V)

    def count_segments(self):
        return lmtof_count_segments(self.ctx)

    def autotune(self, use_cache: bool = False):
        return lmtof_autotune(self.ctx, use_cache)

    def read_packed_events(self, out=None):
        return lmtof_read_packed_events(self.ctx, out)

    def set_regions(self, z_bounds, margin_slices: int = -1):
        lmtof_set_regions(self.ctx, z_bounds, margin_slices)

    def region_info(self, k: int):
        return lmtof_region_info(self.ctx, k)

    def read_region_image(self, k: int, out=None):
        info = self.region_info(k)
        n = int(self.geometry["nx"]) * int(self.geometry["ny"]) * info["nz"]
        return lmtof_read_region_image(self.ctx, k, n, out)

    def event_regions(self, out=None):
        """Region index of every loaded event (caller order) after set_regions."""
        return lmtof_event_regions(self.ctx, lmtof_num_events(self.ctx), out)

    def clear_regions(self):
        lmtof_clear_regions(self.ctx)
