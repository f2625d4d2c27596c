"""FP64 CPU oracle for list-mode TOF-weighted MLEM (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP
library; see ``oracle.c`` for what it computes and which passages of the
paper each part follows.  This wrapper only marshals arrays (and holds the
oracle's own packed-event codec, written with NumPy from the record layout).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

N_PHI = 2048  # azimuth nodes of the acceptance quadrature


def build(force: bool = True) -> str:
    """Compile oracle.c (gcc -O2, IEEE semantics: no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-shared", "-fPIC", "-std=c99",
                               "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Geom(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad_", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
                ("vx", C.c_double), ("vy", C.c_double), ("vz", C.c_double),
                ("R", C.c_double), ("H", C.c_double), ("max_axial_deg", C.c_double),
                ("tof_fwhm_ps", C.c_double), ("trunc_sigmas", C.c_double), ("c_mm_per_ps", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("n_eff", C.c_int64), ("sum_sx", C.c_double), ("loglik", C.c_double)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = C.CDLL(_LIB)
        P = C.POINTER
        G = P(Geom)
        d = P(C.c_double)
        lib.or_sigma_mm.argtypes = [C.c_double, C.c_double]
        lib.or_sigma_mm.restype = C.c_double
        lib.or_system_row.argtypes = [G, d, P(C.c_int64), d, C.c_int64]
        lib.or_system_row.restype = C.c_int64
        lib.or_windows.argtypes = [G, d, C.c_int64, d, d]
        lib.or_forward.argtypes = [G, d, C.c_int64, d, d]
        lib.or_back.argtypes = [G, d, C.c_int64, d, d]
        lib.or_acceptance.argtypes = [G, d, C.c_int]
        lib.or_acceptance.restype = C.c_double
        lib.or_acceptance_points.argtypes = [G, d, C.c_int64, C.c_int, d]
        lib.or_sensitivity.argtypes = [G, C.c_int, d]
        lib.or_mlem.argtypes = [G, d, C.c_int64, d, d, C.c_int, d, P(Stats)]
        lib.or_initial_image.argtypes = [G, d, C.c_int64, d]
        lib.or_num_threads.restype = C.c_int
        lib.or_set_num_threads.argtypes = [C.c_int]
        lib.or_set_num_threads.restype = None
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def geom(g: dict) -> Geom:
    """Oracle geometry from a plain dict (mm, ps): nx ny nz x0 y0 z0 vx vy vz
    scanner_radius scanner_half_length max_axial_angle_deg tof_fwhm_ps
    tof_trunc_sigmas c_mm_per_ps."""
    o = Geom()
    o.nx, o.ny, o.nz = int(g["nx"]), int(g["ny"]), int(g["nz"])
    o.x0, o.y0, o.z0 = float(g["x0"]), float(g["y0"]), float(g["z0"])
    o.vx, o.vy, o.vz = float(g["vx"]), float(g["vy"]), float(g["vz"])
    o.R, o.H = float(g["scanner_radius"]), float(g["scanner_half_length"])
    o.max_axial_deg = float(g.get("max_axial_angle_deg", 0.0))
    o.tof_fwhm_ps = float(g.get("tof_fwhm_ps", 0.0))
    o.trunc_sigmas = float(g.get("tof_trunc_sigmas", 3.0))
    o.c_mm_per_ps = float(g.get("c_mm_per_ps", 0.299792458))
    return o


def _ev64(ev) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(ev, dtype=np.float64).reshape(-1, 7))
    return a


def sigma_mm(fwhm_ps: float, c_mm_per_ps: float = 0.299792458) -> float:
    return _L().or_sigma_mm(fwhm_ps, c_mm_per_ps)


def system_row(g: dict, ev):
    """(voxel indices, weights) of one event's row of A."""
    G = geom(g)
    e = _ev64(ev)[0]
    cap = G.nx + G.ny + G.nz + 5
    jj = np.empty(cap, np.int64)
    aa = np.empty(cap, np.float64)
    m = _L().or_system_row(C.byref(G), _dp(e), jj.ctypes.data_as(C.POINTER(C.c_int64)), _dp(aa), cap)
    return jj[:m].copy(), aa[:m].copy()


def system_matrix(g: dict, ev) -> np.ndarray:
    """Dense A (n_events x n_voxels); tiny problems only."""
    e = _ev64(ev)
    V = int(g["nx"]) * int(g["ny"]) * int(g["nz"])
    A = np.zeros((len(e), V))
    for i in range(len(e)):
        j, a = system_row(g, e[i])
        np.add.at(A[i], j, a)
    return A


def windows(g: dict, ev):
    G = geom(g)
    e = _ev64(ev)
    lo = np.empty(len(e))
    hi = np.empty(len(e))
    _L().or_windows(C.byref(G), _dp(e), len(e), _dp(lo), _dp(hi))
    return lo, hi


def forward(g: dict, ev, x) -> np.ndarray:
    G = geom(g)
    e = _ev64(ev)
    xx = np.ascontiguousarray(np.asarray(x, np.float64).ravel())
    f = np.empty(len(e))
    _L().or_forward(C.byref(G), _dp(e), len(e), _dp(xx), _dp(f))
    return f


def back(g: dict, ev, w) -> np.ndarray:
    G = geom(g)
    e = _ev64(ev)
    ww = np.ascontiguousarray(np.asarray(w, np.float64).ravel())
    b = np.empty(G.nx * G.ny * G.nz)
    _L().or_back(C.byref(G), _dp(e), len(e), _dp(ww), _dp(b))
    return b


def acceptance(g: dict, pts, n_phi: int = N_PHI) -> np.ndarray:
    G = geom(g)
    p = np.ascontiguousarray(np.asarray(pts, np.float64).reshape(-1, 3))
    out = np.empty(len(p))
    _L().or_acceptance_points(C.byref(G), _dp(p), len(p), n_phi, _dp(out))
    return out


def sensitivity(g: dict, n_phi: int = N_PHI) -> np.ndarray:
    G = geom(g)
    s = np.empty(G.nx * G.ny * G.nz)
    _L().or_sensitivity(C.byref(G), n_phi, _dp(s))
    return s


def initial_image(g: dict, s, n_events: int) -> np.ndarray:
    G = geom(g)
    ss = np.ascontiguousarray(np.asarray(s, np.float64).ravel())
    x = np.empty_like(ss)
    _L().or_initial_image(C.byref(G), _dp(ss), int(n_events), _dp(x))
    return x


def mlem(g: dict, ev, s, n_iter: int, x0: Optional[np.ndarray] = None, history: bool = False):
    """Run n_iter MLEM iterations.  Returns (x, stats[, hist]) where stats is a
    list of dicts (n_eff, sum_sx, loglik) and hist is (n_iter, V)."""
    G = geom(g)
    e = _ev64(ev)
    ss = np.ascontiguousarray(np.asarray(s, np.float64).ravel())
    x = initial_image(g, ss, len(e)) if x0 is None else np.array(x0, np.float64).ravel().copy()
    st = (Stats * max(n_iter, 1))()
    hist = np.empty((n_iter, len(ss))) if history else None
    _L().or_mlem(C.byref(G), _dp(e), len(e), _dp(ss), _dp(x), n_iter,
                 _dp(hist) if history else None, st)
    stats = [dict(n_eff=int(st[k].n_eff), sum_sx=st[k].sum_sx, loglik=st[k].loglik) for k in range(n_iter)]
    return (x, stats, hist) if history else (x, stats)


def num_threads() -> int:
    return _L().or_num_threads()


def set_num_threads(n: int) -> None:
    """Threads the oracle's parallel loops use from now on."""
    _L().or_set_num_threads(int(n))


# ------------------------------------------------------------ packed codec
# Record: int16 q[6] (P1.xyz, P2.xyz in 0.1 mm quanta, scanner-centred),
# uint16 dt (IEEE binary16 bits, ps), uint16 spare.  16 bytes.
PACK_QUANTUM_MM = 0.1


def pack_events(ev) -> np.ndarray:
    """Oracle-side packer: q = round-half-even(x * 10) in FP32 arithmetic,
    dt rounded to binary16 (nearest even).  Raises on int16 overflow."""
    e = np.asarray(ev, np.float32).reshape(-1, 7)
    q = np.rint(e[:, :6] * np.float32(10.0))
    if np.any(np.abs(q) > 32767):
        raise OverflowError("coordinate outside the int16 range at 0.1 mm")
    out = np.zeros((len(e), 8), np.int16)
    out[:, :6] = q.astype(np.int16)
    out[:, 6] = e[:, 6].astype(np.float16).view(np.int16)
    return out


def decode_packed(p) -> np.ndarray:
    """Packed records -> FP64 (n, 7): coordinate = q * 0.1 mm, dt exact."""
    p = np.asarray(p, np.int16).reshape(-1, 8)
    out = np.empty((len(p), 7))
    out[:, :6] = p[:, :6].astype(np.float64) * PACK_QUANTUM_MM
    out[:, 6] = p[:, 6].view(np.float16).astype(np.float64)
    return out


def median3(x, nx: int, ny: int, nz: int) -> np.ndarray:
    """Median sieve applied to the image between MLEM iterations (Section
    2.4): each voxel becomes the median of the 3 x 3 x 3 block around it,
    voxels outside the grid counting as 0 (the paper notes that null
    neighbours pull border voxels down).  The kernel size and the zero border
    are readings (the paper states neither).  With 27 values the median is
    the 14th smallest, an element of the input: no rounding.  x is x-fastest."""
    a = np.asarray(x).reshape(nz, ny, nx)
    p = np.zeros((nz + 2, ny + 2, nx + 2), a.dtype)
    p[1:-1, 1:-1, 1:-1] = a
    block = np.stack([p[dz:dz + nz, dy:dy + ny, dx:dx + nx]
                      for dz in range(3) for dy in range(3) for dx in range(3)])
    return np.sort(block, axis=0)[13].reshape(-1)


def attenuation_factors(g: dict, ev, mu) -> np.ndarray:
    """Attenuation correction factor of every event (Section 2.4): the
    inverse of the probability that both photons survive, exp(+ line
    integral of mu along the whole LOR inside the grid), mu in 1/mm per voxel
    (x fastest).  The line integral is the non-TOF row of A applied to mu."""
    g0 = dict(g, tof_fwhm_ps=0.0)
    return np.exp(forward(g0, ev, np.asarray(mu, np.float64)))


def mlem_weighted(g: dict, ev, s, n_iter: int, w, x0) -> np.ndarray:
    """MLEM with a weight per event multiplying its ratio (the paper's
    attenuation correction on the LOR, Section 2.4): x <- x / s * A^T (w / A x),
    events with (A x)_i = 0 contributing nothing, voxels with s = 0 held at
    0.  Written from the definition with the oracle's forward and back
    projections."""
    x = np.asarray(x0, np.float64).copy()
    s = np.asarray(s, np.float64)
    w = np.asarray(w, np.float64)
    for _ in range(n_iter):
        f = forward(g, ev, x)
        r = np.where(f > 0, w / np.where(f > 0, f, 1.0), 0.0)
        b = back(g, ev, r)
        x = np.where(s > 0, x * b / np.where(s > 0, s, 1.0), 0.0)
    return x


SAMPLED_N = 32  # samples per event of the paper's sampled TOF projector


def sampled_system(g: dict, ev, n_samples: int = SAMPLED_N):
    """The paper's own TOF projector (Section 2.3): n_samples equally spaced
    points along the LOR, at the midpoints of n_samples equal steps over the
    kernel window [-K sigma, K sigma] around the TOF centre, each weighted by
    the Gaussian density there, the weights normalised to sum to 1; each
    point adds its weight to the voxel holding it ("direct voxel filling"),
    points outside the grid are dropped.  Returns (voxel index per sample,
    -1 outside; the weights; each sample's distance in mm to the nearest
    voxel plane, for bracketing decisions that rounding can flip)."""
    e = _ev64(ev)
    nx, ny, nz = int(g["nx"]), int(g["ny"]), int(g["nz"])
    v = np.array([g["vx"], g["vy"], g["vz"]], float)
    o = np.array([g["x0"], g["y0"], g["z0"]], float)
    n = np.array([nx, ny, nz])
    c = float(g.get("c_mm_per_ps", 0.0) or 0.299792458)
    K = float(g.get("tof_trunc_sigmas", 0.0) or 3.0)
    sig = sigma_mm(float(g["tof_fwhm_ps"]), c)
    t = -K * sig + (np.arange(n_samples) + 0.5) * (2.0 * K * sig / n_samples)
    w = np.exp(-0.5 * (t / sig) ** 2)
    w /= w.sum()
    d = e[:, 3:6] - e[:, :3]
    u = d / np.linalg.norm(d, axis=1)[:, None]
    mu = 0.5 * (e[:, :3] + e[:, 3:6]) + (c * e[:, 6] / 2.0)[:, None] * u
    p = mu[:, None, :] + t[None, :, None] * u[:, None, :]          # (n, S, 3)
    q = (p - o) / v
    cell = np.floor(q)
    inside = np.all((cell >= 0) & (cell < n), axis=2)
    frac = q - cell
    near = np.min(np.minimum(frac, 1.0 - frac) * v, axis=2)
    ci = cell.astype(np.int64)
    idx = np.where(inside, (ci[:, :, 2] * ny + ci[:, :, 1]) * nx + ci[:, :, 0], -1)
    return idx, w, near


def sampled_forward(g: dict, ev, x) -> np.ndarray:
    """f_i = sum over event i's samples inside the grid of w_k x_voxel."""
    idx, w, _ = sampled_system(g, ev)
    xv = np.asarray(x, np.float64)[np.maximum(idx, 0)]
    return np.sum(np.where(idx >= 0, w[None, :] * xv, 0.0), axis=1)


def sampled_back(g: dict, ev, r) -> np.ndarray:
    """b_j = sum over samples in voxel j of w_k r_i (the adjoint)."""
    idx, w, _ = sampled_system(g, ev)
    b = np.zeros(int(g["nx"]) * int(g["ny"]) * int(g["nz"]))
    m = idx >= 0
    np.add.at(b, idx[m], (np.asarray(r, np.float64)[:, None] * w[None, :])[m])
    return b


TOF_REJECT_Z = 1.959964  # two-sided 95 % quantile of the normal distribution


def tof_keep(g: dict, ev, mask, z: float = TOF_REJECT_Z, grow: float = 0.0, min_piece: float = 0.0) -> np.ndarray:
    """TOF scatter rejection (Section 2.2, Fig. 2): an event is kept when the
    stretch of its LOR within z sigma of the TOF centre (z = 1.96: the 95 %
    confidence interval of the annihilation point) passes through the body
    outline, given as a voxel mask on the reconstruction grid (non-zero =
    body; x fastest).  The stretch is cut by the grid box and walked voxel by
    voxel (sorted plane crossings); the event is kept if a piece longer than
    min_piece lies in a body voxel.  grow widens the stretch by grow mm at
    both ends (negative: narrows it), which the tests use to bracket events
    whose decision turns on rounding.  FP64; one event at a time."""
    e = _ev64(ev)
    m = np.asarray(mask).reshape(-1) != 0
    nx, ny, nz = int(g["nx"]), int(g["ny"]), int(g["nz"])
    v = np.array([g["vx"], g["vy"], g["vz"]], float)
    o = np.array([g["x0"], g["y0"], g["z0"]], float)
    n = np.array([nx, ny, nz])
    c = float(g.get("c_mm_per_ps", 0.0) or 0.299792458)
    half = z * sigma_mm(float(g["tof_fwhm_ps"]), c) + grow
    keep = np.zeros(len(e), bool)
    for i in range(len(e)):
        p1, p2, dt = e[i, :3], e[i, 3:6], e[i, 6]
        d = p2 - p1
        u = d / np.sqrt(d @ d)
        mu = 0.5 * (p1 + p2) + (c * dt / 2.0) * u
        t0, t1 = -half, half
        for k in range(3):  # cut by the grid box (slab method)
            lo, hi = o[k], o[k] + n[k] * v[k]
            if u[k] == 0.0:
                if not lo <= mu[k] < hi:
                    t0, t1 = 1.0, 0.0
                continue
            a, b = (lo - mu[k]) / u[k], (hi - mu[k]) / u[k]
            t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
        if not t0 < t1:
            continue
        ts = [t0, t1]
        for k in range(3):
            if u[k] == 0.0:
                continue
            planes = o[k] + v[k] * np.arange(n[k] + 1)
            tk = (planes - mu[k]) / u[k]
            ts.extend(tk[(tk > t0) & (tk < t1)])
        ts = np.sort(np.array(ts))
        for a, b in zip(ts[:-1], ts[1:]):
            if b - a <= min_piece:
                continue
            pt = mu + 0.5 * (a + b) * u
            idx = np.clip(np.floor((pt - o) / v).astype(int), 0, n - 1)
            if m[(idx[2] * ny + idx[1]) * nx + idx[0]]:
                keep[i] = True
                break
    return keep


def rel_l2(a, ref) -> float:
    a = np.asarray(a, np.float64).ravel()
    r = np.asarray(ref, np.float64).ravel()
    return float(np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-300))
