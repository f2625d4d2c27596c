"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and bench.py.

The module only simulates list-mode data (phantoms, emission, detection,
blur).  It holds none of the reconstruction arithmetic, so sharing it does
not couple the FP64 oracle to the HIP path.  The heavy lifting is in
``synth.c`` (OpenMP, per-event SplitMix64 streams: output does not depend on
the thread count).

Workload shapes follow the paper's studies: a uniform cylinder with hot
spheres (Section 2.1.1) and a whole-body phantom with organ uptake and small
lesions at the paper's lesion sites (Sections 2.1.2-2.1.3), on a single-bed,
long-axial-field-of-view cylinder with a 45 degree axial acceptance cut.
The concrete numbers are this project's own synthetic stand-ins for the
paper's GEANT4/NCAT data.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")

FWHM_TO_SIGMA = 1.0 / (2.0 * np.sqrt(2.0 * np.log(2.0)))
C_MM_PER_PS = 0.299792458


def build(force: bool = True) -> str:
    """Compile synth.c into libsynth.so next to it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Shape(C.Structure):
    _fields_ = [("kind", C.c_int32), ("mode", C.c_int32),
                ("cx", C.c_double), ("cy", C.c_double), ("cz", C.c_double),
                ("ax", C.c_double), ("ay", C.c_double), ("az", C.c_double),
                ("z0", C.c_double), ("z1", C.c_double), ("value", C.c_double)]


class _Scanner(C.Structure):
    _fields_ = [("R", C.c_double), ("H", C.c_double), ("tan_lmax", C.c_double),
                ("pos_sigma", C.c_double), ("tof_sigma_ps", C.c_double),
                ("c_mm_per_ps", C.c_double)]


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
                ("vx", C.c_double), ("vy", C.c_double), ("vz", C.c_double)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = C.CDLL(_LIB)
        P = C.POINTER
        lib.synth_phantom_eval.argtypes = [P(_Shape), C.c_int, P(C.c_double), C.c_int64, P(C.c_double)]
        lib.synth_voxelize.argtypes = [P(_Shape), C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                       C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, P(C.c_float)]
        lib.synth_trues_continuous.argtypes = [P(_Shape), C.c_int, P(C.c_double), P(C.c_double), C.c_double,
                                               P(_Scanner), C.c_int64, C.c_uint64, C.c_int64, P(C.c_float)]
        lib.synth_trues_continuous.restype = C.c_int
        lib.synth_events_voxel.argtypes = [P(C.c_float), P(_Grid), P(_Scanner), C.c_double, C.c_double,
                                           C.c_int64, C.c_uint64, C.c_int64, P(C.c_float), P(C.c_uint8)]
        lib.synth_events_voxel.restype = C.c_int
        lib.synth_point_source.argtypes = [P(_Scanner), P(C.c_double), C.c_int64, C.c_uint64, P(C.c_float)]
        lib.synth_point_source.restype = C.c_int64
        lib.synth_num_threads.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# ----------------------------------------------------------------- shapes
@dataclass
class Shape:
    kind: str                      # "ellipsoid" | "ecyl" (elliptic cylinder along z)
    centre: Tuple[float, float, float]
    axes: Tuple[float, float, float]
    value: float
    mode: str = "set"              # "set" | "mul"
    z0: float = 0.0
    z1: float = 0.0


def _shape_array(shapes: Sequence[Shape]):
    arr = (_Shape * len(shapes))()
    for k, s in enumerate(shapes):
        arr[k].kind = 0 if s.kind == "ellipsoid" else 1
        arr[k].mode = 0 if s.mode == "set" else 1
        arr[k].cx, arr[k].cy, arr[k].cz = s.centre
        arr[k].ax, arr[k].ay, arr[k].az = s.axes
        arr[k].z0, arr[k].z1 = s.z0, s.z1
        arr[k].value = s.value
    return arr


def sphere(c, r, v, mode="set"):
    return Shape("ellipsoid", tuple(c), (r, r, r), v, mode)


def ellipsoid(c, a, v, mode="set"):
    return Shape("ellipsoid", tuple(c), tuple(a), v, mode)


def ecyl(cx, cy, ax, ay, z0, z1, v, mode="set"):
    return Shape("ecyl", (cx, cy, 0.0), (ax, ay, 1.0), v, mode, z0, z1)


def cylinder_phantom() -> List[Shape]:
    """Uniform water-like cylinder r = 120 mm, |z| <= 100 mm, activity 1, with
    three r = 10 mm spheres at 4:1 contrast (cf. the paper's six spheres in a
    homogeneous background, Section 2.1.1)."""
    return [ecyl(0, 0, 120, 120, -100, 100, 1.0),
            sphere((60.0, 0.0, -40.0), 10, 4.0),
            sphere((-30.0, 51.96, 0.0), 10, 4.0),
            sphere((-30.0, -51.96, 40.0), 10, 4.0)]


def wholebody_phantom() -> List[Shape]:
    """Ellipsoidal torso/head/limbs with organ uptake 1-8x background and ten
    3:1 lesions: six at the paper's lesion sites (cervical, sub-clavicular,
    axillary, inguinal, knee, foot; Section 2.1.3) plus liver, brain, lung and
    abdomen.  Feet towards -z, head towards +z."""
    s = []
    # body outline, uptake 1
    s.append(ellipsoid((0, 0, 500), (75, 90, 110), 1.0))           # head
    s.append(ecyl(0, 0, 50, 50, 340, 390, 1.0))                     # neck
    s.append(ecyl(0, 0, 170, 110, -350, 340, 1.0))                  # torso
    s.append(ecyl(215, 0, 40, 40, -150, 300, 1.0))                  # arms
    s.append(ecyl(-215, 0, 40, 40, -150, 300, 1.0))
    s.append(ecyl(90, 0, 65, 65, -1080, -350, 1.0))                 # legs
    s.append(ecyl(-90, 0, 65, 65, -1080, -350, 1.0))
    s.append(ellipsoid((90, 40, -1120), (45, 100, 40), 1.0))        # feet
    s.append(ellipsoid((-90, 40, -1120), (45, 100, 40), 1.0))
    # organs
    s.append(ellipsoid((0, 0, 510), (65, 80, 90), 6.0))             # brain
    s.append(ellipsoid((-80, 0, 60), (90, 70, 80), 2.0))            # liver
    s.append(ellipsoid((100, 30, 70), (35, 30, 50), 2.0))           # spleen
    s.append(ellipsoid((70, 60, -20), (30, 25, 55), 4.0))           # kidneys
    s.append(ellipsoid((-70, 60, -20), (30, 25, 55), 4.0))
    s.append(ellipsoid((0, -30, -300), (40, 35, 35), 8.0))          # bladder
    s.append(ellipsoid((30, -20, 200), (55, 45, 60), 8.0))          # myocardium (outer)
    s.append(ellipsoid((30, -20, 200), (45, 35, 50), 1.0))          # blood pool
    # lesions, 3x host
    for c, r in [((25, 30, 360), 5), ((-90, -60, 300), 6), ((160, 0, 260), 7), ((60, -50, -330), 8),
                 ((90, 0, -760), 9), ((90, 40, -1110), 10), ((-80, 0, 40), 8), ((30, 0, 540), 6),
                 ((-90, 0, 150), 7), ((0, 40, -150), 10)]:
        s.append(sphere(c, r, 3.0, mode="mul"))
    return s


# ------------------------------------------------------------- workloads
@dataclass
class Workload:
    """Geometry + data recipe of one synthetic reconstruction problem."""
    name: str
    nx: int
    ny: int
    nz: int
    voxel: float                  # mm (cubic)
    radius: float                 # scanner radius (mm)
    half_length: float            # scanner half length (mm)
    max_axial_deg: float          # 0 = no cut
    tof_fwhm_ps: float
    n_events: int
    n_iter: int
    seed: int
    kind: str                     # "cylinder" | "wholebody"
    scatter_frac: float = 0.0
    pos_fwhm_mm: float = 0.4
    trunc_sigmas: float = 3.0
    c_mm_per_ps: float = C_MM_PER_PS
    z0: Optional[float] = None    # default: grid centred

    @property
    def origin(self) -> Tuple[float, float, float]:
        z0 = -self.nz * self.voxel / 2 if self.z0 is None else self.z0
        return (-self.nx * self.voxel / 2, -self.ny * self.voxel / 2, z0)

    @property
    def n_voxels(self) -> int:
        return self.nx * self.ny * self.nz

    def geometry(self) -> dict:
        """Plain dict of the reconstruction geometry (mm, ps)."""
        x0, y0, z0 = self.origin
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, vx=self.voxel, vy=self.voxel, vz=self.voxel,
                    x0=x0, y0=y0, z0=z0, scanner_radius=self.radius,
                    scanner_half_length=self.half_length, max_axial_angle_deg=self.max_axial_deg,
                    tof_fwhm_ps=self.tof_fwhm_ps, tof_trunc_sigmas=self.trunc_sigmas,
                    c_mm_per_ps=self.c_mm_per_ps)


def cylinder_workload(n_events: int = 100_000, seed: int = 1706, tof_fwhm_ps: float = 300.0,
                      n_iter: int = 5) -> Workload:
    """64^3 voxels of 4 mm, scanner R = 400 mm, axial length 256 mm, no axial cut."""
    return Workload("cylinder-64^3-4mm", 64, 64, 64, 4.0, 400.0, 128.0, 0.0, tof_fwhm_ps,
                    n_events, n_iter, seed, "cylinder")


def wholebody_workload(n_events: int = 146_000_000, seed: int = 7075, tof_fwhm_ps: float = 300.0,
                       n_iter: int = 10) -> Workload:
    """150x150x600 voxels of 4 mm, R = 450 mm, axial length 2400 mm, 45 deg cut,
    67 % trues + 33 % scatter-like LORs through the body."""
    return Workload("wholebody-150x150x600-4mm", 150, 150, 600, 4.0, 450.0, 1200.0, 45.0, tof_fwhm_ps,
                    n_events, n_iter, seed, "wholebody", scatter_frac=0.33)


def scanner_struct(w: Workload) -> _Scanner:
    sc = _Scanner()
    sc.R, sc.H = w.radius, w.half_length
    sc.tan_lmax = np.tan(np.deg2rad(w.max_axial_deg)) if w.max_axial_deg > 0 else 0.0
    sc.pos_sigma = w.pos_fwhm_mm * FWHM_TO_SIGMA
    sc.tof_sigma_ps = w.tof_fwhm_ps * FWHM_TO_SIGMA
    sc.c_mm_per_ps = w.c_mm_per_ps
    return sc


def phantom_eval(shapes: Sequence[Shape], pts: np.ndarray) -> np.ndarray:
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.empty(len(pts), np.float64)
    arr = _shape_array(shapes)
    _L().synth_phantom_eval(arr, len(shapes), _ptr(pts, C.c_double), len(pts), _ptr(out, C.c_double))
    return out


def voxelize(shapes: Sequence[Shape], w: Workload, supersample: int = 2) -> np.ndarray:
    """Mean activity per voxel, shape (nz, ny, nx) float32 (x fastest)."""
    out = np.empty((w.nz, w.ny, w.nx), np.float32)
    x0, y0, z0 = w.origin
    arr = _shape_array(shapes)
    _L().synth_voxelize(arr, len(shapes), w.nx, w.ny, w.nz, x0, y0, z0, w.voxel, w.voxel, w.voxel,
                        supersample, _ptr(out, C.c_float))
    return out


_phantom_cache = {}


def wholebody_activity(w: Workload) -> np.ndarray:
    key = (w.nx, w.ny, w.nz, w.voxel, w.origin)
    if key not in _phantom_cache:
        _phantom_cache.clear()
        _phantom_cache[key] = voxelize(wholebody_phantom(), w, supersample=2)
    return _phantom_cache[key]


def events(w: Workload, n: Optional[int] = None, first: int = 0, with_labels: bool = False):
    """Generate events [first, first + n) of workload w as float32 (n, 7).

    Event i depends only on (w.seed, i), so any slice can be regenerated on
    its own and any prefix is a representative sample."""
    n = w.n_events if n is None else n
    out = np.empty((n, 7), np.float32)
    labels = np.zeros(n, np.uint8) if with_labels else None
    sc = scanner_struct(w)
    if w.kind == "cylinder":
        shapes = cylinder_phantom()
        arr = _shape_array(shapes)
        lo = (C.c_double * 3)(-120.0, -120.0, -100.0)
        hi = (C.c_double * 3)(120.0, 120.0, 100.0)
        rc = _L().synth_trues_continuous(arr, len(shapes), lo, hi, 4.0, C.byref(sc), n, w.seed, first,
                                         _ptr(out, C.c_float))
    elif w.kind == "wholebody":
        act = np.ascontiguousarray(wholebody_activity(w))
        g = _Grid()
        g.nx, g.ny, g.nz = w.nx, w.ny, w.nz
        g.x0, g.y0, g.z0 = w.origin
        g.vx = g.vy = g.vz = w.voxel
        rc = _L().synth_events_voxel(_ptr(act, C.c_float), C.byref(g), C.byref(sc), w.scatter_frac, 4.0, n,
                                     w.seed, first, _ptr(out, C.c_float),
                                     _ptr(labels, C.c_uint8) if labels is not None else None)
    else:
        raise ValueError(w.kind)
    if rc != 0:
        raise RuntimeError(f"synthetic event generation failed (code {rc})")
    return (out, labels) if with_labels else out


def point_source(w: Workload, p, n_emit: int, seed: int = 11, keep_events: bool = False):
    """Fire n_emit isotropic pairs from point p; return the accepted count
    (and the accepted records if keep_events)."""
    sc = scanner_struct(w)
    pp = (C.c_double * 3)(*[float(v) for v in p])
    buf = np.empty((n_emit, 7), np.float32) if keep_events else None
    acc = _L().synth_point_source(C.byref(sc), pp, n_emit, seed,
                                  _ptr(buf, C.c_float) if keep_events else None)
    return (acc, buf[:acc].copy()) if keep_events else acc


def random_events_in_box(n: int, seed: int, radius: float, half_length: float,
                         tof_sigma_ps: float = 127.4, box: float = 60.0, c=C_MM_PER_PS) -> np.ndarray:
    """Generic test events: emission point uniform in a centred cube of half
    side `box`, isotropic direction, both ends on the cylinder (no |z| cut:
    the line is extended to the barrel), Gaussian dt blur.  Pure NumPy; for
    small unit tests only."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(-box, box, size=(n, 3))
    sl = rng.uniform(-0.8, 0.8, n)
    ph = rng.uniform(0, 2 * np.pi, n)
    cl = np.sqrt(1 - sl * sl)
    u = np.stack([cl * np.cos(ph), cl * np.sin(ph), sl], 1)
    a = u[:, 0] ** 2 + u[:, 1] ** 2
    b = p[:, 0] * u[:, 0] + p[:, 1] * u[:, 1]
    cc = p[:, 0] ** 2 + p[:, 1] ** 2 - radius ** 2
    sq = np.sqrt(b * b - a * cc)
    sp, sm = (-b + sq) / a, (-b - sq) / a
    P1 = p + sm[:, None] * u
    P2 = p + sp[:, None] * u
    dt = (-sm - sp) / c + rng.normal(0, tof_sigma_ps, n)
    return np.concatenate([P1, P2, dt[:, None]], 1).astype(np.float32)


def num_threads() -> int:
    return _L().synth_num_threads()
