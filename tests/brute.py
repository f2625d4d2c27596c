"""Dense brute-force system matrix for tiny grids (NumPy, FP64).

An independent route to the TOF-weighted system matrix used to pin the
oracle: instead of merging plane crossings along the ray (Siddon), every
voxel of the grid is intersected with the line on its own (slab method on
the voxel box), the interval is clipped to the event's window, and the
truncated Gaussian is integrated over it.  O(events x voxels): tiny grids only.
"""
import numpy as np
from scipy.special import ndtr


def sigma_mm(fwhm_ps, c):
    return c * fwhm_ps / 2.0 / (2.0 * np.sqrt(2.0 * np.log(2.0)))


def ray(g, ev):
    ev = np.asarray(ev, np.float64)
    P1, P2, dt = ev[:3], ev[3:6], ev[6]
    d = P2 - P1
    u = d / np.linalg.norm(d)
    tof = g.get("tof_fwhm_ps", 0.0) > 0
    mu = 0.5 * (P1 + P2) + (g["c_mm_per_ps"] * dt / 2.0 if tof else 0.0) * u
    return mu, u


def _interval(lo, hi, mu, u):
    """Parameter interval of the line mu + t u inside the box [lo, hi)."""
    t0, t1 = -np.inf, np.inf
    for k in range(3):
        if u[k] == 0.0:
            if not (lo[k] <= mu[k] < hi[k]):
                return 1.0, 0.0
            continue
        a, b = (lo[k] - mu[k]) / u[k], (hi[k] - mu[k]) / u[k]
        t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
    return t0, t1


def box(g):
    lo = np.array([g["x0"], g["y0"], g["z0"]], np.float64)
    v = np.array([g["vx"], g["vy"], g["vz"]], np.float64)
    n = np.array([g["nx"], g["ny"], g["nz"]])
    return lo, lo + n * v, v, n


def window(g, ev):
    mu, u = ray(g, ev)
    lo, hi, _, _ = box(g)
    t0, t1 = _interval(lo, hi, mu, u)
    if g.get("tof_fwhm_ps", 0.0) > 0:
        w = g["tof_trunc_sigmas"] * sigma_mm(g["tof_fwhm_ps"], g["c_mm_per_ps"])
        t0, t1 = max(t0, -w), min(t1, w)
    return t0, t1


def dense_row(g, ev):
    """Row i of A over all voxels (x-fastest)."""
    mu, u = ray(g, ev)
    lo, _, v, n = box(g)
    w0, w1 = window(g, ev)
    nx, ny, nz = n
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    idx = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], 1)
    vlo = lo + idx * v
    vhi = vlo + v
    t0 = np.full(len(idx), -np.inf)
    t1 = np.full(len(idx), np.inf)
    for k in range(3):
        if u[k] == 0.0:
            inside = (vlo[:, k] <= mu[k]) & (mu[k] < vhi[:, k])
            t0 = np.where(inside, t0, np.inf)
            continue
        a = (vlo[:, k] - mu[k]) / u[k]
        b = (vhi[:, k] - mu[k]) / u[k]
        t0 = np.maximum(t0, np.minimum(a, b))
        t1 = np.minimum(t1, np.maximum(a, b))
    ta = np.maximum(t0, w0)
    tb = np.minimum(t1, w1)
    keep = tb > ta
    row = np.zeros(len(idx))
    if g.get("tof_fwhm_ps", 0.0) > 0:
        s = sigma_mm(g["tof_fwhm_ps"], g["c_mm_per_ps"])
        K = g["tof_trunc_sigmas"]
        norm = ndtr(K) - ndtr(-K)
        row[keep] = (ndtr(tb[keep] / s) - ndtr(ta[keep] / s)) / norm
    else:
        row[keep] = tb[keep] - ta[keep]
    return row


def dense_matrix(g, evs):
    return np.stack([dense_row(g, e) for e in np.asarray(evs, np.float64).reshape(-1, 7)])


def chord_length(g, ev):
    """Length of the line inside the grid box (non-TOF window)."""
    mu, u = ray(g, ev)
    lo, hi, _, _ = box(g)
    t0, t1 = _interval(lo, hi, mu, u)
    return max(0.0, t1 - t0)
