"""Oracle sensitivity of a centred lattice from one voxel per symmetry orbit.

The acceptance of a voxel centre (the oracle's azimuth midpoint rule) is
unchanged by the x and y mirrors, the x <-> y swap and the z mirror: each
maps the azimuth nodes onto themselves.  The oracle pins check every
generator to 1e-12, and a pin checks this routine against the oracle's full
sensitivity on a small grid.  Used by the whole-body parity tests, where the
oracle's full-grid sensitivity would cost minutes.
"""
import numpy as np

import oracle


def sensitivity_by_orbits(g, n_phi=oracle.N_PHI):
    """Oracle acceptance at every voxel centre of a centred lattice with
    nx = ny, vx = vy and even nx, nz, integrated once per orbit."""
    nx, ny, nz = int(g["nx"]), int(g["ny"]), int(g["nz"])
    assert nx == ny and nx % 2 == 0 and nz % 2 == 0 and g["vx"] == g["vy"]
    cx = g["x0"] + g["vx"] * (np.arange(nx) + 0.5)
    cy = g["y0"] + g["vy"] * (np.arange(ny) + 0.5)
    cz = g["z0"] + g["vz"] * (np.arange(nz) + 0.5)
    assert np.array_equal(cx, -cx[::-1]) and np.array_equal(cy, cx) and np.array_equal(cz, -cz[::-1])
    h, hz = nx // 2, nz // 2
    ia, ib = np.triu_indices(h)          # 0 <= a <= b < h: |x| index a, |y| index b
    A = np.repeat(ia, hz)
    B = np.repeat(ib, hz)
    Z = np.tile(np.arange(hz), ia.size)
    pts = np.stack([cx[h + A], cx[h + B], cz[hz + Z]], axis=1)
    acc = oracle.acceptance(g, pts, n_phi)
    s = np.zeros((nz, ny, nx))
    for zs in (hz + Z, hz - 1 - Z):
        for p, q in ((A, B), (B, A)):
            for xs in (h + p, h - 1 - p):
                for ys in (h + q, h - 1 - q):
                    s[zs, ys, xs] = acc
    return s.reshape(-1)
