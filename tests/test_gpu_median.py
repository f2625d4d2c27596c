"""GPU parity of the median sieve between iterations (Section 2.4) against
the oracle: bit-exact (the median of 27 values is one of them), on ragged
grids, at the whole-body size on sampled voxels, and inside MLEM."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1706_07075_amd import lmtof as L  # noqa: E402


def _say(msg):
    print(msg, flush=True)


def _geom(nx, ny, nz, v=1.0):
    return dict(nx=nx, ny=ny, nz=nz, vx=v, vy=v, vz=v, x0=-nx * v / 2, y0=-ny * v / 2, z0=-nz * v / 2,
                scanner_radius=400.0, scanner_half_length=400.0, max_axial_angle_deg=0.0, tof_fwhm_ps=300.0,
                tof_trunc_sigmas=3.0, c_mm_per_ps=0.299792458)


def _image(shape, seed):
    a = np.random.default_rng(seed).uniform(0.0, 1.0, int(np.prod(shape))).astype(np.float32)
    a[a < 0.25] = 0.0   # zeros tie with the border
    a[a > 0.9] = 0.5    # repeated values
    return a


@pytest.mark.parametrize("shape", [(37, 23, 19), (1, 1, 1), (2, 1, 3), (64, 64, 64), (257, 3, 2)])
def test_median_filter_bit_exact(shape):
    nx, ny, nz = shape
    _say(f"case: median filter {shape}")
    x = _image(shape, 11)
    with L.Reconstruction(_geom(nx, ny, nz)) as r:
        y = r.median_filter(x)
    ref = oracle.median3(x, nx, ny, nz)
    assert np.array_equal(y.view(np.uint32), ref.astype(np.float32).view(np.uint32))


def test_median_filter_wholebody_sampled_device():
    """150 x 150 x 600 image in device memory; 3000 sampled voxels (all
    corners, edge and face voxels among them) against the oracle on the
    sample's 3 x 3 x 3 neighbourhood cropped from the image."""
    w = synth.wholebody_workload(n_events=1000)
    g = w.geometry()
    nx, ny, nz = g["nx"], g["ny"], g["nz"]
    _say("case: median filter whole body, device memory")
    x = _image((nx, ny, nz), 12)
    xd = torch.from_numpy(x).cuda()
    with L.Reconstruction(g) as r:
        yd = r.median_filter(xd)
        torch.cuda.synchronize()
    y = yd.cpu().numpy()
    a = x.reshape(nz, ny, nx)
    rng = np.random.default_rng(13)
    pts = [(px, py, pz) for px in (0, nx - 1) for py in (0, ny - 1) for pz in (0, nz - 1)]
    pts += [(0, 5, 7), (nx - 1, 70, 300), (3, 0, 9), (8, ny - 1, nz - 1), (75, 75, 0)]
    pts += [tuple(int(v) for v in rng.integers(0, (nx, ny, nz))) for _ in range(3000)]
    for px, py, pz in pts:
        x0, x1 = max(px - 1, 0), min(px + 2, nx)
        y0, y1 = max(py - 1, 0), min(py + 2, ny)
        z0, z1 = max(pz - 1, 0), min(pz + 2, nz)
        crop = a[z0:z1, y0:y1, x0:x1]
        cz, cy, cx = crop.shape
        m = oracle.median3(crop.reshape(-1), cx, cy, cz).reshape(cz, cy, cx)
        assert y[(pz * ny + py) * nx + px] == m[pz - z0, py - y0, px - x0], (px, py, pz)


def test_median_filter_errors():
    with L.Reconstruction(_geom(4, 4, 4)) as r:
        x = np.ones(64, np.float32)
        with pytest.raises(L.LmtofError) as e:
            L.lmtof_median_filter(r.ctx, x, 63)
        assert e.value.code == L.LMTOF_EINVAL
        xd = torch.ones(64, device="cuda")
        with pytest.raises(L.LmtofError) as e:
            L.lmtof_median_filter(r.ctx, xd, 64, out=xd)
        assert e.value.code == L.LMTOF_EINVAL
        assert np.array_equal(r.median_filter(x), oracle.median3(x, 4, 4, 4).astype(np.float32))


def test_mlem_with_median_sieve():
    """Two iterations with the sieve on against the oracle's EM step followed
    by its median, from the same FP32 start and sensitivity.  The sieve picks
    one of 27 inputs, so the FP32-vs-FP64 differences of the EM step pass
    through unchanged (or pick a neighbour of nearly equal value)."""
    w = synth.cylinder_workload()
    g = w.geometry()
    ev = synth.events(w)
    s = np.random.default_rng(14).uniform(0.5, 1.5, w.n_voxels).astype(np.float32)
    x0 = np.full(w.n_voxels, len(ev) / float(s.astype(np.float64).sum()), np.float32)
    _say("case: MLEM + median sieve, 64^3, 100k events, 2 iterations")
    with L.Reconstruction(g, median_sieve=1) as r:
        r.load_events(ev)
        r.set_sensitivity(s)
        r.set_image(x0)
        st = r.iterate(2)
        x = r.read_image()
        r.set_option("median_sieve", 0)
        r.set_image(x0)
        r.iterate(1)
        x_plain = r.read_image()
    xr = x0.astype(np.float64)
    for _ in range(2):
        xr, _ = oracle.mlem(g, ev, s.astype(np.float64), 1, x0=xr)
        xr = oracle.median3(xr, g["nx"], g["ny"], g["nz"])
    e = oracle.rel_l2(x, xr)
    _say(f"  rel L2 {e:.2e}")
    assert e < 1e-5
    assert [q["iter"] for q in st] == [0, 1] and all(q["ms"] > 0 for q in st)
    # the sieve is on the path: one plain iteration differs from the sieved one
    x1_plain, _ = oracle.mlem(g, ev, s.astype(np.float64), 1, x0=x0.astype(np.float64))
    assert oracle.rel_l2(x_plain, x1_plain) < 1e-5
