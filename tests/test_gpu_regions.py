"""GPU parity of the TOF-assisted data division (regions run as one batch).

Each region is an independent MLEM problem on its sub-volume (core slab
widened by the margin).  The oracle assigns events to regions itself from
the FP64 TOF centre and runs plain MLEM per region.  Events whose TOF centre
lies within 1e-3 mm of a core boundary (where FP32 and FP64 may disagree)
are dropped from the input that both sides get (2 of 200 000 here).
"""
import numpy as np
import pytest

import oracle
import synth
from tests import brute

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1706_07075_amd import lmtof as L  # noqa: E402


def _mu_z(g, ev):
    mz = []
    for e in ev.astype(np.float64):
        mu, _ = brute.ray(g, e)
        mz.append(mu[2])
    return np.array(mz)


def _assign(g, ev, zb):
    mz = _mu_z(g, ev)
    bounds = g["z0"] + np.asarray(zb, np.float64) * g["vz"]
    r = np.zeros(len(ev), np.int64)
    for k in range(1, len(zb) - 1):
        r[mz >= bounds[k]] = k
    amb = np.min(np.abs(mz[:, None] - bounds[None, 1:-1]), axis=1) < 1e-3 if len(zb) > 2 else np.zeros(len(ev), bool)
    return r, amb


def _smooth_sens(w):
    """A positive, smooth stand-in sensitivity given to both sides."""
    z = (np.arange(w.nz) + 0.5) / w.nz
    y = (np.arange(w.ny) + 0.5) / w.ny
    x = (np.arange(w.nx) + 0.5) / w.nx
    s = 0.3 + 0.2 * np.sin(np.pi * z)[:, None, None] + 0.05 * (x[None, None, :] + y[None, :, None])
    return s.astype(np.float32).ravel()


def unambiguous(w, ev, zb):
    """Drop events whose TOF centre lies within 1e-3 mm of a core boundary
    (FP32 and FP64 may put them on different sides); both sides get the rest."""
    _, amb = _assign(w.geometry(), ev, zb)
    return ev[~amb]


def _region_case(w, ev, zb, n_iter, margin=-1, storage=0):
    g = w.geometry()
    s = _smooth_sens(w)
    r_of, amb = _assign(g, ev, zb)
    assert not amb.any()
    with L.Reconstruction(g, storage=storage) as r:
        r.load_events(ev)
        r.set_sensitivity(s)
        r.set_regions(zb, margin)
        infos = [r.region_info(k) for k in range(len(zb) - 1)]
        r.set_image()
        st = r.iterate(n_iter)
        imgs = [r.read_region_image(k) for k in range(len(zb) - 1)]
        summed = r.read_image()
    return g, s, r_of, infos, st, imgs, summed


def test_regions_cylinder_three_slabs():
    print("case: cylinder, 3 regions", flush=True)
    w = synth.cylinder_workload(n_events=60000)
    zb = [0, 20, 40, 64]
    ev = unambiguous(w, synth.events(w), zb)
    g, s, r_of, infos, st, imgs, summed = _region_case(w, ev, zb, 4)
    plane = w.nx * w.ny
    # default margin: ceil(3 sigma / 4 mm) + ceil(6 mm / 4 mm) = 15 + 2 (no axial cut)
    assert [i["z_lo"] for i in infos] == [0, 3, 23]
    assert [i["nz"] for i in infos] == [37, 54, 41]
    total = np.zeros(w.n_voxels)
    for k, info in enumerate(infos):
        sel = r_of == k
        assert info["n_events"] == int(sel.sum())
        gk = dict(g, z0=g["z0"] + info["z_lo"] * w.voxel, nz=info["nz"])
        sk = s[info["z_lo"] * plane:(info["z_lo"] + info["nz"]) * plane].astype(np.float64)
        xk, stk = oracle.mlem(gk, ev[sel], sk, 4)
        e = oracle.rel_l2(imgs[k], xk)
        print(f"  region {k}: {info}, rel L2 {e:.2e}", flush=True)
        assert e < 1e-5
        # every event's window lies inside its sub-volume: the region rows are the whole-volume rows
        for e_ in ev[sel][:200].astype(np.float64):
            j, a = oracle.system_row(g, e_)
            iz = j // plane
            assert iz.min() >= info["z_lo"] and iz.max() < info["z_lo"] + info["nz"]
        total[info["z_lo"] * plane:(info["z_lo"] + info["nz"]) * plane] += imgs[k]
    assert np.allclose(summed, total, rtol=1e-6, atol=0)
    assert sum(q["n_eff"] for q in st[:1]) <= len(ev)


def test_regions_wholebody_nine_cores_packed_and_plain():
    print("case: whole body, 9 regions", flush=True)
    w = synth.wholebody_workload(n_events=200000)
    zb = [0, 107, 177, 240, 290, 335, 375, 410, 438, 470]
    ev = unambiguous(w, synth.events(w, n=200000), zb)
    g, s, r_of, infos, st, imgs, summed = _region_case(w, ev, zb, 3)
    assert [i["nz"] for i in infos] == [120, 96, 89, 76, 71, 66, 61, 54, 58]
    plane = w.nx * w.ny
    counts = [i["n_events"] for i in infos]
    print("  events per region", counts, flush=True)
    assert sum(counts) == len(ev) and len(ev) > 199000
    for k in (0, 4, 8):
        info = infos[k]
        sel = r_of == k
        assert info["n_events"] == int(sel.sum())
        gk = dict(g, z0=g["z0"] + info["z_lo"] * w.voxel, nz=info["nz"])
        sk = s[info["z_lo"] * plane:(info["z_lo"] + info["nz"]) * plane].astype(np.float64)
        xk, _ = oracle.mlem(gk, ev[sel], sk, 3)
        e = oracle.rel_l2(imgs[k], xk)
        print(f"  region {k} rel L2 {e:.2e}", flush=True)
        assert e < 1e-5
    # packed storage: the same split on the decoded events (oracle packer + decoder)
    dec = oracle.decode_packed(oracle.pack_events(ev))
    r_dec, amb_dec = _assign(g, dec, zb)
    keep = ~amb_dec
    _, _, _, infos_p, _, imgs_p, _ = _region_case(w, ev[keep], zb, 3, storage=1)
    for k in (0, 5):
        info = infos_p[k]
        sel = keep.copy()
        sel[keep] = r_dec[keep] == k
        assert info["n_events"] == int(sel.sum())
        gk = dict(g, z0=g["z0"] + info["z_lo"] * w.voxel, nz=info["nz"])
        sk = s[info["z_lo"] * plane:(info["z_lo"] + info["nz"]) * plane].astype(np.float64)
        xk, _ = oracle.mlem(gk, dec[sel], sk, 3)
        e = oracle.rel_l2(imgs_p[k], xk)
        print(f"  packed region {k} vs oracle on decoded events: rel L2 {e:.2e}", flush=True)
        assert e < 1e-5


def test_region_errors():
    w = synth.cylinder_workload(n_events=2000)
    ev = synth.events(w)
    with L.Reconstruction(w.geometry()) as r:
        r.load_events(ev)
        with pytest.raises(L.LmtofError) as e:
            r.set_regions([0, 32, 64])
        assert e.value.code == L.LMTOF_ESTATE
        r.compute_sensitivity()
        for bad in ([0, 32, 32, 64], [0, 70], [-1, 10]):
            with pytest.raises(L.LmtofError) as e:
                r.set_regions(bad)
            assert e.value.code == L.LMTOF_EINVAL
        r.set_regions([0, 32, 64])
        r.set_image()
        r.iterate(1)
        r.clear_regions()
        r.set_image()
        st = r.iterate(1)
        assert st[0]["n_eff"] > 1500
    g0 = dict(w.geometry(), tof_fwhm_ps=0.0)
    with L.Reconstruction(g0) as r:
        r.load_events(ev)
        r.compute_sensitivity()
        with pytest.raises(L.LmtofError) as e:
            r.set_regions([0, 32, 64])
        assert e.value.code == L.LMTOF_EUNSUPPORTED


def _mu_z_vec(g, ev, chunk=8_000_000):
    """FP64 TOF-centre z of every event (the brute-force ray's mu, vectorised)."""
    out = np.empty(len(ev))
    h = g["c_mm_per_ps"] / 2.0 if g.get("tof_fwhm_ps", 0.0) > 0 else 0.0
    for a in range(0, len(ev), chunk):
        e = ev[a:a + chunk].astype(np.float64)
        d = e[:, 3:6] - e[:, 0:3]
        out[a:a + chunk] = 0.5 * (e[:, 2] + e[:, 5]) + h * e[:, 6] * d[:, 2] / np.sqrt((d * d).sum(1))
    return out


def test_regions_wholebody_full_size():
    """The TOF-assisted division at full size (146 M whole-body events, nine
    regions in one batch, 2 iterations): regions 0, 4 and 8 (the feet, the
    middle and the head slab) against the oracle's MLEM on the events its
    FP64 TOF centres put in them.  Events within 1e-3 mm of a core boundary
    are dropped from both inputs."""
    print("case: whole body at full size, 9 regions", flush=True)
    w = synth.wholebody_workload()
    g = w.geometry()
    zb = [0, 107, 177, 240, 290, 335, 375, 410, 438, 470]
    ev = synth.events(w)
    mz = _mu_z_vec(g, ev)
    bounds = g["z0"] + np.asarray(zb, np.float64) * g["vz"]
    amb = np.zeros(len(ev), bool)
    for z in bounds[1:-1]:
        amb |= np.abs(mz - z) < 1e-3
    r_of = np.searchsorted(bounds[1:-1], mz, side="right")
    ev, r_of = ev[~amb], r_of[~amb]
    del mz
    print(f"  {len(ev)} events ({int(amb.sum())} dropped at core boundaries)", flush=True)
    s = _smooth_sens(w)
    with L.Reconstruction(g) as r:
        r.load_events(ev)
        r.set_sensitivity(s)
        r.set_regions(zb, -1)
        infos = [r.region_info(k) for k in range(len(zb) - 1)]
        r.set_image()
        r.iterate(2)
        imgs = {k: r.read_region_image(k) for k in (0, 4, 8)}
    plane = w.nx * w.ny
    assert sum(i["n_events"] for i in infos) == len(ev)
    for k in (0, 4, 8):
        info = infos[k]
        sel = r_of == k
        assert info["n_events"] == int(sel.sum())
        gk = dict(g, z0=g["z0"] + info["z_lo"] * w.voxel, nz=info["nz"])
        sk = s[info["z_lo"] * plane:(info["z_lo"] + info["nz"]) * plane].astype(np.float64)
        xk, _ = oracle.mlem(gk, ev[sel], sk, 2)
        e = oracle.rel_l2(imgs[k], xk)
        print(f"  region {k}: {info['n_events']} events, rel L2 {e:.2e}", flush=True)
        assert e < 1e-5
