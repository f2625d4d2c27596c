"""GPU parity of the attenuation correction on the LOR (Section 2.4)
against the oracle: correction factors exp(line integral of mu), and MLEM
with per-event ratio weights."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1706_07075_amd import lmtof as L  # noqa: E402


def _say(msg):
    print(msg, flush=True)


def _water_map(w):
    """mu of water at 511 keV (0.0096 / mm) inside the cylinder phantom, 0 outside."""
    g = w.geometry()
    nx, ny, nz = g["nx"], g["ny"], g["nz"]
    x = g["x0"] + g["vx"] * (np.arange(nx) + 0.5)
    y = g["y0"] + g["vy"] * (np.arange(ny) + 0.5)
    z = g["z0"] + g["vz"] * (np.arange(nz) + 0.5)
    zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    return np.where(synth.phantom_eval(synth.cylinder_phantom(), pts) > 0, 0.0096, 0.0).astype(np.float32)


@pytest.fixture(scope="module")
def cyl():
    w = synth.cylinder_workload()
    g = w.geometry()
    ev = synth.events(w)
    mu = _water_map(w)
    acf = oracle.attenuation_factors(g, ev, mu.astype(np.float64))
    return dict(w=w, g=g, ev=ev, mu=mu, acf=acf)


def test_attenuation_factors(cyl):
    _say("case: attenuation factors, 64^3, 100k events")
    with L.Reconstruction(cyl["g"]) as r:
        r.load_events(cyl["ev"])
        a = r.attenuation_factors(cyl["mu"])
        ad = r.attenuation_factors(torch.from_numpy(cyl["mu"]).cuda()).cpu().numpy()
    ref = cyl["acf"]
    rel = np.abs(a - ref) / ref
    _say(f"  rel L2 {oracle.rel_l2(a, ref):.2e}, max rel {rel.max():.2e}, factors {ref.min():.3f}..{ref.max():.3f}")
    assert oracle.rel_l2(a, ref) < 1e-6 and rel.max() < 1e-5
    assert np.array_equal(a, ad)
    assert ref.max() > 2.0  # the map attenuates


def test_weighted_mlem(cyl):
    """Two iterations with the oracle's attenuation factors (rounded to FP32)
    as event weights against the oracle's weighted MLEM from the same FP32
    start and sensitivity; unit weights give the unweighted result bit for
    bit; dropping the weights restores it."""
    w, g, ev = cyl["w"], cyl["g"], cyl["ev"]
    s = np.random.default_rng(61).uniform(0.5, 1.5, w.n_voxels).astype(np.float32)
    x0 = np.full(w.n_voxels, 0.05, np.float32)
    wt = cyl["acf"].astype(np.float32)
    _say("case: weighted MLEM, 64^3, 100k events, 2 iterations")
    with L.Reconstruction(g) as r:
        r.load_events(ev)
        r.set_sensitivity(s)
        r.set_image(x0)
        r.iterate(2)
        x_plain = r.read_image()
        r.set_event_weights(np.ones(len(ev), np.float32))
        r.set_image(x0)
        r.iterate(2)
        x_unit = r.read_image()
        r.set_event_weights(wt)
        r.set_image(x0)
        st = r.iterate(2)
        x_w = r.read_image()
        r.set_event_weights(None)
        r.set_image(x0)
        r.iterate(2)
        x_back = r.read_image()
        with pytest.raises(L.LmtofError) as e:
            r.set_event_weights(np.ones(len(ev) - 1, np.float32))
        assert e.value.code == L.LMTOF_EINVAL
    assert np.array_equal(x_unit, x_plain) and np.array_equal(x_back, x_plain)
    xr = oracle.mlem_weighted(g, ev, s.astype(np.float64), 2, wt.astype(np.float64), x0.astype(np.float64))
    e = oracle.rel_l2(x_w, xr)
    _say(f"  weighted rel L2 {e:.2e}")
    assert e < 1e-5
    # normalisation: sum s x after the second iteration equals the weight sum over events with f > 0
    f = oracle.forward(g, ev, oracle.mlem_weighted(g, ev, s.astype(np.float64), 1, wt.astype(np.float64),
                                                   x0.astype(np.float64)))
    assert abs(st[1]["sum_sx"] - wt.astype(np.float64)[f > 0].sum()) < 1e-5 * wt.sum()
