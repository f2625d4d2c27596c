"""GPU parity of the paper's sampled TOF projector (Section 2.3) against
the oracle.  Which voxel holds a sample is an integer that floating point
decides: events with a sample within 1e-3 mm of a voxel plane (by the
oracle's FP64 positions) may differ and are left out of the elementwise
comparison (and get r = 0 for the back projection); every other event must
agree to FP32 rounding."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1706_07075_amd import lmtof as L  # noqa: E402


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("storage", [0, 1])
def test_sampled_projector_against_oracle(storage):
    w = synth.cylinder_workload()
    g = w.geometry()
    ev = synth.events(w)
    evo = oracle.decode_packed(oracle.pack_events(ev)) if storage else ev
    rng = np.random.default_rng(71)
    x = rng.uniform(0.5, 1.5, w.n_voxels).astype(np.float32)
    _, _, near = oracle.sampled_system(g, evo)
    clean = near.min(axis=1) > 1e-3
    r = np.where(clean, rng.uniform(0.5, 2.0, len(ev)), 0.0).astype(np.float32)
    _say(f"case: sampled projector, 64^3, 100k events, storage {storage}; {(~clean).sum()} borderline events")
    with L.Reconstruction(g, storage=storage) as rec:
        rec.load_events(ev)
        f = rec.sampled_forward_project(x)
        b = rec.sampled_back_project(r)
        fd = rec.sampled_forward_project(torch.from_numpy(x).cuda()).cpu().numpy()
    fr = oracle.sampled_forward(g, evo, x.astype(np.float64))
    br = oracle.sampled_back(g, evo, r.astype(np.float64))
    err = np.abs(f[clean] - fr[clean]) / np.maximum(np.abs(fr[clean]), 1e-30)
    eb = oracle.rel_l2(b, br)
    _say(f"  forward max rel {err.max():.2e} (rel L2 all events {oracle.rel_l2(f, fr):.2e}), back rel L2 {eb:.2e}")
    assert err.max() < 2e-6 and oracle.rel_l2(f, fr) < 1e-2  # borderline samples may flip voxels
    assert eb < 2e-6
    assert np.array_equal(f, fd)
    # adjointness of the GPU pair
    lhs, rhs = float(f.astype(np.float64) @ r), float(x.astype(np.float64) @ b)
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)


def test_sampled_projector_needs_tof():
    w = synth.cylinder_workload()
    g = dict(w.geometry(), tof_fwhm_ps=0.0)
    ev = synth.events(w, n=1000)
    with L.Reconstruction(g) as rec:
        rec.load_events(ev)
        with pytest.raises(L.LmtofError) as e:
            rec.sampled_forward_project(np.ones(w.n_voxels, np.float32))
        assert e.value.code == L.LMTOF_EUNSUPPORTED
