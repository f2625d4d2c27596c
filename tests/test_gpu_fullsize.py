"""GPU parity at the full whole-body size (150x150x600 voxels of 4 mm,
146 M events, 300 ps), in the launch configuration the benchmark times.

The oracle cannot run MLEM on 146 M events in a test, so these checks use
outputs it can compute one by one, and properties that hold at any size:
- forward projection: f_i of 2000 sampled events (the oracle's system row
  times the GPU's image after one iteration), rel L2 <= 2e-6 over the
  sample and each event within 1e-4 relative;
- back projection: weights that are zero except on 5000 sampled events; the
  oracle back-projects only those, and the whole image must agree to rel L2
  <= 2e-6;
- ten iterations: sum_j s_j x_j = N_eff after every update (FP64 sums, 1e-6
  relative), x finite and non-negative;
- packed storage: the same sampled forward check on the decoded events.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

from paper_1706_07075_amd import lmtof as L  # noqa: E402


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def wb():
    w = synth.wholebody_workload()
    _say(f"generating {w.n_events} whole-body events")
    ev = synth.events(w)
    return w, ev, torch.from_numpy(ev).to("cuda:0")


def _sampled_forward(g, ev_rows, x, f_gpu):
    ref = np.array([float(np.dot(a, x[j])) for j, a in (oracle.system_row(g, e) for e in ev_rows)])
    rel = np.abs(f_gpu - ref) / np.maximum(np.abs(ref), 1e-30)
    return oracle.rel_l2(f_gpu, ref), rel[ref > 1e-6 * ref.max()].max()


def test_fullsize_plain_sampled_parity_and_invariants(wb):
    w, ev, evd = wb
    g = w.geometry()
    rng = np.random.default_rng(146)
    with L.Reconstruction(g) as r:
        r.load_events(evd)
        r.compute_sensitivity()
        r.set_image()
        st = r.iterate(1)
        x = r.read_image().astype(np.float64)
        # forward on sampled events
        f = r.forward_project(x.astype(np.float32))
        idx = rng.choice(len(ev), 2000, replace=False)
        e2, emax = _sampled_forward(g, ev[idx].astype(np.float64), x, f[idx])
        _say(f"  forward, 2000 sampled events: rel L2 {e2:.2e}, max rel {emax:.2e}")
        assert e2 < 2e-6 and emax < 1e-4
        # back projection of sparse weights
        sel = rng.choice(len(ev), 5000, replace=False)
        wts = np.zeros(len(ev), np.float32)
        wts[sel] = rng.uniform(0.5, 2.0, len(sel)).astype(np.float32)
        b = r.back_project(wts)
        bref = oracle.back(g, ev[sel].astype(np.float64), wts[sel].astype(np.float64))
        eb = oracle.rel_l2(b, bref)
        _say(f"  back, 5000 weighted events: rel L2 {eb:.2e}")
        assert eb < 2e-6
        # ten iterations: invariants (c) and (d)
        r.set_image()
        st = r.iterate(w.n_iter)
        for s in st:
            assert abs(s["sum_sx"] - s["n_eff"]) <= 1e-6 * s["n_eff"], s
        x = r.read_image()
        assert np.isfinite(x).all() and (x >= 0).all()
        _say(f"  10 iterations: n_eff {st[-1]['n_eff']}, sum s x {st[-1]['sum_sx']:.6e}")


def test_fullsize_packed_sampled_forward(wb):
    w, ev, evd = wb
    g = w.geometry()
    rng = np.random.default_rng(147)
    with L.Reconstruction(g, storage=1) as r:
        r.load_events(evd)
        r.compute_sensitivity()
        r.set_image()
        r.iterate(1)
        x = r.read_image().astype(np.float64)
        f = r.forward_project(x.astype(np.float32))
    idx = rng.choice(len(ev), 2000, replace=False)
    dec = oracle.decode_packed(oracle.pack_events(ev[idx]))
    e2, emax = _sampled_forward(g, dec, x, f[idx])
    _say(f"  packed forward, 2000 sampled events (oracle on decoded events): rel L2 {e2:.2e}, max rel {emax:.2e}")
    assert e2 < 2e-6 and emax < 1e-4
