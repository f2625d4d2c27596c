"""Serving pool: continuous batching of independent reconstructions.

- A request's image is bitwise the same whether it runs alone or batched
  with others joining and leaving at step boundaries (every kernel is
  order-independent for a given request: exact fixed-point back projection,
  per-event forward projection, per-voxel update).
- A served request matches the FP64 oracle like a plain reconstruction.
- Admission by HBM footprint: EAGAIN while it does not fit, ENOMEM if it
  never can; the pool frees a request's memory when it is polled.
- Background admission: a large request is prepared on the pool's own
  thread and stream while the running request keeps stepping.
"""
import time

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1706_07075_amd import lmtof as L  # noqa: E402
from paper_1706_07075_amd import serve  # noqa: E402


def _req(kind, n, seed, n_iter, tof=300.0, storage=0):
    if kind == "cyl":
        w = synth.cylinder_workload(n_events=n, seed=seed, tof_fwhm_ps=tof)
    elif kind == "wb":
        w = synth.wholebody_workload(n_events=n, seed=seed, tof_fwhm_ps=tof)
    else:
        raise ValueError(kind)
    ev = synth.events(w, n=n)
    return w, ev, serve.Request(geometry=w.geometry(), events=ev, n_iter=n_iter, storage=storage, name=kind)


def _run_alone(r, budget=8 << 30):
    with serve.Server(budget) as srv:
        assert srv.try_submit(r)
        while True:
            srv.step()
            if srv.poll(r):
                return r.image


def test_alone_vs_mix_bitwise():
    print("case: alone vs mix", flush=True)
    wa, eva, ra = _req("cyl", 40000, 11, 5)
    wb, evb, rb = _req("cyl", 25000, 12, 3, tof=600.0)
    wc, evc, rc = _req("wb", 60000, 13, 4)
    alone = {}
    for name, r in (("a", ra), ("b", rb), ("c", rc)):
        alone[name] = _run_alone(serve.Request(geometry=r.geometry, events=r.events, n_iter=r.n_iter))
    # mix: a starts, b joins after one step, c after two; they finish at
    # different steps (prepared before their submits return, so the joins
    # happen at exactly those steps)
    with serve.Server(8 << 30, background=False) as srv:
        assert srv.try_submit(ra)
        srv.step()
        assert srv.try_submit(rb)
        srv.step()
        assert srv.try_submit(rc)
        done = {}
        batch = []
        while len(done) < 3:
            batch.append(srv.step())
            for name, r in (("a", ra), ("b", rb), ("c", rc)):
                if name not in done and srv.poll(r):
                    done[name] = r.image
        info = srv.info()
    print(f"  batch sizes {batch}", flush=True)
    assert max(batch) == 3
    assert info["used"] == 0 and info["active"] == 0
    for name in "abc":
        assert np.array_equal(done[name], alone[name]), name


def test_served_request_matches_oracle():
    print("case: served request vs oracle", flush=True)
    w = synth.cylinder_workload(n_events=50000)
    ev = synth.events(w)
    g = w.geometry()
    img = _run_alone(serve.Request(geometry=g, events=ev, n_iter=4))
    s = oracle.sensitivity(g)
    x, _ = oracle.mlem(g, ev, s, 4)
    e = oracle.rel_l2(img, x)
    print(f"  rel L2 {e:.2e}", flush=True)
    assert e < 1e-5


def test_admission_by_footprint():
    print("case: admission", flush=True)
    w, ev, r1 = _req("cyl", 30000, 21, 2)
    _, _, r2 = _req("cyl", 30000, 22, 2)
    q, keep = L.make_request(r1.geometry, r1.events, 2)
    need = L.lmtof_pool_request_bytes(q)
    with serve.Server(int(need * 1.5)) as srv:
        assert srv.try_submit(r1)
        assert not srv.try_submit(r2)          # EAGAIN: does not fit next to r1
        while not srv.poll(r1):
            srv.step()
        assert srv.info()["used"] == 0
        assert srv.try_submit(r2)              # fits once r1 is released
        while not srv.poll(r2):
            srv.step()
    with serve.Server(need // 2) as srv:
        with pytest.raises(L.LmtofError) as e:
            srv.try_submit(r1)
        assert e.value.code == L.LMTOF_ENOMEM


def test_tof_and_nontof_not_mixed():
    w, ev, r1 = _req("cyl", 20000, 31, 3)
    g0 = dict(w.geometry(), tof_fwhm_ps=0.0)
    r0 = serve.Request(geometry=g0, events=ev, n_iter=2)
    with serve.Server(8 << 30) as srv:
        assert srv.try_submit(r1)
        assert not srv.try_submit(r0)
        while not srv.poll(r1):
            srv.step()
        assert srv.try_submit(r0)
        while not srv.poll(r0):
            srv.step()


def test_poisson_loop_small():
    print("case: Poisson loop", flush=True)
    reqs = []
    # arrivals 2 ms apart on average, each request running 30-37 iterations,
    # so that the background preparations overlap running requests
    arrivals = serve.poisson_arrivals(8, 500.0, 5)
    for k in range(8):
        kind = "cyl" if k % 3 else "wb"
        _, ev, r = _req(kind, 20000 + 5000 * k, 40 + k, 30 + k, tof=300.0 if k % 2 else 600.0)
        r.arrival = float(arrivals[k])
        reqs.append(r)
    out = serve.run(reqs, 8 << 30)
    print(f"  {out}", flush=True)
    assert out["requests"] == 8 and out["max_batch"] >= 2
    assert all(r.image is not None and np.isfinite(r.image).all() for r in reqs)
    assert out["latency_ms"]["p99"] >= out["latency_ms"]["p50"] > 0


def test_background_admission_overlaps_running_steps():
    """A whole-body request of 20 M events is admitted while a cylinder
    request is running.  Prepared before its submit returns, it would hold
    the running request for the whole preparation; in the background the
    submit returns at once, the running request keeps stepping (no step
    waits as long as the preparation), and the big request joins at a later
    step.  Both images equal their runs alone, bit for bit."""
    print("case: background admission", flush=True)
    _, _, ra = _req("cyl", 1000000, 51, 400)
    _, evb, rb = _req("wb", 20000000, 52, 2)
    rb.events = torch.from_numpy(evb).cuda()  # staged on the GPU, as the serving pools are
    img_a = _run_alone(serve.Request(geometry=ra.geometry, events=ra.events, n_iter=ra.n_iter), budget=64 << 30)
    with serve.Server(64 << 30, background=False) as srv:
        t = time.perf_counter()
        assert srv.try_submit(rb)
        t_sync = time.perf_counter() - t
        while not srv.poll(rb):
            srv.step()
        img_b = rb.image
    rb.image = None
    with serve.Server(64 << 30) as srv:
        assert srv.try_submit(ra)
        while srv.step() == 0:
            pass
        alone = []
        for _ in range(3):
            t = time.perf_counter()
            assert srv.step() == 1
            alone.append(time.perf_counter() - t)
        t = time.perf_counter()
        assert srv.try_submit(rb)
        t_submit = time.perf_counter() - t
        during = []
        while True:
            t = time.perf_counter()
            n = srv.step()
            if n == 2:
                break
            assert n == 1, "the running request stopped before the admission joined"
            during.append(time.perf_counter() - t)
        done = {}
        while len(done) < 2:
            srv.step()
            for name, r in (("a", ra), ("b", rb)):
                if name not in done and srv.poll(r):
                    done[name] = r.image
    print(f"  synchronous admission {1e3 * t_sync:.1f} ms; background submit {1e3 * t_submit:.2f} ms; "
          f"step alone {1e3 * np.median(alone):.2f} ms; {len(during)} steps during the preparation, "
          f"longest {1e3 * max(during, default=0.0):.2f} ms", flush=True)
    assert t_submit < 0.2 * t_sync
    assert len(during) >= 2
    assert max(during) < 0.5 * t_sync
    assert np.array_equal(done["a"], img_a)
    assert np.array_equal(done["b"], img_b)
