"""The allocation-free sampled forward projection
(lmtof_sampled_forward_project_noalloc) against the allocating entry point
(lmtof_sampled_forward_project) through the C ABI: the same kernels, so the
projections must be bit-identical, on two calls in a row with the second
one smaller, and the event limit of its fixed scratch buffer is refused
with EINVAL, leaving the context usable."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1706_07075_amd import lmtof as L  # noqa: E402

MAX_EVENTS = 1 << 22  # the scratch limit stated in include/lmtof.h


def _say(msg):
    print(msg, flush=True)


def _compare(r, x, n):
    f_ref = r.sampled_forward_project(x)
    f = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    r.sampled_forward_project_noalloc(x, f)
    torch.cuda.synchronize()
    assert f_ref.shape == f.shape == (n,)
    assert torch.equal(f, f_ref), float((f - f_ref).abs().max())
    assert float(f.sum()) > 0.0


def test_noalloc_matches_allocating_entry_point():
    w = synth.cylinder_workload(n_events=200_000)
    g = w.geometry()
    ev = synth.events(w)
    rng = np.random.default_rng(11)
    x = torch.from_numpy(rng.uniform(0.1, 2.0, w.n_voxels).astype(np.float32)).cuda()
    with L.Reconstruction(g, device=0) as r:
        for n in (200_000, 50_003):
            _say(f"case: noalloc sampled forward, {n} events")
            r.load_events(torch.from_numpy(ev[:n]).cuda())
            _compare(r, x, n)


def test_noalloc_refuses_more_events_than_its_scratch():
    w = synth.cylinder_workload(n_events=100_000)
    g = w.geometry()
    ev = synth.events(w)
    big = np.concatenate([ev] * (MAX_EVENTS // len(ev) + 1))[:MAX_EVENTS + 1]
    x = torch.ones(w.n_voxels, dtype=torch.float32, device="cuda")
    with L.Reconstruction(g, device=0) as r:
        _say(f"case: noalloc sampled forward, {len(big)} events (over the limit)")
        r.load_events(torch.from_numpy(big).cuda())
        f = torch.zeros(len(big), dtype=torch.float32, device="cuda")
        with pytest.raises(L.LmtofError) as e:
            r.sampled_forward_project_noalloc(x, f)
        assert e.value.code == L.LMTOF_EINVAL
        del f
        _say("case: noalloc sampled forward after the refusal, 1000 events")
        r.load_events(torch.from_numpy(ev[:1000]).cuda())
        _compare(r, x, 1000)
