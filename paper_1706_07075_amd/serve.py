"""Continuous-batching reconstruction server on one GPU.

The pool in liblmtof.so (lmtof_pool_*) keeps admitted requests resident and
runs one batched MLEM iteration over all of them per step; this module is
the host loop around it: requests arrive (Poisson), are admitted first come
first served whenever their HBM footprint fits, are prepared in the
background (the pool's own thread and stream) while the running batch keeps
stepping, join the batch at the next step after that, and leave when their
iterations are done.  Latency is measured from arrival to the image in host
memory.

    python -m paper_1706_07075_amd.serve --requests 300 --rate 2
"""
from __future__ import annotations

import argparse
import json
import time
from dataclasses import dataclass, field
from typing import Any, Dict, List, Optional

import numpy as np

from . import lmtof as L


@dataclass(eq=False)  # identity: requests hold arrays
class Request:
    geometry: Dict[str, Any]
    events: Any                 # float32 (n, 7) NumPy array or GPU tensor
    n_iter: int
    storage: int = 0
    arrival: float = 0.0        # seconds from the start of the run
    name: str = ""
    # filled in by the server
    rid: Optional[int] = None
    admitted: Optional[float] = None
    finished: Optional[float] = None
    image: Optional[np.ndarray] = None

    @property
    def n_voxels(self) -> int:
        g = self.geometry
        return int(g["nx"]) * int(g["ny"]) * int(g["nz"])

    @property
    def n_events(self) -> int:
        return int(np.prod(self.events.shape)) // 7


class Server:
    """Thin owner of one lmtof pool."""

    def __init__(self, hbm_budget_bytes: int, device: int = 0, background: bool = True):
        self.pool = L.lmtof_pool_create(hbm_budget_bytes, device)
        self.background = background
        self._keep: Dict[int, Any] = {}  # request id -> events kept alive until polled

    def close(self):
        if getattr(self, "pool", None):
            L.lmtof_pool_destroy(self.pool)
            self.pool = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def try_submit(self, r: Request) -> bool:
        q, keep = L.make_request(r.geometry, r.events, r.n_iter, r.storage, background=self.background)
        try:
            r.rid = L.lmtof_pool_submit(self.pool, q)
        except L.LmtofError as e:
            if e.code == L.LMTOF_EAGAIN:
                return False
            raise
        self._keep[r.rid] = keep
        return True

    def step(self) -> int:
        return L.lmtof_pool_step(self.pool)

    def poll(self, r: Request) -> bool:
        img = L.lmtof_pool_poll(self.pool, r.rid, r.n_voxels)
        if img is None:
            return False
        r.image = img
        self._keep.pop(r.rid, None)
        return True

    def info(self):
        return L.lmtof_pool_info(self.pool)


def run(requests: List[Request], hbm_budget_bytes: int, device: int = 0, realtime: bool = True,
        log=None, background: bool = True) -> Dict[str, Any]:
    """Serve `requests` (sorted by arrival).  realtime=False submits each
    request as soon as it fits, ignoring arrival times (offline batch);
    background=False prepares each request before its submit returns."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    queue = list(reqs)
    running: List[Request] = []
    t0 = time.perf_counter()
    steps = 0
    batch_sizes = []
    with Server(hbm_budget_bytes, device, background) as srv:
        while queue or running:
            now = time.perf_counter() - t0
            # admit in arrival order while the head of the queue fits
            while queue and (not realtime or queue[0].arrival <= now):
                if not srv.try_submit(queue[0]):
                    if not running:
                        raise RuntimeError("a request does not fit an empty pool")
                    break
                r = queue.pop(0)
                r.admitted = time.perf_counter() - t0
                running.append(r)
            if running:
                n = srv.step()
                if n:
                    steps += 1
                    batch_sizes.append(n)
                else:
                    time.sleep(2e-4)  # every admitted request is still being prepared
                for r in list(running):
                    if srv.poll(r):
                        r.finished = time.perf_counter() - t0
                        running.remove(r)
                        if log:
                            log(f"done {r.name}: {r.n_events} events x {r.n_iter} it, "
                                f"latency {1e3 * (r.finished - r.arrival):.0f} ms")
            elif queue:
                time.sleep(max(0.0, min(queue[0].arrival - now, 0.05)))
    makespan = max(r.finished for r in reqs) - (min(r.arrival for r in reqs) if realtime else 0.0)
    lat = np.array([r.finished - (r.arrival if realtime else 0.0) for r in reqs])
    work = sum(r.n_events * r.n_iter for r in reqs)
    return {
        "requests": len(reqs),
        "steps": steps,
        "mean_batch": float(np.mean(batch_sizes)) if batch_sizes else 0.0,
        "max_batch": int(max(batch_sizes)) if batch_sizes else 0,
        "makespan_s": makespan,
        "event_iterations_per_s": work / makespan,
        "requests_per_s": len(reqs) / makespan,
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
                       "max": float(lat.max() * 1e3)},
    }


def poisson_arrivals(n: int, rate_hz: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, n))


def make_workload(n_requests: int, rate_hz: float, seed: int, max_events: int, device: str = "cuda:0",
                  pools: Optional[Dict] = None):
    """Serving workload: each request draws a kind (whole body, one body
    region, or the cylinder phantom), an event count log-uniform in
    [1M, max_events], 300 or 600 ps TOF and 5-10 iterations.  Events come
    from a few pre-generated pools held on the GPU (any prefix of a pool is a
    representative sample), so staging is done once.  `pools` may hand in
    pools generated already: {(kind, tof_ps): (workload, GPU events)}, kind
    "whole" or "cylinder"; the dict is filled with the ones generated here."""
    import torch

    import synth

    rng = np.random.default_rng(seed)
    arrivals = poisson_arrivals(n_requests, rate_hz, seed)
    if pools is None:
        pools = {}

    def pool(kind, tof):
        key = (kind, tof)
        if key not in pools:
            if kind == "cylinder":
                w = synth.cylinder_workload(n_events=min(max_events, 10_000_000), tof_fwhm_ps=tof)
            else:
                w = synth.wholebody_workload(n_events=max_events, tof_fwhm_ps=tof)
            ev = synth.events(w)
            pools[key] = (w, torch.from_numpy(ev).to(device))
        return pools[key]

    # region sub-volumes of the whole body (cores feet -> head, 4 mm slices)
    cores = [0, 107, 177, 240, 290, 335, 375, 410, 438, 470]
    region_events = {}

    def region_pool(tof, rk):
        """Events of the whole-body pool whose TOF centre lies in core rk,
        as the library's region split assigns them (Section 2.5)."""
        key = (tof, rk)
        if key not in region_events:
            w, evd = pool("whole", tof)
            if (tof, "assign") not in region_events:
                with L.Reconstruction(w.geometry(), device=int(str(device).split(":")[-1])) as r:
                    r.load_events(evd)
                    r.compute_sensitivity()
                    r.set_regions(cores)
                    region_events[(tof, "assign")] = r.event_regions(
                        torch.empty(evd.shape[0], dtype=torch.int32, device=evd.device))
            region_events[key] = evd[region_events[(tof, "assign")] == rk].contiguous()
        return region_events[key]

    reqs = []
    for k in range(n_requests):
        kind = rng.choice(["whole", "region", "cylinder"], p=[0.4, 0.4, 0.2])
        tof = float(rng.choice([300.0, 600.0]))
        n_iter = int(rng.integers(5, 11))
        w, evd = pool("cylinder" if kind == "cylinder" else "whole", tof)
        g = w.geometry()
        name = f"{kind}-{int(tof)}ps"
        if kind == "region":
            rk = int(rng.integers(0, 9))
            margin = 13 if tof <= 300 else 23  # ceil(3 sigma sin 45 deg / 4 mm) + ceil(6 mm / 4 mm)
            z_lo = max(0, cores[rk] - margin)
            nz = min(w.nz, cores[rk + 1] + margin) - z_lo
            g = dict(g, z0=g["z0"] + z_lo * w.voxel, nz=nz)
            evd = region_pool(tof, rk)
            name += f"-r{rk}"
        n = int(min(evd.shape[0], np.exp(rng.uniform(np.log(1e6), np.log(max_events)))))
        reqs.append(Request(geometry=g, events=evd[:n], n_iter=n_iter, arrival=float(arrivals[k]), name=name))
    return reqs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--rate", type=float, default=2.0)
    ap.add_argument("--seed", type=int, default=1217)
    ap.add_argument("--max-events", type=int, default=150_000_000)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    args = ap.parse_args()
    reqs = make_workload(args.requests, args.rate, args.seed, args.max_events)
    out = run(reqs, int(args.budget_gb * 2 ** 30), log=lambda m: print(m, flush=True))
    out["config"] = {"requests": args.requests, "rate_hz": args.rate, "seed": args.seed,
                     "max_events": args.max_events, "budget_gb": args.budget_gb}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
