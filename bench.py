#!/usr/bin/env python3
"""Throughput benchmark: list-mode TOF MLEM on one MI355X.

One step = one whole reconstruction of the whole-body workload (150x150x600
voxels of 4 mm, 146 M events, 300 ps TOF, 10 iterations) from raw events
already resident in HBM: event ingest and bucketing sort, sensitivity,
uniform start image and 10 graph-replayed MLEM iterations.

value = events x iterations x steps / wall time of the steps
(event-iterations per second, end to end).  The same JSON line carries the
iteration-loop-only rate, the one-time costs, the projector kernel's
roofline position (algorithmic bytes over its HIP-event-timed duration) and
the FP64 oracle timed on the host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# TOF-assisted division of the whole-body grid: nine core slabs (z slices),
# feet to head
REGION_CORES = [0, 107, 177, 240, 290, 335, 375, 410, 438, 470]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_back_chunks_wholebody_146M.json")
PROJECTOR_SRC = os.path.join(ROOT, "paper_1706_07075_amd", "csrc", "project.hip")


def measured_traffic(storage):
    """HBM bytes per launch of the brick kernel from committed rocprofv3
    counter runs, if they were taken on the current projector source."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
        src = hashlib.sha256(open(PROJECTOR_SRC, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    m = rec.get(storage)
    if not m or rec.get("source_sha256") != src:
        return None
    return 1024.0 * (m["fetch_kib"] * rec["fetch_scale"] + m["write_kib"] * rec["write_scale"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--events", type=int, default=146_000_000)
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--storage", choices=["plain", "packed"], default="plain")
    ap.add_argument("--cpu-sample", type=int, default=60_000_000,
                    help="events in the oracle CPU-baseline sample (0 = skip)")
    ap.add_argument("--ept", type=int, default=0)
    ap.add_argument("--regions", action="store_true",
                    help="TOF-assisted 9-region division of the same events (one batched launch per kernel)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--tof-reject", action="store_true",
                    help="also time the TOF scatter rejection pre-pass (3 calls) against the phantom's body outline")
    ap.add_argument("--sampled", action="store_true",
                    help="also time the paper's sampled TOF projector (forward and back, 3 calls each)")
    ap.add_argument("--attenuation", action="store_true",
                    help="also time the attenuation factors of a water map over the body (3 calls) and the "
                         "iteration loop with them as event weights")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (a reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design note, not an implemented path.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1706_07075_amd import lmtof as L

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")

    if args.copy_ref_mib > 0:
        src = torch.ones(args.copy_ref_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy reference: {args.copy_ref_mib} MiB read + {args.copy_ref_mib} MiB written")
        del src, dst

    w = synth.wholebody_workload(n_events=args.events, n_iter=args.iters)
    g = w.geometry()
    t0 = time.perf_counter()
    log(f"generating {w.n_events} events ({w.name}) on {synth.num_threads()} threads")
    ev = synth.events(w)
    log(f"  done in {time.perf_counter() - t0:.1f} s")
    ev_dev = torch.from_numpy(ev).to(dev)
    torch.cuda.synchronize()

    opts = dict(storage=1 if args.storage == "packed" else 0)
    if args.ept:
        opts["events_per_thread"] = args.ept
    r = L.Reconstruction(g, device=0, **opts)

    def one_step():
        t = {}
        a = time.perf_counter()
        r.load_events(ev_dev)
        t["load_ms"] = (time.perf_counter() - a) * 1e3
        a = time.perf_counter()
        r.compute_sensitivity()
        t["sens_ms"] = (time.perf_counter() - a) * 1e3
        a = time.perf_counter()
        if args.regions:
            r.set_regions(REGION_CORES)
        r.set_image()
        t["init_ms"] = (time.perf_counter() - a) * 1e3
        a = time.perf_counter()
        st = r.iterate(w.n_iter)
        t["iter_ms"] = (time.perf_counter() - a) * 1e3
        return t, st

    tuned = None
    if not args.no_autotune:
        r.load_events(ev_dev)
        r.compute_sensitivity()
        if args.regions:
            r.set_regions(REGION_CORES)
        r.set_image()
        chosen, pass_ms = r.autotune()
        tuned = {"events_per_thread": chosen, "pass_ms": pass_ms}
        log(f"autotune: {tuned}")

    for k in range(args.warmup):
        t, st = one_step()
        log(f"warmup {k}: {t}, last iteration n_eff {st[-1]['n_eff']} sum_sx {st[-1]['sum_sx']:.6e}")

    torch.cuda.synchronize()
    times, stats = [], []
    t_start = time.perf_counter()
    for k in range(args.steps):
        a = time.perf_counter()
        t, st = one_step()
        t["step_ms"] = (time.perf_counter() - a) * 1e3
        times.append(t)
        stats.append(st)
        log(f"step {k}: {json.dumps({q: round(v, 2) for q, v in t.items()})}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    N, I, K = w.n_events, w.n_iter, args.steps
    value = N * I * K / wall
    allst = [s for st in stats for s in st]
    mean = lambda key: float(np.mean([s[key] for s in allst]))  # noqa: E731
    proj_ms, fwd_ms, back_ms = mean("project_ms"), mean("forward_ms"), mean("back_ms")
    backk_ms, upd_ms, iter_ms = mean("back_kernel_ms"), mean("update_ms"), mean("ms")
    loop_rate = N / (iter_ms * 1e-3)
    last = stats[-1][-1]

    # Algorithmic bytes (no reuse across events): an event record of E bytes
    # and one 4-byte ratio per event, one 4-byte image access per voxel piece
    # (a gather in the forward pass, a scatter-add in the back pass), and a
    # 20-byte-per-voxel update pass (x, s, b read; x written; b cleared).
    visited, weighted = r.count_segments()
    E = 16 if args.storage == "packed" else 32
    V = w.n_voxels
    bytes_back = N * (E + 4) + 4 * weighted
    bytes_fwd = N * (E + 4) + 4 * visited
    bytes_iter = N * E + 4 * (visited + weighted) + 20 * V
    gbs = lambda b, ms: b / (ms * 1e-3) / 1e9  # noqa: E731
    step_ms = [t["step_ms"] for t in times]

    out = {
        "metric": "event-iterations/s (TOF fwd+back proj) at 146M events; p50/p99 recon latency",
        "value": value,
        "unit": "event-iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": float(np.mean(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "plain" else "i16/f16 events, f32 compute",
        "data": "synthetic",
        "config": {"workload": w.name, "events": N, "iterations": I, "tof_fwhm_ps": w.tof_fwhm_ps,
                   "storage": args.storage, "regions": REGION_CORES if args.regions else None,
                   "step": "ingest+sort+sensitivity+init+10 graph-replayed iterations"},
        "autotune": tuned,
        "iter_loop_event_iterations_per_s": loop_rate,
        "recon_latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "one_time_ms": {k: float(np.mean([t[k] for t in times])) for k in ("load_ms", "sens_ms", "init_ms")},
        "iteration_ms": iter_ms,
        "kernel_ms": {"project": proj_ms, "k_forward": fwd_ms, "back_stage": back_ms, "k_back_chunks": backk_ms,
                      "update_stage": upd_ms},
        "segments_per_event": {"visited": visited / N, "weighted": weighted / N},
        "last_iteration": {"n_eff": last["n_eff"], "sum_sx": last["sum_sx"], "loglik": last["loglik"]},
        "roofline": {"bound": "hbm", "achieved": gbs(bytes_back, backk_ms), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs(bytes_back, backk_ms) / HBM_PEAK_GBS,
                     "traffic": None if args.regions else measured_traffic(args.storage),
                     "kernel": "k_back_chunks", "bytes_per_launch": bytes_back},
        "roofline_forward": {"bound": "hbm", "achieved": gbs(bytes_fwd, fwd_ms), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": gbs(bytes_fwd, fwd_ms) / HBM_PEAK_GBS,
                             "kernel": "k_forward", "bytes_per_launch": bytes_fwd},
        "roofline_iteration": {"bound": "hbm", "achieved": gbs(bytes_iter, iter_ms), "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": gbs(bytes_iter, iter_ms) / HBM_PEAK_GBS,
                               "bytes_per_event_iteration": bytes_iter / N,
                               "hbm_roofline_event_iterations_per_s": HBM_PEAK_GBS * 1e9 / (bytes_iter / N)},
    }
    if args.sampled:
        xs = torch.ones(w.n_voxels, dtype=torch.float32, device=dev)
        rs = torch.ones(N, dtype=torch.float32, device=dev)
        fw_ms, bk_ms = [], []
        for k in range(3):
            torch.cuda.synchronize()
            a = time.perf_counter()
            r.sampled_forward_project(xs)
            torch.cuda.synchronize()
            fw_ms.append((time.perf_counter() - a) * 1e3)
            a = time.perf_counter()
            r.sampled_back_project(rs)
            torch.cuda.synchronize()
            bk_ms.append((time.perf_counter() - a) * 1e3)
        out["sampled_projector"] = {"forward_ms": fw_ms, "back_ms": bk_ms, "samples_per_event": 32}
        log(f"sampled projector: {out['sampled_projector']}")
        del xs, rs
    body = None
    if args.tof_reject or args.attenuation:
        gx = g["x0"] + g["vx"] * (np.arange(g["nx"]) + 0.5)
        gy = g["y0"] + g["vy"] * (np.arange(g["ny"]) + 0.5)
        gz = g["z0"] + g["vz"] * (np.arange(g["nz"]) + 0.5)
        zz, yy, xx = np.meshgrid(gz, gy, gx, indexing="ij")
        pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
        body = (synth.phantom_eval(synth.wholebody_phantom(), pts) > 0).astype(np.uint8)
        del zz, yy, xx, pts
    if args.attenuation:
        mu = torch.from_numpy(body.astype(np.float32) * np.float32(0.0096)).to(dev)  # water at 511 keV, 1/mm
        acf_ms = []
        for k in range(3):
            torch.cuda.synchronize()
            a = time.perf_counter()
            acf = r.attenuation_factors(mu)
            torch.cuda.synchronize()
            acf_ms.append((time.perf_counter() - a) * 1e3)
        r.set_event_weights(acf)
        r.set_image()
        st_w = r.iterate(w.n_iter)
        r.set_event_weights(None)
        out["attenuation"] = {"factors_ms": acf_ms, "factor_range": [float(acf.min()), float(acf.max())],
                              "iteration_ms_weighted": float(np.mean([q["ms"] for q in st_w])),
                              "iteration_ms": iter_ms}
        log(f"attenuation: {out['attenuation']}")
        del mu, acf
    if args.tof_reject:
        mask = torch.from_numpy(body).to(dev)
        rej_ms = []
        for k in range(3):
            torch.cuda.synchronize()
            a = time.perf_counter()
            keep = r.tof_keep(mask)
            torch.cuda.synchronize()
            rej_ms.append((time.perf_counter() - a) * 1e3)
        out["tof_reject"] = {"ms": rej_ms, "kept": int(keep.sum()), "events": N,
                             "body_voxels": int(mask.sum())}
        log(f"tof reject: {out['tof_reject']}")
    r.close()
    del ev_dev
    torch.cuda.empty_cache()

    if args.cpu_sample > 0:
        import oracle
        M = min(args.cpu_sample, N)
        ev_s = ev[:M]
        s_ones = np.ones(w.n_voxels)
        log(f"cpu baseline: oracle MLEM, 1 iteration, first {M} events, {oracle.num_threads()} threads")
        a = time.perf_counter()
        oracle.mlem(g, ev_s, s_ones, 1)
        dt = time.perf_counter() - a
        out["cpu_baseline"] = {"value": M / dt, "unit": "event-iterations/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"first {M} of the {N} whole-body events, 1 MLEM iteration on the full "
                                         f"150x150x600 grid (unit sensitivity; sensitivity time excluded), "
                                         f"{dt:.1f} s"}
        log(f"  {M / dt:.3e} ev-it/s in {dt:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
