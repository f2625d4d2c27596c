#!/usr/bin/env python3
"""Throughput benchmark: list-mode TOF MLEM on one MI355X.

One step = one whole reconstruction of the whole-body workload (150x150x600
voxels of 4 mm, 146 M events, 300 ps TOF, 10 iterations) from raw events
already resident in HBM: event ingest and bucketing sort, sensitivity,
uniform start image and 10 graph-replayed MLEM iterations.

value = events x iterations x steps / wall time of the steps
(event-iterations per second, end to end).  The same JSON line carries the
iteration-loop-only rate, the one-time costs, the dominant projector
kernel's roofline position (algorithmic bytes over its HIP-event-timed
duration), the same workload in packed storage, as a nine-region division
and as a served Poisson request stream, and the FP64 oracle timed on the
host cores on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# TOF-assisted division of the whole-body grid: nine core slabs (z slices),
# feet to head
REGION_CORES = [0, 107, 177, 240, 290, 335, 375, 410, 438, 470]
PROFILES = os.path.join(ROOT, "profiles")
PROJECTOR_SRC = os.path.join(ROOT, "paper_1706_07075_amd", "csrc", "project.hip")


def measured_traffic(kernel, storage):
    """HBM bytes per launch of `kernel` from committed rocprofv3 counter
    runs (FETCH_SIZE and WRITE_SIZE, each scaled by a copy of known size),
    if they were taken on the current projector source; else None."""
    path = os.path.join(PROFILES, f"traffic_{kernel}_wholebody_146M.json")
    try:
        rec = json.load(open(path))
        src = hashlib.sha256(open(PROJECTOR_SRC, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    m = rec.get(storage)
    if not m or rec.get("source_sha256") != src:
        return None
    return 1024.0 * (m["fetch_kib"] * rec["fetch_scale"] + m["write_kib"] * rec["write_scale"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def microbench():
    """Hardware ceilings of the GPU (libmicrobench.so), each a rate."""
    import ctypes
    import torch
    torch.cuda.init()
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1706_07075_amd", "microbench", "libmicrobench.so"))
    lib.mb_run.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    probes = [("hbm_copy_GBps", 0, 4 << 30, 1e-9), ("hbm_read_GBps", 1, 4 << 30, 1e-9),
              ("gather4B_L2_2MiB_G_per_s", 2, 2 << 20, 1e-9), ("gather4B_64MiB_G_per_s", 2, 64 << 20, 1e-9),
              ("gather4B_HBM_4GiB_G_per_s", 2, 4 << 30, 1e-9),
              ("global_atomic_add_f32_64MiB_G_per_s", 3, 64 << 20, 1e-9),
              ("global_atomic_add_f32_4GiB_G_per_s", 3, 4 << 30, 1e-9),
              ("lds_atomic_add_f32_T_per_s", 4, 4096, 1e-12), ("lds_atomic_add_u64_T_per_s", 5, 4096, 1e-12),
              ("lds_read_b32_T_per_s", 6, 4096, 1e-12), ("valu_fma_f32_T_lane_per_s", 7, 4096, 1e-12)]
    out = {}
    for name, which, nbytes, scale in probes:
        rate = ctypes.c_double()
        if lib.mb_run(which, nbytes, 5, ctypes.byref(rate)) != 0:
            raise RuntimeError(f"microbenchmark {name} failed")
        out[name] = round(rate.value * scale, 3)
        log(f"  {name}: {out[name]}")
    return out


def mean_stats(stats, key):
    return float(np.mean([s[key] for st in stats for s in st]))


def run_form(r, ev_dev, n_iter, steps, warmup, regions=False, label=""):
    """Time `steps` whole reconstructions (after `warmup`) on context r;
    returns per-step timings and per-iteration stats."""
    times, stats = [], []
    for k in range(warmup + steps):
        t = {}
        a = time.perf_counter()
        r.load_events(ev_dev)
        t["load_ms"] = (time.perf_counter() - a) * 1e3
        b = time.perf_counter()
        r.compute_sensitivity()
        t["sens_ms"] = (time.perf_counter() - b) * 1e3
        b = time.perf_counter()
        if regions:
            r.set_regions(REGION_CORES)
        r.set_image()
        t["init_ms"] = (time.perf_counter() - b) * 1e3
        b = time.perf_counter()
        st = r.iterate(n_iter)
        t["iter_ms"] = (time.perf_counter() - b) * 1e3
        t["step_ms"] = (time.perf_counter() - a) * 1e3
        if k >= warmup:
            times.append(t)
            stats.append(st)
        log(f"{label}{'warmup' if k < warmup else 'step'} {k if k < warmup else k - warmup}: "
            f"{json.dumps({q: round(v, 2) for q, v in t.items()})}")
    return times, stats


def form_summary(times, stats, N, I):
    wall = sum(t["step_ms"] for t in times) * 1e-3
    it_ms = mean_stats(stats, "ms")
    return {"event_iterations_per_s": N * I * len(times) / wall,
            "iter_loop_event_iterations_per_s": N / (it_ms * 1e-3),
            "ms_per_iteration": it_ms,
            "ms_per_step": float(np.mean([t["step_ms"] for t in times])),
            "forward_stage_ms": mean_stats(stats, "forward_ms"),
            "forward_kernel_ms": mean_stats(stats, "forward_kernel_ms"),
            "k_back_chunks_ms": mean_stats(stats, "back_kernel_ms"),
            "one_time_ms": {k: float(np.mean([t[k] for t in times])) for k in ("load_ms", "sens_ms", "init_ms")},
            "steps": len(times)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--events", type=int, default=146_000_000)
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--storage", choices=["plain", "packed"], default="plain")
    ap.add_argument("--cpu-sample", type=int, default=60_000_000,
                    help="events in the oracle CPU-baseline sample on all host threads (0 = skip)")
    ap.add_argument("--cpu-sample-1core", type=int, default=2_000_000,
                    help="events in the oracle CPU-baseline sample on one thread (0 = skip)")
    ap.add_argument("--ept", type=int, default=0)
    ap.add_argument("--sort-cell-mm", type=int, default=0,
                    help="edge of the bucketing sort's sub-cells (0: the library's default, 16 mm)")
    ap.add_argument("--forward", choices=["bricks", "events"], default="bricks",
                    help="forward projector: brick-owned (LDS-staged image bricks) or event-parallel")
    ap.add_argument("--regions", action="store_true",
                    help="headline form: the TOF-assisted 9-region division (one batched launch per kernel)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the packed, regions and serving comparison legs")
    ap.add_argument("--form-steps", type=int, default=3, help="timed reconstructions per comparison leg")
    ap.add_argument("--serve-requests", type=int, default=60, help="requests per serving leg (0 = skip)")
    ap.add_argument("--serve-rates", default="2,10", help="Poisson arrival rates (req/s) of the serving legs")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--tof-reject", action="store_true",
                    help="also time the TOF scatter rejection pre-pass (3 calls) against the phantom's body outline")
    ap.add_argument("--sampled", action="store_true",
                    help="also time the paper's sampled TOF projector (forward and back, 3 calls each)")
    ap.add_argument("--attenuation", action="store_true",
                    help="also time the attenuation factors of a water map over the body (3 calls) and the "
                         "iteration loop with them as event weights")
    ap.add_argument("--microbench", action="store_true",
                    help="only probe the hardware ceilings (HBM copy/read, random gathers, atomics, LDS, FMA)")
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

    if args.microbench:
        print(json.dumps({"microbench": microbench()}), flush=True)
        return

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

    opts = dict(storage=1 if args.storage == "packed" else 0,
                forward=L.LMTOF_FORWARD_BRICKS if args.forward == "bricks" else L.LMTOF_FORWARD_EVENTS)
    if args.ept:
        opts["events_per_thread"] = args.ept
    if args.sort_cell_mm:
        opts["sort_cell_mm"] = args.sort_cell_mm
    r = L.Reconstruction(g, device=0, **opts)

    tuned = None
    if not args.no_autotune:
        r.load_events(ev_dev)
        r.compute_sensitivity()
        if args.regions:
            r.set_regions(REGION_CORES)
        r.set_image()
        tuned = r.autotune()
        log(f"autotune: {tuned}")

    N, I, K = w.n_events, w.n_iter, args.steps
    run_form(r, ev_dev, I, 0, args.warmup, regions=args.regions)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    times, stats = run_form(r, ev_dev, I, K, 0, regions=args.regions)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    value = N * I * K / wall

    proj_ms, fwd_ms, back_ms = mean_stats(stats, "project_ms"), mean_stats(stats, "forward_ms"), mean_stats(stats, "back_ms")
    fwdk_ms = mean_stats(stats, "forward_kernel_ms")
    backk_ms, upd_ms, iter_ms = mean_stats(stats, "back_kernel_ms"), mean_stats(stats, "update_ms"), mean_stats(stats, "ms")
    loop_rate = N / (iter_ms * 1e-3)
    last = stats[-1][-1]

    # Algorithmic bytes per event-iteration (no reuse across events): the
    # event record (E bytes) once, one 4-byte image gather per voxel piece in
    # the forward pass, one 4-byte scatter-add per weighted piece in the back
    # pass, and 20 bytes per voxel for the update pass (x, s, b read; x
    # written; b cleared).  Per stage: forward N E + 4 visited, back
    # 4 weighted; per iteration their sum plus 20 V.  The forward stage is
    # timed whole (projection kernel and the pass that forms the ratios), the
    # back projection by its brick kernel alone.
    visited, weighted = r.count_segments()
    E = 16 if args.storage == "packed" else 32
    V = w.n_voxels
    bytes_fwd = N * E + 4 * visited
    bytes_back = 4 * weighted
    bytes_iter = N * E + 4 * (visited + weighted) + 20 * V
    gbs = lambda b, ms: b / (ms * 1e-3) / 1e9  # noqa: E731
    fwd_name = ("k_forward_items+k_combine" if args.forward == "bricks" else "k_block_image+k_forward+k_combine")
    kern = {fwd_name: (bytes_fwd, fwd_ms), "k_back_chunks": (bytes_back, backk_ms)}
    dom = max(kern, key=lambda k: kern[k][1])

    def roof(kname):
        b, ms = kern[kname]
        return {"bound": "hbm", "achieved": gbs(b, ms), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs(b, ms) / HBM_PEAK_GBS,
                "traffic": None if args.regions else measured_traffic(kname, args.storage),
                "kernel": kname, "bytes_per_launch": b, "launch_ms": ms}

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
        "recon_latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                             "min": float(np.min(step_ms)), "max": float(np.max(step_ms))},
        "one_time_ms": {k: float(np.mean([t[k] for t in times])) for k in ("load_ms", "sens_ms", "init_ms")},
        "iteration_ms": iter_ms,
        "kernel_ms": {"project": proj_ms, "forward_stage": fwd_ms,
                      ("k_forward_items" if args.forward == "bricks" else "k_forward"): fwdk_ms,
                      "k_combine": fwd_ms - fwdk_ms, "back_stage": back_ms, "k_back_chunks": backk_ms,
                      "update_stage": upd_ms},
        "segments_per_event": {"visited": visited / N, "weighted": weighted / N},
        "last_iteration": {"n_eff": last["n_eff"], "sum_sx": last["sum_sx"], "loglik": last["loglik"]},
        "roofline": roof(dom),
        "roofline_other": roof("k_back_chunks" if dom == fwd_name else fwd_name),
        "roofline_iteration": {"bound": "hbm", "achieved": gbs(bytes_iter, iter_ms), "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": gbs(bytes_iter, iter_ms) / HBM_PEAK_GBS,
                               "bytes_per_event_iteration": bytes_iter / N,
                               "hbm_roofline_event_iterations_per_s": HBM_PEAK_GBS * 1e9 / (bytes_iter / N)},
    }
    log(f"headline: {value:.4e} ev-it/s end to end, iteration {iter_ms:.2f} ms, "
        f"{dom} frac {out['roofline']['frac']:.3f}, iteration frac {out['roofline_iteration']['frac']:.3f}")

    if not args.no_forms and args.form_steps > 0:
        # the same events, reconstructed as the other forms, on this GPU
        if not args.regions:
            tr, sr = run_form(r, ev_dev, I, args.form_steps, 1, regions=True, label="regions ")
            out["regions"] = form_summary(tr, sr, N, I)
            out["regions"]["events_per_region"] = [r.region_info(k)["n_events"] for k in range(9)]
            r.clear_regions()
            log(f"regions: {out['regions']}")
        if args.storage == "plain":
            rp = L.Reconstruction(g, device=0, storage=1, forward=opts["forward"],
                                  **({"events_per_thread": args.ept} if args.ept else {}))
            if tuned:
                for k in ("forward", "events_per_thread", "brick_chunks"):
                    rp.set_option(k, tuned[k])
            tp, sp = run_form(rp, ev_dev, I, args.form_steps, 1, label="packed ")
            out["packed"] = form_summary(tp, sp, N, I)
            rp.close()
            log(f"packed: {out['packed']}")

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
        r.load_events(ev_dev)
        r.compute_sensitivity()
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
        r.load_events(ev_dev)
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
    torch.cuda.empty_cache()

    if not args.no_forms and args.serve_requests > 0:
        from paper_1706_07075_amd import serve
        pools = {("whole", float(w.tof_fwhm_ps)): (w, ev_dev)}
        out["serving"] = {}
        for rate in [float(q) for q in args.serve_rates.split(",") if q]:
            reqs = serve.make_workload(args.serve_requests, rate, 1217, N, pools=pools)
            log(f"serving: {len(reqs)} Poisson requests at {rate} req/s")
            res = serve.run(reqs, 200 << 30)
            res["rate_hz"] = rate
            out["serving"][f"{rate:g}hz"] = res
            log(f"  {res}")
        del pools
    del ev_dev
    torch.cuda.empty_cache()

    if args.cpu_sample > 0 or args.cpu_sample_1core > 0:
        import oracle
        s_ones = np.ones(w.n_voxels)
        cb = {"unit": "event-iterations/s", "kind": "oracle", "cpu_model": cpu_model(),
              "host_threads": os.cpu_count()}
        if args.cpu_sample > 0:
            M = min(args.cpu_sample, N)
            log(f"cpu baseline: oracle MLEM, 1 iteration, first {M} events, {oracle.num_threads()} threads")
            a = time.perf_counter()
            oracle.mlem(g, ev[:M], s_ones, 1)
            dt = time.perf_counter() - a
            cb.update(value=M / dt, cores=oracle.num_threads(),
                      sample=f"first {M} of the {N} whole-body events, 1 MLEM iteration on the full "
                             f"150x150x600 grid (unit sensitivity; sensitivity time excluded), {dt:.1f} s")
            log(f"  {M / dt:.3e} ev-it/s in {dt:.1f} s")
        if args.cpu_sample_1core > 0:
            M1 = min(args.cpu_sample_1core, N)
            n_all = oracle.num_threads()
            oracle.set_num_threads(1)
            a = time.perf_counter()
            oracle.mlem(g, ev[:M1], s_ones, 1)
            dt1 = time.perf_counter() - a
            oracle.set_num_threads(n_all)
            cb["one_core"] = {"value": M1 / dt1, "cores": 1,
                              "sample": f"first {M1} events, 1 MLEM iteration, full grid, {dt1:.1f} s"}
            log(f"  one core: {M1 / dt1:.3e} ev-it/s in {dt1:.1f} s")
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
