"""Which quantisation of the packed record drives its error (oracle only).

Runs FP64 oracle MLEM trajectories on the whole-body workload (default
20 M events, 5 iterations, unit sensitivity) from the original events and
from events with (a) every field packed and decoded, (b) only dt through
binary16, (c) only the endpoints through the 0.1 mm int16 quantum, (d) the
endpoints at 1/60 mm (what the record's 16 spare bits would add as one
base-6 digit per coordinate: 6^6 < 2^16) with dt through binary16, and
prints each one's relative L2 distance from the original trajectory per
iteration, with the quantisation errors themselves.

    python tests/packed_error_study.py [n_events]
"""
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
import synth  # noqa: E402


def main(n: int = 20_000_000, n_iter: int = 5) -> None:
    w = synth.wholebody_workload(n_events=n)
    g = w.geometry()
    ev = synth.events(w, n=n)
    dec = oracle.decode_packed(oracle.pack_events(ev))
    ev64 = ev.astype(np.float64)
    dt_only = ev64.copy()
    dt_only[:, 6] = dec[:, 6]
    ep_only = ev64.copy()
    ep_only[:, :6] = dec[:, :6]
    sixtieth = ev64.copy()
    sixtieth[:, :6] = np.rint(ev[:, :6].astype(np.float32) * np.float32(60.0)).astype(np.float64) / 60.0
    sixtieth[:, 6] = dec[:, 6]
    s = np.ones(g["nx"] * g["ny"] * g["nz"])

    def trajectory(e):
        x = oracle.initial_image(g, s, n)
        out = []
        for _ in range(n_iter):
            x, _ = oracle.mlem(g, e, s, 1, x0=x)
            out.append(x.copy())
        return out

    t = time.time()
    ref = trajectory(ev64)
    for name, e in (("packed", dec), ("dt only", dt_only), ("endpoints only", ep_only),
                    ("1/60 mm + dt", sixtieth)):
        tr = trajectory(e)
        print(f"{name:15s}", " ".join(f"{oracle.rel_l2(a, b):.2e}" for a, b in zip(tr, ref)), flush=True)
    d = dec[:, 6] - ev64[:, 6]
    print(f"dt error: rms {np.sqrt(np.mean(d * d)):.3f} ps, max {np.abs(d).max():.3f} ps")
    d = dec[:, :6] - ev64[:, :6]
    print(f"endpoint error: rms {np.sqrt(np.mean(d * d)):.4f} mm")
    print(f"{n} events, {n_iter} iterations, {oracle.num_threads()} threads, {time.time() - t:.0f} s")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 20_000_000)
