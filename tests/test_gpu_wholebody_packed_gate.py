"""Packed-precision gate on the whole-body workload: 146 M events, 150x150x600
voxels of 4 mm, 300 ps, 10 MLEM iterations, events stored as int16
endpoints at 0.1 mm and binary16 dt (16 bytes), ray accumulation and images
in FP32.

Two errors are measured per iteration, each as relative L2 of the GPU
image against an FP64 oracle trajectory:
- against the oracle on the ORIGINAL FP32 events: input quantisation plus
  arithmetic, gate <= 1e-3;
- against the oracle on the DECODED packed events: arithmetic only, gate
  <= 1e-5 (the plain-path target), over the first few iterations (each
  oracle iteration over 146 M events costs ~25 s on 16 host threads; the
  environment variable LMTOF_GATE_DECODED_ITERS raises the count).

The oracle's sensitivity is integrated at one voxel centre per orbit of the
centred lattice's symmetry group (x and y mirrors, x <-> y swap, z mirror),
which maps the azimuth nodes of the quadrature onto themselves, and copied
to the other voxels of the orbit; the oracle pins check each generator of
that group to 1e-12.

The per-iteration table is written to gpurun_out/packed_gate_wholebody.json,
and a progress line per oracle iteration to
gpurun_out/packed_gate_progress.txt.

The format meets the arithmetic bound and the first iteration's gate; past
the first iteration the quantisation of the endpoints exceeds 1e-3, which the
last test records as an expected (strict) failure rather than a looser bound.
"""
import json
import os
import time

import numpy as np
import pytest

import oracle
import synth
from tests import orbits

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1706_07075_amd import lmtof as L  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "gpurun_out")
GATE_ORIGINAL = 1e-3
GATE_DECODED = 1e-5


def _say(msg):
    print(msg, flush=True)
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "packed_gate_progress.txt"), "a") as fh:
        fh.write(f"{time.strftime('%H:%M:%S')} {msg}\n")


@pytest.fixture(scope="module")
def gate():
    """GPU packed trajectory and both oracle trajectories (computed once)."""
    w = synth.wholebody_workload()
    g = w.geometry()
    N, I = w.n_events, w.n_iter
    _say(f"case: packed gate, whole body, {N} events, {I} iterations")
    ev = synth.events(w)
    k_dec = min(I, int(os.environ.get("LMTOF_GATE_DECODED_ITERS", "3")))

    # GPU: packed storage (the library packs the FP32 events at load)
    xs = []
    with L.Reconstruction(g, device=0, storage=1) as r:
        r.load_events(torch.from_numpy(ev).cuda())
        r.compute_sensitivity()
        r.set_image()
        for k in range(I):
            r.iterate(1)
            xs.append(r.read_image())
    torch.cuda.empty_cache()
    _say("  GPU packed trajectory done")

    s = orbits.sensitivity_by_orbits(g)
    _say("  oracle sensitivity done")
    table = {"events": N, "iterations": I, "gate_original": GATE_ORIGINAL, "gate_decoded": GATE_DECODED,
             "original": [], "decoded": [], "oracle_threads": oracle.num_threads()}

    def trajectory(events64, n_it, key):
        x = oracle.initial_image(g, s, N)
        for k in range(n_it):
            a = time.perf_counter()
            x, _ = oracle.mlem(g, events64, s, 1, x0=x)
            e = oracle.rel_l2(xs[k], x)
            table[key].append(e)
            _say(f"  iteration {k + 1}: GPU packed vs oracle({key}) rel L2 {e:.3e} ({time.perf_counter() - a:.0f} s)")

    ev64 = ev.astype(np.float64)
    trajectory(ev64, I, "original")
    del ev64
    dec = oracle.decode_packed(oracle.pack_events(ev))
    del ev
    trajectory(dec, k_dec, "decoded")
    del dec
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "packed_gate_wholebody.json"), "w") as fh:
        json.dump(table, fh, indent=1)
    return table


def test_packed_arithmetic_matches_decoded_oracle(gate):
    """The GPU's own error on the packed events: the plain-path bound."""
    assert max(gate["decoded"]) <= GATE_DECODED, gate["decoded"]


def test_packed_first_iteration_within_gate(gate):
    assert gate["original"][0] <= GATE_ORIGINAL, gate["original"]


@pytest.mark.xfail(strict=True, reason=(
    "the packed record's input quantisation, not the arithmetic, exceeds 1e-3 from the second iteration "
    "(measured 6.6e-4, 1.2e-3, ... 5.0e-3 over 10 iterations against the oracle on the original events; "
    "1e-7 against the oracle on the decoded ones).  The 0.1 mm endpoint quantum accounts for nearly all of "
    "it, dt through binary16 for ~2 % (tests/packed_error_study.py); the error falls as 1/sqrt(events) and "
    "grows with the iterations"))
def test_packed_all_iterations_within_gate(gate):
    assert max(gate["original"]) <= GATE_ORIGINAL, gate["original"]
