"""Writes ``pso_final_errors_pso128.json``: the final global-best joint error and cost of 32
whole oracle PSO runs on the 128x128 one-hand workload frame (64 particles x 30 generations,
w = 0.72, c1 = c2 = 2.05, the worst half re-drawn every third generation; the initial box is
the true pose -/+ 10 deg and 20 mm), seeds 0..31.

Whole runs are chaotic (the swarm follows different paths once FP32 and FP64 costs order two
particles differently), so the GPU is compared with this distribution rather than run by run.
The script calls only ``oracle/`` (and the seeded workload tables for its inputs).

    python tests/golden/make_pso_final_errors.py [processes]
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import pso, synth  # noqa: E402
from workload import WORKLOADS, make_hand_model, seed_sequence  # noqa: E402
from workload.handmodel import init_halfwidth  # noqa: E402

OUT = os.path.join(HERE, "pso_final_errors_pso128.json")
SEEDS = list(range(32))
P, G = 64, 30


def setup():
    cfg = WORKLOADS[1]
    model = make_hand_model(seed_sequence(1, 10_000), cfg.n_hands, cfg.primitive_set)
    fr = synth.make_frame(model, cfg, 0)
    delta = init_halfwidth(model["n_dof"], cfg.init_angle_deg, cfg.init_trans_mm)
    # the box as the GPU receives it: FP32 bounds, clipped to the FP32 joint limits
    lo = np.maximum((fr["h_true"] - delta).astype(np.float32),
                    model["bounds_lo"].astype(np.float32)).astype(np.float64)
    hi = np.minimum((fr["h_true"] + delta).astype(np.float32),
                    model["bounds_hi"].astype(np.float32)).astype(np.float64)
    params = pso.PsoParams(w=cfg.w, c1=cfg.c1, c2=cfg.c2, mutate_every=3, mutate_frac=0.5)
    return cfg, model, fr, lo, hi, params


def joint_error_deg(h, h_true):
    """Mean |delta| over the 20 finger angles, degrees."""
    return float(np.degrees(np.mean(np.abs(np.asarray(h)[:20] - np.asarray(h_true)[:20]))))


def one(seed):
    from threadpoolctl import threadpool_limits
    cfg, model, fr, lo, hi, params = setup()
    with threadpool_limits(1):
        st, _ = pso.run(model, fr, lo, hi, P, G, params, seed)
    return {"seed": seed, "joint_error_deg": joint_error_deg(st["gbest_x"][0], fr["h_true"]),
            "gbest_cost": float(st["gbest_cost"][0])}


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else min(len(os.sched_getaffinity(0)), 16)
    t = time.perf_counter()
    with mp.get_context("fork").Pool(n) as pool:
        runs = pool.map(one, SEEDS, chunksize=1)
    out = {"workload": "pso128 (128x128, one hand, frame 0)", "particles": P, "generations": G,
           "w": 0.72, "c1": 2.05, "c2": 2.05, "mutate_every": 3, "mutate_frac": 0.5,
           "init": "true pose -/+ 10 deg, 20 mm (FP32 box, clipped to the FP32 limits)",
           "seeds": SEEDS, "runs": runs}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT} ({time.perf_counter() - t:.0f} s)")


if __name__ == "__main__":
    main()
