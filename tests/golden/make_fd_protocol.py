"""Writes ``fd_protocol_adjoint320x240.npz``: the finite-difference protocol of the gradient
on the 320x240 one-hand workload frame, computed by the oracle alone.

For 32 seeded poses (the workload's particle distribution: the true pose -/+ 10 deg per angle
and 20 mm per translation, rounded to FP32 as the GPU receives them):

  * the pixel mask: ``oracle.grad.fd_protocol_mask`` (2 px from silhouette, occlusion and
    crease edges, and far enough from the kinks of |.| and min(., d_M) for the fixed steps);
  * the FP64 analytic gradient of E restricted to the mask (``analytic_gradient``);
  * the central difference of the masked smooth cost with sum(o_s or r_m) frozen at the pose,
    steps 1e-3 rad for angles and 1e-2 mm for translations (``fd_gradient``);
  * per pose parameter, the cancellation ratio sum_p |term_p| / |sum_p term_p| of the
    per-pixel terms of the depth part of the analytic gradient (0 where no pixel contributes).

The gradient is not in the paper (its cost is Eq. 4-5); this is the protocol by which the
analytic gradient, and the GPU's against it, are checked.

    python tests/golden/make_fd_protocol.py [processes]
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import cost, grad, synth  # noqa: E402
from workload import WORKLOADS, make_hand_model, seed_sequence  # noqa: E402
from workload.handmodel import perturbed_particles  # noqa: E402

OUT = os.path.join(HERE, "fd_protocol_adjoint320x240.npz")
N_POSES = 32
STEP_RAD, STEP_MM = 1e-3, 1e-2


def setup():
    cfg = WORKLOADS[2]
    model = make_hand_model(seed_sequence(2, 10_000), cfg.n_hands, cfg.primitive_set)
    fr = synth.make_frame(model, cfg, 0)
    rng = np.random.default_rng(seed_sequence(2, 32_000))
    poses = perturbed_particles(rng, fr["h_true"], N_POSES, cfg.init_angle_deg,
                                cfg.init_trans_mm, model["bounds_lo"], model["bounds_hi"])
    return model, fr, poses.astype(np.float32)


def one_pose(args):
    model, fr, pose = args
    h = pose.astype(np.float64)
    E, parts = cost.objective(model, h, fr, return_parts=True)
    mask = grad.fd_protocol_mask(model, h, parts["render"], fr, STEP_RAD, STEP_MM)
    _, g = grad.analytic_gradient(model, h, fr, pixel_mask=mask)
    g_fd = grad.fd_gradient(model, h, fr, mask, parts["S_or"], step_rad=STEP_RAD,
                            step_mm=STEP_MM)
    terms = grad.gradient_terms(model, h, fr, pixel_mask=mask).reshape(model["n_dof"], -1)
    total = np.abs(terms.sum(axis=1))
    spread = np.abs(terms).sum(axis=1)
    ratio = np.where(total > 0.0, spread / np.where(total > 0.0, total, 1.0), 0.0)
    return mask, g, g_fd, ratio, float(E), int(parts["S_or"]), int((mask & parts["render"]["hit"]).sum())


def main():
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else min(8, os.cpu_count() or 1)
    model, fr, poses = setup()
    t = time.time()
    with mp.get_context("fork").Pool(procs) as pool:
        out = pool.map(one_pose, [(model, fr, p) for p in poses], chunksize=1)
    masks, g, g_fd, ratio, E, S_or, n_hit = (np.array(v) for v in zip(*out))
    np.savez_compressed(OUT, poses=poses, masks=np.packbits(masks, axis=-1), mask_shape=masks.shape,
                        g_analytic=g, g_fd=g_fd, cancellation=ratio, cost=E, S_or=S_or,
                        mask_hit_pixels=n_hit, steps=np.array([STEP_RAD, STEP_MM]))
    rel = np.max(np.abs(g - g_fd), axis=1) / np.max(np.abs(g_fd), axis=1)
    print(f"{len(poses)} poses in {time.time() - t:.0f} s; analytic vs FD: max relative "
          f"{rel.max():.2e}; masked hit pixels {n_hit.min()}..{n_hit.max()}; cancellation "
          f"ratio median {np.median(ratio[ratio > 0]):.2f}, max {ratio.max():.1f}")


if __name__ == "__main__":
    main()
