"""Write the seeded synthetic observations of the workloads to workload/data/*.npz.

Every stored value comes from the CPU oracle: a seeded true pose per frame is rendered by the
oracle and the noise model of the workloads is applied (the simulation protocol of section
V.A.1 with sensor noise); the algorithmic work per evaluation (for roofline figures) comes
from the oracle's coverage counts on a sample of particles drawn like the swarm's initial
particles.

    python -m workload.make_data            # all configs
    python -m workload.make_data 1 4        # some
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

from oracle import flops, raycast, synth
from workload import WORKLOADS, make_hand_model, seed_sequence
from workload.handmodel import perturbed_particles

DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def model_seed(idx: int):
    return seed_sequence(idx, 10_000)


def make(idx: int, flop_samples: int = 8) -> str:
    cfg = WORKLOADS[idx]
    model = make_hand_model(model_seed(idx), cfg.n_hands, cfg.primitive_set)
    out = {}
    cams, hs = [], []
    seq = synth.make_sequence(model, cfg) if cfg.sequence else None
    for f in range(cfg.n_frames):
        fr = seq[f] if seq is not None else synth.make_frame(model, cfg, f)
        out[f"depth_{f}"] = fr["depth"]
        out[f"skin_{f}"] = fr["skin"]
        cams.append(fr["cam"])
        hs.append(fr["h_true"])
    out["cam"] = np.array(cams, np.float64)
    out["h_true"] = np.array(hs, np.float64)
    out["bg"] = np.float64(synth.BACKGROUND_MM)
    # algorithmic work per evaluation on particles drawn like the swarm's initial ones: the
    # fragments per primitive type, the ROI pixels and the pixels of the 8x8 tiles holding a
    # model hit, and the FLOP figures built from them
    rng = np.random.default_rng(seed_sequence(idx, 20_000))
    covs, pixels, tile_px = [], [], []
    frames = rng.choice(cfg.n_frames, size=min(flop_samples, cfg.n_frames), replace=False) \
        if cfg.n_frames > 1 else np.zeros(1, int)
    per_frame = max(1, flop_samples // len(frames))
    for f in frames:
        H, W = out[f"depth_{f}"].shape
        poses = perturbed_particles(rng, out["h_true"][f], per_frame, cfg.init_angle_deg,
                                    cfg.init_trans_mm, model["bounds_lo"], model["bounds_hi"])
        for h in poses:
            res = raycast.render(model, h, W, H, tuple(out["cam"][f]), synth.BACKGROUND_MM)
            w = flops.work_counts(res, model["prim_type"])
            covs.append(w["cov_per_type"])
            pixels.append(w["pixels"])
            tile_px.append(w["hit_tile_pixels"])
    out["cov_per_eval"] = np.mean(np.array(covs, np.float64), axis=0)
    out["pixels_per_eval"] = np.float64(np.mean(pixels))
    out["hit_tile_pixels_per_eval"] = np.float64(np.mean(tile_px))
    out["flops_per_eval"] = np.float64(flops.flops_from_counts(out["cov_per_eval"],
                                                               out["pixels_per_eval"]))
    out["flops_hit_tiles_per_eval"] = np.float64(
        flops.flops_from_counts(out["cov_per_eval"], out["hit_tile_pixels_per_eval"]))
    out["flops_sample"] = np.int64(len(covs))
    os.makedirs(DATA, exist_ok=True)
    path = os.path.join(DATA, f"config{idx}.npz")
    np.savez_compressed(path, **out)
    return path


if __name__ == "__main__":
    which = [int(a) for a in sys.argv[1:]] or sorted(WORKLOADS)
    for i in which:
        t = time.time()
        p = make(i)
        print(f"config {i}: {p} ({os.path.getsize(p) / 1e6:.2f} MB, {time.time() - t:.1f} s)",
              flush=True)
