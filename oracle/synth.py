"""Synthetic observations O = (O_s, O_d) by the simulation protocol of section V.A.1.

A seeded true pose is rendered by the oracle (``raycast``) and the render is used as the
observation, as the paper does in simulation, with a sensor-like noise model added (a
reading; the paper does not specify one): o_d = round-half-even(r_d + N(0, sigma^2)) clamped to
[1, 65535] mm, then Bernoulli(p_drop) pixels set to 0 (undefined depth); o_s = the true hit
mask with Bernoulli(p_flip) pixels flipped.  One numpy PCG64 stream per frame.
"""
from __future__ import annotations

import numpy as np

from workload import handmodel
from workload.configs import BACKGROUND_MM, camera_for_roi, seed_sequence

from . import fk, raycast


def hand_centre(model: dict, h, hand: int = 0) -> np.ndarray:
    """Centre of the axis-aligned box around the bounding spheres of one hand's primitives."""
    prims = fk.camera_primitives(model, h)
    per = model["n_prim"] // (model["n_dof"] // handmodel.DOF_PER_HAND)
    lo, hi = np.full(3, np.inf), np.full(3, -np.inf)
    for p in prims[hand * per:(hand + 1) * per]:
        if p["type"] == raycast.CYLINDER:
            r = p["size"][0]
            ends = [p["p"], p["p"] + p["size"][1] * p["R"][:, 2]]
        elif p["type"] in (raycast.CONE, raycast.ECYLINDER):
            r = max(p["size"][0], p["size"][2])
            ends = [p["p"], p["p"] + p["size"][1] * p["R"][:, 2]]
        else:
            r = float(np.max(p["size"]))
            ends = [p["p"]]
        for e in ends:
            lo, hi = np.minimum(lo, e - r), np.maximum(hi, e + r)
    return 0.5 * (lo + hi)


def place_pose(model: dict, h_raw, cam, targets_px) -> np.ndarray:
    """Set each hand's wrist x, y so its centre projects to the given pixel (u, v)."""
    h = np.array(h_raw, np.float64)
    fx, fy, cx, cy = cam
    for hand, (tu, tv) in enumerate(targets_px):
        b = hand * handmodel.DOF_PER_HAND + handmodel.WRIST_DOF
        h[b:b + 2] = 0.0
        c = hand_centre(model, h, hand)
        h[b] = (tu - cx) * c[2] / fx - c[0]
        h[b + 1] = (tv - cy) * c[2] / fy - c[1]
    return h


def true_pose(model: dict, cfg, frame: int, W: int, H: int, cam) -> np.ndarray:
    rng = np.random.default_rng(seed_sequence(cfg.idx, frame, 1))
    h = handmodel.draw_true_pose_angles(rng, cfg.n_hands)
    targets = []
    fx, fy, cx, cy = cam
    for hand in range(cfg.n_hands):
        if cfg.n_hands == 1:
            tu = cx + rng.uniform(-0.05, 0.05) * W
        else:
            # hands side by side at x = hand_x_mm at the drawn depth
            z = h[hand * handmodel.DOF_PER_HAND + 22]
            tu = cx + fx * cfg.hand_x_mm[hand] / z
        tv = cy + rng.uniform(-0.05, 0.05) * H
        targets.append((tu, tv))
    return place_pose(model, h, cam, targets)


def observe(render_res, rng, sigma=2.0, p_drop=0.05, p_flip=0.02):
    """Noise model applied to an oracle render; returns (depth uint16, skin uint8)."""
    d = render_res["depth"] + rng.normal(0.0, sigma, size=render_res["depth"].shape)
    d = np.clip(np.round(d), 1, 65535)
    d[rng.uniform(size=d.shape) < p_drop] = 0
    skin = render_res["hit"] ^ (rng.uniform(size=d.shape) < p_flip)
    return d.astype(np.uint16), skin.astype(np.uint8)


def make_frame(model: dict, cfg, frame: int) -> dict:
    W, H = cfg.frame_roi(frame)
    cam = camera_for_roi(W, H, cfg.full_frame)
    h = true_pose(model, cfg, frame, W, H, cam)
    res = raycast.render(model, h, W, H, cam, BACKGROUND_MM)
    rng = np.random.default_rng(seed_sequence(cfg.idx, frame, 2))
    depth, skin = observe(res, rng, cfg.noise_sigma_mm, cfg.dropout_p, cfg.skin_flip_p)
    return {"depth": depth, "skin": skin, "cam": cam, "bg": BACKGROUND_MM, "h_true": h}


def make_sequence(model: dict, cfg) -> list[dict]:
    """A tracked sequence: frame 0 as ``make_frame``; each later true pose is a random-walk
    step (``workload.handmodel.pose_walk_step``) of the previous one, rendered and observed
    with the same noise model."""
    W, H = cfg.frame_roi(0)
    cam = camera_for_roi(W, H, cfg.full_frame)
    frames = [make_frame(model, cfg, 0)]
    walk = np.random.default_rng(seed_sequence(cfg.idx, 3_000_000))
    h = frames[0]["h_true"]
    for t in range(1, cfg.n_frames):
        h = handmodel.pose_walk_step(walk, h, model["kc_pairs"], model["bounds_lo"],
                                     model["bounds_hi"], cfg.seq_step_deg, cfg.seq_step_mm)
        res = raycast.render(model, h, W, H, cam, BACKGROUND_MM)
        rng = np.random.default_rng(seed_sequence(cfg.idx, t, 2))
        depth, skin = observe(res, rng, cfg.noise_sigma_mm, cfg.dropout_p, cfg.skin_flip_p)
        frames.append({"depth": depth, "skin": skin, "cam": cam, "bg": BACKGROUND_MM,
                       "h_true": h})
    return frames


def clean_observation(model: dict, h, W, H, cam, bg=BACKGROUND_MM) -> dict:
    """Noise-free, dropout-free, flip-free float64 observation of pose h (for pins)."""
    res = raycast.render(model, h, W, H, cam, bg)
    return {"depth": res["depth"].copy(), "skin": res["hit"].astype(np.uint8), "cam": cam,
            "bg": bg, "h_true": np.asarray(h, np.float64)}
