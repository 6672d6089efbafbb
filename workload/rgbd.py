"""Seeded synthetic RGB-D frames for the preprocessing step (data only): a hand mask and
depth from a render are painted with skin tones over a non-skin background, with a
skin-coloured distractor farther away and a non-skin object nearer than the hand."""
from __future__ import annotations

import numpy as np


def paint(hit, depth, rng: np.random.Generator, distractor_mm=1200, near_mm=None):
    """RGB uint8 [H, W, 3] and raw depth uint16 [H, W] from a hit mask and a depth map
    (mm, background already at its plane depth)."""
    H, W = hit.shape
    rgb = np.empty((H, W, 3), np.int64)
    # background: bluish-grey texture (chroma well outside the skin box)
    base = np.array([70, 90, 140])
    rgb[:] = base + rng.integers(-25, 26, size=(H, W, 3))
    # skin: tone around (205, 150, 125) with per-pixel variation
    tone = np.array([205, 150, 125]) + rng.integers(-12, 13, size=(H, W, 3))
    rgb[hit] = tone[hit]
    d = np.asarray(depth, np.float64).copy()
    # a skin-coloured distractor (a face-like disc) behind the hand
    cy, cx, rad = H * 0.25, W * 0.8, max(3, min(H, W) // 8)
    v, u = np.mgrid[0:H, 0:W]
    disc = ((v - cy) ** 2 + (u - cx) ** 2 <= rad * rad) & ~hit
    rgb[disc] = tone[disc]
    d[disc] = distractor_mm
    # a non-skin object nearer than the hand
    if near_mm is not None:
        box = (v > H * 0.75) & (u < W * 0.2) & ~hit
        rgb[box] = np.array([40, 160, 60])
        d[box] = near_mm
    return np.clip(rgb, 0, 255).astype(np.uint8), np.clip(np.round(d), 0, 65535).astype(np.uint16)
