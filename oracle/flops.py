"""Algorithmic floating-point work of one hypothesis evaluation (for roofline figures).

Test infrastructure: only the tests, the benchmark's CPU baseline and the workload writer use
this module; the library never does.

W = sum_k cov_k * f_k + N * f_px, where cov_k is the number of pixels whose ray hits
primitive k (the fragments a rasteriser would shade), f_k an operation count of the
per-ray intersection of that primitive type, N the ROI pixels (Eq. 4 sums over all of them)
and f_px the per-pixel ray set-up plus the cost terms of Eq. 4.  Each add, multiply,
compare, min, square root or division counts as one operation; dense ray-primitive tests
that an implementation may perform and discard are not counted.  The per-unit counts are the
orientation figures fixed for this project's roofline before any kernel existed:

  sphere     13      cylinder (with its two caps)  60      ellipsoid  35      pixel  10

and, for the paper's own primitive set, the cylinder's count plus what the shapes add to it:

  truncated cone     70  (the radius at the reference point 2, the slope terms of the side
                          quadratic 5, two cap radii 2, a safe root for a vanishing leading
                          coefficient 1)
  elliptic cylinder  66  (the map of the ray to the unit-radius frame 6)

A second figure charges the per-pixel term only for the pixels of the 8x8 tiles that hold a
model hit: outside those tiles every pixel renders the background plane, whose Eq. 4 terms are
fixed by the observation alone and can be summed once per observation, not per hypothesis.
"""
from __future__ import annotations

import numpy as np

F_PRIM = {0: 13, 1: 60, 2: 35, 3: 70, 4: 66}
F_PIXEL = 10
TILE = 8


def hit_tile_pixels(hit, tile: int = TILE) -> int:
    """Pixels of the tile x tile blocks (clipped to the image) that contain a hit pixel."""
    hit = np.asarray(hit, bool)
    H, W = hit.shape
    total = 0
    for y0 in range(0, H, tile):
        for x0 in range(0, W, tile):
            blk = hit[y0:y0 + tile, x0:x0 + tile]
            if blk.any():
                total += blk.size
    return total


def work_counts(render_res, prim_types) -> dict:
    """Fragments per primitive type, ROI pixels and hit-tile pixels of one evaluation."""
    n = len(prim_types)
    cov = render_res["prim_hit"].reshape(n, -1).sum(axis=1)
    per_type = np.zeros(len(F_PRIM), np.int64)
    for c, t in zip(cov, prim_types):
        per_type[int(t)] += int(c)
    return {"cov_per_type": per_type, "pixels": int(render_res["depth"].size),
            "hit_tile_pixels": hit_tile_pixels(render_res["hit"])}


def flops_from_counts(cov_per_type, pixels) -> float:
    """sum_type cov_type * f_type + pixels * f_px."""
    return float(sum(float(c) * F_PRIM[t] for t, c in enumerate(cov_per_type)) +
                 float(pixels) * F_PIXEL)


def eval_flops(render_res, prim_types) -> int:
    """W of one evaluation, every ROI pixel charged with the per-pixel term."""
    w = work_counts(render_res, prim_types)
    return int(flops_from_counts(w["cov_per_type"], w["pixels"]))
