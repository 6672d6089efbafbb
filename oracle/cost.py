"""Discrepancy D (Eq. 4), collision term kc and objective E (Eq. 5), in float64.

Per pixel (section III.A): r_m = 1 where the model depth r_d differs from the observed depth
o_d by less than d_m or o_d is undefined; the reading used here also requires a model hit
(r_m is the model's matched-depth mask, so background pixels are never "matched model").
Undefined observed depth is o_d == 0.  Then, with the sums over every pixel of the ROI,

  D = sum min(|o_d - r_d|, d_M) / sum(o_s or r_m)
      + lambda * (1 - 2 sum(o_s and r_m) / (sum(o_s and r_m) + sum(o_s or r_m)))
  kc = sum over the three adjacent non-thumb finger pairs of -min(phi, 0),
       phi = abduction(finger nearer the thumb) - abduction(other finger)
  E = D + lambda_k * kc

with d_m = 1 cm, d_M = 4 cm, lambda = 20, lambda_k = 10 (values of section III.A; lengths in
mm here).  If sum(o_s or r_m) == 0 (empty skin mask and nothing matched) the reading is
D = lambda.  A pose with a non-finite component scores +inf.
"""
from __future__ import annotations

import numpy as np

from . import raycast

D_MATCH_MM = 10.0     # d_m
D_CLAMP_MM = 40.0     # d_M
LAMBDA = 20.0
LAMBDA_K = 10.0


def pixel_terms(o_d, o_s, r_d, hit):
    """Per-pixel (clamped depth difference, r_m, o_s and r_m, o_s or r_m)."""
    o_d = np.asarray(o_d, np.float64)
    o_s = np.asarray(o_s).astype(bool)
    hit = np.asarray(hit).astype(bool)
    diff = np.abs(o_d - np.asarray(r_d, np.float64))
    t_d = np.minimum(diff, D_CLAMP_MM)
    r_m = hit & ((diff < D_MATCH_MM) | (o_d == 0.0))
    return t_d, r_m, o_s & r_m, o_s | r_m


def discrepancy_from_sums(S_d, S_and, S_or):
    if S_or == 0:
        return LAMBDA
    return S_d / S_or + LAMBDA * (1.0 - 2.0 * S_and / (S_and + S_or))


def discrepancy(o_d, o_s, r_d, hit):
    """Eq. 4 from per-pixel images; returns (D, S_d, S_and, S_or)."""
    t_d, r_m, a, o = pixel_terms(o_d, o_s, r_d, hit)
    S_d, S_and, S_or = float(np.sum(t_d)), int(np.sum(a)), int(np.sum(o))
    return discrepancy_from_sums(S_d, S_and, S_or), S_d, S_and, S_or


def kc(model: dict, h) -> float:
    h = np.asarray(h, np.float64)
    total = 0.0
    for a, b in model["kc_pairs"]:
        phi = h[a] - h[b]
        total += -min(phi, 0.0)
    return total


def kc_grad(model: dict, h) -> np.ndarray:
    h = np.asarray(h, np.float64)
    g = np.zeros_like(h)
    for a, b in model["kc_pairs"]:
        if h[a] - h[b] < 0.0:
            g[a] -= 1.0
            g[b] += 1.0
    return g


def objective(model: dict, h, obs: dict, return_parts: bool = False):
    """E(h, O) of Eq. 5 for one hypothesis.  ``obs`` holds depth (H, W), skin (H, W),
    cam (fx, fy, cx, cy) and bg (background plane depth)."""
    h = np.asarray(h, np.float64)
    if not np.all(np.isfinite(h)):
        return (np.inf, {}) if return_parts else np.inf
    H, W = obs["depth"].shape
    res = raycast.render(model, h, W, H, obs["cam"], obs["bg"])
    D, S_d, S_and, S_or = discrepancy(obs["depth"], obs["skin"], res["depth"], res["hit"])
    k = kc(model, h)
    E = D + LAMBDA_K * k
    if return_parts:
        return E, {"D": D, "S_d": S_d, "S_and": S_and, "S_or": S_or, "kc": k, "render": res}
    return E
