"""Shared helpers of the GPU parity tests: contexts, seeded frames and the resolved-oracle
comparison of the parity bar (exact masks outside margin < 1e-5 pixels, 1e-3 mm depths,
1e-5 relative costs)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import cost as ocost
from oracle import raycast, synth
from workload import WORKLOADS, make_hand_model, seed_sequence
from workload.handmodel import perturbed_particles

MARGIN_TAU = 1e-5          # pixels whose ray-surface margin is below this are ambiguous
DEPTH_TOL_MM = 1e-3
COST_RTOL = 1e-5
RM_AMBIG_MM = 1e-3         # | |o_d - r_d| - d_m | below this: r_m decided by float rounding
# the ambiguous pixels are excluded from the exact comparisons, so their number is bounded:
# at most this fraction of the hit pixels (one pixel allowed in any case)
MAX_AMBIGUOUS_FRAC = 0.005


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def frame_for(cfg_idx: int, frame: int = 0, model_seed: int = 0,
              primitive_set: str = "cylinders"):
    cfg = WORKLOADS[cfg_idx]
    model = make_hand_model(seed_sequence(cfg_idx, 10_000 + model_seed), cfg.n_hands,
                            primitive_set)
    fr = synth.make_frame(model, cfg, frame)
    return cfg, model, fr


def particles_for(model, fr, n, seed, angle_deg=10.0, trans_mm=20.0):
    rng = np.random.default_rng(seed)
    p = perturbed_particles(rng, fr["h_true"], n, angle_deg, trans_mm, model["bounds_lo"],
                            model["bounds_hi"])
    return p.astype(np.float32)


def make_ctx(model, frames):
    import paper_2005_07068_amd as ht
    ctx = ht.Context(0)
    ctx.set_model(model)
    for slot, fr in enumerate(frames):
        ctx.set_observation(slot, fr["depth"], fr["skin"], fr["cam"], fr["bg"])
    return ctx


def eval_debug(ctx, poses, slot, W, H):
    torch = torch_cuda()
    dev = torch.device("cuda:0")
    P = len(poses)
    dbg = {"slot": slot,
           "depth": torch.empty((P, H, W), device=dev, dtype=torch.float32),
           "hit": torch.empty((P, H, W), device=dev, dtype=torch.uint8),
           "rm": torch.empty((P, H, W), device=dev, dtype=torch.uint8),
           "winner": torch.empty((P, H, W), device=dev, dtype=torch.int32)}
    slots = torch.tensor([slot], dtype=torch.int32, device=dev)
    p = torch.tensor(np.asarray(poses, np.float32), device=dev)
    cost = ctx.eval(p, slots, debug=dbg)
    torch.cuda.synchronize()
    return cost.cpu().numpy(), {k: (v.cpu().numpy() if k != "slot" else v) for k, v in dbg.items()}


def check_particle(model, fr, pose, gpu_cost, gdbg, i, depth_rounding_atol=False):
    """Compare one particle's GPU images and cost with the oracle; returns diagnostics.

    With ``depth_rounding_atol`` the cost may also differ by the FP32 rounding of the rendered
    depths it sums (hit pixels x one FP32 ulp of the largest depth / S_or): for an ROI of a few
    pixels E is a sub-millimetre residual and the relative bar alone is finer than FP32 depth."""
    h = np.asarray(pose, np.float32).astype(np.float64)
    H, W = fr["depth"].shape
    res = raycast.render(model, h, W, H, fr["cam"], fr["bg"])
    cls = raycast.classify_pixels(res, MARGIN_TAU)
    amb = cls["ambiguous"]
    n_hits = int(res["hit"].sum())
    assert amb.sum() <= max(1, MAX_AMBIGUOUS_FRAC * n_hits), \
        f"particle {i}: {amb.sum()} ambiguous pixels for {n_hits} hits"
    g_hit = gdbg["hit"][i].astype(bool)
    g_depth = gdbg["depth"][i].astype(np.float64)
    g_rm = gdbg["rm"][i].astype(bool)
    bad_hit = (g_hit != res["hit"]) & ~amb
    assert not bad_hit.any(), f"particle {i}: {bad_hit.sum()} hit/miss mismatches off the margin"
    rob = cls["robust_hit"]
    derr = np.abs(g_depth - res["depth"])[rob]
    assert derr.size == 0 or derr.max() <= DEPTH_TOL_MM, \
        f"particle {i}: depth error {derr.max():.3e} mm on robust pixels"
    miss = cls["robust_miss"]
    assert np.all(g_depth[miss] == res["depth"][miss])
    # r_m exact where neither the hit nor the d_m test is decided by rounding
    o_d = fr["depth"].astype(np.float64)
    t_d, r_m, _, _ = ocost.pixel_terms(o_d, fr["skin"], res["depth"], res["hit"])
    rm_amb = amb | (np.abs(np.abs(o_d - res["depth"]) - ocost.D_MATCH_MM) < RM_AMBIG_MM)
    bad_rm = (g_rm != r_m) & ~rm_amb
    assert not bad_rm.any(), f"particle {i}: {bad_rm.sum()} r_m mismatches"
    # resolved oracle: the GPU's decisions at ambiguous pixels, the oracle's elsewhere
    r_d = np.where(amb, g_depth, res["depth"])
    hit = np.where(amb, g_hit, res["hit"])
    t_d, r_m, _, _ = ocost.pixel_terms(o_d, fr["skin"], r_d, hit)
    r_m = np.where(rm_amb, g_rm, r_m)
    o_s = fr["skin"].astype(bool)
    S_d, S_and, S_or = t_d.sum(), int((o_s & r_m).sum()), int((o_s | r_m).sum())
    E = ocost.discrepancy_from_sums(S_d, S_and, S_or) + ocost.LAMBDA_K * ocost.kc(model, h)
    tol = COST_RTOL * abs(E)
    if depth_rounding_atol and S_or > 0:
        tol += int(hit.sum()) * float(np.spacing(np.float32(np.max(r_d)))) / S_or
    assert abs(gpu_cost - E) <= tol, f"particle {i}: cost {gpu_cost} vs {E}"
    return {"ambiguous": int(amb.sum()), "hits": n_hits,
            "max_depth_err": float(derr.max()) if derr.size else 0.0,
            "cost_rel": abs(gpu_cost - E) / abs(E)}
