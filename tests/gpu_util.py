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
MARGIN_ATOL = 1e-4         # FP32 evaluation of the margin in the debug images
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
           "winner": torch.empty((P, H, W), device=dev, dtype=torch.int32),
           "margin": torch.empty((P, H, W), device=dev, dtype=torch.float32)}
    slots = torch.tensor([slot], dtype=torch.int32, device=dev)
    p = torch.tensor(np.asarray(poses, np.float32), device=dev)
    cost = ctx.eval(p, slots, debug=dbg)
    torch.cuda.synchronize()
    return cost.cpu().numpy(), {k: (v.cpu().numpy() if k != "slot" else v) for k, v in dbg.items()}


def oracle_render(model, fr, pose):
    """The oracle's render of the FP32 pose and its pixel classification (CPU only)."""
    h = np.asarray(pose, np.float32).astype(np.float64)
    H, W = fr["depth"].shape
    res = raycast.render(model, h, W, H, fr["cam"], fr["bg"])
    return res, raycast.classify_pixels(res, MARGIN_TAU)


def _oracle_render_job(args):
    return oracle_render(*args)


def oracle_renders(model, frames_and_poses):
    """oracle_render for many (frame, pose) pairs, spread over the host cores (at most 16
    processes, started fresh: the workers run NumPy only and never touch the GPU)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os
    jobs = [(model, fr, pose) for fr, pose in frames_and_poses]
    workers = min(16, len(os.sched_getaffinity(0)), len(jobs))
    if workers <= 1:
        return [oracle_render(*j) for j in jobs]
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_oracle_render_job, jobs))


def check_particle(model, fr, pose, gpu_cost, gdbg, i, depth_rounding_atol=False,
                   rendered=None):
    """Compare one particle's GPU images and cost with the oracle; returns diagnostics.

    With ``depth_rounding_atol`` the cost may also differ by the FP32 rounding of the rendered
    depths it sums (hit pixels x one FP32 ulp of the largest depth / S_or): for an ROI of a few
    pixels E is a sub-millimetre residual and the relative bar alone is finer than FP32 depth.
    ``rendered``: the oracle_render of this pose, if already computed."""
    h = np.asarray(pose, np.float32).astype(np.float64)
    res, cls = rendered if rendered is not None else oracle_render(model, fr, pose)
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
    # the margin of the debug images: the winner's on robust hits (FP32 evaluation of the
    # oracle's definition), at most the robust-miss bound elsewhere
    if "margin" in gdbg:
        g_m = gdbg["margin"][i].astype(np.float64)
        # the GPU's nearest primitive (two entries within rounding of each other may order
        # differently from the oracle's)
        win = gdbg["winner"][i]
        yy, xx = np.nonzero(rob & (win >= 0))
        m_ref = res["prim_margin"][win[yy, xx], yy, xx]
        merr = np.abs(g_m[yy, xx] - m_ref)
        assert merr.size == 0 or merr.max() <= MARGIN_ATOL, \
            f"particle {i}: margin error {merr.max():.3e} on robust pixels"
        assert np.all(g_m[miss] < MARGIN_TAU), f"particle {i}: positive margin at a miss"
    # r_m exact where neither the hit nor the d_m test is decided by rounding
    o_d = fr["depth"].astype(np.float64)
    t_d, r_m, _, _ = ocost.pixel_terms(o_d, fr["skin"], res["depth"], res["hit"])
    rm_amb = amb | (np.abs(np.abs(o_d - res["depth"]) - ocost.D_MATCH_MM) < RM_AMBIG_MM)
    bad_rm = (g_rm != r_m) & ~rm_amb
    assert not bad_rm.any(), f"particle {i}: {bad_rm.sum()} r_m mismatches"
    r_d, hit, S_d, S_and, S_or = resolved_sums(fr, res, cls, g_depth, g_hit, g_rm)
    E = ocost.discrepancy_from_sums(S_d, S_and, S_or) + ocost.LAMBDA_K * ocost.kc(model, h)
    tol = COST_RTOL * abs(E)
    if depth_rounding_atol and S_or > 0:
        tol += int(hit.sum()) * float(np.spacing(np.float32(np.max(r_d)))) / S_or
    assert abs(gpu_cost - E) <= tol, f"particle {i}: cost {gpu_cost} vs {E}"
    return {"ambiguous": int(amb.sum()), "hits": n_hits,
            "max_depth_err": float(derr.max()) if derr.size else 0.0,
            "cost_rel": abs(gpu_cost - E) / abs(E)}


def resolved_sums(fr, res, cls, g_depth, g_hit, g_rm):
    """The resolved oracle: the GPU's decisions (r_d, hit, r_m of its debug images) at the
    pixels the oracle classifies as ambiguous (margin < 1e-5, or the d_m test within 1e-3 mm),
    the oracle's elsewhere.  Returns r_d, hit and the sums S_d, S_and, S_or of Eq. 4."""
    o_d = fr["depth"].astype(np.float64)
    amb = cls["ambiguous"]
    rm_amb = amb | (np.abs(np.abs(o_d - res["depth"]) - ocost.D_MATCH_MM) < RM_AMBIG_MM)
    r_d = np.where(amb, g_depth, res["depth"])
    hit = np.where(amb, g_hit, res["hit"])
    t_d, r_m, _, _ = ocost.pixel_terms(o_d, fr["skin"], r_d, hit)
    r_m = np.where(rm_amb, g_rm, r_m)
    o_s = fr["skin"].astype(bool)
    return r_d, hit, t_d.sum(), int((o_s & r_m).sum()), int((o_s | r_m).sum())


def resolved_gradient(model, fr, h, gdbg, i):
    """The FP64 analytic gradient of E (the oracle's formula) with the GPU's decisions, from
    its debug images of particle i at the same FP32 pose, at the pixels where the oracle finds
    them within the parity tolerances: hit (margin < 1e-5), the nearest of two surfaces
    (entries within twice the depth bar), the sign of r_d - o_d and the d_M clamp (|r_d - o_d|
    within twice the depth bar of 0 or d_M), and sum(o_s or r_m) as resolved for the cost.
    Returns (E, g) or (E, None) when the GPU hits where the oracle has no entry point (a
    margin-ambiguous miss: its depth derivative is not defined there)."""
    from oracle import grad as ograd
    h = np.asarray(h, np.float32).astype(np.float64)
    H, W = fr["depth"].shape
    res, cls = oracle_render(model, fr, h)
    g_depth = gdbg["depth"][i].astype(np.float64)
    g_hit = gdbg["hit"][i].astype(bool)
    g_win = gdbg["winner"][i]
    amb = cls["ambiguous"]
    r_d, hit, S_d, S_and, S_or = resolved_sums(fr, res, cls, g_depth, g_hit,
                                                gdbg["rm"][i].astype(bool))
    E = ocost.discrepancy_from_sums(S_d, S_and, S_or) + ocost.LAMBDA_K * ocost.kc(model, h)
    if np.any(amb & g_hit & ~res["hit"]):
        return E, None
    # the nearest surface: the GPU's where two entries are within twice the depth bar
    pt = np.sort(res["prim_t"], axis=0)
    with np.errstate(invalid="ignore"):
        crease = res["hit"] & (pt[1] - pt[0] < 2 * DEPTH_TOL_MM)
    swap = crease & g_hit & (g_win >= 0) & (g_win != res["winner"])
    rr = res
    if swap.any():
        win = res["winner"].copy()
        win[swap] = g_win[swap]
        zmin = res["zmin"].copy()
        yy, xx = np.nonzero(swap)
        zmin[swap] = res["prim_t"][win[swap], yy, xx]
        if not np.all(np.isfinite(zmin[swap])):
            return E, None
        rr = dict(res, winner=win, zmin=zmin)
    dz = ograd.depth_gradient(model, h, rr, W, H, fr["cam"])
    # s_p with the GPU's depth where its sign or clamp is decided within twice the depth bar
    o_d = fr["depth"].astype(np.float64)
    diff = res["depth"] - o_d
    close = (np.abs(diff) < 2 * DEPTH_TOL_MM) | \
        (np.abs(np.abs(diff) - ocost.D_CLAMP_MM) < 2 * DEPTH_TOL_MM)
    diff = np.where(close | amb, g_depth - o_d, diff)
    s = np.where(hit & (np.abs(diff) < ocost.D_CLAMP_MM), np.sign(diff), 0.0)
    g = np.einsum("jhw,hw->j", dz, s) / S_or if S_or > 0 else np.zeros(model["n_dof"])
    return E, g + ocost.LAMBDA_K * ocost.kc_grad(model, h)
