"""GPU parity with the paper's primitive set (section II.A: truncated-cone phalanges, an
elliptic-cylinder palm capped by ellipsoids, joint spheres, an ellipsoidal thumb phalanx)
against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

from gpu_util import (check_particle, eval_debug, frame_for, make_ctx, oracle_renders,
                      particles_for, torch_cuda)
from oracle import cost as ocost
from oracle import grad as ograd
from oracle import raycast, synth
from workload import CONE, ECYLINDER, make_hand_model, seed_sequence

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg_idx,n", [(0, 16), (2, 16), (5, 16)])
def test_paper_model_parity_masks_depths_costs(cfg_idx, n):
    """The paper's primitive set at 64x64 and 320x240 (one hand) and 640x480 (two hands, the
    workload-5 frame): every particle against the resolved oracle."""
    cfg, model, fr = frame_for(cfg_idx, primitive_set="paper")
    per_hand = 1 if cfg_idx != 5 else 2
    assert (model["prim_type"] == CONE).sum() == 14 * per_hand
    assert (model["prim_type"] == ECYLINDER).sum() == per_hand
    poses = particles_for(model, fr, n, seed=11)
    poses[0] = fr["h_true"].astype(np.float32)
    H, W = fr["depth"].shape
    ctx = make_ctx(model, [fr])
    cost, dbg = eval_debug(ctx, poses, 0, W, H)
    ctx.close()
    rendered = oracle_renders(model, [(fr, poses[i]) for i in range(n)])
    diags = [check_particle(model, fr, poses[i], cost[i], dbg, i, rendered=rendered[i])
             for i in range(n)]
    print("paper model", cfg_idx, diags[:3])
    # the cones and the palm are really seen
    res = rendered[0][0]
    seen = model["prim_type"][res["winner"][res["hit"]]]
    assert (seen == CONE).sum() > 0.01 * W * H and (seen == ECYLINDER).sum() > 0.002 * W * H


def _end_on_model():
    """A one-hand model whose palm carries only a widening cone and an elliptic cylinder with
    their axes pointing away from the camera: rays enter through the near caps and, around
    them, through the cone's flank at angles steeper than the flank (alpha < 0)."""
    m = make_hand_model(seed_sequence(0, 4242), 1, "paper")
    m = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in m.items()}
    m["n_prim"] = 2
    m["prim_type"] = np.array([CONE, ECYLINDER], np.int32)
    m["prim_seg"] = np.zeros(2, np.int32)
    fr = np.zeros((2, 3, 4))
    fr[:, :, :3] = np.eye(3)
    fr[0, :, 3] = (-22.0, 0.0, 0.0)
    fr[1, :, 3] = (25.0, 5.0, 0.0)
    m["prim_frame"] = fr
    m["prim_size"] = np.array([[9.0, 30.0, 20.0], [14.0, 25.0, 7.0]])
    return m


def test_end_on_cone_flank_and_caps():
    torch_cuda()
    model = _end_on_model()
    W, H = 96, 64
    cam = (260.0, 260.0, 47.5, 31.5)
    h = np.zeros(26)
    h[22] = 520.0
    h[24] = np.deg2rad(8.0)
    rng = np.random.default_rng(4)
    res = raycast.render(model, h, W, H, cam, 1500.0)
    depth, skin = synth.observe(res, rng)
    fr = {"depth": depth, "skin": skin, "cam": cam, "bg": 1500.0, "h_true": h}
    poses = particles_for(model, fr, 8, seed=12, angle_deg=3.0, trans_mm=4.0)
    poses[0] = h.astype(np.float32)
    ctx = make_ctx(model, [fr])
    cost, dbg = eval_debug(ctx, poses, 0, W, H)
    for i in range(len(poses)):
        check_particle(model, fr, poses[i], cost[i], dbg, i)
    # what the test exercises: flank entries of the cone with alpha < 0, and cap entries
    from oracle import fk
    cone = fk.camera_primitives(model, h)[0]
    d = raycast.pixel_directions(W, H, cam)
    e = d @ cone["R"]
    k = (cone["size"][2] - cone["size"][0]) / cone["size"][1]
    alpha = e[..., 0] ** 2 + e[..., 1] ** 2 - (k * e[..., 2]) ** 2
    flank = res["hit"] & (res["winner"] == 0) & (res["prim_surface"][0] == 0)
    assert (flank & (alpha < 0)).sum() > 50
    for j in (0, 1):
        assert (res["hit"] & (res["winner"] == j) & (res["prim_surface"][j] == 1)).sum() > 50


@pytest.mark.parametrize("i", [0, 1, 2])
def test_paper_model_adjoint_matches_fp64_gradient(i):
    torch = torch_cuda()
    cfg, model, fr = frame_for(2, primitive_set="paper")
    poses = particles_for(model, fr, 3, seed=31, angle_deg=5.0, trans_mm=8.0)
    h = poses[i].astype(np.float64)
    E, parts = ocost.objective(model, h, fr, return_parts=True)
    mask = ograd.fd_mask(parts["render"], fr["depth"])
    _, g_ref = ograd.analytic_gradient(model, h, fr, pixel_mask=mask)
    ctx = make_ctx(model, [fr])
    dev = torch.device("cuda:0")
    m = torch.tensor(mask.astype(np.uint8), device=dev)
    c, g = ctx.eval_grad(torch.tensor(poses[i:i + 1], device=dev),
                         torch.zeros(1, dtype=torch.int32, device=dev), pixel_mask=m)
    g = g.cpu().numpy()[0].astype(np.float64)
    scale = np.max(np.abs(g_ref))
    err = np.max(np.abs(g - g_ref))
    print(f"paper pose {i}: |g_ref|inf {scale:.4g}, max err {err:.3g}, rel {err / scale:.3g}")
    assert err <= 1e-5 * scale
