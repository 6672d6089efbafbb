"""GPU adjoint (d cost / d pose) against the FP64 oracle's analytic gradient on pixels away
from silhouette / occlusion edges, and the autograd wrapper."""
import numpy as np
import pytest

import paper_2005_07068_amd as ht
from gpu_util import frame_for, make_ctx, particles_for, torch_cuda
from oracle import cost as ocost
from oracle import grad as ograd

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("i", [0, 1, 2, 3])
def test_adjoint_matches_fp64_gradient_on_smooth_pixels(i):
    torch = torch_cuda()
    cfg, model, fr = frame_for(2)
    poses = particles_for(model, fr, 4, seed=21, angle_deg=5.0, trans_mm=8.0)
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
    print(f"pose {i}: |g_ref|inf {scale:.4g}, max err {err:.3g}, rel {err / scale:.3g}")
    assert err <= 1e-5 * scale


@pytest.mark.parametrize("i", [3, 20])
def test_two_hand_adjoint_in_a_refinement_sized_launch(i):
    """Two hands (52 pose parameters, 32 segments) at 640x480, 32 particles in one gradient
    launch (the refinement's top-K size, where each workgroup takes about one work item with
    interleaved tiles): particle i's gradient against the FP64 analytic gradient on its smooth
    pixels (the pixel mask is particle i's; the other particles only share the launch)."""
    torch = torch_cuda()
    cfg, model, fr = frame_for(4)
    poses = particles_for(model, fr, 32, seed=31, angle_deg=5.0, trans_mm=8.0)
    h = poses[i].astype(np.float64)
    E, parts = ocost.objective(model, h, fr, return_parts=True)
    mask = ograd.fd_mask(parts["render"], fr["depth"])
    _, g_ref = ograd.analytic_gradient(model, h, fr, pixel_mask=mask)
    ctx = make_ctx(model, [fr])
    dev = torch.device("cuda:0")
    m = torch.tensor(mask.astype(np.uint8), device=dev)
    c, g = ctx.eval_grad(torch.tensor(poses, device=dev),
                         torch.zeros(1, dtype=torch.int32, device=dev), pixel_mask=m)
    ctx.close()
    g = g.cpu().numpy()[i].astype(np.float64)
    scale = np.max(np.abs(g_ref))
    err = np.max(np.abs(g - g_ref))
    print(f"pose {i}: |g_ref|inf {scale:.4g}, max err {err:.3g}, rel {err / scale:.3g}")
    assert np.count_nonzero(g_ref) > 26
    assert err <= 1e-5 * scale


def test_autograd_function_backward():
    torch = torch_cuda()
    cfg, model, fr = frame_for(0)
    poses = particles_for(model, fr, 8, seed=5)
    ctx = make_ctx(model, [fr])
    dev = torch.device("cuda:0")
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    p = torch.tensor(poses, device=dev, requires_grad=True)
    cost = ht.HandCost.apply(p, ctx, slots)
    w = torch.arange(1, 9, device=dev, dtype=torch.float32)
    (cost * w).sum().backward()
    c2, g2 = ctx.eval_grad(p.detach(), slots)
    assert torch.equal(cost.detach(), c2)
    assert torch.allclose(p.grad, w[:, None] * g2)
    c3 = ctx.eval(p.detach(), slots)
    assert torch.allclose(c3, c2, rtol=1e-6, atol=0)


def test_nonfinite_pose_gives_infinite_cost_and_zero_gradient():
    """A pose with a NaN or an infinite component scores +inf with a zero gradient (not an
    error), in a launch beside finite poses whose results are unaffected."""
    torch = torch_cuda()
    cfg, model, fr = frame_for(0)
    poses = particles_for(model, fr, 4, seed=8)
    ctx = make_ctx(model, [fr])
    dev = torch.device("cuda:0")
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    c_ref, g_ref = ctx.eval_grad(torch.tensor(poses, device=dev), slots)
    bad = poses.copy()
    bad[1, 5] = np.nan
    bad[3, 21] = -np.inf
    c, g = ctx.eval_grad(torch.tensor(bad, device=dev), slots)
    ctx.close()
    c, g = c.cpu().numpy(), g.cpu().numpy()
    c_ref, g_ref = c_ref.cpu().numpy(), g_ref.cpu().numpy()
    assert c[1] == np.inf and c[3] == np.inf
    assert np.all(g[1] == 0.0) and np.all(g[3] == 0.0)
    for i in (0, 2):
        assert c[i] == c_ref[i] and np.array_equal(g[i], g_ref[i])
        assert np.any(g[i] != 0.0)
