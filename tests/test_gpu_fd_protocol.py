"""GPU adjoint against the FP64 analytic gradient of the finite-difference protocol on the
320x240 workload frame (32 seeded poses, each with its protocol mask as the pixel mask),
stored by tests/golden/make_fd_protocol.py from the oracle alone."""
import os

import numpy as np
import pytest

from gpu_util import frame_for, make_ctx, torch_cuda

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fd_protocol_adjoint320x240.npz")


def test_adjoint_matches_the_fd_protocol_gradients():
    torch = torch_cuda()
    d = np.load(GOLDEN)
    masks = np.unpackbits(d["masks"], axis=-1)[..., :int(d["mask_shape"][-1])]
    cfg, model, fr = frame_for(2)
    ctx = make_ctx(model, [fr])
    dev = torch.device("cuda:0")
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    worst = 0.0
    for i, pose in enumerate(d["poses"]):
        m = torch.tensor(masks[i], dtype=torch.uint8, device=dev)
        c, g = ctx.eval_grad(torch.tensor(pose[None], device=dev), slots, pixel_mask=m)
        g = g.cpu().numpy()[0].astype(np.float64)
        g_ref = d["g_analytic"][i]
        scale = np.max(np.abs(g_ref))
        err = np.max(np.abs(g - g_ref))
        worst = max(worst, err / scale)
        assert err <= 1e-5 * scale, (i, err / scale)
        # the cost beside it: the oracle's (stored) up to pixels decided within the margin,
        # which the cost parity tests resolve (one such pixel moves E by about 1e-4)
        assert abs(float(c.cpu()[0]) - d["cost"][i]) <= 1e-3 * d["cost"][i], i
    ctx.close()
    c = d["cancellation"]
    print(f"fd protocol: 32 poses, worst relative gradient difference {worst:.2e}; "
          f"cancellation ratio median {np.median(c[c > 0]):.2f}, max {c.max():.1f}")


def test_per_frame_slot_masks_in_one_gradient_call():
    """The protocol's masks set per frame slot (ht_set_pixel_mask): one gradient call over two
    frames (the same observation in slots 0 and 1, each slot with the mask of its own pose, one
    pose per frame) meets the protocol bar against the stored FP64 gradients of both poses; a
    one-frame call with only the slot mask equals the call that passes the same mask as its
    pixel_mask bit for bit; None, and a new observation of the slot, clear the mask (the call
    is then the unmasked one, bit for bit)."""
    torch = torch_cuda()
    d = np.load(GOLDEN)
    masks = np.unpackbits(d["masks"], axis=-1)[..., :int(d["mask_shape"][-1])]
    cfg, model, fr = frame_for(2)
    ctx = make_ctx(model, [fr, fr])
    dev = torch.device("cuda:0")
    i0, i1 = 3, 17
    ctx.set_pixel_mask(0, masks[i0])
    ctx.set_pixel_mask(1, torch.tensor(masks[i1], dtype=torch.uint8, device=dev))
    poses = torch.tensor(np.stack([d["poses"][i0], d["poses"][i1]])[:, None], device=dev)
    both = torch.tensor([0, 1], dtype=torch.int32, device=dev)
    _, g = ctx.eval_grad(poses, both)
    for f, i in enumerate((i0, i1)):
        g_ref = d["g_analytic"][i]
        err = np.max(np.abs(g.cpu().numpy()[f, 0].astype(np.float64) - g_ref))
        assert err <= 1e-5 * np.max(np.abs(g_ref)), (f, i, err)
    one = torch.zeros(1, dtype=torch.int32, device=dev)
    c_slot, g_slot = ctx.eval_grad(poses[0], one)
    m0 = torch.tensor(masks[i0], dtype=torch.uint8, device=dev)
    c_call, g_call = ctx.eval_grad(poses[0], one, pixel_mask=m0)
    assert torch.equal(c_slot, c_call) and torch.equal(g_slot, g_call)
    # the call's own mask is used instead of the slot's
    ones = torch.ones_like(m0)
    _, g_all = ctx.eval_grad(poses[0], one, pixel_mask=ones)
    ctx.set_pixel_mask(0, None)
    _, g_none = ctx.eval_grad(poses[0], one)
    assert torch.equal(g_all, g_none) and not torch.equal(g_none, g_slot)
    ctx.set_pixel_mask(0, masks[i0])
    ctx.set_observation(0, fr["depth"], fr["skin"], fr["cam"], fr["bg"])
    _, g_new = ctx.eval_grad(poses[0], one)
    assert torch.equal(g_new, g_none)
    with pytest.raises(ValueError):
        ctx.set_pixel_mask(1, masks[i0][:-1])
    ctx.close()
