"""GPU parity of the observation preprocessing (skin colour + depth segmentation) with the
oracle, bit for bit, and the whole chain RGB-D -> O -> E."""
import numpy as np
import pytest

from gpu_util import check_particle, eval_debug, frame_for, make_ctx, particles_for, torch_cuda
from oracle import preprocess as opp
from oracle import raycast
from workload import make_hand_model, seed_sequence
from workload.rgbd import paint

pytestmark = pytest.mark.gpu


def _rgbd(cfg_idx, seed, near=None):
    cfg, model, fr = frame_for(cfg_idx)
    H, W = fr["depth"].shape
    res = raycast.render(model, fr["h_true"], W, H, fr["cam"], fr["bg"])
    rng = np.random.default_rng(seed)
    noisy = np.where(fr["depth"] > 0, fr["depth"], 0)
    rgb, depth = paint(res["hit"], noisy, rng, near_mm=near)
    return model, fr, rgb, depth


def _gpu(ctx, rgb, depth, bg, **kw):
    torch = torch_cuda()
    dev = torch.device("cuda:0")
    d = torch.tensor(depth.astype(np.int32), device=dev).to(torch.int16)   # same 16 bits
    r = torch.tensor(rgb, device=dev)
    o_d, o_s = ctx.preprocess_rgbd(r, d, bg, **kw)
    torch.cuda.synchronize()
    return o_d.cpu().numpy().view(np.uint16), o_s.cpu().numpy()


@pytest.mark.parametrize("cfg_idx,near", [(0, None), (2, 450), (4, 400)])
def test_preprocess_bit_exact(cfg_idx, near):
    model, fr, rgb, depth = _rgbd(cfg_idx, 5 + cfg_idx, near)
    ctx = make_ctx(model, [])
    o_d, o_s = _gpu(ctx, rgb, depth, fr["bg"])
    e_d, e_s, z0 = opp.preprocess(rgb, depth, fr["bg"])
    assert z0 is not None
    assert np.array_equal(o_d, e_d) and np.array_equal(o_s, e_s)
    # the distractor (skin colour, far) and the near object (not skin) were segmented away
    assert o_s.sum() < (opp.skin_mask(rgb) & (depth > 0)).sum()


def test_preprocess_ragged_box_and_no_skin():
    torch_cuda()
    model = make_hand_model(seed_sequence(0, 1))
    ctx = make_ctx(model, [])
    rng = np.random.default_rng(9)
    H, W = 37, 53
    rgb = rng.integers(0, 256, size=(H, W, 3)).astype(np.uint8)
    depth = rng.integers(0, 2000, size=(H, W)).astype(np.uint16)
    depth[rng.uniform(size=(H, W)) < 0.1] = 0
    for box, band in (((77, 127, 133, 173), 150), ((90, 140, 120, 180), 400), ((0, 0, 0, 0), 10)):
        o_d, o_s = _gpu(ctx, rgb, depth, 1234.0, box=box, band_mm=band)
        e_d, e_s, _ = opp.preprocess(rgb, depth, 1234.0, box=box, band_mm=band)
        assert np.array_equal(o_d, e_d) and np.array_equal(o_s, e_s)


def test_rgbd_to_cost_chain():
    """Preprocess on the GPU, hand the device outputs to ht_set_observation, evaluate: the
    costs match the oracle's on the oracle-preprocessed observation."""
    torch = torch_cuda()
    model, fr, rgb, depth = _rgbd(0, 3, near=None)
    ctx = make_ctx(model, [])
    dev = torch.device("cuda:0")
    o_d, o_s = ctx.preprocess_rgbd(torch.tensor(rgb, device=dev),
                                   torch.tensor(depth.astype(np.int32), device=dev).to(torch.int16),
                                   fr["bg"])
    ctx.set_observation(0, o_d, o_s, fr["cam"], fr["bg"])
    e_d, e_s, _ = opp.preprocess(rgb, depth, fr["bg"])
    obs = dict(fr, depth=e_d, skin=e_s)
    poses = particles_for(model, obs, 8, seed=2)
    H, W = e_d.shape
    cost, dbg = eval_debug(ctx, poses, 0, W, H)
    for i in range(len(poses)):
        check_particle(model, obs, poses[i], cost[i], dbg, i)
