"""GPU parity on the degenerate cases of the cost (Eq. 4-5) against the FP64 oracle: S_or = 0,
a hypothesis that renders nothing (outside the view, or behind the background plane), an
observation without any defined depth, and ROIs smaller than one tile (down to 1x1)."""
import numpy as np
import pytest

from gpu_util import check_particle, eval_debug, frame_for, make_ctx, torch_cuda
from oracle import cost as ocost
from oracle import synth

pytestmark = pytest.mark.gpu


def _eval(ctx, poses):
    torch = torch_cuda()
    dev = torch.device("cuda:0")
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    return ctx.eval(torch.tensor(np.asarray(poses, np.float32), device=dev), slots).cpu().numpy()


def _away(model, h, dx=0.0, dz=0.0):
    """Pose h with its wrist moved by (dx, 0, dz) mm (every hand)."""
    g = np.array(h, np.float64)
    for k in range(model["n_dof"] // 26):
        g[26 * k + 20] += dx
        g[26 * k + 22] += dz
    return g.astype(np.float32)


def test_s_or_zero_gives_lambda():
    """No skin and a hypothesis that renders nothing: S_or = 0, so D = lambda exactly and
    E = lambda + lambda_k kc."""
    torch_cuda()
    cfg, model, fr = frame_for(0)
    fr = dict(fr)
    fr["skin"] = np.zeros_like(fr["skin"])
    h = _away(model, fr["h_true"], dx=5000.0)
    ctx = make_ctx(model, [fr])
    c = _eval(ctx, [h])
    ctx.close()
    E = ocost.objective(model, h.astype(np.float64), fr)
    assert E == ocost.LAMBDA + ocost.LAMBDA_K * ocost.kc(model, h.astype(np.float64))
    assert abs(c[0] - E) <= 1e-6 * E


@pytest.mark.parametrize("where", ["outside", "behind"])
def test_hypothesis_that_renders_nothing(where):
    """All-miss hypotheses (the hand far to the side, or beyond the background plane at 1.5 m):
    every pixel renders the background; the cost matches the oracle's."""
    torch_cuda()
    cfg, model, fr = frame_for(1)
    h = _away(model, fr["h_true"], dx=5000.0) if where == "outside" else \
        _away(model, fr["h_true"], dz=2000.0)
    H, W = fr["depth"].shape
    ctx = make_ctx(model, [fr])
    cost, dbg = eval_debug(ctx, [h], 0, W, H)
    ctx.close()
    assert not dbg["hit"].any()
    assert np.all(dbg["depth"] == np.float32(fr["bg"]))
    check_particle(model, fr, h, cost[0], dbg, 0)


def test_observation_without_defined_depth():
    """Every depth pixel undefined (0): each pixel's depth term is the clamp d_M and every
    rendered pixel is matched (r_m = hit)."""
    torch_cuda()
    cfg, model, fr = frame_for(1)
    fr = dict(fr)
    fr["depth"] = np.zeros_like(fr["depth"])
    H, W = fr["depth"].shape
    poses = [fr["h_true"].astype(np.float32), _away(model, fr["h_true"], dx=15.0)]
    ctx = make_ctx(model, [fr])
    cost, dbg = eval_debug(ctx, poses, 0, W, H)
    ctx.close()
    for i in range(len(poses)):
        check_particle(model, fr, poses[i], cost[i], dbg, i)
        assert np.array_equal(dbg["rm"][i].astype(bool), dbg["hit"][i].astype(bool))


@pytest.mark.parametrize("W,H", [(1, 1), (1, 9), (9, 1), (7, 7), (8, 1), (1, 8)])
def test_roi_smaller_than_a_tile(W, H):
    """ROIs of one pixel up to one partial tile, looking at the hand's centre."""
    torch_cuda()
    cfg, model, fr0 = frame_for(1)
    h = fr0["h_true"]
    # the hand's centre at the middle of the ROI
    c = synth.hand_centre(model, h, 0)
    cam = (600.0, 600.0, (W - 1) / 2.0 - 600.0 * c[0] / c[2], (H - 1) / 2.0 - 600.0 * c[1] / c[2])
    ob = synth.clean_observation(model, h, W, H, cam)
    fr = {"depth": np.clip(np.round(ob["depth"]), 0, 65535).astype(np.uint16),
          "skin": ob["skin"].astype(np.uint8), "cam": cam, "bg": ob["bg"], "h_true": h}
    poses = [h.astype(np.float32), _away(model, h, dx=3.0), _away(model, h, dx=5000.0)]
    ctx = make_ctx(model, [fr])
    cost, dbg = eval_debug(ctx, poses, 0, W, H)
    ctx.close()
    for i in range(len(poses)):
        check_particle(model, fr, poses[i], cost[i], dbg, i, depth_rounding_atol=True)


def test_gradient_of_a_hypothesis_that_renders_nothing():
    """Nothing rendered: the depth term has no gradient, so dE/dh is the collision term's alone,
    -/+ lambda_k on the two angles of each violated pair (pairs violated on purpose here)."""
    torch = torch_cuda()
    cfg, model, fr = frame_for(1)
    h = _away(model, fr["h_true"], dx=5000.0).astype(np.float64)
    used, n = set(), 0
    for a, b in model["kc_pairs"]:              # violate two pairs with no angle in common
        if n < 2 and a not in used and b not in used:
            h[a], h[b] = -0.2, 0.1
            used |= {int(a), int(b)}
            n += 1
    h = h.astype(np.float32)
    ctx = make_ctx(model, [fr])
    dev = torch.device("cuda:0")
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    c, g = ctx.eval_grad(torch.tensor(h[None], device=dev), slots)
    ctx.close()
    g = g.cpu().numpy()[0]
    ref = ocost.LAMBDA_K * ocost.kc_grad(model, h.astype(np.float64))
    assert np.count_nonzero(ref) >= 4
    assert np.array_equal(g, ref.astype(np.float32))
    E = ocost.objective(model, h.astype(np.float64), fr)
    assert abs(c.cpu().numpy()[0] - E) <= 1e-5 * E


@pytest.mark.parametrize("tilt", [0.0, 4e-4, -7e-4])
def test_cylinder_seen_along_its_axis(tilt):
    """A cylinder whose axis runs along the optical axis, 2-3 mm off it, so that the principal
    point's ray (and, tilted by a fraction of a milliradian, a ray next to it) lies within
    1e-3 rad of the axis: such rays take the slab-centred reference and the side test at the
    slab's middle, and their wavefront takes the general path.  Depths, masks and costs
    against the FP64 oracle; the principal point's pixel hits the near cap."""
    from oracle import fk, raycast
    from workload import CYLINDER, make_hand_model, seed_sequence
    torch_cuda()
    m = make_hand_model(seed_sequence(0, 4243), 1)
    m = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in m.items()}
    m["n_prim"] = 1
    m["prim_type"] = np.array([CYLINDER], np.int32)
    m["prim_seg"] = np.zeros(1, np.int32)
    frame = np.zeros((1, 3, 4))
    frame[0, :, :3] = np.eye(3)
    frame[0, :, 3] = (2.0, -3.0, 0.0)
    m["prim_frame"] = frame
    m["prim_size"] = np.array([[9.0, 30.0, 0.0]])
    W, H = 96, 64
    # pixel (48, 32) looks along the optical axis, its neighbours 1e-3 rad off it; the
    # cylinder's image is a disc of about 950 pixels
    cam = (1000.0, 1000.0, 48.0, 32.0)
    h = np.zeros(26)
    h[22] = 520.0
    h[23] = tilt
    rng = np.random.default_rng(6)
    res = raycast.render(m, h, W, H, cam, 1500.0)
    depth, skin = synth.observe(res, rng)
    fr = {"depth": depth, "skin": skin, "cam": cam, "bg": 1500.0, "h_true": h}
    # what the test exercises: hit pixels whose rays lie within 1e-3 rad of the axis
    cyl = fk.camera_primitives(m, h)[0]
    d = raycast.pixel_directions(W, H, cam)
    cos = (d @ cyl["R"][:, 2]) / np.linalg.norm(d, axis=-1)
    near = res["hit"] & (np.sqrt(np.maximum(1.0 - cos ** 2, 0.0)) < 1e-3)
    assert near[32, 48] and near.sum() >= 1
    poses = [h.astype(np.float32), _away(m, h, dx=1.0), _away(m, h, dz=-40.0)]
    ctx = make_ctx(m, [fr])
    cost, dbg = eval_debug(ctx, poses, 0, W, H)
    ctx.close()
    for i in range(len(poses)):
        check_particle(m, fr, poses[i], cost[i], dbg, i)
    assert dbg["hit"][0][32, 48] == 1
