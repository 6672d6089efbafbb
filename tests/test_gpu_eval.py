"""GPU parity of the evaluation path (kinematics, ray cast, Eq. 4-5 cost, reduction) against
the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import paper_2005_07068_amd as ht

from gpu_util import (check_particle, eval_debug, frame_for, make_ctx, oracle_renders,
                      particles_for, torch_cuda)
from oracle import synth
from workload import WORKLOADS, make_hand_model, seed_sequence
from workload.configs import camera_for_roi

pytestmark = pytest.mark.gpu


def test_fwd64_parity_masks_depths_costs():
    """64x64 workload: 40 primitives, 16 particles around the true pose."""
    cfg, model, fr = frame_for(0)
    poses = particles_for(model, fr, cfg.n_particles, seed=1)
    poses[0] = fr["h_true"].astype(np.float32)
    ctx = make_ctx(model, [fr])
    cost, dbg = eval_debug(ctx, poses, 0, 64, 64)
    diags = [check_particle(model, fr, poses[i], cost[i], dbg, i) for i in range(len(poses))]
    print("fwd64", diags[:3])
    assert sum(d["hits"] for d in diags) > 1000


def test_ragged_roi_and_off_centre_camera():
    """ROI sizes that are not multiples of the 8x8 tile, a non-square camera (fx != fy)."""
    model = make_hand_model(seed_sequence(0, 777))
    W, H = 61, 53
    cam = (150.0, 128.0, 29.0, 27.5)
    rng = np.random.default_rng(5)
    from workload.handmodel import draw_true_pose_angles
    h = synth.place_pose(model, draw_true_pose_angles(rng), cam, [(31.0, 26.0)])
    from oracle import raycast
    res = raycast.render(model, h, W, H, cam, 1500.0)
    depth, skin = synth.observe(res, rng)
    fr = {"depth": depth, "skin": skin, "cam": cam, "bg": 1500.0, "h_true": h}
    poses = particles_for(model, fr, 6, seed=3)
    ctx = make_ctx(model, [fr])
    cost, dbg = eval_debug(ctx, poses, 0, W, H)
    for i in range(len(poses)):
        check_particle(model, fr, poses[i], cost[i], dbg, i)


def test_no_background_plane_and_far_hand():
    """B <= 0 (misses render 0) and a hypothesis entirely out of view."""
    cfg, model, fr = frame_for(0, model_seed=1)
    fr = dict(fr, bg=0.0)
    poses = particles_for(model, fr, 4, seed=7)
    poses[3, 20] += 3000.0
    ctx = make_ctx(model, [fr])
    cost, dbg = eval_debug(ctx, poses, 0, 64, 64)
    for i in range(len(poses)):
        check_particle(model, fr, poses[i], cost[i], dbg, i)
    assert not dbg["hit"][3].any()


def test_debug_and_plain_costs_identical_and_deterministic():
    torch = torch_cuda()
    cfg, model, fr = frame_for(1)
    poses = particles_for(model, fr, 64, seed=2)
    ctx = make_ctx(model, [fr])
    c_dbg, _ = eval_debug(ctx, poses, 0, 128, 128)
    dev = torch.device("cuda:0")
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    p = torch.tensor(poses, device=dev)
    c1 = ctx.eval(p, slots).cpu().numpy()
    c2 = ctx.eval(p, slots).cpu().numpy()
    assert np.array_equal(c1, c2)
    assert np.array_equal(c1, c_dbg)
    for tpi, gpc, cull in ((4, 1, 0), (64, 8, 1), (16, 2, 0)):
        ctx.set_launch_config(tpi, gpc, cull)
        c3 = ctx.eval(p, slots).cpu().numpy()
        assert np.allclose(c3, c1, rtol=1e-6, atol=0)


@pytest.mark.parametrize("prims", ["cylinders", "paper"])
def test_culling_is_conservative_on_two_hand_frames(prims):
    """640x480, two hands: launches with and without the capsule culling (image extent and
    image-segment reach) give bit-identical costs and per-pixel images, near the true pose and
    far from it."""
    torch_cuda()
    cfg, model, fr = frame_for(4, primitive_set=prims)
    near = particles_for(model, fr, 12, seed=9)
    far = particles_for(model, fr, 6, seed=10, angle_deg=40.0, trans_mm=80.0)
    poses = np.concatenate([near, far])
    ctx = make_ctx(model, [fr])
    H, W = fr["depth"].shape
    out = {}
    for cull in (0, 1):
        ctx.set_launch_config(16, 4, cull)
        out[cull] = eval_debug(ctx, poses, 0, W, H)
    ctx.close()
    (c0, d0), (c1, d1) = out[0], out[1]
    assert np.array_equal(c0, c1)
    for k in ("depth", "hit", "rm", "winner"):
        assert np.array_equal(d0[k], d1[k]), k
    assert d1["hit"].any()


def test_nonfinite_pose_unset_slot_and_empty_call():
    torch = torch_cuda()
    cfg, model, fr = frame_for(0)
    poses = particles_for(model, fr, 3, seed=4)
    poses[1, 7] = np.nan
    poses[2, 22] = np.inf
    ctx = make_ctx(model, [fr])
    dev = torch.device("cuda:0")
    c = ctx.eval(torch.tensor(poses, device=dev), torch.zeros(1, dtype=torch.int32, device=dev))
    c = c.cpu().numpy()
    assert np.isfinite(c[0]) and c[1] == np.inf and c[2] == np.inf
    # a frame slot that was never set scores NaN (no fault) and raises the device error flag;
    # slot numbers out of range too
    assert ctx.device_errors() == 0
    c = ctx.eval(torch.tensor(poses[:1], device=dev),
                 torch.full((1,), 5, dtype=torch.int32, device=dev)).cpu().numpy()
    assert np.isnan(c[0])
    assert ctx.device_errors(reset=True) == ht.HT_DEVERR_UNSET_SLOT
    assert ctx.device_errors() == 0
    c = ctx.eval(torch.tensor(poses[:1], device=dev),
                 torch.full((1,), -3, dtype=torch.int32, device=dev)).cpu().numpy()
    assert np.isnan(c[0]) and ctx.device_errors(reset=True) == ht.HT_DEVERR_UNSET_SLOT
    empty = torch.zeros((0, model["n_dof"]), device=dev)
    out = ctx.eval(empty, torch.zeros(1, dtype=torch.int32, device=dev))
    assert out.numel() == 0


def test_batched_frames_equal_per_frame_calls_and_the_oracle():
    """The uneven-ROI workload's frames (48..192 px per side): one batched launch over 8 frames
    x 16 particles == one call per frame, bit for bit; every cost of the batched launch against
    the resolved oracle at the 1e-5 bar (the per-frame debug calls, bit-identical to the
    batched launch, give the GPU's decisions at ambiguous pixels)."""
    torch = torch_cuda()
    cfg = WORKLOADS[3]
    model = make_hand_model(seed_sequence(3, 10_000))
    frames = [synth.make_frame(model, cfg, f) for f in range(8)]
    ctx = make_ctx(model, frames)
    dev = torch.device("cuda:0")
    P = 16
    poses = np.stack([particles_for(model, fr, P, seed=10 + i) for i, fr in enumerate(frames)])
    slots = torch.arange(len(frames), dtype=torch.int32, device=dev)
    batched = ctx.eval(torch.tensor(poses, device=dev), slots).cpu().numpy()
    dbgs = []
    for f, fr in enumerate(frames):
        one = ctx.eval(torch.tensor(poses[f], device=dev),
                       torch.tensor([f], dtype=torch.int32, device=dev)).cpu().numpy()
        assert np.array_equal(one, batched[f])
        H, W = fr["depth"].shape
        c_dbg, dbg = eval_debug(ctx, poses[f], f, W, H)
        assert np.array_equal(c_dbg, batched[f])
        dbgs.append(dbg)
    ctx.close()
    rendered = oracle_renders(model, [(frames[f], poses[f, i]) for f in range(len(frames))
                                      for i in range(P)])
    rel = []
    for f, fr in enumerate(frames):
        for i in range(P):
            d = check_particle(model, fr, poses[f, i], batched[f, i], dbgs[f], i,
                               rendered=rendered[f * P + i])
            rel.append(d["cost_rel"])
    print(f"batched: {len(rel)} costs, max relative difference {max(rel):.2e}")
    assert len({fr["depth"].shape for fr in frames}) == len(frames)   # uneven ROIs


def test_full_size_adjoint_shape_sampled_particles():
    """320x240 workload (256 particles in one launch): every cost computed, every 8th
    particle (32, first and last included) against the resolved oracle."""
    cfg, model, fr = frame_for(2)
    poses = particles_for(model, fr, cfg.n_particles, seed=11)
    ctx = make_ctx(model, [fr])
    cost, dbg = eval_debug(ctx, poses, 0, 320, 240)
    ctx.close()
    assert np.all(np.isfinite(cost))
    idx = list(range(0, 256, 8)) + [255]
    rendered = oracle_renders(model, [(fr, poses[i]) for i in idx])
    for i, rd in zip(idx, rendered):
        check_particle(model, fr, poses[i], cost[i], dbg, i, rendered=rd)


def test_full_frame_two_hands_sampled_particles():
    """640x480 workload: two hands (80 primitives, 52-D), 1024 particles in one launch; 32 of
    them (every 32nd, first and last included) against the resolved oracle."""
    cfg, model, fr = frame_for(4)
    poses = particles_for(model, fr, cfg.n_particles, seed=12)
    ctx = make_ctx(model, [fr])
    cost, dbg = eval_debug(ctx, poses, 0, 640, 480)
    ctx.close()
    assert np.all(np.isfinite(cost))
    idx = list(range(0, 1024, 33)) + [1023]
    assert len(idx) >= 32
    rendered = oracle_renders(model, [(fr, poses[i]) for i in idx])
    for i, rd in zip(idx, rendered):
        check_particle(model, fr, poses[i], cost[i], dbg, i, rendered=rd)


def test_camera_helper_and_config_shapes():
    assert camera_for_roi(64, 64) == (144.0, 144.0, 31.5, 31.5)
    assert camera_for_roi(640, 480, True)[0] == 575.0


def test_launch_shapes_and_autotuner_keep_costs_bit_identical():
    """Every launch shape gives bit-identical costs (partials are combined in item order and
    the FP64 depth sums are exact), the autotuner returns one of its candidates and keeps it,
    and out-of-range shapes are rejected."""
    import paper_2005_07068_amd as ht
    torch = torch_cuda()
    cfg, model, fr = frame_for(4)
    poses = particles_for(model, fr, 64, seed=9)
    ctx = make_ctx(model, [fr])
    dev = torch.device("cuda:0")
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    x = torch.tensor(poses, device=dev)
    ref = None
    for tpi, gpc, cull in [(4, 1, 0), (16, 2, 1), (64, 8, 1), (1024, 64, 1), (8, 3, 0)]:
        ctx.set_launch_config(tpi, gpc, cull)
        assert ctx.launch_config() == (tpi, gpc, cull)
        c = ctx.eval(x, slots).cpu().numpy()
        if ref is None:
            ref = c
        assert np.array_equal(c, ref), (tpi, gpc, cull)
    lc = ctx.autotune(x[None], slots, repeats=2)
    assert lc[0] in (4, 8, 16, 32, 64) and lc[1] in (1, 2, 4, 8) and lc[2] in (0, 1)
    assert ctx.launch_config() == lc
    assert np.array_equal(ctx.eval(x, slots).cpu().numpy(), ref)
    for bad in [(3, 1, 1), (2048, 1, 1), (16, 0, 1), (16, 65, 1), (16, 1, 2)]:
        with pytest.raises(Exception):
            ctx.set_launch_config(*bad)
    assert ctx.launch_config() == lc
    ctx.close()


def test_work_lists_built_in_the_ray_cast_and_by_the_work_list_kernel_agree():
    """Launches of at most 256 particles build their work list inside the ray cast (items in a
    static stride, at most six workgroups per CU); larger ones take the work-list kernel's list
    and the dequeue counter.  The same particles evaluated in one launch of 300, in launches of
    256 + 44 and of 150 + 150 (and with debug images, which always take the work-list kernel)
    get bit-identical costs, and the device counts every evaluation once; gradients (FP32
    wrench rows summed per item, items cut differently) agree to 1e-5 of the largest
    component."""
    torch = torch_cuda()
    cfg, model, fr = frame_for(4)
    P = 300
    poses = particles_for(model, fr, P, seed=21)
    ctx = make_ctx(model, [fr])
    dev = torch.device("cuda:0")
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    x = torch.tensor(poses, device=dev)
    ctx.eval_counts(reset=True)
    whole = ctx.eval(x, slots).cpu().numpy()
    for cut in (256, 150):
        parts = np.concatenate([ctx.eval(x[:cut], slots).cpu().numpy(),
                                ctx.eval(x[cut:], slots).cpu().numpy()])
        assert np.array_equal(parts, whole), cut
    assert ctx.eval_counts(reset=True) == (3 * P, 0)
    H, W = fr["depth"].shape
    c_dbg, _ = eval_debug(ctx, poses[:40], 0, W, H)
    assert np.array_equal(c_dbg, whole[:40])
    c_all, g_all = ctx.eval_grad(x, slots)
    c_cut = torch.cat([ctx.eval_grad(x[:256], slots)[0], ctx.eval_grad(x[256:], slots)[0]])
    g_cut = torch.cat([ctx.eval_grad(x[:256], slots)[1], ctx.eval_grad(x[256:], slots)[1]])
    assert np.array_equal(c_all.cpu().numpy(), whole) and torch.equal(c_cut, c_all)
    g_all, g_cut = g_all.cpu().numpy(), g_cut.cpu().numpy()
    scale = np.max(np.abs(g_all), axis=1, keepdims=True)
    assert np.all(np.abs(g_cut - g_all) <= 1e-5 * scale)
    ctx.close()


def test_self_scheduled_workgroup_with_two_items_of_one_particle():
    """A self-scheduled launch gives workgroup g the items g, g + grid, ...; with one workgroup
    per CU, four tiles per item and a hand that covers more than four tiles per CU (a three
    times upsampled 1920x1440 observation, focal lengths tripled) a workgroup takes two items of the
    same particle back to back, with no staging between them.  Its cost equals, bit for bit,
    the one the work-list kernel's launch (300 copies of the particle) and the debug launch
    give; the gradient agrees to 1e-5 of its largest component."""
    torch = torch_cuda()
    cfg, model, fr = frame_for(4)
    pose = particles_for(model, fr, 1, seed=21)
    up = 3
    depth = np.repeat(np.repeat(fr["depth"], up, axis=0), up, axis=1)
    skin = np.repeat(np.repeat(fr["skin"], up, axis=0), up, axis=1)
    fx, fy, cx, cy = (float(c) for c in fr["cam"])
    # pixel u of the source image is pixels up u .. up u + up - 1 here (centre up u + 1)
    cam = (up * fx, up * fy, up * cx + (up - 1) / 2, up * cy + (up - 1) / 2)
    ctx = make_ctx(model, [dict(fr, depth=depth, skin=skin, cam=cam)])
    ctx.set_launch_config(4, 1, 1)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    H, W = depth.shape
    c_dbg, dbg = eval_debug(ctx, pose, 0, W, H)
    hit = dbg["hit"][0] == 1
    hit_tiles = hit[:H // 8 * 8, :W // 8 * 8].reshape(H // 8, 8, W // 8, 8).any(axis=(1, 3))
    # more than 4 n_cu tiles in the hand's region: more items of 4 tiles than workgroups
    assert hit_tiles.sum() > 4 * n_cu, (hit_tiles.sum(), n_cu)
    dev = torch.device("cuda:0")
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    x1 = torch.tensor(pose, device=dev)
    x300 = x1.expand(300, -1).contiguous()
    one = ctx.eval(x1, slots).cpu().numpy()
    many = ctx.eval(x300, slots).cpu().numpy()
    assert np.array_equal(one, c_dbg) and np.all(many == one[0])
    g1 = ctx.eval_grad(x1, slots)[1].cpu().numpy()
    g300 = ctx.eval_grad(x300, slots)[1].cpu().numpy()
    scale = np.max(np.abs(g300[0]))
    assert scale > 0 and np.all(np.abs(g300 - g1[0]) <= 1e-5 * scale)
    ctx.close()


def test_depth_error_against_the_ray_surface_margin():
    """The worst GPU depth error on hit pixels, binned by the oracle's margin of the winning
    primitive (m; dimensionless, 0 at the silhouette): FP32 conditioning grows like
    delta / sqrt(m) towards the silhouette, and the bar of 1e-3 mm must hold on every robust
    pixel, the grazing ones included (two-hand 640x480 frame, 8 particles)."""
    cfg, model, fr = frame_for(4)
    poses = particles_for(model, fr, 8, seed=13)
    ctx = make_ctx(model, [fr])
    H, W = fr["depth"].shape
    cost, dbg = eval_debug(ctx, poses, 0, W, H)
    ctx.close()
    rendered = oracle_renders(model, [(fr, p) for p in poses])
    edges = [1e-5, 1e-4, 1e-3, 1e-2, 1e-1, 1.0]
    worst = np.zeros(len(edges) - 1)
    count = np.zeros(len(edges) - 1, np.int64)
    for i, (res, cls) in enumerate(rendered):
        rob = cls["robust_hit"] & (dbg["hit"][i] == 1)
        win = res["winner"]
        yy, xx = np.nonzero(rob)
        m = res["prim_margin"][win[yy, xx], yy, xx]
        err = np.abs(dbg["depth"][i][yy, xx].astype(np.float64) - res["depth"][yy, xx])
        for b in range(len(edges) - 1):
            sel = (m >= edges[b]) & (m < edges[b + 1])
            count[b] += sel.sum()
            if sel.any():
                worst[b] = max(worst[b], float(err[sel].max()))
    print("margin bin: pixels, worst depth error (mm)")
    for b in range(len(edges) - 1):
        print(f"  [{edges[b]:.0e}, {edges[b + 1]:.0e}): {count[b]:7d}  {worst[b]:.2e}")
    assert count[:2].sum() > 0 and count[-1] > 1000
    assert np.all(worst <= 1e-3)
