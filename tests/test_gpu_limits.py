"""GPU parity at the library's size limits (HT_MAX_PRIM primitives, HT_MAX_SEG segments,
HT_MAX_KC collision pairs, HT_MAX_ROI pixels per side), against the FP64 oracle."""
import os

import numpy as np
import pytest

from gpu_util import check_particle, eval_debug, make_ctx, particles_for, torch_cuda
from oracle import synth
from workload import WORKLOADS, make_hand_model, seed_sequence

pytestmark = pytest.mark.gpu

MAX_PRIM, MAX_SEG, MAX_KC, MAX_ROI = 128, 32, 16, 4096
DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "workload",
                    "data")


def _observation(model, h, W, H, cam):
    """The clean render of pose h as the boundary takes it (uint16 mm, 0/1 skin)."""
    ob = synth.clean_observation(model, h, W, H, cam)
    depth = np.clip(np.round(ob["depth"]), 0, 65535).astype(np.uint16)
    return {"depth": depth, "skin": ob["skin"].astype(np.uint8), "cam": cam, "bg": ob["bg"],
            "h_true": ob["h_true"]}


def _padded_two_hand_model():
    """The two-hand model (32 segments, 80 primitives) padded with small spheres on seeded
    segments to 128 primitives, and with collision pairs up to 16."""
    model = make_hand_model(seed_sequence(4, 10_000), 2, "cylinders")
    assert model["n_seg"] == MAX_SEG
    rng = np.random.default_rng(seed_sequence(4, 77))
    extra = MAX_PRIM - model["n_prim"]
    frames = np.zeros((extra, 3, 4))
    frames[:, :, :3] = np.eye(3)
    frames[:, :, 3] = rng.uniform(-12.0, 12.0, (extra, 3))
    sizes = np.zeros((extra, 3))
    sizes[:, 0] = rng.uniform(4.0, 8.0, extra)
    m = dict(model)
    m["prim_type"] = np.concatenate([model["prim_type"], np.zeros(extra, model["prim_type"].dtype)])
    m["prim_seg"] = np.concatenate([model["prim_seg"],
                                    rng.integers(0, MAX_SEG, extra).astype(model["prim_seg"].dtype)])
    m["prim_frame"] = np.concatenate([model["prim_frame"], frames])
    m["prim_size"] = np.concatenate([model["prim_size"], sizes])
    m["n_prim"] = MAX_PRIM
    # further pairs of finger flexion angles (thumb vs index, ...), both hands
    more = [(1 + 26 * k + 4 * a, 1 + 26 * k + 4 * b) for k in range(2)
            for a, b in ((0, 1), (0, 2), (1, 3), (2, 4), (0, 4))]
    m["kc_pairs"] = np.concatenate([model["kc_pairs"],
                                    np.array(more, model["kc_pairs"].dtype)])[:MAX_KC]
    assert len(m["kc_pairs"]) == MAX_KC
    return m


def test_model_at_the_primitive_segment_and_pair_limits():
    """128 primitives (both culling halves full), 32 segments, 16 collision pairs: the
    full-frame two-hand pose at 160x120 (the 640x480 field of view), particles around it."""
    torch_cuda()
    model = _padded_two_hand_model()
    h = np.load(os.path.join(DATA, "config4.npz"))["h_true"][0]
    cam = (575.0 / 4, 575.0 / 4, 79.5, 59.5)
    fr = _observation(model, h, 160, 120, cam)
    poses = particles_for(model, fr, 8, seed=5)
    poses[0] = h.astype(np.float32)
    ctx = make_ctx(model, [fr])
    cost, dbg = eval_debug(ctx, poses, 0, 160, 120)
    ctx.close()
    hits = 0
    for i in range(len(poses)):
        hits += check_particle(model, fr, poses[i], cost[i], dbg, i)["hits"]
    assert hits > 0


@pytest.mark.parametrize("W,H", [(MAX_ROI, 8), (8, MAX_ROI), (MAX_ROI, 13)])
def test_roi_at_the_side_limit(W, H):
    """Observation strips 4096 pixels long (a ragged 13-pixel height too), one hand across
    them."""
    torch_cuda()
    cfg = WORKLOADS[1]
    model = make_hand_model(seed_sequence(1, 10_000), cfg.n_hands, cfg.primitive_set)
    h = np.load(os.path.join(DATA, "config1.npz"))["h_true"][0]
    cam = (600.0, 600.0, (W - 1) / 2.0, (H - 1) / 2.0)
    fr = _observation(model, h, W, H, cam)
    assert fr["skin"].any()
    poses = particles_for(model, fr, 4, seed=6)
    ctx = make_ctx(model, [fr])
    cost, dbg = eval_debug(ctx, poses, 0, W, H)
    ctx.close()
    for i in range(len(poses)):
        check_particle(model, fr, poses[i], cost[i], dbg, i)


def test_roi_beyond_the_side_limit_is_rejected():
    import paper_2005_07068_amd as ht
    torch_cuda()
    cfg = WORKLOADS[0]
    model = make_hand_model(seed_sequence(0, 10_000), cfg.n_hands, cfg.primitive_set)
    ctx = ht.Context(0)
    ctx.set_model(model)
    depth = np.zeros((2, MAX_ROI + 1), np.uint16)
    with pytest.raises(Exception):
        ctx.set_observation(0, depth, np.zeros_like(depth, np.uint8), (600.0, 600.0, 0.0, 0.0),
                            1500.0)
    ctx.close()
