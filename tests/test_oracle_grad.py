"""Pins of the oracle's analytic gradient: central finite differences on smooth pixels,
a closed-form sphere derivative, and exact zeros for an unseen finger."""
import numpy as np
import pytest

from oracle import cost, grad, raycast, synth
from workload import make_hand_model, finger_dof


@pytest.fixture(scope="module")
def model():
    return make_hand_model(21)


def _pose(model, seed):
    """A fairly open hand near 500 mm, so that many pixels are away from edges."""
    rng = np.random.default_rng(seed)
    h = rng.uniform(model["bounds_lo"], model["bounds_hi"])
    flex = [4 * f + j for f in range(5) for j in (0, 2, 3)]
    h[flex] = rng.uniform(0.0, 0.6, len(flex))
    for a, b in model["kc_pairs"]:
        h[b] = min(h[b], h[a] - 0.02)
    h[20:23] = [rng.uniform(-10, 10), rng.uniform(-50, -30), rng.uniform(480, 520)]
    h[23:26] = rng.uniform(-0.3, 0.3, 3)
    return h


@pytest.fixture(scope="module")
def paper_model():
    return make_hand_model(22, 1, "paper")


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_analytic_matches_central_fd_on_smooth_pixels(model, seed):
    _fd_check(model, seed)


@pytest.mark.parametrize("seed", [0, 1])
def test_analytic_matches_central_fd_paper_primitives(paper_model, seed):
    """The same with truncated-cone phalanges and the elliptic-cylinder palm."""
    # grazing views of the tapered phalanges give depth derivatives of ~200 mm/rad with a
    # large third derivative: a smaller step keeps the central-difference truncation small
    _fd_check(paper_model, 10 + seed, step_rad=2e-4, step_mm=2e-3)


def _fd_check(model, seed, step_rad=1e-3, step_mm=1e-2):
    W = H = 160
    cam = (360.0, 360.0, 79.5, 79.5)
    h_true = _pose(model, 100 + seed)
    obs = synth.clean_observation(model, h_true, W, H, cam)
    rng = np.random.default_rng(seed)
    obs["depth"] = obs["depth"] + rng.normal(0, 2.0, obs["depth"].shape)
    h = h_true + rng.uniform(-1, 1, 26) * np.r_[np.full(20, 0.05), [4, 4, 4], np.full(3, 0.03)]
    E, parts = cost.objective(model, h, obs, return_parts=True)
    mask = grad.fd_mask(parts["render"], obs["depth"])
    assert (mask & parts["render"]["hit"]).sum() > 200
    _, g = grad.analytic_gradient(model, h, obs, pixel_mask=mask)
    g_fd = grad.fd_gradient(model, h, obs, mask, parts["S_or"], step_rad=step_rad,
                            step_mm=step_mm)
    scale = np.max(np.abs(g_fd))
    assert scale > 0
    # central differences with 1e-3 rad / 1e-2 mm steps: truncation error well below 5e-5
    assert np.max(np.abs(g - g_fd)) <= 5e-5 * scale, (g, g_fd)


def test_sphere_translation_derivative_closed_form():
    """One-sphere 'hand': d r_d / d x_wrist from the quadratic root vs the oracle."""
    m = make_hand_model(1)
    one = dict(m)
    one["n_prim"] = 1
    one["prim_type"] = np.array([raycast.SPHERE], np.int32)
    one["prim_seg"] = np.array([0], np.int32)
    one["prim_frame"] = np.zeros((1, 3, 4))
    one["prim_frame"][0, :, :3] = np.eye(3)
    one["prim_size"] = np.array([[15.0, 0, 0]])
    W = H = 40
    cam = (400.0, 400.0, 19.5, 19.5)
    h = np.zeros(26)
    h[20:23] = [3.0, -2.0, 500.0]
    res = raycast.render(one, h, W, H, cam, 1500.0)
    dz = grad.depth_gradient(one, h, res, W, H, cam)
    d = raycast.pixel_directions(W, H, cam)
    c = h[20:23]
    a = np.einsum("hwi,hwi->hw", d, d)
    b = d @ c
    disc = b * b - a * (c @ c - 15.0 ** 2)
    hit = res["hit"]
    expect = (d[..., 0] - (b * d[..., 0] - a * c[0]) / np.sqrt(np.where(hit, disc, 1.0))) / a
    assert hit.sum() > 100
    assert np.allclose(dz[20][hit], expect[hit], rtol=1e-9, atol=1e-9)
    assert np.all(dz[:, ~hit] == 0.0)


def test_unseen_finger_has_exactly_zero_gradient(model):
    W = H = 64
    h = np.zeros(26)
    h[finger_dof(4, 0)] = 0.3
    h[20:26] = [0.0, -45.0, 600.0, 0.0, 0.0, 0.0]
    # shift the principal point so that the little-finger side leaves the image
    cam_cut = (144.0, 144.0, -1.5, 31.5)
    obs = synth.clean_observation(model, h, W, H, cam_cut)
    rng = np.random.default_rng(0)
    obs["depth"] = obs["depth"] + rng.normal(0, 2.0, obs["depth"].shape)
    hp = h.copy()
    hp[20] += 3.0
    _, parts = cost.objective(model, hp, obs, return_parts=True)
    little = [5 + 7 * 4 + j for j in range(7)]
    assert not parts["render"]["prim_hit"][little].any()
    assert parts["render"]["hit"].sum() > 200
    _, g = grad.analytic_gradient(model, hp, obs)
    assert np.all(g[[finger_dof(4, j) for j in range(4)]] == 0.0)
    assert np.any(g[[finger_dof(1, j) for j in range(4)]] != 0.0)
