"""Pins of the oracle's kinematics (Eq. 1-3), discrepancy (Eq. 4) and objective (Eq. 5)."""
import numpy as np
import pytest

from oracle import cost, fk, raycast, synth
from workload import make_hand_model, finger_dof
from workload.handmodel import joint_bounds_one_hand


@pytest.fixture(scope="module")
def model():
    return make_hand_model(3)


def tip_centre(model, h, finger):
    """Centre of the fingertip sphere (last primitive of the finger's block)."""
    prims = fk.camera_primitives(model, h)
    return prims[5 + 7 * finger + 6]["p"]


def finger_lengths(model, finger):
    s1 = 1 + 3 * finger
    return (model["seg_offset"][s1 + 1][1, 3], model["seg_offset"][s1 + 2][1, 3],
            model["prim_frame"][5 + 7 * finger + 6][1, 3])


def test_zero_pose_fingertip_is_straight(model):
    h = np.zeros(26)
    h[22] = 600.0
    for f in (1, 2, 3, 4):
        base = model["seg_offset"][1 + 3 * f][:, 3]
        L1, L2, L3 = finger_lengths(model, f)
        expect = base + np.array([0.0, L1 + L2 + L3, 600.0])
        assert np.allclose(tip_centre(model, h, f), expect, atol=1e-9)


def test_flexion_bends_towards_palmar_z(model):
    f = 2
    base = model["seg_offset"][1 + 3 * f][:, 3]
    L1, L2, L3 = finger_lengths(model, f)
    h = np.zeros(26)
    h[22] = 600.0
    h[finger_dof(f, 0)] = np.pi / 2          # MP flexion 90 deg: whole finger along +z
    assert np.allclose(tip_centre(model, h, f), base + [0, 0, 600 + L1 + L2 + L3], atol=1e-9)
    h[finger_dof(f, 0)] = 0.0
    h[finger_dof(f, 2)] = np.pi / 2          # PIP 90 deg: middle + distal along +z
    assert np.allclose(tip_centre(model, h, f), base + [0, L1, 600 + L2 + L3], atol=1e-9)


def test_abduction_turns_towards_thumb(model):
    h = np.zeros(26)
    h[22] = 600.0
    x0 = tip_centre(model, h, 1)[0]
    h[finger_dof(1, 1)] = 0.2
    assert tip_centre(model, h, 1)[0] > x0 + 1.0


def test_wrist_rotation_order_z_y_x(model):
    h = np.zeros(26)
    h[20:23] = [10.0, -20.0, 700.0]
    h[23] = np.pi / 2      # theta_x
    h[25] = np.pi / 2      # theta_z
    T = fk.segment_transforms(model, h)[0]
    # Rz(90) Ry(0) Rx(90) maps hand +y to camera +z (Rx Rz would give -x)
    assert np.allclose(T[:3, :3] @ [0, 1, 0], [0, 0, 1], atol=1e-12)
    assert np.allclose(T[:3, 3], [10, -20, 700])
    R_expected = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]], float)
    assert np.allclose(T[:3, :3], R_expected, atol=1e-12)


def test_bounds_are_tables_1_and_2_in_radians_and_mm():
    lo, hi = joint_bounds_one_hand()
    assert np.rad2deg(hi[finger_dof(0, 1)]) == pytest.approx(60.0)
    assert np.rad2deg(lo[finger_dof(4, 1)]) == pytest.approx(-45.0)
    assert np.rad2deg(hi[finger_dof(1, 2)]) == pytest.approx(100.0)
    assert (lo[20], hi[20], lo[22], hi[22]) == (-900, 900, 500, 1500)
    assert np.rad2deg(lo[23]) == pytest.approx(-30) and np.rad2deg(hi[24]) == pytest.approx(75)


def _pose(model, rng):
    lo, hi = model["bounds_lo"], model["bounds_hi"]
    h = rng.uniform(lo, hi)
    for a, b in model["kc_pairs"]:
        h[b] = min(h[b], h[a])
    h[20:23] = [rng.uniform(-10, 10), rng.uniform(-60, -20), rng.uniform(570, 630)]
    h[23:26] = rng.uniform(-0.3, 0.3, 3)
    return h


def test_clean_float_observation_scores_zero(model):
    rng = np.random.default_rng(1)
    W = H = 64
    cam = (144.0, 144.0, 31.5, 31.5)
    for _ in range(3):
        h = _pose(model, rng)
        assert cost.kc(model, h) == 0.0
        obs = synth.clean_observation(model, h, W, H, cam)
        E, parts = cost.objective(model, h, obs, return_parts=True)
        assert parts["S_d"] == pytest.approx(0.0, abs=1e-9)
        assert parts["S_and"] == parts["S_or"] == int(obs["skin"].sum()) > 0
        assert E == pytest.approx(0.0, abs=1e-12)


def test_uint16_rounding_residual_is_exact(model):
    rng = np.random.default_rng(2)
    W = H = 48
    cam = (108.0, 108.0, 23.5, 23.5)
    h = _pose(model, rng)
    res = raycast.render(model, h, W, H, cam, 1500.0)
    obs = {"depth": np.round(res["depth"]).astype(np.uint16), "skin": res["hit"].astype(np.uint8),
           "cam": cam, "bg": 1500.0}
    E, parts = cost.objective(model, h, obs, return_parts=True)
    resid = np.abs(np.round(res["depth"]) - res["depth"])[res["hit"]]
    assert np.all(resid <= 0.5)
    assert parts["S_d"] == pytest.approx(resid.sum(), rel=1e-12)
    assert parts["D"] == pytest.approx(resid.sum() / parts["S_or"], rel=1e-12)


def test_all_miss_hypothesis_and_dice_identity(model):
    rng = np.random.default_rng(3)
    W = H = 48
    cam = (108.0, 108.0, 23.5, 23.5)
    h = _pose(model, rng)
    obs = synth.clean_observation(model, h, W, H, cam)
    far = h.copy()
    far[20] += 5000.0                       # entirely out of view
    E, parts = cost.objective(model, far, obs, return_parts=True)
    assert parts["S_and"] == 0
    assert parts["D"] == pytest.approx(parts["S_d"] / parts["S_or"] + cost.LAMBDA)
    # Dice identity: sum(a and b) + sum(a or b) == sum(a) + sum(b)
    h2 = h.copy()
    h2[20] += 6.0
    E2, p2 = cost.objective(model, h2, obs, return_parts=True)
    _, r_m, _, _ = cost.pixel_terms(obs["depth"], obs["skin"], p2["render"]["depth"],
                                    p2["render"]["hit"])
    assert p2["S_and"] + p2["S_or"] == int(obs["skin"].sum()) + int(r_m.sum())


def test_dropout_pixels_contribute_constant_d_M(model):
    rng = np.random.default_rng(4)
    W = H = 40
    cam = (90.0, 90.0, 19.5, 19.5)
    h = _pose(model, rng)
    obs = synth.clean_observation(model, h, W, H, cam)
    drop = rng.uniform(size=(H, W)) < 0.1
    obs2 = dict(obs, depth=np.where(drop, 0.0, obs["depth"]))
    for hh in (h, _pose(model, rng)):
        r = raycast.render(model, hh, W, H, cam, 1500.0)
        t_d, r_m, _, _ = cost.pixel_terms(obs2["depth"], obs2["skin"], r["depth"], r["hit"])
        assert np.all(t_d[drop] == cost.D_CLAMP_MM)
        # undefined depth counts as matched wherever the model is hit
        assert np.array_equal(r_m[drop], r["hit"][drop])


def test_objective_nonnegative_and_degenerate_cases(model):
    rng = np.random.default_rng(5)
    W = H = 32
    cam = (72.0, 72.0, 15.5, 15.5)
    obs = synth.clean_observation(model, _pose(model, rng), W, H, cam)
    for _ in range(5):
        assert cost.objective(model, rng.uniform(model["bounds_lo"], model["bounds_hi"]), obs) >= 0
    empty = dict(obs, skin=np.zeros_like(obs["skin"]))
    far = _pose(model, rng)
    far[20] += 5000.0
    assert cost.objective(model, far, empty) == cost.LAMBDA      # S_or == 0 reading
    bad = _pose(model, rng)
    bad[3] = np.nan
    assert cost.objective(model, bad, obs) == np.inf


def test_kc_closed_form_and_gradient(model):
    h = np.zeros(26)
    h[finger_dof(1, 1)], h[finger_dof(2, 1)] = -0.1, 0.05    # index crosses middle by 0.15
    h[finger_dof(3, 1)], h[finger_dof(4, 1)] = -0.2, -0.1    # ring crosses little by 0.1
    assert cost.kc(model, h) == pytest.approx(0.25)
    g = cost.kc_grad(model, h)
    assert g[finger_dof(1, 1)] == -1 and g[finger_dof(2, 1)] == 1
    assert g[finger_dof(3, 1)] == -1 and g[finger_dof(4, 1)] == 1
    assert np.count_nonzero(g) == 4


def test_brute_force_search_recovers_planted_pose(model):
    """A noise-free observation on a 24x24 image; a grid over (x, y, index PIP) with the
    planted values on the grid has its unique E = 0 minimiser at the planted pose."""
    W = H = 24
    cam = (54.0, 54.0, 11.5, 11.5)
    h0 = np.zeros(26)
    h0[20:23] = [4.0, -45.0, 600.0]
    h0[finger_dof(1, 2)] = 0.6
    obs = synth.clean_observation(model, h0, W, H, cam)
    best, arg = np.inf, None
    values = []
    for x in (-8.0, -2.0, 4.0, 10.0):
        for y in (-57.0, -51.0, -45.0, -39.0):
            for pip in (0.0, 0.6, 1.2):
                h = h0.copy()
                h[20], h[21], h[finger_dof(1, 2)] = x, y, pip
                E = cost.objective(model, h, obs)
                values.append(E)
                if E < best:
                    best, arg = E, (x, y, pip)
    assert arg == (4.0, -45.0, 0.6)
    assert best == pytest.approx(0.0, abs=1e-12)
    assert sorted(values)[1] > 0.1
