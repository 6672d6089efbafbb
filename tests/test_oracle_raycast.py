"""Pins of the oracle's ray caster against closed forms, a library root finder and
rendering invariances (section III.A depth image; primitive shapes of section II.A)."""
import numpy as np
import pytest

from oracle import fk, raycast
from workload import make_hand_model


def sphere(p, r):
    return {"type": raycast.SPHERE, "p": np.asarray(p, float), "R": np.eye(3),
            "size": np.array([r, 0.0, 0.0])}


def cylinder(p0, axis, r, L):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    # any orthonormal frame with z = axis
    a = np.array([1.0, 0, 0]) if abs(axis[0]) < 0.9 else np.array([0, 1.0, 0])
    x = np.cross(a, axis)
    x /= np.linalg.norm(x)
    y = np.cross(axis, x)
    return {"type": raycast.CYLINDER, "p": np.asarray(p0, float),
            "R": np.stack([x, y, axis], axis=1), "size": np.array([r, L, 0.0])}


def ellipsoid(c, R, semi):
    return {"type": raycast.ELLIPSOID, "p": np.asarray(c, float), "R": np.asarray(R, float),
            "size": np.asarray(semi, float)}


def test_sphere_on_optical_axis():
    W = H = 33
    cam = (100.0, 100.0, 16.0, 16.0)
    res = raycast.render_primitives([sphere((0, 0, 600), 10.0)], W, H, cam, 1500.0)
    assert res["hit"][16, 16]
    assert res["depth"][16, 16] == pytest.approx(590.0, abs=1e-9)


def test_sphere_centre_on_pixel_ray_closed_form():
    rng = np.random.default_rng(0)
    W, H = 40, 30
    cam = (90.0, 90.0, (W - 1) / 2, (H - 1) / 2)
    d = raycast.pixel_directions(W, H, cam)
    for _ in range(20):
        u, v = rng.integers(0, W), rng.integers(0, H)
        s = rng.uniform(400, 900)
        c = s * d[v, u]
        r = rng.uniform(5, 15)
        res = raycast.render_primitives([sphere(c, r)], W, H, cam, 1500.0)
        expect = c[2] * (1.0 - r / np.linalg.norm(c))
        assert res["depth"][v, u] == pytest.approx(expect, abs=1e-9)


def test_sphere_hit_set_matches_cross_product_distance():
    W, H = 48, 40
    cam = (60.0, 60.0, (W - 1) / 2, (H - 1) / 2)
    c, r = np.array([13.0, -7.0, 420.0]), 21.0
    res = raycast.render_primitives([sphere(c, r)], W, H, cam, 1500.0)
    d = raycast.pixel_directions(W, H, cam)
    dh = d / np.linalg.norm(d, axis=-1, keepdims=True)
    rho = np.linalg.norm(np.cross(dh, c), axis=-1)
    assert np.array_equal(res["hit"], rho <= r)
    m = res["prim_margin"][0]
    assert np.allclose(m, 1.0 - rho ** 2 / r ** 2, atol=1e-12)


def test_cylinder_side_on_closed_form():
    W, H = 41, 41
    f = 80.0
    cam = (f, f, 20.0, 20.0)
    Z, r, L = 500.0, 12.0, 60.0
    res = raycast.render_primitives([cylinder((-L / 2, 0, Z), (1, 0, 0), r, L)], W, H, cam,
                                    1500.0)
    for v in range(H):
        b = (v - 20.0) / f
        disc = Z * Z - (1 + b * b) * (Z * Z - r * r)
        for u in range(W):
            a = (u - 20.0) / f
            if disc < 0:
                assert not res["hit"][v, u]
                continue
            t = (Z - np.sqrt(disc)) / (1 + b * b)
            if abs(a * t) < L / 2 - 1e-6:
                assert res["hit"][v, u]
                assert res["depth"][v, u] == pytest.approx(t, abs=1e-9)
                assert res["prim_surface"][0, v, u] == 0


def test_cylinder_end_on_cap_depth():
    W = H = 41
    f = 100.0
    cam = (f, f, 20.0, 20.0)
    Z, r, L = 600.0, 10.0, 40.0
    res = raycast.render_primitives([cylinder((0, 0, Z - L / 2), (0, 0, 1), r, L)], W, H, cam,
                                    1500.0)
    d = raycast.pixel_directions(W, H, cam)
    radial = np.hypot(d[..., 0], d[..., 1]) * (Z - L / 2)
    assert np.array_equal(res["hit"], radial <= r)
    assert np.allclose(res["depth"][res["hit"]], Z - L / 2, atol=1e-9)
    assert np.all(res["prim_surface"][0][res["hit"]] == 1)


def test_ellipsoid_axis_aligned_centre_depth():
    W = H = 33
    cam = (100.0, 100.0, 16.0, 16.0)
    res = raycast.render_primitives([ellipsoid((0, 0, 700), np.eye(3), (20, 11, 7))], W, H, cam,
                                    1500.0)
    assert res["depth"][16, 16] == pytest.approx(693.0, abs=1e-9)


def test_rotated_ellipsoid_against_numpy_roots():
    rng = np.random.default_rng(3)
    W, H = 30, 24
    cam = (120.0, 120.0, (W - 1) / 2, (H - 1) / 2)
    R = fk.rot_axis(np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8]), 0.9)
    c, semi = np.array([5.0, -3.0, 300.0]), np.array([30.0, 12.0, 20.0])
    res = raycast.render_primitives([ellipsoid(c, R, semi)], W, H, cam, 1500.0)
    Q = R @ np.diag(1.0 / semi ** 2) @ R.T
    d = raycast.pixel_directions(W, H, cam)
    n_hit = 0
    for v in range(H):
        for u in range(W):
            dv = d[v, u]
            roots = np.roots([dv @ Q @ dv, -2.0 * dv @ Q @ c, c @ Q @ c - 1.0])
            real = roots[np.abs(roots.imag) < 1e-9].real
            real = real[real > 0]
            if real.size:
                n_hit += 1
                assert res["hit"][v, u]
                assert res["depth"][v, u] == pytest.approx(real.min(), rel=1e-9)
            else:
                assert not res["hit"][v, u]
    assert n_hit > 50


def _hand_pose(z=600.0):
    h = np.zeros(26)
    h[[0, 2, 6, 10, 14, 18]] = [0.3, 0.4, 0.5, 0.2, 0.6, 0.3]
    h[20:26] = [3.0, -40.0, z, 0.2, -0.15, 0.1]
    return h


def test_composition_is_pixelwise_min():
    model = make_hand_model(7)
    W, H = 64, 64
    cam = (144.0, 144.0, 31.5, 31.5)
    h = _hand_pose()
    full = raycast.render(model, h, W, H, cam, 1500.0)
    prims = fk.camera_primitives(model, h)
    zs = np.stack([raycast.render_primitives([p], W, H, cam, 1500.0)["depth"] for p in prims])
    assert np.array_equal(full["depth"], zs.min(axis=0))
    assert full["hit"].sum() > 300


def test_rotation_about_optical_axis_permutes_pixels():
    model = make_hand_model(11)
    W = H = 64
    cam = (144.0, 144.0, 31.5, 31.5)
    h = _hand_pose()
    a = raycast.render(model, h, W, H, cam, 1500.0)
    h2 = h.copy()
    h2[20], h2[21] = -h[21], h[20]
    h2[25] = h[25] + np.pi / 2
    b = raycast.render(model, h2, W, H, cam, 1500.0)
    # (u, v) -> (cx - (v - cy), cy + (u - cx))
    v, u = np.mgrid[0:H, 0:W]
    u2 = (31.5 - (v - 31.5)).astype(int)
    v2 = (31.5 + (u - 31.5)).astype(int)
    assert np.array_equal(b["hit"][v2, u2], a["hit"])
    assert np.allclose(b["depth"][v2, u2], a["depth"], atol=1e-9)


def test_x_mirror_of_scene_mirrors_image():
    model = make_hand_model(5)
    W, H = 50, 44
    cam = (110.0, 110.0, (W - 1) / 2, (H - 1) / 2)
    prims = fk.camera_primitives(model, _hand_pose())
    M = np.diag([-1.0, 1.0, 1.0])
    mir = [dict(p, p=M @ p["p"], R=M @ p["R"]) for p in prims]
    a = raycast.render_primitives(prims, W, H, cam, 1500.0)
    b = raycast.render_primitives(mir, W, H, cam, 1500.0)
    assert np.array_equal(b["hit"], a["hit"][:, ::-1])
    assert np.allclose(b["depth"], a["depth"][:, ::-1], atol=1e-9)


def test_rigid_motion_of_scene_and_camera_is_invisible():
    rng = np.random.default_rng(2)
    model = make_hand_model(9)
    W, H = 48, 48
    cam = (108.0, 108.0, 23.5, 23.5)
    prims = fk.camera_primitives(model, _hand_pose())
    a = raycast.render_primitives(prims, W, H, cam, 1500.0)
    for _ in range(3):
        axis = rng.normal(size=3)
        Rt = fk.rot_axis(axis / np.linalg.norm(axis), rng.uniform(0, 2 * np.pi))
        tt = rng.normal(size=3) * 200
        moved = [dict(p, p=Rt @ p["p"] + tt, R=Rt @ p["R"]) for p in prims]
        b = raycast.render_primitives(moved, W, H, cam, 1500.0, cam_pose=(Rt, tt))
        assert np.array_equal(a["hit"], b["hit"])
        assert np.allclose(a["depth"], b["depth"], atol=1e-8)


def test_background_plane_hides_far_primitives_and_zero_plane():
    W = H = 21
    cam = (50.0, 50.0, 10.0, 10.0)
    far = raycast.render_primitives([sphere((0, 0, 2000), 50.0)], W, H, cam, 1500.0)
    assert not far["hit"].any() and np.all(far["depth"] == 1500.0)
    nob = raycast.render_primitives([sphere((0, 0, 2000), 50.0)], W, H, cam, 0.0)
    assert nob["hit"][10, 10] and nob["depth"][10, 10] == pytest.approx(1950.0)
    assert nob["depth"][0, 0] == 0.0
