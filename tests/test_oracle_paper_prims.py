"""Pins of the oracle's truncated cone and elliptic cylinder (the phalanx and palm primitives of
section II.A) against the circular-cylinder routine they reduce to, closed forms and brute
force along each ray."""
import numpy as np
import pytest

from oracle import raycast


def frame(axis, rng=None):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    a = np.array([1.0, 0, 0]) if abs(axis[0]) < 0.9 else np.array([0, 1.0, 0])
    x = np.cross(a, axis)
    x /= np.linalg.norm(x)
    y = np.cross(axis, x)
    if rng is not None:                     # random rotation about the axis
        g = rng.uniform(0, 2 * np.pi)
        x, y = np.cos(g) * x + np.sin(g) * y, -np.sin(g) * x + np.cos(g) * y
    return np.stack([x, y, axis], axis=1)


def random_rays(rng, n, target, spread):
    """Rays from the camera origin towards points scattered around ``target``."""
    pts = target[None, :] + rng.normal(size=(n, 3)) * spread
    return pts / pts[:, 2:3]


def inside_cone(x, p0, R, r0, L, r1):
    y = (x - p0) @ R
    k = (r1 - r0) / L
    return (y[..., 0] ** 2 + y[..., 1] ** 2 <= (r0 + k * y[..., 2]) ** 2) & \
        (y[..., 2] >= 0) & (y[..., 2] <= L)


def inside_ecyl(x, p0, R, a, L, b):
    y = (x - p0) @ R
    return ((y[..., 0] / a) ** 2 + (y[..., 1] / b) ** 2 <= 1.0) & (y[..., 2] >= 0) & \
        (y[..., 2] <= L)


def brute_entry(inside, d, t_lo, t_hi, step):
    """First sampled ray parameter inside the solid (inf if none)."""
    ts = np.arange(t_lo, t_hi, step)
    out = np.full(d.shape[0], np.inf)
    for i in range(d.shape[0]):
        ins = inside(ts[:, None] * d[i][None, :])
        j = np.argmax(ins)
        if ins[j]:
            out[i] = ts[j]
    return out


def test_cone_with_equal_radii_is_the_cylinder():
    rng = np.random.default_rng(3)
    for _ in range(5):
        ax = rng.normal(size=3)
        R = frame(ax, rng)
        p0 = np.array([rng.uniform(-30, 30), rng.uniform(-30, 30), rng.uniform(450, 700)])
        r, L = rng.uniform(6, 14), rng.uniform(20, 50)
        d = random_rays(rng, 3000, p0 + R[:, 2] * L / 2, 25.0)
        tc, hc, mc, sc = raycast.intersect_cone(np.zeros(3), d, p0, R, r, L, r)
        ty, hy, my, sy = raycast.intersect_cylinder(np.zeros(3), d, p0, R[:, 2], r, L)
        assert np.array_equal(hc, hy)
        assert hc.any() and (~hc).any()
        assert np.allclose(tc[hc], ty[hc], rtol=0, atol=1e-8)
        assert np.array_equal(sc[hc], sy[hc])
        assert np.allclose(mc, my, atol=1e-9)


def test_cone_closed_forms():
    # axis along +z away from the camera: the ray along the axis enters the near cap
    p0 = np.array([0.0, 0.0, 500.0])
    R = np.eye(3)
    r0, L, r1 = 10.0, 40.0, 6.0
    t, h, m, s = raycast.intersect_cone(np.zeros(3), np.array([[0.0, 0.0, 1.0]]), p0, R, r0, L,
                                        r1)
    assert h[0] and t[0] == pytest.approx(500.0, abs=1e-12) and s[0] == 1
    # axis along x at depth Z: the ray through the axis point at s enters the side at
    # distance R(s) = r0 + k s in front of the axis (the ray is perpendicular to the axis)
    Z = 600.0
    Rx = frame((1.0, 0.0, 0.0))
    p0 = np.array([-20.0, 0.0, Z])
    for s_ax in (2.0, 15.0, 33.0):
        x = -20.0 + s_ax
        d = np.array([[x / Z, 0.0, 1.0]])
        t, h, _, surf = raycast.intersect_cone(np.zeros(3), d, p0, Rx, r0, L, r1)
        # the point at t lies on the cone side and on the ray; its distance from the axis
        # equals the radius at its own axial position
        pt = t[0] * d[0]
        y = (pt - p0) @ Rx
        k = (r1 - r0) / L
        assert h[0] and surf[0] == 0
        assert np.hypot(y[0], y[1]) == pytest.approx(r0 + k * y[2], abs=1e-9)
        # and it is the nearest such point: for a ray perpendicular to the axis the entry
        # lies between the tangent-free bounds Z - max(r0, r1) and Z - min(r0, r1)
        assert Z - max(r0, r1) - 1e-9 <= pt[2] <= Z - min(r0, r1) + 1e-9


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cone_entry_against_brute_force(seed):
    rng = np.random.default_rng(10 + seed)
    R = frame(rng.normal(size=3), rng)
    p0 = np.array([rng.uniform(-20, 20), rng.uniform(-20, 20), rng.uniform(500, 650)])
    r0, L, r1 = rng.uniform(6, 12), rng.uniform(20, 45), rng.uniform(4, 12)
    d = random_rays(rng, 120, p0 + R[:, 2] * L / 2, 18.0)
    t, h, m, _ = raycast.intersect_cone(np.zeros(3), d, p0, R, r0, L, r1)
    step = 2e-3
    tb = brute_entry(lambda x: inside_cone(x, p0, R, r0, L, r1), d, p0[2] - 80, p0[2] + 80,
                     step)
    robust = np.abs(m) > 1e-3
    assert np.array_equal(h[robust], np.isfinite(tb)[robust])
    both = h & np.isfinite(tb)
    # the sampled entry is the first sample at or after the exact entry
    assert np.all(tb[both] - t[both] >= -1e-9)
    assert np.all(tb[both] - t[both] < step * 1.0001)
    assert h.sum() > 20


def test_ecylinder_with_equal_axes_is_the_cylinder():
    rng = np.random.default_rng(5)
    R = frame(rng.normal(size=3), rng)
    p0 = np.array([4.0, -9.0, 580.0])
    r, L = 11.0, 38.0
    d = random_rays(rng, 3000, p0 + R[:, 2] * L / 2, 25.0)
    te, he, me, se = raycast.intersect_ecylinder(np.zeros(3), d, p0, R, r, L, r)
    ty, hy, my, sy = raycast.intersect_cylinder(np.zeros(3), d, p0, R[:, 2], r, L)
    assert np.array_equal(he, hy) and he.any()
    assert np.allclose(te[he], ty[he], rtol=0, atol=1e-8)
    assert np.array_equal(se[he], sy[he])
    assert np.allclose(me, my, atol=1e-9)


def test_ecylinder_semi_axes_closed_form():
    # axis along y (in the image plane), semi-axis a along x, b along z (towards the camera)
    a, b, L, Z = 20.0, 8.0, 30.0, 700.0
    R = np.stack([np.array([1.0, 0, 0]), np.array([0, 0, -1.0]), np.array([0, 1.0, 0])],
                 axis=1)
    p0 = np.array([0.0, -L / 2, Z])
    t, h, _, s = raycast.intersect_ecylinder(np.zeros(3), np.array([[0.0, 0.0, 1.0]]), p0, R,
                                             a, L, b)
    assert h[0] and s[0] == 0 and t[0] == pytest.approx(Z - b, abs=1e-9)
    # swap the roles: now a faces the camera
    R2 = np.stack([np.array([0, 0, -1.0]), np.array([1.0, 0, 0]), np.array([0, 1.0, 0])],
                  axis=1)
    t, h, _, _ = raycast.intersect_ecylinder(np.zeros(3), np.array([[0.0, 0.0, 1.0]]), p0, R2,
                                             a, L, b)
    assert h[0] and t[0] == pytest.approx(Z - a, abs=1e-9)
    # a ray parallel to the optical axis at x just beyond / within the ellipse's x extremity
    # misses / hits, with a margin near zero
    for x, expect in ((a * (1 + 1e-6), False), (a * (1 - 1e-6), True)):
        _, h, m, _ = raycast.intersect_ecylinder(np.array([x, 0.0, 0.0]),
                                                 np.array([[0.0, 0.0, 1.0]]), p0, R, a, L, b)
        assert h[0] == expect and abs(m[0]) < 1e-4


@pytest.mark.parametrize("seed", [0, 1])
def test_ecylinder_entry_against_brute_force(seed):
    rng = np.random.default_rng(20 + seed)
    R = frame(rng.normal(size=3), rng)
    p0 = np.array([rng.uniform(-20, 20), rng.uniform(-20, 20), rng.uniform(500, 650)])
    a, L, b = rng.uniform(15, 30), rng.uniform(20, 45), rng.uniform(6, 12)
    d = random_rays(rng, 120, p0 + R[:, 2] * L / 2, 20.0)
    t, h, m, _ = raycast.intersect_ecylinder(np.zeros(3), d, p0, R, a, L, b)
    step = 2e-3
    tb = brute_entry(lambda x: inside_ecyl(x, p0, R, a, L, b), d, p0[2] - 80, p0[2] + 80, step)
    robust = np.abs(m) > 1e-3
    assert np.array_equal(h[robust], np.isfinite(tb)[robust])
    both = h & np.isfinite(tb)
    assert np.all(tb[both] - t[both] >= -1e-9)
    assert np.all(tb[both] - t[both] < step * 1.0001)
    assert h.sum() > 20
