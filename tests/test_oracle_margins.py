"""Pins of the ray-surface margins that decide which pixels the GPU parity tests treat as
ambiguous, and of the pixel classification built on them.

Each margin is checked against a closed form derived by hand for a special geometry: the
radial slack (r^2 - rho^2)/r^2 of a cylinder seen side-on, its axial slacks s/L and (L-s)/L
and cap slacks along the centre row, 1 - rho'^2 of an axis-aligned ellipsoid, the radial
slack of a truncated cone and of an elliptic cylinder seen side-on.  The margin must also
vanish on the exact hit boundary, found by bisection on the hit flag alone.  Closed forms
agree to 1e-9: the rounding of the discriminant's cancellation, four orders below the 1e-5
threshold of the classification."""
import numpy as np
import pytest

from oracle import raycast

TAU = 1e-5


def _frame(axis):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    a = np.array([1.0, 0, 0]) if abs(axis[0]) < 0.9 else np.array([0, 1.0, 0])
    x = np.cross(a, axis)
    x /= np.linalg.norm(x)
    return np.stack([x, np.cross(axis, x), axis], axis=1)


def _rays(a, b):
    a, b = np.broadcast_arrays(np.asarray(a, float), np.asarray(b, float))
    return np.stack([a, b, np.ones_like(a)], axis=-1).reshape(-1, 3)


def test_cylinder_side_on_radial_slack_closed_form():
    """Axis along x through (0, 0, Z), the middle of its length on the optical axis.  The
    rays of the centre column (slope a = 0, row slope b) cross the axis at s = L/2, so both
    axial slacks are 1/2, and they are parallel to the cap planes (no cap crossing): the
    margin is min(1 - Z^2 b^2 / ((1 + b^2) r^2), 1/2)."""
    Z, r, L = 500.0, 12.0, 60.0
    b = np.linspace(-0.04, 0.04, 801)
    t, hit, m, _ = raycast.intersect_cylinder(np.zeros(3), _rays(0.0, b),
                                              np.array([-L / 2, 0.0, Z]),
                                              np.array([1.0, 0, 0]), r, L)
    expect = np.minimum(1.0 - Z * Z * b * b / ((1.0 + b * b) * r * r), 0.5)
    assert np.allclose(m, expect, rtol=0, atol=1e-9)
    assert np.array_equal(hit, expect >= 0.0)
    assert hit.any() and (~hit).any()


def test_cylinder_axial_and_cap_slacks_closed_form():
    """Same cylinder, rays of the centre row (b = 0, column slope a): the side is crossed at
    t = Z -/+ r (the ray passes through the axis), at axial positions s = a t + L/2 with
    slacks min(1, s/L, 1 - s/L); the cap planes s = 0 and s = L are crossed at
    t = -/+ L / (2a) with radial slack 1 - (t - Z)^2 / r^2.  The margin is the largest of the
    four, and the hit decision is its sign."""
    Z, r, L = 500.0, 12.0, 60.0
    a = np.linspace(-0.09, 0.09, 1201)
    a = a[np.abs(a) > 1e-9]
    t, hit, m, _ = raycast.intersect_cylinder(np.zeros(3), _rays(a, 0.0),
                                              np.array([-L / 2, 0.0, Z]),
                                              np.array([1.0, 0, 0]), r, L)
    slacks = []
    for ts in (Z - r, Z + r):
        s = a * ts + L / 2
        slacks.append(np.minimum(1.0, np.minimum(s / L, 1.0 - s / L)))
    for s_cap in (0.0, L):
        tc = (s_cap - L / 2) / a
        slacks.append(1.0 - (tc - Z) ** 2 / (r * r))
    expect = np.max(slacks, axis=0)
    assert np.allclose(m, expect, rtol=0, atol=1e-9)
    assert np.array_equal(hit, expect >= 0.0)
    assert hit.any() and (~hit).any()


def test_ellipsoid_axis_aligned_closed_form():
    """Semi-axes (A, B, C) along the camera axes, centre (0, 0, Z).  With q = a^2/A^2 +
    b^2/B^2 for the ray (a, b, 1), the squared distance of the ray from the centre in the
    unit-sphere frame is Z^2 q / (1 + C^2 q), so m = 1 - Z^2 q / (1 + C^2 q)."""
    A, B, C, Z = 20.0, 11.0, 7.0, 700.0
    g = np.linspace(-0.04, 0.04, 161)
    aa, bb = np.meshgrid(g, g)
    _, hit, m = raycast.intersect_ellipsoid(np.zeros(3), _rays(aa, bb), np.array([0, 0, Z]),
                                            np.eye(3), np.array([A, B, C]))
    q = (aa / A) ** 2 + (bb / B) ** 2
    expect = (1.0 - Z * Z * q / (1.0 + C * C * q)).reshape(-1)
    assert np.allclose(m, expect, rtol=0, atol=1e-9)
    assert np.array_equal(hit, expect >= 0.0)
    assert hit.any() and (~hit).any()


def test_truncated_cone_side_on_closed_form():
    """Cone with its axis along x, first cap at x = -20 (radius r0), length L, second radius
    r1, axis at depth Z.  The centre column (a = 0) is perpendicular to the axis and crosses
    it at s = 20, where the radius is R = r0 + (r1 - r0) 20 / L; in that cross-section the
    side quadratic's discriminant over |A| is R^2 - rho^2 with rho^2 = Z^2 b^2 / (1 + b^2),
    normalised by the larger radius squared; the axial slacks are 20/L and 1 - 20/L."""
    Z, r0, L, r1 = 600.0, 10.0, 40.0, 6.0
    b = np.linspace(-0.03, 0.03, 601)
    R = _frame((1.0, 0.0, 0.0))
    t, hit, m, _ = raycast.intersect_cone(np.zeros(3), _rays(0.0, b),
                                          np.array([-20.0, 0.0, Z]), R, r0, L, r1)
    Rs = r0 + (r1 - r0) * 20.0 / L
    rho2 = Z * Z * b * b / (1.0 + b * b)
    expect = np.minimum((Rs * Rs - rho2) / max(r0, r1) ** 2, min(20.0 / L, 1.0 - 20.0 / L))
    assert np.allclose(m, expect, rtol=0, atol=1e-9)
    assert np.array_equal(hit, expect >= 0.0)
    assert hit.any() and (~hit).any()


def test_elliptic_cylinder_side_on_closed_form():
    """Elliptic cylinder with its axis along x (s = L/2 on the optical axis), semi-axis a_y
    along the camera y and b_z along z, at depth Z.  In the frame that makes it the unit
    cylinder the centre-column ray (0, b, 1) lies at squared distance
    Z^2 b^2 / (a_y^2 + b^2 b_z^2) from the axis, so m = min(1 - that, 1/2)."""
    ay, bz, L, Z = 18.0, 8.0, 50.0, 650.0
    R = np.stack([np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0]),
                  np.array([1.0, 0.0, 0.0])], axis=1)
    assert np.isclose(np.linalg.det(R), 1.0)
    b = np.linspace(-0.05, 0.05, 1001)
    _, hit, m, _ = raycast.intersect_ecylinder(np.zeros(3), _rays(0.0, b),
                                               np.array([-L / 2, 0.0, Z]), R, ay, L, bz)
    expect = np.minimum(1.0 - Z * Z * b * b / (ay * ay + b * b * bz * bz), 0.5)
    assert np.allclose(m, expect, rtol=0, atol=1e-9)
    assert np.array_equal(hit, expect >= 0.0)
    assert hit.any() and (~hit).any()


def _prim(kind, rng):
    p = np.array([rng.uniform(-30, 30), rng.uniform(-30, 30), rng.uniform(450, 700)])
    R = _frame(rng.normal(size=3))
    if kind == raycast.SPHERE:
        return {"type": kind, "p": p, "R": np.eye(3), "size": np.array([rng.uniform(6, 12), 0, 0])}
    if kind == raycast.CYLINDER:
        return {"type": kind, "p": p, "R": R, "size": np.array([rng.uniform(6, 12),
                                                                rng.uniform(20, 45), 0])}
    if kind == raycast.ELLIPSOID:
        return {"type": kind, "p": p, "R": R, "size": rng.uniform(6, 22, 3)}
    if kind == raycast.CONE:
        return {"type": kind, "p": p, "R": R, "size": np.array([rng.uniform(6, 12),
                                                                rng.uniform(20, 45),
                                                                rng.uniform(4, 12)])}
    return {"type": kind, "p": p, "R": R, "size": np.array([rng.uniform(12, 25),
                                                            rng.uniform(20, 45),
                                                            rng.uniform(6, 12)])}


@pytest.mark.parametrize("kind", [raycast.SPHERE, raycast.CYLINDER, raycast.ELLIPSOID,
                                  raycast.CONE, raycast.ECYLINDER])
def test_margin_vanishes_on_the_hit_boundary(kind):
    """Between a hitting and a missing ray, bisection on the hit flag alone finds the
    boundary ray to 1e-13 in slope; there the margin is within 1e-8 of zero, and rays
    with a margin of at least 1e-3 keep their decision under a 1e-9 change of slope."""
    rng = np.random.default_rng(100 + kind)
    found = 0
    for _ in range(40):
        prim = _prim(kind, rng)
        centre = prim["p"] + (prim["R"][:, 2] * prim["size"][1] / 2 if kind in
                              (raycast.CYLINDER, raycast.CONE, raycast.ECYLINDER) else 0.0)
        d_in = centre / centre[2]
        d_out = d_in + rng.normal(size=3) * np.array([1, 1, 0]) * 0.2
        h_in = raycast.intersect_primitive(np.zeros(3), d_in[None], prim)[1][0]
        h_out = raycast.intersect_primitive(np.zeros(3), d_out[None], prim)[1][0]
        if not h_in or h_out:
            continue
        lo, hi = d_in, d_out
        for _ in range(80):
            mid = 0.5 * (lo + hi)
            if raycast.intersect_primitive(np.zeros(3), mid[None], prim)[1][0]:
                lo = mid
            else:
                hi = mid
        assert np.max(np.abs(hi - lo)) < 1e-13
        m_lo = raycast.intersect_primitive(np.zeros(3), lo[None], prim)[2][0]
        m_hi = raycast.intersect_primitive(np.zeros(3), hi[None], prim)[2][0]
        assert m_lo >= 0.0 > m_hi
        assert abs(m_lo) < 1e-8 and abs(m_hi) < 1e-8
        found += 1
        # robust rays keep their decision under a tiny change of direction
        ds = centre / centre[2] + rng.normal(size=(400, 3)) * np.array([1, 1, 0]) * 0.05
        _, h0, m0, *_ = raycast.intersect_primitive(np.zeros(3), ds, prim)
        jit = ds + rng.normal(size=ds.shape) * np.array([1, 1, 0]) * 1e-9
        _, h1, *_ = raycast.intersect_primitive(np.zeros(3), jit, prim)
        rob = np.abs(m0) >= 1e-3
        assert np.array_equal(h0[rob], h1[rob])
    assert found >= 10


def _tangent_sphere(d, r, s, offset):
    """A sphere of radius r whose centre lies at distance r * (1 + offset) from the ray
    t * d, at depth about s along it."""
    dh = d / np.linalg.norm(d)
    n = np.cross(dh, [0.0, 1.0, 0.0])
    n /= np.linalg.norm(n)
    c = s * dh + r * (1.0 + offset) * n
    return {"type": raycast.SPHERE, "p": c, "R": np.eye(3), "size": np.array([r, 0.0, 0.0])}


def _render(prims, W=9, H=9):
    cam = (60.0, 60.0, 4.0, 4.0)
    return raycast.render_primitives(prims, W, H, cam, 1500.0), raycast.pixel_directions(
        W, H, cam)


def test_classify_tangent_central_and_far_rays():
    """A sphere tangent to the centre pixel's ray (distance r (1 + 1e-7), margin about
    -2e-7) makes that pixel ambiguous; a sphere centred on a pixel's ray makes it a robust
    hit; pixels no primitive comes near are robust misses."""
    _, d = _render([])
    res, _ = _render([_tangent_sphere(d[4, 4], 8.0, 600.0, 1e-7)])
    cls = raycast.classify_pixels(res, TAU)
    assert cls["ambiguous"][4, 4] and not res["hit"][4, 4]
    assert cls["robust_miss"][0, 0]
    c = 600.0 * d[2, 6] / np.linalg.norm(d[2, 6])
    res, _ = _render([{"type": raycast.SPHERE, "p": c, "R": np.eye(3),
                       "size": np.array([3.0, 0, 0])}])
    cls = raycast.classify_pixels(res, TAU)
    assert cls["robust_hit"][2, 6] and not cls["ambiguous"][2, 6]
    assert cls["robust_miss"][8, 0]
    assert cls["ambiguous"].sum() == 0


def test_classify_near_margin_primitive_in_front_of_the_winner():
    """A robust hit of a far sphere at the centre pixel becomes ambiguous when a small sphere
    tangent to that ray (either side of the boundary) lies in front of it; behind the winner
    a tangent sphere that just hits leaves it robust, one that just misses (entry depth
    unknown) makes it ambiguous."""
    _, d = _render([])
    dc = d[4, 4] / np.linalg.norm(d[4, 4])
    far = {"type": raycast.SPHERE, "p": 900.0 * dc, "R": np.eye(3),
           "size": np.array([20.0, 0, 0])}
    res, _ = _render([far])
    assert raycast.classify_pixels(res, TAU)["robust_hit"][4, 4]
    for offset in (1e-7, -1e-7):
        res, _ = _render([far, _tangent_sphere(d[4, 4], 5.0, 600.0, offset)])
        cls = raycast.classify_pixels(res, TAU)
        assert cls["ambiguous"][4, 4], offset
    res, _ = _render([far, _tangent_sphere(d[4, 4], 5.0, 1200.0, -1e-7)])
    cls = raycast.classify_pixels(res, TAU)
    assert res["prim_hit"][1, 4, 4] and cls["robust_hit"][4, 4]
    res, _ = _render([far, _tangent_sphere(d[4, 4], 5.0, 1200.0, 1e-7)])
    cls = raycast.classify_pixels(res, TAU)
    assert not res["prim_hit"][1, 4, 4] and cls["ambiguous"][4, 4]
