"""The image-disc bound behind the ray caster's tile culling, checked by sampling.

The kernels bound the perspective image of a sphere (centre q, radius r, q_z > r) by a disc
whose centre lies at normalised radius (tan(theta + alpha) + tan(theta - alpha)) / 2 from the
principal point, along the direction of q, with radius (tan(theta + alpha) -
tan(theta - alpha)) / 2; theta is the angle of q from the optical axis and sin(alpha) =
r / |q|.  A capsule's image (the convex hull of its end spheres' images) then lies within the
larger radius of the segment joining the two centres.  These tests sample surface points and
check both statements in FP64.
"""
import numpy as np


def image_disc(q, r):
    q = np.asarray(q, np.float64)
    rad = np.hypot(q[0], q[1])
    n = np.linalg.norm(q)
    st, ct, sa = rad / n, q[2] / n, r / n
    ca = np.sqrt(1.0 - sa * sa)
    tp = (st * ca + ct * sa) / (ct * ca - st * sa)
    tm = (st * ca - ct * sa) / (ct * ca + st * sa)
    e = q[:2] / rad if rad > 0 else np.array([1.0, 0.0])
    return e * 0.5 * (tp + tm), 0.5 * (tp - tm)


def sphere_points(rng, q, r, n):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return np.asarray(q) + r * v


def test_sphere_image_in_disc():
    rng = np.random.default_rng(7)
    worst = -np.inf
    for _ in range(300):
        r = rng.uniform(2.0, 60.0)
        Z = rng.uniform(r * 1.05, 1500.0)
        q = np.array([rng.uniform(-1.5, 1.5) * Z, rng.uniform(-1.5, 1.5) * Z, Z])
        c, h = image_disc(q, r)
        pts = sphere_points(rng, q, r, 4000)
        img = pts[:, :2] / pts[:, 2:3]
        d = np.linalg.norm(img - c, axis=1)
        worst = max(worst, float(np.max(d - h) / h))
    assert worst <= 1e-9


def test_disc_is_tight_on_axis():
    # on the optical axis the image is a circle of normalised radius tan(alpha)
    c, h = image_disc([0.0, 0.0, 500.0], 30.0)
    assert np.allclose(c, 0.0)
    assert abs(h - np.tan(np.arcsin(30.0 / 500.0))) < 1e-12


def test_capsule_image_within_reach_of_segment():
    rng = np.random.default_rng(11)
    for _ in range(200):
        r = rng.uniform(3.0, 15.0)
        q0 = np.array([rng.uniform(-300, 300), rng.uniform(-300, 300), rng.uniform(200, 1200)])
        q1 = q0 + rng.normal(size=3) * rng.uniform(5, 60)
        if min(q0[2], q1[2]) <= 1.01 * r:
            continue
        c0, h0 = image_disc(q0, r)
        c1, h1 = image_disc(q1, r)
        reach = max(h0, h1)
        s = rng.random((3000, 1))
        pts = sphere_points(rng, np.zeros(3), r, 3000) * rng.random((3000, 1)) ** (1 / 3)
        pts = pts + (1 - s) * q0 + s * q1            # points of the solid capsule
        img = pts[:, :2] / pts[:, 2:3]
        v = c1 - c0
        vv = v @ v
        t = np.clip(((img - c0) @ v) / vv, 0.0, 1.0) if vv > 0 else np.zeros(len(img))
        dist = np.linalg.norm(img - (c0 + t[:, None] * v), axis=1)
        assert np.max(dist) <= reach * (1 + 1e-9)
