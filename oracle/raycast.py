"""Depth image r_d(h, C) of a hand hypothesis by exact ray casting, in float64.

Section III.A obtains the model depth image by projecting the model with the camera's focal
length and view C; the paper rasterises tessellated primitives with OpenGL.  Here the image
is the exact one: for every pixel the ray through the pixel is intersected analytically with
each primitive (closed solids) and the nearest entry point in front of the camera is kept.

Camera (a reading; the paper gives no intrinsics): pinhole, no distortion, ray of pixel
(u, v) through integer pixel coordinates with direction ((u-cx)/fx, (v-cy)/fy, 1), so the ray
parameter t of a point *is* its depth (camera z).  An optional camera pose (rotation and
centre, world-from-camera) is supported for invariance checks.

Every intersector returns, per ray, the entry parameter t (inf on a miss), the hit flag and a
dimensionless margin m whose sign decides hit (m >= 0) or miss and whose size measures how
far the ray is from flipping that decision:
  sphere     m = 1 - rho^2 / r^2, rho = distance from the centre to the ray line
  ellipsoid  m = 1 - rho'^2, the same in the frame where the ellipsoid is the unit sphere
  cylinder   max over its three surfaces of that surface's smallest slack: the side's radial
             slack (r^2 - rho^2)/r^2 and axial slacks s/L, (L-s)/L at each side crossing,
             each cap's radial slack (r^2 - rho_cap^2)/r^2 where the ray crosses its plane.
  truncated cone   the same with the side's slack disc / (|A| r_max^2) of its quadratic
             A t^2 + 2 B t + C (the cylinder's radial slack when r0 = r1) and each cap's radial
             slack against that cap's radius.
  elliptic cylinder   the cylinder's margin in the frame where it is the unit-radius cylinder.

Section II.A builds the hand from spheres, truncated cones (phalanges), ellipsoids and an
elliptic-cylinder palm; the circular cylinder is the truncated cone with equal radii.
"""
from __future__ import annotations

import numpy as np

from . import fk

SPHERE, CYLINDER, ELLIPSOID, CONE, ECYLINDER = 0, 1, 2, 3, 4


def pixel_directions(W: int, H: int, cam) -> np.ndarray:
    """Camera-frame ray directions [H, W, 3] with unit z component."""
    fx, fy, cx, cy = (float(c) for c in cam)
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    d = np.empty((H, W, 3))
    d[..., 0] = (u - cx) / fx
    d[..., 1] = (v - cy) / fy
    d[..., 2] = 1.0
    return d


def intersect_sphere(o, d, c, r):
    """Rays o + t d against the solid sphere |x - c| <= r.  d: [N, 3]."""
    w = np.asarray(o, np.float64) - c
    a = np.einsum("ij,ij->i", d, d)
    b = d @ w
    cc = w @ w - r * r
    disc = b * b - a * cc
    margin = disc / (a * r * r)
    hit = disc >= 0.0
    t = np.where(hit, (-b - np.sqrt(np.where(hit, disc, 0.0))) / a, np.inf)
    hit &= t > 0.0
    t = np.where(hit, t, np.inf)
    return t, hit, margin


def intersect_ellipsoid(o, d, c, R, semi):
    """Rays against the solid ellipsoid with centre c, axes R[:, i] and semi-axes semi[i]."""
    Minv = (R / semi[None, :]).T          # maps camera offsets to unit-sphere coordinates
    w = Minv @ (np.asarray(o, np.float64) - c)
    e = d @ Minv.T
    A = np.einsum("ij,ij->i", e, e)
    B = e @ w
    C = w @ w - 1.0
    disc = B * B - A * C
    margin = disc / A
    hit = disc >= 0.0
    t = np.where(hit, (-B - np.sqrt(np.where(hit, disc, 0.0))) / A, np.inf)
    hit &= t > 0.0
    t = np.where(hit, t, np.inf)
    return t, hit, margin


def intersect_cylinder(o, d, p0, axis, r, L):
    """Rays against the closed circular cylinder from p0 to p0 + L*axis with radius r."""
    w = np.asarray(o, np.float64) - p0
    da = d @ axis
    wa = w @ axis
    dp = d - da[:, None] * axis[None, :]
    wp = w - wa * axis
    r2 = r * r
    n = d.shape[0]
    cand_t = []
    slacks = []
    # side: |wp + t dp|^2 = r^2
    A = np.einsum("ij,ij->i", dp, dp)
    B = dp @ wp
    C = wp @ wp - r2
    disc = B * B - A * C
    with np.errstate(divide="ignore", invalid="ignore"):
        radial_slack = np.where(A > 0.0, disc / (A * r2), -np.inf)
        sq = np.sqrt(np.where(disc >= 0.0, disc, 0.0))
        for sign in (-1.0, 1.0):
            t = np.where(A > 0.0, (-B + sign * sq) / A, np.inf)
            s = wa + t * da
            slack = np.minimum(radial_slack, np.minimum(s / L, (L - s) / L))
            slack = np.where(A > 0.0, np.where(disc >= 0.0, slack, radial_slack), -np.inf)
            cand_t.append(np.where((slack >= 0.0) & (t > 0.0), t, np.inf))
            slacks.append(slack)
        # caps: planes s = 0 and s = L
        for s_cap in (0.0, L):
            t = np.where(da != 0.0, (s_cap - wa) / da, np.inf)
            q = wp[None, :] + t[:, None] * dp
            rad2 = np.einsum("ij,ij->i", q, q)
            slack = np.where(da != 0.0, (r2 - rad2) / r2, -np.inf)
            cand_t.append(np.where((slack >= 0.0) & (t > 0.0), t, np.inf))
            slacks.append(slack)
    cand = np.stack(cand_t)
    t_entry = np.min(cand, axis=0)
    margin = np.max(np.stack(slacks), axis=0)
    hit = np.isfinite(t_entry)
    # which surface the entry lies on: 0 side, 1 cap at s = 0, 2 cap at s = L
    surface = np.array([0, 0, 1, 2])[np.argmin(cand, axis=0)]
    assert t_entry.shape == (n,)
    return t_entry, hit, margin, surface


def intersect_cone(o, d, p0, R, r0, L, r1):
    """Rays against the closed truncated cone whose axis is R[:, 2] from p0 (s = 0, radius r0)
    to p0 + L R[:, 2] (s = L, radius r1), capped by flat discs.  In the cone's frame a point y
    is inside when y0^2 + y1^2 <= (r0 + k y2)^2 with k = (r1 - r0) / L and 0 <= y2 <= L."""
    w = (np.asarray(o, np.float64) - p0) @ R          # local ray origin
    e = d @ R                                          # local directions [N, 3]
    k = (r1 - r0) / L
    rw = r0 + k * w[2]                                 # radius at the origin's axial position
    A = e[:, 0] ** 2 + e[:, 1] ** 2 - (k * e[:, 2]) ** 2
    B = w[0] * e[:, 0] + w[1] * e[:, 1] - k * e[:, 2] * rw
    C = w[0] ** 2 + w[1] ** 2 - rw ** 2
    disc = B * B - A * C
    rmax2 = max(r0, r1) ** 2
    cand_t, slacks = [], []
    with np.errstate(divide="ignore", invalid="ignore"):
        disc_slack = np.where(A != 0.0, disc / (np.abs(A) * rmax2), np.inf)
        sq = np.sqrt(np.where(disc >= 0.0, disc, 0.0))
        # the two side roots in a form that stays finite as A -> 0
        q = -(B + np.where(B >= 0.0, 1.0, -1.0) * sq)
        roots = (np.where(q != 0.0, q / A, np.inf), np.where(q != 0.0, C / q, np.inf))
        for t in roots:
            s_ax = w[2] + t * e[:, 2]
            slack = np.minimum(disc_slack, np.minimum(s_ax / L, (L - s_ax) / L))
            slack = np.where(disc >= 0.0, slack, disc_slack)
            ok = (disc >= 0.0) & np.isfinite(t) & (slack >= 0.0) & (t > 0.0)
            cand_t.append(np.where(ok, t, np.inf))
            slacks.append(np.where(np.isfinite(t), slack, -np.inf))
        for s_cap, r_cap in ((0.0, r0), (L, r1)):
            t = np.where(e[:, 2] != 0.0, (s_cap - w[2]) / e[:, 2], np.inf)
            rad2 = (w[0] + t * e[:, 0]) ** 2 + (w[1] + t * e[:, 1]) ** 2
            slack = np.where(e[:, 2] != 0.0, (r_cap * r_cap - rad2) / (r_cap * r_cap), -np.inf)
            cand_t.append(np.where((slack >= 0.0) & (t > 0.0), t, np.inf))
            slacks.append(slack)
    cand = np.stack(cand_t)
    t_entry = np.min(cand, axis=0)
    margin = np.max(np.stack(slacks), axis=0)
    hit = np.isfinite(t_entry)
    surface = np.array([0, 0, 1, 2])[np.argmin(cand, axis=0)]
    return t_entry, hit, margin, surface


def intersect_ecylinder(o, d, p0, R, a, L, b):
    """Rays against the closed elliptic cylinder with first cap centre p0, axis R[:, 2], length
    L and semi-axes a along R[:, 0], b along R[:, 1].  An affine map (which keeps the ray
    parameter) takes it to the unit-radius circular cylinder."""
    S = np.array([1.0 / a, 1.0 / b, 1.0])
    w = ((np.asarray(o, np.float64) - p0) @ R) * S
    e = (d @ R) * S[None, :]
    return intersect_cylinder(w, e, np.zeros(3), np.array([0.0, 0.0, 1.0]), 1.0, L)


def intersect_primitive(o, d, prim):
    typ, p, R, size = prim["type"], prim["p"], prim["R"], prim["size"]
    zero = np.zeros(d.shape[0], np.int64)
    if typ == SPHERE:
        return intersect_sphere(o, d, p, size[0]) + (zero,)
    if typ == CYLINDER:
        return intersect_cylinder(o, d, p, R[:, 2], size[0], size[1])
    if typ == ELLIPSOID:
        return intersect_ellipsoid(o, d, p, R, size) + (zero,)
    if typ == CONE:
        return intersect_cone(o, d, p, R, size[0], size[1], size[2])
    if typ == ECYLINDER:
        return intersect_ecylinder(o, d, p, R, size[0], size[1], size[2])
    raise ValueError(f"unknown primitive type {typ}")


def render_primitives(prims, W, H, cam, bg_depth, cam_pose=None):
    """Render a list of camera-space primitives.

    Returns a dict with, per pixel: ``depth`` r_d, ``hit``, ``winner`` (primitive index of the
    nearest entry, lowest index on ties, -1 on a miss), ``zmin``; and per primitive
    ``prim_t`` [n, H, W], ``prim_hit``, ``prim_margin``, ``prim_surface`` (cylinders, cones and
    elliptic cylinders: entry on 0 the side, 1 the cap at s = 0, 2 the cap at s = L).

    Background reading: with bg_depth B > 0 the scene has a plane at depth B, a model point
    behind it is hidden, misses render B and hit = (nearest entry < B).  With B <= 0 there is
    no plane and misses render 0.
    """
    d_cam = pixel_directions(W, H, cam).reshape(-1, 3)
    if cam_pose is None:
        o, d = np.zeros(3), d_cam
    else:
        Rc, oc = cam_pose
        o, d = np.asarray(oc, np.float64), d_cam @ np.asarray(Rc, np.float64).T
    n = len(prims)
    prim_t = np.full((n, H * W), np.inf)
    prim_hit = np.zeros((n, H * W), bool)
    prim_margin = np.zeros((n, H * W))
    prim_surface = np.zeros((n, H * W), np.int64)
    for k, prim in enumerate(prims):
        t, hit, m, surf = intersect_primitive(o, d, prim)
        prim_t[k], prim_hit[k], prim_margin[k], prim_surface[k] = t, hit, m, surf
    if n:
        winner = np.argmin(prim_t, axis=0)
        zmin = prim_t[winner, np.arange(H * W)]
    else:
        winner = np.zeros(H * W, np.int64)
        zmin = np.full(H * W, np.inf)
    if bg_depth > 0.0:
        hit = zmin < bg_depth
        depth = np.where(hit, zmin, bg_depth)
    else:
        hit = np.isfinite(zmin)
        depth = np.where(hit, zmin, 0.0)
    winner = np.where(hit, winner, -1)
    shp = (H, W)
    return {
        "depth": depth.reshape(shp), "hit": hit.reshape(shp), "winner": winner.reshape(shp),
        "zmin": zmin.reshape(shp),
        "prim_t": prim_t.reshape((n,) + shp), "prim_hit": prim_hit.reshape((n,) + shp),
        "prim_margin": prim_margin.reshape((n,) + shp),
        "prim_surface": prim_surface.reshape((n,) + shp),
    }


def render(model: dict, h, W: int, H: int, cam, bg_depth: float, cam_pose=None):
    """r_d(h, C): forward kinematics, then ray casting of every primitive."""
    return render_primitives(fk.camera_primitives(model, h), W, H, cam, bg_depth, cam_pose)


def classify_pixels(res, tau: float = 1e-5):
    """Robust-hit / robust-miss / ambiguous classification of each pixel.

    Robust hit: some primitive margin >= tau and no primitive with |margin| < tau lies in
    front of the nearest robust entry.  Robust miss: every margin <= -tau.  Everything else
    (including hits behind the background plane decided within tau) is ambiguous.
    """
    m = res["prim_margin"]
    near = np.abs(m) < tau
    robust_miss = np.all(m <= -tau, axis=0)
    robust_t = np.where(m >= tau, res["prim_t"], np.inf)
    best_robust = np.min(robust_t, axis=0)
    # a near-boundary primitive whose (possible) entry lies in front of the robust winner;
    # for a primitive that misses we do not know t, so any near-boundary primitive counts
    near_in_front = np.any(near & ((res["prim_t"] <= best_robust[None]) | ~res["prim_hit"]),
                           axis=0)
    robust_hit = np.isfinite(best_robust) & ~near_in_front
    ambiguous = ~(robust_hit | robust_miss)
    return {"robust_hit": robust_hit, "robust_miss": robust_miss, "ambiguous": ambiguous,
            "near_boundary_any": np.any(near, axis=0)}
