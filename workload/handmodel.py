"""Seeded tables of the sphere / cylinder / ellipsoid hand (data only).

Pose layout per hand (Eq. 1-3 of the paper): indices 0..19 are the five fingers in the
order of Table 1 (thumb, index, middle, ring, little), each as (MP flexion, MP abduction,
PIP, DIP); indices 20..25 are the wrist (x, y, z, theta_x, theta_y, theta_z).  Angles are in
radians, lengths in millimetres.  A two-hand model is two consecutive 26-blocks.

Kinematic tree (read by both the HIP library and the oracle): every segment has a parent
(-1 for the root), a fixed rigid offset from its parent frame (3x4, rotation | translation)
and up to two revolute joints given as a unit axis in the segment frame and a pose index.
A segment frame is  parent * offset * Rot(axis0, h[dof0]) * Rot(axis1, h[dof1]).
A root segment is placed by the six wrist parameters starting at ``seg_root_dof``:
Trans(x, y, z) * Rz(theta_z) * Ry(theta_y) * Rx(theta_x) * offset.

Hand frame: +y runs along the fingers, +x points to the thumb side, +z is palmar.  Positive
flexion turns a phalanx from +y towards +z; positive MP abduction turns a finger towards the
thumb (so the abduction axis is -z), which matches the signs of Table 1 where the ring and
little finger ranges are non-positive.

Primitive table: type, segment, a local rigid frame (3x4 in the segment frame) and three
sizes:
  sphere             centre = frame origin, size = (r, 0, 0)
  cylinder           closed, flat caps; first cap centre = frame origin, axis = frame z,
                     size = (r, L, 0)
  ellipsoid          centre = frame origin, semi-axes (a, b, c) along frame x, y, z
  truncated cone     closed, flat caps; first cap centre = frame origin, axis = frame z,
                     size = (r0, L, r1): radius r0 at the first cap, r1 at the second
  elliptic cylinder  closed, flat caps; first cap centre = frame origin, axis = frame z,
                     size = (a, L, b): semi-axes a along frame x and b along frame y

Two primitive sets share the kinematic tree:
  "cylinders" (40 per hand: 16 spheres, 16 circular cylinders, 8 ellipsoids) - the workloads'
      hand: palm body cylinder capped by two ellipsoids, thenar ellipsoid, forearm stub,
      per finger a knuckle ellipsoid (thumb: ellipsoidal metacarpal), three phalanx
      cylinders and joint / tip spheres;
  "paper" (38 per hand, section II.A): the palm is an elliptic cylinder capped at both ends by
      ellipsoids; every finger has three truncated-cone phalanges and four spheres (three
      joints and the tip), except that the thumb's largest phalanx is an ellipsoid.
Radii lie in [5, 14] mm and lengths in [20, 50] mm, drawn from a seed.
"""
from __future__ import annotations

import numpy as np

DOF_PER_HAND = 26
SEG_PER_HAND = 16
PRIM_PER_HAND = 40                 # the "cylinders" set
PRIM_PER_HAND_PAPER = 38           # the "paper" set
WRIST_DOF = 20
SPHERE, CYLINDER, ELLIPSOID, CONE, ECYLINDER = 0, 1, 2, 3, 4

# Table 1 (degrees): rows thumb, index, middle, ring, little; columns MPx, MPz, PIP, DIP.
TABLE1_DEG = np.array([
    [[0, 90], [-15, 60], [0, 50], [-15, 70]],
    [[0, 90], [-15, 15], [0, 100], [0, 60]],
    [[0, 90], [-10, 10], [0, 100], [0, 60]],
    [[0, 90], [-30, 0], [0, 100], [0, 60]],
    [[0, 90], [-45, 0], [0, 100], [0, 60]],
], dtype=np.float64)
# Table 2: x, y, z in mm (converted from metres), rotations in degrees.
TABLE2 = np.array([[-900, 900], [-680, 680], [500, 1500], [-30, 120], [-70, 75], [-35, 20]],
                  dtype=np.float64)


def finger_dof(finger: int, joint: int) -> int:
    """Pose index of ``joint`` (0 MPx, 1 MPz, 2 PIP, 3 DIP) of ``finger`` (0 thumb .. 4 little)."""
    return 4 * finger + joint


def _rx(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])


def _ry(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def _rz(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def _frame(R=None, t=(0.0, 0.0, 0.0)):
    F = np.zeros((3, 4))
    F[:, :3] = np.eye(3) if R is None else R
    F[:, 3] = t
    return F


# Frames whose z axis points along segment +y (phalanx cylinders) or segment +x (palm body).
_ALONG_Y = _rx(-np.pi / 2)
_ALONG_X = _ry(np.pi / 2)


def joint_bounds_one_hand() -> tuple[np.ndarray, np.ndarray]:
    lo = np.zeros(DOF_PER_HAND)
    hi = np.zeros(DOF_PER_HAND)
    lo[:20] = np.deg2rad(TABLE1_DEG[:, :, 0].reshape(-1))
    hi[:20] = np.deg2rad(TABLE1_DEG[:, :, 1].reshape(-1))
    lo[20:23], hi[20:23] = TABLE2[:3, 0], TABLE2[:3, 1]
    lo[23:26], hi[23:26] = np.deg2rad(TABLE2[3:, 0]), np.deg2rad(TABLE2[3:, 1])
    return lo, hi


def _one_hand(rng: np.random.Generator):
    """Tables of one hand; returns (segments, prims) as python lists."""
    def radius(lo=6.0, hi=12.0):
        return float(rng.uniform(lo, hi))

    def length():
        return float(rng.uniform(20.0, 45.0))

    segs = []   # (parent, offset 3x4, [(axis, dof), ...])
    prims = []  # (type, seg, frame 3x4, size 3)
    Yk = 52.0                           # knuckle line
    segs.append((-1, _frame(), []))     # 0: palm (root)

    # palm: body cylinder across the hand capped by two ellipsoids, thenar ellipsoid,
    # forearm stub cylinder
    rb = radius(9.0, 12.0)
    Lb = length()
    prims.append((CYLINDER, 0, _frame(_ALONG_X, (-Lb / 2, Yk - 12.0, 0.0)), (rb, Lb, 0.0)))
    for side in (-1.0, 1.0):
        prims.append((ELLIPSOID, 0, _frame(None, (side * Lb / 2, Yk - 12.0, 0.0)),
                      (length() / 2, radius(9.0, 12.0), radius())))
    prims.append((ELLIPSOID, 0, _frame(_rz(-0.6), (22.0, 18.0, 2.0)),
                  (radius(), length() / 2, radius())))
    Lf = length()
    prims.append((CYLINDER, 0, _frame(_ALONG_Y, (0.0, Yk - 12.0 - Lf, 0.0)),
                  (radius(9.0, 12.0), Lf, 0.0)))

    abd_axis = np.array([0.0, 0.0, -1.0])
    flex_axis = np.array([1.0, 0.0, 0.0])
    bases = {0: (30.0, 16.0, 0.0), 1: (24.0, Yk, 0.0), 2: (8.0, Yk, 0.0),
             3: (-8.0, Yk, 0.0), 4: (-24.0, Yk, 0.0)}
    thumb_rot = _rz(-np.pi / 4) @ _ry(-np.pi / 3)
    for f in range(5):
        L = sorted([length() for _ in range(3)], reverse=True)
        r1 = radius(7.5, 12.0)
        r2, r3 = max(6.0, 0.9 * r1), max(6.0, 0.8 * r1)
        s1 = len(segs)
        R0 = thumb_rot if f == 0 else None
        segs.append((0, _frame(R0, bases[f]),
                     [(abd_axis, finger_dof(f, 1)), (flex_axis, finger_dof(f, 0))]))
        segs.append((s1, _frame(None, (0.0, L[0], 0.0)), [(flex_axis, finger_dof(f, 2))]))
        segs.append((s1 + 1, _frame(None, (0.0, L[1], 0.0)), [(flex_axis, finger_dof(f, 3))]))
        if f == 0:
            # thumb: CMC sphere, metacarpal ellipsoid, MCP sphere, proximal cylinder,
            # IP sphere, distal cylinder, tip sphere
            prims.append((SPHERE, s1, _frame(), (r1, 0.0, 0.0)))
            prims.append((ELLIPSOID, s1, _frame(None, (0.0, L[0] / 2, 0.0)),
                          (radius(), L[0] / 2, radius())))
            prims.append((SPHERE, s1 + 1, _frame(), (max(6.0, 0.95 * r1), 0.0, 0.0)))
        else:
            # finger: knuckle ellipsoid, proximal cylinder, PIP sphere
            prims.append((ELLIPSOID, s1, _frame(), (length() / 2, r1, max(6.0, 0.9 * r1))))
            prims.append((CYLINDER, s1, _frame(_ALONG_Y), (r1, L[0], 0.0)))
            prims.append((SPHERE, s1 + 1, _frame(), (max(6.0, 0.95 * r1), 0.0, 0.0)))
        prims.append((CYLINDER, s1 + 1, _frame(_ALONG_Y), (r2, L[1], 0.0)))
        prims.append((SPHERE, s1 + 2, _frame(), (max(6.0, 0.95 * r2), 0.0, 0.0)))
        prims.append((CYLINDER, s1 + 2, _frame(_ALONG_Y), (r3, L[2], 0.0)))
        prims.append((SPHERE, s1 + 2, _frame(None, (0.0, L[2], 0.0)), (r3, 0.0, 0.0)))
    assert len(segs) == SEG_PER_HAND and len(prims) == PRIM_PER_HAND
    return segs, prims


def _one_hand_paper(rng: np.random.Generator):
    """Tables of one hand with the primitive set of section II.A (38 primitives)."""
    segs = []
    prims = []
    Yk = 52.0                           # knuckle line
    segs.append((-1, _frame(), []))     # 0: palm (root)

    # palm: elliptic cylinder across the hand (axis +x), its cross-section a (thickness, along
    # z) by b (along the fingers, y), capped at both ends by ellipsoids of the same section
    a_p = float(rng.uniform(10.0, 13.0))
    b_p = float(rng.uniform(24.0, 30.0))
    L_p = float(rng.uniform(38.0, 48.0))
    y_p = Yk - b_p + 4.0
    # _ALONG_X: frame z = hand +x, frame x = hand -z, frame y = hand +y
    prims.append((ECYLINDER, 0, _frame(_ALONG_X, (-L_p / 2, y_p, 0.0)), (a_p, L_p, b_p)))
    for side in (-1.0, 1.0):
        prims.append((ELLIPSOID, 0, _frame(None, (side * L_p / 2, y_p, 0.0)),
                      (float(rng.uniform(8.0, 12.0)), b_p, a_p)))

    abd_axis = np.array([0.0, 0.0, -1.0])
    flex_axis = np.array([1.0, 0.0, 0.0])
    bases = {0: (L_p / 2 + 4.0, y_p - 10.0, 0.0), 1: (24.0, Yk, 0.0), 2: (8.0, Yk, 0.0),
             3: (-8.0, Yk, 0.0), 4: (-24.0, Yk, 0.0)}
    thumb_rot = _rz(-np.pi / 4) @ _ry(-np.pi / 3)
    for f in range(5):
        L = sorted([float(rng.uniform(20.0, 45.0)) for _ in range(3)], reverse=True)
        r1 = float(rng.uniform(8.0, 11.0))
        rad = [r1, max(5.0, 0.9 * r1), max(5.0, 0.8 * r1), max(5.0, 0.7 * r1)]
        s1 = len(segs)
        R0 = thumb_rot if f == 0 else None
        segs.append((0, _frame(R0, bases[f]),
                     [(abd_axis, finger_dof(f, 1)), (flex_axis, finger_dof(f, 0))]))
        segs.append((s1, _frame(None, (0.0, L[0], 0.0)), [(flex_axis, finger_dof(f, 2))]))
        segs.append((s1 + 1, _frame(None, (0.0, L[1], 0.0)), [(flex_axis, finger_dof(f, 3))]))
        # joint spheres at the three segment origins and the fingertip
        for j in range(3):
            prims.append((SPHERE, s1 + j, _frame(), (rad[j], 0.0, 0.0)))
        prims.append((SPHERE, s1 + 2, _frame(None, (0.0, L[2], 0.0)), (rad[3], 0.0, 0.0)))
        # phalanges: truncated cones tapering from joint to joint (thumb: its largest phalanx
        # is an ellipsoid)
        for j in range(3):
            if f == 0 and j == 0:
                prims.append((ELLIPSOID, s1, _frame(None, (0.0, L[0] / 2, 0.0)),
                              (rad[0], L[0] / 2, max(5.0, 0.85 * rad[0]))))
            else:
                prims.append((CONE, s1 + j, _frame(_ALONG_Y), (rad[j], L[j], rad[j + 1])))
    assert len(segs) == SEG_PER_HAND and len(prims) == PRIM_PER_HAND_PAPER
    return segs, prims


def make_hand_model(seed, n_hands: int = 1, primitive_set: str = "cylinders") -> dict:
    """Build the model tables for ``n_hands`` identical hands (two-hand particles are 52-D).

    ``seed`` is anything ``numpy.random.default_rng`` accepts; ``primitive_set`` is
    "cylinders" (40 primitives per hand) or "paper" (38, section II.A).  All returned arrays
    are contiguous; float tables are float64.
    """
    if n_hands not in (1, 2):
        raise ValueError("n_hands must be 1 or 2")
    rng = np.random.default_rng(seed)
    if primitive_set == "cylinders":
        segs, prims = _one_hand(rng)
    elif primitive_set == "paper":
        segs, prims = _one_hand_paper(rng)
    else:
        raise ValueError(f"unknown primitive set {primitive_set!r}")
    per = len(prims)
    n_seg, n_prim, n_dof = SEG_PER_HAND * n_hands, per * n_hands, DOF_PER_HAND * n_hands
    m = {
        "n_dof": n_dof, "n_seg": n_seg, "n_prim": n_prim,
        "seg_parent": np.full(n_seg, -1, np.int32),
        "seg_root_dof": np.full(n_seg, -1, np.int32),
        "seg_offset": np.zeros((n_seg, 3, 4)),
        "seg_joint_axis": np.zeros((n_seg, 2, 3)),
        "seg_joint_dof": np.full((n_seg, 2), -1, np.int32),
        "prim_type": np.zeros(n_prim, np.int32),
        "prim_seg": np.zeros(n_prim, np.int32),
        "prim_frame": np.zeros((n_prim, 3, 4)),
        "prim_size": np.zeros((n_prim, 3)),
        "bounds_lo": np.zeros(n_dof), "bounds_hi": np.zeros(n_dof),
        "mutate_mask": np.zeros(n_dof, np.uint8),
        "kc_pairs": np.zeros((3 * n_hands, 2), np.int32),
    }
    lo, hi = joint_bounds_one_hand()
    for hnd in range(n_hands):
        so, po, do = hnd * SEG_PER_HAND, hnd * per, hnd * DOF_PER_HAND
        for i, (parent, off, joints) in enumerate(segs):
            m["seg_parent"][so + i] = -1 if parent < 0 else parent + so
            m["seg_offset"][so + i] = off
            for j, (axis, dof) in enumerate(joints):
                m["seg_joint_axis"][so + i, j] = axis
                m["seg_joint_dof"][so + i, j] = dof + do
        m["seg_root_dof"][so] = do + WRIST_DOF
        for k, (typ, seg, frame, size) in enumerate(prims):
            m["prim_type"][po + k] = typ
            m["prim_seg"][po + k] = seg + so
            m["prim_frame"][po + k] = frame
            m["prim_size"][po + k] = size
        m["bounds_lo"][do:do + DOF_PER_HAND] = lo
        m["bounds_hi"][do:do + DOF_PER_HAND] = hi
        m["mutate_mask"][do:do + 20] = 1
        # collision pairs: abduction of (index, middle), (middle, ring), (ring, little);
        # the first of each pair is the finger nearer the thumb
        for q, (fa, fb) in enumerate(((1, 2), (2, 3), (3, 4))):
            m["kc_pairs"][3 * hnd + q] = (do + finger_dof(fa, 1), do + finger_dof(fb, 1))
    for key, val in m.items():
        if isinstance(val, np.ndarray):
            m[key] = np.ascontiguousarray(val)
    return m


def draw_true_pose_angles(rng: np.random.Generator, n_hands: int = 1) -> np.ndarray:
    """Raw draws of a true pose, translation (x, y) left at 0 for the caller to place.

    Finger angles are uniform within Table 1, redrawn until the abductions of index, middle,
    ring and little are non-increasing (no collision penalty); wrist rotations are uniform in
    [-20, 20] degrees; z is uniform in [570, 630] mm.
    """
    lo, hi = joint_bounds_one_hand()
    out = np.zeros(DOF_PER_HAND * n_hands)
    for hnd in range(n_hands):
        while True:
            fingers = rng.uniform(lo[:20], hi[:20])
            abd = fingers[[finger_dof(f, 1) for f in (1, 2, 3, 4)]]
            if np.all(np.diff(abd) <= 0.0):
                break
        h = np.zeros(DOF_PER_HAND)
        h[:20] = fingers
        h[22] = rng.uniform(570.0, 630.0)
        h[23:26] = np.deg2rad(rng.uniform(-20.0, 20.0, 3))
        out[hnd * DOF_PER_HAND:(hnd + 1) * DOF_PER_HAND] = h
    return out


def perturbed_particles(rng: np.random.Generator, h_true, n: int, angle_deg: float,
                        trans_mm: float, lo, hi) -> np.ndarray:
    """``n`` poses drawn uniformly in [h_true -/+ delta] intersected with [lo, hi], where delta
    is ``trans_mm`` for the wrist translations and ``angle_deg`` for every angle."""
    h_true = np.asarray(h_true, np.float64)
    delta = init_halfwidth(h_true.size, angle_deg, trans_mm)
    a, b = np.maximum(h_true - delta, lo), np.minimum(h_true + delta, hi)
    return a + rng.uniform(size=(n, h_true.size)) * (b - a)


def pose_walk_step(rng: np.random.Generator, h, kc_pairs, lo, hi, step_deg: float,
                   step_mm: float) -> np.ndarray:
    """One step of a smooth random walk of a true pose (a tracked hand between two frames):
    every angle moves by U(-step_deg, step_deg) degrees and every wrist translation by
    U(-step_mm, step_mm) mm, within [lo, hi]; the abductions stay ordered (kc = 0)."""
    h = np.asarray(h, np.float64)
    delta = init_halfwidth(h.size, step_deg, step_mm)
    out = np.clip(h + rng.uniform(-1.0, 1.0, h.size) * delta, lo, hi)
    for a, b in kc_pairs:
        out[b] = min(out[b], out[a])
    return out


def init_halfwidth(n_dof: int, angle_deg: float, trans_mm: float) -> np.ndarray:
    delta = np.full(n_dof, np.deg2rad(angle_deg))
    for hnd in range(n_dof // DOF_PER_HAND):
        b = hnd * DOF_PER_HAND + WRIST_DOF
        delta[b:b + 3] = trans_mm
    return delta
