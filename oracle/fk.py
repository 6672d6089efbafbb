"""Forward kinematics of the hand model, in float64 (section II.A, Eq. 1-3).

The pose h lists, per hand, the four angles of each finger (Eq. 1) followed by the wrist
position and orientation (Eq. 2); Eq. 3 stacks them.  The paper places every part with
"graphical matrices" without stating axes or rotation order; the readings used here are:
wrist transform Trans(x, y, z) * Rz(theta_z) * Ry(theta_y) * Rx(theta_x), and every other
segment is parent * fixed offset * Rot(axis0, angle0) * Rot(axis1, angle1) with the axes
given by the model table.  All transforms are 4x4 homogeneous matrices mapping segment
coordinates to camera coordinates (camera at the origin looking along +z, x right, y down).
"""
from __future__ import annotations

import numpy as np


def rot_axis(axis, angle: float) -> np.ndarray:
    """Rotation matrix about a unit ``axis`` by ``angle`` (Rodrigues' formula)."""
    a = np.asarray(axis, dtype=np.float64)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) + np.sin(angle) * K + (1.0 - np.cos(angle)) * (K @ K)


def rot_x(a):
    return rot_axis((1.0, 0.0, 0.0), a)


def rot_y(a):
    return rot_axis((0.0, 1.0, 0.0), a)


def rot_z(a):
    return rot_axis((0.0, 0.0, 1.0), a)


def homog(R=None, t=None) -> np.ndarray:
    T = np.eye(4)
    if R is not None:
        T[:3, :3] = R
    if t is not None:
        T[:3, 3] = t
    return T


def from_3x4(F) -> np.ndarray:
    T = np.eye(4)
    T[:3, :] = F
    return T


def wrist_transform(q6) -> np.ndarray:
    """Eq. 2 parameters (x, y, z, theta_x, theta_y, theta_z) -> camera-from-wrist."""
    x, y, z, tx, ty, tz = (float(v) for v in q6)
    return homog(rot_z(tz) @ rot_y(ty) @ rot_x(tx), (x, y, z))


def segment_transforms(model: dict, h) -> np.ndarray:
    """Camera-from-segment transforms [n_seg, 4, 4] for pose ``h``."""
    h = np.asarray(h, dtype=np.float64)
    n_seg = model["n_seg"]
    out = np.zeros((n_seg, 4, 4))
    done = np.zeros(n_seg, dtype=bool)

    def solve(s):
        if done[s]:
            return out[s]
        parent = int(model["seg_parent"][s])
        if parent < 0:
            b = int(model["seg_root_dof"][s])
            base = wrist_transform(h[b:b + 6])
        else:
            base = solve(parent)
        T = base @ from_3x4(model["seg_offset"][s])
        for j in range(2):
            dof = int(model["seg_joint_dof"][s, j])
            if dof >= 0:
                T = T @ homog(rot_axis(model["seg_joint_axis"][s, j], h[dof]))
        out[s] = T
        done[s] = True
        return T

    for s in range(n_seg):
        solve(s)
    return out


def primitive_frames(model: dict, h) -> np.ndarray:
    """Camera-from-primitive frames [n_prim, 4, 4]."""
    T = segment_transforms(model, h)
    n = model["n_prim"]
    out = np.zeros((n, 4, 4))
    for k in range(n):
        out[k] = T[model["prim_seg"][k]] @ from_3x4(model["prim_frame"][k])
    return out


def camera_primitives(model: dict, h) -> list[dict]:
    """Each primitive in camera coordinates: type, origin p, rotation R (columns = local
    axes), sizes.  Sphere: centre p, radius size[0].  Cylinder: first cap centre p, axis R[:,2],
    radius size[0], length size[1].  Ellipsoid: centre p, semi-axes size along R's columns.
    Truncated cone: first cap centre p, axis R[:,2], radii size[0] (s = 0) and size[2]
    (s = L), length size[1].  Elliptic cylinder: first cap centre p, axis R[:,2], semi-axes
    size[0] along R[:,0] and size[2] along R[:,1], length size[1]."""
    F = primitive_frames(model, h)
    prims = []
    for k in range(model["n_prim"]):
        prims.append({
            "type": int(model["prim_type"][k]),
            "p": F[k, :3, 3].copy(),
            "R": F[k, :3, :3].copy(),
            "size": np.asarray(model["prim_size"][k], dtype=np.float64).copy(),
            "seg": int(model["prim_seg"][k]),
        })
    return prims
