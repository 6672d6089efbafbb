"""Gradient of E with respect to the pose, in float64: analytic and finite-difference.

The paper optimises E only with PSO and gives no gradient.  E is piecewise smooth: the Dice
term and sum(o_s or r_m) are piecewise constant (zero derivative almost everywhere), so the
derivative comes from the clamped depth sum of Eq. 4 and from kc (Eq. 5):

  dE/dh = (1 / sum(o_s or r_m)) * sum_p s_p * d r_d(p) / dh + lambda_k * d kc / dh,
  s_p = sign(r_d - o_d) on hit pixels with |o_d - r_d| < d_M, else 0.

d r_d / dh is obtained by forward-mode differentiation of the forward kinematics (the
derivative of every segment transform with respect to every pose parameter) and implicit
differentiation of the nearest primitive's surface equation G(y) = 0 at the entry point
x = t d, y = R^T (x - p):  dt/dh = -(dG/dy . dy/dh) / (dG/dy . R^T d).

``fd_mask`` selects pixels away from silhouette / occlusion edges, creases between two
primitives and the kinks of |.|, min(., d_M) and the d_m test, where E is smooth in h; on that
mask a central difference of the masked smooth cost (sum(o_s or r_m) frozen at the base pose)
must agree with the analytic gradient.
"""
from __future__ import annotations

import numpy as np

from . import cost, fk, raycast


def _skew(a):
    return np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])


def transform_derivatives(model: dict, h):
    """Segment transforms T [n_seg, 4, 4] and their derivatives dT [n_dof, n_seg, 4, 4]."""
    h = np.asarray(h, np.float64)
    n_seg, n_dof = model["n_seg"], model["n_dof"]
    T = np.zeros((n_seg, 4, 4))
    dT = np.zeros((n_dof, n_seg, 4, 4))
    done = np.zeros(n_seg, bool)

    def solve(s):
        if done[s]:
            return
        parent = int(model["seg_parent"][s])
        if parent < 0:
            b = int(model["seg_root_dof"][s])
            x, y, z, tx, ty, tz = h[b:b + 6]
            Rx, Ry, Rz = fk.rot_x(tx), fk.rot_y(ty), fk.rot_z(tz)
            base = fk.homog(Rz @ Ry @ Rx, (x, y, z))
            dbase = np.zeros((n_dof, 4, 4))
            for i in range(3):
                dbase[b + i, i, 3] = 1.0
            dbase[b + 3, :3, :3] = Rz @ Ry @ (_skew((1.0, 0, 0)) @ Rx)
            dbase[b + 4, :3, :3] = Rz @ (_skew((0, 1.0, 0)) @ Ry) @ Rx
            dbase[b + 5, :3, :3] = (_skew((0, 0, 1.0)) @ Rz) @ Ry @ Rx
        else:
            solve(parent)
            base, dbase = T[parent], dT[:, parent]
        off = fk.from_3x4(model["seg_offset"][s])
        mats, dmats = [], []
        for j in range(2):
            dof = int(model["seg_joint_dof"][s, j])
            if dof >= 0:
                axis = model["seg_joint_axis"][s, j]
                Rj = fk.rot_axis(axis, h[dof])
                mats.append((dof, fk.homog(Rj)))
                dR = np.zeros((4, 4))
                dR[:3, :3] = _skew(axis) @ Rj
                dmats.append(dR)
        local = off.copy()
        for _, M in mats:
            local = local @ M
        T[s] = base @ local
        dT[:, s] = dbase @ local
        for i, (dof, _) in enumerate(mats):
            left = base @ off
            for _, M in mats[:i]:
                left = left @ M
            right = np.eye(4)
            for _, M in mats[i + 1:]:
                right = right @ M
            dT[dof, s] += left @ dmats[i] @ right
        done[s] = True

    for s in range(n_seg):
        solve(s)
    return T, dT


def depth_gradient(model: dict, h, res, W, H, cam):
    """d r_d / dh per pixel [n_dof, H, W] (zero at pixels that miss)."""
    n_dof = model["n_dof"]
    T, dT = transform_derivatives(model, h)
    d = raycast.pixel_directions(W, H, cam).reshape(-1, 3)
    winner = res["winner"].reshape(-1)
    zmin = res["zmin"].reshape(-1)
    out = np.zeros((n_dof, H * W))
    for k in np.unique(winner[winner >= 0]):
        pix = np.nonzero(winner == k)[0]
        s = int(model["prim_seg"][k])
        PF = fk.from_3x4(model["prim_frame"][k])
        F = T[s] @ PF
        dF = dT[:, s] @ PF
        R, p = F[:3, :3], F[:3, 3]
        t = zmin[pix]
        x = t[:, None] * d[pix]
        y = (x - p) @ R                       # rows: R^T (x - p)
        yd = d[pix] @ R                       # R^T d
        typ = int(model["prim_type"][k])
        size = model["prim_size"][k]
        if typ == raycast.SPHERE:
            gy = 2.0 * y
        elif typ == raycast.ELLIPSOID:
            gy = 2.0 * y / (size ** 2)[None, :]
        else:
            # capped solids: side surface G(y) = 0 below, caps y2 = 0 and y2 = L
            surf = res["prim_surface"][k].reshape(-1)[pix]
            gy = np.zeros_like(y)
            side = surf == 0
            if typ == raycast.CYLINDER:
                gy[side, 0] = 2.0 * y[side, 0]
                gy[side, 1] = 2.0 * y[side, 1]
            elif typ == raycast.CONE:          # y0^2 + y1^2 - (r0 + k y2)^2
                kk = (size[2] - size[0]) / size[1]
                gy[side, 0] = 2.0 * y[side, 0]
                gy[side, 1] = 2.0 * y[side, 1]
                gy[side, 2] = -2.0 * kk * (size[0] + kk * y[side, 2])
            else:                              # (y0 / a)^2 + (y1 / b)^2 - 1
                gy[side, 0] = 2.0 * y[side, 0] / size[0] ** 2
                gy[side, 1] = 2.0 * y[side, 1] / size[2] ** 2
            gy[surf == 1, 2] = -1.0
            gy[surf == 2, 2] = 1.0
        denom = np.einsum("ij,ij->i", gy, yd)
        for j in range(n_dof):
            dR, dp = dF[j, :3, :3], dF[j, :3, 3]
            if not (np.any(dR) or np.any(dp)):
                continue
            dy = (x - p) @ dR - dp @ R        # dR^T (x - p) - R^T dp
            out[j, pix] = -np.einsum("ij,ij->i", gy, dy) / denom
    return out.reshape(n_dof, H, W)


def depth_sign(obs_depth, res):
    """s_p of the clamped depth term: sign(r_d - o_d) where hit and |o_d - r_d| < d_M."""
    diff = res["depth"] - np.asarray(obs_depth, np.float64)
    active = res["hit"] & (np.abs(diff) < cost.D_CLAMP_MM)
    return np.where(active, np.sign(diff), 0.0)


def analytic_gradient(model: dict, h, obs: dict, pixel_mask=None):
    """(E, dE/dh) with the depth term restricted to ``pixel_mask`` (None = all pixels)."""
    h = np.asarray(h, np.float64)
    E, parts = cost.objective(model, h, obs, return_parts=True)
    if not np.isfinite(E):
        return E, np.zeros(model["n_dof"])
    res = parts["render"]
    H, W = obs["depth"].shape
    dz = depth_gradient(model, h, res, W, H, obs["cam"])
    s = depth_sign(obs["depth"], res)
    if pixel_mask is not None:
        s = s * np.asarray(pixel_mask, bool)
    g = np.zeros(model["n_dof"])
    if parts["S_or"] > 0:
        g = np.einsum("jhw,hw->j", dz, s) / parts["S_or"]
    g += cost.LAMBDA_K * cost.kc_grad(model, h)
    return E, g


def _dilate(mask, r):
    out = mask.copy()
    H, W = mask.shape
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            ys, yd = (slice(max(dy, 0), H), slice(0, H - max(dy, 0))) if dy >= 0 else \
                     (slice(0, H + dy), slice(-dy, H))
            xs, xd = (slice(max(dx, 0), W), slice(0, W - max(dx, 0))) if dx >= 0 else \
                     (slice(0, W + dx), slice(-dx, W))
            out[yd, xd] |= mask[ys, xs]
    return out


def fd_mask(res, obs_depth, border: int = 2, occlusion_dz: float = 1.0,
            kink_mm: float = 0.1, crease_mm: float = 0.5):
    """Pixels where the masked depth sum is smooth in h (see the module docstring)."""
    hit, win, z = res["hit"], res["winner"], res["depth"]
    H, W = hit.shape
    edge = np.zeros((H, W), bool)
    for dy, dx in ((0, 1), (1, 0), (1, 1), (1, -1)):
        a = (slice(0, H - dy), slice(max(-dx, 0), W - max(dx, 0)))
        b = (slice(dy, H), slice(max(dx, 0), W - max(-dx, 0)))
        sil = hit[a] != hit[b]
        occ = (win[a] != win[b]) & (np.abs(z[a] - z[b]) > occlusion_dz)
        e = sil | occ
        edge[a] |= e
        edge[b] |= e
    bad = _dilate(edge, border)
    diff = np.abs(np.asarray(obs_depth, np.float64) - z)
    for kink in (0.0, cost.D_MATCH_MM, cost.D_CLAMP_MM):
        bad |= np.abs(diff - kink) < kink_mm
    pt = np.sort(res["prim_t"], axis=0)
    if pt.shape[0] >= 2:
        with np.errstate(invalid="ignore"):
            bad |= hit & (pt[1] - pt[0] < crease_mm)
    return ~bad


def dof_is_translation(model: dict) -> np.ndarray:
    """True for the wrist translations (mm), False for the angles (rad)."""
    trans = np.zeros(model["n_dof"], bool)
    for b in model["seg_root_dof"][model["seg_root_dof"] >= 0]:
        trans[b:b + 3] = True
    return trans


def fd_protocol_mask(model, h, res, obs, step_rad=1e-3, step_mm=1e-2, **kw):
    """``fd_mask`` narrowed for central differences with fixed steps: a step moves a pixel's
    depth by up to reach = max_j |d r_d / d h_j| * step_j (first order), so the kinks of |.| and
    min(., d_M) and the crease to the second-nearest surface must be farther than twice that
    for the pixel's term to stay on one smooth piece over [h - step, h + step].  Every change
    of the nearest primitive between neighbouring pixels is also an edge here, whatever the
    depth step across it (a primitive emerging from another's surface makes a crease that the
    pixels beside it, where the emerging primitive misses, cannot see)."""
    H, W = obs["depth"].shape
    base = fd_mask(res, obs["depth"], **kw)
    win = res["winner"]
    crease = np.zeros((H, W), bool)
    for dy, dx in ((0, 1), (1, 0), (1, 1), (1, -1)):
        a = (slice(0, H - dy), slice(max(-dx, 0), W - max(dx, 0)))
        b = (slice(dy, H), slice(max(dx, 0), W - max(-dx, 0)))
        e = win[a] != win[b]
        crease[a] |= e
        crease[b] |= e
    base &= ~_dilate(crease, kw.get("border", 2))
    dz = depth_gradient(model, h, res, W, H, obs["cam"])
    steps = np.where(dof_is_translation(model), step_mm, step_rad)
    reach = np.max(np.abs(dz) * steps[:, None, None], axis=0)
    diff = np.abs(np.asarray(obs["depth"], np.float64) - res["depth"])
    bad = (diff < 2.0 * reach) | (np.abs(diff - cost.D_CLAMP_MM) < 2.0 * reach)
    pt = np.sort(res["prim_t"], axis=0)
    if pt.shape[0] >= 2:
        with np.errstate(invalid="ignore"):
            bad |= res["hit"] & (pt[1] - pt[0] < 2.0 * reach)
    return base & ~bad


def gradient_terms(model, h, obs, pixel_mask=None):
    """Per-pixel terms of the depth part of dE/dh, [n_dof, H, W]: s_p * d r_d(p) / dh /
    sum(o_s or r_m) (their sum over the pixels plus lambda_k dkc/dh is the analytic
    gradient)."""
    h = np.asarray(h, np.float64)
    E, parts = cost.objective(model, h, obs, return_parts=True)
    res = parts["render"]
    H, W = obs["depth"].shape
    s = depth_sign(obs["depth"], res)
    if pixel_mask is not None:
        s = s * np.asarray(pixel_mask, bool)
    if parts["S_or"] == 0:
        return np.zeros((model["n_dof"], H, W))
    return depth_gradient(model, h, res, W, H, obs["cam"]) * s[None] / parts["S_or"]


def masked_smooth_cost(model, h, obs, mask, S_or_fixed):
    """(1 / S_or_fixed) * sum over ``mask`` of min(|o_d - r_d(h)|, d_M) + lambda_k kc(h)."""
    H, W = obs["depth"].shape
    res = raycast.render(model, h, W, H, obs["cam"], obs["bg"])
    t_d = np.minimum(np.abs(np.asarray(obs["depth"], np.float64) - res["depth"]),
                     cost.D_CLAMP_MM)
    return float(np.sum(t_d[mask])) / S_or_fixed + cost.LAMBDA_K * cost.kc(model, h)


def fd_gradient(model, h, obs, mask, S_or_fixed, step_rad=1e-3, step_mm=1e-2, dofs=None):
    """Central differences of ``masked_smooth_cost``; translation dims use ``step_mm``."""
    h = np.asarray(h, np.float64)
    g = np.zeros(model["n_dof"])
    trans = dof_is_translation(model)
    for j in (range(model["n_dof"]) if dofs is None else dofs):
        step = step_mm if trans[j] else step_rad
        hp, hm = h.copy(), h.copy()
        hp[j] += step
        hm[j] -= step
        g[j] = (masked_smooth_cost(model, hp, obs, mask, S_or_fixed)
                - masked_smooth_cost(model, hm, obs, mask, S_or_fixed)) / (2.0 * step)
    return g
