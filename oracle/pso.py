"""Particle swarm optimisation of E (section III.B, Eq. 6-7), in float64.

Each particle is a pose h; a swarm per frame holds positions x, velocities v, personal bests
P (position and cost) and the global best G.  One generation, as read here:

 1. the costs E(x) of the current positions are given (evaluated by the caller);
 2. personal bests take every strictly better cost; G is the personal best of lowest cost
    (ties: lowest particle index);
 3. every ``mutate_every``-th generation (k + 1 divisible by it; the paper uses 3) the worst
    floor(P * mutate_frac) particles by current cost (ties: the higher index is worse) get
    their finger dimensions (the mutate mask, the 20 finger angles) re-drawn uniformly within
    the joint limits, their velocity zeroed in those dimensions, and skip step 4;
 4. every other particle moves by Eq. 6-7: v <- w (v + c1 r1 (P - x) + c2 r2 (G - x)),
    x <- x + v, with r1, r2 uniform in [0, 1) per dimension; a coordinate that leaves the
    joint limits (Tables 1-2) is clamped to the limit and its velocity zeroed;
 5. the generation counter advances.

Stop rule (section III.B stops at E < 1.0): with stop_cost > 0, a frame whose global best
after step 2 is below stop_cost keeps that generation's personal and global bests, skips
steps 3-4, records the generation count in ``stop_gen`` and is left unchanged afterwards.

Tracking (section II: the observation is a video; each frame's search starts from the
previous frame's solution): the initial box of frame t is c -/+ halfwidth clipped to the
joint limits, with c the previous frame's global best clipped to the limits (``box_around``).

The constriction factor of section III.B is w = 2 / |2 - psi - sqrt(psi^2 - 4 psi)| with
psi = c1 + c2.  Random numbers come from ``philox`` (see its docstring for the counters).

Gradient refinement (not in the paper): the ``refine_topk`` particles of lowest current cost
(ties: lower index first) take up to ``refine_steps`` steps of normalised steepest descent in
the space scaled by eta (eta_rot rad for angles, eta_trans mm for translations): with
g_s = eta * dE/dh the step is  x <- clamp(x - eta * g_s / max|g_s|), halved up to three
times until E decreases; a step that never decreases E ends the particle's refinement.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import cost, grad, philox


@dataclass
class PsoParams:
    w: float = 0.72
    c1: float = 2.05
    c2: float = 2.05
    mutate_every: int = 3
    mutate_frac: float = 0.5
    refine_topk: int = 0
    refine_steps: int = 0
    eta_rot: float = 0.02
    eta_trans: float = 2.0
    stop_cost: float = 0.0


def constriction(c1: float, c2: float) -> float:
    psi = c1 + c2
    return 2.0 / abs(2.0 - psi - np.sqrt(psi * psi - 4.0 * psi))


def init_state(init_lo, init_hi, n_particles: int, seed: int) -> dict:
    """Uniform positions in [init_lo, init_hi] (arrays [F, D]); zero velocity; no bests."""
    init_lo = np.atleast_2d(np.asarray(init_lo, np.float64))
    init_hi = np.atleast_2d(np.asarray(init_hi, np.float64))
    F, D = init_lo.shape
    P = n_particles
    x = np.zeros((F, P, D))
    for f in range(F):
        u, _ = philox.uniforms(seed, np.arange(D), f * P + np.arange(P), 0, philox.STREAM_INIT)
        x[f] = init_lo[f] + u * (init_hi[f] - init_lo[f])
    return {
        "x": x, "v": np.zeros((F, P, D)), "pbest_x": x.copy(),
        "pbest_cost": np.full((F, P), np.inf), "gbest_x": x[:, 0].copy(),
        "gbest_cost": np.full(F, np.inf), "gen": np.zeros(F, np.int64),
        "stop_gen": np.zeros(F, np.int64),
    }


def worst_set(costs, n_mut: int) -> np.ndarray:
    """Indices of the ``n_mut`` worst particles (ties: the higher index is worse)."""
    P = len(costs)
    order = sorted(range(P), key=lambda i: (-costs[i], -i))
    return np.array(sorted(order[:n_mut]), dtype=np.int64)


def update(state: dict, costs, params: PsoParams, lo, hi, mutate_mask, seed: int) -> dict:
    """Steps 2-5 of a generation for every frame, given the current costs [F, P]."""
    s = {k: np.array(v, copy=True) for k, v in state.items()}
    costs = np.asarray(costs, np.float64)
    F, P, D = s["x"].shape
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    mmask = np.asarray(mutate_mask).astype(bool)
    dims = np.arange(D)
    if "stop_gen" not in s:
        s["stop_gen"] = np.zeros(F, np.int64)
    for f in range(F):
        if s["stop_gen"][f] != 0:
            continue
        k = int(s["gen"][f])
        better = costs[f] < s["pbest_cost"][f]
        s["pbest_cost"][f][better] = costs[f][better]
        s["pbest_x"][f][better] = s["x"][f][better]
        g = int(np.argmin(s["pbest_cost"][f]))
        s["gbest_cost"][f] = s["pbest_cost"][f][g]
        s["gbest_x"][f] = s["pbest_x"][f][g]
        if params.stop_cost > 0.0 and s["gbest_cost"][f] < params.stop_cost:
            s["gen"][f] = k + 1
            s["stop_gen"][f] = k + 1
            continue
        gparts = f * P + np.arange(P)
        mutated = np.zeros(P, bool)
        if params.mutate_every > 0 and (k + 1) % params.mutate_every == 0:
            n_mut = int(np.floor(P * params.mutate_frac))
            mutated[worst_set(costs[f], n_mut)] = True
            u, _ = philox.uniforms(seed, dims, gparts, k, philox.STREAM_MUTATE)
            for i in np.nonzero(mutated)[0]:
                s["x"][f, i, mmask] = lo[mmask] + u[i, mmask] * (hi[mmask] - lo[mmask])
                s["v"][f, i, mmask] = 0.0
        r1, r2 = philox.uniforms(seed, dims, gparts, k, philox.STREAM_SWARM)
        for i in np.nonzero(~mutated)[0]:
            x, v = s["x"][f, i], s["v"][f, i]
            v = params.w * (v + params.c1 * r1[i] * (s["pbest_x"][f, i] - x)
                            + params.c2 * r2[i] * (s["gbest_x"][f] - x))
            x = x + v
            below, above = x < lo, x > hi
            x = np.where(below, lo, np.where(above, hi, x))
            v = np.where(below | above, 0.0, v)
            s["x"][f, i], s["v"][f, i] = x, v
        s["gen"][f] = k + 1
    return s


def eta_vector(model: dict, params: PsoParams) -> np.ndarray:
    eta = np.full(model["n_dof"], params.eta_rot)
    for b in model["seg_root_dof"][model["seg_root_dof"] >= 0]:
        eta[b:b + 3] = params.eta_trans
    return eta


def top_k(costs, K: int) -> np.ndarray:
    """The K lowest costs (ties: lower index first)."""
    order = sorted(range(len(costs)), key=lambda i: (costs[i], i))
    return np.array(order[:K], dtype=np.int64)


def refine_particle(model, obs, x, E, params: PsoParams, lo, hi, objective=None,
                    gradient=None, trace=None):
    """Normalised steepest-descent refinement of one particle; returns (x, E).

    Each step takes the gradient g at x, scales it by eta (g_s = eta * g) and tries the
    step eta * g_s / max|g_s| and its halves (1/2, 1/4, 1/8) in that order, each clipped to
    [lo, hi]; the first candidate whose cost is strictly below E(x) is taken.  No decrease
    (or a zero or non-finite g_s) ends the refinement.  ``objective(x) -> E`` and
    ``gradient(x) -> (E, g)`` default to the hand cost of Eq. 5 and its analytic gradient.
    With ``trace`` (a list), one entry per step is appended: the index j of the accepted
    length 2^-j, -1 for a rejected step, or None when g_s vanished."""
    if objective is None:
        def objective(xx):
            return cost.objective(model, xx, obs)
    if gradient is None:
        def gradient(xx):
            return grad.analytic_gradient(model, xx, obs)
    eta = eta_vector(model, params)
    x = np.asarray(x, np.float64).copy()
    for _ in range(params.refine_steps):
        E0, g = gradient(x)
        gs = eta * g
        n = np.max(np.abs(gs))
        if not np.isfinite(n) or n == 0.0:
            if trace is not None:
                trace.append(None)
            break
        delta = eta * gs / n
        accepted = -1
        for j in range(4):
            cand = np.clip(x - delta * 2.0 ** -j, lo, hi)
            Ec = objective(cand)
            if Ec < E0:
                x, E, accepted = cand, Ec, j
                break
        if trace is not None:
            trace.append(accepted)
        if accepted < 0:
            break
    return x, E


def box_around(center, halfwidth, lo, hi):
    """Initial box of a tracked frame: c -/+ halfwidth within [lo, hi], c = clip(center)."""
    c = np.clip(np.asarray(center, np.float64), lo, hi)
    return np.maximum(c - halfwidth, lo), np.minimum(c + halfwidth, hi)


def run(model, obs, init_lo, init_hi, n_particles, n_generations, params: PsoParams, seed):
    """A whole single-frame PSO run (FP64, slow); returns (state, gbest cost per generation)."""
    lo, hi = model["bounds_lo"], model["bounds_hi"]
    st = init_state(np.clip(init_lo, lo, hi), np.clip(init_hi, lo, hi), n_particles, seed)
    history = []
    for _ in range(n_generations):
        c = np.array([[cost.objective(model, st["x"][0, i], obs) for i in range(n_particles)]])
        if params.refine_topk > 0 and params.refine_steps > 0:
            for i in top_k(c[0], params.refine_topk):
                st["x"][0, i], c[0, i] = refine_particle(model, obs, st["x"][0, i], c[0, i],
                                                         params, lo, hi)
        st = update(st, c, params, lo, hi, model["mutate_mask"], seed)
        history.append(float(st["gbest_cost"][0]))
        if st["stop_gen"][0] != 0:
            break
    return st, history
