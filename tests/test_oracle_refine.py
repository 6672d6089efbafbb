"""Pins of the oracle's gradient refinement (not in the paper; the refined swarm of the
two-hand workload) and of its top-K selection.

The step logic is pinned on objectives whose minimiser, gradient and every candidate cost are
known in closed form, so the normalisation by max|eta * g|, the halvings, the strict-decrease
acceptance, the clip to the bounds and the early stop are each decided by hand.  The
selection is pinned by a hand-worked example with ties and by brute force over all orderings
of small arrays."""
import itertools

import numpy as np
import pytest

from oracle import pso
from workload import make_hand_model, seed_sequence

WX = 20          # wrist x (a translation: eta_trans)


@pytest.fixture(scope="module")
def model():
    return make_hand_model(seed_sequence(0, 10_000))


def _quadratic(a, weights):
    """f(x) = sum_d w_d (x_d - a_d)^2 with its gradient."""
    a, w = np.asarray(a, np.float64), np.asarray(weights, np.float64)

    def f(x):
        return float(np.sum(w * (x - a) ** 2))

    def g(x):
        return f(x), 2.0 * w * (x - a)
    return f, g


def _wide_bounds(n):
    return np.full(n, -1e6), np.full(n, 1e6)


def test_eta_vector_marks_the_wrist_translations(model):
    p = pso.PsoParams(eta_rot=0.02, eta_trans=2.0)
    eta = pso.eta_vector(model, p)
    assert np.all(eta[20:23] == 2.0)
    assert np.all(eta[:20] == 0.02) and np.all(eta[23:26] == 0.02)


def test_full_step_then_half_step_then_stop(model):
    """1-D quadratic in wrist x, minimum at a, start a + 3 mm.  The normalised step is
    eta_trans = 2 mm towards a: a + 1 (cost 1 < 9, accepted at full length); from a + 1 the
    full step lands on a - 1 (cost 1, not below 1: rejected), the half step on a (cost 0:
    accepted); at a the gradient vanishes and the refinement ends."""
    D = model["n_dof"]
    a = np.zeros(D)
    a[WX] = 10.0
    w = np.zeros(D)
    w[WX] = 1.0
    f, g = _quadratic(a, w)
    x0 = a.copy()
    x0[WX] += 3.0
    lo, hi = _wide_bounds(D)
    trace = []
    x, E = pso.refine_particle(model, None, x0, f(x0),
                               pso.PsoParams(refine_steps=3, eta_trans=2.0), lo, hi,
                               objective=f, gradient=g, trace=trace)
    assert trace == [0, 1, None]
    assert x[WX] == 10.0 and E == 0.0
    assert np.array_equal(np.delete(x, WX), np.delete(x0, WX))


def test_every_length_overshoots_so_the_first_step_is_rejected(model):
    """Start 0.1 mm from the minimum: the four lengths 2, 1, 1/2, 1/4 mm land 1.9, 0.9, 0.4
    and 0.15 mm beyond it, all costlier than 0.01: the step is rejected, the particle keeps
    its position and cost, and no further step is tried."""
    D = model["n_dof"]
    a = np.zeros(D)
    w = np.zeros(D)
    w[WX] = 1.0
    f, g = _quadratic(a, w)
    x0 = a.copy()
    x0[WX] = 0.1
    lo, hi = _wide_bounds(D)
    trace = []
    E0 = f(x0)
    x, E = pso.refine_particle(model, None, x0, E0, pso.PsoParams(refine_steps=3), lo, hi,
                               objective=f, gradient=g, trace=trace)
    assert trace == [-1]
    assert np.array_equal(x, x0) and E == E0


def test_normalisation_by_the_largest_scaled_component(model):
    """Two active dimensions, an angle (eta 0.02 rad) and wrist x (eta 2 mm), with gradient
    components 3 and 0.5: g_s = (0.06, 1.0), so the step is eta * g_s / 1.0 = (0.0012 rad,
    2 mm): the translation moves by its full eta, the angle by eta_rot * 0.06."""
    D = model["n_dof"]

    def f(x):
        return 3.0 * x[0] + 0.5 * x[WX] + 100.0

    def g(x):
        gg = np.zeros(D)
        gg[0], gg[WX] = 3.0, 0.5
        return f(x), gg
    x0 = np.zeros(D)
    x0[0], x0[WX] = 0.5, 50.0
    lo, hi = _wide_bounds(D)
    trace = []
    x, E = pso.refine_particle(model, None, x0, f(x0), pso.PsoParams(refine_steps=1), lo, hi,
                               objective=f, gradient=g, trace=trace)
    assert trace == [0]
    assert x[0] == pytest.approx(0.5 - 0.02 * 0.06, abs=1e-15)
    assert x[WX] == pytest.approx(48.0, abs=1e-12)
    assert E == pytest.approx(f(x))
    assert np.count_nonzero(x - x0) == 2


def test_candidates_are_clipped_to_the_bounds(model):
    """A linear cost falling towards +x with the upper bound 0.3 mm above the start: every
    candidate is clipped to the bound, so the full length is accepted there, and the next
    step (same direction) only reproduces the bound: no decrease, stop."""
    D = model["n_dof"]

    def f(x):
        return -x[WX]

    def g(x):
        gg = np.zeros(D)
        gg[WX] = -1.0
        return f(x), gg
    x0 = np.zeros(D)
    lo, hi = _wide_bounds(D)
    hi[WX] = 0.3
    trace = []
    x, E = pso.refine_particle(model, None, x0, f(x0), pso.PsoParams(refine_steps=3), lo, hi,
                               objective=f, gradient=g, trace=trace)
    assert trace == [0, -1]
    assert x[WX] == 0.3 and E == -0.3


def test_non_finite_gradient_ends_the_refinement(model):
    D = model["n_dof"]

    def f(x):
        return 1.0

    def g(x):
        gg = np.zeros(D)
        gg[3] = np.nan
        return 1.0, gg
    x0 = np.zeros(D)
    trace = []
    x, E = pso.refine_particle(model, None, x0, 1.0, pso.PsoParams(refine_steps=3),
                               *_wide_bounds(D), objective=f, gradient=g, trace=trace)
    assert trace == [None] and np.array_equal(x, x0) and E == 1.0


def test_refinement_on_the_hand_cost_never_raises_it(model):
    """On the hand cost itself (a 48x48 clean render of an open hand at 500 mm, the start
    6 mm and 3 degrees off): the first step is accepted, each accepted step strictly lowers
    E, and the returned cost is E at the returned position."""
    from oracle import cost, synth
    rng = np.random.default_rng(5)
    h_true = rng.uniform(model["bounds_lo"], model["bounds_hi"])
    h_true[[4 * f + j for f in range(5) for j in (0, 2, 3)]] = 0.2
    for a, b in model["kc_pairs"]:
        h_true[b] = min(h_true[b], h_true[a] - 0.02)
    h_true[20:26] = (0.0, -40.0, 500.0, 0.1, -0.1, 0.05)
    obs = synth.clean_observation(model, h_true, 48, 48, (108.0, 108.0, 23.5, 23.5))
    x0 = h_true.copy()
    x0[20] += 6.0
    x0[1] += np.deg2rad(3.0)
    E0 = cost.objective(model, x0, obs)
    trace = []
    x, E = pso.refine_particle(model, obs, x0, E0, pso.PsoParams(refine_steps=3),
                               model["bounds_lo"], model["bounds_hi"], trace=trace)
    assert E == cost.objective(model, x, obs)
    assert trace[0] is not None and trace[0] >= 0 and E < E0


def test_top_k_hand_worked_with_ties():
    c = [3.0, 1.0, 2.0, 1.0, 5.0, 2.0, 1.0]
    assert pso.top_k(c, 3).tolist() == [1, 3, 6]
    assert pso.top_k(c, 5).tolist() == [1, 3, 6, 2, 5]
    assert pso.top_k(c, 0).tolist() == []
    assert pso.top_k(c, 7).tolist() == [1, 3, 6, 2, 5, 0, 4]


@pytest.mark.parametrize("seed", range(6))
def test_top_k_against_brute_force(seed):
    """Among all K-subsets, the selection is the one with the smallest sorted (cost, index)
    sequence: every chosen pair precedes every excluded pair in (cost, index) order."""
    rng = np.random.default_rng(seed)
    n = 7
    c = rng.integers(0, 3, n).astype(np.float64)
    for K in range(n + 1):
        sel = pso.top_k(c, K)
        best = min(itertools.combinations(range(n), K),
                   key=lambda s: sorted((c[i], i) for i in s))
        assert sorted(sel.tolist()) == sorted(best)
        keys = [(c[i], i) for i in sel]
        assert keys == sorted(keys)
        # every chosen (cost, index) precedes every excluded one
        out = [(c[e], e) for e in range(n) if e not in set(sel.tolist())]
        assert all(k < o for k in keys for o in out)
