"""Pins of the oracle's swarm update (Eq. 6-7, mutation of section III.B) and of Philox."""
import numpy as np
import pytest

from oracle import philox, pso


def test_constriction_factor_of_section_3b():
    assert pso.constriction(2.8, 1.3) == pytest.approx(0.7298437881, abs=1e-10)
    assert pso.constriction(2.05, 2.05) == pytest.approx(0.7298437881, abs=1e-10)


def test_philox_4x64_matches_numpy_and_4x32_known_answers():
    bg = np.random.Philox(counter=[4, 7, 9, 11], key=[123, 456])
    ref = [int(x) for x in bg.random_raw(4)]          # numpy bumps the counter first
    assert philox.philox4([5, 7, 9, 11], [123, 456], width=64) == ref
    # Random123 known-answer vectors for Philox4x32-10
    assert philox.philox4([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C,
                                                    0x9B00DBD8]
    assert philox.philox4([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [0x408F276D, 0x41C83B0E,
                                                                  0xA20BC7C6, 0x6D5451FD]
    assert philox.philox4([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
                          [0xA4093822, 0x299F31D0]) == [0xD16CFE09, 0x94FDCCEB, 0x5001E420,
                                                        0x24126EA1]
    w = philox.philox4x32_vec(np.array([0x243F6A88]), np.array([0x85A308D3]),
                              np.array([0x13198A2E]), np.array([0x03707344]),
                              0xA4093822, 0x299F31D0)
    assert [int(x[0]) for x in w] == [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]
    u = philox.to_unit(np.array([0, 0xFFFFFFFF], np.uint32))
    assert u[0] == 0.0 and u[1] == 1.0 - 2.0 ** -24


def _state(F, P, D, rng):
    x = rng.uniform(-1, 1, (F, P, D))
    return {"x": x, "v": rng.uniform(-0.1, 0.1, (F, P, D)), "pbest_x": x.copy(),
            "pbest_cost": np.full((F, P), np.inf), "gbest_x": x[:, 0].copy(),
            "gbest_cost": np.full(F, np.inf), "gen": np.zeros(F, np.int64)}


def test_no_attraction_and_no_velocity_keeps_x():
    rng = np.random.default_rng(0)
    st = _state(2, 8, 26, rng)
    st["v"][:] = 0.0
    p = pso.PsoParams(c1=0.0, c2=0.0, mutate_every=0)
    lo, hi = np.full(26, -2.0), np.full(26, 2.0)
    out = pso.update(st, rng.uniform(size=(2, 8)), p, lo, hi, np.ones(26), seed=5)
    assert np.array_equal(out["x"], st["x"])
    assert np.all(out["gen"] == 1)


def test_eq6_eq7_single_particle_by_hand():
    D = 4
    st = {"x": np.array([[[0.5, -0.5, 1.9, 0.0]]]), "v": np.array([[[0.1, 0.2, 0.3, -0.4]]]),
          "pbest_x": np.array([[[1.0, 1.0, 1.0, 1.0]]]), "pbest_cost": np.array([[0.5]]),
          "gbest_x": np.zeros((1, D)), "gbest_cost": np.array([0.5]), "gen": np.array([4])}
    p = pso.PsoParams(w=0.7, c1=1.5, c2=1.0, mutate_every=3)
    lo, hi = np.full(D, -2.0), np.full(D, 2.0)
    out = pso.update(st, np.array([[0.25]]), p, lo, hi, np.ones(D), seed=99)
    # cost 0.25 < 0.5: personal and global best become x
    assert np.array_equal(out["pbest_x"][0, 0], st["x"][0, 0])
    assert out["gbest_cost"][0] == 0.25
    r1, r2 = philox.uniforms(99, np.arange(D), [0], 4, philox.STREAM_SWARM)
    x, v = st["x"][0, 0], st["v"][0, 0]
    v_new = 0.7 * (v + 1.5 * r1[0] * (x - x) + 1.0 * r2[0] * (x - x))
    x_new = x + v_new
    clamped = x_new > 2.0
    assert clamped[2]                                   # 1.9 + 0.7*0.3 > 2
    assert np.allclose(out["x"][0, 0], np.minimum(x_new, 2.0))
    assert np.allclose(out["v"][0, 0], np.where(clamped, 0.0, v_new))


def test_mutation_worst_half_finger_dims_only():
    rng = np.random.default_rng(1)
    F, P, D = 1, 10, 26
    st = _state(F, P, D, rng)
    st["gen"][:] = 2                                    # (2 + 1) % 3 == 0
    costs = np.array([[5.0, 1.0, 5.0, 2.0, 9.0, 0.5, 3.0, 5.0, 0.1, 7.0]])
    mask = np.r_[np.ones(20), np.zeros(6)]
    lo, hi = np.full(D, -3.0), np.full(D, 3.0)
    out = pso.update(st, costs, pso.PsoParams(), lo, hi, mask, seed=7)
    worst = pso.worst_set(costs[0], 5)
    # 9 (idx 4), 7 (idx 9), then the three 5.0s: all of 0, 2, 7 rank worse than 3.0
    assert list(worst) == [0, 2, 4, 7, 9]
    assert list(pso.worst_set(costs[0], 4)) == [2, 4, 7, 9]   # tie: higher index is worse
    u, _ = philox.uniforms(7, np.arange(D), np.arange(P), 2, philox.STREAM_MUTATE)
    for i in worst:
        assert np.allclose(out["x"][0, i, :20], -3.0 + 6.0 * u[i, :20])
        assert np.all(out["v"][0, i, :20] == 0.0)
        assert np.array_equal(out["x"][0, i, 20:], st["x"][0, i, 20:])
        assert np.array_equal(out["v"][0, i, 20:], st["v"][0, i, 20:])
    others = [i for i in range(P) if i not in worst]
    assert not np.allclose(out["x"][0, others], st["x"][0, others])


def test_sphere_function_converges_and_gbest_monotone():
    D, P = 26, 64
    lo, hi = np.full(D, -5.0), np.full(D, 5.0)
    st = pso.init_state(lo[None], hi[None], P, seed=3)
    p = pso.PsoParams(w=pso.constriction(2.05, 2.05), mutate_every=0)
    hist = []
    for _ in range(300):
        c = np.sum(st["x"] ** 2, axis=2)
        st = pso.update(st, c, p, lo, hi, np.zeros(D), seed=3)
        hist.append(st["gbest_cost"][0])
    assert np.all(np.diff(hist) <= 0.0)
    assert hist[0] > 10.0 and hist[-1] < 1e-3


def test_stop_rule_keeps_bests_and_freezes_the_frame():
    """Section III.B stop rule: the generation whose global best falls below the threshold
    records its personal / global bests, moves nobody, and nothing changes afterwards; a frame
    above the threshold runs on."""
    rng = np.random.default_rng(4)
    F, P, D = 2, 6, 5
    st = _state(F, P, D, rng)
    lo, hi = np.full(D, -1.0), np.full(D, 1.0)
    c = np.array([[0.5, 0.2, 0.9, 0.4, 0.3, 0.8], [5.0, 6.0, 7.0, 8.0, 9.0, 4.0]])
    p = pso.PsoParams(w=0.7, c1=1.5, c2=1.5, mutate_every=1, stop_cost=1.0)
    s1 = pso.update(st, c, p, lo, hi, np.ones(D), seed=1)
    # frame 0 stopped in generation 1: bests recorded, positions and velocities untouched
    assert s1["stop_gen"][0] == 1 and s1["gen"][0] == 1
    assert s1["gbest_cost"][0] == 0.2 and np.array_equal(s1["gbest_x"][0], st["x"][0, 1])
    assert np.array_equal(s1["pbest_cost"][0], c[0])
    assert np.array_equal(s1["x"][0], st["x"][0]) and np.array_equal(s1["v"][0], st["v"][0])
    # frame 1 is above the threshold: it moved
    assert s1["stop_gen"][1] == 0 and not np.array_equal(s1["x"][1], st["x"][1])
    # a later generation leaves frame 0 exactly as it was, even with better costs
    s2 = pso.update(s1, np.zeros((F, P)), p, lo, hi, np.ones(D), seed=1)
    for k in ("x", "v", "pbest_x", "pbest_cost"):
        assert np.array_equal(s2[k][0], s1[k][0])
    assert s2["gbest_cost"][0] == 0.2 and s2["gen"][0] == 1
    # and frame 1 now stops (cost 0 < 1)
    assert s2["stop_gen"][1] == 2


def test_tracking_box_and_moving_minimum():
    """The tracking box is c -/+ halfwidth inside the limits with c the clipped previous best;
    tracking a drifting quadratic minimum stays close to it in every frame."""
    lo, hi = np.array([-1.0, 0.0, 5.0]), np.array([1.0, 2.0, 9.0])
    a, b = pso.box_around(np.array([0.9, -3.0, 7.0]), np.array([0.5, 0.5, 10.0]), lo, hi)
    assert np.array_equal(a, [0.4, 0.0, 5.0]) and np.array_equal(b, [1.0, 0.5, 9.0])
    D, P = 6, 32
    lo, hi = np.full(D, -10.0), np.full(D, 10.0)
    hw = np.full(D, 1.0)
    rng = np.random.default_rng(2)
    target = rng.uniform(-2, 2, D)
    center = target.copy()
    p = pso.PsoParams(w=pso.constriction(2.8, 1.3), c1=2.8, c2=1.3, mutate_every=0)
    for t in range(8):
        target = target + 0.3 * rng.uniform(-1, 1, D)          # the minimum drifts
        bl, bh = pso.box_around(center, hw, lo, hi)
        st = pso.init_state(bl[None], bh[None], P, seed=10 + t)
        for _ in range(40):
            c = np.sum((st["x"] - target) ** 2, axis=2)
            st = pso.update(st, c, p, lo, hi, np.zeros(D), seed=10 + t)
        center = st["gbest_x"][0]
        assert np.max(np.abs(center - target)) < 0.05
