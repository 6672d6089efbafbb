"""GPU swarm kernels against the oracle's swarm update (Eq. 6-7, mutation of section III.B):
initialisation and single generations given identical state and costs; graph replay."""
import numpy as np
import pytest

import paper_2005_07068_amd as ht
from gpu_util import frame_for, make_ctx, oracle_renders, torch_cuda
from oracle import philox, pso

pytestmark = pytest.mark.gpu


def _setup(cfg_idx=1, P=64):
    torch = torch_cuda()
    cfg, model, fr = frame_for(cfg_idx)
    ctx = make_ctx(model, [fr])
    dev = torch.device("cuda:0")
    from workload.handmodel import init_halfwidth
    delta = init_halfwidth(model["n_dof"], 10.0, 20.0)
    lo = (fr["h_true"] - delta).astype(np.float32)
    hi = (fr["h_true"] + delta).astype(np.float32)
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    sw = ctx.swarm(slots, P, torch.tensor(lo), torch.tensor(hi), seed=123456789012345)
    return torch, ctx, model, fr, sw, lo, hi


def _host(sw):
    return {k: sw[k].cpu().numpy().astype(np.float64) if k != "gen" else
            sw[k].cpu().numpy().astype(np.int64)
            for k in ("x", "v", "pbest_x", "pbest_cost", "gbest_x", "gbest_cost", "gen")}


def test_init_matches_oracle():
    torch, ctx, model, fr, sw, lo, hi = _setup()
    ctx.pso_init(sw)
    torch.cuda.synchronize()
    ref = pso.init_state(np.maximum(lo, model["bounds_lo"].astype(np.float32)).astype(np.float64),
                         np.minimum(hi, model["bounds_hi"].astype(np.float32)).astype(np.float64),
                         64, 123456789012345)
    x = sw["x"].cpu().numpy()
    assert np.allclose(x, ref["x"], rtol=0, atol=1e-4)
    assert np.all(sw["v"].cpu().numpy() == 0) and np.all(sw["gen"].cpu().numpy() == 0)
    assert np.all(np.isinf(sw["pbest_cost"].cpu().numpy()))


W_PAPER = float(pso.constriction(2.8, 1.3))
CONSTANTS = {
    # the workloads' literal constants, with the mutation of section III.B
    "workload": dict(w=0.72, c1=2.05, c2=2.05, mutate_every=3),
    # section III.B: c1 = 2.8, c2 = 1.3 and the constriction factor w of psi = c1 + c2
    "paper": dict(w=W_PAPER, c1=2.8, c2=1.3, mutate_every=3),
    # without the mutation step
    "no_mutation": dict(w=0.72, c1=2.05, c2=2.05, mutate_every=0),
    "paper_no_mutation": dict(w=W_PAPER, c1=2.8, c2=1.3, mutate_every=0),
}


@pytest.mark.parametrize("consts", sorted(CONSTANTS))
@pytest.mark.parametrize("gen", [0, 2])
def test_single_generation_matches_oracle(gen, consts):
    """One generation from a mid-run state against the oracle's update, for each set of swarm
    constants (generation 2 is a mutation generation when the mutation is on)."""
    kw = CONSTANTS[consts]
    torch, ctx, model, fr, sw, lo, hi = _setup()
    ctx.pso_init(sw)
    rng = np.random.default_rng(gen)
    # a mid-run state: random velocities and personal bests, generation counter `gen`
    sw["v"].copy_(torch.tensor(rng.uniform(-0.05, 0.05, sw["v"].shape).astype(np.float32)))
    pb = sw["x"].cpu().numpy() + rng.uniform(-0.02, 0.02, sw["x"].shape).astype(np.float32)
    sw["pbest_x"].copy_(torch.tensor(pb))
    sw["pbest_cost"].copy_(torch.tensor(rng.uniform(28, 60, (1, 64)).astype(np.float32)))
    sw["gen"].fill_(gen)
    torch.cuda.synchronize()
    before = _host(sw)
    params = ht.pso_params(**kw)
    ctx.pso_step(sw, params)
    torch.cuda.synchronize()
    costs = sw["cost"].cpu().numpy().astype(np.float64)
    after = _host(sw)
    ref = pso.update(before, costs, pso.PsoParams(w=float(np.float32(kw["w"])), c1=kw["c1"],
                                                  c2=kw["c2"], mutate_every=kw["mutate_every"]),
                     model["bounds_lo"].astype(np.float32), model["bounds_hi"].astype(np.float32),
                     model["mutate_mask"], 123456789012345)
    assert np.array_equal(after["pbest_cost"], ref["pbest_cost"])
    assert np.array_equal(after["gbest_cost"], ref["gbest_cost"])
    assert after["gen"][0] == gen + 1
    for k in ("x", "v", "pbest_x", "gbest_x"):
        assert np.allclose(after[k], ref[k], rtol=1e-5, atol=2e-5), k
    # mutated particles (only in a mutation generation with the mutation on): their finger
    # dimensions are re-drawn and their velocity there zeroed
    zeroed = np.all(after["v"][0, :, :20] == 0.0, axis=1)
    if gen == 2 and kw["mutate_every"] == 3:
        assert zeroed.sum() >= 32
    else:
        assert not zeroed.any()


@pytest.mark.parametrize("P", [100, 600, 1000])
def test_mutation_generation_matches_oracle_with_ties(P):
    """A mutation generation (the worst half by current cost re-drawn, ties: the higher index is
    worse) at swarm sizes whose ranking sorts one key per thread across several wavefronts
    (100, 1000 particles) or several keys per thread (600); duplicated positions give exactly
    tied costs."""
    torch, ctx, model, fr, sw, lo, hi = _setup(P=P)
    ctx.pso_init(sw)
    x = sw["x"].clone()
    x[0, 1::7] = x[0, 0]
    sw["x"].copy_(x)
    sw["gen"].fill_(2)
    torch.cuda.synchronize()
    before = _host(sw)
    params = ht.pso_params(w=0.72, c1=2.05, c2=2.05)
    ctx.pso_step(sw, params)
    torch.cuda.synchronize()
    costs = sw["cost"].cpu().numpy().astype(np.float64)
    assert len(np.unique(costs)) < P            # ties present
    after = _host(sw)
    ref = pso.update(before, costs, pso.PsoParams(w=0.72, c1=2.05, c2=2.05),
                     model["bounds_lo"].astype(np.float32), model["bounds_hi"].astype(np.float32),
                     model["mutate_mask"], 123456789012345)
    moved_gpu = np.any(after["x"][0] != before["x"][0], axis=1)
    moved_ref = np.any(ref["x"][0] != before["x"][0], axis=1)
    # mutated particles are exactly the oracle's (their re-drawn dimensions differ from any
    # Eq. 6-7 move); the others follow Eq. 6-7 within FP32 rounding
    mutated_ref = np.zeros(P, bool)
    order = sorted(range(P), key=lambda i: (costs[0, i], i))
    mutated_ref[order[P - P // 2:]] = True
    mask = model["mutate_mask"].astype(bool)
    assert np.allclose(after["x"][0][mutated_ref][:, mask], ref["x"][0][mutated_ref][:, mask],
                       rtol=1e-6, atol=1e-6)
    assert np.all(after["v"][0][mutated_ref][:, mask] == 0.0)
    assert np.allclose(after["x"], ref["x"], rtol=1e-5, atol=2e-5)
    assert np.allclose(after["v"], ref["v"], rtol=1e-5, atol=2e-5)
    assert np.array_equal(moved_gpu, moved_ref)


def test_graph_replay_equals_eager_and_gbest_monotone():
    torch, ctx, model, fr, sw, lo, hi = _setup()
    params = ht.pso_params()
    ctx.pso_init(sw)
    hist = []
    for _ in range(8):
        ctx.pso_step(sw, params)
        hist.append(float(sw["gbest_cost"].cpu()[0]))
    eager = sw["gbest_x"].cpu().numpy().copy()
    assert all(b <= a for a, b in zip(hist, hist[1:]))
    for _ in range(3):
        sw["x"].zero_()
        ctx.pso_run_graph(sw, params, 8)
        torch.cuda.synchronize()
        assert np.array_equal(sw["gbest_x"].cpu().numpy(), eager)
        assert float(sw["gbest_cost"].cpu()[0]) == hist[-1]
        # eager work between replays
        ctx.eval(sw["x"][0], sw["frame_slots"])


def test_refinement_never_raises_the_cost():
    torch, ctx, model, fr, sw, lo, hi = _setup(P=64)
    ctx.pso_init(sw)
    plain = ht.pso_params(mutate_every=0)
    ctx.pso_step(sw, plain)
    x = sw["x"].clone()
    c0 = ctx.eval(x[0], sw["frame_slots"]).cpu().numpy()
    refine = ht.pso_params(mutate_every=0, refine_topk=8, refine_steps=3)
    # the step evaluates x, refines the 8 best, then moves the swarm; the refined costs land
    # in sw["cost"] before the move
    ctx.pso_step(sw, refine)
    c1 = sw["cost"].cpu().numpy()[0]
    top = np.argsort(c0, kind="stable")[:8]
    assert np.all(c1[top] <= c0[top])
    assert np.any(c1[top] < c0[top])
    others = np.setdiff1d(np.arange(64), top)
    assert np.array_equal(c1[others], c0[others])


def test_refinement_reusing_the_swarm_kinematics_matches_recomputing_them():
    """The refinement's first gradient evaluation reads the swarm evaluation's kinematic tables
    through the selection when the workspace already holds them with a wrench buffer (after
    reserve), and computes them again when the workspace must grow first (no reserve, first
    step): the swarms agree bit for bit after one step and after three."""
    runs = []
    for reserve in (False, True):
        torch, ctx, model, fr, sw, lo, hi = _setup(P=64)
        if reserve:
            ctx.reserve(64 * 4, fr["depth"].size)
        ctx.pso_init(sw)
        p = ht.pso_params(mutate_every=0, refine_topk=8, refine_steps=2)
        states = []
        for _ in range(3):
            ctx.pso_step(sw, p)
            states.append({k: sw[k].cpu().numpy().copy()
                           for k in ("x", "cost", "pbest_cost", "gbest_x", "gbest_cost")})
        ctx.close()
        runs.append(states)
    for a, b in zip(*runs):
        for k in a:
            assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("P,K", [(100, 40), (1000, 64), (100, 80)])
def test_refinement_selects_exactly_the_k_lowest(P, K):
    """The refined set is the K lowest current costs (ties: lower index), for a particle count
    that is not a multiple of the wavefront, the largest fast-path K and the full-sort path;
    duplicated positions create exact cost ties."""
    torch, ctx, model, fr, sw, lo, hi = _setup(P=P)
    ctx.pso_init(sw)
    plain = ht.pso_params(mutate_every=0)
    ctx.pso_step(sw, plain)
    # duplicate some positions so that their costs tie exactly
    x = sw["x"].clone()
    x[0, 1::7] = x[0, 0]
    sw["x"].copy_(x)
    c0 = ctx.eval(x[0], sw["frame_slots"]).cpu().numpy()
    ctx.pso_step(sw, ht.pso_params(mutate_every=0, refine_topk=K, refine_steps=1))
    c1 = sw["cost"].cpu().numpy()[0]
    top = np.array(sorted(range(P), key=lambda i: (c0[i], i))[:K])
    others = np.setdiff1d(np.arange(P), top)
    assert np.array_equal(c1[others], c0[others])
    assert np.all(c1[top] <= c0[top])


def test_whole_runs_match_the_oracle_distribution():
    """Whole 64 x 30 runs on the 128x128 frame, seeds 0..31, against the oracle's
    (golden/pso_final_errors_pso128.json, written from the oracle alone by
    golden/make_pso_final_errors.py).  Whole runs are chaotic, so the final joint errors and
    global-best costs are compared as distributions: two-sample Kolmogorov-Smirnov p > 0.01 and
    means within three standard errors of their difference."""
    import json
    import os

    from scipy import stats

    from workload.handmodel import init_halfwidth
    path = os.path.join(os.path.dirname(__file__), "golden", "pso_final_errors_pso128.json")
    with open(path) as f:
        ref = json.load(f)
    torch = torch_cuda()
    cfg, model, fr = frame_for(1)
    ctx = make_ctx(model, [fr])
    dev = torch.device("cuda:0")
    delta = init_halfwidth(model["n_dof"], cfg.init_angle_deg, cfg.init_trans_mm)
    lo = torch.tensor((fr["h_true"] - delta).astype(np.float32))
    hi = torch.tensor((fr["h_true"] + delta).astype(np.float32))
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    params = ht.pso_params(w=ref["w"], c1=ref["c1"], c2=ref["c2"],
                           mutate_every=ref["mutate_every"], mutate_frac=ref["mutate_frac"])
    errs, costs = [], []
    for s in ref["seeds"]:
        sw = ctx.swarm(slots, ref["particles"], lo, hi, seed=s)
        ctx.pso_init(sw)
        for _ in range(ref["generations"]):
            ctx.pso_step(sw, params)
        g = sw["gbest_x"].cpu().numpy()[0].astype(np.float64)
        errs.append(float(np.degrees(np.mean(np.abs(g[:20] - fr["h_true"][:20])))))
        costs.append(float(sw["gbest_cost"].cpu().numpy()[0]))
    ctx.close()
    r_err = [r["joint_error_deg"] for r in ref["runs"]]
    r_cost = [r["gbest_cost"] for r in ref["runs"]]
    for a, b in ((errs, r_err), (costs, r_cost)):
        assert stats.ks_2samp(a, b).pvalue > 0.01
        se = np.sqrt(np.var(a, ddof=1) / len(a) + np.var(b, ddof=1) / len(b))
        assert abs(np.mean(a) - np.mean(b)) <= 3.0 * se


def test_kernel_tracing_counts_one_refined_generation():
    """The per-kernel trace of one generation with refinement (K = 8, 2 steps, workspace
    reserved, so the first gradient evaluation reuses the swarm's kinematics): the swarm
    evaluation, the gradient evaluation of the 8 best, a gradient and a forward evaluation of
    the 32 candidates (each of these three assembled by the update kernel that follows it, not
    by a finalize launch), the select and three updates, and the swarm update."""
    torch, ctx, model, fr, sw, lo, hi = _setup(P=64)
    ctx.reserve(64 * 4, fr["depth"].size)
    ctx.pso_init(sw)
    torch.cuda.synchronize()
    ctx.profile_begin()
    ctx.pso_step(sw, ht.pso_params(mutate_every=0, refine_topk=8, refine_steps=2))
    st = ctx.profile_end()
    ctx.close()
    launches = {k: v["launches"] for k, v in st.items()}
    # every evaluation here has at most 256 particles, so the ray casts build their own work
    # lists (no work-list launch)
    assert launches == {"fk": 3, "sched": 0, "raycast": 2, "raycast_grad": 2, "finalize": 1,
                        "pso": 1, "refine": 4}, launches
    assert st["fk"]["particles"] == 64 + 2 * 32
    assert st["raycast_grad"]["particles"] == 8 + 32
    assert st["raycast"]["particles"] == 64 + 32
    assert all(v["ms"] > 0.0 for v in st.values() if v["launches"])


def test_refinement_matches_the_oracle_step_by_step():
    """The HIP refinement (gradient, four step lengths, accept, write-back into the swarm)
    against oracle.pso.refine_particle, one step at a time from the GPU's state (single-step
    parity, as for the swarm update), on the 128x128 frame: 12 particles within 1 deg / 1 mm
    of the true pose (steps halved or rejected, some at the first step) and 12 within
    3 deg / 3 mm (mostly full steps), all 24 refined (K = P), 3 steps.  With w = c1 = c2 = 0
    and no mutation a generation moves nobody, so the swarm's positions after each generation
    are the refined ones.

    Per step and particle, the oracle takes one step from the GPU's FP32 position with the
    resolved FP64 gradient (the oracle's formula, with the GPU's per-pixel decisions where the
    oracle finds them within the parity tolerances, from its debug images at that position).
    A step is compared when its accept decision is clear (every candidate cost differs from
    the current one by more than 1e-4 relative, the FP32 costs agree with the oracle's to
    about 1e-5, plus the most the candidate's margin-ambiguous pixels can move it): the new
    position must equal the oracle's to 1e-3 of the step scale eta per
    parameter (a different decision moves the parameter with the largest |eta g| by at least
    eta / 16), and the new cost must be the resolved oracle's cost there (1e-5 relative).
    Finally the three steps chained in one generation (candidates evaluated with their
    gradients, a stopped particle proposing nothing new) end where the single steps end."""
    torch, ctx, model, fr, sw, lo, hi = _setup(P=24)
    from gpu_util import check_particle, eval_debug, particles_for, resolved_gradient
    from oracle import cost as ocost
    from oracle import raycast
    near = particles_for(model, fr, 12, seed=7, angle_deg=1.0, trans_mm=1.0)
    mid = particles_for(model, fr, 12, seed=8, angle_deg=3.0, trans_mm=3.0)
    x0 = np.concatenate([near, mid])
    K, S = 24, 3
    H, W = fr["depth"].shape
    blo = model["bounds_lo"].astype(np.float32).astype(np.float64)
    bhi = model["bounds_hi"].astype(np.float32).astype(np.float64)
    one = pso.PsoParams(mutate_every=0, refine_topk=K, refine_steps=1)
    eta = pso.eta_vector(model, one)
    ctx.pso_init(sw)
    sw["x"].copy_(torch.tensor(x0[None]))
    step_p = ht.pso_params(w=0.0, c1=0.0, c2=0.0, mutate_every=0, refine_topk=K, refine_steps=1)
    n_cmp, rejected, halved, skipped = 0, 0, 0, 0
    first_rejected = set()
    for step in range(S):
        xs = sw["x"].cpu().numpy()[0].copy()
        c_s, dbg = eval_debug(ctx, xs, 0, W, H)
        ctx.pso_step(sw, step_p)
        torch.cuda.synchronize()
        xn = sw["x"].cpu().numpy()[0].astype(np.float64)
        cn = sw["cost"].cpu().numpy()[0]
        assert np.all(cn <= c_s)
        for i in range(K):
            clear, cur = [], [None]

            def objective(xx):
                # the decision E(candidate) < E(x) is clear when the gap exceeds 1e-4 of E
                # plus what the pixels decided within the margin can move E: each at most
                # (d_M + 2 lambda) / sum(o_s or r_m)
                e, parts = ocost.objective(model, xx, fr, return_parts=True)
                n_amb = int(raycast.classify_pixels(parts["render"])["ambiguous"].sum())
                per_px = (ocost.D_CLAMP_MM + 2 * ocost.LAMBDA) / max(parts["S_or"], 1)
                bound = 1e-4 * e + n_amb * per_px
                clear.append(abs(e - cur[0]) > bound)
                return e

            def gradient(xx, i=i):
                e, g = resolved_gradient(model, fr, xx, dbg, i)
                cur[0] = e
                return e, (g if g is not None else np.full(model["n_dof"], np.nan))

            trace = []
            xr, _ = pso.refine_particle(model, fr, xs[i].astype(np.float64), None, one, blo,
                                        bhi, objective=objective, gradient=gradient,
                                        trace=trace)
            if trace == [None] or not all(clear):
                skipped += 1          # undefined resolved gradient or a near-tie decision
                continue
            n_cmp += 1
            rejected += trace == [-1]
            halved += trace[0] > 0
            if step == 0 and trace == [-1]:
                first_rejected.add(i)
            err = np.abs(xn[i] - xr)
            assert np.all(err <= 1e-3 * eta), (step, i, trace, float(np.max(err / eta)))
            if trace == [-1]:
                assert np.array_equal(xn[i], xs[i].astype(np.float64)) and cn[i] == c_s[i]
        # the new costs are the GPU's evaluations at the new positions: the resolved oracle
        c_new, dbg_new = eval_debug(ctx, xn.astype(np.float32), 0, W, H)
        assert np.array_equal(c_new, cn)
        rendered = oracle_renders(model, [(fr, xn[i]) for i in range(K)])
        for i in range(K):
            check_particle(model, fr, xn[i], cn[i], dbg_new, i, rendered=rendered[i])
    print(f"refinement: {n_cmp} of {S * K} steps compared ({skipped} not), {rejected} "
          f"rejected ({len(first_rejected)} at the first step), {halved} halved")
    assert n_cmp >= 0.75 * S * K and first_rejected and halved >= 8
    # the chained refinement of one generation ends where the single steps end
    x_steps = sw["x"].cpu().numpy()[0].astype(np.float64)
    ctx.pso_init(sw)
    sw["x"].copy_(torch.tensor(x0[None]))
    ctx.pso_step(sw, ht.pso_params(w=0.0, c1=0.0, c2=0.0, mutate_every=0, refine_topk=K,
                                   refine_steps=S))
    x_chain = sw["x"].cpu().numpy()[0].astype(np.float64)
    ctx.close()
    assert np.all(np.abs(x_chain - x_steps) <= 1e-3 * eta)


def test_eval_counts_and_skipped_refinement_candidates():
    """The device evaluation counts: every evaluated particle once (forward or with
    gradients), in eager calls and graph replays; the candidates of refined particles that
    have stopped refining are not evaluated.  Particles placed out of view render nothing and
    have no collision term, so their gradient is zero and their refinement stops at once: a
    generation then evaluates the swarm (forward) and the K selected (with gradients) only."""
    torch, ctx, model, fr, sw, lo, hi = _setup(P=64)
    ctx.eval_counts(reset=True)
    ctx.pso_init(sw)
    x = sw["x"].clone()
    ctx.eval(x[0], sw["frame_slots"])
    ctx.eval_grad(x[0, :10], sw["frame_slots"])
    assert ctx.eval_counts(reset=True) == (64, 10)
    # refinement: K = 8, 2 steps; in view, every candidate of an active particle is evaluated
    p = ht.pso_params(mutate_every=0, refine_topk=8, refine_steps=2)
    ctx.pso_step(sw, p)
    f, g = ctx.eval_counts(reset=True)
    assert g >= 8 and f >= 64 and f + g <= 64 + 8 + 4 * 8 * 2
    # out of view (x far to the side, angles with kc = 0): gradients vanish, nothing proposed
    far = sw["x"].clone()
    far[0, :, 20] += 5000.0
    sw["x"].copy_(far)
    c_far = ctx.eval(far[0], sw["frame_slots"]).cpu().numpy()
    _, g_far = ctx.eval_grad(far[0], sw["frame_slots"])
    ctx.eval_counts(reset=True)
    kc_free = np.all(g_far.cpu().numpy() == 0.0, axis=1)
    assert kc_free.sum() >= 8
    ctx.pso_step(sw, p)
    torch.cuda.synchronize()
    # the 8 selected (lowest costs: nothing rendered, so E = D + lambda_k kc is lowest where
    # kc = 0) have zero gradients, stop at once and propose nothing
    assert ctx.eval_counts(reset=True) == (64, 8)
    assert np.array_equal(sw["cost"].cpu().numpy()[0], c_far)
    # graph replays count every replay
    ctx.reserve(64 * 4, fr["depth"].size)
    plain = ht.pso_params(mutate_every=0)
    ctx.pso_run_graph(sw, plain, 3)
    ctx.eval_counts(reset=True)
    for _ in range(2):
        ctx.pso_run_graph(sw, plain, 3)
    assert ctx.eval_counts(reset=True) == (2 * 3 * 64, 0)
    ctx.close()


def test_device_seed_replays_with_new_random_numbers():
    """A swarm whose Philox key is read from device memory: after one capture, rewriting the
    key makes the same cached graph replay the run of a swarm seeded with the new key (bit for
    bit), without a new capture."""
    torch, ctx, model, fr, sw, lo, hi = _setup(P=32)
    ctx.reserve(32 * 4, fr["depth"].size)
    dev = sw["x"].device
    slots = sw["frame_slots"]
    params = ht.pso_params()
    dsw = ctx.swarm(slots, 32, torch.tensor(lo), torch.tensor(hi), seed=5, device_seed=True)
    ctx.pso_run_graph(dsw, params, 4)
    for key in (9, 123456789):
        dsw["seed_dev"].fill_(key)
        ctx.pso_run_graph(dsw, params, 4)
        ref = ctx.swarm(slots, 32, torch.tensor(lo), torch.tensor(hi), seed=key)
        ctx.pso_init(ref)
        for _ in range(4):
            ctx.pso_step(ref, params)
        torch.cuda.synchronize()
        for k in ("x", "v", "pbest_x", "pbest_cost", "gbest_x", "gbest_cost"):
            assert torch.equal(dsw[k], ref[k]), (key, k)
    assert dev.type == "cuda"
    ctx.close()
