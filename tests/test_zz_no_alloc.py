"""ht_eval_particles_noalloc (the evaluation for callers that cannot allocate: its workspace is
the library's fixed per-GPU scratch array) against ht_eval_particles, through the C ABI: two
calls in a row, the second smaller, bit-identical costs; the size limit; a call captured in a
HIP graph on a context that never reserved a workspace."""
import numpy as np
import pytest

import paper_2005_07068_amd as ht
from gpu_util import frame_for, make_ctx, particles_for, torch_cuda
from oracle import synth
from workload import WORKLOADS, make_hand_model, seed_sequence

pytestmark = pytest.mark.gpu


def test_noalloc_equals_eval_two_calls_second_smaller():
    torch = torch_cuda()
    dev = torch.device("cuda:0")
    cfg, model, fr = frame_for(4)                 # 640x480, two hands
    ctx = make_ctx(model, [fr])
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    for n, seed in ((1024, 51), (100, 52)):
        x = torch.tensor(particles_for(model, fr, n, seed=seed), device=dev)
        ref = ctx.eval(x, slots).cpu().numpy()
        got = ctx.eval_noalloc(x, slots).cpu().numpy()
        assert np.all(np.isfinite(ref))
        assert np.array_equal(got, ref), n
    ctx.close()


def test_noalloc_batched_frames_and_the_size_limit():
    """Uneven-ROI frames in one call (twice, the second with fewer frames), then a call beyond
    the scratch array is rejected with an error and enqueues nothing."""
    torch = torch_cuda()
    dev = torch.device("cuda:0")
    cfg = WORKLOADS[3]
    model = make_hand_model(seed_sequence(3, 10_000))
    frames = [synth.make_frame(model, cfg, f) for f in range(6)]
    ctx = make_ctx(model, frames)
    for F, P in ((6, 64), (3, 16)):
        poses = np.stack([particles_for(model, frames[f], P, seed=60 + f) for f in range(F)])
        x = torch.tensor(poses, device=dev)
        slots = torch.arange(F, dtype=torch.int32, device=dev)
        ref = ctx.eval(x, slots).cpu().numpy()
        got = ctx.eval_noalloc(x, slots).cpu().numpy()
        assert np.array_equal(got, ref), (F, P)
    big = torch.zeros((1, 60_000, model["n_dof"]), device=dev)
    out = torch.full((1, 60_000), 7.0, device=dev)
    with pytest.raises(ht.HandtrackError, match="scratch"):
        ctx.eval_noalloc(big, torch.zeros(1, dtype=torch.int32, device=dev), out)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
    ctx.close()


def test_noalloc_under_graph_capture_without_reserve():
    """A fresh context (no ht_reserve, so ht_eval_particles would have to grow its workspace,
    which capture refuses) captures the no-allocation call; every replay, with eager work in
    between, equals the eager result."""
    torch = torch_cuda()
    dev = torch.device("cuda:0")
    cfg, model, fr = frame_for(1)
    ctx = make_ctx(model, [fr])
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    x = torch.tensor(particles_for(model, fr, 64, seed=70), device=dev)
    cost = torch.empty((1, 64), device=dev)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.eval_noalloc(x[None], slots, cost)
    eager = ctx.eval(x, slots).cpu().numpy()
    for _ in range(3):
        cost.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(cost.cpu().numpy()[0], eager)
        ctx.eval(x[:8], slots)                   # eager work between the replays
    ctx.close()
