"""GPU adjoint against the FP64 analytic gradient of the finite-difference protocol on the
320x240 workload frame (32 seeded poses, each with its protocol mask as the pixel mask),
stored by tests/golden/make_fd_protocol.py from the oracle alone."""
import os

import numpy as np
import pytest

from gpu_util import frame_for, make_ctx, torch_cuda

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fd_protocol_adjoint320x240.npz")


def test_adjoint_matches_the_fd_protocol_gradients():
    torch = torch_cuda()
    d = np.load(GOLDEN)
    masks = np.unpackbits(d["masks"], axis=-1)[..., :int(d["mask_shape"][-1])]
    cfg, model, fr = frame_for(2)
    ctx = make_ctx(model, [fr])
    dev = torch.device("cuda:0")
    slots = torch.zeros(1, dtype=torch.int32, device=dev)
    worst = 0.0
    for i, pose in enumerate(d["poses"]):
        m = torch.tensor(masks[i], dtype=torch.uint8, device=dev)
        c, g = ctx.eval_grad(torch.tensor(pose[None], device=dev), slots, pixel_mask=m)
        g = g.cpu().numpy()[0].astype(np.float64)
        g_ref = d["g_analytic"][i]
        scale = np.max(np.abs(g_ref))
        err = np.max(np.abs(g - g_ref))
        worst = max(worst, err / scale)
        assert err <= 1e-5 * scale, (i, err / scale)
        # the cost beside it: the oracle's (stored) up to pixels decided within the margin,
        # which the cost parity tests resolve (one such pixel moves E by about 1e-4)
        assert abs(float(c.cpu()[0]) - d["cost"][i]) <= 1e-3 * d["cost"][i], i
    ctx.close()
    c = d["cancellation"]
    print(f"fd protocol: 32 poses, worst relative gradient difference {worst:.2e}; "
          f"cancellation ratio median {np.median(c[c > 0]):.2f}, max {c.max():.1f}")
