"""The gradient's finite-difference protocol on the 320x240 workload frame, stored by
tests/golden/make_fd_protocol.py from the oracle alone: on 32 seeded poses the FP64 analytic
gradient agrees with central differences (1e-3 rad / 1e-2 mm) of the masked smooth cost, and
the stored file is what the oracle computes now (one pose re-derived)."""
import os

import numpy as np
import pytest

from oracle import cost, grad

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fd_protocol_adjoint320x240.npz")
# central differences carry a truncation error of step^2 / 6 times the third derivative:
# at 1e-3 rad that is below 1e-4 of the gradient's largest component on these poses
FD_RTOL = 1e-4


@pytest.fixture(scope="module")
def golden():
    d = np.load(GOLDEN)
    masks = np.unpackbits(d["masks"], axis=-1)[..., :int(d["mask_shape"][-1])].astype(bool)
    return d, masks


def test_analytic_matches_central_differences_on_32_poses(golden):
    d, masks = golden
    g, g_fd = d["g_analytic"], d["g_fd"]
    assert g.shape == (32, 26) and masks.shape == (32, 240, 320)
    for i in range(32):
        scale = np.max(np.abs(g_fd[i]))
        assert scale > 0.0
        assert np.max(np.abs(g[i] - g_fd[i])) <= FD_RTOL * scale, i
    # enough smooth model pixels in every mask, and the ratios are >= 1 where defined
    assert np.all(d["mask_hit_pixels"] >= 500)
    c = d["cancellation"]
    assert np.all((c == 0.0) | (c >= 1.0 - 1e-12))


def test_stored_protocol_is_the_oracle_as_it_stands(golden):
    """Pose 0 recomputed: the same mask, analytic gradient and (three parameters') central
    differences as stored."""
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    import make_fd_protocol as mk
    d, masks = golden
    model, fr, poses = mk.setup()
    assert np.array_equal(poses, d["poses"])
    h = poses[0].astype(np.float64)
    E, parts = cost.objective(model, h, fr, return_parts=True)
    mask = grad.fd_protocol_mask(model, h, parts["render"], fr, mk.STEP_RAD, mk.STEP_MM)
    assert np.array_equal(mask, masks[0])
    _, g = grad.analytic_gradient(model, h, fr, pixel_mask=mask)
    assert np.allclose(g, d["g_analytic"][0], rtol=1e-12, atol=1e-15)
    dofs = [1, 20, 25]
    g_fd = grad.fd_gradient(model, h, fr, mask, parts["S_or"], step_rad=mk.STEP_RAD,
                            step_mm=mk.STEP_MM, dofs=dofs)
    assert np.allclose(g_fd[dofs], d["g_fd"][0][dofs], rtol=1e-9, atol=1e-12)
    # the per-pixel terms sum to the depth part of the gradient
    terms = grad.gradient_terms(model, h, fr, pixel_mask=mask)
    assert np.allclose(terms.sum(axis=(1, 2)) + cost.LAMBDA_K * cost.kc_grad(model, h), g,
                       rtol=1e-12, atol=1e-15)
