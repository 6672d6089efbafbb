"""Pins of the algorithmic work counts behind the roofline figures: fragment counts against
the closed-form hit set of a sphere, the per-unit operation counts, and the hit-tile pixel
count against a hand-made mask."""
import numpy as np

from oracle import flops, raycast


def test_per_unit_counts():
    assert flops.F_PRIM == {0: 13, 1: 60, 2: 35, 3: 70, 4: 66}
    assert flops.F_PIXEL == 10


def test_sphere_fragments_and_flops_closed_form():
    """One sphere: its fragments are the pixels whose ray passes within r of the centre
    (cross-product distance), so W = 13 * that count + 10 * W * H."""
    W, H = 48, 40
    cam = (60.0, 60.0, (W - 1) / 2, (H - 1) / 2)
    c, r = np.array([13.0, -7.0, 420.0]), 21.0
    prim = {"type": raycast.SPHERE, "p": c, "R": np.eye(3), "size": np.array([r, 0.0, 0.0])}
    res = raycast.render_primitives([prim], W, H, cam, 1500.0)
    d = raycast.pixel_directions(W, H, cam)
    dh = d / np.linalg.norm(d, axis=-1, keepdims=True)
    n_cov = int((np.linalg.norm(np.cross(dh, c), axis=-1) <= r).sum())
    assert 0 < n_cov < W * H
    w = flops.work_counts(res, [raycast.SPHERE])
    assert w["cov_per_type"].tolist() == [n_cov, 0, 0, 0, 0]
    assert w["pixels"] == W * H
    assert flops.eval_flops(res, [raycast.SPHERE]) == 13 * n_cov + 10 * W * H


def test_hit_tile_pixels_hand_made_mask():
    """A 20 x 13 image (tiles of 8: columns 0-7, 8-15, 16-19; rows 0-7, 8-12): hits in the
    first tile, in the ragged corner tile (4 x 5 pixels) and two in the middle-bottom tile
    (8 x 5) count 64 + 20 + 40 pixels."""
    hit = np.zeros((13, 20), bool)
    hit[0, 0] = hit[3, 5] = True
    hit[12, 19] = True
    hit[9, 9] = hit[11, 14] = True
    assert flops.hit_tile_pixels(hit) == 64 + 20 + 40
    assert flops.hit_tile_pixels(np.zeros((13, 20), bool)) == 0
    assert flops.hit_tile_pixels(np.ones((13, 20), bool)) == 13 * 20
