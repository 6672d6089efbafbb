"""Pins of the oracle's observation preprocessing (section II.B: skin colour and depth
segmentation) against the BT.601 chroma formula it approximates and hand-made images."""
import numpy as np

from oracle import preprocess as pp


def test_integer_chroma_is_bt601_within_one_level():
    rng = np.random.default_rng(0)
    rgb = rng.integers(0, 256, size=(200, 300, 3)).astype(np.uint8)
    cb, cr = pp.chroma(rgb)
    r, g, b = (rgb[..., i].astype(np.float64) for i in range(3))
    cb_f = 128.0 - 0.168736 * r - 0.331264 * g + 0.5 * b
    cr_f = 128.0 + 0.5 * r - 0.418688 * g - 0.081312 * b
    assert np.max(np.abs(cb - cb_f)) <= 1.0 and np.max(np.abs(cr - cr_f)) <= 1.0
    # greys have neutral chroma exactly
    grey = np.repeat(np.arange(256, dtype=np.uint8)[:, None, None], 3, axis=2)
    cbg, crg = pp.chroma(grey)
    assert np.all(cbg == 128) and np.all(crg == 128)


def test_segmentation_rule_on_a_hand_made_frame():
    skin = np.array([205, 150, 125], np.uint8)       # Cb 106, Cr 158: inside the box
    blue = np.array([70, 90, 140], np.uint8)         # Cb 156, Cr 114: outside
    rgb = np.empty((3, 4, 3), np.uint8)
    rgb[:] = blue
    rgb[0, 0] = rgb[0, 1] = rgb[1, 1] = rgb[2, 3] = skin
    depth = np.array([[600, 0, 640, 900],
                      [700, 651, 749, 750],
                      [599, 760, 0, 1200]], np.uint16)
    o_d, o_s, z0 = pp.preprocess(rgb, depth, 1500, band_mm=150)
    # skin pixels with a defined depth: 600, 651, 1200 -> z0 = 600, band [600, 750]
    assert z0 == 600
    assert o_d.tolist() == [[600, 0, 640, 1500], [700, 651, 749, 750], [1500, 1500, 0, 1500]]
    assert o_s.tolist() == [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 0]]


def test_no_skin_means_background_everywhere():
    rgb = np.zeros((5, 6, 3), np.uint8)
    rgb[:] = (70, 90, 140)
    depth = np.arange(30, dtype=np.uint16).reshape(5, 6)
    o_d, o_s, z0 = pp.preprocess(rgb, depth, 1500)
    assert z0 is None and not o_s.any()
    assert np.array_equal(o_d, np.where(depth > 0, 1500, 0))
