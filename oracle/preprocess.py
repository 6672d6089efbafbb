"""Observation preprocessing (section II.B): from an RGB-D frame to O = (O_s, O_d).

The paper extracts the hand with skin-colour detection and depth segmentation and names no
method; this module fixes one (a reading), in exact integer arithmetic so that any
implementation can match it bit for bit:

  skin colour   YCbCr chroma of ITU-R BT.601 in the 8-bit fixed-point form
                  Cb = 128 + ((-43 R - 85 G + 128 B + 128) >> 8)
                  Cr = 128 + ((128 R - 107 G - 21 B + 128) >> 8)
                (">>" an arithmetic shift, i.e. floor division by 256) and the skin box
                cb_lo <= Cb <= cb_hi, cr_lo <= Cr <= cr_hi (default 77..127 and 133..173, the
                Chai-Ngan box);
  depth band    z0 = the smallest defined depth (> 0) among skin pixels; a pixel belongs to
                the hand's depth band when z0 <= depth <= z0 + band_mm (default 150 mm);
  output        O_s = skin and in the band; O_d = the depth inside the band, 0 where the
                depth is undefined, and the background plane depth B elsewhere (segmented
                away = background, which is what the model renders at misses).  With no skin
                pixel of defined depth, O_s = 0 everywhere and every defined depth becomes B.
"""
from __future__ import annotations

import numpy as np

SKIN_BOX = (77, 127, 133, 173)      # cb_lo, cb_hi, cr_lo, cr_hi
BAND_MM = 150


def chroma(rgb):
    """(Cb, Cr) int arrays of an [H, W, 3] uint8 image."""
    r, g, b = (rgb[..., i].astype(np.int64) for i in range(3))
    cb = 128 + ((-43 * r - 85 * g + 128 * b + 128) >> 8)
    cr = 128 + ((128 * r - 107 * g - 21 * b + 128) >> 8)
    return cb, cr


def skin_mask(rgb, box=SKIN_BOX):
    cb, cr = chroma(rgb)
    cb_lo, cb_hi, cr_lo, cr_hi = box
    return (cb >= cb_lo) & (cb <= cb_hi) & (cr >= cr_lo) & (cr <= cr_hi)


def preprocess(rgb, depth, bg_mm, box=SKIN_BOX, band_mm=BAND_MM):
    """(O_d uint16 [H, W], O_s uint8 [H, W], z0 or None) of an RGB-D frame."""
    depth = np.asarray(depth)
    skin = skin_mask(rgb, box)
    defined = depth > 0
    cand = depth[skin & defined]
    if cand.size == 0:
        o_d = np.where(defined, int(bg_mm), 0).astype(np.uint16)
        return o_d, np.zeros(depth.shape, np.uint8), None
    z0 = int(cand.min())
    band = defined & (depth >= z0) & (depth <= z0 + band_mm)
    o_d = np.where(band, depth, np.where(defined, int(bg_mm), 0)).astype(np.uint16)
    o_s = (skin & band).astype(np.uint8)
    return o_d, o_s, z0
