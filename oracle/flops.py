"""Algorithmic floating-point work of one hypothesis evaluation (for roofline figures).

W = sum_k cov_k * f_k + N * f_px, where cov_k is the number of pixels whose ray hits
primitive k (the fragments a rasteriser would shade), f_k the operation count of the
oracle's per-ray intersection formulas for that primitive type, N the ROI pixels and f_px
the per-pixel ray set-up plus cost terms of Eq. 4.  Each add, multiply, compare, min,
square root or division counts as one operation; dense ray-primitive tests that an
implementation may perform and discard are not counted.

  sphere     16  (d.w 5, discriminant 3, test 1, sqrt 1, root 2, t > 0 1, nearest-depth 3)
  ellipsoid  35  (map of d to the unit frame 15, e.e 5, e.w 5, discriminant 3, test 1,
                  sqrt 1, root 2, nearest-depth 3)
  cylinder   68  (axial part of d 5, perpendicular part 6, side quadratic 13, two side
                  roots 4, their axial slabs 4 + 4 tests, two caps 2 x 14, nearest of four
                  candidates 3, nearest-depth 1)
  cone       78  (as the cylinder, plus the radius at the reference point 2, the k terms of
                  the side quadratic 5, two cap radii 2, and the quadratic's A -> 0 safe
                  roots 1)
  elliptic cylinder  74  (map of d to the unit-radius frame 6, then the cylinder's 68)
  pixel      19  (ray direction 4, d.d 5, |o_d - r_d| 2, clamp 1, two depth tests 2, the
                  three Boolean terms 3, three accumulations 3, minus the shared 1)
"""
from __future__ import annotations

import numpy as np

F_PRIM = {0: 16, 1: 68, 2: 35, 3: 78, 4: 74}
F_PIXEL = 19


def eval_flops(render_res, prim_types) -> int:
    cov = render_res["prim_hit"].reshape(len(prim_types), -1).sum(axis=1)
    N = render_res["depth"].size
    return int(sum(int(c) * F_PRIM[int(t)] for c, t in zip(cov, prim_types)) + N * F_PIXEL)
