"""The synthetic workloads and their seed / camera recipes (data only).

Camera: pinhole with fx = fy = f, principal point at the ROI centre ((W-1)/2, (H-1)/2), so
pixel ray directions (u - cx, v - cy, f) are exact binary fractions; f = 2.25 * min(W, H)
for hand-centred ROIs and 575 for the full 640x480 frame (a Kinect-like focal length; the
paper does not give its intrinsics).  The background plane sits at 1500 mm.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 2005_07068
BACKGROUND_MM = 1500.0


def seed_sequence(config_idx: int, *extra: int) -> np.random.SeedSequence:
    return np.random.SeedSequence([ROOT_SEED, config_idx, *extra])


def camera_for_roi(W: int, H: int, full_frame: bool = False) -> tuple[float, float, float, float]:
    f = 575.0 if full_frame else 2.25 * min(W, H)
    return (f, f, (W - 1) / 2.0, (H - 1) / 2.0)


@dataclass(frozen=True)
class WorkloadConfig:
    idx: int
    name: str
    n_frames: int
    roi: tuple[int, int] | None          # (W, H); None = drawn per frame
    roi_range: tuple[int, int] = (48, 192)
    n_hands: int = 1
    n_particles: int = 16
    n_generations: int = 1
    full_frame: bool = False
    w: float = 0.72
    c1: float = 2.05
    c2: float = 2.05
    refine_topk: int = 0
    refine_steps: int = 0
    init_angle_deg: float = 10.0
    init_trans_mm: float = 20.0
    hand_x_mm: tuple[float, ...] = field(default=(0.0,))
    primitive_set: str = "cylinders"     # or "paper" (section II.A: cones, elliptic palm)
    # a tracked sequence (frames are consecutive video frames of one moving hand) instead of
    # independent frames; per-frame random-walk steps of the true pose
    sequence: bool = False
    seq_step_deg: float = 3.0
    seq_step_mm: float = 4.0
    # observation noise model
    noise_sigma_mm: float = 2.0
    dropout_p: float = 0.05
    skin_flip_p: float = 0.02

    def frame_roi(self, frame: int) -> tuple[int, int]:
        if self.roi is not None:
            return self.roi
        rng = np.random.default_rng(seed_sequence(self.idx, 1_000_000 + frame))
        lo, hi = self.roi_range
        W, H = rng.integers(lo, hi + 1, size=2)
        return int(W), int(H)


WORKLOADS = {
    0: WorkloadConfig(0, "fwd64", 1, (64, 64), n_particles=16, n_generations=1),
    1: WorkloadConfig(1, "pso128", 1, (128, 128), n_particles=64, n_generations=30),
    2: WorkloadConfig(2, "adjoint320x240", 1, (320, 240), n_particles=256, n_generations=1),
    3: WorkloadConfig(3, "batched64", 64, None, n_particles=64, n_generations=30),
    4: WorkloadConfig(4, "hybrid640x480", 1, (640, 480), n_hands=2, n_particles=1024,
                      n_generations=20, full_frame=True, refine_topk=32, refine_steps=3,
                      hand_x_mm=(-120.0, 120.0)),
    # a 30-frame tracked sequence (15 fps-like motion), one hand at 320x240, with the paper's
    # swarm constants (c1 = 2.8, c2 = 1.3 and the constriction factor)
    6: WorkloadConfig(6, "track320x240", 30, (320, 240), n_particles=64, n_generations=30,
                      sequence=True, w=0.7298437881, c1=2.8, c2=1.3),
    # workload 4 with the paper's own primitive set (38 per hand)
    5: WorkloadConfig(5, "hybrid640x480_paper", 1, (640, 480), n_hands=2, n_particles=1024,
                      n_generations=20, full_frame=True, refine_topk=32, refine_steps=3,
                      hand_x_mm=(-120.0, 120.0), primitive_set="paper"),
}
