"""Seeded synthetic inputs shared by the HIP library's callers and by the CPU oracle.

Everything in this package is *input data*: the hand-model tables (kinematic tree,
primitive list, joint limits, collision pairs), the camera recipe and raw uniform draws.
It holds no kinematics, no ray casting and no cost arithmetic, so that the product path and
the oracle can both consume the same inputs without sharing any of the method's code.
"""
from .handmodel import (  # noqa: F401
    DOF_PER_HAND, SEG_PER_HAND, PRIM_PER_HAND, PRIM_PER_HAND_PAPER, SPHERE, CYLINDER,
    ELLIPSOID, CONE, ECYLINDER, make_hand_model, finger_dof, WRIST_DOF,
)
from .configs import WORKLOADS, WorkloadConfig, camera_for_roi, seed_sequence  # noqa: F401
