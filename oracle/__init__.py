"""CPU FP64 oracle for the hand-tracking hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, pixel-by-pixel (vectorised over pixels, one primitive at a time) NumPy
implementation of what the paper defines: forward kinematics of the 26-DOF hand (Eq. 1-3,
section II.A), the depth image of the hypothesis (section III.A), the discrepancy D (Eq. 4),
the collision term kc and the objective E (Eq. 5), the particle-swarm update (Eq. 6-7 with
the mutation of section III.B), plus the analytic gradient used to check the adjoint kernel
and a central finite-difference gradient that checks the analytic one.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may import
this package.  It shares no code with the HIP library; the only common inputs are the seeded
tables of the ``workload`` package.
"""
from . import fk, raycast, cost, grad, philox, pso, synth, flops  # noqa: F401
