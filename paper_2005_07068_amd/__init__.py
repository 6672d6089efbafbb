"""MI355X (gfx950) hot path of model-based 26-DOF hand tracking with particle swarms.

The compute lives in ``libhandtrack.so`` (HIP kernels behind the C ABI of
``include/handtrack.h``); this package is its thin Python binding plus a
``torch.autograd.Function`` around the adjoint kernel.
"""
from .binding import (  # noqa: F401
    HT_DEVERR_UNSET_SLOT, Context, HandtrackError, load_library, pso_params, header_functions,
)
from .autograd import HandCost  # noqa: F401
