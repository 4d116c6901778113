"""MI355X (gfx950) implementation of the capacitance -> B_z path of
reconfigurable resonant loop arrays and its gradient.

The numerical work runs in ``libcosim.so`` (hand-written HIP kernels behind
the C ABI of ``include/cosim.h``); this package only marshals arguments.
PyTorch supplies device memory and streams.
"""
from ._lib import CosimError, load_library, library_path  # noqa: F401
from .api import (  # noqa: F401
    FP64, FP32, BF16X3, LOSS_MAG, LOSS_COMPLEX, LOSS_RATIO,
    SYS_BAD_INPUT, SYS_SINGULAR, SYS_NONFINITE, SYS_NEGATIVE_C,
    Geometry, Plan, CosimField, cosim_field, adam_step, loss_and_grad_many, ManyCall,
    capture_loss_and_grad_many,
    SParamPlan, sp_rc, sp_rc_backward, tanh_projection, clip_,
)
