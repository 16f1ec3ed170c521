"""lmmew: list-mode multi-energy-window OSEM SPECT on MI355X (arXiv 2305.17111).

The reconstruction runs in the HIP library ``liblmmew.so`` (C ABI in
``include/lmmew.h``).  This package is a thin binding with the same names: it
marshals torch tensors (device memory) and the current HIP stream into the C
calls.  There is no CPU fallback: importing the binding raises if the library
is missing.
"""
from .binding import (  # noqa: F401
    LmmewError,
    calibrate,
    Context,
    Plan,
    Mlp,
    events_to_device,
    line_mask,
    plan_maps,
    roi_metrics,
    system_from_params,
    library_path,
)
