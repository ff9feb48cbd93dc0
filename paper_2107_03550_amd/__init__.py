"""MI355X (gfx950) spectral BIEM hot path for mildly non-planar faults.

The compute path is the C ABI of ``lib/libsbiem.so`` (declared in
``include/sbiem.h``); this package is a thin ctypes binding with the same
names.  Importing it loads the library and raises ``ImportError`` if it has
not been built (``python -m paper_2107_03550_amd.build``): there is no other
implementation to fall back to.
"""

from ._lib import (  # noqa: F401
    SBIEM_FP64, SBIEM_FP32CONV, SBIEM_THETA_PAPER, SBIEM_THETA_EXP, SBIEM_RULE_MIDPOINT,
    SBIEM_RULE_INTERVAL, ADAPT_OUTCOMES, kernel_primitive_eval, slip_scaling,
    SbiemError, Plan, Batch, lib, lib_path, kernel_eval, abi_version,
    set_torch_allocator, set_default_allocator, EXPORTED_NAMES, closure_train_noalloc,
    CLOSURE_TRAIN_MAX_BATCH, CLOSURE_PARAMS, closure_eval, ClosureTrainer,
)
