"""MI355X (gfx950) implementation of Iterative Charted Refinement (ICR).

The library libicr.so (HIP kernels behind the C ABI in include/icr.h) does all
the work; this package binds it with ctypes and wraps it for PyTorch autograd.
"""

from .icr import (ICRError, IcrConfig, Plan, icr_adjoint, icr_adjoint_level,  # noqa: F401
                  icr_build_matrices, icr_cg_metric, icr_cg_workspace_bytes, icr_forward,
                  icr_forward_level,
                  icr_last_error, icr_metric_apply, icr_plan_copy_level0,
                  icr_plan_copy_refinement, icr_plan_destroy, icr_plan_set_level0,
                  icr_plan_set_refinement, icr_plan_get_info, icr_version,
                  load_library, make_config, workspace_for)


def __getattr__(name):
    if name in ("ICRFunction", "icr_sample"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
