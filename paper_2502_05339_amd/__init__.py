"""MI355X-native DMD hot path (fit, batched reconstruction, adjoint) over a C ABI.

The compute runs in libdmdmi.so (hand-written HIP kernels for gfx950); this
package is the thin Python binding.  See include/dmdmi.h for the C ABI.
"""
from ._lib import DMDError, lib, status_string
from .api import (BatchedFit, DMDLoss, DMDLossStats, Model, PreparedReconstruction, RefitStats, autotune_fit,
                  autotune_reconstruct, edit_modes, fit, fit_opts, integrate, loss_grad, lowres_project, project,
                  reconstruct, refit, reverse, rollout, status_word, upsample)

__all__ = [
    "DMDError", "lib", "status_string", "BatchedFit", "DMDLoss", "DMDLossStats", "Model", "PreparedReconstruction",
    "RefitStats",
    "autotune_fit", "autotune_reconstruct", "edit_modes", "fit",
    "fit_opts", "integrate", "loss_grad", "project", "reconstruct", "refit", "reverse", "rollout", "lowres_project", "upsample",
    "status_word",
]
