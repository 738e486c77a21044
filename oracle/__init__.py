"""FP64 CPU oracle for the DMD hot path.  TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The HIP library never links it and the product path never calls
it.  See oracle/dmd.py for the method and the readings it takes of the paper.
"""
from .dmd import (LOW_FREQ_CUT, DMDFit, block_average_matrix, canonical_order, cluster_edit, edit_modes,
                  fit_exact, fit_optdmd, fit_randomized, frequency_clusters, integrate, kkt_project,
                  koopman_least_squares, loss, loss_grad, powers, project,
                  range_finder, reconstruct, reverse, rollout, split_snapshots, thin_svd, upsample_evolve,
                  vandermonde, varpro, varpro_normal_equations, varpro_residual, varpro_trial,
                  thin_svd_qr_route)
from .metrics import (amplitude_weights, complex_modes_from_folded, eig_errors,
                      field_errors, match_eigs)

__all__ = [
    "LOW_FREQ_CUT", "DMDFit", "canonical_order", "cluster_edit", "edit_modes",
    "frequency_clusters", "reverse", "rollout", "block_average_matrix", "kkt_project", "upsample_evolve",
    "fit_optdmd", "vandermonde", "varpro", "varpro_normal_equations", "varpro_residual", "varpro_trial", "fit_exact", "fit_randomized", "integrate",
    "koopman_least_squares", "loss", "loss_grad", "powers", "project",
    "range_finder", "reconstruct", "split_snapshots", "thin_svd",
    "thin_svd_qr_route", "amplitude_weights", "complex_modes_from_folded",
    "eig_errors", "field_errors", "match_eigs",
]
