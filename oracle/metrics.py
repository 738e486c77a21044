"""Error metrics used to compare a fit or a reconstruction with the oracle.  TEST INFRASTRUCTURE ONLY.

Several results are equally correct (the order of the eigenvalues, the scale of
each eigenvector), so comparisons use only what is unique:
  * eigenvalue sets are matched by an optimal assignment on |lambda_a - lambda_b|;
  * modes are compared through phi_i * b_i, which does not depend on the
    eigenvector scale;
  * fields are compared frame by frame.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import linear_sum_assignment


def match_eigs(la, lb):
    """Index arrays (ia, ib) pairing la[ia] with lb[ib] at minimum total |difference|."""
    la = np.asarray(la, dtype=np.complex128)
    lb = np.asarray(lb, dtype=np.complex128)
    cost = np.abs(la[:, None] - lb[None, :])
    return linear_sum_assignment(cost)


def eig_errors(la, lb, weights=None):
    """Max-relative, norm-relative and weighted-relative distance of two eigenvalue sets.

    weights (aligned with lb) default to 1; the weighted error is
    sum w_i |dlambda_i| / sum w_i |lambda_i|.
    """
    ia, ib = match_eigs(la, lb)
    d = np.abs(np.asarray(la)[ia] - np.asarray(lb)[ib])
    ref = np.abs(np.asarray(lb)[ib])
    w = np.ones_like(ref) if weights is None else np.asarray(weights)[ib]
    return {
        "max_rel": float(np.max(d / np.maximum(ref, 1e-300))),
        "norm_rel": float(np.linalg.norm(d) / np.linalg.norm(ref)),
        "weighted_rel": float(np.sum(w * d) / np.sum(w * ref)),
    }


def amplitude_weights(phi, b):
    """w_i = |b_i| * ||phi_i||."""
    return np.abs(np.asarray(b)) * np.linalg.norm(np.asarray(phi), axis=0)


def field_errors(U, Uref):
    """Per-frame ||u - u_ref|| / ||u_ref||: max over frames, and the aggregate Frobenius ratio."""
    U = np.asarray(U, dtype=np.float64)
    Uref = np.asarray(Uref, dtype=np.float64)
    num = np.linalg.norm(U - Uref, axis=0)
    den = np.linalg.norm(Uref, axis=0)
    return {
        "max_frame": float(np.max(num / np.maximum(den, 1e-300))),
        "fro": float(np.linalg.norm(U - Uref) / np.linalg.norm(Uref)),
    }


def complex_modes_from_folded(phi_f, kind):
    """Complex modes from the real folded storage of a real-data DMD model.

    kind[i] = 0: real mode phi_i = phi_f[:, i];  kind[i] = 1 and kind[i+1] = 2:
    a conjugate pair phi_i = phi_f[:, i] + 1j phi_f[:, i+1], phi_{i+1} = conj(phi_i).
    This is a pure storage convention (the one LAPACK uses for real eigenvectors).
    """
    phi_f = np.asarray(phi_f, dtype=np.float64)
    r = len(kind)
    out = np.zeros((phi_f.shape[0], r), dtype=np.complex128)
    i = 0
    while i < r:
        if kind[i] == 0:
            out[:, i] = phi_f[:, i]
            i += 1
        elif kind[i] == 1:
            out[:, i] = phi_f[:, i] + 1j * phi_f[:, i + 1]
            out[:, i + 1] = phi_f[:, i] - 1j * phi_f[:, i + 1]
            i += 2
        else:
            raise ValueError(f"bad mode kind sequence at {i}: {list(kind)}")
    return out
