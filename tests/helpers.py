"""Shared test helpers: oracle fits in the library's folded storage, error metrics."""
import functools

import numpy as np


def folded_from_complex(phi, lam, b, tol=1e-9):
    """Folded real storage of a conjugate-paired complex model (pairs adjacent, Im > 0 first).

    Returns (phi_folded N x r, lam, b, kind).  Raises if the pair structure is broken.
    """
    phi = np.asarray(phi)
    lam = np.asarray(lam, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    r = lam.size
    folded = np.zeros((phi.shape[0], r))
    kind = np.zeros(r, dtype=np.int32)
    i = 0
    while i < r:
        if abs(lam[i].imag) <= tol * max(1.0, abs(lam[i])):
            folded[:, i] = phi[:, i].real
            kind[i] = 0
            i += 1
            continue
        assert lam[i].imag > 0 and i + 1 < r, "pair must start with Im > 0"
        assert abs(lam[i + 1] - np.conj(lam[i])) <= tol * abs(lam[i]), "conjugate partner missing"
        folded[:, i] = phi[:, i].real
        folded[:, i + 1] = phi[:, i].imag
        kind[i], kind[i + 1] = 1, 2
        i += 2
    return folded, lam, b, kind


def model_from_oracle(fit, dtype, device="cuda", dt=1.0):
    """A library Model holding an oracle fit (folded modes in the given torch dtype)."""
    import torch
    from paper_2502_05339_amd import Model
    folded, lam, b, kind = folded_from_complex(fit.phi, fit.lam, fit.b)
    n, r = folded.shape
    m = Model.empty(n, r, dtype, device, dt)
    m.phi[:, :r].copy_(torch.from_numpy(folded).to(dtype))
    m.lam.copy_(torch.from_numpy(lam))
    m.b.copy_(torch.from_numpy(b))
    m.kind.copy_(torch.from_numpy(kind))
    return m


def rel_fro(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_frame_rel(U, Uref):
    """max over frames (rows of (K, N) arrays) of ||u - u_ref|| / ||u_ref||."""
    U = np.asarray(U, dtype=np.float64)
    Uref = np.asarray(Uref, dtype=np.float64)
    num = np.linalg.norm(U - Uref, axis=1)
    den = np.linalg.norm(Uref, axis=1)
    return float(np.max(num / np.maximum(den, 1e-300)))


@functools.lru_cache(maxsize=1)
def rank150_fit():
    """Oracle exact fit of rank 150 (2 x 64 x 64 grid, 160 snapshot pairs of a rank-180
    signal with persistent modes): a model whose FP64 products against one column span
    more than 128 columns.  Its folded modes have condition number about 8."""
    import oracle
    import synth
    cfg = synth.Config("rank150", (2, 64, 64), 161, 90, 0.99, 1e-6, 618, r=150, p=0, q=0, jitter=True, dtype="f64")
    g = synth.generate(cfg)
    return cfg, g, oracle.fit_exact(g.Z, cfg.r)
