"""Seeded synthetic snapshot generators shared by the tests, the benchmark and smoke().

The paper's training data are velocity fields from full-space fluid solvers on
staggered grids (Sec. 4.1, "Constructing Training Data"; Sec. 5, Table
"experiment_setup": 2D 256x512 .. 1024x512, 3D 128x128x256, 300-500 frames,
r = 2..150).  None of those datasets is available, so every workload here is a
synthetic linear system with the same shapes: snapshots

    z_j = Re( sum_i phi_i * s_i(j) ) + sigma * eps_j,   s_i(j+1) = lambda_i * s_i(j),
    s_i(0) = b_i,

i.e. the state of a known diagonal linear recurrence seen through a set of
complex spatial modes (the setting of Sec. 3.1, eqs. reduced_koopman and
reduced_koopman_simulation, with the ground truth known in closed form).

This module only *draws* inputs.  It holds none of the DMD method's arithmetic
(no SVD, no eigen-decomposition, no powers by exp/log, no projection): the
snapshots are produced by stepping the recurrence one frame at a time.  Random
numbers the method itself consumes (the Gaussian sketch of the randomized SVD,
Sec. 4.3) are drawn here as well and passed to both the oracle and the GPU path
as explicit inputs.

Random stream: numpy PCG64 (``np.random.default_rng(seed)``); draw order is
modes, |lambda|, arg(lambda), b, then the noise column by column.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Config", "CONFIGS", "config", "draw_eigs", "draw_amplitudes",
    "orthonormal_modes", "smooth_modes", "snapshots", "sketch", "generate",
    "Scene", "c5b_scenes", "synthetic_model",
]


@dataclasses.dataclass(frozen=True)
class Config:
    """One synthetic workload.

    n_grid: grid shape (components first), N = prod(n_grid).
    m: number of snapshots (columns of Z); X and X' have m-1 columns.
    nc: number of complex terms in the generating sum (rank 2*nc once Re() is taken).
    lam_lo: |lambda| ~ U[lam_lo, 1].
    arg: (lo, hi) of arg(lambda) ~ U[lo, hi] in radians per frame.
    jitter: draw arg(lambda) on a jittered grid instead (well-conditioned variant).
    sigma: additive Gaussian noise level.
    modes: "orthonormal" (QR of a complex Gaussian matrix) or "smooth"
        (complex white noise, periodic Gaussian filter of width 4 cells).
    r, p, q: DMD rank, sketch oversampling, power iterations.
    K: number of reconstructed frames (k = 0..K-1 unless ks is given).
    dtype: element type handed to the fit ("f64" or "f32").
    """

    name: str
    n_grid: tuple
    m: int
    nc: int
    lam_lo: float
    sigma: float
    seed: int
    r: int
    p: int = 10
    q: int = 2
    K: int = 100
    arg: tuple = (0.01, 0.5)
    jitter: bool = False
    modes: str = "orthonormal"
    dtype: str = "f32"

    @property
    def N(self) -> int:
        return int(np.prod(self.n_grid))

    @property
    def l(self) -> int:
        return self.r + self.p


CONFIGS = {
    # Plain FP64 DMD, exact SVD: 2D 64x64 velocity grid, 8 conjugate pairs.
    "c1": Config("c1", (2, 64, 64), 65, 8, 0.97, 1e-8, 101, r=16, p=0, q=0,
                 K=100, dtype="f64"),
    # Closed-form variant of c1: noise free, jittered-grid frequencies.
    "c1-cf": Config("c1-cf", (2, 64, 64), 65, 8, 0.97, 0.0, 102, r=16, p=0,
                    q=0, K=100, jitter=True, dtype="f64"),
    # Randomized-SVD DMD on a 2D 256x256x2 grid, rank 150 system.
    "c2": Config("c2", (2, 256, 256), 200, 75, 0.95, 1e-4, 201, r=150, p=10,
                 q=2, K=1000),
    # Well-posed variant of c2 (signal far above noise, separated frequencies).
    "c2-wp": Config("c2-wp", (2, 256, 256), 200, 75, 0.95, 1e-6, 202, r=150,
                    p=10, q=2, K=1000, jitter=True),
    # 3D plume-shaped fit, 3x128^3 smooth modes, rank-200 system, r=150.
    "c3": Config("c3", (3, 128, 128, 128), 300, 100, 0.98, 1e-3, 301, r=150,
                 p=10, q=2, K=300, modes="smooth"),
    # Adjoint refit: rank-40 system with strong noise.
    "c4": Config("c4", (2, 256, 256), 200, 20, 0.95, 1e-2, 401, r=40, p=10,
                 q=2, K=200),
    # Batched reconstruction of a synthetic 3D model: 75 smooth conjugate pairs.
    "c5a": Config("c5a", (3, 192, 96, 96), 0, 75, 0.98, 0.0, 501, r=150, p=0,
                  q=0, K=4096, modes="smooth"),
}


def config(name: str, **overrides) -> Config:
    """Return a named configuration, optionally with fields replaced."""
    return dataclasses.replace(CONFIGS[name], **overrides)


def draw_eigs(rng, nc, lam_lo, arg=(0.01, 0.5), jitter=False):
    """|lambda| ~ U[lam_lo, 1]; arg ~ U[arg] or a jittered grid on (0.05, pi-0.05)."""
    mod = rng.uniform(lam_lo, 1.0, nc)
    if jitter:
        lo = 0.05
        h = (math.pi - 0.1) / nc
        u = rng.uniform(-0.25, 0.25, nc)
        ang = lo + h * (np.arange(nc) + 0.5 + u)
    else:
        ang = rng.uniform(arg[0], arg[1], nc)
    return mod * np.exp(1j * ang)


def draw_amplitudes(rng, nc):
    """b ~ CN(0, 1)."""
    return (rng.standard_normal(nc) + 1j * rng.standard_normal(nc)) / math.sqrt(2.0)


def orthonormal_modes(rng, N, nc):
    """Random complex N x nc matrix with orthonormal columns (QR of a complex Gaussian)."""
    g = rng.standard_normal((N, nc)) + 1j * rng.standard_normal((N, nc))
    q, _ = np.linalg.qr(g)
    return q


def _gauss_transfer(n, sigma):
    """Fourier multiplier of a periodic Gaussian blur of width sigma cells on n points."""
    f = np.fft.fftfreq(n)
    return np.exp(-2.0 * (math.pi * sigma * f) ** 2)


def smooth_modes(rng, n_grid, nc, sigma_cells=4.0, dtype=np.complex64, progress=None):
    """Spatially smooth complex modes on a component-major grid.

    Each component of each mode is complex white noise on the grid, blurred by a
    periodic Gaussian of width ``sigma_cells`` (applied in Fourier space), then
    every mode is scaled to unit 2-norm.  Flattening is component-major:
    n = ((c*Z + z)*Y + y)*X + x for a 3D grid (c, Z, Y, X).
    """
    ncomp, spatial = n_grid[0], tuple(n_grid[1:])
    mult = None
    for ax, n in enumerate(spatial):
        t = _gauss_transfer(n, sigma_cells)
        shape = [1] * len(spatial)
        shape[ax] = n
        t = t.reshape(shape)
        mult = t if mult is None else mult * t
    N = int(np.prod(n_grid))
    out = np.empty((N, nc), dtype=dtype)
    per = int(np.prod(spatial))
    for i in range(nc):
        for c in range(ncomp):
            w = rng.standard_normal(spatial) + 1j * rng.standard_normal(spatial)
            out[c * per:(c + 1) * per, i] = np.fft.ifftn(np.fft.fftn(w) * mult).ravel()
        nrm = np.linalg.norm(out[:, i].astype(np.complex128))
        out[:, i] /= nrm
        if progress is not None and (i + 1) % 10 == 0:
            progress(f"smooth modes {i + 1}/{nc}")
    return out


def snapshots(modes, lam, b, m, sigma, rng, out_dtype=np.float64, row_block=1 << 18, progress=None):
    """Z[:, j] = Re(modes @ s(j)) + sigma * eps_j with s(0) = b, s(j+1) = lam * s(j).

    The state is advanced one frame at a time (a recurrence, not a power).  The
    noise is drawn column by column after everything else.
    """
    N = modes.shape[0]
    S = np.empty((lam.shape[0], m), dtype=np.complex128)
    s = b.astype(np.complex128).copy()
    for j in range(m):
        S[:, j] = s
        s = s * lam
    Z = np.empty((N, m), dtype=out_dtype, order="F")
    Sr = np.ascontiguousarray(S.real)
    Si = np.ascontiguousarray(S.imag)
    for r0 in range(0, N, row_block):
        blk = modes[r0:r0 + row_block]
        re = blk.real.astype(np.float64)
        im = blk.imag.astype(np.float64)
        Z[r0:r0 + row_block, :] = re @ Sr - im @ Si
        if progress is not None and (r0 // row_block) % 8 == 7:
            progress(f"snapshot rows {min(N, r0 + row_block)}/{N}")
    if sigma > 0:
        for j in range(m):
            Z[:, j] += sigma * rng.standard_normal(N)
            if progress is not None and j % 50 == 49:
                progress(f"noise columns {j + 1}/{m}")
    return Z


def sketch(seed, m, l, dtype=np.float32):
    """Gaussian test matrix of the randomized SVD, (m-1) x l, column-major.

    Drawn from its own stream (seed + 10**6) and rounded to the fit's element
    type, so the oracle's randomized twin and the GPU path see identical values.
    """
    g = np.random.default_rng(seed + 10 ** 6).standard_normal((m - 1, l))
    return np.asfortranarray(g.astype(dtype))


@dataclasses.dataclass
class Generated:
    cfg: Config
    Z: np.ndarray          # N x m, column-major, cfg.dtype
    lam: np.ndarray        # nc prescribed eigenvalues (Im > 0 half of each pair)
    b: np.ndarray          # nc prescribed amplitudes
    modes: np.ndarray      # N x nc prescribed complex modes
    Omega: np.ndarray | None


def generate(cfg: Config, with_sketch=True, progress=None) -> Generated:
    """Draw one workload: modes, |lambda|, arg(lambda), b, noise; then the sketch.

    ``progress``, if given, is called with a short text now and then (long draws)."""
    rng = np.random.default_rng(cfg.seed)
    if cfg.modes == "orthonormal":
        modes = orthonormal_modes(rng, cfg.N, cfg.nc)
    else:
        modes = smooth_modes(rng, cfg.n_grid, cfg.nc, progress=progress)
    lam = draw_eigs(rng, cfg.nc, cfg.lam_lo, cfg.arg, cfg.jitter)
    b = draw_amplitudes(rng, cfg.nc)
    dt = np.float64 if cfg.dtype == "f64" else np.float32
    Z = snapshots(modes, lam, b, cfg.m, cfg.sigma, rng, out_dtype=np.float64, progress=progress)
    if dt is np.float32:
        Z = np.asfortranarray(Z.astype(np.float32))
    Om = sketch(cfg.seed, cfg.m, cfg.l, dtype=dt) if (with_sketch and cfg.p > 0) else None
    return Generated(cfg, Z, lam, b, modes, Om)


@dataclasses.dataclass(frozen=True)
class Scene:
    """One scene of the multi-scene fit batch."""
    N: int
    m: int
    seed: int


def c5b_scenes():
    """Eight fits of uneven size: N from 65,536 to 2,097,152 rows, m from 100 to 300."""
    ms = [300, 100, 243, 157, 214, 129, 271, 186]
    out = []
    for i in range(8):
        N = 256 * int(round(65536 * 32 ** (i / 7) / 256))
        out.append(Scene(N, ms[i], 510 + i))
    return out


def c5b_config(scene: Scene) -> Config:
    """Configuration of one multi-scene member: 32 orthonormal pairs, r=64, p=10, q=2."""
    return Config("c5b", (scene.N,), scene.m, 32, 0.95, 1e-4, scene.seed, r=64,
                  p=10, q=2, K=100)


def synthetic_model(cfg: Config, modes_dtype=np.float32, progress=None):
    """A prescribed (not fitted) model with exact conjugate pairs, for reconstruction-only work.

    Returns (phi_pairs, lam, b): phi_pairs is N x nc complex (one member of each
    pair), lam/b the matching nc values.  The full model is the 2*nc modes
    {phi, conj(phi)} with {lam, conj(lam)} and {b, conj(b)}.
    """
    rng = np.random.default_rng(cfg.seed)
    if cfg.modes == "orthonormal":
        modes = orthonormal_modes(rng, cfg.N, cfg.nc)
    else:
        modes = smooth_modes(rng, cfg.n_grid, cfg.nc, progress=progress)
    lam = draw_eigs(rng, cfg.nc, cfg.lam_lo, cfg.arg, cfg.jitter)
    b = draw_amplitudes(rng, cfg.nc)
    return modes.astype(np.complex64 if modes_dtype == np.float32 else np.complex128), lam, b


def c5a_frames(K=4096, kmax=5000):
    """k_j = floor(j * kmax / (K-1)), j = 0..K-1."""
    j = np.arange(K, dtype=np.int64)
    return (j * kmax) // (K - 1)
