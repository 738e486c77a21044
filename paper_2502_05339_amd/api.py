"""Python binding of the MI355X DMD library: argument marshalling over the C ABI.

Every step of the method runs in the HIP library (libdmdmi.so); this module only
allocates torch tensors for outputs and workspace, fills the C structs and calls
the C entry points on torch's current HIP stream.  There is no CPU fallback: a
missing library or GPU raises.

Layouts
  * snapshots: a (m, N) tensor whose row j is frame u_j (row-major (m, N) is the
    column-major N x m matrix Z of the C ABI); X = Z[:-1], X' = Z[1:].
  * Model.phi: (N, ldphi) row-major folded real modes (see include/dmdmi.h).
  * reconstructions: (K, N) tensors, row k = frame k.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib
from ._lib import (DMD_F32, DMD_F64, FIT_ASYNC, FIT_CHECK_FINITE, FIT_FP64_EXACT, FIT_FP64_RANDOMIZED,
                   FIT_MIXED, FIT_OPTDMD, RECON_BF16, RECON_BF16X3, RECON_FP32, RECON_FP64, check)

PRECISIONS = {"mixed": FIT_MIXED, "fp64": FIT_FP64_RANDOMIZED, "fp64_exact": FIT_FP64_EXACT}
RECON_MODES = {"fp64": RECON_FP64, "fp32": RECON_FP32, "bf16": RECON_BF16, "bf16x3": RECON_BF16X3}

_ws_cache: dict = {}


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _require_gpu(t: torch.Tensor, name: str):
    if not torch.cuda.is_available():
        raise RuntimeError("the DMD library needs a HIP GPU (no CPU fallback)")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")


def _workspace(nbytes: int, device) -> torch.Tensor:
    """A cached byte workspace per (device, stream), grown on demand (stream-ordered reuse)."""
    key = (str(device), _stream())
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def _ptr(t) -> int:
    return 0 if t is None else t.data_ptr()


def _size_t():
    return ctypes.c_size_t(0)


@dataclasses.dataclass
class Model:
    """A fitted (or prescribed) DMD model held in device memory."""

    phi: torch.Tensor      # (N, ldphi) float32/float64, folded real modes
    lam: torch.Tensor      # (r,) complex128
    b: torch.Tensor        # (r,) complex128
    sigma: torch.Tensor    # (r,) float64
    kind: torch.Tensor     # (r,) int32
    info: torch.Tensor     # (8,) int32
    dt: float = 1.0

    @property
    def n(self) -> int:
        return self.phi.shape[0]

    @property
    def r(self) -> int:
        return self.lam.shape[0]

    @property
    def dtype_code(self) -> int:
        return DMD_F32 if self.phi.dtype == torch.float32 else DMD_F64

    def struct(self, lam: torch.Tensor | None = None, b: torch.Tensor | None = None) -> _lib.ModelStruct:
        s = _lib.ModelStruct()
        s.n = self.n
        s.r = self.r
        s.dtype = self.dtype_code
        s.dt = float(self.dt)
        s.phi = self.phi.data_ptr()
        s.ldphi = self.phi.stride(0)
        s.lam = (self.lam if lam is None else lam).data_ptr()
        s.b = (self.b if b is None else b).data_ptr()
        s.sigma = self.sigma.data_ptr()
        s.kind = self.kind.data_ptr()
        s.info = self.info.data_ptr()
        return s

    @staticmethod
    def empty(n: int, r: int, dtype: torch.dtype, device, dt: float = 1.0, zero: bool = True) -> "Model":
        """Storage for a model; zero=False leaves it uninitialised (for a fit, which writes
        every entry of phi, including its padding columns, and clears info itself)."""
        ld = int(_lib.lib().dmd_phi_ld(r))
        new = torch.zeros if zero else torch.empty
        return Model(
            phi=new((n, ld), dtype=dtype, device=device),
            lam=new(r, dtype=torch.complex128, device=device),
            b=new(r, dtype=torch.complex128, device=device),
            sigma=new(r, dtype=torch.float64, device=device),
            kind=new(r, dtype=torch.int32, device=device),
            info=new(_lib.INFO_WORDS, dtype=torch.int32, device=device),
            dt=dt,
        )

    @staticmethod
    def from_pairs(phi_pairs: np.ndarray, lam_pairs: np.ndarray, b_pairs: np.ndarray, dtype=torch.float32,
                   device="cuda", dt: float = 1.0) -> "Model":
        """Prescribed model with exact conjugate pairs: modes {phi, conj(phi)}, eigenvalues
        {lam, conj(lam)}, amplitudes {b, conj(b)}; lam_pairs should have Im > 0."""
        nc = lam_pairs.shape[0]
        r = 2 * nc
        n = phi_pairs.shape[0]
        m = Model.empty(n, r, dtype, device, dt)
        folded = np.zeros((n, m.phi.shape[1]), dtype=np.float64 if dtype == torch.float64 else np.float32)
        folded[:, 0:r:2] = phi_pairs.real
        folded[:, 1:r:2] = phi_pairs.imag
        m.phi.copy_(torch.from_numpy(folded))
        lam = np.empty(r, dtype=np.complex128)
        bb = np.empty(r, dtype=np.complex128)
        lam[0::2], lam[1::2] = lam_pairs, np.conj(lam_pairs)
        bb[0::2], bb[1::2] = b_pairs, np.conj(b_pairs)
        kind = np.tile(np.array([1, 2], dtype=np.int32), nc)
        m.lam.copy_(torch.from_numpy(lam))
        m.b.copy_(torch.from_numpy(bb))
        m.kind.copy_(torch.from_numpy(kind))
        return m

    # ---- host views
    def lam_host(self) -> np.ndarray:
        return self.lam.cpu().numpy()

    def b_host(self) -> np.ndarray:
        return self.b.cpu().numpy()

    def kind_host(self) -> np.ndarray:
        return self.kind.cpu().numpy()

    def complex_modes(self, rows=None) -> np.ndarray:
        """Complex modes (N x r, or a row subset) built from the folded storage."""
        ph = self.phi[:, : self.r] if rows is None else self.phi[rows, : self.r]
        ph = ph.double().cpu().numpy()
        kind = self.kind_host()
        out = np.zeros((ph.shape[0], self.r), dtype=np.complex128)
        i = 0
        while i < self.r:
            if kind[i] == 0:
                out[:, i] = ph[:, i]
                i += 1
            else:
                out[:, i] = ph[:, i] + 1j * ph[:, i + 1]
                out[:, i + 1] = np.conj(out[:, i])
                i += 2
        return out

    # ---- evaluation
    def reconstruct(self, ks, mode: str | None = None, out: torch.Tensor | None = None,
                    check_status: bool = False) -> torch.Tensor:
        return reconstruct(self, ks, mode, out, check_status)

    def integrate(self, ts, mode: str | None = None, out: torch.Tensor | None = None,
                  check_status: bool = False) -> torch.Tensor:
        return integrate(self, ts, mode, out, check_status)

    def project(self, u: torch.Tensor) -> torch.Tensor:
        return project(self, u)

    # ---- checkpoint (versioned model file, written and read by the library)
    def save(self, path: str):
        """Write the model file (dmd_model_save: header, lambda, b, sigma, kind, Phi)."""
        ms = self.struct()
        check(_lib.lib().dmd_model_save(_stream(), ctypes.byref(ms), str(path).encode()), "dmd_model_save")

    @staticmethod
    def file_info(path: str):
        """(N, r, dtype code, dt) from a model file's header (host only)."""
        n, r, dt_code, dt = ctypes.c_int64(0), ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0.0)
        check(_lib.lib().dmd_model_file_info(str(path).encode(), ctypes.byref(n), ctypes.byref(r),
                                             ctypes.byref(dt_code), ctypes.byref(dt)), "dmd_model_file_info")
        return n.value, r.value, dt_code.value, dt.value

    @staticmethod
    def load(path: str, device="cuda") -> "Model":
        """Read a model file into new device tensors (dmd_model_load)."""
        n, r, code, dt = Model.file_info(path)
        m = Model.empty(n, r, torch.float64 if code == DMD_F64 else torch.float32, device, dt)
        _require_gpu(m.phi, "model.phi")
        ms = m.struct()
        check(_lib.lib().dmd_model_load(_stream(), str(path).encode(), ctypes.byref(ms)), "dmd_model_load")
        m.dt = ms.dt
        return m


def status_word(ws: torch.Tensor) -> int:
    """Device status (DMD_OK, DMD_ERR_DOMAIN or DMD_ERR_OVERFLOW) of the last coefficient
    pass that used workspace `ws`; waits for the current stream."""
    st = ctypes.c_int32(0)
    check(_lib.lib().dmd_status_word(_stream(), ws.data_ptr(), ctypes.byref(st)), "dmd_status_word")
    return st.value


def _check_status(ws: torch.Tensor, where: str):
    check(status_word(ws), where)


def _xview(Z: torch.Tensor | None, X: torch.Tensor | None, Xp: torch.Tensor | None):
    """(x_ptr, xp_ptr, n, ncols, ldx, ldxp, dtype_code) from a snapshot buffer or an (X, X') pair."""
    if Z is not None:
        if Z.dim() != 2 or Z.stride(1) != 1:
            raise ValueError("snapshots must be a (m, N) tensor with unit stride along N")
        m, n = Z.shape
        x, xp, ld, ldp = Z.data_ptr(), Z[1].data_ptr(), Z.stride(0), Z.stride(0)
        ncols = m - 1
        dt = Z.dtype
    else:
        if X.shape != Xp.shape or X.stride(1) != 1 or Xp.stride(1) != 1:
            raise ValueError("X and X' must be (m-1, N) tensors with unit stride along N")
        ncols, n = X.shape
        x, xp, ld, ldp = X.data_ptr(), Xp.data_ptr(), X.stride(0), Xp.stride(0)
        dt = X.dtype
    code = DMD_F32 if dt == torch.float32 else DMD_F64
    return x, xp, n, ncols, ld, ldp, code


def fit_opts(r: int, p: int = 10, q: int = 2, precision: str = "mixed", omega: torch.Tensor | None = None,
             dt: float = 1.0, rank_tol: float = 0.0, check_finite: bool = False, asynchronous: bool = False,
             optdmd: bool = False, optdmd_trials: int = 0):
    o = _lib.FitOpts()
    o.r, o.p, o.q = int(r), int(p), int(q)
    o.precision = PRECISIONS[precision]
    o.dt = float(dt)
    o.rank_tol = float(rank_tol)
    o.omega = _ptr(omega)
    o.flags = ((FIT_CHECK_FINITE if check_finite else 0) | (FIT_ASYNC if asynchronous else 0) |
               (FIT_OPTDMD if optdmd else 0))
    o.optdmd_trials = int(optdmd_trials)
    return o


def fit(Z: torch.Tensor | None = None, r: int = 0, *, X: torch.Tensor | None = None, Xp: torch.Tensor | None = None,
        p: int = 10, q: int = 2, omega: torch.Tensor | None = None, precision: str = "mixed", dt: float = 1.0,
        rank_tol: float = 0.0, check_finite: bool = False, asynchronous: bool = False,
        optdmd: bool = False, optdmd_trials: int = 0) -> Model:
    """Fit a rank-r DMD model (Sec. 4.3 randomized SVD, then Sec. 3.1).

    optdmd=True refines the eigenvalues and modes by variable projection over all
    snapshots of X (OptDMD, Sec. 4.2), with Levenberg-Marquardt decisions taken on the
    device.  A waiting call runs it to its stopping rule; with asynchronous=True it
    enqueues optdmd_trials trial points (0: 64).  model.info[4..6]: kept steps, trial
    points, outcome (0 stopped by its rule, 1 out of trial points, 2 not applied).

    Z: (m, N) snapshots (or X, Xp: (m-1, N) each); omega: (l, m-1) tensor holding the
    column-major (m-1) x l Gaussian sketch (i.e. omega.T is the sketch), same dtype as Z;
    precision: "mixed" (FP32 input), "fp64" (FP64 input, randomized) or "fp64_exact".
    """
    src = Z if Z is not None else X
    _require_gpu(src, "snapshots")
    x, xp, n, ncols, ld, ldp, code = _xview(Z, X, Xp)
    o = fit_opts(r, p, q, precision, omega, dt, rank_tol, check_finite, asynchronous, optdmd, optdmd_trials)
    L = _lib.lib()
    nb = ctypes.c_size_t(0)
    check(L.dmd_fit_workspace_size(n, ncols, code, ctypes.byref(o), ctypes.byref(nb)), "dmd_fit_workspace_size")
    ws = _workspace(nb.value, src.device)
    model = Model.empty(n, r, torch.float32 if code == DMD_F32 else torch.float64, src.device, dt, zero=False)
    ms = model.struct()
    st = L.dmd_fit(_stream(), x, xp, n, ncols, ld, ldp, code, ctypes.byref(o), ws.data_ptr(), ws.numel(),
                   ctypes.byref(ms))
    check(st, "dmd_fit")
    return model


def _default_mode(model: Model) -> str:
    return "fp64" if model.dtype_code == DMD_F64 else "bf16x3"


def _recon_common(model: Model, K: int, mode: str | None, out: torch.Tensor | None):
    mode = mode or _default_mode(model)
    mcode = RECON_MODES[mode]
    odt = torch.float64 if mcode == RECON_FP64 else torch.float32
    if out is None:
        out = torch.empty((K, model.n), dtype=odt, device=model.phi.device)
    if out.dtype != odt or out.shape[0] != K or out.shape[1] != model.n or out.stride(1) != 1:
        raise ValueError("output must be a (K, N) tensor of the mode's dtype with unit stride along N")
    L = _lib.lib()
    nb = ctypes.c_size_t(0)
    check(L.dmd_reconstruct_workspace_size(model.r, K, mcode, ctypes.byref(nb)), "dmd_reconstruct_workspace_size")
    ws = _workspace(nb.value, model.phi.device)
    return mcode, out, ws


def reconstruct(model: Model, ks, mode: str | None = None, out: torch.Tensor | None = None,
                check_status: bool = False) -> torch.Tensor:
    """U[k] = Re(Phi diag(lambda^k) b) for every integer k in ks (Sec. 4.4).

    check_status=True waits for the device and raises DMDError for DMD_ERR_DOMAIN
    (a power of lambda = 0 with k < 0) or DMD_ERR_OVERFLOW (|b| |lambda|^k past FP32/FP64)."""
    _require_gpu(model.phi, "model.phi")
    k = np.ascontiguousarray(np.asarray(ks, dtype=np.int64).ravel())
    mcode, out, ws = _recon_common(model, k.size, mode, out)
    ms = model.struct()
    st = _lib.lib().dmd_reconstruct(_stream(), ctypes.byref(ms), k.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    k.size, mcode, out.data_ptr(), out.stride(0), ws.data_ptr(), ws.numel())
    check(st, "dmd_reconstruct")
    if check_status:
        _check_status(ws, "dmd_reconstruct")
    return out


class PreparedReconstruction:
    """Coefficients b lambda^k for one exponent list, kept in a private workspace so
    that the reconstruction GEMM can be replayed (dmd_reconstruct_prepare / _apply)."""

    def __init__(self, model: Model, ks=None, ts=None, mode: str | None = None):
        _require_gpu(model.phi, "model.phi")
        self.model = model
        self.mode = mode or _default_mode(model)
        self.mcode = RECON_MODES[self.mode]
        L = _lib.lib()
        if ks is not None:
            self._k = np.ascontiguousarray(np.asarray(ks, dtype=np.int64).ravel())
            kp, tp, K = self._k.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), None, self._k.size
        else:
            self._t = np.ascontiguousarray(np.asarray(ts, dtype=np.float64).ravel())
            kp, tp, K = None, self._t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self._t.size
        self.K = K
        nb = ctypes.c_size_t(0)
        check(L.dmd_reconstruct_workspace_size(model.r, K, self.mcode, ctypes.byref(nb)), "workspace")
        self.ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=model.phi.device)
        ms = model.struct()
        check(L.dmd_reconstruct_prepare(_stream(), ctypes.byref(ms), kp, tp, K, self.mcode, self.ws.data_ptr(),
                                        self.ws.numel()), "dmd_reconstruct_prepare")

    def apply(self, out: torch.Tensor | None = None) -> torch.Tensor:
        odt = torch.float64 if self.mcode == RECON_FP64 else torch.float32
        if out is None:
            out = torch.empty((self.K, self.model.n), dtype=odt, device=self.model.phi.device)
        ms = self.model.struct()
        check(_lib.lib().dmd_reconstruct_apply(_stream(), ctypes.byref(ms), self.K, self.mcode, out.data_ptr(),
                                               out.stride(0), self.ws.data_ptr(), self.ws.numel()),
              "dmd_reconstruct_apply")
        return out


def integrate(model: Model, ts, mode: str | None = None, out: torch.Tensor | None = None,
              check_status: bool = False) -> torch.Tensor:
    """U[j] = Re(Phi exp(Omega t_j) b), Omega = Log(Lambda)/dt (Sec. 6.1); check_status as
    for reconstruct (lambda = 0 has no logarithm: negative or fractional t/dt is a domain error)."""
    _require_gpu(model.phi, "model.phi")
    t = np.ascontiguousarray(np.asarray(ts, dtype=np.float64).ravel())
    mcode, out, ws = _recon_common(model, t.size, mode, out)
    ms = model.struct()
    st = _lib.lib().dmd_integrate(_stream(), ctypes.byref(ms), t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  t.size, mcode, out.data_ptr(), out.stride(0), ws.data_ptr(), ws.numel())
    check(st, "dmd_integrate")
    if check_status:
        _check_status(ws, "dmd_integrate")
    return out


LOW_FREQ_CUT = 0.01


def _pair(v, name):
    a = np.broadcast_to(np.asarray(v, dtype=np.float64), (2,))
    if not np.all(np.isfinite(a)):
        raise ValueError(f"{name} must be finite")
    return a


def edit_modes(model: Model, weight=1.0, re_scale=1.0, re_shift=0.0, im_scale=1.0,
               freq_cut: float = LOW_FREQ_CUT, per_mode: torch.Tensor | None = None, inplace: bool = False):
    """Temporal editing (Sec. 6.1, eq. edit_temporal); returns (edited Model, cluster labels).

    Omega = Log(lambda)/dt; per frequency cluster (0: |Im Omega| < freq_cut, 1: the rest)
    Re Omega' = re_scale Re Omega + re_shift, Im Omega' = im_scale Im Omega, b' = weight b.
    weight, re_scale, re_shift, im_scale: a scalar for both clusters or a (low, high) pair.
    per_mode: optional (r, 4) float64 device tensor of (w, re_scale, re_shift, im_scale)
    rows that replaces the cluster parameters.  The edited model shares phi and kind
    with `model`; with inplace=True it also shares (and overwrites) lam and b.
    """
    _require_gpu(model.lam, "model.lam")
    e = _lib.EditStruct()
    e.freq_cut = float(freq_cut)
    for name, v in (("weight", weight), ("re_scale", re_scale), ("re_shift", re_shift), ("im_scale", im_scale)):
        a = _pair(v, name)
        getattr(e, name)[0], getattr(e, name)[1] = float(a[0]), float(a[1])
    pm = 0
    if per_mode is not None:
        _require_gpu(per_mode, "per_mode")
        if per_mode.dtype != torch.float64 or tuple(per_mode.shape) != (model.r, 4) or not per_mode.is_contiguous():
            raise ValueError("per_mode must be a contiguous (r, 4) float64 device tensor")
        pm = per_mode.data_ptr()
    lam = model.lam if inplace else torch.empty_like(model.lam)
    b = model.b if inplace else torch.empty_like(model.b)
    clusters = torch.empty(model.r, dtype=torch.int32, device=model.lam.device)
    ms = model.struct()
    check(_lib.lib().dmd_edit_modes(_stream(), ctypes.byref(ms), ctypes.byref(e), pm, lam.data_ptr(), b.data_ptr(),
                                    clusters.data_ptr()), "dmd_edit_modes")
    edited = model if inplace else dataclasses.replace(model, lam=lam, b=b)
    return edited, clusters


def reverse(model: Model, u: torch.Tensor, ks, mode: str | None = None, out: torch.Tensor | None = None):
    """Backward roll-out (Sec. 6.2, eq. reverse_simulation): z = Phi^+ u, then frame j is
    Re(Phi Lambda^-ks[j] z), the state ks[j] steps before u."""
    z = project(model, u)
    back = dataclasses.replace(model, b=z)
    return reconstruct(back, -np.asarray(ks, dtype=np.int64), mode, out)


def rollout(model: Model, forcing: torch.Tensor | None = None, steps: int | None = None,
            z0: torch.Tensor | None = None, mode: str | None = None, frames: bool = True):
    """Forced reduced roll-out (Sec. 4.6, eq. external_forces): z_{s+1} = Lambda z_s + dt Phi^+ f_s.

    forcing: (T, N) tensor of the model's dtype, row s = full-space forcing of step s (the
    paper's sum of B_i q_i and f_j), or None with `steps` = T for the unforced recurrence.
    z0: (r,) complex128 device tensor, default the model's amplitudes b.
    Returns (states (T+1, r) complex128, frames (T+1, N) or None): frame s = Re(Phi z_s).
    """
    _require_gpu(model.phi, "model.phi")
    if forcing is not None:
        _require_gpu(forcing, "forcing")
        if forcing.dim() != 2 or forcing.shape[1] != model.n or forcing.stride(1) != 1 or forcing.dtype != model.phi.dtype:
            raise ValueError("forcing must be a (T, N) tensor of the model's dtype with unit stride along N")
        T = forcing.shape[0]
        fptr, ldf = forcing.data_ptr(), forcing.stride(0)
    else:
        if steps is None or steps < 1:
            raise ValueError("steps must be given (>= 1) without forcing")
        T, fptr, ldf = int(steps), 0, model.n
    if z0 is not None:
        _require_gpu(z0, "z0")
        if z0.dtype != torch.complex128 or z0.numel() != model.r or not z0.is_contiguous():
            raise ValueError("z0 must be a contiguous (r,) complex128 tensor")
    m = mode or _default_mode(model)
    mcode = RECON_MODES[m]
    L = _lib.lib()
    nb = ctypes.c_size_t(0)
    check(L.dmd_rollout_workspace_size(model.n, model.r, T, mcode, ctypes.byref(nb)), "dmd_rollout_workspace_size")
    ws = _workspace(nb.value, model.phi.device)
    states = torch.empty((T + 1, model.r), dtype=torch.complex128, device=model.phi.device)
    U = None
    if frames:
        odt = torch.float64 if mcode == RECON_FP64 else torch.float32
        U = torch.empty((T + 1, model.n), dtype=odt, device=model.phi.device)
    ms = model.struct()
    check(L.dmd_rollout(_stream(), ctypes.byref(ms), _ptr(z0), fptr, ldf, T, mcode, _ptr(U),
                        U.stride(0) if U is not None else model.n, states.data_ptr(), ws.data_ptr(), ws.numel()),
          "dmd_rollout")
    return states, U


def upsample(model: Model, h0: torch.Tensor, guide: torch.Tensor, low, mode: str | None = None,
             frames: bool = True):
    """Upsampling evolution (Sec. 6.3.1): R_0 = Phi^+ h0, R_t = S^L Phi^+ l_t + S^H Lambda R_{t-1}.

    h0: (N,) high-res initial field; guide: (T, N) guide frames l_1 .. l_T on the high-res
    grid (model dtype); low: r booleans, True for the low-order modes taken from the guide.
    Returns (states (T+1, r) complex128, frames (T+1, N) or None), frame t = Re(Phi R_t).
    """
    _require_gpu(model.phi, "model.phi")
    for t, name in ((h0, "h0"), (guide, "guide")):
        _require_gpu(t, name)
        if t.dtype != model.phi.dtype or t.stride(-1) != 1:
            raise ValueError(f"{name} must have the model's dtype and unit stride along N")
    if h0.numel() != model.n or guide.dim() != 2 or guide.shape[1] != model.n:
        raise ValueError("h0 must hold N values and guide must be (T, N)")
    flags = np.ascontiguousarray(np.asarray(low, dtype=bool).astype(np.int32).ravel())
    if flags.size != model.r:
        raise ValueError("low must hold one flag per mode")
    T = guide.shape[0]
    mcode = RECON_MODES[mode or _default_mode(model)]
    L = _lib.lib()
    nb = ctypes.c_size_t(0)
    check(L.dmd_upsample_workspace_size(model.n, model.r, T, mcode, ctypes.byref(nb)), "dmd_upsample_workspace_size")
    ws = _workspace(nb.value, model.phi.device)
    states = torch.empty((T + 1, model.r), dtype=torch.complex128, device=model.phi.device)
    U = None
    if frames:
        odt = torch.float64 if mcode == RECON_FP64 else torch.float32
        U = torch.empty((T + 1, model.n), dtype=odt, device=model.phi.device)
    ms = model.struct()
    check(L.dmd_upsample(_stream(), ctypes.byref(ms), h0.data_ptr(), guide.data_ptr(), guide.stride(0), T,
                         flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), mcode, _ptr(U),
                         U.stride(0) if U is not None else model.n, states.data_ptr(), ws.data_ptr(), ws.numel()),
          "dmd_upsample")
    return states, U


def lowres_project(h: torch.Tensor, l: torch.Tensor, grid, factor: int, out: torch.Tensor | None = None):
    """Projection of Sec. 6.3.2: the fields closest to h whose block averages equal l.

    h: (F, N) or (N,) fine frames on grid = (ncomp, nz, ny, nx) (component-major, x fastest;
    nz = 1 for 2D); l: the coarse frames, (F, M) or (M,); factor: block size per axis.
    out may be h (in place).  Returns out.
    """
    _require_gpu(h, "h")
    _require_gpu(l, "l")
    ncomp, nz, ny, nx = (int(v) for v in grid)
    h2 = h.reshape(-1, h.shape[-1])
    l2 = l.reshape(-1, l.shape[-1])
    if h2.stride(-1) != 1 or l2.stride(-1) != 1 or l.dtype != h.dtype or h2.shape[0] != l2.shape[0]:
        raise ValueError("h and l must share dtype and frame count, with unit stride along the grid")
    x = torch.empty_like(h2) if out is None else out.reshape(-1, h.shape[-1])
    dcode = DMD_F64 if h.dtype == torch.float64 else DMD_F32
    check(_lib.lib().dmd_lowres_project(_stream(), dcode, h2.data_ptr(), h2.stride(0), l2.data_ptr(), l2.stride(0),
                                         x.data_ptr(), x.stride(0), h2.shape[0], ncomp, nz, ny, nx, int(factor)),
          "dmd_lowres_project")
    return x.reshape(h.shape)


def project(model: Model, u: torch.Tensor) -> torch.Tensor:
    """z = Phi^+ u (Sec. 3.1, eq. projection); returns (r,) complex128 on the device."""
    _require_gpu(u, "u")
    if u.dtype != model.phi.dtype or u.numel() != model.n or not u.is_contiguous():
        raise ValueError("u must be a contiguous N-vector of the model's dtype")
    L = _lib.lib()
    nb = ctypes.c_size_t(0)
    check(L.dmd_project_workspace_size(model.n, model.r, ctypes.byref(nb)), "dmd_project_workspace_size")
    ws = _workspace(nb.value, u.device)
    z = torch.empty(model.r, dtype=torch.complex128, device=u.device)
    ms = model.struct()
    check(L.dmd_project(_stream(), ctypes.byref(ms), u.data_ptr(), z.data_ptr(), ws.data_ptr(), ws.numel()),
          "dmd_project")
    return z


def loss_grad(model: Model, lam: torch.Tensor, b: torch.Tensor, X: torch.Tensor, ks):
    """(loss, grad_lambda, grad_b) of sum_j ||x_j - Re(Phi (b lambda^{k_j}))||^2 (modes fixed).

    X: (ncols, N) target frames (row j = frame compared with lambda^{k_j}), model dtype.
    Gradients follow complex autograd (dL/dRe + i dL/dIm).  Returns device tensors.
    """
    _require_gpu(X, "X")
    if X.dtype != model.phi.dtype or X.stride(1) != 1 or X.shape[1] != model.n:
        raise ValueError("X must be (ncols, N) of the model's dtype with unit stride along N")
    lam = lam.detach().to(torch.complex128).contiguous()
    b = b.detach().to(torch.complex128).contiguous()
    k = np.ascontiguousarray(np.asarray(ks, dtype=np.int64).ravel())
    if k.size != X.shape[0]:
        raise ValueError("one exponent per target frame")
    L = _lib.lib()
    nb = ctypes.c_size_t(0)
    check(L.dmd_loss_grad_workspace_size(model.n, model.r, k.size, model.dtype_code, ctypes.byref(nb)),
          "dmd_loss_grad_workspace_size")
    ws = _workspace(nb.value, X.device)
    # the library writes [loss, grad_lambda, grad_b] (1 + 4r doubles) from element 1 of a
    # fresh buffer, so that the complex gradients start on 16-byte boundaries and are
    # returned as views
    buf = torch.empty(2 + 4 * model.r, dtype=torch.float64, device=X.device)
    ms = model.struct()
    st = L.dmd_loss_grad(_stream(), ctypes.byref(ms), lam.data_ptr(), b.data_ptr(), X.data_ptr(), X.stride(0),
                         k.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), k.size, buf[1:].data_ptr(),
                         ws.data_ptr(), ws.numel())
    check(st, "dmd_loss_grad")
    r = model.r
    gl = torch.view_as_complex(buf[2:2 + 2 * r].view(r, 2))
    gb = torch.view_as_complex(buf[2 + 2 * r:].view(r, 2))
    return buf[1], gl, gb


class DMDLoss(torch.autograd.Function):
    """L(lambda, b) = sum_j ||x_j - Re(Phi (b .* lambda^{k_j}))||^2 with the modes fixed.

    forward runs the library's fused residual / adjoint; backward returns the
    gradients it produced (hand-written adjoint, no autograd graph through the kernels).
    """

    @staticmethod
    def forward(ctx, lam, b, model: Model, X: torch.Tensor, ks):
        loss, gl, gb = loss_grad(model, lam, b, X, ks)
        ctx.save_for_backward(gl.clone(), gb.clone())
        return loss.clone()

    @staticmethod
    def backward(ctx, g):
        gl, gb = ctx.saved_tensors
        return g * gl, g * gb, None, None, None


class RefitStats:
    """The statistics G0 = Phi_f^T X, M = Phi_f^T Phi_f and ||X||^2 of the target frames
    (dmd_refit_prepare), from which dmd_refit_loss_grad gives the loss and adjoint of
    loss_grad for any (lambda, b) without touching X again."""

    def __init__(self, model: Model, X: torch.Tensor, ks):
        _require_gpu(X, "X")
        if X.dtype != model.phi.dtype or X.stride(1) != 1 or X.shape[1] != model.n:
            raise ValueError("X must be (ncols, N) of the model's dtype with unit stride along N")
        k = np.ascontiguousarray(np.asarray(ks, dtype=np.int64).ravel())
        if k.size != X.shape[0]:
            raise ValueError("one exponent per target frame")
        L = _lib.lib()
        nb = ctypes.c_size_t(0)
        check(L.dmd_refit_workspace_size(model.n, model.r, k.size, ctypes.byref(nb)), "dmd_refit_workspace_size")
        self.ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=X.device)
        self.model = model
        self.ncols = int(k.size)
        self.ms = model.struct()
        check(L.dmd_refit_prepare(_stream(), ctypes.byref(self.ms), X.data_ptr(), X.stride(0),
                                  k.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), k.size, self.ws.data_ptr(),
                                  self.ws.numel()), "dmd_refit_prepare")

    def loss_grad(self, lam: torch.Tensor, b: torch.Tensor):
        """(loss, grad_lambda, grad_b) as loss_grad returns them (device tensors)."""
        lam = lam.detach().to(torch.complex128).contiguous()
        b = b.detach().to(torch.complex128).contiguous()
        r = self.model.r
        out = torch.empty(1 + 4 * r, dtype=torch.float64, device=self.ws.device)
        check(_lib.lib().dmd_refit_loss_grad(_stream(), ctypes.byref(self.ms), lam.data_ptr(), b.data_ptr(), self.ncols,
                                             out.data_ptr(), self.ws.data_ptr(), self.ws.numel()),
              "dmd_refit_loss_grad")
        gl = torch.view_as_complex(out[1:1 + 2 * r].clone().view(r, 2))
        gb = torch.view_as_complex(out[1 + 2 * r:].clone().view(r, 2))
        return out[0], gl, gb


class DMDLossStats(torch.autograd.Function):
    """DMDLoss evaluated from RefitStats (the same loss and hand-written adjoint)."""

    @staticmethod
    def forward(ctx, lam, b, stats: RefitStats):
        loss, gl, gb = stats.loss_grad(lam, b)
        ctx.save_for_backward(gl, gb)
        return loss.clone()

    @staticmethod
    def backward(ctx, g):
        gl, gb = ctx.saved_tensors
        return g * gl, g * gb, None


def refit(model: Model, X: torch.Tensor, ks, steps: int = 200, lr: float = 1e-3, optimizer: str = "adam",
          stats: bool = True):
    """Refit lambda and b by gradient steps on the full-space loss (modes fixed).

    A noise-robust refit in the spirit of OptDMD (Sec. 4.2): every snapshot of the
    horizon enters the loss at once.  With stats=True the frames are read once
    (RefitStats) and every step is O(r^2 ncols); stats=False evaluates DMDLoss on the
    frames at every step.  Returns (lam, b, losses) and leaves the model unchanged.
    """
    lam = model.lam.clone().requires_grad_(True)
    b = model.b.clone().requires_grad_(True)
    opt = torch.optim.Adam([lam, b], lr=lr) if optimizer == "adam" else torch.optim.SGD([lam, b], lr=lr)
    rs = RefitStats(model, X, ks) if stats else None
    losses = []
    for _ in range(steps):
        opt.zero_grad(set_to_none=True)
        loss = DMDLossStats.apply(lam, b, rs) if stats else DMDLoss.apply(lam, b, model, X, ks)
        loss.backward()
        opt.step()
        losses.append(loss.detach())
    return lam.detach(), b.detach(), torch.stack(losses).cpu().numpy()


class BatchedFit:
    """Several independent fits captured once into a HIP graph (one forked stream per scene)."""

    def __init__(self, scenes, capture: bool = True):
        """scenes: list of dicts with keys Z (m, N tensor), r, p, q, omega, precision, dt, and
        optionally optdmd (bool) and optdmd_trials (trial points enqueued, 0: 64)."""
        L = _lib.lib()
        self.models = []
        self._keep = []
        n = len(scenes)
        self._sc = (_lib.SceneStruct * n)()
        self._ms = (_lib.ModelStruct * n)()
        for i, s in enumerate(scenes):
            Z = s["Z"]
            _require_gpu(Z, "Z")
            x, xp, nn, ncols, ld, ldp, code = _xview(Z, None, None)
            o = fit_opts(s["r"], s.get("p", 10), s.get("q", 2), s.get("precision", "mixed"), s.get("omega"),
                         s.get("dt", 1.0), 0.0, False, True, bool(s.get("optdmd", False)),
                         int(s.get("optdmd_trials", 0)))
            nb = ctypes.c_size_t(0)
            check(L.dmd_fit_workspace_size(nn, ncols, code, ctypes.byref(o), ctypes.byref(nb)), "workspace")
            ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=Z.device)
            m = Model.empty(nn, s["r"], torch.float32 if code == DMD_F32 else torch.float64, Z.device,
                            s.get("dt", 1.0))
            self.models.append(m)
            self._keep += [Z, ws, s.get("omega")]
            sc = self._sc[i]
            sc.x, sc.xp, sc.n, sc.ncols, sc.xdtype, sc.ldx, sc.ldxp = x, xp, nn, ncols, code, ld, ldp
            sc.opts = o
            sc.ws, sc.ws_bytes = ws.data_ptr(), ws.numel()
            self._ms[i] = m.struct()
        self.graph = ctypes.c_void_p(0)
        self.capture = capture
        # capture and replay on a stream of our own (default priority): the legacy null
        # stream cannot be captured
        self.stream = torch.cuda.Stream(device=scenes[0]["Z"].device)
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            if capture:
                check(L.dmd_fit_batched(_stream(), n, self._sc, self._ms, 1, ctypes.byref(self.graph)),
                      "dmd_fit_batched")
            else:
                check(L.dmd_fit_batched(_stream(), n, self._sc, self._ms, 0, None), "dmd_fit_batched")
        torch.cuda.current_stream().wait_stream(self.stream)

    def launch(self):
        """Replay the captured batch, ordered after the caller's current stream."""
        if not self.capture:
            raise RuntimeError("not captured")
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        check(_lib.lib().dmd_graph_launch(self.graph, self.stream.cuda_stream), "dmd_graph_launch")
        cur.wait_stream(self.stream)

    def statuses(self):
        return [int(m.info[0].item()) for m in self.models]

    def close(self):
        if self.capture and self.graph.value:
            _lib.lib().dmd_graph_destroy(self.graph)
            self.graph = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_fit(Z: torch.Tensor, r: int, *, p: int = 10, q: int = 2, omega: torch.Tensor | None = None,
                 precision: str = "mixed", dt: float = 1.0, cache_path: str | None = None) -> Model:
    """Fit once while timing every tile candidate of the fit's TN products for this shape
    class (dmd_autotune_fit); later fits of the class take the fastest.  Returns the model."""
    _require_gpu(Z, "snapshots")
    x, xp, n, ncols, ld, ldp, code = _xview(Z, None, None)
    o = fit_opts(r, p, q, precision, omega, dt)
    L = _lib.lib()
    nb = ctypes.c_size_t(0)
    check(L.dmd_fit_workspace_size(n, ncols, code, ctypes.byref(o), ctypes.byref(nb)), "dmd_fit_workspace_size")
    ws = _workspace(nb.value, Z.device)
    model = Model.empty(n, r, torch.float32 if code == DMD_F32 else torch.float64, Z.device, dt)
    ms = model.struct()
    check(L.dmd_autotune_fit(_stream(), x, xp, n, ncols, ld, ldp, code, ctypes.byref(o), ws.data_ptr(), ws.numel(),
                             ctypes.byref(ms), None if cache_path is None else cache_path.encode()),
          "dmd_autotune_fit")
    return model


def autotune_reconstruct(model: Model, K: int, mode: str | None = None, cache_path: str | None = None) -> int:
    """Time the reconstruction kernel's tile-shape candidates on this model; keep the fastest."""
    mcode, out, ws = _recon_common(model, K, mode, None)
    ms = model.struct()
    best = ctypes.c_int32(-1)
    st = _lib.lib().dmd_autotune_reconstruct(_stream(), ctypes.byref(ms), K, mcode, out.data_ptr(), out.stride(0),
                                             ws.data_ptr(), ws.numel(),
                                             None if cache_path is None else cache_path.encode(), ctypes.byref(best))
    check(st, "dmd_autotune_reconstruct")
    return best.value
