"""Plain FP64 CPU oracle of the DMD hot path.  TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The product path (the HIP library and its Python binding)
never calls it.  It shares no code with the GPU path: it uses NumPy / LAPACK in
float64 / complex128 and writes every step the way the paper defines it.

Paper: Chen et al., "Fast Subspace Fluid Simulation with a Temporally-Aware
Basis" (ACM TOG 2025).

Readings where the paper is silent or garbled:
  * X = U S V^T is the ordinary thin SVD (the paper's Sec. 3.1 swaps the names
    of the singular-vector factors).
  * Modes are the exact DMD modes  Phi = X' V_r S_r^-1 W  (the paper writes the
    projected relation w_i = U^T phi_i; both give identical reconstructions once
    the amplitudes absorb the scale).
  * Projections use the pseudo-inverse Phi^+ (DMD modes are not orthogonal);
    the paper's Phi^* is read as Phi^+, as its Sec. 6.2 writes.
  * The amplitudes are b = Phi^+ x_0 (least squares on the first snapshot).
  * Re() is taken after the sum over modes.
  * Powers are lambda^e = exp(e * Log lambda) on the principal branch, for
    integer e (arbitrary time step, Sec. 4.4) and real e = t / dt (Sec. 6.1).
  * lambda = 0: 0^0 = 1, 0^k = 0 for k > 0.
  * Temporal editing (Sec. 6.1): the printed sum drops the imaginary unit in
    front of sin(k theta); it is read as exp(i k theta).  "Adjusting" Re(Omega)
    and Im(Omega) is read as Re Omega' = s_re Re Omega + c_re and
    Im Omega' = s_im Im Omega; the mode weight w multiplies the amplitude.
    lambda = 0 (no logarithm) stays 0 under any edit.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class DMDFit:
    """Result of a fit: eigenvalues, full-space complex modes, amplitudes.

    lam: (r,) complex128;  phi: (N, r) complex128 (N may be a row subset);
    b: (r,) complex128;  sigma: (r,) singular values kept;  atilde: (r, r) reduced
    operator;  w: (r, r) eigenvectors of atilde;  v: (m-1, r) right singular
    vectors kept.
    """

    lam: np.ndarray
    phi: np.ndarray
    b: np.ndarray
    sigma: np.ndarray
    atilde: np.ndarray
    w: np.ndarray
    v: np.ndarray


def split_snapshots(Z):
    """X = [u_0 .. u_{T-1}], X' = [u_1 .. u_T]: Sec. 3.1, eq. reduced_koopman."""
    Z = np.asarray(Z, dtype=np.float64)
    return Z[:, :-1], Z[:, 1:]


def thin_svd(X):
    """Thin SVD X = U diag(s) V^T with s descending (LAPACK gesdd)."""
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    return U, s, Vt.T


def thin_svd_qr_route(Z):
    """Thin SVD of X = Z[:, :-1] through a Householder QR of Z.

    Z = Q R, so X = Q R[:, :-1] and the SVD of the small R[:, :-1] gives the SVD
    of X with U = Q U_R.  Returns (U, s, V, QtXp) where QtXp = Q^T X' = R[:, 1:].
    """
    Q, R = np.linalg.qr(np.asarray(Z, dtype=np.float64))
    Ur, s, Vt = np.linalg.svd(R[:, :-1], full_matrices=False)
    return Q @ Ur, s, Vt.T, Ur.T @ R[:, 1:]


def reduced_operator(Ur_t_Xp, V_r, s_r):
    """Atilde = U_r^T X' V_r S_r^-1 (Sec. 3.1, after eq. reduced_koopman_solution).

    Ur_t_Xp is the r x (m-1) product U_r^T X'.
    """
    return (Ur_t_Xp @ V_r) / s_r[None, :]


def dmd_from_svd(Xp, U_t_Xp, s, V, r, x0, rows=None):
    """Steps shared by the exact and randomized oracles once an SVD is known.

    U_t_Xp: U^T X' for all available left singular vectors (rows beyond r are
    ignored); s, V: singular values and right singular vectors (descending).
    rows: None, or the rows of Phi to return (for inputs too tall to hold Phi whole).
    Phi = X' M then never exists in full; b = Phi^+ x0 is the same least-squares
    solution written through its normal equations (Phi^H Phi) b = Phi^H x0, with
    Phi^H Phi = M^H (X'^T X') M and Phi^H x0 = M^H (X'^T x0) (Phi has full column rank).
    """
    s_r = s[:r]
    V_r = V[:, :r]
    at = reduced_operator(U_t_Xp[:r], V_r, s_r)          # r x r
    lam, W = np.linalg.eig(at)                             # LAPACK geev, unit columns
    M = (V_r / s_r[None, :]) @ W                           # (m-1) x r complex
    if rows is None:
        phi = Xp @ M                                       # exact modes X' V S^-1 W
        b = np.linalg.lstsq(phi, x0.astype(np.complex128), rcond=None)[0]   # b = Phi^+ x0
    else:
        phi = np.asarray(Xp[rows], dtype=np.float64) @ M
        G = M.conj().T @ (Xp.T @ Xp) @ M
        b = np.linalg.solve(G, M.conj().T @ (Xp.T @ x0))
    order = canonical_order(lam)
    return DMDFit(lam[order], phi[:, order], b[order], s_r.copy(), at, W[:, order], V_r)


def fit_exact(Z, r, route="svd"):
    """Exact DMD of rank r (Sec. 3.1, eqs. reduced_koopman .. reduced_koopman_simulation).

    route="svd": thin SVD of X by LAPACK; route="qr": the same SVD through a
    Householder QR of Z (see thin_svd_qr_route).
    """
    X, Xp = split_snapshots(Z)
    if route == "svd":
        U, s, V = thin_svd(X)
        U_t_Xp = U[:, :r].T @ Xp
    elif route == "qr":
        _, s, V, U_t_Xp = thin_svd_qr_route(Z)
    else:
        raise ValueError(route)
    return dmd_from_svd(Xp, U_t_Xp, s, V, r, X[:, 0])


def range_finder(X, Omega, q):
    """Randomized subspace iteration (Halko, Martinsson & Tropp 2011, Alg. 4.4).

    Y = X Omega, Q = qr(Y); then q times: W = qr(X^T Q), Q = qr(X W).  Householder
    QR throughout.  This is the basis Q with X ~ Q Q^T X of Sec. 4.3.
    """
    Q, _ = np.linalg.qr(X @ Omega)
    for _ in range(q):
        Wq, _ = np.linalg.qr(X.T @ Q)
        Q, _ = np.linalg.qr(X @ Wq)
    return Q


def fit_randomized(Z, r, Omega, q, rows=None):
    """FP64 randomized twin of the GPU fit (Sec. 4.3 then Sec. 3.1).

    Uses the given sketch Omega ((m-1) x l, the values handed to the GPU), the
    basis Q from range_finder, B = Q^T X and Q^T X' from one product Q^T Z, the
    SVD of the small B, then the same reduced operator / eigen / mode / amplitude
    steps as the exact DMD.  rows: return Phi on these rows only (see dmd_from_svd).
    """
    X, Xp = split_snapshots(Z)
    Q = range_finder(X, np.asarray(Omega, dtype=np.float64), q)
    Bz = Q.T @ np.asarray(Z, dtype=np.float64)
    B, Bp = Bz[:, :-1], Bz[:, 1:]
    Ub, s, Vt = np.linalg.svd(B, full_matrices=False)
    return dmd_from_svd(Xp, Ub.T @ Bp, s, Vt.T, r, X[:, 0], rows)


def canonical_order(lam):
    """Ascending |arg lambda|, ties by descending |lambda|, conjugate pairs with Im > 0 first.

    (The paper sorts modes by the size of the imaginary part, Sec. 6.3.1.)
    """
    lam = np.asarray(lam)
    keys = [(round(abs(np.angle(z)), 12), -round(abs(z), 12), -np.sign(z.imag), i)
            for i, z in enumerate(lam)]
    return np.array([k[-1] for k in sorted(keys)], dtype=np.int64)


def powers(lam, e):
    """lambda^e = exp(e * Log lambda) for an array of exponents e (Sec. 4.4, Sec. 6.1).

    Returns an (r, len(e)) complex128 array.  lambda = 0 gives 1 for e = 0 and 0
    for e > 0.
    """
    lam = np.asarray(lam, dtype=np.complex128)
    e = np.asarray(e, dtype=np.float64)
    out = np.zeros((lam.size, e.size), dtype=np.complex128)
    nz = lam != 0
    out[nz] = np.exp(np.outer(np.log(lam[nz]), e))
    if (~nz).any():
        out[~nz] = np.where(e == 0, 1.0, 0.0)[None, :]
    return out


def reconstruct(phi, lam, b, ks):
    """U[:, j] = Re(Phi diag(lambda^{k_j}) b): eq. large_time_step (Sec. 4.4)."""
    P = powers(lam, ks) * np.asarray(b, dtype=np.complex128)[:, None]
    return (np.asarray(phi, dtype=np.complex128) @ P).real


def integrate(phi, lam, b, ts, dt=1.0):
    """u(t) = Re(Phi exp(Omega t) b) with Omega = Log(Lambda) / dt: eq. edit_temporal (Sec. 6.1)."""
    Om = np.log(np.asarray(lam, dtype=np.complex128)) / dt
    P = np.exp(np.outer(Om, np.asarray(ts, dtype=np.float64))) * np.asarray(b)[:, None]
    return (np.asarray(phi, dtype=np.complex128) @ P).real


LOW_FREQ_CUT = 0.01


def frequency_clusters(lam, dt, cut=LOW_FREQ_CUT):
    """Cluster label of each mode (Sec. 6.1): 0 when |Im Omega| < cut (low frequency), else 1.

    Omega = Log(lambda) / dt, so Im Omega = arg(lambda) / dt.
    """
    lam = np.asarray(lam, dtype=np.complex128)
    theta = np.arctan2(lam.imag, lam.real)
    return np.where(np.abs(theta / dt) < cut, 0, 1).astype(np.int32)


def edit_modes(lam, b, dt, w, re_scale, re_shift, im_scale):
    """Temporal editing of eq. edit_temporal (Sec. 6.1), one parameter set per mode.

    Each eigenvalue is written as lambda = r exp(i theta) with r its modulus and
    theta = atan2(Im, Re) its phase, so Omega = (log r + i theta) / dt.  The
    edited rate and frequency are
        Re Omega' = re_scale * Re Omega + re_shift,   Im Omega' = im_scale * Im Omega,
    giving r' = exp(Re Omega' dt), theta' = Im Omega' dt and
    lambda' = r' (cos theta' + i sin theta').  The mode's weight w scales its
    amplitude: b' = w b.  Returns (lambda', b').
    """
    lam = np.asarray(lam, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    r = lam.size
    w, re_scale, re_shift, im_scale = (np.broadcast_to(np.asarray(v, dtype=np.float64), (r,))
                                       for v in (w, re_scale, re_shift, im_scale))
    lam_new = np.zeros(r, dtype=np.complex128)
    for i in range(r):
        mod = abs(lam[i])
        if mod == 0.0:
            continue
        theta = math.atan2(lam[i].imag, lam[i].real)
        om_re = math.log(mod) / dt
        om_im = theta / dt
        om_re_new = re_scale[i] * om_re + re_shift[i]
        om_im_new = im_scale[i] * om_im
        mod_new = math.exp(om_re_new * dt)
        th_new = om_im_new * dt
        lam_new[i] = complex(mod_new * math.cos(th_new), mod_new * math.sin(th_new))
    return lam_new, w * b


def cluster_edit(lam, b, dt, weight, re_scale, re_shift, im_scale, cut=LOW_FREQ_CUT):
    """edit_modes with one parameter set per frequency cluster (index 0 low, 1 high).

    Returns (lambda', b', clusters).
    """
    c = frequency_clusters(lam, dt, cut)
    pick = lambda v: np.asarray(v, dtype=np.float64)[c]
    lam_new, b_new = edit_modes(lam, b, dt, pick(weight), pick(re_scale), pick(re_shift), pick(im_scale))
    return lam_new, b_new, c


def reverse(phi, lam, u, ks):
    """Backward roll-out of eq. reverse_simulation (Sec. 6.2): z = Phi^+ u, then
    u(t - k dt) = Re(Phi Lambda^-k z) for k in ks, with u the state at time t."""
    z = project(phi, u)
    return reconstruct(phi, lam, z, -np.asarray(ks, dtype=np.float64))


def rollout(phi, lam, z0, F=None, dt=1.0, steps=None):
    """Forced reduced roll-out, eq. external_forces (Sec. 4.6, DMD with control).

    z_0 = z0 and, for s = 0 .. T-1,  z_{s+1} = Lambda z_s + dt Phi^+ f_s, where f_s is
    column s of the full-space forcing F (N x T; the paper's sum of B_i q_i and f_j at
    step s) and Phi^+ is the least-squares projection of eq. projection.  F = None runs
    `steps` unforced steps.  Returns (Z, U): the states Z (T+1, r) and the frames
    U = Re(Phi z_s) (N, T+1).
    """
    phi = np.asarray(phi, dtype=np.complex128)
    lam = np.asarray(lam, dtype=np.complex128)
    if F is None:
        T = int(steps)
        G = np.zeros((lam.size, T), dtype=np.complex128)
    else:
        F = np.asarray(F, dtype=np.float64)
        T = F.shape[1]
        G = np.linalg.lstsq(phi, F.astype(np.complex128), rcond=None)[0]   # Phi^+ f_s, all s
    Z = np.zeros((T + 1, lam.size), dtype=np.complex128)
    Z[0] = np.asarray(z0, dtype=np.complex128)
    for s in range(T):
        Z[s + 1] = lam * Z[s] + dt * G[:, s]
    U = (phi @ Z.T).real
    return Z, U


def upsample_evolve(phi, lam, h0, L, low):
    """Upsampling evolution of Sec. 6.3.1 (high-res basis, low-res guide).

    R_0 = Phi^+ h0; for t = 1 .. T:  R*_t = Lambda R_{t-1},  P_t = Phi^+ l_t,
    R_t = S^L P_t + S^H R*_t (low-order modes from the guide, the others evolved),
    and H_t = Re(Phi R_t).  L (N x T) holds the guide frames l_1 .. l_T on the high-res
    grid; low (r bools) marks the low-order modes.  Returns (R (T+1, r), H (N, T+1)).
    """
    phi = np.asarray(phi, dtype=np.complex128)
    lam = np.asarray(lam, dtype=np.complex128)
    low = np.asarray(low, dtype=bool)
    L = np.asarray(L, dtype=np.float64)
    T = L.shape[1]
    R = np.zeros((T + 1, lam.size), dtype=np.complex128)
    R[0] = project(phi, h0)
    for t in range(1, T + 1):
        r_star = lam * R[t - 1]
        P = project(phi, L[:, t - 1])
        R[t] = np.where(low, P, r_star)
    return R, (phi @ R.T).real


def block_average_matrix(ncomp, nz, ny, nx, f):
    """Dense downsampling operator A of Sec. 6.3.2: each coarse cell of each component is
    the mean of its f x f (x f) fine cells; fields are component-major (c, z, y, x) with x
    fastest, z not coarsened when nz = 1."""
    fz = 1 if nz == 1 else f
    cz, cy, cx = nz // fz, ny // f, nx // f
    A = np.zeros((ncomp * cz * cy * cx, ncomp * nz * ny * nx))
    w = 1.0 / (fz * f * f)
    for c in range(ncomp):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    row = ((c * cz + z // fz) * cy + y // f) * cx + x // f
                    col = ((c * nz + z) * ny + y) * nx + x
                    A[row, col] = w
    return A


def kkt_project(h, l, A):
    """argmin_x 1/2 ||x - h||^2 subject to A x = l (Sec. 6.3.2), from the KKT system
    [[I, A^T], [A, 0]] [x; mu] = [h; l]."""
    h = np.asarray(h, dtype=np.float64)
    l = np.asarray(l, dtype=np.float64)
    n, m = h.size, l.size
    K = np.block([[np.eye(n), A.T], [A, np.zeros((m, m))]])
    return np.linalg.solve(K, np.concatenate([h, l]))[:n]


def vandermonde(alpha, T):
    """Phi(alpha) of eq. variable_projection: entry (i, j) = alpha_j^(i-1), i = 1 .. T."""
    alpha = np.asarray(alpha, dtype=np.complex128)
    return alpha[None, :] ** np.arange(T)[:, None]


def varpro_residual(alpha, Y):
    """B = Phi(alpha)^+ Y (least squares) and the residual Y - Phi(alpha) B."""
    Phi = vandermonde(alpha, Y.shape[0])
    B = np.linalg.lstsq(Phi, Y, rcond=None)[0]
    return Y - Phi @ B, B, Phi


def varpro_trial(alpha, Y):
    """(R, B, Phi, cost) at a trial point of the Levenberg-Marquardt iteration.  A point
    whose basis overflows (|alpha|^(T-1) beyond the double range) gets an infinite cost,
    so the iteration rejects it like any point that raises the cost."""
    with np.errstate(over="ignore", invalid="ignore"):
        Phi = vandermonde(alpha, Y.shape[0])
    if not np.all(np.isfinite(Phi)):
        return None, None, Phi, np.inf
    R, B, Phi = varpro_residual(alpha, Y)
    return R, B, Phi, float(np.sum(np.abs(R) ** 2))


def varpro_normal_equations(alpha, Y, R, B, Phi):
    """Gauss-Newton normal matrix and gradient of the variable-projection residual with
    the Kaufman Jacobian J_j = -P_perp (dPhi/dalpha_j) B (Askham & Kutz 2018).

    Column j of dPhi/dalpha_j is d_j(t) = t alpha_j^(t-1); J_j is the rank-one matrix
    -(P_perp d_j) B[j, :], so <J_j, J_k> = (D~^H D~)_jk (conj(B) B^T)_jk and
    <J_j, R> = -sum_l (D~^H R)_jl conj(B_jl), with D~ = P_perp D.
    """
    T = Y.shape[0]
    t = np.arange(T)[:, None]
    D = t * np.asarray(alpha)[None, :] ** (t - 1)
    Qb, _ = np.linalg.qr(Phi)
    Dt = D - Qb @ (Qb.conj().T @ D)
    JhJ = (Dt.conj().T @ Dt) * (B.conj() @ B.T)
    g = -np.sum((Dt.conj().T @ R) * B.conj(), axis=1)
    return JhJ, g


def varpro(Y, alpha0, max_iter=200, tol=1e-13):
    """min over alpha, B of ||Y - Phi(alpha) B||_F, eq. variable_projection (Sec. 4.2).

    B is eliminated by least squares and alpha takes Levenberg-Marquardt steps
    (J^H J + mu diag(J^H J)) delta = -J^H r; a step is kept when it lowers the cost,
    then mu shrinks, else mu grows and the step is retried.  Stops when a kept step
    lowers the cost by less than tol relative.  Returns (alpha, B, cost, iterations).
    """
    Y = np.asarray(Y, dtype=np.complex128)
    alpha = np.asarray(alpha0, dtype=np.complex128).copy()
    R, B, Phi = varpro_residual(alpha, Y)
    cost = float(np.sum(np.abs(R) ** 2))
    mu = 1e-3
    it = 0
    for it in range(1, max_iter + 1):
        JhJ, g = varpro_normal_equations(alpha, Y, R, B, Phi)
        dg = np.diag(np.diag(JhJ).real)
        while True:
            delta = np.linalg.solve(JhJ + mu * dg, -g)
            a_new = alpha + delta
            R_new, B_new, Phi_new, c_new = varpro_trial(a_new, Y)
            if c_new < cost:
                break
            mu *= 4.0
            if mu > 1e20:
                return alpha, B, cost, it
        gain = cost - c_new
        alpha, R, B, Phi, cost = a_new, R_new, B_new, Phi_new, c_new
        mu = max(mu / 4.0, 1e-12)
        if gain <= tol * cost:
            break
    return alpha, B, cost, it


def fit_optdmd(U_r, s_r, V_r, alpha0, max_iter=200, tol=1e-13):
    """OptDMD of Sec. 4.2: with X ~ U_r S_r V_r^T, solve eq. variable_projection on
    Y = conj(V_r) S_r starting from alpha0, then the modes of eq. phi_optdmd,
    phi_i = U_r B^T(:, i) / ||U_r B^T(:, i)||, with amplitudes b_i = ||U_r B^T(:, i)||
    (so that x_t ~ sum_i phi_i b_i alpha_i^t, t = 0 .. T-1).
    Returns (alpha, phi, b, cost, iterations)."""
    Y = np.conj(np.asarray(V_r, dtype=np.complex128)) * np.asarray(s_r)[None, :]
    alpha, B, cost, it = varpro(Y, alpha0, max_iter, tol)
    M = np.asarray(U_r, dtype=np.complex128) @ B.T
    b = np.linalg.norm(M, axis=0)
    return alpha, M / b[None, :], b.astype(np.complex128), cost, it


def project(phi, u):
    """z = Phi^+ u: eq. projection (Sec. 3.1)."""
    return np.linalg.lstsq(np.asarray(phi, dtype=np.complex128),
                           np.asarray(u, dtype=np.complex128), rcond=None)[0]


def loss(phi, lam, b, Xt, ks):
    """L(lambda, b) = sum_j || x_{k_j} - Re(Phi (b * lambda^{k_j})) ||^2."""
    R = np.asarray(Xt, dtype=np.float64) - reconstruct(phi, lam, b, ks)
    return float(np.sum(R * R))


def loss_grad(phi, lam, b, Xt, ks):
    """Closed-form gradient of L with respect to lambda and b.

    With R_j = x_j - Re(Phi c_j), c_ij = b_i lambda_i^{k_j} and G = Phi^T R
    (transpose, not conjugate transpose):
        dL/dc_ij  = -2 conj(G_ij)                 (as  dL/dRe + i dL/dIm)
        grad_b_i  = -2 conj( sum_j G_ij lambda_i^{k_j} )
        grad_l_i  = -2 conj( sum_j G_ij k_j b_i lambda_i^{k_j - 1} )
    which is the convention of complex autograd (grad = dL/dRe + i dL/dIm).
    """
    phi = np.asarray(phi, dtype=np.complex128)
    lam = np.asarray(lam, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    ks = np.asarray(ks, dtype=np.float64)
    R = np.asarray(Xt, dtype=np.float64) - reconstruct(phi, lam, b, ks)
    G = phi.T @ R                                              # r x ncols complex
    Pk = powers(lam, ks)                                       # lambda^k
    Pkm1 = np.zeros_like(Pk)
    for j, k in enumerate(ks):                                 # k lambda^{k-1}, 0 when k = 0
        if k != 0:
            Pkm1[:, j] = k * powers(lam, [k - 1])[:, 0]
    grad_b = -2.0 * np.conj(np.sum(G * Pk, axis=1))
    grad_l = -2.0 * np.conj(np.sum(G * Pkm1, axis=1) * b)
    return float(np.sum(R * R)), grad_l, grad_b


def koopman_least_squares(X, Xp):
    """K = X' X^+ : the minimiser of ||X' - K X||_F (Sec. 3.1, eq. reduced_koopman_solution)."""
    return Xp @ np.linalg.pinv(X)
