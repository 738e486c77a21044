"""Pins of the FP64 oracle against mathematics the paper fixes (CPU only).

The paper prints no numerical worked example, eigenvalue table or field error
value, so no pin here uses a number from it ("parity unpinned" by the paper);
every pin comes from a closed form, a textbook special case, an invariant the
paper states, or brute force on tiny inputs.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle.metrics import eig_errors, field_errors

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _truth(g):
    lam = np.concatenate([g.lam, np.conj(g.lam)])
    return lam


# ---------------------------------------------------------------- closed form
@pytest.mark.parametrize("seed", [102, 103, 104])
def test_closed_form_linear_system(seed):
    """Noise-free snapshots of a rank-16 linear system: DMD returns its eigenvalues
    and rebuilds the data (Sec. 3.1: a mode representable in the reduced space
    keeps its eigenvalue)."""
    cfg = synth.config("c1-cf", seed=seed)
    g = synth.generate(cfg)
    f = oracle.fit_exact(g.Z, cfg.r)
    e = eig_errors(f.lam, _truth(g))
    assert e["max_rel"] <= 1e-10
    U = oracle.reconstruct(f.phi, f.lam, f.b, np.arange(cfg.m))
    assert field_errors(U, g.Z)["max_frame"] <= 1e-12


def test_rotation_golden():
    """Hand-built 2x2 rotation-scaling system lifted to 5 DOFs (tests/golden/rotation_2x2.json).

    u_{j+1} = P A P^T u_j with A = rho [[cos t, -sin t], [sin t, cos t]] and P
    with orthonormal columns; its nonzero Koopman eigenvalues are rho e^{+-it}.
    """
    with open(os.path.join(GOLDEN, "rotation_2x2.json")) as fh:
        gd = json.load(fh)
    rho, th = gd["rho"], gd["theta"]
    P = np.array(gd["P"], dtype=np.float64)
    A = rho * np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    u = P @ np.array(gd["y0"], dtype=np.float64)
    Z = np.empty((5, gd["m"]))
    for j in range(gd["m"]):
        Z[:, j] = u
        u = P @ (A @ (P.T @ u))
    f = oracle.fit_exact(Z, 2)
    expect = np.array([rho * complex(math.cos(th), math.sin(th)),
                       rho * complex(math.cos(th), -math.sin(th))])
    assert np.allclose(f.lam, expect, rtol=0, atol=1e-13)
    assert f.lam[0].imag > 0          # canonical order: Im > 0 member first
    # stored expectation written by hand from the closed form
    assert abs(f.lam[0] - complex(*gd["lambda_plus"])) <= 1e-12
    U = oracle.reconstruct(f.phi, f.lam, f.b, np.arange(gd["m"]))
    assert np.abs(U - Z).max() <= 1e-13


# ---------------------------------------------------------- textbook / brute
def test_textbook_koopman_tiny():
    """At full rank, DMD eigenvalues are the nonzero eigenvalues of K = X' X^+ and
    K Phi = Phi Lambda (Sec. 3.1, eq. reduced_koopman_solution)."""
    rng = np.random.default_rng(7)
    N, m = 9, 6
    Z = rng.standard_normal((N, m))
    X, Xp = oracle.split_snapshots(Z)
    r = m - 1
    f = oracle.fit_exact(Z, r)
    K = oracle.koopman_least_squares(X, Xp)
    ev = np.linalg.eigvals(K)
    ev = ev[np.argsort(-np.abs(ev))][:r]
    assert eig_errors(f.lam, ev)["max_rel"] <= 1e-10
    res = K @ f.phi - f.phi * f.lam[None, :]
    assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(f.phi)


def test_var1_special_case():
    """More frames than DOFs: full-rank DMD is the VAR(1) least-squares fit X' = A X
    (Sec. 7, eq. var) and its eigenvalues are those of A."""
    rng = np.random.default_rng(11)
    N, m = 4, 40
    A = rng.standard_normal((N, N)) * 0.4
    Z = np.empty((N, m))
    Z[:, 0] = rng.standard_normal(N)
    for j in range(1, m):
        Z[:, j] = A @ Z[:, j - 1] + 1e-2 * rng.standard_normal(N)
    X, Xp = oracle.split_snapshots(Z)
    A_ls = np.linalg.lstsq(X.T, Xp.T, rcond=None)[0].T
    f = oracle.fit_exact(Z, N)
    assert eig_errors(f.lam, np.linalg.eigvals(A_ls))["max_rel"] <= 1e-11


@pytest.mark.parametrize("shape", [(7, 5), (30, 9), (12, 13)])
def test_svd_routes_brute_force(shape):
    """Thin SVD by LAPACK, by the QR route, and by eig(X^T X) agree on tiny inputs."""
    rng = np.random.default_rng(sum(shape))
    Z = rng.standard_normal(shape)
    X, Xp = oracle.split_snapshots(Z)
    U, s, V = oracle.thin_svd(X)
    U2, s2, V2, QtXp = oracle.thin_svd_qr_route(Z)
    ev = np.sort(np.linalg.eigvalsh(X.T @ X))[::-1][:len(s)]
    assert np.allclose(s, s2, rtol=1e-12, atol=1e-13)
    assert np.allclose(s ** 2, ev, rtol=1e-10, atol=1e-12)
    assert np.allclose((U * s) @ V.T, X, atol=1e-12)
    assert np.allclose((U2 * s2) @ V2.T, X, atol=1e-12)
    k = min(len(s), Z.shape[1] - 1)
    assert np.allclose(np.abs(U2[:, :k].T @ Xp), np.abs(QtXp[:k]), atol=1e-11)


def test_routes_agree_on_fit():
    """Exact DMD through LAPACK SVD and through the QR route give the same result."""
    cfg = synth.config("c1-cf", seed=103)
    g = synth.generate(cfg)
    f1 = oracle.fit_exact(g.Z, cfg.r, route="svd")
    f2 = oracle.fit_exact(g.Z, cfg.r, route="qr")
    assert eig_errors(f1.lam, f2.lam)["max_rel"] <= 1e-12
    ks = np.arange(100)
    U1 = oracle.reconstruct(f1.phi, f1.lam, f1.b, ks)
    U2 = oracle.reconstruct(f2.phi, f2.lam, f2.b, ks)
    assert field_errors(U2, U1)["max_frame"] <= 1e-11


# --------------------------------------------------------------- randomized
def test_randomized_equals_exact_low_rank():
    """Halko et al.: with rank(X) <= l the randomized range finder is exact, so the
    randomized twin equals the exact DMD (Sec. 4.3)."""
    cfg = synth.Config("lowrank", (2, 32, 32), 60, 10, 0.95, 0.0, 31, r=20,
                       p=6, q=1, jitter=True)
    g = synth.generate(cfg)
    Z = g.Z.astype(np.float64)
    fe = oracle.fit_exact(Z, cfg.r)
    fr = oracle.fit_randomized(Z, cfg.r, g.Omega, cfg.q)
    assert eig_errors(fr.lam, fe.lam)["max_rel"] <= 1e-9
    ks = np.arange(cfg.m)
    Ue = oracle.reconstruct(fe.phi, fe.lam, fe.b, ks)
    Ur = oracle.reconstruct(fr.phi, fr.lam, fr.b, ks)
    assert field_errors(Ur, Ue)["max_frame"] <= 1e-9


def test_randomized_equals_exact_well_posed():
    """Signal far above the noise and r equal to the signal rank: twin == exact."""
    cfg = synth.Config("wp", (2, 48, 48), 120, 30, 0.95, 1e-6, 202, r=60, p=10,
                       q=2, jitter=True)
    g = synth.generate(cfg)
    Z = g.Z.astype(np.float64)
    fe = oracle.fit_exact(Z, cfg.r)
    fr = oracle.fit_randomized(Z, cfg.r, g.Omega, cfg.q)
    assert eig_errors(fr.lam, fe.lam)["max_rel"] <= 1e-8
    assert eig_errors(fe.lam, _truth(g))["max_rel"] <= 1e-4
    ks = np.arange(cfg.m)
    Ue = oracle.reconstruct(fe.phi, fe.lam, fe.b, ks)
    Ur = oracle.reconstruct(fr.phi, fr.lam, fr.b, ks)
    assert field_errors(Ur, Ue)["max_frame"] <= 1e-8


def test_range_finder_orthonormal():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((200, 40))
    Q = oracle.range_finder(X, rng.standard_normal((40, 12)), 2)
    assert np.allclose(Q.T @ Q, np.eye(12), atol=1e-13)


# --------------------------------------------------------------- invariants
def _periodic_diff(n):
    D = np.zeros((n, n))
    for i in range(n):
        D[i, (i + 1) % n] = 0.5
        D[i, (i - 1) % n] = -0.5
    return D


def test_constraint_inherited():
    """C X = 0 implies C Phi = 0 (Sec. 4.5): divergence-free data give
    divergence-free modes."""
    n = 16
    D = _periodic_diff(n)
    I = np.eye(n)
    Dx = np.kron(I, D)          # d/dx on a row-major n x n grid
    Dy = np.kron(D, I)
    C = np.hstack([Dx, Dy])     # discrete divergence of (u, v)
    rng = np.random.default_rng(5)
    nc = 6
    psi = rng.standard_normal((n * n, nc)) + 1j * rng.standard_normal((n * n, nc))
    modes = np.vstack([Dy @ psi, -(Dx @ psi)])
    lam = synth.draw_eigs(rng, nc, 0.9, jitter=True)
    b = synth.draw_amplitudes(rng, nc)
    Z = synth.snapshots(modes, lam, b, 40, 0.0, rng)
    assert np.linalg.norm(C @ Z) <= 1e-13 * np.linalg.norm(C) * np.linalg.norm(Z)
    f = oracle.fit_exact(Z, 2 * nc)
    rel = np.linalg.norm(C @ f.phi) / (np.linalg.norm(C) * np.linalg.norm(f.phi))
    assert rel <= 1e-14


def test_powers_exp_log_vs_repeated_multiplication():
    """lambda^k by exp(k Log lambda) equals k single steps (Sec. 4.4 vs eq.
    reduced_koopman_simulation)."""
    rng = np.random.default_rng(9)
    lam = synth.draw_eigs(rng, 20, 0.95)
    P = oracle.powers(lam, [5000])[:, 0]
    z = np.ones_like(lam)
    for _ in range(5000):
        z = z * lam
    assert np.max(np.abs(P - z) / np.abs(z)) <= 1e-12
    P0 = oracle.powers(np.array([0.0, 0.5]), [0, 1, 2])
    assert np.allclose(P0, [[1, 0, 0], [1, 0.5, 0.25]])


def test_time_reversal_round_trip():
    """Lambda^-1 reverses the reduced dynamics (Sec. 6.2, eq. reverse_simulation)."""
    cfg = synth.config("c1-cf", seed=104)
    g = synth.generate(cfg)
    f = oracle.fit_exact(g.Z, cfg.r)
    k = 37
    zk = f.b * oracle.powers(f.lam, [k])[:, 0]
    back = zk * oracle.powers(f.lam, [-k])[:, 0]
    assert np.allclose(back, f.b, rtol=1e-12, atol=1e-14)
    Uback = oracle.reconstruct(f.phi, f.lam, zk, [-k])
    assert field_errors(Uback, g.Z[:, :1])["max_frame"] <= 1e-11


# ---------------------------------------------------- temporal editing (Sec. 6.1)
def _edit_case(seed=41, nc=12, dt=0.5):
    rng = np.random.default_rng(seed)
    lam_p = synth.draw_eigs(rng, nc, 0.9, arg=(0.001, 2.5))
    lam = np.concatenate([lam_p, np.conj(lam_p), [0.93, -0.7]])
    b = np.concatenate([synth.draw_amplitudes(rng, nc)] * 2 + [[0.4 - 0.1j, 1.2 + 0.3j]])
    b[nc:2 * nc] = np.conj(b[:nc])
    return lam, b, dt


def test_edit_identity():
    """Unit weights and scales and zero shift leave every eigenvalue and amplitude unchanged."""
    lam, b, dt = _edit_case()
    l2, b2 = oracle.edit_modes(lam, b, dt, 1.0, 1.0, 0.0, 1.0)
    assert np.max(np.abs(l2 - lam) / np.abs(lam)) <= 4e-16 * 8
    assert np.array_equal(b2, b)


def test_edit_closed_forms():
    """Doubling Omega squares lambda, negating it inverts lambda, a shift of
    log(s)/dt scales lambda by s, a zero frequency scale leaves |lambda|."""
    lam, b, dt = _edit_case(dt=0.37)
    l2, _ = oracle.edit_modes(lam, b, dt, 1.0, 2.0, 0.0, 2.0)
    assert np.max(np.abs(l2 - lam * lam) / np.abs(lam * lam)) <= 1e-14
    li, _ = oracle.edit_modes(lam, b, dt, 1.0, -1.0, 0.0, -1.0)
    assert np.max(np.abs(li - 1.0 / lam) * np.abs(lam)) <= 1e-14
    ls, _ = oracle.edit_modes(lam, b, dt, 1.0, 1.0, math.log(1.5) / dt, 1.0)
    assert np.max(np.abs(ls - 1.5 * lam) / np.abs(lam)) <= 1e-14
    la, _ = oracle.edit_modes(lam, b, dt, 1.0, 1.0, 0.0, 0.0)
    assert np.max(np.abs(la - np.abs(lam)) / np.abs(lam)) <= 1e-15
    lu, _ = oracle.edit_modes(lam, b, dt, 1.0, 0.0, 0.0, 1.0)
    assert np.max(np.abs(lu - lam / np.abs(lam))) <= 1e-15
    lz, bz = oracle.edit_modes(np.array([0.0, 0.5]), np.array([1.0, 1.0]), dt, 3.0, 2.0, 0.1, 2.0)
    assert lz[0] == 0 and np.array_equal(bz, [3.0, 3.0])


def test_edit_clusters_brute_force():
    """|Im Omega| = |arg lambda| / dt against the 0.01 cut, by hand."""
    dt = 0.5
    th = np.array([0.0, 0.004, -0.004, 0.0049, 0.0051, 0.006, -0.2, np.pi])
    lam = 0.9 * np.exp(1j * th)
    lam[-1] = -0.9
    c = oracle.frequency_clusters(lam, dt)
    assert list(c) == [0, 0, 0, 0, 1, 1, 1, 1]
    assert list(oracle.frequency_clusters(lam, 1.0)) == [0, 0, 0, 0, 0, 0, 1, 1]


def test_edit_reconstruction_semigroup_and_weights():
    """Reconstructing the Omega-doubled model at k equals the original at 2k;
    cluster weights (a, c) give a U_low + c U_high."""
    cfg = synth.config("c1-cf", seed=102)
    g = synth.generate(cfg)
    f = oracle.fit_exact(g.Z, cfg.r)
    dt = 0.25
    ks = np.array([0, 1, 5, 33])
    l2, b2 = oracle.edit_modes(f.lam, f.b, dt, 1.0, 2.0, 0.0, 2.0)
    U2 = oracle.reconstruct(f.phi, l2, b2, ks)
    U1 = oracle.reconstruct(f.phi, f.lam, f.b, 2 * ks)
    assert field_errors(U2, U1)["max_frame"] <= 1e-12
    cut = np.median(np.abs(np.angle(f.lam))) / dt
    lw, bw, c = oracle.cluster_edit(f.lam, f.b, dt, (2.0, 3.0), (1, 1), (0, 0), (1, 1), cut=cut)
    assert 0 < c.sum() < c.size
    assert np.array_equal(lw, oracle.edit_modes(f.lam, f.b, dt, 1, 1, 0, 1)[0])
    Uw = oracle.reconstruct(f.phi, lw, bw, ks)
    lo, hi = c == 0, c == 1
    Ulo = oracle.reconstruct(f.phi[:, lo], f.lam[lo], f.b[lo], ks)
    Uhi = oracle.reconstruct(f.phi[:, hi], f.lam[hi], f.b[hi], ks)
    assert field_errors(Uw, 2 * Ulo + 3 * Uhi)["max_frame"] <= 1e-12


def test_reverse_recovers_earlier_snapshots():
    """Backward roll-out from the last snapshot of an exactly linear sequence
    returns the earlier snapshots (Sec. 6.2, eq. reverse_simulation)."""
    cfg = synth.config("c1-cf", seed=103)
    g = synth.generate(cfg)
    f = oracle.fit_exact(g.Z, cfg.r)
    T = g.Z.shape[1] - 1
    ks = np.array([1, 2, 10, T])
    U = oracle.reverse(f.phi, f.lam, g.Z[:, T], ks)
    assert field_errors(U, g.Z[:, T - ks])["max_frame"] <= 1e-9


# ------------------------------------------- forced roll-out (Sec. 4.6, DMDc)
def _paired_vector(rng, kind_like):
    """A complex vector conjugate-paired like a fitted eigenvalue list."""
    v = rng.standard_normal(kind_like.size) + 1j * rng.standard_normal(kind_like.size)
    i = 0
    while i < kind_like.size:
        if abs(kind_like[i].imag) < 1e-12:
            v[i] = v[i].real
            i += 1
        else:
            v[i + 1] = np.conj(v[i])
            i += 2
    return v


def test_rollout_unforced_is_reconstruction():
    cfg = synth.config("c1-cf", seed=102)
    g = synth.generate(cfg)
    f = oracle.fit_exact(g.Z, cfg.r)
    Z, U = oracle.rollout(f.phi, f.lam, f.b, None, dt=0.3, steps=40)
    assert field_errors(U, oracle.reconstruct(f.phi, f.lam, f.b, np.arange(41)))["max_frame"] <= 1e-13
    assert np.allclose(Z[17], f.b * f.lam ** 17, rtol=1e-12, atol=0)


def test_rollout_constant_forcing_geometric_series():
    """f_s = Phi c for every s gives z_s = lambda^s z0 + dt (1 - lambda^s) / (1 - lambda) c."""
    cfg = synth.config("c1-cf", seed=103)
    g = synth.generate(cfg)
    f = oracle.fit_exact(g.Z, cfg.r)
    rng = np.random.default_rng(4)
    c = _paired_vector(rng, f.lam)
    fs = (f.phi @ c).real
    T, dt = 25, 0.4
    F = np.repeat(fs[:, None], T, axis=1)
    Z, _ = oracle.rollout(f.phi, f.lam, f.b, F, dt=dt)
    s = np.arange(T + 1)[:, None]
    expect = f.lam[None, :] ** s * f.b[None, :] + dt * (1 - f.lam[None, :] ** s) / (1 - f.lam[None, :]) * c[None, :]
    assert np.max(np.abs(Z - expect)) <= 1e-10 * np.max(np.abs(expect))


def test_rollout_orthogonal_forcing_and_linearity():
    """Forcing orthogonal to the modes' real span changes nothing; the response is linear in F."""
    cfg = synth.config("c1-cf", seed=104)
    g = synth.generate(cfg)
    f = oracle.fit_exact(g.Z, cfg.r)
    rng = np.random.default_rng(5)
    T = 12
    basis = np.concatenate([f.phi.real, f.phi.imag], axis=1)
    F = rng.standard_normal((f.phi.shape[0], T))
    Fperp = F - basis @ np.linalg.lstsq(basis, F, rcond=None)[0]
    Z0, _ = oracle.rollout(f.phi, f.lam, f.b, None, steps=T)
    Zp, _ = oracle.rollout(f.phi, f.lam, f.b, Fperp, dt=0.7)
    assert np.max(np.abs(Zp - Z0)) <= 1e-10 * np.max(np.abs(Z0))
    F1, F2 = rng.standard_normal((2, f.phi.shape[0], T))
    Za, _ = oracle.rollout(f.phi, f.lam, f.b, F1, dt=0.7)
    Zb, _ = oracle.rollout(f.phi, f.lam, f.b, F2, dt=0.7)
    Zc, _ = oracle.rollout(f.phi, f.lam, f.b, F1 + F2, dt=0.7)
    assert np.max(np.abs((Zc - Z0) - (Za - Z0) - (Zb - Z0))) <= 1e-10 * np.max(np.abs(Zc))


def test_rollout_two_mode_by_hand():
    """Orthonormal complex pair: Phi^+ = Phi^H; two steps written out."""
    v = np.array([1.0, 1j, 0.0]) / np.sqrt(2.0)
    phi = np.stack([v, np.conj(v)], axis=1)
    lam = np.array([0.9 * np.exp(0.2j), 0.9 * np.exp(-0.2j)])
    z0 = np.array([1 + 1j, 1 - 1j])
    F = np.array([[1.0, 0.0], [0.0, 2.0], [5.0, 5.0]])     # the third row is outside the span
    dt = 0.5
    g = np.conj(phi).T @ F                                   # Phi^H f_s
    z1 = lam * z0 + dt * g[:, 0]
    z2 = lam * z1 + dt * g[:, 1]
    Z, U = oracle.rollout(phi, lam, z0, F, dt=dt)
    assert np.allclose(Z, [z0, z1, z2], rtol=0, atol=1e-14)
    assert np.allclose(U[:, 2], (phi @ z2).real, atol=1e-14)


# ------------------------------------------------- upsampling (Sec. 6.3)
def _upsample_case(seed=102):
    cfg = synth.config("c1-cf", seed=seed)
    g = synth.generate(cfg)
    return oracle.fit_exact(g.Z, cfg.r)


def test_upsample_all_high_is_dmd_evolution():
    f = _upsample_case()
    rng = np.random.default_rng(6)
    h0 = rng.standard_normal(f.phi.shape[0])
    L = rng.standard_normal((f.phi.shape[0], 9))
    R, H = oracle.upsample_evolve(f.phi, f.lam, h0, L, np.zeros(f.lam.size, bool))
    z0 = oracle.project(f.phi, h0)
    assert field_errors(H, oracle.reconstruct(f.phi, f.lam, z0, np.arange(10)))["max_frame"] <= 1e-12


def test_upsample_guide_in_span_and_zero_guide():
    """A guide inside the modes' span is reproduced by the low-order modes; with a zero
    guide the low-order modes vanish and the others follow Lambda^t."""
    f = _upsample_case(103)
    rng = np.random.default_rng(7)
    T = 6
    cs = [_paired_vector(rng, f.lam) for _ in range(T + 1)]
    L = np.stack([(f.phi @ c).real for c in cs[1:]], axis=1)
    h0 = (f.phi @ cs[0]).real
    R, H = oracle.upsample_evolve(f.phi, f.lam, h0, L, np.ones(f.lam.size, bool))
    assert field_errors(H[:, 1:], L)["max_frame"] <= 1e-10
    low = np.abs(np.angle(f.lam)) < np.median(np.abs(np.angle(f.lam)))
    R0, H0 = oracle.upsample_evolve(f.phi, f.lam, h0, np.zeros_like(L), low)
    expect = np.where(low[None, :], 0.0, cs[0][None, :] * f.lam[None, :] ** np.arange(T + 1)[:, None])
    expect[0] = cs[0]                                        # R_0 = Phi^+ h0 in every mode
    assert np.max(np.abs(R0 - expect)) <= 1e-10 * np.max(np.abs(expect))


def test_block_average_and_kkt_projection():
    """x = argmin ||x - h|| with A x = l: the constraint holds, x - h is constant over each
    block (it lies in the range of A^T), a feasible h is kept, and a 4 x 4 case by hand."""
    rng = np.random.default_rng(8)
    for (nc, nz, ny, nx, fct) in [(2, 1, 8, 8, 2), (1, 4, 6, 6, 2), (3, 1, 9, 6, 3)]:
        A = oracle.block_average_matrix(nc, nz, ny, nx, fct)
        assert np.allclose(A.sum(axis=1), 1.0) and np.allclose(A @ A.T, np.eye(A.shape[0]) * A.max())
        h = rng.standard_normal(A.shape[1])
        l = rng.standard_normal(A.shape[0])
        x = oracle.kkt_project(h, l, A)
        assert np.max(np.abs(A @ x - l)) <= 1e-12
        d = x - h                                            # in the range of A^T
        assert np.max(np.abs(d - A.T @ np.linalg.lstsq(A.T, d, rcond=None)[0])) <= 1e-12
        assert np.max(np.abs(oracle.kkt_project(x, l, A) - x)) <= 1e-12
    h = np.arange(16.0)
    l = np.array([1.0, 2.0, 3.0, 4.0])
    A = oracle.block_average_matrix(1, 1, 4, 4, 2)
    x = oracle.kkt_project(h, l, A).reshape(4, 4)
    H = h.reshape(4, 4)
    for by in range(2):
        for bx in range(2):
            blk = H[2 * by:2 * by + 2, 2 * bx:2 * bx + 2]
            assert np.allclose(x[2 * by:2 * by + 2, 2 * bx:2 * bx + 2], blk - (blk.mean() - l[2 * by + bx]), atol=1e-12)


# ------------------------------------------------ OptDMD (Sec. 4.2, varpro)
def test_varpro_recovers_exact_exponentials():
    """Noise-free data Y = Phi(alpha) B: from a perturbed start the fit returns alpha."""
    rng = np.random.default_rng(21)
    T, nc = 40, 3
    ap = 0.97 * np.exp(1j * np.array([0.1, 0.25, 0.4]))
    at = np.concatenate([ap, ap.conj(), [0.9, -0.5]])
    r = at.size
    B = rng.standard_normal((r, r)) + 1j * rng.standard_normal((r, r))
    Y = oracle.vandermonde(at, T) @ B
    a0 = at * (1 + 1e-3 * rng.standard_normal(r))
    a, Bo, cost, it = oracle.varpro(Y, a0)
    assert np.max(np.abs(a - at)) <= 1e-10
    assert cost <= 1e-20 * np.sum(np.abs(Y) ** 2)


def test_varpro_trial_rejects_overflowing_basis():
    """A trial point whose Vandermonde basis overflows gets an infinite cost (rejected),
    and one in range gets the plain residual norm."""
    rng = np.random.default_rng(23)
    Y = rng.standard_normal((200, 3)) + 1j * rng.standard_normal((200, 3))
    R, B, Phi, c = oracle.varpro_trial(np.array([0.9, 40.0, 0.5j]), Y)
    assert R is None and c == np.inf
    al = np.array([0.9, 0.8 * np.exp(0.2j), 0.5j])
    R, B, Phi, c = oracle.varpro_trial(al, Y)
    Rr, _, _ = oracle.varpro_residual(al, Y)
    assert c == float(np.sum(np.abs(Rr) ** 2)) and np.isfinite(c)


def test_varpro_normal_equations_match_explicit_jacobian():
    """The structured J^H J and J^H r equal products with the explicit Kaufman Jacobian."""
    rng = np.random.default_rng(22)
    T, r = 9, 3
    al = np.array([0.9 * np.exp(0.3j), 0.8, 0.95 * np.exp(-0.7j)])
    Y = rng.standard_normal((T, r)) + 1j * rng.standard_normal((T, r))
    R, B, Phi = oracle.varpro_residual(al, Y)
    JhJ, g = oracle.varpro_normal_equations(al, Y, R, B, Phi)
    t = np.arange(T)[:, None]
    D = t * al[None, :] ** (t - 1)
    P = np.eye(T) - Phi @ np.linalg.pinv(Phi)
    J = np.stack([-np.outer(P @ D[:, j], B[j, :]).ravel() for j in range(r)], axis=1)
    assert np.max(np.abs(J.conj().T @ J - JhJ)) <= 1e-13
    assert np.max(np.abs(J.conj().T @ R.ravel() - g)) <= 1e-13
    # and J is the derivative of the projected residual (finite differences, Kaufman drops
    # a term that vanishes at a zero residual, so compare on exact data)
    Ye = oracle.vandermonde(al, T) @ B
    Re, Be, Pe = oracle.varpro_residual(al, Ye)
    h = 1e-7
    ap = al.copy()
    ap[1] += h
    Rp, _, _ = oracle.varpro_residual(ap, Ye)
    Je = -np.outer((np.eye(T) - Pe @ np.linalg.pinv(Pe)) @ D[:, 1], Be[1, :])
    assert np.max(np.abs((Rp - Re) / h - Je)) <= 1e-5 * max(1.0, np.max(np.abs(Je)))


def test_optdmd_beats_dmd_on_noisy_data():
    """With noise, eq. variable_projection over all snapshots gives eigenvalues closer to
    the truth than the one-step fit of eq. reduced_koopman_solution (the reason for
    OptDMD in Sec. 4.2); the lifted modes reproduce the rank-r data."""
    for seed in (11, 12, 13):
        cfg = synth.config("c1-cf", seed=seed, sigma=1e-2)
        g = synth.generate(cfg)
        f = oracle.fit_exact(g.Z, cfg.r)
        X, _ = oracle.split_snapshots(g.Z)
        U, s, V = oracle.thin_svd(X)
        a, phi, b, cost, it = oracle.fit_optdmd(U[:, :cfg.r], s[:cfg.r], V[:, :cfg.r], f.lam)
        truth = _truth(g)
        assert eig_errors(a, truth)["max_rel"] < 0.25 * eig_errors(f.lam, truth)["max_rel"]
        # conjugate pairs stay paired (real data)
        assert eig_errors(np.conj(a), a)["max_rel"] <= 1e-10
        Xr = (U[:, :cfg.r] * s[:cfg.r]) @ V[:, :cfg.r].T
        Ur = oracle.reconstruct(phi, a, b, np.arange(X.shape[1]))
        assert np.linalg.norm(Ur - Xr) ** 2 <= 1.0001 * cost


def test_integrate_matches_integer_steps_and_semigroup():
    """exp(Omega t) at t = k dt equals Lambda^k; exp(Omega(t1+t2)) = exp(Omega t1) exp(Omega t2)."""
    cfg = synth.config("c1-cf", seed=102)
    g = synth.generate(cfg)
    f = oracle.fit_exact(g.Z, cfg.r)
    dt = 0.25
    ks = np.array([0, 1, 7, 64])
    U1 = oracle.reconstruct(f.phi, f.lam, f.b, ks)
    U2 = oracle.integrate(f.phi, f.lam, f.b, ks * dt, dt=dt)
    assert field_errors(U2, U1)["max_frame"] <= 1e-13
    t1, t2 = 3.3, 11.45
    b1 = f.b * np.exp(np.log(f.lam) / dt * t1)
    Ua = oracle.integrate(f.phi, f.lam, f.b, [t1 + t2], dt=dt)
    Ub = oracle.integrate(f.phi, f.lam, b1, [t2], dt=dt)
    assert field_errors(Ub, Ua)["max_frame"] <= 1e-12


def test_project_recovers_amplitudes():
    """z = Phi^+ u (eq. projection) applied to the k = 0 reconstruction returns b."""
    cfg = synth.config("c1-cf", seed=103)
    g = synth.generate(cfg)
    f = oracle.fit_exact(g.Z, cfg.r)
    u0 = oracle.reconstruct(f.phi, f.lam, f.b, [0])[:, 0]
    z = oracle.project(f.phi, u0)
    assert np.allclose(z, f.b, rtol=1e-10, atol=1e-12)


# ------------------------------------------------------------------ adjoint
def _small_problem(seed=21, N=40, r=6, ncols=9):
    rng = np.random.default_rng(seed)
    phi = rng.standard_normal((N, r)) + 1j * rng.standard_normal((N, r))
    lam = synth.draw_eigs(rng, r, 0.9)
    b = synth.draw_amplitudes(rng, r)
    Xt = rng.standard_normal((N, ncols))
    ks = np.arange(ncols)
    return phi, lam, b, Xt, ks


def test_adjoint_matches_autograd():
    torch = pytest.importorskip("torch")
    phi, lam, b, Xt, ks = _small_problem()
    L, gl, gb = oracle.loss_grad(phi, lam, b, Xt, ks)
    tl = torch.tensor(lam, dtype=torch.complex128, requires_grad=True)
    tb = torch.tensor(b, dtype=torch.complex128, requires_grad=True)
    tphi = torch.tensor(phi, dtype=torch.complex128)
    tk = torch.tensor(ks, dtype=torch.float64)
    P = torch.exp(torch.outer(torch.log(tl), tk.to(torch.complex128))) * tb[:, None]
    R = torch.tensor(Xt) - (tphi @ P).real
    Lt = (R * R).sum()
    Lt.backward()
    assert abs(L - Lt.item()) <= 1e-12 * abs(L)
    assert np.allclose(gl, tl.grad.numpy(), rtol=1e-10, atol=1e-10)
    assert np.allclose(gb, tb.grad.numpy(), rtol=1e-10, atol=1e-10)


def test_adjoint_matches_finite_differences():
    """Central differences (h = 1e-6) on Re and Im parts separately."""
    phi, lam, b, Xt, ks = _small_problem(seed=22)
    _, gl, gb = oracle.loss_grad(phi, lam, b, Xt, ks)
    h = 1e-6
    for which, g in (("lam", gl), ("b", gb)):
        for i in range(len(lam)):
            for unit in (1.0, 1j):
                lp, ln, bp, bn = lam.copy(), lam.copy(), b.copy(), b.copy()
                if which == "lam":
                    lp[i] += h * unit
                    ln[i] -= h * unit
                else:
                    bp[i] += h * unit
                    bn[i] -= h * unit
                fd = (oracle.loss(phi, lp, bp, Xt, ks) - oracle.loss(phi, ln, bn, Xt, ks)) / (2 * h)
                an = g[i].real if unit == 1.0 else g[i].imag
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (which, i, unit, fd, an)


def test_loss_zero_at_exact_model():
    cfg = synth.config("c1-cf", seed=102)
    g = synth.generate(cfg)
    f = oracle.fit_exact(g.Z, cfg.r)
    ks = np.arange(cfg.m)
    L, gl, gb = oracle.loss_grad(f.phi, f.lam, f.b, g.Z, ks)
    assert L <= 1e-20 * np.sum(g.Z ** 2)
    assert np.max(np.abs(gb)) <= 1e-8


# ------------------------------------------------------------------ metrics
def test_metrics_invariant_to_order_and_folding():
    rng = np.random.default_rng(2)
    lam = synth.draw_eigs(rng, 10, 0.9)
    perm = rng.permutation(10)
    assert eig_errors(lam[perm], lam)["max_rel"] == 0.0
    phi = rng.standard_normal((8, 2)) + 1j * rng.standard_normal((8, 2))
    folded = np.stack([phi[:, 0].real, phi[:, 0].imag, phi[:, 1].real], axis=1)
    cm = oracle.complex_modes_from_folded(folded, [1, 2, 0])
    assert np.allclose(cm[:, 0], phi[:, 0]) and np.allclose(cm[:, 1], np.conj(phi[:, 0]))
    assert np.allclose(cm[:, 2], phi[:, 1].real)


def test_canonical_order():
    lam = np.array([0.9 * np.exp(-0.3j), 0.5, 0.9 * np.exp(0.3j), 0.95])
    o = oracle.canonical_order(lam)
    assert list(o) == [3, 1, 2, 0]


# ---------------------------------------------- planted mistakes are caught
def test_planted_missing_sigma_inverse_is_caught(monkeypatch):
    """Dropping S_r^-1 from the reduced operator must break the closed-form pin."""
    import oracle.dmd as od
    monkeypatch.setattr(od, "reduced_operator", lambda UtXp, V, s: UtXp @ V)
    cfg = synth.config("c1-cf", seed=102)
    g = synth.generate(cfg)
    f = od.fit_exact(g.Z, cfg.r)
    assert eig_errors(f.lam, _truth(g))["max_rel"] > 1e-3


def test_planted_gradient_sign_is_caught(monkeypatch):
    """A dropped conjugate in the gradient must disagree with finite differences."""
    import oracle.dmd as od
    phi, lam, b, Xt, ks = _small_problem(seed=23)
    real = od.loss_grad
    monkeypatch.setattr(od, "loss_grad", lambda *a: (lambda L, gl, gb: (L, np.conj(gl), gb))(*real(*a)))
    _, gl, _ = od.loss_grad(phi, lam, b, Xt, ks)
    h = 1e-6
    lp, ln = lam.copy(), lam.copy()
    lp[0] += 1j * h
    ln[0] -= 1j * h
    fd = (od.loss(phi, lp, b, Xt, ks) - od.loss(phi, ln, b, Xt, ks)) / (2 * h)
    assert abs(fd - gl[0].imag) > 1e-3 * max(1.0, abs(fd))


def test_planted_swapped_snapshots_is_caught(monkeypatch):
    """Swapping X and X' (fitting the backward map) must break the closed-form pin."""
    import oracle.dmd as od
    real = od.split_snapshots
    monkeypatch.setattr(od, "split_snapshots", lambda Z: real(Z)[::-1])
    cfg = synth.config("c1-cf", seed=103)
    g = synth.generate(cfg)
    f = od.fit_exact(g.Z, cfg.r)
    assert eig_errors(f.lam, _truth(g))["max_rel"] > 1e-3


def test_planted_wrong_real_part_is_caught(monkeypatch):
    """Taking Im instead of Re of the mode sum must break the rebuild pin."""
    import oracle.dmd as od
    monkeypatch.setattr(od, "reconstruct", lambda phi, lam, b, ks: (
        np.asarray(phi) @ (od.powers(lam, ks) * np.asarray(b)[:, None])).imag)
    cfg = synth.config("c1-cf", seed=102)
    g = synth.generate(cfg)
    f = od.fit_exact(g.Z, cfg.r)
    U = od.reconstruct(f.phi, f.lam, f.b, np.arange(cfg.m))
    assert field_errors(U, g.Z)["max_frame"] > 1e-3


def test_planted_cluster_without_dt_is_caught(monkeypatch):
    """Comparing arg(lambda) instead of arg(lambda)/dt with the cut must fail the cluster pin."""
    import oracle.dmd as od
    real = od.frequency_clusters
    monkeypatch.setattr(od, "frequency_clusters", lambda lam, dt, cut=0.01: real(lam, 1.0, cut))
    th = np.array([0.0049, 0.0051])
    assert list(od.frequency_clusters(0.9 * np.exp(1j * th), 0.5)) != [0, 1]


def test_planted_edit_without_imaginary_unit_is_caught(monkeypatch):
    """The printed form cos + sin (no i) must fail the squaring pin."""
    import oracle.dmd as od
    real = od.edit_modes

    def garbled(lam, b, dt, w, s_re, c_re, s_im):
        l2, b2 = real(lam, b, dt, w, s_re, c_re, s_im)
        return np.abs(l2) * (np.cos(np.angle(l2)) + np.sin(np.angle(l2))), b2
    monkeypatch.setattr(od, "edit_modes", garbled)
    lam, b, dt = _edit_case()
    l2, _ = od.edit_modes(lam, b, dt, 1.0, 2.0, 0.0, 2.0)
    assert np.max(np.abs(l2 - lam * lam) / np.abs(lam * lam)) > 1e-3


def test_planted_rollout_without_dt_is_caught(monkeypatch):
    """Dropping dt from the forcing term must fail the geometric-series pin."""
    import oracle.dmd as od
    real = od.rollout
    monkeypatch.setattr(od, "rollout", lambda phi, lam, z0, F=None, dt=1.0, steps=None: real(phi, lam, z0, F, 1.0, steps))
    _geometric_check(od, expect_pass=False)


def _geometric_check(od, expect_pass=True):
    cfg = synth.config("c1-cf", seed=103)
    g = synth.generate(cfg)
    f = od.fit_exact(g.Z, cfg.r)
    c = _paired_vector(np.random.default_rng(4), f.lam)
    F = np.repeat((f.phi @ c).real[:, None], 25, axis=1)
    Z, _ = od.rollout(f.phi, f.lam, f.b, F, dt=0.4)
    s = np.arange(26)[:, None]
    expect = f.lam ** s * f.b + 0.4 * (1 - f.lam ** s) / (1 - f.lam) * c
    ok = np.max(np.abs(Z - expect)) <= 1e-10 * np.max(np.abs(expect))
    assert ok == expect_pass


def test_planted_swapped_selection_is_caught(monkeypatch):
    """Taking the evolved state for the low-order modes (S^L and S^H swapped) must fail the
    zero-guide pin."""
    import oracle.dmd as od
    real = od.upsample_evolve
    swapped = lambda phi, lam, h0, L, low: real(phi, lam, h0, L, ~np.asarray(low))
    monkeypatch.setattr(od, "upsample_evolve", swapped)
    monkeypatch.setattr(oracle, "upsample_evolve", swapped)
    with pytest.raises(AssertionError):
        test_upsample_guide_in_span_and_zero_guide()


def test_amplitude_weights_hand_case_and_invariance():
    """w_i = |b_i| ||phi_i||: the size of mode i's term phi_i b_i, the weight of the
    amplitude-weighted eigenvalue error.  Pinned by a hand-computed case, by the scale
    freedom of an eigenvector (phi_i -> c phi_i, b_i -> b_i / c leaves the model and so the
    weight unchanged; a weight from |b| or ||phi|| alone changes), and by the norm of the
    single-mode field at k = 0 for a real mode."""
    phi = np.array([[3.0, 0.0], [4.0, 0.0], [0.0, 1.0]], dtype=np.complex128)
    b = np.array([2j, -0.5])
    assert np.allclose(oracle.amplitude_weights(phi, b), [10.0, 0.5], rtol=0, atol=1e-15)
    rng = np.random.default_rng(11)
    phi = rng.standard_normal((40, 6)) + 1j * rng.standard_normal((40, 6))
    b = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    c = rng.standard_normal(6) * 3 + 1j * rng.standard_normal(6)
    w = oracle.amplitude_weights(phi, b)
    assert np.allclose(oracle.amplitude_weights(phi * c, b / c), w, rtol=1e-13)
    assert not np.allclose(np.abs(b / c), np.abs(b), rtol=1e-3)      # |b| alone would move
    # a real mode: its weight is the norm of its field at k = 0
    phr = rng.standard_normal((40, 1))
    br = np.array([-1.7])
    u0 = oracle.reconstruct(phr, np.array([0.9]), br, np.array([0]))[:, 0]
    assert abs(oracle.amplitude_weights(phr, br)[0] - np.linalg.norm(u0)) <= 1e-13 * np.linalg.norm(u0)


def test_weighted_eig_error_follows_the_weights():
    """A large eigenvalue error on a mode of negligible weight hardly moves the weighted
    error, while the same error on the heavy mode moves it in full."""
    lam = np.array([0.9 + 0.1j, 0.5 - 0.3j, 0.99])
    w = np.array([1.0, 1e-8, 1.0])
    bad_light = lam + np.array([0, 0.1, 0])
    bad_heavy = lam + np.array([0.1, 0, 0])
    e_light = oracle.eig_errors(bad_light, lam, w)
    e_heavy = oracle.eig_errors(bad_heavy, lam, w)
    assert e_light["weighted_rel"] < 1e-8 and e_light["max_rel"] > 0.1
    assert abs(e_heavy["weighted_rel"] - 0.1 / np.sum(w * np.abs(lam))) < 1e-12


def test_row_subset_route_matches_full_fit():
    """fit_randomized(rows=...) returns the same eigenvalues, the same modes on the chosen
    rows and the same least-squares amplitudes (normal equations instead of lstsq) as
    the full fit, on an input small enough to hold Phi whole."""
    cfg = synth.Config("rows", (2, 40, 40), 70, 18, 0.95, 1e-4, 314, r=30, p=8, q=2)
    g = synth.generate(cfg)
    Zd = g.Z.astype(np.float64)
    Om = g.Omega.astype(np.float64)
    full = oracle.fit_randomized(Zd, cfg.r, Om, cfg.q)
    rows = np.sort(np.random.default_rng(1).choice(cfg.N, 500, replace=False))
    sub = oracle.fit_randomized(Zd, cfg.r, Om, cfg.q, rows=rows)
    assert np.array_equal(sub.lam, full.lam)
    assert np.allclose(sub.phi, full.phi[rows], rtol=0, atol=1e-13 * np.abs(full.phi).max())
    assert np.allclose(sub.b, full.b, rtol=1e-9, atol=1e-12 * np.abs(full.b).max())
    ks = np.arange(cfg.m)
    U1 = oracle.reconstruct(full.phi[rows], full.lam, full.b, ks)
    U2 = oracle.reconstruct(sub.phi, sub.lam, sub.b, ks)
    assert np.linalg.norm(U1 - U2) <= 1e-10 * np.linalg.norm(U1)
