"""GPU parity of the fit (Sec. 4.3 randomized SVD, Sec. 3.1 exact DMD) against the
FP64 oracle, through the C ABI.

Gates (the tolerances come from the target accuracy of the mixed-precision
path: 1e-5 relative in lambda and 1e-4 in the fields):
  G1  FP64 exact path on the noise-free closed form: lambda <= 1e-10 against the
      prescribed eigenvalues, snapshots rebuilt to <= 1e-12.
  G2  mixed path against the FP64 randomized twin fed the same sketch: fields
      <= 1e-4, amplitude-weighted lambda <= 1e-5.
  G3  mixed path against the exact oracle on the well-posed variant: max-relative
      lambda <= 1e-5, fields <= 1e-4.
Eigenvalue sets are compared after an optimal matching; modes only through the
fields they produce (their scale is not unique).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import max_frame_rel

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _gpu_fit(g, cfg, precision):
    import paper_2502_05339_amd as dmd
    dt = torch.float64 if precision != "mixed" else torch.float32
    Z = torch.from_numpy(np.ascontiguousarray(g.Z.T).astype(np.float64 if dt == torch.float64 else np.float32)).cuda()
    om = None
    if precision != "fp64_exact":
        Om = np.ascontiguousarray(g.Omega.T).astype(np.float64 if dt == torch.float64 else np.float32)
        om = torch.from_numpy(Om).cuda()
    m = dmd.fit(Z, cfg.r, p=cfg.p, q=cfg.q, omega=om, precision=precision)
    return m, Z


def _fields(m, ks, mode, rows=None):
    U = m.reconstruct(ks, mode)
    if rows is not None:
        U = U[:, torch.from_numpy(rows).cuda()]
    return U.cpu().numpy()


def _weights(m):
    phi = m.complex_modes()
    return np.abs(m.b_host()) * np.linalg.norm(phi, axis=0)


@pytest.mark.parametrize("seed", [102, 103, 104])
def test_g1_fp64_exact_closed_form(gpu_lib, seed):
    cfg = synth.config("c1-cf", seed=seed)
    _print(f"case: G1 c1-cf seed {seed}, fp64_exact")
    g = synth.generate(cfg)
    m, Z = _gpu_fit(g, cfg, "fp64_exact")
    truth = np.concatenate([g.lam, np.conj(g.lam)])
    e = oracle.eig_errors(m.lam_host(), truth)
    _print(f"  lambda max rel {e['max_rel']:.3e}")
    assert e["max_rel"] <= 1e-10
    U = _fields(m, np.arange(cfg.m), "fp64")
    err = max_frame_rel(U, g.Z.T)
    _print(f"  rebuild max-frame {err:.3e}")
    assert err <= 1e-12
    kind = m.kind_host()
    assert set(kind.tolist()) <= {0, 1, 2}
    lam = m.lam_host()
    assert np.all(np.diff(np.abs(np.angle(lam))) >= -1e-12)      # canonical order


def test_fp64_exact_vs_oracle_literal_c1(gpu_lib):
    """Literal c1 (noise 1e-8, ill-conditioned frequencies, sigma_16 / sigma_1 ~ 2e-7): the
    exact path's triangular-factor route keeps relative accuracy about n u kappa
    (64 x 1.1e-16 x 5e6 = 3.5e-8) in every kept singular value, so all 16 are held to 1e-7
    against the oracle's LAPACK SVD, and the fields to 1e-8 on the fitted frames and 1e-6
    with extrapolation (a Gram route would lose u kappa^2 ~ 3e-3 in sigma_16)."""
    cfg = synth.config("c1")
    _print("case: c1 literal fp64_exact vs oracle")
    g = synth.generate(cfg)
    m, Z = _gpu_fit(g, cfg, "fp64_exact")
    f = oracle.fit_exact(g.Z, cfg.r)
    ks = np.arange(cfg.K)
    U = _fields(m, ks, "fp64")
    Uo = oracle.reconstruct(f.phi, f.lam, f.b, ks).T
    fitted = max_frame_rel(U[: cfg.m], Uo[: cfg.m])
    extrap = max_frame_rel(U, Uo)
    _print(f"  fields vs oracle: fitted frames {fitted:.3e}, with extrapolated frames {extrap:.3e}")
    s = m.sigma.cpu().numpy()
    srel = np.abs(s - f.sigma) / f.sigma
    _print(f"  sigma relative errors: max {np.max(srel):.3e} (sigma_r / sigma_1 = {f.sigma[-1] / f.sigma[0]:.2e})")
    assert np.max(srel) <= 1e-7
    assert fitted <= 1e-8
    assert extrap <= 1e-6


def _small_randomized_cfg(sigma=1e-4, seed=211, jitter=False):
    return synth.Config("c2-small", (2, 96, 96), 120, 30, 0.95, sigma, seed, r=60, p=10, q=2, jitter=jitter)


@pytest.mark.parametrize("precision,tol_lam,tol_field", [("mixed", 1e-5, 1e-4), ("fp64", 1e-9, 1e-9)])
def test_randomized_vs_twin_small(gpu_lib, precision, tol_lam, tol_field):
    cfg = _small_randomized_cfg()
    _print(f"case: small randomized {precision} vs FP64 twin")
    g = synth.generate(cfg)
    if precision == "fp64":
        g.Omega = g.Omega.astype(np.float64)
    m, Z = _gpu_fit(g, cfg, precision)
    Zd = g.Z.astype(np.float64)
    tw = oracle.fit_randomized(Zd, cfg.r, g.Omega.astype(np.float64), cfg.q)
    e = oracle.eig_errors(m.lam_host(), tw.lam, weights=None)
    w = oracle.amplitude_weights(tw.phi, tw.b)
    ia, ib = oracle.match_eigs(m.lam_host(), tw.lam)
    d = np.abs(m.lam_host()[ia] - tw.lam[ib])
    wrel = float(np.sum(w[ib] * d) / np.sum(w[ib] * np.abs(tw.lam[ib])))
    ks = np.arange(cfg.m)
    U = _fields(m, ks, "fp64" if precision == "fp64" else "fp32")
    Uo = oracle.reconstruct(tw.phi, tw.lam, tw.b, ks).T
    ferr = max_frame_rel(U, Uo)
    _print(f"  lambda max {e['max_rel']:.3e} weighted {wrel:.3e} fields {ferr:.3e}")
    assert wrel <= tol_lam
    assert ferr <= tol_field
    assert int(m.info[0].item()) == 0


@pytest.mark.parametrize("grid", [(3, 61, 67), (2, 50, 98)])
@pytest.mark.parametrize("precision,tol_lam,tol_field", [("mixed", 1e-5, 1e-4), ("fp64", 1e-9, 1e-9)])
def test_randomized_vs_twin_ragged_n(gpu_lib, precision, tol_lam, tol_field, grid):
    """N = 3*61*67 = 12261 (odd): the products take their guarded paths (no 16-byte loads
    for N not a multiple of 4, ragged last row chunks).  N = 2*50*98 = 9800 (a multiple of
    4, not of the 128-row tile of the NN product): the 16-byte path whose last row tile
    reads clamped rows and zeroes them.  Both against the FP64 twin."""
    cfg = synth.Config("ragged", grid, 90, 20, 0.95, 1e-4, 223, r=36, p=8, q=2)
    _print(f"case: ragged N={cfg.N} randomized {precision} vs FP64 twin")
    g = synth.generate(cfg)
    if precision == "fp64":
        g.Omega = g.Omega.astype(np.float64)
    m, Z = _gpu_fit(g, cfg, precision)
    tw = oracle.fit_randomized(g.Z.astype(np.float64), cfg.r, g.Omega.astype(np.float64), cfg.q)
    w = oracle.amplitude_weights(tw.phi, tw.b)
    ia, ib = oracle.match_eigs(m.lam_host(), tw.lam)
    d = np.abs(m.lam_host()[ia] - tw.lam[ib])
    wrel = float(np.sum(w[ib] * d) / np.sum(w[ib] * np.abs(tw.lam[ib])))
    ks = np.arange(cfg.m)
    U = _fields(m, ks, "fp64" if precision == "fp64" else "fp32")
    Uo = oracle.reconstruct(tw.phi, tw.lam, tw.b, ks).T
    ferr = max_frame_rel(U, Uo)
    _print(f"  lambda weighted {wrel:.3e} fields {ferr:.3e}")
    assert wrel <= tol_lam
    assert ferr <= tol_field
    assert int(m.info[0].item()) == 0


def test_g3_mixed_vs_exact_well_posed_c2(gpu_lib):
    """Full-size c2-wp (N = 131072, m = 200, r = 150, p = 10, q = 2)."""
    cfg = synth.config("c2-wp")
    _print("case: G3 c2-wp mixed vs exact oracle (full size)")
    g = synth.generate(cfg)
    m, Z = _gpu_fit(g, cfg, "mixed")
    f = oracle.fit_exact(g.Z.astype(np.float64), cfg.r)
    e = oracle.eig_errors(m.lam_host(), f.lam)
    rows = np.sort(np.random.default_rng(5).choice(cfg.N, 4096, replace=False))
    ks = np.arange(cfg.m)
    U = _fields(m, ks, "fp32", rows)
    Uo = oracle.reconstruct(f.phi[rows], f.lam, f.b, ks).T
    ferr = max_frame_rel(U, Uo)
    _print(f"  lambda max {e['max_rel']:.3e} fields {ferr:.3e}")
    assert e["max_rel"] <= 1e-5
    assert ferr <= 1e-4


def test_g2_mixed_vs_twin_c2(gpu_lib):
    """Full-size literal c2 (noise 1e-4): the rank-150 cut lies in the noise bulk, so the
    gate is the twin fed the same sketch, with the amplitude-weighted eigenvalue error.
    Most of the twin's eigenvalues are fitted to the noise (148 of 150 lie 1e-3 or more
    from every generating eigenvalue) and move with any perturbation of the data, so each
    one is held to its first-order perturbation bound instead of a fixed tolerance:
    |d lambda_i| <= kappa_i ||dAtilde||, kappa_i = ||y_i|| ||w_i|| / |y_i^H w_i| from the
    twin's eigenvectors, and FP32 operands perturb Atilde = U^T X' V S^-1 by about
    u32 sigma_1 / sigma_r in norm (u32 = 2^-24)."""
    cfg = synth.config("c2")
    _print("case: G2 c2 mixed vs FP64 twin (full size)")
    g = synth.generate(cfg)
    m, Z = _gpu_fit(g, cfg, "mixed")
    tw = oracle.fit_randomized(g.Z.astype(np.float64), cfg.r, g.Omega.astype(np.float64), cfg.q)
    w = oracle.amplitude_weights(tw.phi, tw.b)
    ia, ib = oracle.match_eigs(m.lam_host(), tw.lam)
    d = np.abs(m.lam_host()[ia] - tw.lam[ib])
    wrel = float(np.sum(w[ib] * d) / np.sum(w[ib] * np.abs(tw.lam[ib])))
    rows = np.sort(np.random.default_rng(6).choice(cfg.N, 4096, replace=False))
    ks = np.arange(cfg.m)
    U = _fields(m, ks, "fp32", rows)
    Uo = oracle.reconstruct(tw.phi[rows], tw.lam, tw.b, ks).T
    ferr = max_frame_rel(U, Uo)
    kappa = np.linalg.norm(np.linalg.inv(tw.w), axis=1) * np.linalg.norm(tw.w, axis=0)
    bound = kappa[ib] * 2.0 ** -24 * tw.sigma[0] / tw.sigma[-1]
    _print(f"  lambda weighted {wrel:.3e} max abs {np.max(d):.3e}; largest ratio to the perturbation bound "
           f"{np.max(d / bound):.3f} (kappa {kappa.min():.2f}..{kappa.max():.2f}, sigma_1/sigma_r "
           f"{tw.sigma[0] / tw.sigma[-1]:.1f}); fields {ferr:.3e}")
    assert wrel <= 1e-5
    assert np.all(d <= bound)
    assert ferr <= 1e-4


def test_fit_separate_x_xp_matches_shifted_view(gpu_lib):
    """X and X' passed as separate buffers give the same model as the shifted views of Z."""
    import paper_2502_05339_amd as dmd
    cfg = _small_randomized_cfg(seed=212)
    _print("case: separate X / X' buffers")
    g = synth.generate(cfg)
    m1, Z = _gpu_fit(g, cfg, "mixed")
    X = Z[:-1].clone()
    Xp = Z[1:].clone()
    om = torch.from_numpy(np.ascontiguousarray(g.Omega.T)).cuda()
    m2 = dmd.fit(None, cfg.r, X=X, Xp=Xp, p=cfg.p, q=cfg.q, omega=om)
    assert np.allclose(m1.lam_host(), m2.lam_host(), rtol=1e-6, atol=1e-6)


def test_fit_errors_raise(gpu_lib):
    import paper_2502_05339_amd as dmd
    _print("case: error statuses")
    Z = torch.zeros((20, 1000), dtype=torch.float32, device="cuda")
    om = torch.zeros((30, 19), dtype=torch.float32, device="cuda")
    with pytest.raises(dmd.DMDError) as ei:
        dmd.fit(Z, 25, p=5, omega=om)
    assert ei.value.code == 2
    # rank tolerance: snapshots of a rank-4 system, ask for r = 8 with a tolerance
    rng = np.random.default_rng(0)
    cfg = synth.Config("rk", (4000,), 40, 2, 0.9, 0.0, 5, r=8, p=0, q=0, dtype="f64")
    g = synth.generate(cfg)
    Zd = torch.from_numpy(np.ascontiguousarray(g.Z.T)).cuda()
    with pytest.raises(dmd.DMDError) as ei:
        dmd.fit(Zd, 8, p=0, q=0, precision="fp64_exact", rank_tol=1e-8)
    assert ei.value.code == 6
    # non-finite input, checked on request
    Zn = torch.randn((40, 4000), dtype=torch.float64, device="cuda")
    Zn[3, 17] = float("nan")
    with pytest.raises(dmd.DMDError) as ei:
        dmd.fit(Zn, 4, p=0, q=0, precision="fp64_exact", check_finite=True)
    assert ei.value.code == 4


def test_rank_deficient_sketch_reports_or_recovers(gpu_lib):
    """Noise-free rank-16 data with l = 26: CholeskyQR breaks down; the shifted retry
    either recovers (status 0, info[3] > 0) or the call reports breakdown; it never
    returns silently non-finite eigenvalues."""
    import paper_2502_05339_amd as dmd
    cfg = synth.Config("rd", (2, 48, 48), 60, 8, 0.95, 0.0, 41, r=16, p=10, q=1, jitter=True)
    _print("case: rank-deficient sketch")
    g = synth.generate(cfg)
    try:
        m, Z = _gpu_fit(g, cfg, "mixed")
        assert np.all(np.isfinite(m.lam_host()))
        truth = np.concatenate([g.lam, np.conj(g.lam)])
        e = oracle.eig_errors(m.lam_host(), truth)
        _print(f"  recovered: lambda max {e['max_rel']:.3e}, shifted retries {int(m.info[3].item())}")
        assert e["max_rel"] <= 1e-4
    except dmd.DMDError as err:
        _print(f"  reported: {err}")
        assert err.code == 5


def test_fit_deterministic(gpu_lib):
    cfg = _small_randomized_cfg(seed=213)
    _print("case: bitwise-repeatable fit")
    g = synth.generate(cfg)
    m1, _ = _gpu_fit(g, cfg, "mixed")
    m2, _ = _gpu_fit(g, cfg, "mixed")
    assert torch.equal(m1.phi, m2.phi) and torch.equal(m1.lam, m2.lam) and torch.equal(m1.b, m2.b)


def test_batched_graph_matches_single_fits(gpu_lib):
    """Uneven scenes fitted in one captured graph, replayed three times with eager work
    and synchronisation in between: every replay equals the single-call fits bitwise."""
    import paper_2502_05339_amd as dmd
    _print("case: batched fit graph (3 scenes)")
    scenes, singles = [], []
    for i, (N, m_) in enumerate([(20000, 60), (7777, 45), (33000, 80)]):
        cfg = synth.Config(f"s{i}", (N,), m_, 12, 0.95, 1e-4, 600 + i, r=24, p=6, q=1)
        g = synth.generate(cfg)
        m1, Z = _gpu_fit(g, cfg, "mixed")
        singles.append(m1)
        om = torch.from_numpy(np.ascontiguousarray(g.Omega.T)).cuda()
        scenes.append(dict(Z=Z, r=cfg.r, p=cfg.p, q=cfg.q, omega=om))
    bf = dmd.BatchedFit(scenes, capture=True)
    for rep in range(3):
        for mm in bf.models:
            mm.phi.zero_()
            mm.lam.zero_()
        bf.launch()
        torch.cuda.synchronize()
        _ = torch.randn(1000, device="cuda").sum().item()
        assert bf.statuses() == [0, 0, 0]
        for a, b in zip(bf.models, singles):
            assert torch.equal(a.lam, b.lam) and torch.equal(a.phi, b.phi) and torch.equal(a.b, b.b)
    bf.close()


# Ranks at both ends of the supported range: r = 1 (a single real eigenvalue), r = 2
# and 3 (one pair, a pair plus a real value), r = 149 (odd) and r = 150 with l = r + p =
# 160, the largest sketch, and r = 160 (the eigen-solver limit) with p = 0; the FP64
# products of one column against the modes then span more than 128 columns.  Signals are
# rank 6-180 with
# persistent modes (|lambda| >= 0.99) so the truncation falls between two singular
# values at least 1e-3 apart (relative to the largest): the twin comparison is then well
# conditioned.  The tolerances are the gates of the two precisions.
_EDGE = {
    "r1": (1, 10, 3, 611, 200),
    "r2": (2, 10, 3, 612, 200),
    "r3": (3, 10, 4, 613, 200),
    "r149-l159": (149, 10, 90, 614, 200),
    "r150-l160": (150, 10, 90, 615, 200),
    "r160-p0": (160, 0, 90, 621, 200),
}


def _edge_cfg(name):
    r, p, nc, seed, m = _EDGE[name]
    return synth.Config(f"edge-{name}", (2, 64, 64), m, nc, 0.99, 1e-6, seed, r=r, p=p, q=2, jitter=True)


def _edge_generate(cfg):
    g = synth.generate(cfg)
    if g.Omega is None:                  # p = 0: the sketch still has l = r columns
        g.Omega = synth.sketch(cfg.seed, cfg.m, cfg.l)
    return g


def _twin_errors(m, g, cfg, precision):
    tw = oracle.fit_randomized(g.Z.astype(np.float64), cfg.r, g.Omega.astype(np.float64), cfg.q)
    w = oracle.amplitude_weights(tw.phi, tw.b)
    lam = m.lam_host()
    assert lam.shape == tw.lam.shape
    ia, ib = oracle.match_eigs(lam, tw.lam)
    d = np.abs(lam[ia] - tw.lam[ib])
    wrel = float(np.sum(w[ib] * d) / np.sum(w[ib] * np.abs(tw.lam[ib])))
    ks = np.arange(cfg.m)
    U = _fields(m, ks, "fp64" if precision == "fp64" else "fp32")
    Uo = oracle.reconstruct(tw.phi, tw.lam, tw.b, ks).T
    return wrel, max_frame_rel(U, Uo)


def _check_canonical(m):
    """Modes in canonical order: |arg lambda| non-decreasing, then |lambda| non-increasing;
    a conjugate pair is (kind 1, kind 2) with the Im > 0 member first; real modes kind 0."""
    lam, kind = m.lam_host(), m.kind.cpu().numpy()
    heads = [i for i in range(lam.size) if kind[i] != 2]
    keys = [(abs(np.angle(lam[i])), -abs(lam[i])) for i in heads]
    for a, b in zip(keys, keys[1:]):
        assert a[0] < b[0] + 1e-12 and (a[0] < b[0] - 1e-12 or a[1] <= b[1] + 1e-12), (a, b)
    for i in range(lam.size):
        if kind[i] == 1:
            assert i + 1 < lam.size and kind[i + 1] == 2 and lam[i].imag > 0
            assert lam[i + 1] == np.conj(lam[i])
        elif kind[i] == 0:
            assert lam[i].imag == 0
        else:
            assert i > 0 and kind[i - 1] == 1


@pytest.mark.parametrize("name", list(_EDGE))
def test_rank_extremes_fp64_vs_twin(gpu_lib, name):
    cfg = _edge_cfg(name)
    _print(f"case: rank extreme {name} (r={cfg.r}, l={cfg.l}) fp64 vs FP64 twin")
    g = _edge_generate(cfg)
    g.Omega = g.Omega.astype(np.float64)
    s = np.linalg.svd(g.Z[:, :-1].astype(np.float64), compute_uv=False)
    assert (s[cfg.r - 1] - s[cfg.r]) / s[0] >= 1e-3      # the premise of the tolerances
    m, _ = _gpu_fit(g, cfg, "fp64")
    wrel, ferr = _twin_errors(m, g, cfg, "fp64")
    _print(f"  lambda weighted {wrel:.3e} fields {ferr:.3e}")
    assert int(m.info[0].item()) == 0
    assert wrel <= 1e-9
    assert ferr <= 1e-9
    _check_canonical(m)


@pytest.mark.parametrize("name", ["r150-l160", "r160-p0"])
def test_rank_extreme_mixed_max_sketch(gpu_lib, name):
    cfg = _edge_cfg(name)
    _print(f"case: rank extreme {name} mixed vs FP64 twin")
    g = _edge_generate(cfg)
    m, _ = _gpu_fit(g, cfg, "mixed")
    wrel, ferr = _twin_errors(m, g, cfg, "mixed")
    _print(f"  lambda weighted {wrel:.3e} fields {ferr:.3e}")
    assert int(m.info[0].item()) == 0
    assert wrel <= 1e-5
    assert ferr <= 1e-4


def test_exact_path_max_rank_and_columns(gpu_lib):
    """FP64 exact path at its limits: r = 160 (eigen-solver) from m - 1 = 192 columns
    (Gram eigen-decomposition), against the oracle's SVD-based exact DMD."""
    cfg = synth.Config("edge-exact", (2, 64, 64), 193, 90, 0.99, 1e-6, 618, r=160, p=0, q=0, jitter=True,
                       dtype="f64")
    _print("case: fp64_exact r=160, m-1=192 vs oracle")
    g = synth.generate(cfg)
    s = np.linalg.svd(g.Z[:, :-1], compute_uv=False)
    assert (s[cfg.r - 1] - s[cfg.r]) / s[0] >= 1e-3
    m, _ = _gpu_fit(g, cfg, "fp64_exact")
    f = oracle.fit_exact(g.Z, cfg.r)
    ks = np.arange(cfg.m)
    err = max_frame_rel(_fields(m, ks, "fp64"), oracle.reconstruct(f.phi, f.lam, f.b, ks).T)
    _print(f"  fields vs oracle {err:.3e}")
    assert int(m.info[0].item()) == 0
    assert err <= 1e-9


def test_sketch_beyond_limit_is_unsupported(gpu_lib):
    """l = r + p above the sketch limit is refused before any launch (status 11)."""
    import paper_2502_05339_amd as dmd
    cfg = synth.Config("edge-l161", (2, 32, 32), 200, 80, 0.99, 1e-6, 619, r=150, p=11, q=1, jitter=True)
    g = synth.generate(cfg)
    with pytest.raises(dmd.DMDError) as ei:
        _gpu_fit(g, cfg, "mixed")
    assert ei.value.code == 11


def test_autotune_fit_tiles(gpu_lib, tmp_path):
    """dmd_autotune_fit times every TN tile candidate of the fit's products per shape class and
    keeps the fastest; it writes one cache line per class, a fit after it (tuned tiles) still
    matches the FP64 twin to the mixed path's bar, and the cache file loads again."""
    import paper_2502_05339_amd as dmd
    from paper_2502_05339_amd import _lib
    cfg = _small_randomized_cfg(seed=212)
    _print("case: fit autotuner")
    g = synth.generate(cfg)
    Z = torch.from_numpy(np.ascontiguousarray(g.Z.T)).cuda()
    om = torch.from_numpy(np.ascontiguousarray(g.Omega.T)).cuda()
    path = tmp_path / "tune.txt"
    m1 = dmd.autotune_fit(Z, cfg.r, p=cfg.p, q=cfg.q, omega=om, cache_path=str(path))
    lines = [ln for ln in open(path) if ln.startswith("tn ")]
    _print("  " + "; ".join(ln.strip() for ln in lines))
    assert len(lines) >= 2 and int(m1.info[0].item()) == 0
    m2 = dmd.fit(Z, cfg.r, p=cfg.p, q=cfg.q, omega=om)
    tw = oracle.fit_randomized(g.Z.astype(np.float64), cfg.r, g.Omega.astype(np.float64), cfg.q)
    w = oracle.amplitude_weights(tw.phi, tw.b)
    for m in (m1, m2):
        ia, ib = oracle.match_eigs(m.lam_host(), tw.lam)
        d = np.abs(m.lam_host()[ia] - tw.lam[ib])
        wrel = float(np.sum(w[ib] * d) / np.sum(w[ib] * np.abs(tw.lam[ib])))
        _print(f"  lambda weighted vs twin {wrel:.3e}")
        assert wrel <= 1e-5
    assert _lib.lib().dmd_autotune_load(str(path).encode()) == 0
