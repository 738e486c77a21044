"""GPU parity of the batched reconstruction (Sec. 4.4) and arbitrary-time
integration (Sec. 6.1) against the FP64 oracle, through the C ABI.

Tolerances (relative Frobenius error per frame against the FP64 oracle):
  FP64 1e-12; FP32 1e-4 (FP32 products and accumulation over r <= 160 terms,
  expected ~1e-6); BF16X3 1e-4 (split-BF16, ~16 mantissa bits per operand,
  expected ~1e-5); BF16 is reported against 3e-2 only (8 mantissa bits, the
  paper fixes no precision; it cannot meet 1e-4).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import max_frame_rel, model_from_oracle, rank150_fit

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-4, "bf16x3": 1e-4, "bf16": 3e-2}


def _print(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def c1cf_fit():
    cfg = synth.config("c1-cf")
    g = synth.generate(cfg)
    return cfg, g, oracle.fit_exact(g.Z, cfg.r)


def test_reconstruct_fp64_oracle_model(gpu_lib, c1cf_fit):
    cfg, g, f = c1cf_fit
    _print("case: c1-cf oracle model, fp64 reconstruct k=0..99")
    m = model_from_oracle(f, torch.float64)
    ks = np.arange(100)
    U = m.reconstruct(ks, "fp64").cpu().numpy()
    Uo = oracle.reconstruct(f.phi, f.lam, f.b, ks).T
    assert max_frame_rel(U, Uo) <= TOL["fp64"]


@pytest.mark.parametrize("mode", ["fp32", "bf16x3", "bf16"])
def test_reconstruct_fp32_modes_oracle_model(gpu_lib, c1cf_fit, mode):
    cfg, g, f = c1cf_fit
    _print(f"case: c1-cf oracle model, {mode} reconstruct")
    m = model_from_oracle(f, torch.float32)
    ks = np.arange(100)
    U = m.reconstruct(ks, mode).cpu().numpy()
    # the oracle sees the same FP32-rounded modes
    phi32 = m.complex_modes()
    Uo = oracle.reconstruct(phi32, f.lam, f.b, ks).T
    err = max_frame_rel(U, Uo)
    _print(f"  {mode} max-frame rel err {err:.3e}")
    assert err <= TOL[mode]


@pytest.mark.parametrize("N,nc,K", [(8192 + 37, 11, 37), (5000, 3, 1), (130, 16, 130)])
def test_reconstruct_ragged_shapes(gpu_lib, N, nc, K):
    """N not a multiple of the row tile, r not a multiple of 32, odd K, negative k."""
    _print(f"case: ragged N={N} nc={nc} K={K}")
    rng = np.random.default_rng(N + nc)
    phi = synth.orthonormal_modes(rng, N, nc)
    lam = synth.draw_eigs(rng, nc, 0.9)
    b = synth.draw_amplitudes(rng, nc)
    from paper_2502_05339_amd import Model
    ks = rng.integers(-40, 300, size=K)
    for dtype, mode in ((torch.float64, "fp64"), (torch.float32, "fp32"), (torch.float32, "bf16x3")):
        m = Model.from_pairs(phi, lam, b, dtype=dtype)
        U = m.reconstruct(ks, mode).cpu().numpy()
        phic = m.complex_modes()
        Uo = oracle.reconstruct(phic, m.lam_host(), m.b_host(), ks).T
        err = max_frame_rel(U, Uo)
        _print(f"  {mode} err {err:.3e}")
        assert err <= TOL[mode]


def test_reconstruct_real_modes_and_strided_output(gpu_lib):
    """A model with real eigenvalues (kind 0) next to pairs, written into a strided output."""
    _print("case: real + paired modes, strided output")
    rng = np.random.default_rng(3)
    N, nc = 3000, 5
    phi_p = synth.orthonormal_modes(rng, N, nc)
    lam_p = synth.draw_eigs(rng, nc, 0.9)
    b_p = synth.draw_amplitudes(rng, nc)
    from paper_2502_05339_amd import Model
    m = Model.from_pairs(phi_p, lam_p, b_p, dtype=torch.float64)
    # append two real modes by hand
    r = m.r + 2
    m2 = Model.empty(N, r, torch.float64, "cuda")
    m2.phi[:, : m.r].copy_(m.phi[:, : m.r])
    real_modes = rng.standard_normal((N, 2))
    m2.phi[:, m.r:r].copy_(torch.from_numpy(real_modes))
    lam = np.concatenate([m.lam_host(), [0.97, -0.5]])
    b = np.concatenate([m.b_host(), [1.5, -0.25]])
    kind = np.concatenate([m.kind_host(), [0, 0]]).astype(np.int32)
    m2.lam.copy_(torch.from_numpy(lam))
    m2.b.copy_(torch.from_numpy(b))
    m2.kind.copy_(torch.from_numpy(kind))
    ks = np.arange(-3, 20)
    big = torch.zeros((len(ks), N + 10), dtype=torch.float64, device="cuda")
    out = big[:, :N]
    m2.reconstruct(ks, "fp64", out=out)
    Uo = oracle.reconstruct(m2.complex_modes(), lam, b, ks).T
    assert max_frame_rel(out.cpu().numpy(), Uo) <= 1e-12
    assert torch.count_nonzero(big[:, N:]).item() == 0


def test_reconstruct_c2_shape_sampled_rows(gpu_lib):
    """Full c2 reconstruction shape (N = 131072, r = 150, K = 1000) in the launch
    configuration the benchmark times; the oracle checks a random row sample."""
    cfg = synth.config("c2")
    _print("case: c2-shaped synthetic model, K=1000, bf16x3/fp32/fp64, sampled rows")
    phi, lam, b = synth.synthetic_model(cfg, np.float64)
    from paper_2502_05339_amd import Model
    ks = np.arange(1000)
    rows = np.sort(np.random.default_rng(7).choice(cfg.N, 2048, replace=False))
    for dtype, mode in ((torch.float32, "bf16x3"), (torch.float32, "fp32"), (torch.float64, "fp64")):
        m = Model.from_pairs(phi, lam, b, dtype=dtype)
        U = m.reconstruct(ks, mode)
        Us = U[:, torch.from_numpy(rows).cuda()].cpu().numpy()
        Uo = oracle.reconstruct(m.complex_modes(rows), m.lam_host(), m.b_host(), ks).T
        err = max_frame_rel(Us, Uo)
        _print(f"  {mode} err {err:.3e}")
        assert err <= TOL[mode]
        del U


def test_integrate_matches_oracle_and_integer_steps(gpu_lib, c1cf_fit):
    cfg, g, f = c1cf_fit
    _print("case: integrate (real t, dt = 0.5) vs oracle and vs reconstruct")
    m = model_from_oracle(f, torch.float64, dt=0.5)
    ts = np.array([0.0, 0.25, 1.0, 3.3, 17.75, -2.5])
    U = m.integrate(ts, "fp64").cpu().numpy()
    Uo = oracle.integrate(f.phi, f.lam, f.b, ts, dt=0.5).T
    assert max_frame_rel(U, Uo) <= 1e-12
    ks = np.array([0, 2, 7, 40])
    Ui = m.integrate(ks * 0.5, "fp64").cpu().numpy()
    Uk = m.reconstruct(ks, "fp64").cpu().numpy()
    assert max_frame_rel(Ui, Uk) <= 1e-13


def test_time_reversal_round_trip(gpu_lib, c1cf_fit):
    """Negative k runs the reduced model backwards (Sec. 6.2): projecting frame k and
    stepping -k returns frame 0."""
    cfg, g, f = c1cf_fit
    _print("case: reversal round trip through project + negative k")
    m = model_from_oracle(f, torch.float64)
    k = 25
    uk = m.reconstruct([k], "fp64")[0].contiguous()
    z = m.project(uk)
    from paper_2502_05339_amd import Model
    m2 = Model(phi=m.phi, lam=m.lam, b=z, sigma=m.sigma, kind=m.kind, info=m.info)
    u0 = m2.reconstruct([-k], "fp64").cpu().numpy()
    U0 = m.reconstruct([0], "fp64").cpu().numpy()
    assert max_frame_rel(u0, U0) <= 1e-10


def test_project_matches_oracle(gpu_lib, c1cf_fit):
    cfg, g, f = c1cf_fit
    _print("case: project z = Phi^+ u")
    m = model_from_oracle(f, torch.float64)
    u = torch.from_numpy(np.ascontiguousarray(g.Z[:, 5])).cuda()
    z = m.project(u).cpu().numpy()
    zo = oracle.project(m.complex_modes(), g.Z[:, 5])
    assert np.max(np.abs(z - zo)) <= 1e-9 * np.max(np.abs(zo))


def test_project_rank150_matches_oracle(gpu_lib):
    """z = Phi^+ u for a rank-150 FP64 model (one column against 150 modes)."""
    cfg, g, f = rank150_fit()
    _print("case: project z = Phi^+ u, r = 150")
    m = model_from_oracle(f, torch.float64)
    u = torch.from_numpy(np.ascontiguousarray(g.Z[:, 7])).cuda()
    z = m.project(u).cpu().numpy()
    zo = oracle.project(m.complex_modes(), g.Z[:, 7])
    assert np.max(np.abs(z - zo)) <= 1e-9 * np.max(np.abs(zo))


def test_reconstruct_deterministic(gpu_lib):
    _print("case: bitwise repeatability")
    cfg = synth.config("c2")
    rng = np.random.default_rng(1)
    phi = synth.orthonormal_modes(rng, 20000, 40)
    lam = synth.draw_eigs(rng, 40, 0.95)
    b = synth.draw_amplitudes(rng, 40)
    from paper_2502_05339_amd import Model
    m = Model.from_pairs(phi, lam, b, dtype=torch.float32)
    a = m.reconstruct(np.arange(300), "bf16x3").clone()
    c = m.reconstruct(np.arange(300), "bf16x3")
    assert torch.equal(a, c)


@pytest.mark.parametrize("N,nc,K", [(8192 + 37, 11, 37), (130, 16, 130), (5000, 75, 70)])
def test_every_bf16_tile_candidate(gpu_lib, tmp_path, N, nc, K):
    """Every tile candidate of the BF16 modes (forced through the tuning-cache loader) on
    ragged shapes: N not a multiple of any row tile, K not a multiple of any frame chunk,
    ranks 22, 32 and 150 (one to ten 16-mode groups)."""
    from paper_2502_05339_amd import Model, _lib
    import paper_2502_05339_amd as dmd
    _print(f"case: every BF16 tile candidate N={N} nc={nc} K={K}")
    rng = np.random.default_rng(N + 3 * nc)
    phi = synth.orthonormal_modes(rng, N, nc)
    lam = synth.draw_eigs(rng, nc, 0.9)
    b = synth.draw_amplitudes(rng, nc)
    ks = rng.integers(-20, 200, size=K)
    m = Model.from_pairs(phi, lam, b, dtype=torch.float32)
    Uo = oracle.reconstruct(m.complex_modes(), m.lam_host(), m.b_host(), ks).T
    rp = int(_lib.lib().dmd_phi_ld(2 * nc))
    key = f"{rp} {int(N).bit_length() - 1} {int(K).bit_length() - 1}"
    L = _lib.lib()
    try:
        for mode in ("bf16x3", "bf16"):
            mc = dmd.api.RECON_MODES[mode]
            for cfg in range(6):
                path = tmp_path / f"tune_{mode}_{cfg}.txt"
                path.write_text(f"{mc} {key} {cfg} 0.0\n")
                assert L.dmd_autotune_load(str(path).encode()) == 0
                err = max_frame_rel(m.reconstruct(ks, mode).cpu().numpy(), Uo)
                _print(f"  {mode} candidate {cfg}: err {err:.3e}")
                assert err <= TOL[mode]
    finally:
        # back to the default candidate for this shape class
        path = tmp_path / "tune_default.txt"
        path.write_text("".join(f"{dmd.api.RECON_MODES[md]} {key} 0 0.0\n" for md in ("bf16x3", "bf16")))
        L.dmd_autotune_load(str(path).encode())
