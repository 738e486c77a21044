"""GPU checks of the C ABI's boundary behaviour: the device status word of the
coefficient pass (Sec. 6.1 defines Omega = Log(lambda) / dt, undefined at lambda = 0;
powers beyond the output type's range), model files written and read by the library,
a fit into an exactly sized workspace with the widest valid ldphi, and the shifted
CholeskyQR retry on a sketch whose Gram is numerically singular."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import max_frame_rel, model_from_oracle

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _tiny_model(lam, b, dtype=torch.float32):
    """A model of real modes (kind 0) on N = 64 rows with the given eigenvalues/amplitudes."""
    import paper_2502_05339_amd as dmd
    r = len(lam)
    rng = np.random.default_rng(9)
    m = dmd.Model.empty(64, r, dtype, "cuda")
    phi = rng.standard_normal((64, r))
    m.phi[:, :r].copy_(torch.from_numpy(phi).to(dtype))
    m.lam.copy_(torch.from_numpy(np.asarray(lam, dtype=np.complex128)))
    m.b.copy_(torch.from_numpy(np.asarray(b, dtype=np.complex128)))
    return m, phi


def test_status_domain_for_zero_eigenvalue(gpu_lib):
    """lambda = 0: k = 0 gives 0^0 = 1, k > 0 gives 0, both fine; k < 0 or a fractional
    time is DMD_ERR_DOMAIN in the status word (the call itself is asynchronous)."""
    import paper_2502_05339_amd as dmd
    _print("case: status word, lambda = 0")
    m, phi = _tiny_model([0.0, 0.9], [1.0, 2.0])
    U = m.reconstruct([0, 1, 3], "fp32", check_status=True).cpu().numpy()
    ref = oracle.reconstruct(phi.astype(np.complex128), np.array([0.0, 0.9]), np.array([1.0, 2.0]), np.array([0, 1, 3]))
    assert max_frame_rel(U, ref.T) <= 1e-6
    with pytest.raises(dmd.DMDError) as ei:
        m.reconstruct([2, -1], "fp32", check_status=True)
    assert ei.value.code == 8
    with pytest.raises(dmd.DMDError) as ei:
        m.integrate([0.5], "fp32", check_status=True)
    assert ei.value.code == 8
    # integer times through integrate are fine, and the word is cleared by the next call
    m.integrate([0.0, 2.0], "fp32", check_status=True)


def test_status_overflow(gpu_lib):
    """|b| |lambda|^k past FP32's range (2^200) is DMD_ERR_OVERFLOW for FP32 output and
    fine in FP64; past FP64's range (2^1100) it is DMD_ERR_OVERFLOW there as well."""
    import paper_2502_05339_amd as dmd
    _print("case: status word, overflow")
    m, _ = _tiny_model([2.0, 0.5], [1.0, 1.0])
    m.reconstruct([0, 100], "fp32", check_status=True)                 # 2^100 = 1.3e30 fits FP32
    with pytest.raises(dmd.DMDError) as ei:
        m.reconstruct([0, 200], "fp32", check_status=True)
    assert ei.value.code == 9
    m64, _ = _tiny_model([2.0, 0.5], [1.0, 1.0], torch.float64)
    m64.reconstruct([200], "fp64", check_status=True)
    with pytest.raises(dmd.DMDError) as ei:
        m64.reconstruct([1100], "fp64", check_status=True)
    assert ei.value.code == 9
    # a growing state of the forced roll-out overflows FP32 frames as well
    states, _ = dmd.rollout(m, steps=200, mode="fp32")
    assert dmd.status_word(dmd.api._ws_cache[(str(m.phi.device), dmd.api._stream())]) == 9


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_model_file_round_trip(gpu_lib, tmp_path, dtype):
    """A fitted model written by dmd_model_save and read by dmd_model_load reconstructs
    the same frames bit for bit; a corrupted byte is refused."""
    import paper_2502_05339_amd as dmd
    _print(f"case: model file round trip {dtype}")
    cfg = synth.Config("io", (2, 32, 32), 40, 6, 0.95, 1e-5, 77, r=12, p=4, q=1,
                       dtype="f64" if dtype == torch.float64 else "f32")
    g = synth.generate(cfg)
    Z = torch.from_numpy(np.ascontiguousarray(g.Z.T)).cuda()
    om = torch.from_numpy(np.ascontiguousarray(g.Omega.T)).cuda()
    m = dmd.fit(Z, cfg.r, p=cfg.p, q=cfg.q, omega=om, precision="mixed" if dtype == torch.float32 else "fp64",
                dt=0.25)
    path = str(tmp_path / "model.dmd")
    m.save(path)
    n, r, code, dt = dmd.Model.file_info(path)
    assert (n, r, dt) == (cfg.N, cfg.r, 0.25)
    m2 = dmd.Model.load(path)
    assert torch.equal(m2.phi, m.phi) and torch.equal(m2.lam, m.lam) and torch.equal(m2.b, m.b)
    assert torch.equal(m2.kind, m.kind) and torch.equal(m2.sigma, m.sigma) and m2.dt == 0.25
    mode = "fp64" if dtype == torch.float64 else "bf16x3"
    ks = np.arange(50)
    assert torch.equal(m2.reconstruct(ks, mode), m.reconstruct(ks, mode))
    raw = bytearray(open(path, "rb").read())
    raw[100] ^= 0x40
    bad = str(tmp_path / "bad.dmd")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(dmd.DMDError) as ei:
        dmd.Model.load(bad)
    assert ei.value.code == 12


def test_fit_widest_ldphi_exact_workspace_guard_band(gpu_lib):
    """Separate X and X' buffers (no shifted view), a model with ldphi = 192 and a
    workspace of exactly the queried size followed by a guard band: the guard band is
    untouched and the model equals the one fitted with the minimal ldphi."""
    import paper_2502_05339_amd as dmd
    from paper_2502_05339_amd import _lib
    _print("case: ldphi = 192 into an exactly sized workspace")
    cfg = synth.Config("ld192", (2, 48, 48), 90, 40, 0.95, 1e-4, 88, r=70, p=10, q=1)
    g = synth.generate(cfg)
    Z = torch.from_numpy(np.ascontiguousarray(g.Z.T)).cuda()
    X, Xp = Z[:-1].clone(), Z[1:].clone()
    om = torch.from_numpy(np.ascontiguousarray(g.Omega.T)).cuda()
    ref = dmd.fit(None, cfg.r, X=X, Xp=Xp, p=cfg.p, q=cfg.q, omega=om)
    L = _lib.lib()
    o = dmd.fit_opts(cfg.r, cfg.p, cfg.q, "mixed", om)
    nb = ctypes.c_size_t(0)
    assert L.dmd_fit_workspace_size(cfg.N, cfg.m - 1, 0, ctypes.byref(o), ctypes.byref(nb)) == 0
    guard = 1 << 20
    buf = torch.full((nb.value + guard,), 0x5A, dtype=torch.uint8, device="cuda")
    m = dmd.Model.empty(cfg.N, cfg.r, torch.float32, "cuda")
    m.phi = torch.zeros((cfg.N, 192), dtype=torch.float32, device="cuda")
    ms = m.struct()
    assert ms.ldphi == 192
    st = L.dmd_fit(dmd.api._stream(), X.data_ptr(), Xp.data_ptr(), cfg.N, cfg.m - 1, X.stride(0), Xp.stride(0), 0,
                   ctypes.byref(o), buf.data_ptr(), nb.value, ctypes.byref(ms))
    assert st == 0
    torch.cuda.synchronize()
    assert bool(torch.all(buf[nb.value:] == 0x5A).item())
    assert torch.allclose(m.lam, ref.lam, rtol=1e-6, atol=1e-7)
    assert torch.allclose(m.phi[:, : cfg.r], ref.phi[:, : cfg.r], rtol=1e-5, atol=1e-6)
    assert bool(torch.all(m.phi[:, cfg.r:] == 0).item())


def test_shifted_cholesky_retry_fires_and_recovers(gpu_lib):
    """FP64 randomized fit of noise-free data whose pair amplitudes fall by 10x per pair
    (13 pairs, sketch l = 26): the sketch's condition number is near 1e13, so the FP64
    Gram of the first CholeskyQR pass is numerically singular and its Cholesky breaks
    down.  The shifted retry (shifted CholeskyQR3) must fire (info[3] > 0) and the fit
    must still match the Householder-QR twin on the modes that carry the data."""
    import paper_2502_05339_amd as dmd
    _print("case: shifted CholeskyQR retry")
    rng = np.random.default_rng(4242)
    N, m, nc = 4608, 60, 13
    modes = synth.orthonormal_modes(rng, N, nc)
    lam = synth.draw_eigs(rng, nc, 0.97, jitter=True)
    b = synth.draw_amplitudes(rng, nc) * 10.0 ** (-np.arange(nc))
    Z = synth.snapshots(modes, lam, b, m, 0.0, rng)
    r, p, q = 16, 10, 1
    Om = synth.sketch(4242, m, r + p, dtype=np.float64)
    Zt = torch.from_numpy(np.ascontiguousarray(Z.T)).cuda()
    om = torch.from_numpy(np.ascontiguousarray(Om.T)).cuda()
    mod = dmd.fit(Zt, r, p=p, q=q, omega=om, precision="fp64")
    retries = int(mod.info[3].item())
    tw = oracle.fit_randomized(Z, r, Om, q)
    w = oracle.amplitude_weights(tw.phi, tw.b)
    ia, ib = oracle.match_eigs(mod.lam_host(), tw.lam)
    d = np.abs(mod.lam_host()[ia] - tw.lam[ib])
    wrel = float(np.sum(w[ib] * d) / np.sum(w[ib] * np.abs(tw.lam[ib])))
    ks = np.arange(m)
    U = mod.reconstruct(ks, "fp64").cpu().numpy()
    Uo = oracle.reconstruct(tw.phi, tw.lam, tw.b, ks).T
    ferr = max_frame_rel(U, Uo)
    _print(f"  shifted retries {retries}, lambda weighted {wrel:.3e}, fields {ferr:.3e}")
    assert retries > 0
    assert np.all(np.isfinite(mod.lam_host()))
    assert wrel <= 1e-4 and ferr <= 1e-6


def test_exactly_singular_sketch_reports_breakdown(gpu_lib):
    """A zero column in the sketch gives an exactly singular Gram that no shift can
    repair (the basis keeps a zero column): the retry fires and the fit reports
    DMD_ERR_CHOL_BREAKDOWN instead of returning eigenvalues."""
    import paper_2502_05339_amd as dmd
    _print("case: exactly singular sketch")
    cfg = synth.Config("sing", (2, 32, 32), 50, 10, 0.95, 1e-4, 99, r=12, p=6, q=1, dtype="f64")
    g = synth.generate(cfg)
    Om = np.array(g.Omega, dtype=np.float64)
    Om[:, 5] = 0.0
    Zt = torch.from_numpy(np.ascontiguousarray(g.Z.T)).cuda()
    om = torch.from_numpy(np.ascontiguousarray(Om.T)).cuda()
    with pytest.raises(dmd.DMDError) as ei:
        dmd.fit(Zt, cfg.r, p=cfg.p, q=cfg.q, omega=om, precision="fp64")
    assert ei.value.code == 5
