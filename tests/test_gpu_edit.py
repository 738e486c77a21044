"""GPU parity of temporal mode editing (Sec. 6.1, eq. edit_temporal) and of the
backward roll-out (Sec. 6.2, eq. reverse_simulation) against the FP64 oracle,
through the C ABI.

Tolerances: edited eigenvalues and amplitudes 1e-13 relative (one log, atan2,
exp and sincos each in FP64; the device and host math libraries differ by a few
ulp); cluster labels bit-exact (both sides compare the FP64 atan2 / dt with the
cut; inputs within 1e-9 of the cut are left out); reconstructions as in the
reconstruction tests (FP64 1e-12, bf16x3 1e-4).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import max_frame_rel, model_from_oracle

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _lams(seed, nc, dt, cut):
    """Conjugate pairs with phases spread across the cut, a positive, a negative and a zero eigenvalue."""
    rng = np.random.default_rng(seed)
    th = np.concatenate([rng.uniform(0.0, 3.0 * cut * dt, nc // 2), rng.uniform(0.0, 3.0, nc - nc // 2)])
    th = th[np.abs(th / dt - cut) > 1e-9]
    mod = rng.uniform(0.8, 1.02, th.size)
    lp = mod * np.exp(1j * th)
    lam = np.concatenate([np.stack([lp, np.conj(lp)], 1).ravel(), [0.97, -0.6, 0.0]])
    bp = rng.standard_normal(th.size) + 1j * rng.standard_normal(th.size)
    b = np.concatenate([np.stack([bp, np.conj(bp)], 1).ravel(), [0.3, -1.1 + 0.2j, 0.5]])
    kind = np.concatenate([np.tile([1, 2], th.size), [0, 0, 0]]).astype(np.int32)
    return lam, b, kind


def _model(lam, b, kind, dt, dtype=torch.float32):
    from paper_2502_05339_amd import Model
    m = Model.empty(64, lam.size, dtype, "cuda", dt)
    m.lam.copy_(torch.from_numpy(lam))
    m.b.copy_(torch.from_numpy(b))
    m.kind.copy_(torch.from_numpy(kind))
    return m


def _rel(a, ref):
    a, ref = np.asarray(a), np.asarray(ref)
    return float(np.max(np.abs(a - ref) / np.maximum(np.abs(ref), 1e-300)))


@pytest.mark.parametrize("seed,nc,dt", [(1, 40, 0.5), (2, 77, 1.0), (3, 3, 0.05)])
def test_cluster_edit_parity(gpu_lib, seed, nc, dt):
    from paper_2502_05339_amd import edit_modes
    cut = 0.01
    lam, b, kind = _lams(seed, nc, dt, cut)
    _print(f"case: cluster edit seed={seed} r={lam.size} dt={dt}")
    m = _model(lam, b, kind, dt)
    params = dict(weight=(0.5, 1.5), re_scale=(1.0, 0.5), re_shift=(0.0, 0.02), im_scale=(1.0, 1.5))
    em, cl = edit_modes(m, freq_cut=cut, **params)
    lo, bo, co = oracle.cluster_edit(lam, b, dt, params["weight"], params["re_scale"], params["re_shift"],
                                     params["im_scale"], cut=cut)
    assert np.array_equal(cl.cpu().numpy(), co)
    assert 0 < co.sum() < co.size
    l2, b2 = em.lam.cpu().numpy(), em.b.cpu().numpy()
    nz = lo != 0
    assert _rel(l2[nz], lo[nz]) <= 1e-13 and np.all(l2[~nz] == 0)
    assert _rel(b2, bo) <= 1e-15
    # conjugate pairs stay conjugate
    pairs = np.nonzero(kind == 1)[0]
    assert np.max(np.abs(l2[pairs + 1] - np.conj(l2[pairs]))) <= 1e-15
    # the source model is untouched
    assert np.array_equal(m.lam.cpu().numpy(), lam)


def test_per_mode_edit_parity_and_inplace(gpu_lib):
    from paper_2502_05339_amd import edit_modes
    dt = 0.25
    lam, b, kind = _lams(7, 60, dt, 0.01)
    r = lam.size
    _print(f"case: per-mode edit r={r}")
    rng = np.random.default_rng(8)
    pm = np.stack([rng.uniform(0, 2, r), rng.uniform(-1.5, 2, r), rng.uniform(-0.1, 0.1, r),
                   rng.uniform(-2, 2, r)], 1)
    m = _model(lam, b, kind, dt)
    em, _ = edit_modes(m, per_mode=torch.from_numpy(pm).cuda())
    lo, bo = oracle.edit_modes(lam, b, dt, pm[:, 0], pm[:, 1], pm[:, 2], pm[:, 3])
    l2 = em.lam.cpu().numpy()
    nz = lo != 0
    assert _rel(l2[nz], lo[nz]) <= 1e-13
    assert _rel(em.b.cpu().numpy(), bo) <= 1e-15
    m2 = _model(lam, b, kind, dt)
    ei, _ = edit_modes(m2, per_mode=torch.from_numpy(pm).cuda(), inplace=True)
    assert ei is m2
    assert np.array_equal(m2.lam.cpu().numpy(), l2)
    assert np.array_equal(m2.b.cpu().numpy(), em.b.cpu().numpy())


def test_identity_edit(gpu_lib):
    from paper_2502_05339_amd import edit_modes
    lam, b, kind = _lams(11, 50, 1.0, 0.01)
    em, _ = edit_modes(_model(lam, b, kind, 1.0))
    l2 = em.lam.cpu().numpy()
    nz = lam != 0
    assert _rel(l2[nz], lam[nz]) <= 1e-14
    assert np.array_equal(em.b.cpu().numpy(), b)


@pytest.fixture(scope="module")
def c1cf():
    cfg = synth.config("c1-cf", seed=103)
    g = synth.generate(cfg)
    return cfg, g, oracle.fit_exact(g.Z, cfg.r)


@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_edited_reconstruction_parity(gpu_lib, c1cf, mode):
    from paper_2502_05339_amd import edit_modes
    cfg, g, f = c1cf
    dt = 0.5
    cut = float(np.median(np.abs(np.angle(f.lam))) / dt)
    dtype = torch.float64 if mode == "fp64" else torch.float32
    m = model_from_oracle(f, dtype, dt=dt)
    _print(f"case: c1-cf edited reconstruction {mode}, cut={cut:.4g}")
    params = dict(weight=(1.0, 2.0), re_scale=(1.0, 0.7), re_shift=(0.0, -0.01), im_scale=(1.0, 1.3))
    em, cl = edit_modes(m, freq_cut=cut, **params)
    lam_h, b_h = m.lam.cpu().numpy(), m.b.cpu().numpy()
    lo, bo, co = oracle.cluster_edit(lam_h, b_h, dt, params["weight"], params["re_scale"], params["re_shift"],
                                     params["im_scale"], cut=cut)
    assert np.array_equal(cl.cpu().numpy(), co)
    ks = np.arange(0, 150, 3)
    U = em.reconstruct(ks, mode).cpu().numpy()
    Uo = oracle.reconstruct(m.complex_modes(), lo, bo, ks).T
    err = max_frame_rel(U, Uo)
    _print(f"  max-frame rel err {err:.3e}")
    assert err <= (1e-12 if mode == "fp64" else 1e-4)


def test_inverse_edit_equals_negative_exponents(gpu_lib, c1cf):
    """re_scale = im_scale = -1 gives lambda^-1: reconstructing it at k equals the model at -k."""
    from paper_2502_05339_amd import edit_modes
    cfg, g, f = c1cf
    m = model_from_oracle(f, torch.float64, dt=0.2)
    em, _ = edit_modes(m, re_scale=-1.0, im_scale=-1.0)
    ks = np.arange(0, 60)
    Ua = em.reconstruct(ks, "fp64").cpu().numpy()
    Ub = m.reconstruct(-ks, "fp64").cpu().numpy()
    assert max_frame_rel(Ua, Ub) <= 1e-12


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-9), (torch.float32, 2e-4)])
def test_reverse_roll_out(gpu_lib, c1cf, dtype, tol):
    """From the last snapshot back to the first (Sec. 6.2), against the oracle and the data."""
    from paper_2502_05339_amd import reverse
    cfg, g, f = c1cf
    m = model_from_oracle(f, dtype)
    T = g.Z.shape[1] - 1
    _print(f"case: reverse roll-out {dtype} T={T}")
    ks = np.arange(1, T + 1)
    u = torch.from_numpy(np.ascontiguousarray(g.Z[:, T])).to(dtype).cuda()
    mode = "fp64" if dtype == torch.float64 else "fp32"
    U = reverse(m, u, ks, mode).cpu().numpy()
    Uo = oracle.reverse(m.complex_modes(), m.lam.cpu().numpy(), u.double().cpu().numpy(), ks).T
    err_o = max_frame_rel(U, Uo)
    err_d = max_frame_rel(U, g.Z[:, T - ks].T)
    _print(f"  vs oracle {err_o:.3e}, vs data {err_d:.3e}")
    assert err_o <= tol and err_d <= max(tol, 1e-8)


def test_edit_argument_errors(gpu_lib):
    from paper_2502_05339_amd import DMDError, edit_modes
    lam, b, kind = _lams(5, 10, 1.0, 0.01)
    m = _model(lam, b, kind, 1.0)
    for kw in (dict(weight=float("nan")), dict(freq_cut=-1.0), dict(im_scale=(1.0, float("inf")))):
        with pytest.raises((DMDError, ValueError)):
            edit_modes(m, **kw)
    m.dt = 0.0
    with pytest.raises(DMDError):
        edit_modes(m)
    m.dt = 1.0
    with pytest.raises(ValueError):
        edit_modes(m, per_mode=torch.zeros((m.r, 3), dtype=torch.float64, device="cuda"))
