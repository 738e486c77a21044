"""GPU parity of the upsampling evolution (Sec. 6.3.1) and of the constrained
projection onto a low-res guide (Sec. 6.3.2) against the FP64 oracle, through the C ABI.

Tolerances: FP64 models 1e-10 (evolution states and frames; normal equations of the
FP64 Gram against the oracle's QR least squares); FP32 models 2e-5 on states and 1e-4
on FP32 / bf16x3 frames (the oracle sees the FP32-rounded modes and fields).  The
projection is one subtraction per cell after an FP64 block mean: FP64 1e-12, FP32 1e-6
relative, against the oracle's dense KKT solve; at a full-size grid the constraint and
the block-constant correction are checked directly.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import max_frame_rel, model_from_oracle, rank150_fit

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def c1cf():
    cfg = synth.config("c1-cf", seed=103)
    g = synth.generate(cfg)
    return cfg, g, oracle.fit_exact(g.Z, cfg.r)


def _rel(Z, Zo):
    return float(np.max(np.abs(Z - Zo)) / np.max(np.abs(Zo)))


@pytest.mark.parametrize("T", [1, 7, 70])
def test_upsample_fp64_parity(gpu_lib, c1cf, T):
    from paper_2502_05339_amd import upsample
    cfg, g, f = c1cf
    m = model_from_oracle(f, torch.float64)
    lam = m.lam.cpu().numpy()
    low = np.abs(np.angle(lam)) < np.median(np.abs(np.angle(lam)))
    rng = np.random.default_rng(T)
    h0 = rng.standard_normal(m.n)
    L = rng.standard_normal((T, m.n))
    _print(f"case: upsample fp64 N={m.n} r={m.r} T={T} low={int(low.sum())}")
    R, H = upsample(m, torch.from_numpy(h0).cuda(), torch.from_numpy(L).cuda(), low, mode="fp64")
    Ro, Ho = oracle.upsample_evolve(m.complex_modes(), lam, h0, L.T, low)
    es, ef = _rel(R.cpu().numpy(), Ro), max_frame_rel(H.cpu().numpy(), Ho.T)
    _print(f"  states {es:.3e} frames {ef:.3e}")
    assert es <= 1e-10 and ef <= 1e-10


@pytest.mark.parametrize("T", [1, 30])
def test_upsample_fp64_parity_rank150(gpu_lib, T):
    from paper_2502_05339_amd import upsample
    cfg, g, f = rank150_fit()
    m = model_from_oracle(f, torch.float64)
    lam = m.lam.cpu().numpy()
    low = np.abs(np.angle(lam)) < np.median(np.abs(np.angle(lam)))
    rng = np.random.default_rng(2000 + T)
    h0 = rng.standard_normal(m.n)
    L = rng.standard_normal((T, m.n))
    _print(f"case: upsample fp64 N={m.n} r={m.r} T={T} low={int(low.sum())}")
    R, H = upsample(m, torch.from_numpy(h0).cuda(), torch.from_numpy(L).cuda(), low, mode="fp64")
    Ro, Ho = oracle.upsample_evolve(m.complex_modes(), lam, h0, L.T, low)
    es, ef = _rel(R.cpu().numpy(), Ro), max_frame_rel(H.cpu().numpy(), Ho.T)
    _print(f"  states {es:.3e} frames {ef:.3e}")
    assert es <= 1e-10 and ef <= 1e-10


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_upsample_fp32_parity(gpu_lib, c1cf, mode):
    from paper_2502_05339_amd import upsample
    cfg, g, f = c1cf
    m = model_from_oracle(f, torch.float32)
    lam = m.lam.cpu().numpy()
    low = np.abs(np.angle(lam)) < np.median(np.abs(np.angle(lam)))
    rng = np.random.default_rng(5)
    h0 = rng.standard_normal(m.n).astype(np.float32)
    L = rng.standard_normal((40, m.n)).astype(np.float32)
    R, H = upsample(m, torch.from_numpy(h0).cuda(), torch.from_numpy(L).cuda(), low, mode=mode)
    Ro, Ho = oracle.upsample_evolve(m.complex_modes(), lam, h0.astype(np.float64), L.T.astype(np.float64), low)
    es, ef = _rel(R.cpu().numpy(), Ro), max_frame_rel(H.cpu().numpy(), Ho.T)
    _print(f"case: upsample fp32 {mode}: states {es:.3e} frames {ef:.3e}")
    assert es <= 2e-5 and ef <= 1e-4


def test_upsample_all_high_is_reconstruction(gpu_lib, c1cf):
    from paper_2502_05339_amd import upsample
    cfg, g, f = c1cf
    m = model_from_oracle(f, torch.float64)
    h0 = torch.from_numpy(np.ascontiguousarray(g.Z[:, 3])).cuda()
    L = torch.zeros((12, m.n), dtype=torch.float64, device="cuda")
    R, H = upsample(m, h0, L, np.zeros(m.r, bool), mode="fp64")
    z0 = m.project(h0)
    from paper_2502_05339_amd import Model
    import dataclasses
    Ur = dataclasses.replace(m, b=z0).reconstruct(np.arange(13), "fp64").cpu().numpy()
    assert max_frame_rel(H.cpu().numpy(), Ur) <= 1e-11


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-6)])
@pytest.mark.parametrize("grid,fct", [((2, 1, 16, 16), 2), ((1, 4, 8, 8), 2), ((3, 1, 12, 9), 3), ((1, 1, 5, 5), 1),
                                      ((2, 1, 16, 16), 4), ((1, 8, 8, 8), 4), ((1, 1, 16, 16), 8)])
def test_lowres_project_parity(gpu_lib, grid, fct, dtype, tol):
    from paper_2502_05339_amd import lowres_project
    nc, nz, ny, nx = grid
    A = oracle.block_average_matrix(nc, nz, ny, nx, fct)
    rng = np.random.default_rng(nc * 100 + nx)
    F = 3
    npdt = np.float64 if dtype == torch.float64 else np.float32
    h = rng.standard_normal((F, A.shape[1])).astype(npdt)
    l = rng.standard_normal((F, A.shape[0])).astype(npdt)
    _print(f"case: lowres_project grid={grid} factor={fct} {dtype}")
    x = lowres_project(torch.from_numpy(h).cuda(), torch.from_numpy(l).cuda(), grid, fct).cpu().numpy()
    for fr in range(F):
        xo = oracle.kkt_project(h[fr].astype(np.float64), l[fr].astype(np.float64), A)
        assert np.max(np.abs(x[fr] - xo)) <= tol * np.max(np.abs(xo))
    # in place
    ht = torch.from_numpy(h).cuda()
    lowres_project(ht, torch.from_numpy(l).cuda(), grid, fct, out=ht)
    assert np.array_equal(ht.cpu().numpy(), x)


def test_lowres_project_full_grid_properties(gpu_lib):
    """c2's grid (2 x 256 x 256), factor 4, FP32: A x = l and x - h constant per block."""
    from paper_2502_05339_amd import lowres_project
    nc, ny, nx, fct = 2, 256, 256, 4
    gen = torch.Generator(device="cuda").manual_seed(3)
    h = torch.randn((4, nc * ny * nx), device="cuda", generator=gen)
    l = torch.randn((4, nc * (ny // fct) * (nx // fct)), device="cuda", generator=gen)
    x = lowres_project(h, l, (nc, 1, ny, nx), fct)
    xb = x.double().reshape(4, nc, ny // fct, fct, nx // fct, fct)
    d = (x.double() - h.double()).reshape(4, nc, ny // fct, fct, nx // fct, fct)
    mean = xb.mean(dim=(3, 5)).reshape(4, -1)
    assert float((mean - l.double()).abs().max()) <= 1e-5
    assert float((d - d[:, :, :, :1, :, :1]).abs().max()) <= 1e-5


def test_upsample_and_project_argument_errors(gpu_lib, c1cf):
    from paper_2502_05339_amd import DMDError, lowres_project, upsample
    cfg, g, f = c1cf
    m = model_from_oracle(f, torch.float64)
    h0 = torch.zeros(m.n, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        upsample(m, h0, torch.zeros((3, m.n), dtype=torch.float64, device="cuda"), np.zeros(m.r - 1, bool))
    with pytest.raises(DMDError):
        lowres_project(torch.zeros((1, 2 * 10 * 10), device="cuda"), torch.zeros((1, 2 * 3 * 3), device="cuda"),
                       (2, 1, 10, 10), 3)
