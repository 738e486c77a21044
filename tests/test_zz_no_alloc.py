"""GPU test of dmd_reconstruct_noalloc, the reconstruction entry point without a workspace
argument (its coefficients live in a library-owned device array): through the C ABI its
frames equal dmd_reconstruct's on the same model and exponents, bit for bit (the same
kernels on the same coefficients), on two calls in a row, the second with fewer frames;
the status word reaches the caller's device int; requests beyond the array's size are
refused before any device work."""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _model(dtype, nc=20, n=3000, seed=11):
    import paper_2502_05339_amd as dmd
    rng = np.random.default_rng(seed)
    phi = synth.orthonormal_modes(rng, n, nc)
    lam = synth.draw_eigs(rng, nc, 0.95)
    b = synth.draw_amplitudes(rng, nc)
    return dmd.Model.from_pairs(phi, lam, b, dtype=dtype)


def _noalloc(model, ks, mcode, U, status=None):
    from paper_2502_05339_amd import _lib
    from paper_2502_05339_amd.api import _stream
    k = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
    ms = model.struct()
    return _lib.lib().dmd_reconstruct_noalloc(_stream(), ctypes.byref(ms), k.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                              k.size, mcode, U.data_ptr(), U.stride(0),
                                              status.data_ptr() if status is not None else None)


@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x3"])
def test_noalloc_matches_workspace_call(gpu_lib, mode):
    import paper_2502_05339_amd as dmd
    from paper_2502_05339_amd.api import RECON_MODES
    dtype = torch.float64 if mode == "fp64" else torch.float32
    _print(f"case: dmd_reconstruct_noalloc vs dmd_reconstruct, {mode}")
    m = _model(dtype)
    mcode = RECON_MODES[mode]
    for K, k0 in ((700, -40), (93, 5)):                     # second call with fewer frames
        ks = np.arange(k0, k0 + K)
        ref = dmd.reconstruct(m, ks, mode)
        U = torch.full((K, m.n), float("nan"), dtype=dtype, device="cuda")
        st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        assert _noalloc(m, ks, mcode, U, st) == 0
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        assert torch.equal(U, ref), float((U - ref).abs().max().item())
        _print(f"  K={K}: equal to the workspace call")


def test_noalloc_status_and_limits(gpu_lib):
    import paper_2502_05339_amd as dmd
    from paper_2502_05339_amd import _lib
    from paper_2502_05339_amd.api import RECON_MODES
    _print("case: dmd_reconstruct_noalloc status word and size limit")
    m = dmd.Model.empty(64, 2, torch.float32, "cuda")
    m.phi[:, :2].copy_(torch.randn(64, 2))
    m.lam.copy_(torch.tensor([0.0, 0.9], dtype=torch.complex128))
    m.b.copy_(torch.tensor([1.0, 2.0], dtype=torch.complex128))
    U = torch.empty((2, 64), dtype=torch.float32, device="cuda")
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    assert _noalloc(m, [2, -1], RECON_MODES["fp32"], U, st) == 0
    torch.cuda.synchronize()
    assert int(st.item()) & 1                               # 0^-1: outside the domain
    assert _noalloc(m, [0, 1], RECON_MODES["fp32"], U, st) == 0
    torch.cuda.synchronize()
    assert int(st.item()) == 0                              # cleared by the next call
    # beyond the array: refused before any device work
    big = _model(torch.float64, nc=75, n=256)
    nb = ctypes.c_size_t(0)
    K = 8000
    assert _lib.lib().dmd_reconstruct_workspace_size(big.r, K, RECON_MODES["fp64"], ctypes.byref(nb)) == 0
    assert nb.value > _lib.NOALLOC_SCRATCH_BYTES
    Ub = torch.empty((K, big.n), dtype=torch.float64, device="cuda")
    assert _noalloc(big, np.arange(K), RECON_MODES["fp64"], Ub) == _lib.DMD_ERR_WORKSPACE
