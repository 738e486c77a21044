"""GPU parity of the forced reduced roll-out (Sec. 4.6, eq. external_forces) against
the FP64 oracle, through the C ABI.

Tolerances: FP64 models 1e-10 relative on states and frames (normal equations of the
FP64 Gram and an FP64 recurrence; the oracle uses a QR least-squares solve and a plain
loop); FP32 models 2e-5 on states (the projection Phi^T F reads FP32 modes and forcing
with FP64 accumulation) and 1e-4 on the FP32 / bf16x3 frames.  The oracle sees the
FP32-rounded modes and forcing.
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
    cfg = synth.config("c1-cf", seed=102)
    g = synth.generate(cfg)
    return cfg, g, oracle.fit_exact(g.Z, cfg.r)


def _rel_states(Z, Zo):
    return float(np.max(np.abs(Z - Zo)) / np.max(np.abs(Zo)))


@pytest.mark.parametrize("T", [1, 63, 64, 65, 200, 333])
def test_rollout_fp64_parity(gpu_lib, c1cf, T):
    from paper_2502_05339_amd import rollout
    cfg, g, f = c1cf
    dt = 0.3
    m = model_from_oracle(f, torch.float64, dt=dt)
    _print(f"case: rollout fp64 N={m.n} r={m.r} T={T}")
    rng = np.random.default_rng(T)
    F = 0.05 * rng.standard_normal((T, m.n))
    Z, U = rollout(m, torch.from_numpy(F).cuda(), mode="fp64")
    Zo, Uo = oracle.rollout(m.complex_modes(), m.lam.cpu().numpy(), m.b.cpu().numpy(), F.T, dt=dt)
    es, ef = _rel_states(Z.cpu().numpy(), Zo), max_frame_rel(U.cpu().numpy(), Uo.T)
    _print(f"  states {es:.3e} frames {ef:.3e}")
    assert es <= 1e-10 and ef <= 1e-10


@pytest.mark.parametrize("T", [1, 100])
def test_rollout_fp64_parity_rank150(gpu_lib, T):
    from paper_2502_05339_amd import rollout
    cfg, g, f = rank150_fit()
    dt = 0.7
    m = model_from_oracle(f, torch.float64, dt=dt)
    _print(f"case: rollout fp64 N={m.n} r={m.r} T={T}")
    rng = np.random.default_rng(1000 + T)
    F = 0.05 * rng.standard_normal((T, m.n))
    Z, U = rollout(m, torch.from_numpy(F).cuda(), mode="fp64")
    Zo, Uo = oracle.rollout(m.complex_modes(), m.lam.cpu().numpy(), m.b.cpu().numpy(), F.T, dt=dt)
    es, ef = _rel_states(Z.cpu().numpy(), Zo), max_frame_rel(U.cpu().numpy(), Uo.T)
    _print(f"  states {es:.3e} frames {ef:.3e}")
    assert es <= 1e-10 and ef <= 1e-10


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_rollout_fp32_parity(gpu_lib, c1cf, mode):
    from paper_2502_05339_amd import rollout
    cfg, g, f = c1cf
    dt, T = 0.5, 150
    m = model_from_oracle(f, torch.float32, dt=dt)
    _print(f"case: rollout fp32 model, {mode} frames, T={T}")
    rng = np.random.default_rng(77)
    F32 = (0.05 * rng.standard_normal((T, m.n))).astype(np.float32)
    Z, U = rollout(m, torch.from_numpy(F32).cuda(), mode=mode)
    Zo, Uo = oracle.rollout(m.complex_modes(), m.lam.cpu().numpy(), m.b.cpu().numpy(), F32.T.astype(np.float64),
                            dt=dt)
    es, ef = _rel_states(Z.cpu().numpy(), Zo), max_frame_rel(U.cpu().numpy(), Uo.T)
    _print(f"  states {es:.3e} frames {ef:.3e}")
    assert es <= 2e-5 and ef <= 1e-4


def test_rollout_unforced_equals_reconstruction(gpu_lib, c1cf):
    from paper_2502_05339_amd import rollout
    cfg, g, f = c1cf
    m = model_from_oracle(f, torch.float64)
    Z, U = rollout(m, None, steps=90, mode="fp64")
    Ur = m.reconstruct(np.arange(91), "fp64").cpu().numpy()
    assert max_frame_rel(U.cpu().numpy(), Ur) <= 1e-12
    lam, b = m.lam.cpu().numpy(), m.b.cpu().numpy()
    assert _rel_states(Z.cpu().numpy()[90], b * lam ** 90) <= 1e-12


def test_rollout_initial_state_and_states_only(gpu_lib, c1cf):
    """An explicit z0 (here the projection of a snapshot) and a call without frames."""
    from paper_2502_05339_amd import rollout
    cfg, g, f = c1cf
    m = model_from_oracle(f, torch.float64, dt=0.25)
    u = torch.from_numpy(np.ascontiguousarray(g.Z[:, 5])).cuda()
    z0 = m.project(u)
    rng = np.random.default_rng(3)
    F = 0.02 * rng.standard_normal((40, m.n))
    Z, U = rollout(m, torch.from_numpy(F).cuda(), z0=z0, frames=False)
    assert U is None
    Zo, _ = oracle.rollout(m.complex_modes(), m.lam.cpu().numpy(), z0.cpu().numpy(), F.T, dt=0.25)
    assert _rel_states(Z.cpu().numpy(), Zo) <= 1e-10


def test_rollout_argument_errors(gpu_lib, c1cf):
    from paper_2502_05339_amd import DMDError, rollout
    cfg, g, f = c1cf
    m = model_from_oracle(f, torch.float32)
    with pytest.raises(ValueError):
        rollout(m, None)
    with pytest.raises(ValueError):
        rollout(m, torch.zeros((3, m.n), dtype=torch.float64, device="cuda"))
    with pytest.raises(DMDError):
        rollout(m, None, steps=4, mode="fp64")          # FP64 frames from an FP32 model
    m.dt = -1.0
    with pytest.raises(DMDError):
        rollout(m, None, steps=4)
