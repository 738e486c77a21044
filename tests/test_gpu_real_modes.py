"""Models with a real negative eigenvalue (odd rank of a conjugate-paired system: the
exact DMD of c1-cf at r = 15 keeps 7 pairs and one real mode near -0.59) through the
calls that take powers or per-mode states: integration at fractional times (where
lambda^t of a negative lambda is complex and only its real part reaches the field), the
forced roll-out and the upsampling evolution, against the FP64 oracle through the C ABI.
Tolerances as in the FP64 tests of those calls (1e-12 fields for integration, 1e-10
states and frames for the roll-outs).
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


@pytest.fixture(scope="module")
def odd_fit():
    cfg = synth.config("c1-cf", seed=104)
    g = synth.generate(cfg)
    f = oracle.fit_exact(g.Z, 15)
    real = np.abs(f.lam.imag) <= 1e-9 * np.abs(f.lam)
    assert real.sum() == 1 and f.lam[real][0].real < 0       # the premise of the cases
    return cfg, g, f


def _rel(Z, Zo):
    return float(np.max(np.abs(Z - Zo)) / np.max(np.abs(Zo)))


def test_integrate_negative_real_mode(gpu_lib, odd_fit):
    cfg, g, f = odd_fit
    _print("case: integrate, r = 15 with a negative real eigenvalue")
    m = model_from_oracle(f, torch.float64, dt=0.5)
    ts = np.array([0.0, 0.25, 0.5, 1.3, 7.75, -1.25])
    U = m.integrate(ts, "fp64").cpu().numpy()
    Uo = oracle.integrate(f.phi, f.lam, f.b, ts, dt=0.5).T
    err = max_frame_rel(U, Uo)
    _print(f"  fields {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("T", [1, 37])
def test_rollout_negative_real_mode(gpu_lib, odd_fit, T):
    from paper_2502_05339_amd import rollout
    cfg, g, f = odd_fit
    dt = 0.4
    m = model_from_oracle(f, torch.float64, dt=dt)
    _print(f"case: rollout fp64 r=15 (real negative mode) T={T}")
    F = 0.05 * np.random.default_rng(300 + T).standard_normal((T, m.n))
    Z, U = rollout(m, torch.from_numpy(F).cuda(), mode="fp64")
    Zo, Uo = oracle.rollout(m.complex_modes(), m.lam.cpu().numpy(), m.b.cpu().numpy(), F.T, dt=dt)
    es, ef = _rel(Z.cpu().numpy(), Zo), max_frame_rel(U.cpu().numpy(), Uo.T)
    _print(f"  states {es:.3e} frames {ef:.3e}")
    assert es <= 1e-10 and ef <= 1e-10


@pytest.mark.parametrize("real_low", [True, False])
def test_upsample_negative_real_mode(gpu_lib, odd_fit, real_low):
    from paper_2502_05339_amd import upsample
    cfg, g, f = odd_fit
    m = model_from_oracle(f, torch.float64)
    lam = m.lam.cpu().numpy()
    kind = m.kind.cpu().numpy()
    low = np.abs(np.angle(lam)) < np.median(np.abs(np.angle(lam)))
    low[kind == 0] = real_low
    rng = np.random.default_rng(41 + int(real_low))
    h0 = rng.standard_normal(m.n)
    L = rng.standard_normal((9, m.n))
    _print(f"case: upsample fp64 r=15, real mode {'low' if real_low else 'high'}")
    R, H = upsample(m, torch.from_numpy(h0).cuda(), torch.from_numpy(L).cuda(), low, mode="fp64")
    Ro, Ho = oracle.upsample_evolve(m.complex_modes(), lam, h0, L.T, low)
    es, ef = _rel(R.cpu().numpy(), Ro), max_frame_rel(H.cpu().numpy(), Ho.T)
    _print(f"  states {es:.3e} frames {ef:.3e}")
    assert es <= 1e-10 and ef <= 1e-10
