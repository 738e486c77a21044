"""GPU parity at the full sizes of the benchmark workloads, in the launch
configurations the benchmark times, against the FP64 oracle on sampled outputs.

  c5a  batched reconstruction, N = 5,308,416 (3 x 192 x 96 x 96), 75 smooth pairs,
       4096 frames k in [0, 5000] in one launch: 2.17e10 output elements, so element
       offsets pass 2^31.  FP32 and bf16x3 gated at 1e-4 (max-frame relative) on 2048
       sampled rows over all frames; BF16 reported.
  c3   3D plume-shaped mixed fit, N = 6,291,456 (7.55 GB of FP32 snapshots, byte offsets
       past 2^31), against the FP64 randomized twin on the full FP64 input: amplitude-
       weighted eigenvalue error <= 1e-5, fields on 65,536 sampled rows <= 1e-4.
  c5b  eight uneven mixed fits replayed from one captured graph, each against its own
       FP64 twin (amplitude-weighted eigenvalues <= 1e-5, fields <= 1e-4).
  OptDMD, mixed path, against the oracle's variable projection started from the FP64
       twin: eigenvalues <= 1e-5 and fields <= 1e-4 at a small well-posed case; at the
       c4 shape, whose minimiser is not unique, the cost the GPU's eigenvalues reach.
"""
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import max_frame_rel
from oracle.metrics import match_eigs

pytestmark = pytest.mark.gpu

T0 = time.perf_counter()


def _print(*a):
    print(f"[{time.perf_counter() - T0:7.1f}s]", *a, flush=True)


def _weighted(lam_gpu, tw):
    w = oracle.amplitude_weights(tw.phi, tw.b)
    ia, ib = match_eigs(lam_gpu, tw.lam)
    d = np.abs(lam_gpu[ia] - tw.lam[ib])
    return float(np.sum(w[ib] * d) / np.sum(w[ib] * np.abs(tw.lam[ib]))), float(np.max(d / np.abs(tw.lam[ib])))


@pytest.mark.timeout(900)
def test_c5a_full_shape_vs_oracle(gpu_lib):
    import paper_2502_05339_amd as dmd
    cfg = synth.config("c5a")
    _print(f"case: c5a N={cfg.N} r={cfg.r} K={cfg.K}; drawing the model")
    phi, lam, b = synth.synthetic_model(cfg, progress=_print)
    model = dmd.Model.from_pairs(phi, lam, b, dtype=torch.float32)
    ks = synth.c5a_frames(cfg.K)
    U = torch.empty((cfg.K, cfg.N), dtype=torch.float32, device="cuda")
    assert U.numel() > 2 ** 31
    rows = np.sort(np.random.default_rng(5).choice(cfg.N, 2048, replace=False))
    rows[-1] = cfg.N - 1                                  # the last row of the last frame
    pc = phi[rows].astype(np.complex128)
    full_phi = np.empty((rows.size, 2 * cfg.nc), dtype=np.complex128)
    full_phi[:, 0::2], full_phi[:, 1::2] = pc, np.conj(pc)
    lam_f = np.empty(2 * cfg.nc, dtype=np.complex128)
    b_f = np.empty(2 * cfg.nc, dtype=np.complex128)
    lam_f[0::2], lam_f[1::2] = lam, np.conj(lam)
    b_f[0::2], b_f[1::2] = b, np.conj(b)
    ref = oracle.reconstruct(full_phi, lam_f, b_f, ks)     # rows x K
    rows_t = torch.from_numpy(rows).cuda()
    errs = {}
    for mode in ("bf16x3", "fp32", "bf16"):
        U.fill_(float("nan"))
        dmd.reconstruct(model, ks, mode, out=U)
        got = U[:, rows_t].double().cpu().numpy().T
        errs[mode] = max_frame_rel(got.T, ref.T)
        _print(f"  {mode}: max-frame rel {errs[mode]:.3e}")
        assert np.all(np.isfinite(got))
        assert bool(torch.isfinite(U[-1]).all().item())      # every element of the last frame written
    assert errs["bf16x3"] <= 1e-4 and errs["fp32"] <= 1e-4
    assert errs["bf16"] <= 2e-2                            # BF16 coefficients and modes: reported, bounded


@pytest.mark.timeout(1200)
def test_c3_mixed_vs_twin_full(gpu_lib):
    import paper_2502_05339_amd as dmd
    cfg = synth.config("c3")
    _print(f"case: c3 N={cfg.N} m={cfg.m} r={cfg.r}; drawing the input")
    g = synth.generate(cfg, progress=_print)
    _print("  input drawn")
    Z = torch.from_numpy(np.ascontiguousarray(g.Z.T)).cuda()
    om = torch.from_numpy(np.ascontiguousarray(g.Omega.T)).cuda()
    assert Z.numel() * 4 > 2 ** 31
    m = dmd.fit(Z, cfg.r, p=cfg.p, q=cfg.q, omega=om, precision="mixed")
    _print(f"  GPU fit done, info {m.info.cpu().tolist()}")
    rows = np.sort(np.random.default_rng(302).choice(cfg.N, 65536, replace=False))
    rows[-1] = cfg.N - 1
    ks = np.arange(cfg.m)
    U = m.reconstruct(ks, "fp32")[:, torch.from_numpy(rows).cuda()].double().cpu().numpy()
    del Z
    Zd = np.asfortranarray(g.Z, dtype=np.float64)
    del g
    tw = oracle.fit_randomized(Zd, cfg.r, synth.sketch(cfg.seed, cfg.m, cfg.l).astype(np.float64), cfg.q,
                               rows=rows)
    _print("  twin done")
    wrel, mx = _weighted(m.lam_host(), tw)
    Uo = oracle.reconstruct(tw.phi, tw.lam, tw.b, ks).T
    ferr = max_frame_rel(U, Uo)
    _print(f"  lambda weighted {wrel:.3e} (max {mx:.3e}), fields {ferr:.3e}")
    assert wrel <= 1e-5
    assert ferr <= 1e-4


@pytest.mark.timeout(900)
def test_c5b_graph_scenes_vs_twins(gpu_lib):
    import paper_2502_05339_amd as dmd
    _print("case: c5b eight scenes in one captured graph vs their FP64 twins")
    scenes, gens = [], []
    for sc in synth.c5b_scenes():
        cfg = synth.c5b_config(sc)
        g = synth.generate(cfg)
        Z = torch.from_numpy(np.ascontiguousarray(g.Z.T)).cuda()
        om = torch.from_numpy(np.ascontiguousarray(g.Omega.T)).cuda()
        scenes.append({"Z": Z, "r": cfg.r, "p": cfg.p, "q": cfg.q, "omega": om, "precision": "mixed"})
        gens.append((cfg, g))
    bf = dmd.BatchedFit(scenes, capture=True)
    for s in scenes:
        s["Z"].mul_(1.0)                                   # eager work between replays
    bf.launch()
    torch.cuda.synchronize()
    bf.launch()
    torch.cuda.synchronize()
    assert bf.statuses() == [0] * 8
    for i, ((cfg, g), m) in enumerate(zip(gens, bf.models)):
        rows = np.sort(np.random.default_rng(600 + i).choice(cfg.N, 4096, replace=False))
        tw = oracle.fit_randomized(g.Z.astype(np.float64), cfg.r, g.Omega.astype(np.float64), cfg.q, rows=rows)
        wrel, mx = _weighted(m.lam_host(), tw)
        ks = np.arange(cfg.m)
        U = m.reconstruct(ks, "fp32")[:, torch.from_numpy(rows).cuda()].double().cpu().numpy()
        ferr = max_frame_rel(U, oracle.reconstruct(tw.phi, tw.lam, tw.b, ks).T)
        _print(f"  scene {i} N={cfg.N} m={cfg.m}: lambda weighted {wrel:.3e} (max {mx:.3e}), fields {ferr:.3e}")
        assert wrel <= 1e-5 and ferr <= 1e-4
    bf.close()


def _twin_svd(g, cfg):
    X, _ = oracle.split_snapshots(g.Z.astype(np.float64))
    Om = np.asarray(g.Omega, dtype=np.float64)
    Q = oracle.range_finder(X, Om, cfg.q)
    Ub, s, Vt = np.linalg.svd(Q.T @ X, full_matrices=False)
    f = oracle.fit_randomized(g.Z.astype(np.float64), cfg.r, Om, cfg.q)
    return Q @ Ub[:, :cfg.r], s[:cfg.r], Vt.T[:, :cfg.r], f.lam


@pytest.mark.parametrize("case", ["small", "c4"])
@pytest.mark.timeout(600)
def test_optdmd_mixed_vs_oracle(gpu_lib, case):
    """The mixed fit's OptDMD refinement against the oracle's variable projection on the
    FP64 twin's SVD, started from the twin's eigenvalues.

    small: a well-posed case (16 modes, 1% noise) whose minimiser is unique: eigenvalues
    and fields are gated.  c4: rank 40 at 1% noise, where the per-entry noise exceeds the
    signal.  The starting eigenvalues there give a Vandermonde basis of condition 2e17
    (numerically singular), and the cost surface has a flat valley: the oracle itself
    stops at different points with different BLAS thread counts (cost 327.93 after 276
    steps on 8 threads, 328.50 after 298 on 16), and the GPU, whose FP64 normal equations
    take the shifted-Cholesky retry at that start, follows another path.  The minimiser
    is not unique, so what is compared is the objective: the oracle's own cost function
    evaluated at the GPU's eigenvalues on the twin's data must take at least 80% of the
    decrease the oracle achieves from the same start."""
    import paper_2502_05339_amd as dmd
    cfg = synth.config("c1-cf", seed=12, sigma=1e-2, p=4, q=1, dtype="f32") if case == "small" else synth.config("c4")
    _print(f"case: optdmd mixed vs oracle, {case} (N={cfg.N}, m={cfg.m}, r={cfg.r})")
    g = synth.generate(cfg)
    Z = torch.from_numpy(np.ascontiguousarray(g.Z.T).astype(np.float32)).cuda()
    om = torch.from_numpy(np.ascontiguousarray(g.Omega.T).astype(np.float32)).cuda()
    m = dmd.fit(Z, cfg.r, p=cfg.p, q=cfg.q, omega=om, precision="mixed", optdmd=True)
    steps = int(m.info.cpu().numpy()[4])
    U_r, s_r, V_r, lam0 = _twin_svd(g, cfg)
    a, phi, b, cost, it = oracle.fit_optdmd(U_r, s_r, V_r, lam0, max_iter=1000)
    lam = m.lam_host()
    Yv = np.conj(V_r.astype(np.complex128)) * s_r[None, :]
    cost_gpu = oracle.varpro_trial(lam, Yv)[3]
    cost_start = oracle.varpro_trial(lam0, Yv)[3]
    ia, ib = match_eigs(lam, a)
    e_par = float(np.max(np.abs(lam[ia] - a[ib]) / np.abs(a[ib])))
    w = oracle.amplitude_weights(phi, b)
    e_w = float(np.sum(w[ib] * np.abs(lam[ia] - a[ib])) / np.sum(w[ib] * np.abs(a[ib])))
    T = cfg.m - 1
    rows = np.sort(np.random.default_rng(7).choice(cfg.N, min(cfg.N, 8192), replace=False))
    U = m.reconstruct(np.arange(T), "fp32")[:, torch.from_numpy(rows).cuda()].double().cpu().numpy()
    Uo = oracle.reconstruct(phi[rows], a, b, np.arange(T)).T
    e_f = max_frame_rel(U, Uo)
    truth = np.concatenate([g.lam, np.conj(g.lam)])
    wt = np.abs(np.concatenate([g.b, np.conj(g.b)]))
    e_truth = oracle.eig_errors(lam, truth, weights=wt)["weighted_rel"]
    e_truth_o = oracle.eig_errors(a, truth, weights=wt)["weighted_rel"]
    gap = (cost_gpu - cost) / (cost_start - cost)
    _print(f"  LM steps {steps} (oracle {it}); lambda vs oracle max {e_par:.3e} weighted {e_w:.3e}; fields {e_f:.3e}; "
           f"cost start {cost_start:.9g} oracle {cost:.9g} GPU {cost_gpu:.9g} (gap {gap:.3e} of the decrease); "
           f"weighted error vs the generating system: GPU {e_truth:.3e}, oracle {e_truth_o:.3e}")
    assert int(m.info[0].item()) == 0
    if case == "small":
        assert e_par <= 1e-5
        assert e_f <= 1e-4
    else:
        assert gap <= 0.2
