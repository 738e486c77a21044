#!/usr/bin/env python3
"""Benchmark of the DMD hot path on one MI355X.

Default workload (the configuration the headline metric is quoted on): randomized-
SVD DMD on a 2 x 256 x 256 velocity grid (N = 131072 DOFs), m = 200 snapshots of
a rank-150 synthetic linear system with noise 1e-4, r = 150, oversampling 10,
2 power iterations, 1000 reconstructed frames.

One step = the whole hot path once: mixed-precision fit (sketch, CholeskyQR2,
power iterations, projection, FP64 small factors, exact modes, amplitudes),
the batched bf16x3 reconstruction of frames k = 0..999, and one evaluation of
the adjoint (loss and gradients in lambda and b over the 200 snapshots).
`value` = reconstructed frames per second of whole steps (K * steps / wall time
of the steps, inputs resident in HBM).

Prints one JSON line.  `--gpus` other than 1 exits with a message: this build has
no multi-GPU path.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DMD fit time + reconstructed frames/s at r=150, mixed vs FP64, HBM% roofline"
HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "recon_bf16x3_c2_traffic.json")
RECON_SRC = os.path.join(ROOT, "paper_2502_05339_amd", "csrc", "recon.hip")


def _events_ms(fn, reps):
    """Average device milliseconds of fn() over reps launches on the current stream."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def _src_hash(path):
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def _traffic(bytes_alg):
    """HBM bytes per launch from the committed counter summary, if the kernel is unchanged."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
        if t.get("source_sha256_16") != _src_hash(RECON_SRC):
            return None
        return float(t["bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def cpu_baseline(g, cfg, rows_sample=65536):
    """The FP64 oracle on the host: the randomized twin fit on the full input (repeated up
    to three times, about 6 s, mean taken), plus the reconstruction of all K frames and one
    loss/gradient on a row sample, scaled to N: about 10 s of host work in all."""
    import numpy as np

    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [os.cpu_count() or 1])
    except Exception:
        threads = os.cpu_count() or 1
    Zd = g.Z.astype(np.float64)
    t_fits = []
    while len(t_fits) < 3 and sum(t_fits) < 6.0:
        t0 = time.perf_counter()
        tw = oracle.fit_randomized(Zd, cfg.r, g.Omega.astype(np.float64), cfg.q)
        t_fits.append(time.perf_counter() - t0)
    t_fit = sum(t_fits) / len(t_fits)
    rows = np.sort(np.random.default_rng(1).choice(cfg.N, rows_sample, replace=False))
    ks = np.arange(cfg.K)
    t0 = time.perf_counter()
    Us = oracle.reconstruct(tw.phi[rows], tw.lam, tw.b, ks)
    t_rec = (time.perf_counter() - t0) * cfg.N / rows_sample
    t0 = time.perf_counter()
    oracle.loss_grad(tw.phi[rows], tw.lam, tw.b, Zd[rows], np.arange(cfg.m))
    t_adj = (time.perf_counter() - t0) * cfg.N / rows_sample
    t_step = t_fit + t_rec + t_adj
    # the same step on one host thread: one twin fit, reconstruction and loss+gradient on
    # a smaller row sample, scaled to N
    single = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            oracle.fit_randomized(Zd, cfg.r, g.Omega.astype(np.float64), cfg.q)
            t_fit1 = time.perf_counter() - t0
            rows1 = rows[: rows_sample // 8]
            t0 = time.perf_counter()
            oracle.reconstruct(tw.phi[rows1], tw.lam, tw.b, ks)
            t_rec1 = (time.perf_counter() - t0) * cfg.N / rows1.size
            t0 = time.perf_counter()
            oracle.loss_grad(tw.phi[rows1], tw.lam, tw.b, Zd[rows1], np.arange(cfg.m))
            t_adj1 = (time.perf_counter() - t0) * cfg.N / rows1.size
        single = {"value": round(cfg.K / (t_fit1 + t_rec1 + t_adj1), 3), "unit": "frames/s", "cores": 1,
                  "sample": (f"the same step on one host thread: twin fit {t_fit1:.2f} s, reconstruction "
                             f"{t_rec1:.2f} s and loss+gradient {t_adj1:.2f} s (the latter two on {rows1.size} rows, "
                             f"scaled to N)")}
    except ImportError:
        pass
    return tw, rows, Us, {
        "value": round(cfg.K / t_step, 3),
        "unit": "frames/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"one step of the FP64 NumPy oracle: randomized-SVD twin fit on the full input "
                   f"({t_fit:.2f} s, mean of {len(t_fits)}), reconstruction of all {cfg.K} frames ({t_rec:.2f} s) and one "
                   f"loss+gradient over {cfg.m} frames ({t_adj:.2f} s), the latter two measured on "
                   f"{rows_sample} of {cfg.N} rows and scaled linearly to N"),
        "fit_s": round(t_fit, 3),
        "single_thread": single,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the host oracle leg")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison path")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling HBM counters)")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5a", "c5b"],
                    help="c2 (default, the headline line); c3 3D plume-shaped fit; c5a batched "
                         "reconstruction of 4096 frames; c5b eight uneven fits in one captured graph")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "bench.py runs on exactly one GPU: this build of the DMD hot path has "
                                   "no multi-GPU path (run with --gpus 1)"}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2502_05339_amd as dmd
    import synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload != "c2":
        out = {"c3": run_c3, "c4": run_c4, "c5a": run_c5a, "c5b": run_c5b}[args.workload](args)
        out.update({"metric": METRIC, "n_gpus": 1, "higher_is_better": True, "vs_baseline": None,
                    "data": "synthetic"})
        print(json.dumps(out), flush=True)
        return
    cfg = synth.config("c2")
    g = synth.generate(cfg)
    Z = torch.from_numpy(np.ascontiguousarray(g.Z.T)).cuda()               # (m, N) float32
    om = torch.from_numpy(np.ascontiguousarray(g.Omega.T)).cuda()          # (l, m-1)
    ks = np.arange(cfg.K)
    kfit = np.arange(cfg.m)
    Ubuf = torch.empty((cfg.K, cfg.N), dtype=torch.float32, device="cuda")
    print(f"# workload c2: N={cfg.N} m={cfg.m} r={cfg.r} p={cfg.p} q={cfg.q} K={cfg.K}", file=sys.stderr, flush=True)

    def fit_mixed():
        return dmd.fit(Z, cfg.r, p=cfg.p, q=cfg.q, omega=om, precision="mixed", asynchronous=True)

    def step():
        m = fit_mixed()
        dmd.reconstruct(m, ks, "bf16x3", out=Ubuf)
        dmd.loss_grad(m, m.lam, m.b, Z, kfit)
        return m

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # tile shapes of the fit's TN products and of the reconstruction for these shape
    # classes, chosen by timing (outside the timed region)
    dmd.autotune_fit(Z, cfg.r, p=cfg.p, q=cfg.q, omega=om, precision="mixed")
    m = step()
    torch.cuda.synchronize()
    recon_cfg = {mode: dmd.autotune_reconstruct(m, cfg.K, mode) for mode in ("bf16x3", "fp32")}
    print(f"# reconstruction tile configs (autotuned): {recon_cfg}", file=sys.stderr, flush=True)
    st = int(m.info[0].item())
    info = m.info.cpu().tolist()
    print(f"# fit info: status {info[0]}, bisection rounds {info[1]}, eigenvalue (Aberth) iterations {info[2]}, "
          f"shifted CholeskyQR retries {info[3]}", file=sys.stderr, flush=True)
    if st != 0:
        print(json.dumps({"error": f"fit status {st}: {dmd.status_string(st)}"}), flush=True)
        sys.exit(1)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # ---- timed region: exactly `steps` whole steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        m = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    print(f"# timed {args.steps} steps: {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)

    # ---- per-stage device times (outside the timed steps)
    reps = 10
    fit_ms = _events_ms(fit_mixed, reps)
    m = fit_mixed()
    prep = dmd.PreparedReconstruction(m, ks, mode="bf16x3")
    recon_ms = _events_ms(lambda: prep.apply(Ubuf), reps)
    prep32 = dmd.PreparedReconstruction(m, ks, mode="fp32")
    recon32_ms = _events_ms(lambda: prep32.apply(Ubuf), reps)
    adj_ms = _events_ms(lambda: dmd.loss_grad(m, m.lam, m.b, Z, kfit), reps)
    recon_full_ms = _events_ms(lambda: dmd.reconstruct(m, ks, "bf16x3", out=Ubuf), reps)
    # temporal editing (Sec. 6.1) and backward roll-out (Sec. 6.2) on the same model
    edit_kw = dict(weight=(1.0, 1.5), re_scale=(1.0, 0.9), im_scale=(1.0, 1.5))
    edit_ms = _events_ms(lambda: dmd.edit_modes(m, **edit_kw), reps)
    em, _ = dmd.edit_modes(m, **edit_kw)
    edited_recon_ms = _events_ms(lambda: dmd.reconstruct(em, ks, "bf16x3", out=Ubuf), reps)
    u_last = Z[-1].contiguous()
    reverse_ms = _events_ms(lambda: dmd.reverse(m, u_last, ks + 1, "bf16x3", out=Ubuf), reps)
    # forced roll-out (Sec. 4.6): K-1 steps of synthetic forcing, K frames
    gen = torch.Generator(device="cuda").manual_seed(11)
    forcing = 1e-3 * torch.randn((cfg.K - 1, cfg.N), device="cuda", generator=gen)
    rollout_ms = _events_ms(lambda: dmd.rollout(m, forcing, mode="bf16x3"), reps)
    rollout_bytes = 4 * cfg.N * (cfg.K - 1) + 4 * cfg.N * cfg.K + 2 * 4 * cfg.N * cfg.r
    # upsampling (Sec. 6.3): K-1 guide frames, low-order half of the modes from the guide;
    # the guide buffer is reused for the constrained projection of the K-1 frames
    low = np.zeros(m.r, dtype=bool)
    low[: m.r // 2] = True
    upsample_ms = _events_ms(lambda: dmd.upsample(m, Z[0], forcing, low, mode="bf16x3"), reps)
    grid, fct = (2, 1, 256, 256), 4
    coarse = torch.randn((cfg.K - 1, cfg.N // fct ** 2), device="cuda", generator=gen)
    lowres_ms = _events_ms(lambda: dmd.lowres_project(forcing, coarse, grid, fct, out=forcing), reps)
    lowres_bytes = 2 * 4 * cfg.N * (cfg.K - 1) + 4 * (cfg.N // fct ** 2) * (cfg.K - 1)
    del forcing, coarse
    # OptDMD refinement (Sec. 4.2) on the same snapshots: the waiting call reads a device
    # flag after every 8 trial points, so wall time
    torch.cuda.synchronize()
    t_opt = time.perf_counter()
    mo = dmd.fit(Z, cfg.r, p=cfg.p, q=cfg.q, omega=om, precision="mixed", optdmd=True)
    torch.cuda.synchronize()
    optdmd_ms = 1e3 * (time.perf_counter() - t_opt)
    info_o = mo.info.cpu().numpy()

    fp64 = None
    if not args.no_fp64:
        Z64 = Z.double()
        om64 = om.double()
        fit64 = lambda: dmd.fit(Z64, cfg.r, p=cfg.p, q=cfg.q, omega=om64, precision="fp64", asynchronous=True)
        fit64_ms = _events_ms(fit64, 5)
        m64 = fit64()
        U64 = torch.empty((cfg.K, cfg.N), dtype=torch.float64, device="cuda")
        prep64 = dmd.PreparedReconstruction(m64, ks, mode="fp64")
        recon64_ms = _events_ms(lambda: prep64.apply(U64), 5)
        dmd.loss_grad(m64, m64.lam, m64.b, Z64, kfit)     # warm-up (workspace allocation)
        adj64_ms = _events_ms(lambda: dmd.loss_grad(m64, m64.lam, m64.b, Z64, kfit), 5)
        torch.cuda.synchronize()
        fp64 = {"fit_ms": round(fit64_ms, 4), "recon_ms": round(recon64_ms, 4),
                "frames_per_s": round(cfg.K / (recon64_ms * 1e-3), 1), "loss_grad_ms": round(adj64_ms, 4),
                "step_ms": round(fit64_ms + recon64_ms + adj64_ms, 4)}
        del U64, Z64

    # ---- roofline of the dominant streaming kernel (the reconstruction)
    rp = int(m.phi.shape[1])
    bytes_alg = 4 * cfg.N * cfg.K + 4 * cfg.N * cfg.r + 4 * cfg.K * cfg.r   # write U, read Phi and C once
    achieved = bytes_alg / (recon_ms * 1e-3)
    roofline = {"bound": "hbm", "achieved": round(achieved / 1e9, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK, 4), "traffic": _traffic(bytes_alg),
                "kernel": "recon_kernel<bf16x3> (dmd_reconstruct_apply)",
                "bytes_per_launch": bytes_alg, "launch_ms": round(recon_ms, 4)}

    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        import oracle
        tw, rows, Us, cpu = cpu_baseline(g, cfg)
        lam = m.lam_host()
        w = oracle.amplitude_weights(tw.phi, tw.b)
        ia, ib = oracle.match_eigs(lam, tw.lam)
        d = np.abs(lam[ia] - tw.lam[ib])
        U = dmd.reconstruct(m, ks, "bf16x3")[:, torch.from_numpy(rows).cuda()].cpu().numpy().T
        ferr = float(np.max(np.linalg.norm(U - Us, axis=0) / np.linalg.norm(Us, axis=0)))
        accuracy = {"reference": "FP64 oracle randomized twin (same sketch)",
                    "lambda_weighted_rel": float(np.sum(w[ib] * d) / np.sum(w[ib] * np.abs(tw.lam[ib]))),
                    "lambda_max_rel": float(np.max(d / np.abs(tw.lam[ib]))),
                    "field_max_frame_rel_bf16x3": ferr, "field_rows_sampled": int(rows.size)}

    out = {
        "metric": METRIC,
        "value": round(cfg.K / (ms_per_step * 1e-3), 1),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c2: randomized-SVD DMD fit + 1000-frame reconstruction + adjoint, "
                               "N=131072 (2x256x256), m=200, r=150, p=10, q=2, noise 1e-4",
                   "N": cfg.N, "m": cfg.m, "r": cfg.r, "p": cfg.p, "q": cfg.q, "K": cfg.K,
                   "fit": "mixed (FP32 MFMA streaming, FP64 Gram/small factors)",
                   "reconstruction": "bf16x3 (split-BF16 MFMA, FP32 accumulate)",
                   "recon_tile_config": recon_cfg},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "mixed": {"fit_ms": round(fit_ms, 4), "recon_ms": round(recon_ms, 4),
                  "recon_with_coeffs_ms": round(recon_full_ms, 4),
                  "frames_per_s": round(cfg.K / (recon_ms * 1e-3), 1),
                  "recon_fp32_ms": round(recon32_ms, 4), "loss_grad_ms": round(adj_ms, 4)},
        "editing": {"edit_ms": round(edit_ms, 4), "edited_recon_ms": round(edited_recon_ms, 4),
                    "reverse_ms": round(reverse_ms, 4),
                    "reverse": "project the last snapshot, then 1000 frames of Lambda^-k (bf16x3)",
                    "rollout_ms": round(rollout_ms, 4),
                    "rollout_gb_s": round(rollout_bytes / (rollout_ms * 1e-3) / 1e9, 1),
                    "rollout": "999 forced steps (N x 999 FP32 forcing projected on the modes) and 1000 "
                               "bf16x3 frames",
                    "upsample_ms": round(upsample_ms, 4),
                    "upsample": "999 guide frames projected, 75 low-order modes from the guide, 75 evolved, "
                                "1000 bf16x3 frames",
                    "lowres_project_ms": round(lowres_ms, 4),
                    "lowres_project_gb_s": round(lowres_bytes / (lowres_ms * 1e-3) / 1e9, 1),
                    "lowres_project": "999 frames of the 2x256x256 grid onto 4x4 block averages, in place",
                    "optdmd_fit_ms": round(optdmd_ms, 3), "optdmd_lm_steps": int(info_o[4]),
                    "optdmd_status": int(info_o[0]),
                    "optdmd": "mixed fit + variable-projection refinement over the 199 snapshots (wall time)"},
        "fp64": fp64,
        "accuracy": accuracy,
        "paper_context": {"precompute_s": 79.0, "subspace_step_us": 8.9,
                          "hardware": "2.10 GHz 32-core Intel CPU, 120 GB RAM (2D plume 256x512)"},
    }
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------- other workloads
def _say(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [os.cpu_count() or 1])
    except Exception:
        return os.cpu_count() or 1


def run_c3(args):
    """3D plume-shaped fit: 3x128^3 smooth modes (N = 6,291,456), m = 300, rank-200 system,
    noise 1e-3, randomized SVD r = 150, p = 10, q = 2; a step is the fit plus the
    reconstruction of the 300 fitted frames.  Mixed and plain FP64 fits on the same input."""
    import numpy as np
    import torch

    import paper_2502_05339_amd as dmd
    import synth

    cfg = synth.config("c3")
    _say(f"workload c3: N={cfg.N} m={cfg.m} r={cfg.r} p={cfg.p} q={cfg.q}; drawing the input")
    t0 = time.perf_counter()
    g = synth.generate(cfg, progress=_say)
    _say(f"input drawn in {time.perf_counter() - t0:.1f} s")
    Z = torch.from_numpy(np.ascontiguousarray(g.Z.T)).cuda()
    om = torch.from_numpy(np.ascontiguousarray(g.Omega.T)).cuda()
    ks = np.arange(cfg.m)
    U = torch.empty((cfg.m, cfg.N), dtype=torch.float32, device="cuda")

    def fit_mixed():
        return dmd.fit(Z, cfg.r, p=cfg.p, q=cfg.q, omega=om, precision="mixed", asynchronous=True)

    def step():
        mm = fit_mixed()
        dmd.reconstruct(mm, ks, "bf16x3", out=U)
        return mm

    # tile shapes of the fit's TN products, chosen by timing (outside the timed region)
    dmd.autotune_fit(Z, cfg.r, p=cfg.p, q=cfg.q, omega=om, precision="mixed")
    m = step()
    torch.cuda.synchronize()
    info = m.info.cpu().tolist()
    _say(f"fit info: status {info[0]}, bisection rounds {info[1]}, eigenvalue (Aberth) iterations {info[2]}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 5))
    t0 = time.perf_counter()
    for _ in range(steps):
        m = step()
    torch.cuda.synchronize()
    ms_per_step = 1e3 * (time.perf_counter() - t0) / steps
    fit_ms = _events_ms(fit_mixed, 3)
    recon_ms = _events_ms(lambda: dmd.reconstruct(m, ks, "bf16x3", out=U), 3)
    _say(f"mixed: step {ms_per_step:.2f} ms, fit {fit_ms:.2f} ms, reconstruction {recon_ms:.2f} ms")

    # plain FP64 path on the same values, and agreement on a row sample
    rows = np.sort(np.random.default_rng(3).choice(cfg.N, 65536, replace=False))
    rows_t = torch.from_numpy(rows).cuda()
    Um = dmd.reconstruct(m, ks, "fp32")[:, rows_t].double().cpu().numpy()
    fp64 = None
    agree = None
    if not args.no_fp64:
        del U
        Z64 = Z.double()
        om64 = om.double()
        fit64 = lambda: dmd.fit(Z64, cfg.r, p=cfg.p, q=cfg.q, omega=om64, precision="fp64", asynchronous=True)
        m64 = fit64()
        torch.cuda.synchronize()
        fit64_ms = _events_ms(fit64, 2)
        U64 = dmd.reconstruct(m64, ks, "fp64")[:, rows_t].cpu().numpy()
        fp64 = {"fit_ms": round(fit64_ms, 3)}
        agree = float(np.linalg.norm(Um - U64) / np.linalg.norm(U64))
        _say(f"fp64: fit {fit64_ms:.2f} ms; mixed vs FP64 fields on {rows.size} rows: {agree:.3e}")
        del Z64, m64
    Zs = g.Z[rows].astype(np.float64).T
    resid = float(np.linalg.norm(Um - Zs) / np.linalg.norm(Zs))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        sub = np.sort(np.random.default_rng(4).choice(cfg.N, 131072, replace=False))
        Zd = g.Z[sub].astype(np.float64)
        t0 = time.perf_counter()
        tw = oracle.fit_randomized(Zd, cfg.r, g.Omega.astype(np.float64), cfg.q)
        oracle.reconstruct(tw.phi, tw.lam, tw.b, ks)
        t_sub = time.perf_counter() - t0
        t_full = t_sub * cfg.N / sub.size
        cpu = {"value": round(cfg.m / t_full, 3), "unit": "frames/s", "cores": int(_threads()), "kind": "oracle",
               "sample": (f"FP64 NumPy randomized twin fit + reconstruction of the {cfg.m} fitted frames on "
                          f"{sub.size} of {cfg.N} rows ({t_sub:.2f} s), scaled linearly to N")}
    return {
        "value": round(cfg.m / (ms_per_step * 1e-3), 1), "unit": "frames/s", "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "scaling": "weak", "dtype": "f32",
        "config": {"workload": "c3: 3D plume-shaped randomized-SVD DMD fit + reconstruction of the 300 fitted "
                               "frames, N=6291456 (3x128^3), m=300, r=150, p=10, q=2, noise 1e-3",
                   "N": cfg.N, "m": cfg.m, "r": cfg.r, "p": cfg.p, "q": cfg.q, "K": cfg.m},
        "mixed": {"fit_ms": round(fit_ms, 3), "recon_bf16x3_ms": round(recon_ms, 3),
                  "fit_info": {"bisection_rounds": info[1], "aberth_iterations": info[2]}},
        "fp64": fp64,
        "accuracy": {"fields_mixed_vs_fp64_rel": agree, "fields_vs_data_rel": resid,
                     "rows_sampled": int(rows.size)},
        "cpu_baseline": cpu,
    }


def run_c4(args):
    """Adjoint-driven refit: c2's grid with a rank-40 system and 1% noise; the mixed fit at
    r = 40, then 200 refit steps on (lambda, b) with the modes fixed over k = 0..199; a step
    of the metric is one refit step.  The timed refit reduces the frames once to the
    statistics Phi_f^T X, Phi_f^T Phi_f and ||X||^2 (inside the timed region) and takes each
    step's loss and hand-written adjoint from them; the refit that evaluates the residual
    against the frames at every step is timed beside it.  OptDMD (variable projection) on
    the same input is reported as well."""
    import numpy as np
    import torch

    import oracle
    import paper_2502_05339_amd as dmd
    import synth
    from oracle.metrics import eig_errors

    cfg = synth.config("c4")
    _say(f"workload c4: N={cfg.N} m={cfg.m} r={cfg.r} p={cfg.p} q={cfg.q}; drawing the input")
    g = synth.generate(cfg)
    Z = torch.from_numpy(np.ascontiguousarray(g.Z.T)).cuda()
    om = torch.from_numpy(np.ascontiguousarray(g.Omega.T)).cuda()
    ks = np.arange(cfg.m)
    m = dmd.fit(Z, cfg.r, p=cfg.p, q=cfg.q, omega=om, precision="mixed")
    truth = np.concatenate([g.lam, np.conj(g.lam)])
    wt = np.abs(np.concatenate([g.b, np.conj(g.b)]))          # generating amplitudes (unit modes)
    err = lambda lam: eig_errors(lam, truth, weights=wt)["weighted_rel"]
    e_fit = err(m.lam_host())
    dmd.loss_grad(m, m.lam, m.b, Z, ks)               # warm-up (workspace allocation)
    lg_ms = _events_ms(lambda: dmd.loss_grad(m, m.lam, m.b, Z, ks), 10)
    nsteps = 200
    dmd.refit(m, Z, ks, steps=3)                      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam_r, b_r, losses = dmd.refit(m, Z, ks, steps=nsteps)
    torch.cuda.synchronize()
    refit_s = time.perf_counter() - t0
    # the same refit evaluating the residual against the frames at every step
    t0 = time.perf_counter()
    _, _, losses_res = dmd.refit(m, Z, ks, steps=nsteps, stats=False)
    torch.cuda.synchronize()
    refit_res_s = time.perf_counter() - t0
    rs = dmd.RefitStats(m, Z, ks)
    prep_ms = _events_ms(lambda: dmd.RefitStats(m, Z, ks), 5)
    lgs_ms = _events_ms(lambda: rs.loss_grad(m.lam, m.b), 10)
    e_refit = err(lam_r.cpu().numpy())
    t0 = time.perf_counter()
    mo = dmd.fit(Z, cfg.r, p=cfg.p, q=cfg.q, omega=om, precision="mixed", optdmd=True)
    torch.cuda.synchronize()
    opt_ms = 1e3 * (time.perf_counter() - t0)
    e_opt = err(mo.lam_host())
    _say(f"loss+grad {lg_ms:.3f} ms (from the statistics {lgs_ms:.3f} ms, statistics {prep_ms:.3f} ms); "
         f"{nsteps} refit steps {refit_s:.3f} s ({refit_res_s:.3f} s on the residual path); "
         f"amplitude-weighted lambda error vs "
         f"the generating system: fit {e_fit:.3e}, refit {e_refit:.3e}, OptDMD {e_opt:.3e}")
    cpu = None
    if not args.no_cpu_baseline:
        rows = np.sort(np.random.default_rng(5).choice(cfg.N, 32768, replace=False))
        phi = m.complex_modes(torch.from_numpy(rows).cuda())
        lam, b = m.lam_host(), m.b_host()
        Xt = g.Z[rows].astype(np.float64)
        t0 = time.perf_counter()
        oracle.loss_grad(phi, lam, b, Xt, ks)
        t_sub = time.perf_counter() - t0
        cpu = {"value": round(rows.size / cfg.N / t_sub, 3), "unit": "refit steps/s", "cores": int(_threads()),
               "kind": "oracle",
               "sample": (f"one FP64 NumPy loss + closed-form gradient on {rows.size} of {cfg.N} rows "
                          f"({t_sub:.3f} s), scaled linearly to N")}
    return {
        "value": round(nsteps / refit_s, 1), "unit": "refit steps/s", "steps": nsteps, "warmup": 3,
        "ms_per_step": round(1e3 * refit_s / nsteps, 4), "scaling": "weak", "dtype": "f32",
        "config": {"workload": "c4: rank-40 system on c2's grid (N=131072), 200 snapshots, noise 1e-2; mixed "
                               "fit r=40, then Adam refit of (lambda, b) with the modes fixed over k=0..199",
                   "N": cfg.N, "m": cfg.m, "r": cfg.r, "p": cfg.p, "q": cfg.q},
        "loss_grad_ms": round(lg_ms, 4),
        "refit_statistics": {"prepare_ms": round(prep_ms, 4), "loss_grad_ms": round(lgs_ms, 4),
                             "residual_path_steps_per_s": round(nsteps / refit_res_s, 1),
                             "largest_relative_loss_difference_of_the_two_paths":
                                 float(np.max(np.abs(losses - losses_res) / np.abs(losses_res)))},
        "loss_first_last": [float(losses[0]), float(losses[-1])],
        "lambda_weighted_error_vs_truth": {"fit": e_fit, "refit": e_refit, "optdmd": e_opt,
                                           "weights": "generating amplitudes |b|"},
        "optdmd_fit_ms": round(opt_ms, 3), "optdmd_lm_steps": int(mo.info.cpu().numpy()[4]),
        "cpu_baseline": cpu,
    }


def run_c5a(args):
    """Batched reconstruction: a synthetic 3D model (3x192x96x96 = 5,308,416 DOFs, 75 smooth
    conjugate pairs, r = 150), 4096 frames k in [0, 5000] in one persistent launch."""
    import numpy as np
    import torch

    import oracle
    import paper_2502_05339_amd as dmd
    import synth

    cfg = synth.config("c5a")
    _say(f"workload c5a: N={cfg.N} r={cfg.r} K={cfg.K}; drawing the model")
    phi, lam, b = synth.synthetic_model(cfg, progress=_say)
    model = dmd.Model.from_pairs(phi, lam, b, dtype=torch.float32)
    ks = synth.c5a_frames(cfg.K)
    U = torch.empty((cfg.K, cfg.N), dtype=torch.float32, device="cuda")
    _say(f"output buffer {U.numel() * 4 / 2 ** 30:.1f} GiB")
    res = {}
    tiles = {}
    for mode in ("bf16", "bf16x3", "fp32"):
        tiles[mode] = dmd.autotune_reconstruct(model, cfg.K, mode)
        prep = dmd.PreparedReconstruction(model, ks, mode=mode)
        prep.apply(U)
        torch.cuda.synchronize()
        t = _events_ms(lambda: prep.apply(U), 3)
        res[mode] = t
        _say(f"{mode}: {t:.2f} ms per {cfg.K} frames")
    # parity on a row sample against the oracle (complex modes, both members of each pair)
    rows = np.sort(np.random.default_rng(5).choice(cfg.N, 2048, replace=False))
    pc = phi[rows].astype(np.complex128)
    full_phi = np.empty((rows.size, 2 * cfg.nc), dtype=np.complex128)
    full_phi[:, 0::2], full_phi[:, 1::2] = pc, np.conj(pc)
    lam_f = np.empty(2 * cfg.nc, dtype=np.complex128)
    b_f = np.empty(2 * cfg.nc, dtype=np.complex128)
    lam_f[0::2], lam_f[1::2] = lam, np.conj(lam)
    b_f[0::2], b_f[1::2] = b, np.conj(b)
    ref = oracle.reconstruct(full_phi, lam_f, b_f, ks)
    rows_t = torch.from_numpy(rows).cuda()
    err = {}
    for mode in ("bf16", "bf16x3", "fp32"):
        dmd.PreparedReconstruction(model, ks, mode=mode).apply(U)
        got = U[:, rows_t].double().cpu().numpy().T
        fr = np.linalg.norm(got - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)
        err[mode] = float(fr.max())
    t = res["bf16"]
    bytes_alg = 4 * cfg.N * cfg.K + 4 * cfg.N * cfg.r + 2 * cfg.K * cfg.r
    cpu = None
    if not args.no_cpu_baseline:
        sub = rows[:1024]
        t0 = time.perf_counter()
        oracle.reconstruct(full_phi[:sub.size], lam_f, b_f, ks)
        t_sub = time.perf_counter() - t0
        cpu = {"value": round(cfg.K / (t_sub * cfg.N / sub.size), 3), "unit": "frames/s", "cores": int(_threads()),
               "kind": "oracle", "sample": f"FP64 NumPy reconstruction of all {cfg.K} frames on {sub.size} of "
                                           f"{cfg.N} rows ({t_sub:.2f} s), scaled linearly to N"}
    return {
        "value": round(cfg.K / (t * 1e-3), 1), "unit": "frames/s", "steps": 3, "warmup": 1,
        "ms_per_step": round(t, 3), "scaling": "weak", "dtype": "bf16",
        "config": {"workload": "c5a: batched reconstruction, N=5308416 (3x192x96x96), r=150 (75 smooth pairs), "
                               "4096 frames k in [0, 5000], BF16 modes and coefficients, FP32 accumulation",
                   "N": cfg.N, "r": cfg.r, "K": cfg.K},
        "roofline": {"bound": "hbm", "achieved": round(bytes_alg / (t * 1e-3) / 1e9, 1), "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": round(bytes_alg / (t * 1e-3) / HBM_PEAK, 4), "traffic": None,
                     "kernel": "recon_kernel<bf16>", "bytes_per_launch": bytes_alg, "launch_ms": round(t, 3)},
        "modes_ms": {k: round(v, 3) for k, v in res.items()},
        "recon_tile_config": tiles,
        "accuracy": {"reference": "FP64 oracle reconstruction on 2048 sampled rows, all frames",
                     "field_max_frame_rel": err},
        "cpu_baseline": cpu,
    }


def run_c5b(args):
    """Eight fits of uneven size (N 65,536 .. 2,097,152, m 100 .. 300, r = 64, p = 10, q = 2)
    captured into one HIP graph, against the same fits launched one after another."""
    import numpy as np
    import torch

    import paper_2502_05339_amd as dmd
    import synth

    scenes = []
    total_frames = 0
    for sc in synth.c5b_scenes():
        cfg = synth.c5b_config(sc)
        g = synth.generate(cfg)
        Z = torch.from_numpy(np.ascontiguousarray(g.Z.T)).cuda()
        om = torch.from_numpy(np.ascontiguousarray(g.Omega.T)).cuda()
        scenes.append({"Z": Z, "r": cfg.r, "p": cfg.p, "q": cfg.q, "omega": om, "precision": "mixed"})
        total_frames += cfg.m
        _say(f"scene N={cfg.N} m={cfg.m} drawn")
    # tile shapes of every scene's TN products, chosen by timing before the graph is captured
    for s in scenes:
        dmd.autotune_fit(s["Z"], s["r"], p=s["p"], q=s["q"], omega=s["omega"], precision="mixed")
    bf = dmd.BatchedFit(scenes, capture=True)
    for _ in range(2):
        bf.launch()
    torch.cuda.synchronize()
    st = bf.statuses()
    t_graph = _events_ms(bf.launch, 5)

    def seq():
        for s in scenes:
            dmd.fit(s["Z"], s["r"], p=s["p"], q=s["q"], omega=s["omega"], precision="mixed", asynchronous=True)
    seq()
    torch.cuda.synchronize()
    t_seq = _events_ms(seq, 3)
    _say(f"graph {t_graph:.2f} ms, sequential {t_seq:.2f} ms, statuses {st}")
    bf.close()
    return {
        "value": round(total_frames / (t_graph * 1e-3), 1), "unit": "frames/s", "steps": 5, "warmup": 2,
        "ms_per_step": round(t_graph, 3), "scaling": "weak", "dtype": "f32",
        "config": {"workload": "c5b: 8 randomized-SVD DMD fits of uneven size (N 65536..2097152, m 100..300, "
                               "r=64, p=10, q=2) in one captured HIP graph; value = snapshots fitted per second",
                   "scenes": [[int(s["Z"].shape[1]), int(s["Z"].shape[0])] for s in scenes]},
        "graph_ms": round(t_graph, 3), "sequential_ms": round(t_seq, 3), "statuses": st,
        "cpu_baseline": None,
    }


if __name__ == "__main__":
    main()
