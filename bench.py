"""Benchmark: ms per linear system to relative residual 1e-10, local vs global PCG,
plus SpMV HBM GB/s, on one MI355X.

Workload (default): the 2-D 1024x1024 five-point FP64 sequence of 20 backward-
Euler systems with log-normal conductivity (sigma = 1) and a radius-40 disk
source moving 4 cells per system.  Setup (untimed) evolves the sequence on the
GPU, so every system's x^(0) = x_{k-1} and b_k are resident in HBM before the
timed region.  One step = one system solved by Algorithm 1 (local domain by
residual, Algorithm 3, E_max = 1), cycling through the 20 systems.  The global
Jacobi-PCG from the same x^(0) is timed the same way as the baseline, and the
gradient-based local domain (Algorithm 2) as a second variant.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=40)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--cpu-seconds", type=float, default=20.0)
    p.add_argument("--nx", type=int, default=1024)
    p.add_argument("--skip-spmv-hbm", action="store_true")
    return p.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is a design "
                                   "description only (see DESIGN.md)", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2001_01158_amd import lcs, workloads as W

    dev = "cuda:0"
    torch.cuda.set_device(0)
    nx = args.nx
    w = W.c2_moving_disk(nx=nx, ny=nx)
    n = w.n
    log(f"workload {w.name} N={n} systems={w.n_systems}")
    A = lcs.matrix_from_numpy(w.kind, w.nx, w.ny, w.nz, w.coef, dev)
    ctx = lcs.Context()
    stream = torch.cuda.current_stream()
    inv_dt = 1.0 / w.dt
    eps = 1e-10
    opts = lcs.Options(eps=eps, precond="jacobi", n_smooth=1, check_every=8)

    # ---- setup: evolve the sequence (untimed) ----
    X = [torch.zeros(n, dtype=torch.float64, device=dev)]          # X[k] = x_{k-1}
    Bs = []
    for k in range(w.n_systems):
        q = torch.as_tensor(W.disk_source(nx, nx, nx / 4.0 + 4.0 * k, nx / 2.0, 40.0, 1.0)).to(dev)
        b = X[-1] * inv_dt + q
        x = X[-1].clone()
        lcs.solve_global(A, b, x, opts, ctx=ctx)
        Bs.append(b)
        X.append(x)
    torch.cuda.synchronize()
    log("sequence ready")
    x = torch.empty(n, dtype=torch.float64, device=dev)

    def run_leg(kind: str, steps: int, warm: int, collect: bool):
        stats = []
        for s in range(warm):
            k = s % w.n_systems
            x.copy_(X[k])
            one(kind, k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            k = s % w.n_systems
            x.copy_(X[k])
            st = one(kind, k)
            if collect:
                stats.append(st)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps, stats

    def one(kind, k):
        b = Bs[k]
        if kind == "global":
            return lcs.solve_global(A, b, x, opts, ctx=ctx)
        if kind == "residual":
            return lcs.solve_local_then_global(A, b, x, "residual", "paper", eps, 1, opts, ctx=ctx)
        if kind == "residual_relmax":
            return lcs.solve_local_then_global(A, b, x, "residual", "relmax", 1e-3, 1, opts, ctx=ctx)
        return lcs.solve_local_then_global(A, b, x, "gradient", "relmax", 1e-4, 1, opts, ctx=ctx)

    # ---- timed legs ----
    ms_local, st_local = run_leg("residual", args.steps, args.warmup, True)
    log(f"local (residual, paper threshold): {ms_local:.3f} ms/system")
    ms_global, st_global = run_leg("global", args.steps, max(2, args.warmup // 2), True)
    log(f"global PCG: {ms_global:.3f} ms/system")
    ms_grad, st_grad = run_leg("gradient", args.steps, max(2, args.warmup // 2), True)
    log(f"local (gradient): {ms_grad:.3f} ms/system")
    ms_relmax, st_relmax = run_leg("residual_relmax", args.steps, max(2, args.warmup // 2), True)
    log(f"local (residual, relmax 1e-3): {ms_relmax:.3f} ms/system")

    def summary(sts):
        return {"K_mean": float(np.mean([s.K for s in sts])),
                "eta_mean": float(np.mean([s.K for s in sts]) / n),
                "its_local_mean": float(np.mean([s.its_local for s in sts])),
                "its_global_mean": float(np.mean([s.its_global for s in sts])),
                "relres_final_max": float(np.max([s.relres_final for s in sts])),
                "global_finish_fraction": float(np.mean([s.its_global > 0 for s in sts]))}

    # ---- SpMV GB/s ----
    def time_spmv(M, xx, yy, reps=50):
        lcs.spmv(M, xx, yy, reps=5, ctx=ctx)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lcs.spmv(M, xx, yy, reps=reps, ctx=ctx)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    xs = torch.rand(n, dtype=torch.float64, device=dev)
    ys = torch.empty_like(xs)
    spmv_ms = time_spmv(A, xs, ys)
    spmv_bytes = n * (3 * 8 + 8 + 8)      # C, E, N + x + y
    spmv = {"c2_5pt_fp64": {"n": n, "ms": spmv_ms, "GBs": spmv_bytes / spmv_ms / 1e6,
                            "bytes_per_row": 40, "note": "working set 40 MB: Infinity-Cache resident"}}
    hbm = None
    if not args.skip_spmv_hbm:
        n3 = 4096
        c9 = W.assemble_9pt(n3, n3, 0.25, 100.0, 30.0)
        A9 = lcs.matrix_from_numpy(W.KIND_9PT, n3, n3, 1, c9, dev, with32=True)
        del c9
        x9 = torch.rand(n3 * n3, dtype=torch.float32, device=dev)
        y9 = torch.empty_like(x9)
        ms9 = time_spmv(A9, x9, y9)
        b9 = n3 * n3 * (5 * 4 + 4 + 4)
        hbm = {"n": n3 * n3, "ms": ms9, "GBs": b9 / ms9 / 1e6, "bytes_per_row": 28,
               "frac_of_8TBs": b9 / ms9 / 1e6 / HBM_PEAK_GBS}
        spmv["c3_9pt_fp32_4096x4096"] = hbm
        log(f"SpMV 9pt FP32 4096^2: {ms9 * 1e3:.1f} us, {hbm['GBs']:.0f} GB/s")
        del A9, x9, y9

    roof = {"bound": "hbm", "kernel": "k_spmv<Stencil9<float>> (9-point FP32 SpMV, 4096x4096)",
            "achieved": hbm["GBs"] if hbm else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (hbm["GBs"] / HBM_PEAK_GBS) if hbm else None, "traffic": None}

    # ---- CPU baseline: the oracle on the same systems ----
    cpu = None
    if not args.no_cpu:
        import oracle
        Ah = oracle.csr_from_stencil(w.kind, w.nx, w.ny, w.nz, w.coef)
        t_used, done, t_glob, n_glob = 0.0, 0, 0.0, 0
        k = 1
        while t_used < args.cpu_seconds * 0.5 and done < w.n_systems:
            b = Bs[k % w.n_systems].cpu().numpy()
            x0 = X[k % w.n_systems].cpu().numpy()
            t = time.perf_counter()
            oracle.local_then_global(Ah, b, x0, oracle.MODE_RESIDUAL, eps, oracle.TH_PAPER, 1,
                                     oracle.Options(eps=eps))
            t_used += time.perf_counter() - t
            done += 1
            k += 1
        while t_glob < args.cpu_seconds * 0.5 and n_glob < 5:
            b = Bs[(n_glob + 1) % w.n_systems].cpu().numpy()
            x0 = X[(n_glob + 1) % w.n_systems].cpu().numpy()
            t = time.perf_counter()
            oracle.solve_global(Ah, b, x0, oracle.Options(eps=eps))
            t_glob += time.perf_counter() - t
            n_glob += 1
        cpu = {"value": t_used * 1e3 / done, "unit": "ms per system", "cores": 1, "kind": "oracle",
               "sample": f"oracle (serial FP64 C) Algorithm 1 with the paper threshold on {done} "
                         f"systems of the same sequence, from the GPU's x_(k-1); oracle global "
                         f"Jacobi-PCG {t_glob * 1e3 / max(n_glob, 1):.1f} ms/system on {n_glob} systems",
               "global_ms_per_system": t_glob * 1e3 / max(n_glob, 1)}
        log(f"CPU oracle: local {cpu['value']:.1f} ms/system, global {cpu['global_ms_per_system']:.1f}")

    out = {
        "metric": "ms per linear system to rel. residual 1e-10, local vs global PCG; SpMV HBM GB/s",
        "value": ms_local,
        "unit": "ms per system",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_local,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded log-normal conductivity, moving disk source)",
        "config": {"workload": f"2D {nx}x{nx} 5-point FP64, 20-system backward-Euler sequence, "
                               "sigma=1 log-normal conductivity, disk radius 40 moving 4 cells/system; "
                               "Algorithm 1, residual local domain (paper threshold eps||b||/sqrt(N), "
                               "E_max=1), Jacobi-PCG, eps=1e-10", "N": n, "systems": w.n_systems,
                   "dt": w.dt},
        "global_pcg_ms_per_system": ms_global,
        "speedup_vs_global": ms_global / ms_local,
        "local_gradient_ms_per_system": ms_grad,
        "local_residual_relmax_ms_per_system": ms_relmax,
        "local_residual": summary(st_local),
        "local_gradient": summary(st_grad),
        "local_residual_relmax": summary(st_relmax),
        "global": summary(st_global),
        "spmv": spmv,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
