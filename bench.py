"""Benchmark: time to relative residual 1e-6 and stencil-apply HBM bandwidth.

One step is one complete solve of the correlated log-normal 256^3 system
(sigma = 2, Gaussian correlation length 8 cells, c = 1e-3, x-plane Dirichlet
1/0) from a zero initial guess to a true relative residual of 1e-6: FP32
matrix-free CG with the apply fused into the vector updates and reductions,
then the FP64 true residual and, if needed, FP64 refinement. Inputs (the
coefficients and the right-hand side) are resident in device memory before
the timed region starts.

Besides the headline time it measures, on the grid's own stream with HIP
events: the stencil apply (24 algorithmic bytes per cell) against the MI355X
HBM peak, the library's streaming copy (the achievable ceiling), and the
FP64 oracle on the host (SciPy CSR CG, one thread) on a 64^3 crop of the same
field as the CPU baseline.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, published peak
APPLY_BYTES_PER_CELL = 24       # x, a, Tx, Ty, Tz read; y written (FP32)
CG_BYTES_PER_CELL_ITER = 52     # fused phase A (40) + phase B (12), FP32
METRIC = "time to rel-resid 1e-6 (learned FCG vs plain CG); stencil-apply HBM GB/s"


def cells_iter_rate(cells: float, iters: float, seconds: float) -> float:
    """The paper's throughput unit (Table III): cells x iterations / time."""
    return cells * iters / seconds


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(k, c, tol, crop=64):
    """Oracle FP64 CG (SciPy CSR product, single thread) on a crop of the field."""
    import numpy as np
    from oracle import tpfa, krylov
    kc = np.ascontiguousarray(k[:crop, :crop, :crop])
    T = tpfa.round_to_f32(*tpfa.transmissibility(kc))
    dm, pd = tpfa.x_plane_dirichlet(kc.shape)
    A, b = tpfa.assemble(*T, float(np.float32(c)), dm, pd)
    Auu, bu, _ = tpfa.reduce_to_unknowns(A, b, dm)
    t0 = time.perf_counter()
    res = krylov.cg(Auu, bu, tol=tol, max_iter=20000)
    dt = time.perf_counter() - t0
    return {
        "value": cells_iter_rate(kc.size, res.iters, dt),
        "unit": "cell*iter/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{crop}^3 crop [0:{crop}]^3 of the same field with its own x-plane Dirichlet "
                   f"planes; FP64 CG to rel-resid {tol:g}: {res.iters} iterations in {dt:.2f} s "
                   f"(SciPy CSR matvec, 1 thread of {os.cpu_count()} host cores)"),
        "time_to_solution_s": dt,
        "iters": res.iters,
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lognormal_corr8_256cube")
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-jacobi", action="store_true")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "x-slab design is described but not built.", flush=True)
        return 2

    import numpy as np
    import torch
    from paper_2408_03452_amd import mffv
    from synth import WORKLOADS, workload_field

    w = WORKLOADS[args.workload]
    nx, ny, nz = w.shape
    n = w.n
    log(f"{mffv.version()}; workload {w.name} {w.shape}, generating the field")
    k = workload_field(w)
    dev = torch.device("cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        kd = torch.from_numpy(k.ravel()).to(dev)
        tx, ty, tz, b = (torch.empty(n, dtype=torch.float32, device=dev) for _ in range(4))
        mffv.perm_to_trans(nx, ny, nz, kd, w.kz_ratio, tx, ty, tz, stream=s)
        g = mffv.create_grid(nx, ny, nz, stream=s)
        mffv.set_transmissibility(g, tx, ty, tz, accum_scalar=w.c, b_out=b)
        del kd
        x = torch.zeros(n, dtype=torch.float32, device=dev)
        opts = mffv.default_opts(tol=w.tol, precision=mffv.FP32_IR, check_every=16, use_graph=1)

        def step():
            x.zero_()
            st, info = mffv.cg_solve(g, b, x, opts)
            if st != mffv.OK:
                raise RuntimeError(f"solve did not converge: {info}")
            return info

        log(f"warmup x{args.warmup}")
        for _ in range(args.warmup):
            info = step()
        torch.cuda.synchronize()
        log(f"timed x{args.steps}")
        infos = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            infos.append(step())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms_per_step = (t1 - t0) * 1e3 / args.steps
        iters = statistics.mean(i["iters"] for i in infos)
        log(f"solve: {ms_per_step:.2f} ms, {iters:.0f} iterations, true rel-res "
            f"{infos[-1]['rel_res_true']:.3e}, ir_steps {infos[-1]['ir_steps']}")

        # Jacobi-PCG on the same system (context for the preconditioned comparison)
        jac = None
        if not args.no_jacobi:
            jopts = mffv.default_opts(tol=w.tol, precision=mffv.FP32_IR,
                                      precond=mffv.PRECOND_JACOBI, check_every=16, use_graph=1)
            x.zero_()
            mffv.cg_solve(g, b, x, jopts)
            x.zero_()
            torch.cuda.synchronize()
            tj = time.perf_counter()
            st, jinfo = mffv.cg_solve(g, b, x, jopts)
            torch.cuda.synchronize()
            jac = {"ms": (time.perf_counter() - tj) * 1e3, "iters": jinfo["iters"],
                   "rel_res_true": jinfo["rel_res_true"]}
            log(f"jacobi-pcg: {jac['ms']:.2f} ms, {jac['iters']} iterations")

        # stencil apply: HIP events on the grid's stream around back-to-back launches
        xa = torch.randn(n, dtype=torch.float32, device=dev)
        ya = torch.empty_like(xa)
        for _ in range(5):
            mffv.apply(g, xa, ya)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(args.apply_reps):
            mffv.apply(g, xa, ya)
        e1.record(s)
        e1.synchronize()
        apply_ms = e0.elapsed_time(e1) / args.apply_reps
        apply_gbps = APPLY_BYTES_PER_CELL * n / (apply_ms * 1e-3) / 1e9
        log(f"apply: {apply_ms * 1e3:.1f} us/launch, {apply_gbps:.0f} GB/s algorithmic")

        # achievable streaming ceiling: the library's own copy kernel, 1 GiB
        nbytes = 1 << 30
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            mffv.copy_probe(dst, src, nbytes, stream=s)
        e0.record(s)
        for _ in range(20):
            mffv.copy_probe(dst, src, nbytes, stream=s)
        e1.record(s)
        e1.synchronize()
        copy_ms = e0.elapsed_time(e1) / 20
        copy_gbps = 2 * nbytes / (copy_ms * 1e-3) / 1e9
        log(f"copy probe: {copy_gbps:.0f} GB/s (read + write)")
        del src, dst
    torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, 64^3 crop)")
        cpu = cpu_baseline(k, w.c, w.tol)
        log(f"cpu: {cpu['value'] / 1e6:.1f} Mcell*iter/s, {cpu['iters']} iterations")

    gpu_rate = cells_iter_rate(n, iters, ms_per_step * 1e-3)
    line = {
        "metric": METRIC,
        "value": ms_per_step * 1e-3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Gaussian-filtered log-normal permeability)",
        "config": {"workload": w.name, "grid": list(w.shape), "cells": n,
                   "sigma": w.sigma, "corr_len_cells": w.corr_len, "accumulation": w.c,
                   "tol": w.tol, "precision": "FP32 CG + FP64 true residual/refinement",
                   "precond": "none", "initial_guess": "zero"},
        "iters": iters,
        "rel_res_true": infos[-1]["rel_res_true"],
        "ir_steps": infos[-1]["ir_steps"],
        "cells_iter_per_s": gpu_rate,
        "cg_effective_GBps": CG_BYTES_PER_CELL_ITER * gpu_rate / 1e9,
        "apply_us": apply_ms * 1e3,
        "apply_GBps": apply_gbps,
        "copy_probe_GBps": copy_gbps,
        "jacobi_pcg": jac,
        "roofline": {
            "kernel": "stencil_v4<apply> (mffv_apply)",
            "bound": "hbm",
            "achieved": apply_gbps,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": apply_gbps / HBM_PEAK_GBPS,
            "traffic": None,
            "bytes_per_cell": APPLY_BYTES_PER_CELL,
            "cells_per_launch": n,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    g.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
