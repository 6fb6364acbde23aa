"""Benchmark: time to relative residual 1e-6 (learned flexible CG vs plain CG)
and stencil-apply HBM bandwidth.

One step is one complete solve of a held-out realisation of the channelised
two-facies 128^3 workload (1000 / 1 mD sinusoidal channels, c = 1e-3, x-plane
Dirichlet 1/0; held-out seeds 3500 + i) with flexible CG preconditioned by the
library's 3D-convolution network, from a zero initial guess to an FP64 true
relative residual of 1e-6 (FP32 iterations, FP64 true residual and
refinement; the FP64 field is returned). The network is trained first, on the
GPU, by the library's own kernels, on held-in realisations (not timed). Each
held-out realisation is also solved by plain CG and by Jacobi-PCG to the same
true residual. ``value`` is the median learned-FCG time over the timed steps;
the line also carries both other methods, the network layers' per-launch
times, the hidden convolution against its roofline (HBM: at 216 FLOP per byte
it lies below the BF16 ridge point; its matrix-core fraction is given too),
and each result's field error against the FP64 oracle on 64^3 crop problems.

Further sections (each a key of the JSON line): the 256^3 correlated
log-normal solve and the stencil kernels against the HBM peak and their
streaming ceilings, the 512 x 512 x 1024 anisotropic system (apply GB/s, CG
rate), 64 batched uneven systems, backward-Euler time steps with wells, the
256^3 field as a face-list mesh, and the oracle on the host as the CPU
baseline.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] ...
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
# Algorithmic bytes per cell (FP32). With a scalar accumulation and the x-plane
# Dirichlet set (every workload here) the identity coefficient is the
# accumulation itself away from the Dirichlet planes and is not a per-cell
# stream: the kernels read it only on the four planes at the ends.
APPLY_BYTES_PER_CELL = 20       # x, Tx, Ty, Tz read; y written
CG_BYTES_PER_CELL_ITER = 46     # fused phase A (34 on average) + phase B (12)
PHASE_B_BYTES_PER_CELL = 12     # r, q read; r written
# face-list apply: a, x, y per cell (12 B) and, per face, two entries (one in
# each cell's row) of neighbour index and T (16 B); the gathered neighbour
# values are taken as cache hits, slice padding is not counted


def face_apply_bytes(n: int, nfaces: int) -> int:
    return 12 * n + 16 * nfaces


STEP_RHS_BYTES_PER_CELL = 21
# arrays read / written per cell by each kernel (FP32), for the streaming probe
STREAM_MIXES = {"apply": (4, 1), "phase_a_odd": (5, 2), "phase_a_even": (7, 3), "phase_b": (2, 1)}    # b, p_old, WI, pw (4 B each) and the Dirichlet mask (1 B) read; rhs written


def phase_a_bytes(k: int) -> int:
    """Algorithmic bytes per cell of phase A of iteration k. It reads r and the
    faces Tx, Ty, Tz and writes p and q; from k = 1 on it also reads p_{k-1};
    on even k >= 2 it applies two deferred solution steps, reading x and
    p_{k-2} and writing x."""
    if k == 0:
        return 24
    return 40 if k % 2 == 0 else 28


def phase_a_bytes_mean(iters: int) -> float:
    """Mean algorithmic bytes per cell over the phase-A launches of iterations 0..iters-1."""
    iters = max(1, int(iters))
    return sum(phase_a_bytes(k) for k in range(iters)) / iters


PHASE_A_BYTES_PER_CELL = 34     # steady-state mean of phase_a_bytes over two iterations
MERGED_BYTES_PER_CELL = 44      # single-reduction iteration: r, q, p, x, Tx, Ty, Tz read;
                                # r, p, q, x written
METRIC = "time to rel-resid 1e-6 (learned FCG vs plain CG); stencil-apply HBM GB/s"
MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix-core peak
# algorithmic FLOPs per cell of each network layer: 27 taps x cin x cout x 2
NN_LAYER_FLOP_PER_CELL = (27 * 2 * 16 * 2, 27 * 16 * 16 * 2, 27 * 16 * 16 * 2, 27 * 16 * 1 * 2)
# algorithmic HBM bytes per cell of a hidden layer: 16 BF16 channels in, 16 out.
# At 13824 FLOP per 64 bytes (216 FLOP/B) the layer sits below the MI355X ridge
# point (2500 TFLOP/s / 8 TB/s = 312 FLOP/B): its roofline is the HBM one.
NN_HIDDEN_BYTES_PER_CELL = 64
# HBM bytes per launch of the hidden convolution on 128^3 from rocprofv3
# FETCH_SIZE and WRITE_SIZE (FETCH_SIZE scaled by the same counter on a copy of
# known size), or None
NN_TRAFFIC = {"hidden": {"bytes": 146_468_454,  # 38,749.8 KiB x 2 fetched + 65,536 KiB written
                          "profile": "profiles/conv3d_hidden_channelised_128cube_hbm_traffic.md"}}
# launch shapes the stencil autotuner reports: the CG kernels' and the apply's own
LAUNCH_KEYS = ("ci", "remap", "seg", "vec", "blocks", "apply_ci", "apply_remap", "apply_seg", "apply_blocks")
# HBM bytes per launch of the step's dominant kernel on the 256^3 workload from
# rocprofv3 FETCH_SIZE and WRITE_SIZE (kernel_probe at each launch shape given),
# scaled by the same counters on a copy of known size; reported only when this
# run uses that kernel and its autotuner picks one of these shapes
TRAFFIC = {
    "two_phase": {
        "profile": "profiles/stencil_cg_phase_a_lognormal_corr8_256cube_hbm_traffic.md",
        "by_launch": [            # mean over the phase-A launches of a 64-iteration solve
            ({"ci": 8, "remap": 0, "seg": -1}, 689158750),
            ({"ci": 8, "remap": 1, "seg": -1}, 653083314),
            ({"ci": 16, "remap": 0, "seg": -1}, 669059721),
            ({"ci": 16, "remap": 1, "seg": -1}, 642284444),
        ],
    },
    "single_reduction": None,
}


def traffic_for(traffic, tune):
    """Measured HBM bytes per launch at the tuned shape, or None."""
    if not traffic:
        return None
    for launch, nbytes in traffic["by_launch"]:
        if all(tune[k] == v for k, v in launch.items()):
            return nbytes
    return None


def cells_iter_rate(cells: float, iters: float, seconds: float) -> float:
    """The paper's throughput unit (Table III): cells x iterations / time."""
    return cells * iters / seconds


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bench_large(log_fn, solve: bool, cg_iters: int = 200):
    """The 512 x 512 x 1024 anisotropic workload (268 M cells, 1 GiB per FP32
    vector): stencil apply and fused CG phases timed with HIP events on the
    grid's stream at a size no cache holds, a fixed number of CG iterations
    for the per-iteration rate, and with ``solve`` the full FP32 + FP64
    refinement solve to 1e-8."""
    import torch
    from paper_2408_03452_amd import mffv
    from synth import WORKLOADS, workload_field

    w = WORKLOADS["anisotropic_512x512x1024"]
    nx, ny, nz = w.shape
    n = w.n
    t0 = time.perf_counter()
    k = workload_field(w)
    log_fn(f"large: field {w.shape} generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda")
    s = torch.cuda.Stream()
    out = {"workload": w.name, "grid": list(w.shape), "cells": n, "kz_ratio": w.kz_ratio,
           "accumulation": w.c}
    with torch.cuda.stream(s):
        kd = torch.from_numpy(k).to(dev).view(-1)
        del k
        tx, ty, tz, b = (torch.empty(n, dtype=torch.float32, device=dev) for _ in range(4))
        mffv.perm_to_trans(nx, ny, nz, kd, w.kz_ratio, tx, ty, tz, stream=s)
        del kd
        g = mffv.create_grid(nx, ny, nz, stream=s)
        mffv.set_transmissibility(g, tx, ty, tz, accum_scalar=w.c, b_out=b)
        del tx, ty, tz
        tune = mffv.autotune(g, tune_cache())
        out["launch"] = {kk: tune[kk] for kk in LAUNCH_KEYS}
        xa = torch.randn(n, dtype=torch.float32, device=dev)
        ya = torch.empty_like(xa)
        for _ in range(3):
            mffv.apply(g, xa, ya)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(20):
            mffv.apply(g, xa, ya)
        e1.record(s)
        e1.synchronize()
        apply_us = e0.elapsed_time(e1) / 20 * 1e3
        del xa, ya
        out["apply_us"] = apply_us
        out["apply_GBps"] = APPLY_BYTES_PER_CELL * n / (apply_us * 1e-6) / 1e9
        x = torch.zeros(n, dtype=torch.float32, device=dev)
        st, info = mffv.cg_solve(g, b, x, mffv.default_opts(tol=1e-30, max_iter=cg_iters, timing=1))
        bpc = MERGED_BYTES_PER_CELL if info["single_reduction"] else phase_a_bytes_mean(info["timed_iters"])
        out["single_reduction"] = info["single_reduction"] == 1
        out["iter_kernel_us"] = info["phase_a_us"]
        out["iter_kernel_GBps"] = bpc * n / (info["phase_a_us"] * 1e-6) / 1e9
        out["iter_kernel_bytes_per_cell"] = bpc
        out["phase_b_us"] = info["phase_b_us"]
        x.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, info = mffv.cg_solve(g, b, x, mffv.default_opts(tol=1e-30, max_iter=cg_iters))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        out["cg_iters_fixed"] = info["iters"]
        out["cg_ms_per_iter"] = dt * 1e3 / max(1, info["iters"])
        out["cells_iter_per_s"] = cells_iter_rate(n, info["iters"], dt)
        log_fn(f"large: apply {apply_us:.0f} us ({out['apply_GBps']:.0f} GB/s), iteration kernel "
               f"{out['iter_kernel_us']:.0f} us ({out['iter_kernel_GBps']:.0f} GB/s), CG "
               f"{out['cg_ms_per_iter']:.3f} ms/iter ({out['cells_iter_per_s'] / 1e9:.1f} Gcell*iter/s)")
        if solve:
            # FP32 CG refined in FP64 to 1e-8: one refinement step per call (each
            # FP32 solve cuts the FP64 residual by 1e2, and stops after 50,000
            # iterations), continuing from the FP64 iterate, so every step
            # reports as it ends
            del x
            x64 = torch.zeros(n, dtype=torch.float64, device=dev)
            b64 = b.double()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            iters, steps, st, rel = 0, 0, mffv.NOT_CONVERGED, 1.0
            while steps < 40:
                st, info = mffv.cg_solve_f64(g, b64, x64, mffv.default_opts(
                    tol=w.tol_refined, precision=mffv.FP32_IR, max_outer=1, inner_tol=1e-2,
                    max_iter=50000, check_every=32))
                iters += info["iters"]
                steps += info["ir_steps"]
                rel = info["rel_res_true"]
                log_fn(f"large: refinement step {steps}: {info['iters']} FP32 iterations, "
                       f"true rel-res {rel:.2e}, {time.perf_counter() - t1:.1f} s")
                if st == mffv.OK or info["iters"] == 0:
                    break
            torch.cuda.synchronize()
            out["solve"] = {"tol": w.tol_refined, "status": st, "s": time.perf_counter() - t1,
                            "iters": iters, "ir_steps": steps, "inner_tol": 1e-2,
                            "inner_max_iter": 50000, "rel_res_true": rel}
            log_fn(f"large: solve to {w.tol_refined:g}: {out['solve']['s']:.1f} s, "
                   f"{iters} iterations, true rel-res {rel:.2e}")
        g.close()
    torch.cuda.synchronize()
    return out


def bench_time_steps(log_fn, shape, tx, ty, tz, nsteps: int = 8):
    """Backward-Euler time steps with wells on the headline grid and field:
    storage c = 2^-7 per cell, an injector column (pw = 2) and a producer
    column (pw = -1) with well index 1 (Peaceman form, so the operator's
    accumulation is c + WI), the x-plane Dirichlet planes at 1 and 0. Each
    step solves from the previous pressure to a true relative residual of 1e-6
    (FP32 CG + FP64 refinement). The mass balance of one more step is checked
    from the fields in FP64; the right-hand-side kernel is timed with HIP
    events."""
    import numpy as np
    import torch
    from paper_2408_03452_amd import mffv

    nx, ny, nz = shape
    n = nx * ny * nz
    c = 2.0 ** -7
    wi = np.zeros(shape, dtype=np.float32)
    pw = np.zeros(shape, dtype=np.float32)
    inj, prod = (nx // 4, ny // 4), (3 * nx // 4, 3 * ny // 4)
    wi[inj[0], inj[1], :] = wi[prod[0], prod[1], :] = 1.0
    pw[inj[0], inj[1], :], pw[prod[0], prod[1], :] = 2.0, -1.0
    dev = torch.device("cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        wi_t, pw_t = (torch.from_numpy(a.ravel()).to(dev) for a in (wi, pw))
        b = torch.empty(n, dtype=torch.float32, device=dev)
        g = mffv.create_grid(nx, ny, nz, stream=s)
        mffv.set_transmissibility(g, tx, ty, tz, accum=wi_t + c, b_out=b)
        mffv.autotune(g, None)
        opts = mffv.default_opts(tol=1e-6, precision=mffv.FP32_IR, check_every=16, use_graph=1)
        p0 = torch.zeros(n, dtype=torch.float32, device=dev)
        p0.view(nx, ny * nz)[0] = 1.0
        p = p0.clone()
        mffv.time_steps(g, 1, b, p, c_scalar=c, wi=wi_t, pw=pw_t, opts=opts)   # warmup
        p.copy_(p0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, infos = mffv.time_steps(g, nsteps, b, p, c_scalar=c, wi=wi_t, pw=pw_t, opts=opts)
        torch.cuda.synchronize()
        ms_step = (time.perf_counter() - t0) * 1e3 / nsteps
        if st != mffv.OK:
            raise RuntimeError(f"time steps did not converge: {infos}")
        p_prev = p.clone()
        mffv.time_steps(g, 1, b, p, c_scalar=c, wi=wi_t, pw=pw_t, opts=opts)
        # right-hand-side kernel: b, p_old, wi, pw and the Dirichlet mask in, rhs out
        rhs = torch.empty_like(b)
        for _ in range(3):
            mffv.step_rhs(g, b, p_prev, rhs, c_scalar=c, wi=wi_t, pw=pw_t)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(50):
            mffv.step_rhs(g, b, p_prev, rhs, c_scalar=c, wi=wi_t, pw=pw_t)
        e1.record(s)
        e1.synchronize()
        rhs_us = e0.elapsed_time(e1) * 1e3 / 50
        # the operator with a per-cell diagonal (c + WI): the apply (24 B/cell)
        # and the fused phase A (4 B/cell more than with a uniform diagonal),
        # HIP events on the grid's stream
        xa = torch.randn(n, dtype=torch.float32, device=dev)
        ya = torch.empty_like(xa)
        for _ in range(3):
            mffv.apply(g, xa, ya)
        e0.record(s)
        for _ in range(20):
            mffv.apply(g, xa, ya)
        e1.record(s)
        e1.synchronize()
        apply_us = e0.elapsed_time(e1) * 1e3 / 20
        xt = p_prev.clone()
        _, tinfo = mffv.cg_solve(g, b, xt, mffv.default_opts(tol=1e-30, max_iter=64, timing=1))
        pa_bytes = phase_a_bytes_mean(tinfo["timed_iters"]) + 4
        del xa, ya, xt
        p0h, p1h = (t.cpu().numpy().astype(np.float64).reshape(shape) for t in (p_prev, p))
        T = [t.cpu().numpy().astype(np.float64).reshape(shape) for t in (tx, ty, tz)]
        g.close()
    # mass balance of the last step: storage change against sources, wells and
    # the flow across the Dirichlet planes (interior fluxes cancel pairwise)
    u = np.ones(shape, dtype=bool)
    u[0] = u[-1] = False
    storage = c * np.sum((p1h - p0h)[u])
    wells = np.sum((wi * (pw - p1h))[u])
    left = np.sum(T[0][0] * (1.0 - p1h[1]))
    right = np.sum(T[0][nx - 2] * (0.0 - p1h[nx - 2]))
    scale = np.sum(np.abs(wi * (pw - p1h))) + np.sum(np.abs(T[0][0] * (1.0 - p1h[1]))) + \
        np.sum(np.abs(T[0][nx - 2] * p1h[nx - 2]))
    balance = abs(storage - (wells + left + right)) / scale
    res = {"nsteps": nsteps, "ms_per_step": ms_step,
           "iters_per_step": [i["iters"] for i in infos],
           "rel_res_true_max": max(i["rel_res_true"] for i in infos),
           "mass_balance_rel": balance,
           "step_rhs_us": rhs_us,
           "step_rhs_GBps": STEP_RHS_BYTES_PER_CELL * n / (rhs_us * 1e-6) / 1e9,
           "per_cell_diagonal": {
               "apply_us": apply_us, "apply_bytes_per_cell": APPLY_BYTES_PER_CELL + 4,
               "apply_GBps": (APPLY_BYTES_PER_CELL + 4) * n / (apply_us * 1e-6) / 1e9,
               "phase_a_us": tinfo["phase_a_us"], "phase_a_bytes_per_cell": pa_bytes,
               "phase_a_GBps": pa_bytes * n / (tinfo["phase_a_us"] * 1e-6) / 1e9,
               "phase_b_us": tinfo["phase_b_us"]},
           "config": {"storage": c, "wells": "injector column pw 2, producer column pw -1, WI 1",
                      "tol": 1e-6, "initial": "p = 0 inside, Dirichlet planes 1 and 0"}}
    pc = res["per_cell_diagonal"]
    log_fn(f"time steps: {ms_step:.1f} ms/step, iterations {res['iters_per_step']}, mass balance "
           f"{balance:.1e}, rhs kernel {rhs_us:.1f} us ({res['step_rhs_GBps']:.0f} GB/s); per-cell diagonal: "
           f"apply {pc['apply_us']:.1f} us ({pc['apply_GBps']:.0f} GB/s at 24 B/cell), phase A "
           f"{pc['phase_a_us']:.1f} us ({pc['phase_a_GBps']:.0f} GB/s at {pc['phase_a_bytes_per_cell']:.1f} B/cell)")
    return res


def bench_faces(log_fn, shape, tx, ty, tz, c, cg_iters: int = 200, rcm: bool = False):
    """The headline grid and field as a face-list mesh (3 x 256^2 x 255 faces):
    the face-list apply in the Cartesian numbering and with the cells randomly
    renumbered, and the face-list CG iteration rate over a fixed number of
    iterations, each timed with HIP events on the grid's stream. With rcm, the
    random numbering is also renumbered by mffv_face_order (reverse
    Cuthill-McKee on the host) and timed again."""
    import numpy as np
    import torch
    from paper_2408_03452_amd import mffv
    from synth import cartesian_faces

    nx, ny, nz = shape
    n = nx * ny * nz
    fk, fl, ax = cartesian_faces(shape)
    dmask = np.zeros(shape, dtype=np.uint8)
    dmask[0] = dmask[-1] = 1
    pd = np.zeros(shape, dtype=np.float32)
    pd[0] = 1.0
    dev = torch.device("cuda")
    s = torch.cuda.Stream()
    nbytes = face_apply_bytes(n, int(fk.size))
    res = {"faces": int(fk.size), "bytes_per_cell": nbytes / n}
    with torch.cuda.stream(s):
        fk_t = torch.from_numpy(fk).to(dev)
        ax_t = torch.from_numpy(ax).to(dev)
        T = torch.where(ax_t == 0, tx[fk_t], torch.where(ax_t == 1, ty[fk_t], tz[fk_t])).contiguous()
        del fk_t, ax_t
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        rng = np.random.default_rng(7)
        rand = rng.permutation(n)
        cases = [("cartesian_order", None), ("random_order", rand)]
        if rcm:
            t0 = time.perf_counter()
            new = mffv.face_order(n, rand[fk], rand[fl])
            res["rcm_host_s"] = time.perf_counter() - t0
            log_fn(f"faces: reverse Cuthill-McKee of the random numbering on the host, {res['rcm_host_s']:.1f} s")
            cases.append(("rcm_of_random_order", new.astype(np.int64)[rand]))
        for label, perm in cases:
            if perm is None:
                g = mffv.create_grid_faces(n, fk, fl, stream=s)
                dm, pdv = dmask.ravel(), pd.ravel()
            else:
                g = mffv.create_grid_faces(n, perm[fk], perm[fl], stream=s)
                dm = np.empty(n, dtype=np.uint8)
                dm[perm] = dmask.ravel()
                pdv = np.empty(n, dtype=np.float32)
                pdv[perm] = pd.ravel()
            b = torch.empty(n, dtype=torch.float32, device=dev)
            mffv.set_face_transmissibility(g, T, accum_scalar=c, dmask=torch.from_numpy(dm).to(dev),
                                           pD=torch.from_numpy(pdv).to(dev), b_out=b)
            xa = torch.randn(n, dtype=torch.float32, device=dev)
            ya = torch.empty_like(xa)
            for _ in range(3):
                mffv.apply(g, xa, ya)
            e0.record(s)
            for _ in range(20):
                mffv.apply(g, xa, ya)
            e1.record(s)
            e1.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / 20
            r = {"apply_us": us, "apply_GBps": nbytes / (us * 1e-6) / 1e9}
            x = torch.zeros(n, dtype=torch.float32, device=dev)
            opts = mffv.default_opts(tol=1e-30, max_iter=cg_iters, check_every=16, use_graph=1)
            mffv.cg_solve(g, b, x, opts)
            x.zero_()
            e0.record(s)
            st, info = mffv.cg_solve(g, b, x, opts)
            e1.record(s)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            r["cg_ms_per_iter"] = ms / info["iters"]
            r["cells_iter_per_s"] = n * info["iters"] / (ms * 1e-3)
            res[label] = r
            log_fn(f"faces ({label}): apply {us:.1f} us ({r['apply_GBps']:.0f} GB/s at "
                   f"{nbytes / n:.1f} B/cell), CG {r['cg_ms_per_iter'] * 1e3:.1f} us/iter "
                   f"({r['cells_iter_per_s'] / 1e9:.1f} Gcell*iter/s)")
            g.close()
            del b, xa, ya, x
    return res


def bench_batched(log_fn):
    """64 independent uneven systems (dims uniform in [32, 128], log-normal
    sigma 1.5, c log-uniform in [1e-4, 1e-2]) in one persistent launch under a
    HIP graph, launch shape picked by the autotuner. Timed twice: with the
    blocks shared by system size (a batch solved for the first time), and with
    the shares the library takes from the previous solve's iteration counts
    (the same batch solved again)."""
    import numpy as np
    import torch
    from paper_2408_03452_amd import mffv
    from synth import batch_systems
    systems = batch_systems()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        grids, bs, xs = [], [], []
        for sy in systems:
            nx, ny, nz = sy.shape
            n = sy.k.size
            kd = torch.from_numpy(sy.k.ravel()).cuda()
            tx, ty, tz, b = (torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(4))
            mffv.perm_to_trans(nx, ny, nz, kd, 1.0, tx, ty, tz, stream=s)
            g = mffv.create_grid(nx, ny, nz, stream=s)
            mffv.set_transmissibility(g, tx, ty, tz, accum_scalar=sy.c, b_out=b)
            grids.append(g)
            bs.append(b)
            xs.append(torch.zeros(n, dtype=torch.float32, device="cuda"))
        opts = mffv.default_opts(tol=1e-6, precision=mffv.FP32_IR)
        # first with block shares by size only (a batch never solved before)
        mffv.set_batched_rebalance(False)
        tune = mffv.autotune_batched(grids, bs, xs, opts)
        log_fn(f"batched autotune: {tune}")

        def timed_solve():
            for x in xs:
                x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, infos = mffv.cg_solve_batched(grids, bs, xs, opts)
            torch.cuda.synchronize()
            return st, infos, time.perf_counter() - t0
        timed_solve()                                    # graph capture
        _, infos0, wall0 = timed_solve()
        # then with shares following the iteration counts of the solve before
        # (a batch solved again, e.g. at the next time step): one solve to see
        # them, one to capture the graph of the new shares, then the timed one
        mffv.set_batched_rebalance(True)
        timed_solve()
        mffv.set_batched_rebalance(False)
        timed_solve()
        st, infos, wall = timed_solve()
    cells = np.array([g.n for g in grids], dtype=np.float64)
    iters = np.array([i["iters"] for i in infos], dtype=np.float64)
    rr = np.array([i["rel_res_recursive"] for i in infos])
    rt = np.array([i["rel_res_true"] for i in infos])
    iters0 = np.array([i["iters"] for i in infos0], dtype=np.float64)
    out = {"workload": "batched_64_uneven", "systems": len(grids), "cells_total": int(cells.sum()),
           "status": st, "wall_ms": 1e3 * wall, "device_ms": infos[0]["ms"],
           "cells_iter_per_s": float((cells * iters).sum() / wall),
           "shares": "cells x iterations of the solve before",
           "size_shares": {"wall_ms": 1e3 * wall0, "device_ms": infos0[0]["ms"],
                           "cells_iter_per_s": float((cells * iters0).sum() / wall0)},
           "iters_min_max": [int(iters.min()), int(iters.max())],
           "rel_res_recursive_max": float(rr.max()), "rel_res_true_max": float(rt.max()),
           "rel_res_true_median": float(np.median(rt)), "launch": tune}
    for g in grids:
        g.close()
    return out


_TUNE_CACHE = None


def tune_cache() -> str:
    """A launch-shape cache file for this run (outside the repository): the
    autotuner measures each grid shape once and every later grid of the same
    shape takes its pick."""
    global _TUNE_CACHE
    if _TUNE_CACHE is None:
        import atexit
        import shutil
        import tempfile
        d = tempfile.mkdtemp(prefix="mffv_tune_")
        atexit.register(shutil.rmtree, d, True)
        _TUNE_CACHE = os.path.join(d, "tune.json")
    return _TUNE_CACHE


def make_problem(k, c, stream, kz_ratio=1.0):
    """Grid handle and right-hand side of a permeability field (x-plane
    Dirichlet 1/0, scalar accumulation c), built through the C ABI."""
    import numpy as np
    import torch
    from paper_2408_03452_amd import mffv
    nx, ny, nz = k.shape
    n = k.size
    kd = torch.from_numpy(np.ascontiguousarray(k).ravel()).cuda()
    tx, ty, tz, b = (torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(4))
    mffv.perm_to_trans(nx, ny, nz, kd, kz_ratio, tx, ty, tz, stream=stream)
    g = mffv.create_grid(nx, ny, nz, stream=stream)
    mffv.set_transmissibility(g, tx, ty, tz, accum_scalar=c, b_out=b)
    mffv.autotune(g, tune_cache())   # CG and stencil launch shapes (measured once per grid shape)
    return g, b


def solve_f64(g, b64, opts):
    """One timed solve from a zero initial guess; returns (seconds, info, x64)."""
    import torch
    from paper_2408_03452_amd import mffv
    x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, info = mffv.cg_solve_f64(g, b64, x, opts)
    torch.cuda.synchronize()
    info["status"] = st
    return time.perf_counter() - t0, info, x


def bench_channelised(log_fn, held_in: int, held_out: int, steps: int, warmup: int, train_seeds=(0, 1, 2)):
    """The headline: learned flexible CG against plain CG and Jacobi-PCG on
    held-out 128^3 channelised realisations, each solve to an FP64 true
    relative residual of 1e-6 (FP32 iterations with FP64 refinement, FP64 field
    out). The network is trained first: one network per training seed on
    held-in 32^3 realisations (seeds 3000+), the one with the fewest flexible-CG
    iterations on two held-in 128^3 realisations kept. Per realisation every method first runs a short untimed solve (its
    graph capture and workspace allocation are set-up), then the timed solve.
    The learned solves of the first ``steps`` realisations are the timed steps
    of the benchmark; the comparison covers all ``held_out`` realisations."""
    import numpy as np
    import torch
    from paper_2408_03452_amd import mffv, learned
    from synth import channelised

    shape = (128, 128, 128)
    c = 1e-3
    s = torch.cuda.Stream()
    out = {"workload": "channelised_128cube", "grid": list(shape), "cells": int(np.prod(shape)),
           "accumulation": c, "held_out": held_out, "held_in_32cube": held_in,
           "tol_true": 1e-6, "precision": "FP32 iterations, FP64 true residual and refinement, FP64 field"}
    with torch.cuda.stream(s):
        t0 = time.perf_counter()
        train = [make_problem(channelised((32, 32, 32), 3000 + i), c, s) for i in range(held_in)]
        # model selection on two held-in realisations at the full size
        select = [make_problem(channelised(shape, 3000 + i), c, s) for i in range(2)]
        net, scores = learned.train_best_of(train, select, seeds=train_seeds, validation=train[:8],
                                            n_white=10 * held_in, epochs=6, lr=2e-3, dagger_rounds=1,
                                            dagger_epochs=2, log=log_fn)
        out["train_s"] = time.perf_counter() - t0
        out["train_seed_scores_128cube_held_in"] = {str(k): v for k, v in scores.items()}
        # the sweeps' weight, chosen with the network on the same held-in 128^3 systems
        omega, wscores = learned.select_smoothing(net, select)
        out["nn_smooth"] = omega
        out["nn_smooth_scores_128cube_held_in"] = {str(w): v for w, v in wscores.items()}
        log_fn(f"channelised: sweep weight {omega} (iterations on the selection systems {wscores})")
        log_fn(f"channelised: trained {len(train_seeds)} networks on {held_in} held-in 32^3 realisations in "
               f"{out['train_s']:.1f} s; selection iterations {scores}")
        for g, _ in train + select:
            g.close()
        del train, select
        methods = {
            "learned_fcg": lambda tol=1e-6, **kw: mffv.default_opts(
                tol=tol, precision=mffv.FP32_IR, precond=mffv.PRECOND_LEARNED, net=net, nn_smooth=omega, **kw),
            "plain": lambda tol=1e-6, **kw: mffv.default_opts(tol=tol, precision=mffv.FP32_IR, **kw),
            "jacobi": lambda tol=1e-6, **kw: mffv.default_opts(
                tol=tol, precision=mffv.FP32_IR, precond=mffv.PRECOND_JACOBI, **kw),
        }
        rows = {m: [] for m in methods}
        step_times = []
        n_eval = max(held_out, steps)
        for i in range(n_eval):
            seed = 3500 + (i % held_out)
            g, b = make_problem(channelised(shape, seed), c, s)
            if i == 0:
                out["launch"] = {kk: v for kk, v in mffv.autotune(g, tune_cache()).items() if kk in LAUNCH_KEYS}
            b64 = b.double()
            for name, mk in methods.items():
                solve_f64(g, b64, mk(max_iter=16))                    # set-up: graphs, workspace
                if i == 0 and name == "learned_fcg":
                    for _ in range(warmup):
                        solve_f64(g, b64, mk())
                    # per-layer times of the network inside flexible CG (HIP events
                    # on the grid's stream), first 32 iterations
                    xt = torch.zeros(g.n, dtype=torch.float32, device="cuda")
                    _, tinfo = mffv.cg_solve(g, b, xt, mffv.default_opts(
                        tol=1e-6, precond=mffv.PRECOND_LEARNED, net=net, nn_smooth=omega, timing=1))
                    out["timing"] = {k: tinfo[k] for k in ("phase_a_us", "phase_b_us", "precond_us",
                                                            "timed_iters", "nn_layer_us", "nn_timed")}
                    # each layer's launch duration: 20 back-to-back launches between
                    # HIP events on this stream (the roofline's figure; the in-solve
                    # events above also count the gap before each launch)
                    feat = torch.empty(g.n, dtype=torch.float32, device="cuda")
                    mffv.grid_feature(g, feat)
                    gen = torch.Generator(device="cuda").manual_seed(11)
                    rh = torch.randn(g.n, dtype=torch.float32, device="cuda", generator=gen)
                    out["layer_us"] = mffv.nn_time_layers(net, shape, rh, feat, reps=20, stream=s)
                    del xt, feat, rh
                dt, info, x = solve_f64(g, b64, mk())
                if i < held_out:
                    rows[name].append((dt, info["iters"], info["ir_steps"], info["rel_res_true"],
                                       info["status"], info["fallbacks"]))
                if name == "learned_fcg" and i < steps:
                    step_times.append(dt)
                if i == 0 and name == "learned_fcg":
                    out["_x_first"] = x.cpu().numpy()
                del x
            if i < held_out and (i % 10 == 9 or i == held_out - 1):
                log_fn(f"channelised: {i + 1}/{held_out} held-out realisations; median so far (ms): " +
                       ", ".join(f"{m} {1e3 * np.median([r[0] for r in v]):.1f}" for m, v in rows.items()))
            g.close()
        out["_params"] = mffv.net_get_params(net)[0]
        net.close()
    for name, r in rows.items():
        t = np.array([v[0] for v in r])
        it = np.array([v[1] for v in r])
        out[name] = {"time_to_1e-6_s_median": float(np.median(t)), "time_to_1e-6_s_mean": float(t.mean()),
                     "iters_median": float(np.median(it)), "iters_min_max": [int(it.min()), int(it.max())],
                     "ir_steps_max": int(max(v[2] for v in r)),
                     "rel_res_true_max": float(max(v[3] for v in r)),
                     "all_converged": all(v[4] == 0 for v in r),
                     "fallbacks_max": int(max(v[5] for v in r))}
    out["learned_vs_plain_speedup"] = (out["plain"]["time_to_1e-6_s_median"] /
                                       out["learned_fcg"]["time_to_1e-6_s_median"])
    out["learned_vs_jacobi_speedup"] = (out["jacobi"]["time_to_1e-6_s_median"] /
                                        out["learned_fcg"]["time_to_1e-6_s_median"])
    out["learned_vs_jacobi_iters"] = out["learned_fcg"]["iters_median"] / out["jacobi"]["iters_median"]
    out["_step_times"] = step_times
    return out


def bench_crop_fields(log_fn, c1_field, c3_params, omega: float = 0.5):
    """GPU fields for the accuracy comparison with the oracle (made by the CPU
    baseline leg): the 32^3 workload (plain CG in FP64 and in FP32 to 1e-6),
    the [0:64]^3 crop of the 256^3 field as its own problem (FP32 CG refined to
    1e-6 and to 1e-8), and the [0:64]^3 crop of held-out channelised realisation
    3500 (learned flexible CG refined to 1e-6 and 1e-8, plain CG and
    Jacobi-PCG refined to 1e-6)."""
    import numpy as np
    import torch
    from paper_2408_03452_amd import mffv
    from synth import WORKLOADS, workload_field, channelised
    s = torch.cuda.Stream()
    res = {}
    with torch.cuda.stream(s):
        w0 = WORKLOADS["lognormal_iid_32cube"]
        k0 = workload_field(w0)
        g, b = make_problem(k0, w0.c, s)
        x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        st, info = mffv.cg_solve_f64(g, b.double(), x, mffv.default_opts(tol=1e-6, precision=mffv.FP64))
        res["c0_fp64_cg_1e-6"] = {"k": k0, "c": w0.c, "x": x.cpu().numpy(), "info": info}
        x32 = torch.zeros(g.n, dtype=torch.float32, device="cuda")
        st, info = mffv.cg_solve(g, b, x32, mffv.default_opts(tol=1e-6))
        res["c0_fp32_cg_1e-6"] = {"k": k0, "c": w0.c, "x": x32.double().cpu().numpy(), "info": info}
        g.close()
        kc = np.ascontiguousarray(c1_field[:64, :64, :64])
        g, b = make_problem(kc, 1e-3, s)
        for tol in (1e-6, 1e-8):
            _, info, x = solve_f64(g, b.double(), mffv.default_opts(tol=tol, precision=mffv.FP32_IR))
            res[f"c1_crop64_fp32_ir_{tol:g}"] = {"k": kc, "c": 1e-3, "x": x.cpu().numpy(), "info": info}
        g.close()
        k3 = np.ascontiguousarray(channelised((128, 128, 128), 3500)[:64, :64, :64])
        g, b = make_problem(k3, 1e-3, s)
        net = mffv.net_create(c3_params)
        for name, pre, tols in (("learned_fcg", mffv.PRECOND_LEARNED, (1e-6, 1e-8)),
                                ("plain", mffv.PRECOND_NONE, (1e-6,)),
                                ("jacobi", mffv.PRECOND_JACOBI, (1e-6,))):
            for tol in tols:
                lk = {"net": net, "nn_smooth": omega} if pre == mffv.PRECOND_LEARNED else {}
                _, info, x = solve_f64(g, b.double(), mffv.default_opts(
                    tol=tol, precision=mffv.FP32_IR, precond=pre, **lk))
                res[f"c3_crop64_{name}_{tol:g}"] = {"k": k3, "c": 1e-3, "x": x.cpu().numpy(), "info": info}
        net.close()
        g.close()
    torch.cuda.synchronize()
    return res


def bench_large_learned(log_fn, c3_params, n_crops: int = 100, n_eval: int = 4, omega: float = 0.5):
    """Learned preconditioner on the 512 x 512 x 1024 anisotropic workload: the
    network trained on the channelised field is fine-tuned on 32^3 crops of this
    field (white noise, then its own flexible-CG residuals), flexible CG with
    either network is compared with Jacobi-PCG and plain CG to 1e-6 on held-out
    128^3 crops, and the iteration time of each method is measured on the full
    grid (a solve of the full grid to 1e-8 with the network is beyond a bench
    run: plain CG alone needs about 400,000 iterations)."""
    import numpy as np
    import torch
    from paper_2408_03452_amd import mffv, learned
    from synth import WORKLOADS, workload_field

    w = WORKLOADS["anisotropic_512x512x1024"]
    nx, ny, nz = w.shape
    t0 = time.perf_counter()
    k = workload_field(w)
    log_fn(f"large-learned: field {w.shape} generated in {time.perf_counter() - t0:.1f} s")
    rng = np.random.default_rng(4100)

    def positions(size, count):
        return [(int(rng.integers(0, nx - size + 1)), int(rng.integers(0, ny - size + 1)),
                 int(rng.integers(0, nz - size + 1))) for _ in range(count)]

    def problem(kc, stream):
        cx, cy, cz = kc.shape
        kd = torch.from_numpy(np.ascontiguousarray(kc).ravel()).cuda()
        tx, ty, tz, b = (torch.empty(kc.size, dtype=torch.float32, device="cuda") for _ in range(4))
        mffv.perm_to_trans(cx, cy, cz, kd, w.kz_ratio, tx, ty, tz, stream=stream)
        g = mffv.create_grid(cx, cy, cz, stream=stream)
        mffv.set_transmissibility(g, tx, ty, tz, accum_scalar=w.c, b_out=b)
        mffv.autotune(g, tune_cache())   # launch shapes, measured once per grid shape
        return g, b

    def crop(pos, size):
        i, j, l = pos
        return k[i:i + size, j:j + size, l:l + size]

    out = {"workload": w.name, "finetune_crops_32cube": n_crops, "eval_crops_128cube": n_eval, "nn_smooth": omega}
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        t1 = time.perf_counter()
        train = [problem(crop(p, 32), s) for p in positions(32, n_crops)]
        tuned = learned.train_preconditioner(train, validation=train[:8], n_white=10 * n_crops, epochs=3,
                                             lr=1e-3, dagger_rounds=1, dagger_epochs=2, init=c3_params,
                                             log=log_fn)
        out["finetune_s"] = time.perf_counter() - t1
        log_fn(f"large-learned: fine-tuned on {n_crops} crops of 32^3 in {out['finetune_s']:.1f} s")
        eval_pos = positions(128, n_eval)
        # the fine-tuned network's own sweep weight, chosen on two held-in 128^3
        # crops that overlap none of the evaluation crops (the 32^3 training
        # crops favour another weight than the 128^3 systems do)
        def overlaps(p, q):
            return all(abs(a - b_) < 128 for a, b_ in zip(p, q))
        sel_pos = []
        while len(sel_pos) < 2:
            cand = positions(128, 1)[0]
            if not any(overlaps(cand, q) for q in eval_pos + sel_pos):
                sel_pos.append(cand)
        sel = [problem(crop(p, 128), s) for p in sel_pos]
        omega_t, wscores = learned.select_smoothing(tuned, sel)
        for g, _ in sel:
            g.close()
        out["nn_smooth_finetuned"] = omega_t
        log_fn(f"large-learned: sweep weight of the fine-tuned network {omega_t} (held-in 128^3 crops {wscores})")
        c3 = mffv.net_create(c3_params)
        # (name, preconditioner, network, sweep weight)
        methods = (("plain", mffv.PRECOND_NONE, None, omega),
                   ("jacobi", mffv.PRECOND_JACOBI, None, omega),
                   ("learned_fcg_channelised_net", mffv.PRECOND_LEARNED, c3, omega),
                   ("learned_fcg_finetuned", mffv.PRECOND_LEARNED, tuned, omega_t))
        rows = {name: [] for name, _, _, _ in methods}
        for pos in eval_pos:
            g, b = problem(crop(pos, 128), s)
            for name, pre, net, w_ in methods:
                x = torch.zeros(g.n, dtype=torch.float32, device="cuda")
                mffv.cg_solve(g, b, x, mffv.default_opts(max_iter=4, precision=mffv.FP32_IR, precond=pre, net=net, nn_smooth=w_))
                x.zero_()
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                st, info = mffv.cg_solve(g, b, x, mffv.default_opts(precision=mffv.FP32_IR, precond=pre, net=net, nn_smooth=w_))
                torch.cuda.synchronize()
                rows[name].append((time.perf_counter() - t2, info["iters"], info["rel_res_true"], st))
            g.close()
        out["crops_128cube"] = {
            name: {"time_to_1e-6_s_median": float(np.median([v[0] for v in r])),
                   "iters_median": float(np.median([v[1] for v in r])),
                   "rel_res_true_max": float(max(v[2] for v in r)),
                   "all_converged": all(v[3] == 0 for v in r)} for name, r in rows.items()}
        log_fn("large-learned: 128^3 crops, median time to 1e-6 (iterations): " + ", ".join(
            f"{n} {v['time_to_1e-6_s_median'] * 1e3:.1f} ms ({v['iters_median']:.0f})"
            for n, v in out["crops_128cube"].items()))
        for g, _ in train:
            g.close()
        # iteration time of each method on the full grid
        g, b = problem(k, s)
        del k
        full = {}
        for name, pre, net, w_ in methods:
            iters = 20 if pre == mffv.PRECOND_LEARNED else 100
            x = torch.zeros(g.n, dtype=torch.float32, device="cuda")
            o = mffv.default_opts(tol=1e-30, max_iter=iters, precond=pre, net=net, nn_smooth=w_)
            mffv.cg_solve(g, b, x, mffv.default_opts(tol=1e-30, max_iter=4, precond=pre, net=net, nn_smooth=w_))
            x.zero_()
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            st, info = mffv.cg_solve(g, b, x, o)
            torch.cuda.synchronize()
            full[name] = {"ms_per_iter": (time.perf_counter() - t3) * 1e3 / max(1, info["iters"]),
                          "iters": info["iters"]}
        out["full_grid_ms_per_iter"] = full
        log_fn("large-learned: full grid ms per iteration: " + ", ".join(
            f"{n} {v['ms_per_iter']:.2f}" for n, v in full.items()))
        g.close()
    return out


def cpu_baseline(c3_params, learned_iters, crop_fields, log_fn, omega: float = 0.5):
    """The CPU baseline leg: the FP64 oracle on the host, one thread.

    * The headline's baseline: one iteration of the oracle's flexible CG with
      the oracle's learned preconditioner (the trained network between two
      damped Jacobi sweeps, as the GPU solve uses it), on the [0:64]^3 crop of
      held-out realisation 3500 (network forward in NumPy plus the CSR
      products and dots), timed and scaled by the cell count (x8 to
      128^3) and by the GPU's median learned-FCG iteration count: the oracle's
      time to 1e-6 on the headline workload, extrapolated.
    * The accuracy of each GPU field of ``bench_crop_fields``: the oracle's
      reference solution (direct for 32^3, Jacobi-PCG to 1e-12 for the 64^3
      crops) and, per field, the relative L2 field error and the FP64 true
      relative residual of the returned field."""
    import numpy as np
    import scipy.sparse.linalg as spla
    from threadpoolctl import threadpool_limits
    from oracle import krylov, nn, tpfa
    from synth import channelised

    def oracle_problem(k, c):
        T = tpfa.round_to_f32(*tpfa.transmissibility(k))
        dm, pd = tpfa.x_plane_dirichlet(k.shape)
        A, b = tpfa.assemble(*T, float(np.float32(c)), dm, pd)
        Auu, bu, u = tpfa.reduce_to_unknowns(A, b, dm)
        return A, b, Auu, bu, u, dm, pd

    out = {}
    with threadpool_limits(limits=1):
        k3 = np.ascontiguousarray(channelised((128, 128, 128), 3500)[:64, :64, :64])
        A, b, Auu, bu, u, dm, pd = oracle_problem(k3, 1e-3)
        d = A.diagonal()
        ld = np.log(d)
        feat = np.where(dm.ravel(), 0.0, ld - ld[u].mean()).reshape(k3.shape)
        M = nn.learned_preconditioner(c3_params, A, dm, feat, omega=omega)

        t0 = time.perf_counter()
        z = M(bu)
        q = Auu @ z
        _ = (z @ bu, z @ q)
        t_iter = time.perf_counter() - t0
        scale = (128 ** 3) / (64 ** 3)
        out.update({
            "value": t_iter * scale * learned_iters, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"one iteration of the oracle's flexible CG with the oracle's learned preconditioner "
                       f"(the network between two damped Jacobi sweeps, omega {omega:g}: FP64 NumPy convolutions "
                       f"on BF16-rounded operands, SciPy CSR products) on the [0:64]^3 crop "
                       f"of held-out channelised realisation 3500: {t_iter:.2f} s on 1 thread of "
                       f"{os.cpu_count()} host cores; scaled x{scale:g} (cells, to 128^3) and x{learned_iters:g} "
                       f"(the GPU's median learned-FCG iteration count): time to 1e-6, extrapolated"),
            "oracle_fcg_iteration_s_64cube": t_iter,
        })
        log_fn(f"cpu: oracle learned-FCG iteration at 64^3 {t_iter:.2f} s -> {out['value']:.0f} s "
               "to 1e-6 at 128^3 (extrapolated)")
        # accuracy of the GPU fields against the oracle's reference solutions
        refs = {}
        acc = {}
        for key, f in crop_fields.items():
            kid = (id(f["k"]), f["c"])
            if kid not in refs:
                A, b, Auu, bu, u, dm, pd = oracle_problem(f["k"], f["c"])
                t1 = time.perf_counter()
                if f["k"].size <= 40 ** 3:
                    xu = spla.spsolve(Auu.tocsc(), bu)
                    how = "direct"
                else:
                    r = krylov.pcg(Auu, bu, krylov.jacobi(Auu), tol=1e-12, max_iter=50000)
                    xu, how = r.x, f"Jacobi-PCG to 1e-12 ({r.iters} iterations)"
                refs[kid] = (tpfa.scatter_solution(xu, u, pd, dm), A, b, dm, how, time.perf_counter() - t1)
            p, A, b, dm, how, tref = refs[kid]
            x = f["x"]
            acc[key] = {"field_rel_err": float(np.linalg.norm(x - p) / np.linalg.norm(p)),
                        "rel_res_true_oracle": float(tpfa.relative_residual(A, b, x, dm)),
                        "rel_res_true_gpu": f["info"]["rel_res_true"], "iters": f["info"]["iters"],
                        "reference": how, "reference_s": tref, "grid": list(f["k"].shape)}
            log_fn(f"accuracy {key}: field error {acc[key]['field_rel_err']:.2e}, true rel-res "
                   f"{acc[key]['rel_res_true_oracle']:.2e} (oracle reference: {how})")
        out["accuracy_vs_oracle"] = acc
    return out


def bench_c1(log_fn, args):
    """The 256^3 correlated log-normal workload: plain FP32 CG refined in FP64
    to the true relative residual 1e-6 and to 1e-8 (the configuration's own
    target), the fused CG kernels and the apply timed with HIP events on the
    grid's stream against the HBM peak and against streaming probes of each
    kernel's mix of arrays, and the streaming copy."""
    import numpy as np
    import torch
    from paper_2408_03452_amd import mffv
    from synth import WORKLOADS, workload_field

    w = WORKLOADS["lognormal_corr8_256cube"]
    nx, ny, nz = w.shape
    n = w.n
    log_fn(f"c1: workload {w.name} {w.shape}, generating the field")
    k = workload_field(w)
    dev = torch.device("cuda")
    s = torch.cuda.Stream()
    res = {"workload": w.name, "grid": list(w.shape), "cells": n, "sigma": w.sigma,
           "corr_len_cells": w.corr_len, "accumulation": w.c}
    with torch.cuda.stream(s):
        kd = torch.from_numpy(k.ravel()).to(dev)
        tx, ty, tz, b = (torch.empty(n, dtype=torch.float32, device=dev) for _ in range(4))
        mffv.perm_to_trans(nx, ny, nz, kd, w.kz_ratio, tx, ty, tz, stream=s)
        g = mffv.create_grid(nx, ny, nz, stream=s)
        mffv.set_transmissibility(g, tx, ty, tz, accum_scalar=w.c, b_out=b)
        del kd
        tune = mffv.autotune(g, None)
        res["launch"] = {kk: tune[kk] for kk in LAUNCH_KEYS}
        log_fn(f"c1 autotune: CG kernels ci {tune['ci']}, remap {tune['remap']}, seg {tune['seg']}, "
               f"{tune['blocks']} blocks, phase A {tune['phase_a_us']:.1f} us; apply ci {tune['apply_ci']}, "
               f"remap {tune['apply_remap']}, {tune['apply_us']:.1f} us")
        b64 = b.double()
        for tol in (1e-6, 1e-8):
            o = mffv.default_opts(tol=tol, precision=mffv.FP32_IR, check_every=16, use_graph=1)
            solve_f64(g, b64, o)                                      # warm
            dt, info, x = solve_f64(g, b64, o)
            res[f"solve_{tol:g}"] = {"s": dt, "iters": info["iters"], "ir_steps": info["ir_steps"],
                                     "rel_res_true": info["rel_res_true"], "status": info["status"],
                                     "cells_iter_per_s": cells_iter_rate(n, info["iters"], dt)}
            log_fn(f"c1: solve to true {tol:g}: {dt:.2f} s, {info['iters']} iterations, "
                   f"{info['ir_steps']} refinement steps, true rel-res {info['rel_res_true']:.2e}")
            del x
        # per-launch times of the fused CG kernels (HIP events, first 32 iterations)
        x = torch.zeros(n, dtype=torch.float32, device=dev)
        forms = {}
        for sr in (0, 1):
            x.zero_()
            _, forms[sr] = mffv.cg_solve(g, b, x, mffv.default_opts(
                tol=w.tol, precision=mffv.FP32_IR, check_every=16, use_graph=1, timing=1, single_reduction=sr))
        tinfo = forms[0]
        phase_a_us, phase_b_us = tinfo["phase_a_us"], tinfo["phase_b_us"]
        pa_bytes = phase_a_bytes_mean(tinfo["timed_iters"])
        phase_a_gbps = pa_bytes * n / (phase_a_us * 1e-6) / 1e9
        phase_b_gbps = PHASE_B_BYTES_PER_CELL * n / (phase_b_us * 1e-6) / 1e9
        merged_us = forms[1]["phase_a_us"]
        res.update({"phase_a_us": phase_a_us, "phase_a_GBps": phase_a_gbps, "phase_b_us": phase_b_us,
                    "phase_b_GBps": phase_b_gbps, "single_reduction_us": merged_us,
                    "single_reduction_GBps": MERGED_BYTES_PER_CELL * n / (merged_us * 1e-6) / 1e9})
        log_fn(f"c1: phase A {phase_a_us:.1f} us ({phase_a_gbps:.0f} GB/s) + phase B {phase_b_us:.1f} us "
               f"({phase_b_gbps:.0f} GB/s); single-reduction {merged_us:.1f} us")
        if not args.no_jacobi:
            o = mffv.default_opts(tol=w.tol, precision=mffv.FP32_IR, precond=mffv.PRECOND_JACOBI)
            solve_f64(g, b64, o)
            dt, info, xj = solve_f64(g, b64, o)
            res["jacobi_pcg_1e-6"] = {"s": dt, "iters": info["iters"], "rel_res_true": info["rel_res_true"]}
            del xj
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
        apply_us = e0.elapsed_time(e1) * 1e3 / args.apply_reps
        res["apply_us"] = apply_us
        res["apply_GBps"] = APPLY_BYTES_PER_CELL * n / (apply_us * 1e-6) / 1e9
        log_fn(f"c1: apply {apply_us:.1f} us/launch, {res['apply_GBps']:.0f} GB/s algorithmic")
        del xa, ya
        # streaming ceilings: the library's copy (1 GiB) and each kernel's mix of arrays
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
        res["copy_probe_GBps"] = 2 * nbytes / (copy_ms * 1e-3) / 1e9
        # the runtime's own device-to-device copy of the same buffers, for comparison
        for _ in range(3):
            dst.copy_(src)
        e0.record(s)
        for _ in range(20):
            dst.copy_(src)
        e1.record(s)
        e1.synchronize()
        res["runtime_copy_GBps"] = 2 * nbytes / (e0.elapsed_time(e1) / 20 * 1e-3) / 1e9
        log_fn(f"c1: copy probe {res['copy_probe_GBps']:.0f} GB/s, runtime copy {res['runtime_copy_GBps']:.0f} GB/s")
        del src, dst
        arrs = [torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0) for _ in range(10)]
        stream_ceil = {}
        for name, (ni, no) in STREAM_MIXES.items():
            ins, outs = arrs[:ni], arrs[ni:ni + no]
            for _ in range(3):
                mffv.stream_probe(ins, outs, stream=s)
            e0.record(s)
            for _ in range(20):
                mffv.stream_probe(ins, outs, stream=s)
            e1.record(s)
            e1.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / 20
            stream_ceil[name] = {"in": ni, "out": no, "us": us, "GBps": 4 * (ni + no) * n / (us * 1e-6) / 1e9}
        del arrs
        pa_ceiling_us = 0.5 * (stream_ceil["phase_a_odd"]["us"] + stream_ceil["phase_a_even"]["us"])
        stream_ceil["phase_a_vs_its_mix"] = pa_ceiling_us / phase_a_us
        stream_ceil["apply_vs_its_mix"] = stream_ceil["apply"]["us"] / apply_us
        res["stream_ceilings"] = stream_ceil
        traffic = TRAFFIC["two_phase"]
        res["stencil_roofline"] = {
            "kernel": "stencil_v4<1> (fused CG phase A: direction update, apply, deferred solution "
                      "update, p.Ap partials)",
            "bound": "hbm", "achieved": phase_a_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": phase_a_gbps / HBM_PEAK_GBPS, "traffic": traffic_for(traffic, tune),
            "traffic_source": traffic["profile"], "bytes_per_cell": pa_bytes, "cells_per_launch": n,
            "launch_us": phase_a_us}
        g.close()
    torch.cuda.synchronize()
    return res, k, tx, ty, tz


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50,
                    help="timed steps: learned-FCG solves of the first K held-out realisations")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--held-out", type=int, default=50,
                    help="held-out 128^3 realisations compared (the configuration's 50)")
    ap.add_argument("--held-in", type=int, default=200)
    ap.add_argument("--train-seeds", type=int, default=3,
                    help="networks trained (seeds 0..N-1); the one with the fewest iterations on two held-in "
                         "128^3 realisations is kept")
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-jacobi", action="store_true")
    ap.add_argument("--no-c1", action="store_true", help="skip the 256^3 section (and the sections on its field)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-timesteps", action="store_true")
    ap.add_argument("--no-faces", action="store_true")
    ap.add_argument("--faces-rcm", action="store_true",
                    help="also renumber the randomly numbered face-list mesh with mffv_face_order (about 30 s on the host)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 512x512x1024 apply / CG-rate measurement")
    ap.add_argument("--no-large-learned", action="store_true",
                    help="skip fine-tuning the learned preconditioner on crops of the 512x512x1024 workload "
                         "and comparing the methods there (on by default)")
    ap.add_argument("--large-solve", action="store_true",
                    help="also solve the 512x512x1024 system to 1e-8 (minutes)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "x-slab design is described but not built.", flush=True)
        return 2

    import numpy as np
    import torch
    from paper_2408_03452_amd import mffv

    log(f"{mffv.version()}; headline: learned flexible CG on channelised 128^3, {args.held_out} held-out "
        f"realisations, {args.steps} timed steps")
    head = bench_channelised(log, args.held_in, args.held_out, args.steps, args.warmup,
                             train_seeds=tuple(range(args.train_seeds)))
    step_times = head.pop("_step_times")
    c3_params = head.pop("_params")
    head.pop("_x_first", None)
    lf = head["learned_fcg"]
    log("channelised: median time to true 1e-6 (iterations): " + ", ".join(
        f"{m} {head[m]['time_to_1e-6_s_median'] * 1e3:.1f} ms ({head[m]['iters_median']:.0f})"
        for m in ("learned_fcg", "plain", "jacobi")))
    # the step's dominant kernel: a hidden 16 -> 16 convolution of the network
    n3 = head["cells"]
    layers = head.get("layer_us", [0.0] * 4)
    hidden_us = 0.5 * (layers[1] + layers[2])
    hidden_tflops = NN_LAYER_FLOP_PER_CELL[1] * n3 / (hidden_us * 1e-6) / 1e12 if hidden_us > 0 else 0.0
    hidden_gbs = NN_HIDDEN_BYTES_PER_CELL * n3 / (hidden_us * 1e-6) / 1e9 if hidden_us > 0 else 0.0
    head["network_layers"] = [
        {"layer": i + 1, "us": layers[i], "flop_per_cell": NN_LAYER_FLOP_PER_CELL[i],
         "TFLOPs": NN_LAYER_FLOP_PER_CELL[i] * n3 / (layers[i] * 1e-6) / 1e12 if layers[i] > 0 else 0.0}
        for i in range(4)]
    log(f"network layers (us): {[round(v, 1) for v in layers]}; hidden layer {hidden_gbs:.0f} GB/s, "
        f"{hidden_tflops:.0f} TFLOP/s")

    c1 = tsteps = face_res = None
    k1 = None
    if not args.no_c1:
        c1, k1, tx, ty, tz = bench_c1(log, args)
        if not args.no_timesteps:
            tsteps = bench_time_steps(log, tuple(c1["grid"]), tx, ty, tz)
        if not args.no_faces:
            face_res = bench_faces(log, tuple(c1["grid"]), tx, ty, tz, c1["accumulation"], rcm=args.faces_rcm)
        del tx, ty, tz
    large = None
    if not args.no_large:
        large = bench_large(log, args.large_solve)
    batched = None
    if not args.no_batched:
        log("batched: 64 uneven systems, one persistent launch")
        batched = bench_batched(log)
        log(f"batched: {batched['cells_iter_per_s'] / 1e9:.1f} Gcell*iter/s (shares by size: "
            f"{batched['size_shares']['cells_iter_per_s'] / 1e9:.1f}), iters "
            f"{batched['iters_min_max']}, worst true rel-res {batched['rel_res_true_max']:.2e}")
    large_learned = None
    if not args.no_large_learned:
        large_learned = bench_large_learned(log, c3_params, omega=head["nn_smooth"])

    cpu = None
    if not args.no_cpu_baseline:
        if k1 is None:
            from synth import WORKLOADS, workload_field
            k1 = workload_field(WORKLOADS["lognormal_corr8_256cube"])
        crops = bench_crop_fields(log, k1, c3_params, omega=head["nn_smooth"])
        log("cpu baseline (oracle on the host)")
        cpu = cpu_baseline(c3_params, lf["iters_median"], crops, log, omega=head["nn_smooth"])

    ms_per_step = 1e3 * float(np.mean(step_times))
    line = {
        "metric": METRIC,
        "value": lf["time_to_1e-6_s_median"],
        "unit": "s",
        "n_gpus": 1,
        "steps": len(step_times),
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded two-facies channelised permeability; trained network, no external data)",
        "config": {"workload": "channelised_128cube", "grid": [128, 128, 128], "cells": n3,
                   "held_out": args.held_out, "held_out_seeds": [3500, 3500 + args.held_out - 1],
                   "held_in_32cube": args.held_in, "accumulation": 1e-3, "tol_true": 1e-6,
                   "method": "flexible CG, 3D-conv network preconditioner (2-16-16-16-1, 3^3, BF16 MFMA)",
                   "precision": "FP32 iterations, FP64 true residual and refinement, FP64 field",
                   "initial_guess": "zero",
                   "value_is": "median over the held-out realisations of the learned-FCG time to true rel-res 1e-6"},
        "learned_fcg": lf,
        "plain_cg": head["plain"],
        "jacobi_pcg": head["jacobi"],
        "learned_vs_plain_speedup": head["learned_vs_plain_speedup"],
        "learned_vs_jacobi_speedup": head["learned_vs_jacobi_speedup"],
        "channelised": {k: v for k, v in head.items() if k not in ("learned_fcg", "plain", "jacobi")},
        "roofline": {
            "kernel": "conv3d<16,0> (hidden 16->16 3^3 convolution + ReLU of the network inside flexible "
                      "CG, BF16 MFMA with FP32 accumulation)",
            "bound": "hbm",
            "achieved": hidden_gbs,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": hidden_gbs / HBM_PEAK_GBPS,
            "traffic": NN_TRAFFIC["hidden"]["bytes"] if NN_TRAFFIC["hidden"] else None,
            "traffic_source": NN_TRAFFIC["hidden"]["profile"] if NN_TRAFFIC["hidden"] else None,
            "bytes_per_cell": NN_HIDDEN_BYTES_PER_CELL,
            "cells_per_launch": n3,
            "launch_us": hidden_us,
            "flop_per_cell": NN_LAYER_FLOP_PER_CELL[1],
            "mfma_tflops": hidden_tflops,
            "mfma_frac": hidden_tflops / MFMA_BF16_PEAK_TFLOPS,
        },
        "c1_256cube": c1,
        "large": large,
        "time_steps": tsteps,
        "faces": face_res,
        "batched": batched,
        "large_learned": large_learned,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
