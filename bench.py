"""Benchmark: time to relative residual 1e-6 and stencil-apply HBM bandwidth.

One step is one complete solve of the correlated log-normal 256^3 system
(sigma = 2, Gaussian correlation length 8 cells, c = 1e-3, x-plane Dirichlet
1/0) from a zero initial guess to a true relative residual of 1e-6: FP32
matrix-free CG with the apply fused into the vector updates and reductions,
then the FP64 true residual and, if needed, FP64 refinement. Inputs (the
coefficients and the right-hand side) are resident in device memory before
the timed region starts.

Besides the headline time it measures, on the grid's own stream with HIP
events: the stencil apply (20 algorithmic bytes per cell) against the MI355X
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
        tune = mffv.autotune(g, None)
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
           "config": {"storage": c, "wells": "injector column pw 2, producer column pw -1, WI 1",
                      "tol": 1e-6, "initial": "p = 0 inside, Dirichlet planes 1 and 0"}}
    log_fn(f"time steps: {ms_step:.1f} ms/step, iterations {res['iters_per_step']}, mass balance "
           f"{balance:.1e}, rhs kernel {rhs_us:.1f} us ({res['step_rhs_GBps']:.0f} GB/s)")
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
    HIP graph, launch shape picked by the autotuner."""
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
        opts = mffv.default_opts(tol=1e-6)
        tune = mffv.autotune_batched(grids, bs, xs, opts)
        log_fn(f"batched autotune: {tune}")
        for x in xs:
            x.zero_()
        mffv.cg_solve_batched(grids, bs, xs, opts)        # graph capture
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, infos = mffv.cg_solve_batched(grids, bs, xs, opts)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    cells = np.array([g.n for g in grids], dtype=np.float64)
    iters = np.array([i["iters"] for i in infos], dtype=np.float64)
    rr = np.array([i["rel_res_recursive"] for i in infos])
    rt = np.array([i["rel_res_true"] for i in infos])
    out = {"workload": "batched_64_uneven", "systems": len(grids), "cells_total": int(cells.sum()),
           "status": st, "wall_ms": 1e3 * wall, "device_ms": infos[0]["ms"],
           "cells_iter_per_s": float((cells * iters).sum() / wall),
           "iters_min_max": [int(iters.min()), int(iters.max())],
           "rel_res_recursive_max": float(rr.max()), "rel_res_true_max": float(rt.max()),
           "rel_res_true_median": float(np.median(rt)), "launch": tune}
    for g in grids:
        g.close()
    return out


def bench_learned(log_fn, held_in: int, held_out: int):
    """Learned preconditioner on the channelised two-facies field: train on
    held-in 32^3 realisations (seeds 3000+), confirm at 128^3 against the zero
    network, then time flexible CG against Jacobi-PCG and plain CG on held-out
    128^3 realisations (seeds 3500+) to 1e-6."""
    import numpy as np
    import torch
    from paper_2408_03452_amd import mffv, learned
    from synth import channelised

    def problem(k, stream):
        nx, ny, nz = k.shape
        n = k.size
        kd = torch.from_numpy(np.ascontiguousarray(k).ravel()).cuda()
        tx, ty, tz, b = (torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(4))
        mffv.perm_to_trans(nx, ny, nz, kd, 1.0, tx, ty, tz, stream=stream)
        g = mffv.create_grid(nx, ny, nz, stream=stream)
        mffv.set_transmissibility(g, tx, ty, tz, accum_scalar=1e-3, b_out=b)
        return g, b

    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        t0 = time.perf_counter()
        train = [problem(channelised((32, 32, 32), 3000 + i), s) for i in range(held_in)]
        confirm = [problem(channelised((128, 128, 128), 3000 + i), s) for i in range(2)]
        # epoch selection on 8 held-in 32^3 systems (the zero network, i.e. Jacobi,
        # is the first candidate)
        net = learned.train_preconditioner(train, validation=train[:8], n_white=10 * held_in,
                                           epochs=6, lr=2e-3, dagger_rounds=1, dagger_epochs=2,
                                           log=log_fn)
        t_train = time.perf_counter() - t0
        log_fn(f"learned: trained on {held_in} held-in 32^3 realisations in {t_train:.1f} s")
        zero = mffv.net_create(learned.init_params(0))
        it_net = learned.fcg_iterations(net, confirm)
        it_zero = learned.fcg_iterations(zero, confirm)
        chosen = net
        log_fn(f"learned: 128^3 held-in check, FCG iterations trained {it_net} vs zero net {it_zero}")
        methods = (("plain", mffv.default_opts()),
                   ("jacobi", mffv.default_opts(precond=mffv.PRECOND_JACOBI)),
                   ("learned_fcg", mffv.default_opts(precond=mffv.PRECOND_LEARNED, net=chosen)))
        rows = {name: [] for name, _ in methods}
        for i in range(held_out):
            g, b = problem(channelised((128, 128, 128), 3500 + i), s)
            for name, opts in methods:
                x = torch.zeros(g.n, dtype=torch.float32, device="cuda")
                if i == 0:
                    mffv.cg_solve(g, b, x, opts)
                    x.zero_()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st, info = mffv.cg_solve(g, b, x, opts)
                torch.cuda.synchronize()
                rows[name].append((time.perf_counter() - t1, info["iters"], info["rel_res_recursive"],
                                   info["rel_res_true"], st))
            g.close()
    out = {"workload": "channelised_128cube", "held_out": held_out, "held_in_32cube": held_in,
           "train_s": t_train, "check_iters_trained_vs_zero": [it_net, it_zero],
           "network": "trained" if chosen is net else "zero (Jacobi)"}
    for name, r in rows.items():
        t = np.array([v[0] for v in r])
        it = np.array([v[1] for v in r])
        out[name] = {"time_to_1e-6_s_median": float(np.median(t)), "iters_median": float(np.median(it)),
                     "rel_res_recursive_max": float(max(v[2] for v in r)),
                     "rel_res_true_max": float(max(v[3] for v in r)),
                     "all_converged": all(v[4] == 0 for v in r)}
    out["learned_vs_plain_speedup"] = out["plain"]["time_to_1e-6_s_median"] / out["learned_fcg"]["time_to_1e-6_s_median"]
    out["learned_vs_jacobi_iters"] = out["learned_fcg"]["iters_median"] / out["jacobi"]["iters_median"]

    for g, _ in train + confirm:
        g.close()
    out["_params"] = mffv.net_get_params(chosen)[0]
    return out


def bench_large_learned(log_fn, c3_params, n_crops: int = 100, n_eval: int = 4):
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
        return g, b

    def crop(pos, size):
        i, j, l = pos
        return k[i:i + size, j:j + size, l:l + size]

    out = {"workload": w.name, "finetune_crops_32cube": n_crops, "eval_crops_128cube": n_eval}
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        t1 = time.perf_counter()
        train = [problem(crop(p, 32), s) for p in positions(32, n_crops)]
        tuned = learned.train_preconditioner(train, validation=train[:8], n_white=10 * n_crops, epochs=3,
                                             lr=1e-3, dagger_rounds=1, dagger_epochs=2, init=c3_params,
                                             log=log_fn)
        out["finetune_s"] = time.perf_counter() - t1
        log_fn(f"large-learned: fine-tuned on {n_crops} crops of 32^3 in {out['finetune_s']:.1f} s")
        c3 = mffv.net_create(c3_params)
        # (name, preconditioner, network)
        methods = (("plain", mffv.PRECOND_NONE, None),
                   ("jacobi", mffv.PRECOND_JACOBI, None),
                   ("learned_fcg_channelised_net", mffv.PRECOND_LEARNED, c3),
                   ("learned_fcg_finetuned", mffv.PRECOND_LEARNED, tuned))
        rows = {name: [] for name, _, _ in methods}
        for pos in positions(128, n_eval):
            g, b = problem(crop(pos, 128), s)
            for name, pre, net in methods:
                x = torch.zeros(g.n, dtype=torch.float32, device="cuda")
                mffv.cg_solve(g, b, x, mffv.default_opts(max_iter=4, precond=pre, net=net))
                x.zero_()
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                st, info = mffv.cg_solve(g, b, x, mffv.default_opts(precond=pre, net=net))
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
        for name, pre, net in methods:
            iters = 20 if pre == mffv.PRECOND_LEARNED else 100
            x = torch.zeros(g.n, dtype=torch.float32, device="cuda")
            o = mffv.default_opts(tol=1e-30, max_iter=iters, precond=pre, net=net)
            mffv.cg_solve(g, b, x, mffv.default_opts(tol=1e-30, max_iter=4, precond=pre, net=net))
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


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lognormal_corr8_256cube")
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-jacobi", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-timesteps", action="store_true")
    ap.add_argument("--no-faces", action="store_true")
    ap.add_argument("--faces-rcm", action="store_true",
                    help="also renumber the randomly numbered face-list mesh with mffv_face_order (about 30 s on the host)")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-held-out", type=int, default=10,
                    help="held-out 128^3 realisations in the learned comparison (50 = full set)")
    ap.add_argument("--learned-held-in", type=int, default=200)
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 512x512x1024 apply / CG-rate measurement")
    ap.add_argument("--large-learned", action="store_true",
                    help="fine-tune the learned preconditioner on crops of the 512x512x1024 workload and "
                         "compare the methods there (needs the learned section)")
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
        # launch shape of the stencil kernels: the library's autotuner (bitwise
        # apply probe, timed phase A), outside the timed region
        tune = mffv.autotune(g, None)
        log(f"autotune: CG kernels ci {tune['ci']}, remap {tune['remap']}, seg {tune['seg']}, {tune['blocks']} "
            f"blocks, phase A {tune['phase_a_us']:.1f} us; apply ci {tune['apply_ci']}, remap "
            f"{tune['apply_remap']}, seg {tune['apply_seg']}, {tune['apply_us']:.1f} us ({tune['candidates']} candidates)")
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

        # the dominant kernel of the step (the single-reduction CG iteration, or
        # phase A of the two-phase iteration), timed per launch with HIP events on
        # the grid's stream during one more (untimed) solve with the same options
        x.zero_()
        st, tinfo = mffv.cg_solve(g, b, x, mffv.default_opts(
            tol=w.tol, precision=mffv.FP32_IR, check_every=16, use_graph=1, timing=1))
        merged = tinfo["single_reduction"] == 1
        dom_us = tinfo["phase_a_us"]
        dom_bytes = MERGED_BYTES_PER_CELL if merged else phase_a_bytes_mean(tinfo["timed_iters"])
        dom_gbps = dom_bytes * n / (dom_us * 1e-6) / 1e9
        log(f"{'single-reduction iteration' if merged else 'phase A'}: {dom_us:.1f} us/launch "
            f"({dom_gbps:.0f} GB/s algorithmic), over {tinfo['timed_iters']} iterations")
        traffic = TRAFFIC["single_reduction" if merged else "two_phase"]
        # both forms of the iteration, per launch (the other one for comparison)
        forms = {}
        for sr in (0, 1):
            if sr == int(merged):
                tf = tinfo
            else:
                x.zero_()
                st, tf = mffv.cg_solve(g, b, x, mffv.default_opts(
                    tol=w.tol, precision=mffv.FP32_IR, check_every=16, use_graph=1, timing=1,
                    single_reduction=sr))
            forms[sr] = tf
        phase_a_us, phase_b_us = forms[0]["phase_a_us"], forms[0]["phase_b_us"]
        phase_a_gbps = phase_a_bytes_mean(forms[0]["timed_iters"]) * n / (phase_a_us * 1e-6) / 1e9
        phase_b_gbps = PHASE_B_BYTES_PER_CELL * n / (phase_b_us * 1e-6) / 1e9
        merged_us = forms[1]["phase_a_us"]
        merged_gbps = MERGED_BYTES_PER_CELL * n / (merged_us * 1e-6) / 1e9
        log(f"two-phase: phase A {phase_a_us:.1f} us ({phase_a_gbps:.0f} GB/s) + phase B {phase_b_us:.1f} us "
            f"({phase_b_gbps:.0f} GB/s); single-reduction: {merged_us:.1f} us ({merged_gbps:.0f} GB/s)")

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
        # each kernel's mix of arrays read and written, streamed without its
        # arithmetic or neighbours: the achievable ceiling of that mix
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
        # phase A alternates between the odd and even mixes
        pa_ceiling_us = 0.5 * (stream_ceil["phase_a_odd"]["us"] + stream_ceil["phase_a_even"]["us"])
        stream_ceil["phase_a_vs_its_mix"] = pa_ceiling_us / phase_a_us
        stream_ceil["apply_vs_its_mix"] = stream_ceil["apply"]["us"] / (apply_ms * 1e3)
        log("stream mixes: " + ", ".join(f"{k} {v['us']:.1f} us ({v['GBps']:.0f} GB/s)"
                                          for k, v in stream_ceil.items() if isinstance(v, dict))
            + f"; phase A runs at {stream_ceil['phase_a_vs_its_mix']:.2f} of its mix's rate, the apply at "
              f"{stream_ceil['apply_vs_its_mix']:.2f}")
    torch.cuda.synchronize()

    tsteps = None
    if not args.no_timesteps:
        tsteps = bench_time_steps(log, w.shape, tx, ty, tz)
    face_res = None
    if not args.no_faces:
        face_res = bench_faces(log, w.shape, tx, ty, tz, w.c, rcm=args.faces_rcm)
    del tx, ty, tz
    large = None
    if not args.no_large:
        large = bench_large(log, args.large_solve)
    batched = None
    if not args.no_batched:
        log("batched: 64 uneven systems, one persistent launch")
        batched = bench_batched(log)
        log(f"batched: {batched['cells_iter_per_s'] / 1e9:.1f} Gcell*iter/s, iters "
            f"{batched['iters_min_max']}, worst true rel-res {batched['rel_res_true_max']:.2e}")
    learned_res = None
    large_learned = None
    if not args.no_learned:
        learned_res = bench_learned(log, args.learned_held_in, args.learned_held_out)
        c3_params = learned_res.pop("_params")
        log("learned: median time to 1e-6 (iterations): " + ", ".join(
            f"{k} {learned_res[k]['time_to_1e-6_s_median']*1e3:.1f} ms ({learned_res[k]['iters_median']:.0f})"
            for k in ("plain", "jacobi", "learned_fcg")))
        if args.large_learned:
            large_learned = bench_large_learned(log, c3_params)
    elif args.large_learned:
        log("large-learned: skipped (it fine-tunes the network of the learned section, which --no-learned removes)")

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
                   "precond": "none", "initial_guess": "zero",
                   "launch": {k: tune[k] for k in LAUNCH_KEYS}},
        "iters": iters,
        "rel_res_true": infos[-1]["rel_res_true"],
        "ir_steps": infos[-1]["ir_steps"],
        "cells_iter_per_s": gpu_rate,
        "cg_effective_GBps": (MERGED_BYTES_PER_CELL if merged else CG_BYTES_PER_CELL_ITER) * gpu_rate / 1e9,
        "single_reduction": merged,
        "apply_us": apply_ms * 1e3,
        "apply_GBps": apply_gbps,
        "copy_probe_GBps": copy_gbps,
        "jacobi_pcg": jac,
        "large": large,
        "stream_ceilings": stream_ceil,
        "time_steps": tsteps,
        "faces": face_res,
        "batched": batched,
        "learned": learned_res,
        "large_learned": large_learned,
        "phase_a_us": phase_a_us,
        "phase_a_GBps": phase_a_gbps,
        "phase_b_us": phase_b_us,
        "phase_b_GBps": phase_b_gbps,
        "single_reduction_us": merged_us,
        "single_reduction_GBps": merged_gbps,
        "roofline": {
            "kernel": ("stencil_v4<3> (single-reduction CG iteration: residual and direction "
                       "updates, apply, deferred solution update, four dot partials)" if merged else
                       "stencil_v4<1> (fused CG phase A: direction update, apply, deferred "
                       "solution update, p.Ap partials)"),
            "bound": "hbm",
            "achieved": dom_gbps,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": dom_gbps / HBM_PEAK_GBPS,
            "traffic": traffic_for(traffic, tune),
            "traffic_source": traffic["profile"] if traffic else None,
            "bytes_per_cell": dom_bytes,
            "cells_per_launch": n,
            "launch_us": dom_us,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    g.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
