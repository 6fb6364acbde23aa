// Matrix-free TPFA stencil kernels: the apply of Eq. 6 / Alg. 2 (sign flipped,
// plus the accumulation diagonal), the CG phase that fuses it with the
// direction update, the deferred solution update and the p.Ap reduction
// (Alg. 1), and the residual b - A x.
//
// Every kernel marches along x: a block owns a contiguous chunk of one plane
// (kThreads*vec cells, z fastest) and walks through m.ci consecutive planes,
// carrying the values of planes i-1, i, i+1 and the face Tx of plane i-1 in
// registers, so each x-neighbour and x-face is read from memory once. The z
// neighbours come from the adjacent lane by a cross-lane shuffle (only the
// first and last lane of a wave load across a wave boundary), the y neighbours
// are the rows +-nz of the same plane, which the chunk itself or the
// neighbouring chunk of the same XCD has just read. Per cell the algorithmic
// traffic of the apply is x, a, Tx, Ty, Tz in and y out: 24 bytes in FP32.
#include "launch.hpp"

#include <type_traits>

namespace mffv {

bool march_seg_ok(const Geom& g, int vec, int seg) {
    return vec == 4 && seg >= 16 && seg <= kThreads * 4 && (seg & (seg - 1)) == 0 && g.nz % seg == 0;
}

March plan_march(const Geom& g, int vec, int ci, int remap, int seg) {
    March m;
    m.vec = vec;
    const int64_t per_block = (int64_t)kThreads * vec;
    if (seg == 0) {
        // default: long rows as segments of 256 cells (4 rows per chunk; a flat
        // chunk would be a single row with every y neighbour outside it)
        seg = (vec == 4 && g.nz > kWave * 4 && g.nz % (kWave * 4) == 0) ? kWave * 4 : -1;
    }
    if (seg > 0 && march_seg_ok(g, vec, seg)) {
        // a chunk is kThreads*4/seg rows x seg cells: taller chunks keep more of
        // the y neighbours inside the chunk, at the price of z neighbours read
        // across the segment ends
        m.seg = seg;
        m.nseg = g.nz / seg;
        m.tps_log2 = 0;
        while ((1 << m.tps_log2) < seg / 4) ++m.tps_log2;
        const int rows = kThreads >> m.tps_log2;
        m.nchunk = ((g.ny + rows - 1) / rows) * m.nseg;
    } else {
        m.seg = 0;
        m.nseg = 0;
        m.tps_log2 = 0;
        m.nchunk = (int)((g.plane + per_block - 1) / per_block);
    }
    if (ci <= 0) {
        // default: enough blocks to give each CU several, but long marches
        const int64_t target = 4096;
        int64_t want = (int64_t)m.nchunk * g.nx / target;
        ci = (int)(want < 1 ? 1 : (want > 64 ? 64 : want));
        if (ci > g.nx) ci = g.nx;
    }
    m.ci = ci;
    m.nich = (g.nx + ci - 1) / ci;
    m.remap = remap;
    return m;
}

namespace {

__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
// Results are written with streaming (nontemporal) stores: they are read again
// only by the next kernel, and keeping them out of the way in L2 leaves room
// for the neighbour rows the other blocks still need.
typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st4(float* p, float4 v) {
    const f4v w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<f4v*>(p));
}
__device__ __forceinline__ float4 f4(float v) { return make_float4(v, v, v, v); }
// Two FP32 values as BF16 (round to nearest even), lo in the low half.
typedef float nn_v2f __attribute__((ext_vector_type(2)));
typedef __bf16 nn_v2bf __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pair(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((nn_v2f){lo, hi}, nn_v2bf));
}
// The network's input channels of one cell from the swept residual r1:
// t = sqrt(dinv) r1 and t f in BF16 (the scale 1/s, a power of two, is
// applied by the first convolution).
__device__ __forceinline__ uint32_t nn_pair(float d, float r1, float f) {
    const float t = sqrtf(d) * r1;
    return bf16_pair(t, t * f);
}
__device__ __forceinline__ float4 axpy4(float a, float4 x, float4 y) {
    return make_float4(y.x + a * x.x, y.y + a * x.y, y.z + a * x.z, y.w + a * x.w);
}

// Start of phase A_k of the fused CG loop. Every block sums the partials of
// the kernels before it (phase B: r.r, r.z, and at k = 0 ||b_U||^2; flexible
// CG: the preconditioner dots) in the same order, tests convergence on r_k and
// forms beta_{k-1}; block 0 records the scalars. Returns false, identically in
// every block, once the loop is over.
template <class real>
struct PhaseA {
    int k;
    real beta;        // beta_{k-1}
    real alpha_prev;  // alpha_{k-1}: the deferred solution update
    real alpha_prev2; // alpha_{k-2}: with it, on even k >= 2 (see phase A below)
    bool fallback;    // flexible CG: this iteration uses z = r / diag(A)
};

template <class real>
__device__ bool phase_a_start(const StencilIO<real>& io, real* lds, PhaseA<real>& o) {
    CgState<real>* st = io.st;
    // r.r; Jacobi: r.z; at k = 0: ||b_U||^2; flexible CG: the preconditioner's
    // z.r, z.q and the Jacobi safeguard's dinv r.r, dinv r.q; summed together
    const int nb = io.nb_b, nf = io.precond == 2 ? io.nb_f : 0;
    const real* parts[7] = {io.pb, io.pb + nb, io.pb + 2 * nb, io.pf, io.pf + nf, io.pf + 2 * nf, io.pf + 3 * nf};
    // The done flag, the loop's scalars and the first batch of partials are
    // read together, in one memory round trip. No block writes any of these
    // scalars during this kernel (block 0 writes other slots, and thresh2 and
    // bnorm2 only at k = 0, where they are formed here rather than read); the
    // ||b_U||^2 partials are loaded before k is known (their buffer always
    // holds nb entries) and added at k = 0 only.
    const int loads[7] = {nb, io.precond == 1 ? nb : 0, nb, nf, nf, nf, nf};
    real first[7][kPartBatch];
    load_partials_first(parts, loads, first);
    const int done = early_load(&st->done), k = early_load(&st->iterA), max_iter = early_load(&st->max_iter);
    const real thresh2_st = early_load(&st->thresh2), bnorm2_st = early_load(&st->bnorm2),
               tol2 = early_load(&st->tol2);
    const real alpha0 = early_load(&st->alpha[0]), alpha1 = early_load(&st->alpha[1]);
    const real rho0 = early_load(&st->rho[0]), rho1 = early_load(&st->rho[1]);
    const real pq0 = early_load(&st->pq[0]), pq1 = early_load(&st->pq[1]);
    if (block_uniform(done)) {
        drain_loads();
        return false;
    }
    const int counts[7] = {nb, io.precond == 1 ? nb : 0, k == 0 ? nb : 0, nf, nf, nf, nf};
    real sums[7];
    sum_partials_n_rest(parts, counts, first, lds, sums);
    const real rr = sums[0];
    real rho = rr, zq = 0;
    bool fallback = false;
    if (io.precond == 1) {
        rho = sums[1];
    } else if (io.precond == 2) {
        const real zr = sums[3], zqv = sums[4], jr = sums[5], jq = sums[6];
        fallback = !(zr > real(0)) || !isfinite(zr) || !isfinite(zqv);
        rho = fallback ? jr : zr;
        zq = fallback ? jq : zqv;
    }
    real thresh2 = thresh2_st, bnorm2 = bnorm2_st;
    if (k == 0) {
        const real bb = sums[2];
        bnorm2 = bb > real(0) ? bb : rr;
        thresh2 = tol2 * bnorm2;
    }
    const bool conv = isfinite(rr) && rr <= thresh2;
    const bool bad = !conv && (!isfinite(rr) || (io.precond != 0 && (!(rho > real(0)) || !isfinite(rho))));
    const bool cap = k >= max_iter;
    if (conv || bad || cap) {
        if (first_thread()) {
            st->done = 1;
            st->status = conv ? 0 : (bad ? -4 : 1);
            st->iters = k;
            // x holds the steps up to the last even k' <= k - 1: one step
            // owed for odd k, two for even k >= 2
            st->tail = k == 0 ? 0 : ((k & 1) ? 1 : 2);
            st->rr = rr;
            if (k == 0) {
                st->thresh2 = thresh2;
                st->bnorm2 = bnorm2;
            }
        }
        return false;
    }
    o.k = k;
    o.fallback = fallback;
    // slot (k - 1) & 1 and slot k & 1 (selects, not indexing: the values stay in registers)
    const bool odd = k & 1;
    o.alpha_prev = k >= 1 ? (odd ? alpha0 : alpha1) : real(0);
    o.alpha_prev2 = k >= 2 ? (odd ? alpha1 : alpha0) : real(0);  // phase B_k has not written it yet
    o.beta = k == 0 ? real(0) : (io.precond == 2 ? -zq / (odd ? pq0 : pq1) : rho / (odd ? rho0 : rho1));
    if (first_thread()) {
        st->rho[k & 1] = rho;
        st->iterB = k;
        st->rr = rr;
        st->beta = o.beta;
        st->fallback = fallback ? 1 : 0;
        if (fallback) st->fallbacks += 1;
        if (k == 0) {
            st->thresh2 = thresh2;
            st->bnorm2 = bnorm2;
        }
    }
    return true;
}

// Start of kernel K of the single-reduction CG (Chronopoulos-Gear style: one
// reduction phase per iteration). Kernel K - 1 left the partial sums of
// p.q, r.r, r.q and q.q of its iterate (pq, rho_{K-1}, rq, qq); every block sums
// them in the same order and forms
//   alpha_{K-1} = rho_{K-1} / pq,
//   rho_K = ||r_{K-1} - alpha q_{K-1}||^2 = rho_{K-1} - 2 alpha rq + alpha^2 qq,
//   beta_{K-1} = rho_K / rho_{K-1},
// the recurrence taking one step from the exact rho_{K-1}, so its rounding does
// not accumulate. The convergence test uses the exact rho_{K-1}: the run stops
// with x_{K-1}, which kernel K-1 completed. Kernel 0 takes r_0 and ||b_U||^2
// from the initial-residual partials. Returns false, identically in every
// block, once the run is over.
struct MergedPh {
    int k;
    float alpha;  // alpha_{K-1} (0 for K = 0)
    float beta;   // beta_{K-1} (0 for K = 0)
};

__device__ bool merged_start(const StencilIO<float>& io, float* lds, MergedPh& o) {
    MergedState* ms = io.ms;
    MergedSlot* cur = &ms->s[io.parity];
    MergedSlot* nxt = &ms->s[io.parity ^ 1];
    if (block_flag(&cur->done)) return false;
    const int K = cur->k;
    float rr, thresh2, bnorm2, alpha = 0.f, beta = 0.f;
    bool bad = false;
    if (K == 0) {
        rr = sum_partials(io.pb, io.nb_b, lds);
        const float bb = sum_partials(io.pb + 2 * io.nb_b, io.nb_b, lds);
        bnorm2 = bb > 0.f ? bb : rr;
        thresh2 = ms->tol2 * bnorm2;
    } else {
        const int nb = io.nb_f;
        const float pq = sum_partials(io.pf, nb, lds);
        rr = sum_partials(io.pf + nb, nb, lds);
        const float rq = sum_partials(io.pf + 2 * nb, nb, lds);
        const float qq = sum_partials(io.pf + 3 * nb, nb, lds);
        thresh2 = cur->thresh2;
        bnorm2 = cur->bnorm2;
        bad = !(pq > 0.f) || !isfinite(pq);
        alpha = rr / pq;
        const float rho = rr - 2.f * alpha * rq + alpha * alpha * qq;
        beta = rho > 0.f ? rho / rr : 0.f;  // a cancelled recurrence restarts the directions
    }
    const bool conv = isfinite(rr) && rr <= thresh2;
    bad = !conv && (bad || !isfinite(rr));
    const int done_iters = K == 0 ? 0 : K - 1;
    const bool cap = done_iters >= ms->max_iter;
    if (conv || bad || cap) {
        if (first_thread()) {
            for (MergedSlot* sl : {nxt, cur}) {
                sl->status = conv ? 0 : (bad ? -4 : 1);
                sl->iters = done_iters;
                sl->rr = rr;
                sl->thresh2 = thresh2;
                sl->bnorm2 = bnorm2;
                sl->done = 1;
            }
        }
        return false;
    }
    if (first_thread()) {
        nxt->k = K + 1;
        nxt->done = 0;
        nxt->rr = rr;
        nxt->thresh2 = thresh2;
        nxt->bnorm2 = bnorm2;
        nxt->beta = beta;
    }
    o.k = K;
    o.alpha = alpha;
    o.beta = beta;
    return true;
}

// ---------------------------------------------------------------------------
// FP32, four cells per thread along z (requires nz % 4 == 0).
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(kThreads) void stencil_v4(Geom g, Coef c, StencilIO<float> io, March m) {
    __shared__ float red[7 * kThreads / kWave];  // phase_a_start sums 7 arrays at once
    // the chunk's own source values and y faces of the current plane (double
    // buffered): y neighbours inside the chunk are read from here, only the
    // rows just outside it from memory
    __shared__ float4 ls[2][kThreads];
    __shared__ float4 lty[2][kThreads];

    constexpr bool kCg = MODE == kFusedCg || MODE == kMergedCg;
    PhaseA<float> ph{0, 0.f, 0.f, 0.f, false};
    if (MODE == kFusedCg && !phase_a_start(io, red, ph)) return;
    if ((MODE == kSweep1 || MODE == kSweep2) && io.done && block_flag(io.done)) return;
    if (MODE == kMergedCg) {
        // r_K = r_{K-1} - alpha q_{K-1} on the fly, then the same direction
        // update and deferred solution update as phase A
        MergedPh mp{0, 0.f, 0.f};
        if (!merged_start(io, red, mp)) return;
        ph.k = mp.k;
        ph.beta = mp.beta;
        ph.alpha_prev = mp.alpha;
    }
    const int it = ph.k;
    const float beta = ph.beta, alpha_prev = ph.alpha_prev, alpha_prev2 = ph.alpha_prev2;
    // Deferred solution update. The single-reduction kernel applies
    // alpha_{k-1} p_{k-1} every iteration. The two-phase CG applies two steps on
    // even k >= 2, x += alpha_{k-2} p_{k-2} + alpha_{k-1} p_{k-1}, and none on odd
    // k: x is read and written every other iteration (p_{k-2} is read at the own
    // cell from the buffer p_k is about to replace). The finalize kernel adds
    // what is owed when the loop stops.
    const bool pending = MODE == kMergedCg ? it > 0 : (it >= 2 && (it & 1) == 0);
    const float* pold = MODE == kMergedCg ? io.pin : ((it & 1) ? io.p0 : io.p1);
    float* pnew = MODE == kMergedCg ? io.pout : ((it & 1) ? io.p1 : io.p0);
    const bool use_pold = kCg && it > 0;
    // flexible CG fallback: the source is r / diag(A) instead of the network's z
    const bool jz = (MODE == kFusedCg) && ph.fallback;
    const float* zsrc = jz ? io.rres : io.src;
    const bool rupd = MODE == kMergedCg && it > 0;  // r_K = r_{K-1} - alpha q_{K-1}

    const int b = m.remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int pc = b % m.nchunk, ic = b / m.nchunk;
    const int i0 = ic * m.ci;
    const int i1 = min(g.nx, i0 + m.ci);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t P = g.plane;
    int64_t r0;
    bool valid;
    int j = 0, k = 0;
    int ystep;  // threads between a cell and its y neighbour inside the chunk
    // z neighbours not held by the adjacent lane (ends of a wave or of a row
    // segment) are read from memory
    bool zl_mem = lane == 0, zr_mem = lane == kWave - 1;
    if (m.nseg) {
        const int tps = 1 << m.tps_log2;
        const int col = (int)threadIdx.x & (tps - 1);
        j = (pc / m.nseg) * (kThreads >> m.tps_log2) + ((int)threadIdx.x >> m.tps_log2);
        k = (pc % m.nseg) * m.seg + col * 4;
        valid = j < g.ny;
        r0 = (int64_t)j * g.nz + k;
        ystep = tps;
        zl_mem = zl_mem || col == 0;
        zr_mem = zr_mem || col == tps - 1;
    } else {
        r0 = ((int64_t)pc * kThreads + threadIdx.x) * 4;
        valid = r0 < P;
        if (valid) {
            j = (int)(r0 / g.nz);
            k = (int)(r0 - (int64_t)j * g.nz);
        }
        ystep = g.nz / 4;
    }
    const bool hasjm = valid && j > 0;
    const bool hasjp = valid && j + 1 < g.ny;
    const bool haskm = valid && k > 0;
    const bool haskp = valid && k + 4 < g.nz;
    const int nz = g.nz;
    // LDS slots of the y neighbours when they lie inside the chunk
    const int jm_slot = (int)threadIdx.x - ystep, jp_slot = (int)threadIdx.x + ystep;
    const bool jm_in = jm_slot >= 0, jp_in = jp_slot < kThreads;

    // source value of the stencil: x, or r + beta p_old in the fused CG phase
    const float sws = MODE == kSweep2 ? *io.sw_scale : 0.f;
    auto Z4 = [&](int64_t idx) -> float4 {
        float4 v = ld4(zsrc + idx);
        if (jz) {
            const float4 d = ld4(io.dinv + idx);
            v = make_float4(v.x * d.x, v.y * d.y, v.z * d.z, v.w * d.w);
        }
        if (MODE == kSweep1) {  // the first sweep's step omega dinv r
            const float4 d = ld4(io.dinv + idx);
            const float w = io.omega;
            v = make_float4(w * d.x * v.x, w * d.y * v.y, w * d.z * v.z, w * d.w * v.w);
        }
        if (MODE == kSweep2) {  // z2 from the network's output v
            const float4 jv = ld4(io.sw_j + idx), q = ld4(io.sw_sq + idx);
            v = make_float4(jv.x + sws * q.x * v.x, jv.y + sws * q.y * v.y, jv.z + sws * q.z * v.z,
                            jv.w + sws * q.w * v.w);
        }
        if (rupd) v = axpy4(-alpha_prev, ld4(io.qin + idx), v);
        return v;
    };
    auto S4 = [&](int64_t idx) -> float4 {
        float4 v = Z4(idx);
        if (use_pold) v = axpy4(beta, ld4(pold + idx), v);
        return v;
    };
    auto S1 = [&](int64_t idx) -> float {
        float v = zsrc[idx];
        if (jz) v *= io.dinv[idx];
        if (MODE == kSweep1) v = io.omega * io.dinv[idx] * v;
        if (MODE == kSweep2) v = io.sw_j[idx] + sws * io.sw_sq[idx] * v;
        if (rupd) v -= alpha_prev * io.qin[idx];
        if (use_pold) v += beta * pold[idx];
        return v;
    };

    float4 sm = f4(0.f), sc = f4(0.f), sp = f4(0.f), txm = f4(0.f);
    float4 poc = f4(0.f), pop = f4(0.f);  // p_old at own cells, planes i and i+1
    float4 zc = f4(0.f), zp = f4(0.f);    // single-reduction CG: r_K at own cells
    float dot = 0.f, d_rr = 0.f, d_rq = 0.f, d_qq = 0.f;
    int64_t base = (int64_t)i0 * P + r0;
    if (valid && i0 < i1) {
        zc = Z4(base);
        if (use_pold) {
            poc = ld4(pold + base);
            sc = axpy4(beta, poc, zc);
        } else {
            sc = zc;
        }
        if (i0 > 0) {
            sm = S4(base - P);
            txm = ld4(c.tx + base - P);
        } else {
            sm = sc;
        }
    }
    int buf = 0;
    for (int i = i0; i < i1; ++i, base += P, buf ^= 1) {
        float4 txc = f4(0.f), tyc = f4(0.f), tzc = f4(0.f), ac = f4(0.f), tyl = f4(0.f);
        float4 sjm = sc, sjp = sc;
        if (valid) {
            if (i + 1 < g.nx) {
                zp = Z4(base + P);
                if (use_pold) {
                    pop = ld4(pold + base + P);
                    sp = axpy4(beta, pop, zp);
                } else {
                    sp = zp;
                }
            } else {
                sp = sc;
            }
            txc = ld4(c.tx + base);
            tyc = ld4(c.ty + base);
            tzc = ld4(c.tz + base);
            ac = coef_plane_uniform(c, i, g.nx) ? f4(c.a_const) : ld4(c.a + base);
        }
        ls[buf][threadIdx.x] = sc;
        lty[buf][threadIdx.x] = tyc;
        __syncthreads();
        if (valid) {
            if (hasjm) {
                if (jm_in) {
                    sjm = ls[buf][jm_slot];
                    tyl = lty[buf][jm_slot];
                } else {
                    tyl = ld4(c.ty + base - nz);
                    sjm = S4(base - nz);
                }
            }
            if (hasjp) sjp = jp_in ? ls[buf][jp_slot] : S4(base + nz);
        }
        // z neighbours across the float4 boundary from the adjacent lanes
        float xl = __shfl_up(sc.w, 1, kWave);
        float tzl = __shfl_up(tzc.w, 1, kWave);
        float xr = __shfl_down(sc.x, 1, kWave);
        if (valid) {
            if (zl_mem && haskm) {
                xl = S1(base - 1);
                tzl = c.tz[base - 1];
            }
            if (zr_mem && haskp) xr = S1(base + 4);
            if (!haskm) {
                xl = sc.x;
                tzl = 0.f;
            }
            if (!haskp) xr = sc.w;

            float4 y;
            y.x = cell_op<float, float>(ac.x, sc.x, txc.x, sp.x, txm.x, sm.x, tyc.x, sjp.x, tyl.x,
                                        sjm.x, tzc.x, sc.y, tzl, xl);
            y.y = cell_op<float, float>(ac.y, sc.y, txc.y, sp.y, txm.y, sm.y, tyc.y, sjp.y, tyl.y,
                                        sjm.y, tzc.y, sc.z, tzc.x, sc.x);
            y.z = cell_op<float, float>(ac.z, sc.z, txc.z, sp.z, txm.z, sm.z, tyc.z, sjp.z, tyl.z,
                                        sjm.z, tzc.z, sc.w, tzc.y, sc.y);
            y.w = cell_op<float, float>(ac.w, sc.w, txc.w, sp.w, txm.w, sm.w, tyc.w, sjp.w, tyl.w,
                                        sjm.w, tzc.w, xr, tzc.z, sc.z);
            if (MODE == kApply) {
                st4(io.out + base, y);
            } else if (kCg) {
                if (pending) {
                    float4 xv = axpy4(alpha_prev, poc, ld4(io.xsol + base));
                    if (MODE == kFusedCg) xv = axpy4(alpha_prev2, ld4(pnew + base), xv);
                    st4(io.xsol + base, xv);
                }
                st4(pnew + base, sc);
                st4(io.out + base, y);
                dot += sc.x * y.x + sc.y * y.y + sc.z * y.z + sc.w * y.w;
                if (MODE == kMergedCg) {
                    st4(io.rout + base, zc);
                    d_rr += zc.x * zc.x + zc.y * zc.y + zc.z * zc.z + zc.w * zc.w;
                    d_rq += zc.x * y.x + zc.y * y.y + zc.z * y.z + zc.w * y.w;
                    d_qq += y.x * y.x + y.y * y.y + y.z * y.z + y.w * y.w;
                }
            } else if (MODE == kSweep1) {
                // r1 = r - A (omega dinv r) and the partial sums of dinv r1^2
                const float4 rv = ld4(io.src + base), d = ld4(io.dinv + base);
                const float4 r1 = make_float4(rv.x - y.x, rv.y - y.y, rv.z - y.z, rv.w - y.w);
                if (io.out) st4(io.out + base, r1);
                if (io.nn_x0) {
                    const float4 f = ld4(io.nn_feat + base);
                    *reinterpret_cast<uint4*>(io.nn_x0 + base) =
                        make_uint4(nn_pair(d.x, r1.x, f.x), nn_pair(d.y, r1.y, f.y), nn_pair(d.z, r1.z, f.z),
                                   nn_pair(d.w, r1.w, f.w));
                }
                dot += d.x * r1.x * r1.x + d.y * r1.y * r1.y + d.z * r1.z * r1.z + d.w * r1.w * r1.w;
                if (io.sw_j) {
                    const float w = io.omega;
                    st4(io.sw_j + base, make_float4(w * d.x * rv.x + d.x * r1.x, w * d.y * rv.y + d.y * r1.y,
                                                    w * d.z * rv.z + d.z * r1.z, w * d.w * rv.w + d.w * r1.w));
                }
            } else if (MODE == kSweep2) {
                // z = z2 + omega dinv (r - A z2); sc is z2 at the own cells
                const float4 rv = ld4(io.rres + base), d = ld4(io.dinv + base);
                const float w = io.omega;
                const float4 zo = make_float4(sc.x + w * d.x * (rv.x - y.x), sc.y + w * d.y * (rv.y - y.y),
                                              sc.z + w * d.z * (rv.z - y.z), sc.w + w * d.w * (rv.w - y.w));
                st4(io.out + base, zo);
                if (io.sw_flex) {  // dot, d_rr, d_rq, d_qq hold z.r, z.q, dinv r.r, dinv r.q here
                    dot += zo.x * rv.x + zo.y * rv.y + zo.z * rv.z + zo.w * rv.w;
                    d_rq += d.x * rv.x * rv.x + d.y * rv.y * rv.y + d.z * rv.z * rv.z + d.w * rv.w * rv.w;
                    if (io.sw_q) {
                        const float4 qv = ld4(io.sw_q + base);
                        d_rr += zo.x * qv.x + zo.y * qv.y + zo.z * qv.z + zo.w * qv.w;
                        d_qq += d.x * rv.x * qv.x + d.y * rv.y * qv.y + d.z * rv.z * qv.z + d.w * rv.w * qv.w;
                    }
                }
            } else {  // residual r = b - A x
                float4 bb;
                if (io.rhs_f64) {
                    const double* bd = static_cast<const double*>(io.rhs) + base;
                    bb = make_float4((float)bd[0], (float)bd[1], (float)bd[2], (float)bd[3]);
                } else {
                    bb = ld4(static_cast<const float*>(io.rhs) + base);
                }
                st4(io.out + base, make_float4(bb.x - y.x, bb.y - y.y, bb.z - y.z, bb.w - y.w));
            }
        }
        sm = sc;
        sc = sp;
        txm = txc;
        poc = pop;
        zc = zp;
    }

    if (MODE == kFusedCg || MODE == kSweep1) {
        const float tot = block_sum(dot, red);
        if (threadIdx.x == 0) io.partials[blockIdx.x] = tot;
    } else if (MODE == kSweep2) {
        if (io.sw_flex) {  // z.r, z.q, dinv r.r, dinv r.q (the order flex_dots writes)
            const int nb = gridDim.x;
            const float a0 = block_sum(dot, red), a1 = block_sum(d_rr, red), a2 = block_sum(d_rq, red),
                        a3 = block_sum(d_qq, red);
            if (threadIdx.x == 0) {
                io.sw_flex[blockIdx.x] = a0;
                io.sw_flex[nb + blockIdx.x] = a1;
                io.sw_flex[2 * nb + blockIdx.x] = a2;
                io.sw_flex[3 * nb + blockIdx.x] = a3;
            }
        }
    } else if (MODE == kMergedCg) {
        const int nb = gridDim.x;
        const float a0 = block_sum(dot, red), a1 = block_sum(d_rr, red), a2 = block_sum(d_rq, red),
                    a3 = block_sum(d_qq, red);
        if (threadIdx.x == 0) {
            io.partials[blockIdx.x] = a0;
            io.partials[nb + blockIdx.x] = a1;
            io.partials[2 * nb + blockIdx.x] = a2;
            io.partials[3 * nb + blockIdx.x] = a3;
        }
    }
}

// ---------------------------------------------------------------------------
// One cell per thread (any nz; FP32 or FP64 vectors, FP32 coefficients).
// ---------------------------------------------------------------------------
template <class real, int MODE>
__global__ __launch_bounds__(kThreads) void stencil_s(Geom g, Coef c, StencilIO<real> io, March m) {
    __shared__ real red[7 * kThreads / kWave];  // phase_a_start sums 7 arrays at once

    PhaseA<real> ph{0, real(0), real(0), real(0), false};
    if (MODE == kFusedCg && !phase_a_start(io, red, ph)) return;
    if ((MODE == kSweep1 || MODE == kSweep2) && io.done && block_flag(io.done)) return;
    const int it = ph.k;
    const real beta = ph.beta, alpha_prev = ph.alpha_prev, alpha_prev2 = ph.alpha_prev2;
    // two deferred steps on even k >= 2, as in the four-cells-per-thread kernel
    const bool pending = it >= 2 && (it & 1) == 0;
    const real* pold = (it & 1) ? io.p0 : io.p1;
    real* pnew = (it & 1) ? io.p1 : io.p0;
    const bool use_pold = (MODE == kFusedCg) && it > 0;
    const bool jz = (MODE == kFusedCg) && ph.fallback;
    const real* zsrc = jz ? io.rres : io.src;

    const int b = m.remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int pc = b % m.nchunk, ic = b / m.nchunk;
    const int i0 = ic * m.ci;
    const int i1 = min(g.nx, i0 + m.ci);
    const int64_t P = g.plane;
    const int64_t r0 = (int64_t)pc * kThreads + threadIdx.x;
    const bool valid = r0 < P;
    int j = 0, k = 0;
    if (valid) {
        j = (int)(r0 / g.nz);
        k = (int)(r0 - (int64_t)j * g.nz);
    }
    const bool hasjm = j > 0, hasjp = j + 1 < g.ny, haskm = k > 0, haskp = k + 1 < g.nz;
    const int nz = g.nz;

    const float sws = MODE == kSweep2 ? *io.sw_scale : 0.f;
    auto Z = [&](int64_t idx) -> real {
        real v = zsrc[idx];
        if (jz) v *= (real)io.dinv[idx];
        if (MODE == kSweep1) v = (real)(io.omega * io.dinv[idx]) * v;
        if (MODE == kSweep2) v = (real)(io.sw_j[idx] + sws * io.sw_sq[idx] * (float)v);
        return v;
    };
    auto S = [&](int64_t idx) -> real {
        real v = Z(idx);
        if (use_pold) v += beta * pold[idx];
        return v;
    };

    real dot = 0, f_zq = 0, f_jr = 0, f_jq = 0;  // kSweep2: the flexible-CG dots
    if (valid && i0 < i1) {
        int64_t base = (int64_t)i0 * P + r0;
        real poc = use_pold ? pold[base] : real(0);
        real sc = use_pold ? Z(base) + beta * poc : Z(base);
        real sm = sc;
        float txm = 0.f;
        if (i0 > 0) {
            sm = S(base - P);
            txm = c.tx[base - P];
        }
        for (int i = i0; i < i1; ++i, base += P) {
            real pop = 0, sp = sc;
            if (i + 1 < g.nx) {
                if (use_pold) {
                    pop = pold[base + P];
                    sp = Z(base + P) + beta * pop;
                } else {
                    sp = Z(base + P);
                }
            }
            const float txc = c.tx[base], tyc = c.ty[base], tzc = c.tz[base];
            const real ac = coef_plane_uniform(c, i, g.nx) ? (real)c.a_const
                            : std::is_same<real, double>::value ? (real)c.a64[base] : (real)c.a[base];
            float tyl = 0.f, tzl = 0.f;
            real sjm = sc, sjp = sc, skm = sc, skp = sc;
            if (hasjm) {
                tyl = c.ty[base - nz];
                sjm = S(base - nz);
            }
            if (hasjp) sjp = S(base + nz);
            if (haskm) {
                tzl = c.tz[base - 1];
                skm = S(base - 1);
            }
            if (haskp) skp = S(base + 1);
            const real y = ac * sc + cell_op<real, float>(0.f, sc, txc, sp, txm, sm, tyc, sjp, tyl,
                                                          sjm, tzc, skp, tzl, skm);
            if (MODE == kApply) {
                io.out[base] = y;
            } else if (MODE == kFusedCg) {
                if (pending) io.xsol[base] += alpha_prev2 * pnew[base] + alpha_prev * poc;
                pnew[base] = sc;
                io.out[base] = y;
                dot += sc * y;
            } else if (MODE == kSweep1) {
                const real r1 = io.src[base] - y;
                if (io.out) io.out[base] = r1;
                const real d = (real)io.dinv[base];
                if (io.nn_x0) io.nn_x0[base] = nn_pair((float)d, (float)r1, io.nn_feat[base]);
                dot += d * r1 * r1;
                if (io.sw_j) io.sw_j[base] = (real)io.omega * d * io.src[base] + d * r1;
            } else if (MODE == kSweep2) {
                const real rv = io.rres[base], d = (real)io.dinv[base];
                const real zo = sc + (real)io.omega * d * (rv - y);
                io.out[base] = zo;
                if (io.sw_flex) {
                    dot += zo * rv;
                    f_jr += d * rv * rv;
                    if (io.sw_q) {
                        const real qv = io.sw_q[base];
                        f_zq += zo * qv;
                        f_jq += d * rv * qv;
                    }
                }
            } else {
                const real bb = io.rhs_f64 ? (real) static_cast<const double*>(io.rhs)[base]
                                           : (real) static_cast<const float*>(io.rhs)[base];
                const real r = bb - y;
                io.out[base] = r;
                dot += r * r;
            }
            sm = sc;
            sc = sp;
            txm = txc;
            poc = pop;
        }
    }

    if (MODE == kFusedCg || MODE == kSweep1 || (MODE == kResidual && io.partials != nullptr)) {
        const real tot = block_sum(dot, red);
        if (threadIdx.x == 0) io.partials[blockIdx.x] = tot;
    }
    if (MODE == kSweep2 && io.sw_flex) {
        const int nb = gridDim.x;
        const real a0 = block_sum(dot, red), a1 = block_sum(f_zq, red), a2 = block_sum(f_jr, red),
                   a3 = block_sum(f_jq, red);
        if (threadIdx.x == 0) {
            io.sw_flex[blockIdx.x] = (float)a0;
            io.sw_flex[nb + blockIdx.x] = (float)a1;
            io.sw_flex[2 * nb + blockIdx.x] = (float)a2;
            io.sw_flex[3 * nb + blockIdx.x] = (float)a3;
        }
    }
}

// ---------------------------------------------------------------------------
// Face-list (unstructured) operator: one thread per cell (grid-stride, so a
// wave always holds one slice of the sliced layout), the cell's faces its
// (neighbour, T) entries, so that y = a x + sum_f T_f (x - x_nbr) as on the
// Cartesian grid. Faces that touch a Dirichlet cell, and padding, carry T = 0
// and are skipped.
// ---------------------------------------------------------------------------
// sum_f T_f (x_K - x_nbr) over cell K's entries. The entries go in groups of
// kGroup: their indices and T, then their gathers, are in flight together,
// and the sum keeps the entry order.
template <class real>
__device__ __forceinline__ real csr_flux(const Coef& c, int64_t K, real xk, const real* __restrict__ x) {
    constexpr int kGroup = 8;
    real flux = 0;
    const int64_t sl = K / kWave;
    const int e1 = c.sp[sl + 1];
    for (int e = c.sp[sl] + (int)(K - sl * kWave); e < e1; e += kGroup * kWave) {
        float t[kGroup];
        int nbr[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            const int eu = e + u * kWave;
            t[u] = eu < e1 ? c.val[eu] : 0.f;
            nbr[u] = eu < e1 ? c.col[eu] : 0;
        }
        real xv[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) xv[u] = t[u] != 0.f ? x[nbr[u]] : xk;
#pragma unroll
        for (int u = 0; u < kGroup; ++u)
            if (t[u] != 0.f) flux += (real)t[u] * (xk - xv[u]);
    }
    return flux;
}

template <class real>
__device__ __forceinline__ real csr_diag(const Coef& c, int64_t K) {
    return std::is_same<real, double>::value ? (real)c.a64[K] : (real)c.a[K];
}

// apply (y = A x) and residual (r = b - A x, with r.r partials if asked)
template <class real, int MODE>
__global__ __launch_bounds__(kThreads) void stencil_csr(int64_t n, Coef c, StencilIO<real> io) {
    __shared__ real red[kThreads / kWave];
    real dot = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t K = (int64_t)blockIdx.x * kThreads + threadIdx.x; K < n; K += stride) {
        const real xk = io.src[K];
        const real y = csr_diag<real>(c, K) * xk + csr_flux(c, K, xk, io.src);
        if (MODE == kApply) {
            io.out[K] = y;
        } else {
            const real bb = io.rhs_f64 ? (real) static_cast<const double*>(io.rhs)[K]
                                       : (real) static_cast<const float*>(io.rhs)[K];
            const real r = bb - y;
            io.out[K] = r;
            dot += r * r;
        }
    }
    if (MODE == kResidual && io.partials != nullptr) {
        const real tot = block_sum(dot, red);
        if (threadIdx.x == 0) io.partials[blockIdx.x] = tot;
    }
}

// The face-list CG step in two kernels. Forming p = r + beta p_old at every
// neighbour on the fly, as the Cartesian kernels do, costs two gathers per
// face here; instead the first kernel forms p elementwise (with the deferred
// solution update) and the second applies A to the stored p, gathering one
// vector. The second finds the iteration in the state the first recorded.
template <class real>
__global__ __launch_bounds__(kThreads) void csr_direction(int64_t n, StencilIO<real> io) {
    __shared__ real red[7 * kThreads / kWave];  // phase_a_start sums 7 arrays at once
    PhaseA<real> ph{0, real(0), real(0), real(0), false};
    if (!phase_a_start(io, red, ph)) return;
    const int it = ph.k;
    const real beta = ph.beta, alpha_prev = ph.alpha_prev, alpha_prev2 = ph.alpha_prev2;
    const bool pending = it >= 2 && (it & 1) == 0;
    const real* pold = (it & 1) ? io.p0 : io.p1;
    real* pnew = (it & 1) ? io.p1 : io.p0;
    const bool use_pold = it > 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t K = (int64_t)blockIdx.x * kThreads + threadIdx.x; K < n; K += stride) {
        const real poc = use_pold ? pold[K] : real(0);
        const real sc = use_pold ? io.src[K] + beta * poc : io.src[K];
        if (pending) io.xsol[K] += alpha_prev2 * pnew[K] + alpha_prev * poc;
        pnew[K] = sc;
    }
}

template <class real>
__global__ __launch_bounds__(kThreads) void csr_apply_dot(int64_t n, Coef c, StencilIO<real> io) {
    __shared__ real red[kThreads / kWave];
    if (block_flag(&io.st->done)) return;
    const int it = io.st->iterB;  // recorded by csr_direction for this iteration
    const real* p = (it & 1) ? io.p1 : io.p0;
    real dot = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t K = (int64_t)blockIdx.x * kThreads + threadIdx.x; K < n; K += stride) {
        const real pk = p[K];
        const real y = csr_diag<real>(c, K) * pk + csr_flux(c, K, pk, p);
        io.out[K] = y;
        dot += pk * y;
    }
    const real tot = block_sum(dot, red);
    if (threadIdx.x == 0) io.partials[blockIdx.x] = tot;
}

template <class real, int MODE>
hipError_t launch_csr(const Geom& g, const Coef& c, const StencilIO<real>& io, const March& m,
                      hipStream_t s) {
    if constexpr (MODE == kFusedCg) {
        hipLaunchKernelGGL((csr_direction<real>), dim3(m.blocks()), dim3(kThreads), 0, s, g.n, io);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((csr_apply_dot<real>), dim3(m.blocks()), dim3(kThreads), 0, s, g.n, c, io);
        return hipGetLastError();
    } else {
        hipLaunchKernelGGL((stencil_csr<real, MODE>), dim3(m.blocks()), dim3(kThreads), 0, s, g.n, c, io);
        return hipGetLastError();
    }
}

template <class real, int MODE>
hipError_t launch_s(const Geom& g, const Coef& c, const StencilIO<real>& io, const March& m,
                    hipStream_t s) {
    hipLaunchKernelGGL((stencil_s<real, MODE>), dim3(m.blocks()), dim3(kThreads), 0, s, g, c, io, m);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_v4(const Geom& g, const Coef& c, const StencilIO<float>& io, const March& m,
                     hipStream_t s) {
    hipLaunchKernelGGL((stencil_v4<MODE>), dim3(m.blocks()), dim3(kThreads), 0, s, g, c, io, m);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stencil_f32(int mode, const Geom& g, const Coef& c, const StencilIO<float>& io,
                              const March& m, hipStream_t s) {
    if (c.sp) {
        switch (mode) {
            case kApply: return launch_csr<float, kApply>(g, c, io, m, s);
            case kFusedCg: return launch_csr<float, kFusedCg>(g, c, io, m, s);
            case kResidual: return launch_csr<float, kResidual>(g, c, io, m, s);
            default: return hipErrorInvalidValue;  // the single-reduction form and the sweeps are Cartesian only
        }
    }
    if (m.vec == 4) {
        switch (mode) {
            case kApply: return launch_v4<kApply>(g, c, io, m, s);
            case kFusedCg: return launch_v4<kFusedCg>(g, c, io, m, s);
            case kMergedCg: return launch_v4<kMergedCg>(g, c, io, m, s);
            case kSweep1: return launch_v4<kSweep1>(g, c, io, m, s);
            case kSweep2: return launch_v4<kSweep2>(g, c, io, m, s);
            default: return launch_v4<kResidual>(g, c, io, m, s);
        }
    }
    if (mode == kMergedCg) return hipErrorInvalidValue;  // float4 path only
    switch (mode) {
        case kApply: return launch_s<float, kApply>(g, c, io, m, s);
        case kFusedCg: return launch_s<float, kFusedCg>(g, c, io, m, s);
        case kSweep1: return launch_s<float, kSweep1>(g, c, io, m, s);
        case kSweep2: return launch_s<float, kSweep2>(g, c, io, m, s);
        default: return launch_s<float, kResidual>(g, c, io, m, s);
    }
}

hipError_t launch_stencil_f64(int mode, const Geom& g, const Coef& c, const StencilIO<double>& io,
                              const March& m, hipStream_t s) {
    if (c.sp) {
        switch (mode) {
            case kApply: return launch_csr<double, kApply>(g, c, io, m, s);
            case kFusedCg: return launch_csr<double, kFusedCg>(g, c, io, m, s);
            default: return launch_csr<double, kResidual>(g, c, io, m, s);
        }
    }
    switch (mode) {
        case kApply: return launch_s<double, kApply>(g, c, io, m, s);
        case kFusedCg: return launch_s<double, kFusedCg>(g, c, io, m, s);
        default: return launch_s<double, kResidual>(g, c, io, m, s);
    }
}

}  // namespace mffv
