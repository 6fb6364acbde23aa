// Batched CG: many independent systems of any sizes solved by one persistent
// launch. Each system owns a contiguous range of the grid's blocks (sized by
// its share of the work) and runs the whole of Alg. 1 inside the kernel: the
// initial residual, then per iteration the fused phase A (direction update,
// matrix-free apply, deferred solution update, p.Ap partial) and phase B
// (residual update, r.r partial), separated by per-system barriers. After each
// barrier every block of the system sums the system's partials in the same
// order, so all of them take the same decisions without further
// communication; converged systems' blocks leave while the others go on.
//
// Every residual that starts a CG pass is computed in FP64 (b - A x with the
// FP32 coefficients upcast). With refinement, a system whose FP64 true
// residual misses the tolerance after a pass runs another FP32 pass on the
// correction equation A dx = r from that residual and adds dx to x, all in
// the same launch.
//
// Barriers spin on agent-scope atomics with a wall-clock watchdog: a block
// that waits longer than the limit records an error and leaves, so a launch
// whose blocks are not all resident ends with an error instead of hanging.
// A limit of 0 makes every wait that is not satisfied at once fail (the
// failure path can then be tested with kernels that all exit normally).
#include "launch.hpp"

namespace mffv {
namespace {

__device__ __forceinline__ bool sys_barrier(unsigned* bar, unsigned nblk, uint64_t limit_ticks,
                                            int* err) {
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        ok = 1;
        if (nblk > 1) {
            const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned prev =
                __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (prev == nblk - 1) {
                __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&bar[1], gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                const uint64_t t0 = wall_clock64();
                while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                    __builtin_amdgcn_s_sleep(1);
                    if (limit_ticks == 0 || wall_clock64() - t0 > limit_ticks) {
                        ok = 0;
                        atomicOr(err, 1);
                        break;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
        }
    }
    __syncthreads();
    return ok != 0;
}

// Exchange of one partial sum per block without a fence. Each block publishes
// its value with the tag of the exchange in one 64-bit relaxed atomic word;
// every block waits until all of the system's words carry that tag and sums
// the values in sum_partials' order (so the result has the same bits). Only
// the values inside these words pass between blocks, which is why no release
// or acquire is needed: use it where the blocks have no other data to share
// (phase B touches only the cells the same thread wrote in phase A). A block
// cannot overwrite its word with the next tag before every block has read
// this one: the fenced barrier at the end of the iteration lies in between.
// Returns false (after recording the error) if a wait exceeds the limit.
__device__ __forceinline__ bool exchange_sum(unsigned long long* xch, int t, int nblk, unsigned tag, float v,
                                             uint64_t limit_ticks, int* err, float* red, float* out) {
    __shared__ int ok;
    if (threadIdx.x == 0) {
        ok = 1;
        __hip_atomic_store(&xch[t], ((unsigned long long)tag << 32) | __float_as_uint(v), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    float s = 0.f;
    bool mine = true;
    for (int i = threadIdx.x; i < nblk; i += kThreads) {
        const uint64_t t0 = wall_clock64();
        unsigned long long w;
        for (;;) {
            w = __hip_atomic_load(&xch[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((unsigned)(w >> 32) == tag) break;
            __builtin_amdgcn_s_sleep(1);
            if (limit_ticks == 0 || wall_clock64() - t0 > limit_ticks) {
                mine = false;
                break;
            }
        }
        if (!mine) break;
        s += __uint_as_float((unsigned)w);
    }
    if (!mine) {
        ok = 0;
        atomicOr(err, 1);
    }
    *out = block_sum(s, red);  // its barriers also publish ok
    return ok != 0;
}

// Own cells of a work item without the stencil.
template <class F>
__device__ __forceinline__ void own_cells(const Geom& g, int pc, int ic, int ci, F f) {
    const int64_t r0 = (int64_t)pc * kThreads + threadIdx.x;
    if (r0 >= g.plane) return;
    const int i0 = ic * ci, i1 = min(g.nx, i0 + ci);
    for (int i = i0; i < i1; ++i) f((int64_t)i * g.plane + r0);
}

// Byte-offset access from a block-uniform base in global memory. The
// system's pointers come from a descriptor in device memory, so the compiler
// cannot infer their address space by itself; without it every access would
// be a flat one (slower to wait on, and able to alias the kernel's own stack,
// which keeps the dot accumulators out of registers). A batched system has
// fewer than 2^30 cells (checked when the batch is planned), so every byte
// offset fits in 32 bits: a scalar base plus one 32-bit vector offset.
typedef __attribute__((address_space(1))) char gchar;
typedef __attribute__((address_space(1))) float gfloat;
__device__ __forceinline__ float ldo(const float* p, uint32_t off) {
    return *(const gfloat*)((const gchar*)p + off);
}
__device__ __forceinline__ void sto(float* p, uint32_t off, float v) { *(gfloat*)((gchar*)p + off) = v; }

// Plane steps whose loads are issued together in phase A and phase B.
#ifndef MFFV_BATCH_UNROLL_A
#define MFFV_BATCH_UNROLL_A 3
#endif
#ifndef MFFV_BATCH_UNROLL_B
#define MFFV_BATCH_UNROLL_B 8
#endif
constexpr int kUnrollA = MFFV_BATCH_UNROLL_A;
constexpr int kUnrollB = MFFV_BATCH_UNROLL_B;

// Raw operands of one plane step of phase A: the direction sources (s_k and
// p_{k-1}) at the next plane and at the four in-plane neighbours, the own
// faces and diagonal, the faces shared with the previous y and z neighbours,
// and the solution value for the deferred update. Loaded before use, so that
// the loads of several plane steps are in flight together.
struct StepA {
    float zp, pp, zjm, pjm, zjp, pjp, zkm, pkm, zkp, pkp;
    float tx, ty, tz, ac, tyl, tzl, xo;
};

struct CellA {
    bool hasjm, hasjp, haskm, haskp;
    bool ldkm, ldkp;   // the z neighbour lies in another wave: loaded (wave's first / last lane)
    uint32_t nz4, P4;  // byte strides of y and x
};

// Wavefront shifts by one lane (DPP wave_shr / wave_shl): lane l gets lane
// l - 1 (l + 1). The z neighbours of a cell are the neighbouring lanes of its
// wave (a work item's cells run along z), except at the wave's ends, where
// the neighbour is loaded, and at a row's ends, where its face is 0.
__device__ __forceinline__ float wave_shr1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float wave_shl1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

__device__ __forceinline__ void load_a(StepA& o, const BatchSys& S, const CellA& cc, const float* src,
                                       const float* pold, const float* xv, bool up, uint32_t off, int i) {
    const Geom& g = S.g;
    o.zp = o.pp = o.zjm = o.pjm = o.zjp = o.pjp = o.zkm = o.pkm = o.zkp = o.pkp = 0.f;
    o.tyl = o.tzl = o.xo = 0.f;
    if (i + 1 < g.nx) {
        o.zp = ldo(src, off + cc.P4);
        if (up) o.pp = ldo(pold, off + cc.P4);
    }
    o.tx = ldo(S.c.tx, off);
    o.ty = ldo(S.c.ty, off);
    o.tz = ldo(S.c.tz, off);
    o.ac = coef_plane_uniform(S.c, i, g.nx) ? S.c.a_const : ldo(S.c.a, off);
    if (cc.hasjm) {
        o.tyl = ldo(S.c.ty, off - cc.nz4);
        o.zjm = ldo(src, off - cc.nz4);
        if (up) o.pjm = ldo(pold, off - cc.nz4);
    }
    if (cc.hasjp) {
        o.zjp = ldo(src, off + cc.nz4);
        if (up) o.pjp = ldo(pold, off + cc.nz4);
    }
    if (cc.ldkm) {
        o.tzl = ldo(S.c.tz, off - 4u);
        o.zkm = ldo(src, off - 4u);
        if (up) o.pkm = ldo(pold, off - 4u);
    }
    if (cc.ldkp) {
        o.zkp = ldo(src, off + 4u);
        if (up) o.pkp = ldo(pold, off + 4u);
    }
    if (up) o.xo = ldo(xv, off);
}

// Phase A of one work item (chunk pc of a plane, planes of group ic): the
// direction update p_k = s_k + beta p_{k-1} at every stencil point, q = A p_k,
// the deferred x += alpha_{k-1} p_{k-1}, and the partial sum of p.q. Two plane
// steps at a time: both steps' loads are issued before either is computed.
__device__ __forceinline__ float phase_a_item(const BatchSys& S, int pc, int ic, const float* src,
                                              const float* pold, float* pnew, float* xv, bool up, float beta,
                                              float alpha_prev) {
    const Geom& g = S.g;
    const uint32_t P = (uint32_t)g.plane;
    const uint32_t r0 = (uint32_t)pc * kThreads + threadIdx.x;
    float dot = 0.f;
    if (r0 >= P) return dot;
    const int i0 = ic * S.ci, i1 = min(g.nx, i0 + S.ci);
    const uint32_t j = r0 / (uint32_t)g.nz, k = r0 - j * (uint32_t)g.nz;
    CellA cc;
    cc.hasjm = j > 0;
    cc.hasjp = (int)j + 1 < g.ny;
    cc.haskm = k > 0;
    cc.haskp = (int)k + 1 < g.nz;
    const int lane = threadIdx.x & 63;
    // the last lane of the wave that has a cell (the plane may end inside it)
    const int last = (int)min(63u, P - 1u - (r0 - (uint32_t)lane));
    cc.ldkm = cc.haskm && lane == 0;
    cc.ldkp = cc.haskp && lane == last;
    cc.nz4 = 4u * (uint32_t)g.nz;
    cc.P4 = 4u * P;
    uint32_t off = 4u * ((uint32_t)i0 * P + r0);
    float poc = up ? ldo(pold, off) : 0.f;
    float sc = up ? ldo(src, off) + beta * poc : ldo(src, off);
    float sm = sc, txm = 0.f;
    if (i0 > 0) {
        sm = up ? ldo(src, off - cc.P4) + beta * ldo(pold, off - cc.P4) : ldo(src, off - cc.P4);
        txm = ldo(S.c.tx, off - cc.P4);
    }
    auto step = [&](const StepA& a, uint32_t o, int i) {
        const float sp = i + 1 < g.nx ? a.zp + beta * a.pp : sc;
        const float sjm = cc.hasjm ? a.zjm + beta * a.pjm : sc;
        const float sjp = cc.hasjp ? a.zjp + beta * a.pjp : sc;
        // z neighbours: the neighbouring lanes' own values (same bits as loading them)
        const float sl = wave_shr1(sc), sr = wave_shl1(sc), tl = wave_shr1(a.tz);
        const float skm = !cc.haskm ? sc : cc.ldkm ? a.zkm + beta * a.pkm : sl;
        const float skp = !cc.haskp ? sc : cc.ldkp ? a.zkp + beta * a.pkp : sr;
        const float tzl = !cc.haskm ? 0.f : cc.ldkm ? a.tzl : tl;
        const float y =
            cell_op<float, float>(a.ac, sc, a.tx, sp, txm, sm, a.ty, sjp, a.tyl, sjm, a.tz, skp, tzl, skm);
        sto(pnew, o, sc);
        sto(S.q, o, y);
        if (up) sto(xv, o, a.xo + alpha_prev * poc);
        dot += sc * y;
        sm = sc;
        sc = sp;
        txm = a.tx;
        poc = a.pp;
    };
    int i = i0;
    for (; i + kUnrollA - 1 < i1; i += kUnrollA, off += kUnrollA * cc.P4) {
        StepA a[kUnrollA];
#pragma unroll
        for (int u = 0; u < kUnrollA; ++u) load_a(a[u], S, cc, src, pold, xv, up, off + u * cc.P4, i + u);
#pragma unroll
        for (int u = 0; u < kUnrollA; ++u) step(a[u], off + u * cc.P4, i + u);
    }
    for (; i < i1; ++i, off += cc.P4) {
        StepA a0;
        load_a(a0, S, cc, src, pold, xv, up, off, i);
        step(a0, off, i);
    }
    return dot;
}

// Phase B of one work item: r -= alpha q (and z = r / diag(A) with Jacobi),
// with the partial sums of r.r and r.z; kUnrollB planes' loads at a time.
__device__ __forceinline__ float2 phase_b_item(const BatchSys& S, int pc, int ic, bool jac, float alpha) {
    const Geom& g = S.g;
    const uint32_t P = (uint32_t)g.plane;
    const uint32_t r0 = (uint32_t)pc * kThreads + threadIdx.x;
    float r2 = 0.f, z2 = 0.f;
    if (r0 >= P) return make_float2(r2, z2);
    const int i0 = ic * S.ci, i1 = min(g.nx, i0 + S.ci);
    const uint32_t P4 = 4u * P;
    uint32_t off = 4u * ((uint32_t)i0 * P + r0);
    int i = i0;
    for (; i + kUnrollB - 1 < i1; i += kUnrollB, off += kUnrollB * P4) {
        float rv[kUnrollB], qv[kUnrollB], dv[kUnrollB];
#pragma unroll
        for (int u = 0; u < kUnrollB; ++u) {
            rv[u] = ldo(S.r, off + u * P4);
            qv[u] = ldo(S.q, off + u * P4);
            dv[u] = jac ? ldo(S.dinv, off + u * P4) : 0.f;
        }
#pragma unroll
        for (int u = 0; u < kUnrollB; ++u) {
            const float r = rv[u] - alpha * qv[u];
            sto(S.r, off + u * P4, r);
            r2 += r * r;
            if (jac) {
                const float z = dv[u] * r;
                sto(S.z, off + u * P4, z);
                z2 += r * z;
            }
        }
    }
    for (; i < i1; ++i, off += P4) {
        const float r = ldo(S.r, off) - alpha * ldo(S.q, off);
        sto(S.r, off, r);
        r2 += r * r;
        if (jac) {
            const float z = ldo(S.dinv, off) * r;
            sto(S.z, off, z);
            z2 += r * z;
        }
    }
    return make_float2(r2, z2);
}

// Raw operands of one plane step of the single-reduction iteration: the
// previous residual, product and direction (r_{K-1}, q_{K-1}, p_{K-1}) at the
// next plane and at the four in-plane neighbours, the own faces and diagonal,
// the faces shared with the previous y and z neighbours, and x.
struct StepM {
    float zp, qp, pp, zjm, qjm, pjm, zjp, qjp, pjp, zkm, qkm, pkm, zkp, qkp, pkp;
    float tx, ty, tz, ac, tyl, tzl, xo;
};

__device__ __forceinline__ void load_m(StepM& o, const BatchSys& S, const CellA& cc, const float* rin,
                                       const float* qin, const float* pold, const float* xv, bool up, uint32_t off,
                                       int i) {
    const Geom& g = S.g;
    o.zp = o.qp = o.pp = o.zjm = o.qjm = o.pjm = o.zjp = o.qjp = o.pjp = 0.f;
    o.zkm = o.qkm = o.pkm = o.zkp = o.qkp = o.pkp = 0.f;
    o.tyl = o.tzl = o.xo = 0.f;
    auto three = [&](uint32_t at, float& z, float& q, float& pp) {
        z = ldo(rin, at);
        if (up) {
            q = ldo(qin, at);
            pp = ldo(pold, at);
        }
    };
    if (i + 1 < g.nx) three(off + cc.P4, o.zp, o.qp, o.pp);
    o.tx = ldo(S.c.tx, off);
    o.ty = ldo(S.c.ty, off);
    o.tz = ldo(S.c.tz, off);
    o.ac = coef_plane_uniform(S.c, i, g.nx) ? S.c.a_const : ldo(S.c.a, off);
    if (cc.hasjm) {
        o.tyl = ldo(S.c.ty, off - cc.nz4);
        three(off - cc.nz4, o.zjm, o.qjm, o.pjm);
    }
    if (cc.hasjp) three(off + cc.nz4, o.zjp, o.qjp, o.pjp);
    if (cc.haskm) {
        o.tzl = ldo(S.c.tz, off - 4u);
        three(off - 4u, o.zkm, o.qkm, o.pkm);
    }
    if (cc.haskp) three(off + 4u, o.zkp, o.qkp, o.pkp);
    if (up) o.xo = ldo(xv, off);
}

// One work item of single-reduction iteration K (Alg. 1 with one reduction
// phase per iteration): r_K = r_{K-1} - alpha q_{K-1} and the direction
// p_K = r_K + beta p_{K-1} on the fly at every stencil point, q_K = A p_K, the
// deferred x_K = x_{K-1} + alpha p_{K-1}, and the partial sums of p.q, r.r,
// r.q and q.q of iteration K; two plane steps' loads at a time. K = 0 (up
// false) takes r_0 as it is.
__device__ __forceinline__ float4 merged_item(const BatchSys& S, int pc, int ic, const float* rin,
                                              const float* qin, const float* pold, float* rout, float* qout,
                                              float* pnew, float* xv, bool up, float alpha, float beta) {
    const Geom& g = S.g;
    const uint32_t P = (uint32_t)g.plane;
    const uint32_t r0 = (uint32_t)pc * kThreads + threadIdx.x;
    float pq = 0.f, rr = 0.f, rq = 0.f, qq = 0.f;
    if (r0 >= P) return make_float4(pq, rr, rq, qq);
    const int i0 = ic * S.ci, i1 = min(g.nx, i0 + S.ci);
    const uint32_t j = r0 / (uint32_t)g.nz, k = r0 - j * (uint32_t)g.nz;
    CellA cc;
    cc.hasjm = j > 0;
    cc.hasjp = (int)j + 1 < g.ny;
    cc.haskm = k > 0;
    cc.haskp = (int)k + 1 < g.nz;
    cc.nz4 = 4u * (uint32_t)g.nz;
    cc.P4 = 4u * P;
    auto resid = [&](float z, float q) { return up ? z - alpha * q : z; };
    auto dir = [&](float z, float q, float pp) { return up ? resid(z, q) + beta * pp : z; };
    uint32_t off = 4u * ((uint32_t)i0 * P + r0);
    float poc = up ? ldo(pold, off) : 0.f;
    float zc = resid(ldo(rin, off), up ? ldo(qin, off) : 0.f);
    float sc = up ? zc + beta * poc : zc;
    float sm = sc, txm = 0.f;
    if (i0 > 0) {
        const uint32_t o = off - cc.P4;
        sm = dir(ldo(rin, o), up ? ldo(qin, o) : 0.f, up ? ldo(pold, o) : 0.f);
        txm = ldo(S.c.tx, o);
    }
    auto step = [&](const StepM& a, uint32_t o, int i) {
        const bool nxt = i + 1 < g.nx;
        const float zn = nxt ? resid(a.zp, a.qp) : zc;
        const float sp = nxt ? (up ? zn + beta * a.pp : zn) : sc;
        const float sjm = cc.hasjm ? dir(a.zjm, a.qjm, a.pjm) : sc;
        const float sjp = cc.hasjp ? dir(a.zjp, a.qjp, a.pjp) : sc;
        const float skm = cc.haskm ? dir(a.zkm, a.qkm, a.pkm) : sc;
        const float skp = cc.haskp ? dir(a.zkp, a.qkp, a.pkp) : sc;
        const float y =
            cell_op<float, float>(a.ac, sc, a.tx, sp, txm, sm, a.ty, sjp, a.tyl, sjm, a.tz, skp, a.tzl, skm);
        sto(rout, o, zc);
        sto(pnew, o, sc);
        sto(qout, o, y);
        if (up) sto(xv, o, a.xo + alpha * poc);
        pq += sc * y;
        rr += zc * zc;
        rq += zc * y;
        qq += y * y;
        sm = sc;
        sc = sp;
        zc = zn;
        txm = a.tx;
        poc = a.pp;
    };
    int i = i0;
    for (; i + 1 < i1; i += 2, off += 2u * cc.P4) {
        StepM a0, a1;
        load_m(a0, S, cc, rin, qin, pold, xv, up, off, i);
        load_m(a1, S, cc, rin, qin, pold, xv, up, off + cc.P4, i + 1);
        step(a0, off, i);
        step(a1, off + cc.P4, i + 1);
    }
    if (i < i1) {
        StepM a0;
        load_m(a0, S, cc, rin, qin, pold, xv, up, off, i);
        step(a0, off, i);
    }
    return make_float4(pq, rr, rq, qq);
}

// Residual pass of one work item: r64 = b - A x' in FP64 at the item's own
// cells (x' = b on Dirichlet cells, x elsewhere; FP32 coefficients upcast, the
// FP64 identity coefficient), r = fl32(r64) on unknown cells and 0 on
// Dirichlet cells, z = dinv r with Jacobi, and dx = 0 when asked. Partial sums:
// r.r and r.z of the rounded r and ||b_U||^2 in FP32, ||r64||^2 and ||b_U||^2
// in FP64.
struct ResidSums {
    float rr, rz, bb;
    double rr64, bb64;
};

__device__ __forceinline__ void residual_item64(const BatchSys& S, int pc, int ic, bool jac, bool zero_dx,
                                                ResidSums& acc) {
    const Geom& g = S.g;
    const Coef& c = S.c;
    const int64_t P = g.plane;
    const int64_t r0 = (int64_t)pc * kThreads + threadIdx.x;
    if (r0 >= P) return;
    const int i0 = ic * S.ci, i1 = min(g.nx, i0 + S.ci);
    const int j = (int)(r0 / g.nz), k = (int)(r0 - (int64_t)j * g.nz);
    const bool hasjm = j > 0, hasjp = j + 1 < g.ny, haskm = k > 0, haskp = k + 1 < g.nz;
    const int nz = g.nz;
    auto X = [&](int64_t l) -> double { return S.dmask[l] ? (double)S.b[l] : (double)S.x[l]; };
    int64_t base = (int64_t)i0 * P + r0;
    double sc = X(base), sm = sc;
    double txm = 0.0;
    if (i0 > 0) {
        sm = X(base - P);
        txm = c.tx[base - P];
    }
    for (int i = i0; i < i1; ++i, base += P) {
        const double sp = (i + 1 < g.nx) ? X(base + P) : sc;
        const double txc = c.tx[base], tyc = c.ty[base], tzc = c.tz[base];
        const double ac = coef_plane_uniform(c, i, g.nx) ? (double)c.a_const : c.a64[base];
        double tyl = 0.0, tzl = 0.0, sjm = sc, sjp = sc, skm = sc, skp = sc;
        if (hasjm) {
            tyl = c.ty[base - nz];
            sjm = X(base - nz);
        }
        if (hasjp) sjp = X(base + nz);
        if (haskm) {
            tzl = c.tz[base - 1];
            skm = X(base - 1);
        }
        if (haskp) skp = X(base + 1);
        const double y = cell_op<double, double>(ac, sc, txc, sp, txm, sm, tyc, sjp, tyl, sjm, tzc, skp, tzl, skm);
        const bool d = S.dmask[base] != 0;
        const double bv = S.b[base];
        const double r64 = d ? 0.0 : bv - y;
        const float r = (float)r64;
        S.r[base] = r;
        acc.rr += r * r;
        if (jac) {
            const float z = S.dinv[base] * r;
            S.z[base] = z;
            acc.rz += r * z;
        }
        if (zero_dx) S.dx[base] = 0.f;
        acc.rr64 += r64 * r64;
        if (!d) {
            acc.bb += (float)bv * (float)bv;
            acc.bb64 += bv * bv;
        }
        sm = sc;
        sc = sp;
        txm = txc;
    }
}

// Outcome of one FP32 CG pass of a system.
struct PassOut {
    int iters;      // iterations of the pass
    int status;     // 0 converged (recursive residual), 1 iteration cap, -4 breakdown
    int tail;       // the deferred step alpha_prev p_{iters-1} is still owed
    float alpha_prev;
    float rr;       // recursive r.r at exit
    bool aborted;   // a wait expired (the error flag is set)
};

// One CG pass: from r (and z) as the residual pass left them, iterate until
// r.r <= thresh2, kmax iterations, or a breakdown, accumulating the solution
// in xv. Exchange tags continue from tag0 so that no tag repeats in a launch.
__device__ PassOut cg_pass(const BatchSys& S, const BatchRun& run, int t, int B, int W, bool jac, float rr,
                           float rz, float thresh2, int kmax, unsigned tag0, float* xv, float* red) {
    PassOut out{0, 1, 0, 0.f, rr, false};
    float* rr_part = S.part + B;
    float* rz_part = S.part + 2 * B;
    float rho = jac ? rz : rr;
    float beta = 0.f, alpha_prev = 0.f;
    int k = 0;
    const float* src = jac ? S.z : S.r;

    if (run.merged) {
        // Single-reduction iteration K: the partial sums of iteration K-1 give
        // alpha_{K-1} = rho_{K-1} / p.q, rho_K = rho_{K-1} - 2 alpha r.q + alpha^2 q.q
        // (one step from the exact rho_{K-1}) and beta_{K-1} = rho_K / rho_{K-1}.
        // Convergence is tested on the exact rho_{K-1}; iteration K-1 completed
        // x_{K-1}, so the pass stops with no owed update. One barrier per iteration.
        //
        // With a single barrier per iteration the partial sums are double
        // buffered: iteration K writes set (K+1) & 1 and iteration K+1 reads it,
        // so no block overwrites sums another block may still be reading (set 0
        // holds the residual pass's sums, read before iteration 0's barrier).
        float alpha = 0.f, bm = 0.f;
        int K = 0;
        for (;;) {
            bool bad = false;
            if (K > 0) {
                const float* rd = S.part + 4 * B * (K & 1);
                const float pq = sum_partials(rd, B, red);
                rr = sum_partials(rd + B, B, red);
                const float rq = sum_partials(rd + 2 * B, B, red);
                const float qq = sum_partials(rd + 3 * B, B, red);
                bad = !(pq > 0.f) || !isfinite(pq);
                alpha = rr / pq;
                const float rnext = rr - 2.f * alpha * rq + alpha * alpha * qq;
                bm = rnext > 0.f ? rnext / rr : 0.f;  // a cancelled recurrence restarts the directions
            }
            const bool conv = isfinite(rr) && rr <= thresh2;
            bad = !conv && (bad || !isfinite(rr));
            const int done = K == 0 ? 0 : K - 1;
            if (conv || bad || done >= kmax) {
                out.status = conv ? 0 : (bad ? -4 : 1);
                out.iters = done;
                out.rr = rr;
                return out;
            }
            const bool up = K > 0;
            const float* rin = (K & 1) ? S.r2 : S.r;
            float* rout = (K & 1) ? S.r : S.r2;
            const float* qin = (K & 1) ? S.q : S.q2;
            float* qout = (K & 1) ? S.q2 : S.q;
            const float* pold = (K & 1) ? S.p0 : S.p1;
            float* pnew = (K & 1) ? S.p1 : S.p0;
            float4 d = make_float4(0.f, 0.f, 0.f, 0.f);
            for (int w = t; w < W; w += B) {
                const float4 v = merged_item(S, w % S.nchunk, w / S.nchunk, rin, qin, pold, rout, qout, pnew, xv,
                                             up, alpha, bm);
                d.x += v.x;
                d.y += v.y;
                d.z += v.z;
                d.w += v.w;
            }
            {
                const float a0 = block_sum(d.x, red), a1 = block_sum(d.y, red), a2 = block_sum(d.z, red),
                            a3 = block_sum(d.w, red);
                if (threadIdx.x == 0) {
                    float* wr = S.part + 4 * B * ((K + 1) & 1);
                    wr[t] = a0;
                    wr[B + t] = a1;
                    wr[2 * B + t] = a2;
                    wr[3 * B + t] = a3;
                }
            }
            if (!sys_barrier(S.bar, B, run.limit_ticks, run.err)) {
                out.aborted = true;
                return out;
            }
            ++K;
        }
    }

    for (;;) {
        const bool conv = isfinite(rr) && rr <= thresh2;
        const bool bad = !conv && (!isfinite(rr) || (jac && (!(rho > 0.f) || !isfinite(rho))));
        if (conv || bad || k >= kmax) {
            out.status = conv ? 0 : (bad ? -4 : 1);
            out.tail = k >= 1 ? 1 : 0;
            break;
        }
        // phase A
        const float* pold = (k & 1) ? S.p0 : S.p1;
        float* pnew = (k & 1) ? S.p1 : S.p0;
        const bool up = k > 0;
        float dot = 0.f;
        for (int w = t; w < W; w += B)
            dot += phase_a_item(S, w % S.nchunk, w / S.nchunk, src, pold, pnew, xv, up, beta, alpha_prev);
        // p.q: a fence-free exchange (phase B needs no other block's data)
        float pq = 0.f;
        if (B > 1) {
            const float a0 = block_sum(dot, red);
            if (!exchange_sum(S.xch, t, B, tag0 + (unsigned)k + 1u, a0, run.limit_ticks, run.err, red, &pq)) {
                out.aborted = true;
                return out;
            }
        } else {
            pq = block_sum(dot, red);
        }
        if (!(pq > 0.f) || !isfinite(pq)) {
            out.status = -4;
            out.tail = 0;
            break;
        }
        const float alpha = rho / pq;
        // phase B
        float r2 = 0.f, z2 = 0.f;
        for (int w = t; w < W; w += B) {
            const float2 v = phase_b_item(S, w % S.nchunk, w / S.nchunk, jac, alpha);
            r2 += v.x;
            z2 += v.y;
        }
        {
            const float a0 = block_sum(r2, red), a1 = block_sum(z2, red);
            if (threadIdx.x == 0) {
                rr_part[t] = a0;
                rz_part[t] = a1;
            }
        }
        if (!sys_barrier(S.bar, B, run.limit_ticks, run.err)) {
            out.aborted = true;
            return out;
        }
        rr = sum_partials(rr_part, B, red);
        const float rho_new = jac ? sum_partials(rz_part, B, red) : rr;
        beta = rho_new / rho;
        rho = rho_new;
        alpha_prev = alpha;
        ++k;
    }
    out.iters = k;
    out.alpha_prev = alpha_prev;
    out.rr = rr;
    return out;
}

__global__ __launch_bounds__(kThreads) void batched_cg(const BatchSys* __restrict__ systems,
                                                       const int* __restrict__ block_sys, BatchRun run) {
    __shared__ float red[kThreads / kWave];
    __shared__ double red64[kThreads / kWave];
    BatchSys S = systems[block_sys[blockIdx.x]];
    {
        // the operator's scalars as set last (they live with the grid, not the plan)
        const CoefScalars cs = *S.cs;
        S.c.a_uniform = cs.a_uniform;
        S.c.a_const = cs.a_const;
    }
    const int t = (int)blockIdx.x - S.blk0, B = S.nblk;
    const int W = S.nchunk * S.nich;
    const bool jac = run.precond == 1;
    float* rr_part = S.part + B;
    float* rz_part = S.part + 2 * B;
    float* bb_part = S.part + 3 * B;

    // Pass 0 solves A x = b from the caller's x in place. With refinement every
    // later pass o solves A dx = r_o for the FP64 true residual r_o of the
    // current x (rounded to FP32), to a reduction min(0.5, max(tol / rho_o,
    // inner_tol)) of |r_o|, and then adds dx to x (one rounding to FP32 per
    // pass), until the FP64 true relative residual rho meets tol.
    int ktot = 0, passes = 0, status = 1;
    float rr = 0.f, bnorm2 = 0.f, rr_exit = 0.f;
    double rr64 = 0.0, bb64 = 0.0;
    for (int outer = 0;; ++outer) {
        // residual pass: r = b - A x' in FP64 (the initial residual, or the true
        // residual of the updated x)
        ResidSums acc{0.f, 0.f, 0.f, 0.0, 0.0};
        for (int w = t; w < W; w += B) residual_item64(S, w % S.nchunk, w / S.nchunk, jac, outer > 0, acc);
        {
            const float a0 = block_sum(acc.rr, red), a1 = block_sum(acc.rz, red), a2 = block_sum(acc.bb, red);
            const double d0 = block_sum(acc.rr64, red64), d1 = block_sum(acc.bb64, red64);
            if (threadIdx.x == 0) {
                rr_part[t] = a0;
                rz_part[t] = a1;
                bb_part[t] = a2;
                S.part64[t] = d0;
                S.part64[B + t] = d1;
            }
        }
        if (!sys_barrier(S.bar, B, run.limit_ticks, run.err)) return;
        rr = sum_partials(rr_part, B, red);
        const float rz = sum_partials(rz_part, B, red);
        rr64 = sum_partials(S.part64, B, red64);
        if (outer == 0) {
            const float bb = sum_partials(bb_part, B, red);
            bnorm2 = bb > 0.f ? bb : rr;
            bb64 = sum_partials(S.part64 + B, B, red64);
        }
        const double rho = bb64 > 0.0 ? sqrt(rr64 / bb64) : sqrt(rr64);
        if (outer > 0) {
            if (run.max_outer == 0 || status < 0) break;   // FP32: the pass's own status stands
            if (rho <= run.tol) {
                status = 0;
                break;
            }
            if (outer > run.max_outer || ktot >= run.max_iter || !isfinite(rho)) {
                status = isfinite(rho) ? 1 : -4;
                break;
            }
        } else if (run.max_outer > 0 && rho <= run.tol) {
            status = 0;                                      // the initial guess meets tol
            break;
        }
        float thresh2 = run.tol2 * bnorm2;
        if (outer > 0) {
            const double inner = fmin(0.5, fmax(run.tol / rho, run.inner_tol));
            thresh2 = (float)(inner * inner * rr64);
        }
        float* xv = outer == 0 ? S.x : S.dx;
        const PassOut po = cg_pass(S, run, t, B, W, jac, rr, rz, thresh2, run.max_iter - ktot,
                                   (unsigned)ktot + (unsigned)outer, xv, red);
        if (po.aborted) return;
        // owed step, the correction, Dirichlet values
        const float* plast = ((po.iters - 1) & 1) ? S.p1 : S.p0;
        for (int w = t; w < W; w += B) {
            const int pc = w % S.nchunk, ic = w / S.nchunk;
            own_cells(S.g, pc, ic, S.ci, [&](int64_t l) {
                if (S.dmask[l]) {
                    S.x[l] = S.b[l];
                } else if (outer == 0) {
                    if (po.tail) S.x[l] += po.alpha_prev * plast[l];
                } else {
                    const float d = po.tail ? S.dx[l] + po.alpha_prev * plast[l] : S.dx[l];
                    S.x[l] = (float)((double)S.x[l] + (double)d);
                }
            });
        }
        ktot += po.iters;
        passes += 1;
        status = po.status;
        rr_exit = po.rr;
        // every block's x is complete before the residual pass reads neighbours
        if (!sys_barrier(S.bar, B, run.limit_ticks, run.err)) return;
    }
    if (t == 0 && threadIdx.x == 0) {
        BatchResult* res = S.res;
        res->iters = ktot;
        res->status = status;
        res->passes = passes;
        res->rr = rr_exit;
        res->bnorm2 = bnorm2;
        res->rr64 = rr64;
        res->bb64 = bb64;
    }
}

// Start of a launch: barrier words, exchange slots and the watchdog flag to 0.
__global__ void clear_barriers(unsigned* bars, int n, int* err) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) bars[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) *err = 0;
}

}  // namespace

int batched_blocks_per_cu() {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched_cg, kThreads, 0) != hipSuccess)
        return 0;
    return per_cu;
}

hipError_t launch_batched_cg(const BatchSys* systems, const int* block_sys, int nblocks,
                             unsigned* bars, int nbars, int* err, const BatchRun& run, hipStream_t s) {
    hipLaunchKernelGGL(clear_barriers, dim3(1), dim3(256), 0, s, bars, nbars, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batched_cg, dim3(nblocks), dim3(kThreads), 0, s, systems, block_sys, run);
    return hipGetLastError();
}

}  // namespace mffv
