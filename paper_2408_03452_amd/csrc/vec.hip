// Streaming kernels of the CG loop and its set-up: the residual update with
// its dot products and the scalar recurrences of Alg. 1 (phase B), flexible-CG
// dots, the final deferred solution update, operator set-up from the face
// transmissibilities (Eq. 3 and 4) and small elementwise helpers.
//
// All reductions are deterministic: per-block partials, then the last block to
// arrive sums them in a fixed order and updates the device-resident scalars.
#include "launch.hpp"

#include <type_traits>

#include <cstring>

namespace mffv {
namespace {

template <class real> struct VT;
template <> struct VT<float> { using V = float4; static constexpr int W = 4; };
template <> struct VT<double> { using V = double2; static constexpr int W = 2; };

template <class real>
__device__ __forceinline__ void ldv(const real* p, real (&v)[VT<real>::W]) {
    typename VT<real>::V t = *reinterpret_cast<const typename VT<real>::V*>(p);
    memcpy(v, &t, sizeof(t));
}
template <class real>
__device__ __forceinline__ void stv(real* p, const real (&v)[VT<real>::W]) {
    typename VT<real>::V t;
    memcpy(&t, v, sizeof(t));
    *reinterpret_cast<typename VT<real>::V*>(p) = t;
}

// ---------------------------------------------------------------------------
// Phase B_k: alpha_k from the phase-A partials (summed by every block), then
// r -= alpha_k q with the per-block partials r.r (and r.z) that phase A_{k+1}
// consumes. The init mode forms the partials of r_0 (and ||b_U||^2) and
// resets the loop state.
// ---------------------------------------------------------------------------
template <class real, int MODE>
__global__ __launch_bounds__(kThreads) void phase_b(int64_t n, VecIO<real> io) {
    __shared__ real red[kThreads / kWave];
    CgState<real>* st = io.st;
    real alpha = 0;
    if (MODE != kBInit) {
        // the done flag, k, rho and the first batch of phase A's partials in
        // one memory round trip (phase A_k wrote rho; no block of this kernel
        // writes it), then the sum in sum_partials' order
        const real* pa[1] = {io.pa};
        const int na[1] = {io.nb_a};
        real first[1][kPartBatch];
        load_partials_first(pa, na, first);
        const int done = early_load(&st->done), k = early_load(&st->iterB);
        const real rho0 = early_load(&st->rho[0]), rho1 = early_load(&st->rho[1]);
        if (block_uniform(done)) {
            drain_loads();
            return;
        }
        real pqs[1];
        sum_partials_n_rest(pa, na, first, red, pqs);
        const real pq = pqs[0];
        if (!(pq > real(0)) || !isfinite(pq)) {
            if (first_thread()) {
                st->done = 1;
                st->status = -4;
                st->iters = k;
                // x_k lacks alpha_{k-1} p_{k-1} when k is odd (phase A applies
                // steps on even k only)
                st->tail = (k & 1) ? 1 : 0;
            }
            return;
        }
        alpha = ((k & 1) ? rho1 : rho0) / pq;
        if (first_thread()) {
            st->alpha[k & 1] = alpha;
            st->pq[k & 1] = pq;
            st->iterA = k + 1;
        }
    }
    const bool jac = (MODE == kBJacobi) || (MODE == kBInit && io.jacobi);
    const bool dd = !jac && io.dinv_dot;
    constexpr int W = VT<real>::W;
    const int64_t nv = n / W;
    real rr = 0, rz = 0, bb = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;

    auto one = [&](int64_t idx, real& r, real q) {
        if (MODE != kBInit) r -= alpha * q;
        rr += r * r;
        if (jac) {
            const real z = (real)io.dinv[idx] * r;
            io.z[idx] = z;
            rz += r * z;
        } else if (dd) {
            rz += r * ((real)io.dinv[idx] * r);
        }
        if (MODE == kBInit && !io.dmask[idx]) {
            const real b = io.b_f64 ? (real) static_cast<const double*>(io.b)[idx]
                                    : (real) static_cast<const float*>(io.b)[idx];
            bb += b * b;
        }
    };

    for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < nv; v += stride) {
        const int64_t e = v * W;
        real r[W], q[W];
        ldv(io.r + e, r);
        if (MODE != kBInit) ldv(io.q + e, q);
#pragma unroll
        for (int t = 0; t < W; ++t) one(e + t, r[t], MODE != kBInit ? q[t] : real(0));
        if (MODE != kBInit) stv(io.r + e, r);
    }
    if (blockIdx.x == 0 && threadIdx.x < n - nv * W) {  // ragged tail
        const int64_t e = nv * W + threadIdx.x;
        real r = io.r[e];
        one(e, r, MODE != kBInit ? io.q[e] : real(0));
        if (MODE != kBInit) io.r[e] = r;
    }

    const int nb = gridDim.x;
    const real t0 = block_sum(rr, red);
    const real t1 = block_sum(rz, red);
    const real t2 = block_sum(bb, red);
    if (threadIdx.x == 0) {
        io.partials[blockIdx.x] = t0;
        io.partials[nb + blockIdx.x] = t1;
        io.partials[2 * nb + blockIdx.x] = t2;
    }
    if (MODE == kBInit && first_thread()) {
        st->iterA = 0;
        st->iterB = 0;
        st->done = 0;
        st->status = 0;
        st->iters = 0;
        st->tail = 0;
        st->tol2 = io.tol2;
        st->max_iter = io.max_iter;
        st->fallback = 0;
        st->fallbacks = 0;
        st->thresh2 = 0;
        st->bnorm2 = 0;
    }
}

// Flexible CG: after the preconditioner wrote z = M(r), per-block partials of
// z.r, z.q and of the Jacobi alternatives (dinv r).r, (dinv r).q; the next
// phase A sums them, takes beta = -(z.q)/(p.q) (the Golub-Ye Polak-Ribiere
// beta, since r_{k+1} - r_k = -alpha q) and falls back to the Jacobi z when
// z.r <= 0 or is not finite.
template <class real>
__global__ __launch_bounds__(kThreads) void flex_dots(int64_t n, VecIO<real> io) {
    __shared__ real red[kThreads / kWave];
    CgState<real>* st = io.st;
    if (block_flag(&st->done)) return;
    const bool first = st->iterA == 0;
    real zr = 0, zq = 0, jr = 0, jq = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    int64_t e0 = 0;
    if (std::is_same<real, float>::value) {
        // four cells per load (every vector is 16-byte aligned); the tail below
        const int64_t n4 = n / 4;
        for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n4; e += stride) {
            const float4 r = reinterpret_cast<const float4*>(io.r)[e];
            const float4 z = reinterpret_cast<const float4*>(io.z)[e];
            const float4 d = reinterpret_cast<const float4*>(io.dinv)[e];
            zr += z.x * r.x + z.y * r.y + z.z * r.z + z.w * r.w;
            jr += d.x * r.x * r.x + d.y * r.y * r.y + d.z * r.z * r.z + d.w * r.w * r.w;
            if (!first) {
                const float4 q = reinterpret_cast<const float4*>(io.q)[e];
                zq += z.x * q.x + z.y * q.y + z.z * q.z + z.w * q.w;
                jq += d.x * r.x * q.x + d.y * r.y * q.y + d.z * r.z * q.z + d.w * r.w * q.w;
            }
        }
        e0 = n4 * 4;
    }
    for (int64_t e = e0 + (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) {
        const real r = io.r[e], z = io.z[e], d = (real)io.dinv[e];
        zr += z * r;
        jr += d * r * r;
        if (!first) {
            const real q = io.q[e];
            zq += z * q;
            jq += d * r * q;
        }
    }
    const int nb = gridDim.x;
    const real a0 = block_sum(zr, red), a1 = block_sum(zq, red), a2 = block_sum(jr, red),
               a3 = block_sum(jq, red);
    if (threadIdx.x == 0) {
        io.partials[blockIdx.x] = a0;
        io.partials[nb + blockIdx.x] = a1;
        io.partials[2 * nb + blockIdx.x] = a2;
        io.partials[3 * nb + blockIdx.x] = a3;
    }
}

// The steps owed when the loop stopped at K iterations: x += alpha_{K-1}
// p_{K-1} (tail 1), and also alpha_{K-2} p_{K-2} (tail 2). p_j is in p1 for odd
// j and p0 for even j; the loop left both.
template <class real>
__global__ void finalize(int64_t n, real* x, const real* p0, const real* p1,
                         const CgState<real>* st) {
    const int tail = st->tail;
    if (!tail) return;
    const int K = st->iters;
    const real* pa = ((K - 1) & 1) ? p1 : p0;
    const real a = st->alpha[(K - 1) & 1];
    const real* pb = ((K - 2) & 1) ? p1 : p0;
    const real b = tail == 2 ? st->alpha[(K - 2) & 1] : real(0);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        x[e] += tail == 2 ? b * pb[e] + a * pa[e] : a * pa[e];
}

// Training pair of the learned preconditioner in the Jacobi-scaled space from
// a residual r (0 on Dirichlet cells): s^2 = sum(dinv r^2) / n_U,
// r_hat = sqrt(dinv) r / s and target = (x* - x) / (sqrt(dinv) s), the scaled
// error (A~ target = r_hat with A~ = D^-1/2 A D^-1/2); both 0 on Dirichlet cells.
__global__ __launch_bounds__(kThreads) void harvest_scale(int64_t n, const float* r, const float* x,
                                                          const double* xstar, const float* dinv,
                                                          const uint8_t* dmask, const float* part,
                                                          int nb, float n_u, float* r_hat,
                                                          float* target, float* s_out) {
    __shared__ float red[kThreads / kWave];
    const float rr = sum_partials(part, nb, red);
    const float s = rr > 0.f ? sqrtf(rr / n_u) : 1.f;
    const float inv = 1.f / s;
    if (first_thread() && s_out) *s_out = s;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride) {
        const bool d = dmask[l] != 0;
        const double sd = sqrt((double)dinv[l]);
        r_hat[l] = d ? 0.f : (float)(sd * r[l]) * inv;
        target[l] = d ? 0.f : (float)((xstar[l] - (double)x[l]) / (sd * (double)s));
    }
}

__global__ __launch_bounds__(kThreads) void dinv_sq_partials(int64_t n, const float* v,
                                                             const float* dinv, float* part) {
    __shared__ float red[kThreads / kWave];
    float s = 0.f;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride)
        s += dinv[l] * v[l] * v[l];
    const float t = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kThreads) void sum_partials_kernel(const double* parts, int n,
                                                                double* out) {
    __shared__ double red[kThreads / kWave];
    const double s = sum_partials(parts, n, red);
    if (threadIdx.x == 0) *out = s;
}

template <class real, class breal>
__global__ void copy_dirichlet(int64_t n, const uint8_t* dmask, const breal* b, real* x) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        if (dmask[e]) x[e] = (real)b[e];
}

template <class vreal>
__global__ __launch_bounds__(kThreads) void masked_norm2(int64_t n, const uint8_t* dmask,
                                                         const vreal* v, double* partials) {
    __shared__ double red[kThreads / kWave];
    double s = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride)
        if (!dmask[e]) {
            const double t = (double)v[e];
            s += t * t;
        }
    const double tot = block_sum(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ void scale_to_f32(int64_t n, const double* r64, const double* norm2, float* r32) {
    const double inv = 1.0 / sqrt(*norm2);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        r32[e] = (float)(r64[e] * inv);
}

__global__ void axpy_f64_from_f32(int64_t n, const double* norm2, const float* d, double* x) {
    const double s = sqrt(*norm2);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        x[e] += s * (double)d[e];
}

template <class A, class B>
__global__ void convert(int64_t n, const A* a, B* b) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        b[e] = (B)a[e];
}

__global__ void fill_f32(int64_t n, float* a, float v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) a[e] = v;
}

// z = r / diag(A) on unknown cells, 0 on Dirichlet cells: the Jacobi step that
// flexible CG takes between applications of the network.
__global__ __launch_bounds__(kThreads) void jacobi_z(int64_t n, const float* __restrict__ r,
                                                     const float* __restrict__ dinv,
                                                     const uint8_t* __restrict__ dmask, float* z) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride)
        z[l] = dmask[l] ? 0.f : dinv[l] * r[l];
}

// out = D^(power/2) v on unknown cells (power +1: v / sqrt(dinv); -1: v sqrt(dinv)), 0 on Dirichlet cells.
__global__ __launch_bounds__(kThreads) void scale_dsqrt(int64_t n, const float* __restrict__ v,
                                                        const float* __restrict__ dinv,
                                                        const uint8_t* __restrict__ dmask, int power, float* out) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride) {
        const float sq = sqrtf(dinv[l]);
        out[l] = dmask[l] ? 0.f : (power > 0 ? v[l] / sq : v[l] * sq);
    }
}

// Scalars of a single-reduction CG run before kernel 0 (plain vector stores).
__global__ void merged_init(MergedState* ms, float tol2, int max_iter) {
    if (threadIdx.x != 0) return;
    for (int i = 0; i < 2; ++i) {
        MergedSlot& sl = ms->s[i];
        sl.k = 0;
        sl.done = 0;
        sl.status = 1;
        sl.iters = 0;
        sl.rr = 0.f;
        sl.thresh2 = 0.f;
        sl.bnorm2 = 0.f;
        sl.beta = 0.f;
    }
    ms->tol2 = tol2;
    ms->max_iter = max_iter;
}

// flag[0] = 1 if the two arrays differ in any bit (flag cleared by the caller);
// every block that finds a difference stores the same value.
__global__ __launch_bounds__(kThreads) void differ(int64_t n, const uint32_t* __restrict__ a,
                                                   const uint32_t* __restrict__ b, int* flag) {
    int d = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) d |= a[e] != b[e];
    d = __syncthreads_or(d);
    if (d && threadIdx.x == 0) flag[0] = 1;
}

// One 16-byte element per thread and a grid of one block per 256 elements:
// blocks finish and are replaced as the memory system drains them, which on
// gfx950 streams faster than fewer resident blocks looping over the array
// (measured on 1 GiB: 6.36 TB/s against 4.3-5.6 TB/s with 2,048-65,536 blocks
// and 1-8 loads in flight per thread). Stores are nontemporal.
typedef unsigned int pu4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kThreads) void copy_probe(const pu4* __restrict__ src, pu4* __restrict__ dst,
                                                       int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n16; e += stride)
        __builtin_nontemporal_store(src[e], dst + e);
}

// Streaming probe: every output array receives the sum of the input arrays,
// four cells per thread, with the nontemporal stores the stencil kernels use:
// the achievable rate of a kernel that streams the same numbers of arrays in
// and out as a given stencil kernel, without its arithmetic or neighbours.
typedef float sp4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kThreads) void stream_probe(int64_t n4, StreamProbeIO io) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n4; e += stride) {
        sp4 v[kStreamProbeIn];
#pragma unroll
        for (int k = 0; k < kStreamProbeIn; ++k)
            if (k < io.nin) v[k] = reinterpret_cast<const sp4*>(io.in[k])[e];
        sp4 sum = v[0];
#pragma unroll
        for (int k = 1; k < kStreamProbeIn; ++k)
            if (k < io.nin) sum += v[k];
#pragma unroll
        for (int j = 0; j < kStreamProbeOut; ++j)
            if (j < io.nout) __builtin_nontemporal_store(sum, reinterpret_cast<sp4*>(io.out[j]) + e);
    }
}

// ---------------------------------------------------------------------------
// Operator set-up.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double harmonic(double ka, double kb) { return 2.0 * ka * kb / (ka + kb); }

__global__ void perm_to_trans(Geom g, const double* __restrict__ k, double kz_ratio, float* tx,
                              float* ty, float* tz) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < g.n; l += stride) {
        const int i = (int)(l / g.plane);
        const int64_t rem = l - (int64_t)i * g.plane;
        const int j = (int)(rem / g.nz);
        const int kk = (int)(rem - (int64_t)j * g.nz);
        const double kc = k[l];
        tx[l] = (i + 1 < g.nx) ? (float)harmonic(kc, k[l + g.plane]) : 0.f;
        ty[l] = (j + 1 < g.ny) ? (float)harmonic(kc, k[l + g.nz]) : 0.f;
        tz[l] = (kk + 1 < g.nz) ? (float)(kz_ratio * harmonic(kc, k[l + 1])) : 0.f;
    }
}

__device__ __forceinline__ bool is_dirichlet(const Geom& g, const uint8_t* dmask, int64_t l, int i) {
    return dmask ? dmask[l] != 0 : (i == 0 || i == g.nx - 1);
}

__device__ __forceinline__ bool bad_face(float t) { return !(t >= 0.f) || !isfinite(t); }

__global__ __launch_bounds__(kThreads) void setup_kernel(Geom g, SetupIn in, SetupOut out) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    int badT = 0, badC = 0, badP = 0, anyC = 0;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < g.n; l += stride) {
        const int i = (int)(l / g.plane);
        const int64_t rem = l - (int64_t)i * g.plane;
        const int j = (int)(rem / g.nz);
        const int k = (int)(rem - (int64_t)j * g.nz);
        const bool D = is_dirichlet(g, in.dmask, l, i);
        // the six faces of the cell: T and whether the neighbour is a Dirichlet cell
        float t[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        bool nd[6] = {false, false, false, false, false, false};
        int64_t nb[6] = {0, 0, 0, 0, 0, 0};
        if (i + 1 < g.nx) { t[0] = in.tx[l]; nb[0] = l + g.plane; nd[0] = is_dirichlet(g, in.dmask, nb[0], i + 1); }
        if (i > 0)        { t[1] = in.tx[l - g.plane]; nb[1] = l - g.plane; nd[1] = is_dirichlet(g, in.dmask, nb[1], i - 1); }
        if (j + 1 < g.ny) { t[2] = in.ty[l]; nb[2] = l + g.nz; nd[2] = is_dirichlet(g, in.dmask, nb[2], i); }
        if (j > 0)        { t[3] = in.ty[l - g.nz]; nb[3] = l - g.nz; nd[3] = is_dirichlet(g, in.dmask, nb[3], i); }
        if (k + 1 < g.nz) { t[4] = in.tz[l]; nb[4] = l + 1; nd[4] = is_dirichlet(g, in.dmask, nb[4], i); }
        if (k > 0)        { t[5] = in.tz[l - 1]; nb[5] = l - 1; nd[5] = is_dirichlet(g, in.dmask, nb[5], i); }
        // validate the faces this cell owns (+x, +y, +z)
        if ((i + 1 < g.nx && bad_face(t[0])) || (j + 1 < g.ny && bad_face(t[2])) ||
            (k + 1 < g.nz && bad_face(t[4])))
            badT = 1;
        const float cl = in.accum ? in.accum[l] : in.accum_scalar;
        if (!(cl >= 0.f) || !isfinite(cl)) badC = 1;
        if (!D && cl > 0.f) anyC = 1;
        out.dmask[l] = D ? 1 : 0;
        // faces kept in the device copy: both cells unknown
        out.tx[l] = (!D && i + 1 < g.nx && !nd[0]) ? t[0] : 0.f;
        out.ty[l] = (!D && j + 1 < g.ny && !nd[2]) ? t[2] : 0.f;
        out.tz[l] = (!D && k + 1 < g.nz && !nd[4]) ? t[4] : 0.f;
        if (D) {
            const float pd = in.pd ? in.pd[l] : (i == 0 ? 1.f : 0.f);
            if (!isfinite(pd)) badP = 1;
            out.a[l] = 1.f;
            out.a64[l] = 1.0;
            out.dinv[l] = 1.f;
            if (out.b) out.b[l] = pd;
        } else {
            double diag = (double)cl, to_d = (double)cl, bsum = 0.0;
            for (int f = 0; f < 6; ++f) {
                diag += (double)t[f];
                if (nd[f]) {
                    to_d += (double)t[f];
                    const int ni = (f == 0) ? i + 1 : (f == 1 ? i - 1 : i);
                    const float pd = in.pd ? in.pd[nb[f]] : (ni == 0 ? 1.f : 0.f);
                    bsum += (double)t[f] * (double)pd;
                }
            }
            out.a[l] = (float)to_d;
            out.a64[l] = to_d;
            out.dinv[l] = (float)(1.0 / diag);
            if (out.b) out.b[l] = (float)bsum;
        }
    }
    // one atomic per block and flag
    badT = __syncthreads_or(badT);
    badC = __syncthreads_or(badC);
    badP = __syncthreads_or(badP);
    anyC = __syncthreads_or(anyC);
    if (threadIdx.x == 0) {
        if (badT) atomicOr(&out.flags[0], 1);
        if (badC) atomicOr(&out.flags[1], 1);
        if (badP) atomicOr(&out.flags[2], 1);
        if (anyC) atomicOr(&out.flags[4], 1);
    }
}

// Face-list operator set-up: one thread per cell over its entries in the
// sliced layout (entry e: neighbour col[e], face ef[e], -1 for padding), with
// the outputs of the Cartesian set-up
// (identity coefficient, masked faces, 1/diag, mask, b, flags). Without a
// mask no cell is Dirichlet; without pD the Dirichlet values are 0.
__global__ __launch_bounds__(kThreads) void csr_setup_kernel(int64_t n, CsrSetupIn in, SetupOut out,
                                                             float* val) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    int badT = 0, badC = 0, badP = 0, anyC = 0;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride) {
        const bool D = in.dmask && in.dmask[l];
        const float cl = in.accum ? in.accum[l] : in.accum_scalar;
        if (!(cl >= 0.f) || !isfinite(cl)) badC = 1;
        if (!D && cl > 0.f) anyC = 1;
        out.dmask[l] = D ? 1 : 0;
        double diag = (double)cl, to_d = (double)cl, bsum = 0.0;
        const int64_t sl = l / kWave;
        const int e1 = in.sp[sl + 1];
        for (int e = in.sp[sl] + (int)(l - sl * kWave); e < e1; e += kWave) {
            if (in.ef[e] < 0) {  // padding of a slice's shorter rows
                val[e] = 0.f;
                continue;
            }
            const float t = in.T[in.ef[e]];
            if (bad_face(t)) badT = 1;
            const int nb = in.col[e];
            const bool nd = in.dmask && in.dmask[nb];
            val[e] = (!D && !nd) ? t : 0.f;
            if (!D) {
                diag += (double)t;
                if (nd) {
                    to_d += (double)t;
                    bsum += (double)t * (double)(in.pd ? in.pd[nb] : 0.f);
                }
            }
        }
        if (D) {
            const float pd = in.pd ? in.pd[l] : 0.f;
            if (!isfinite(pd)) badP = 1;
            out.a[l] = 1.f;
            out.a64[l] = 1.0;
            out.dinv[l] = 1.f;
            if (out.b) out.b[l] = pd;
        } else {
            out.a[l] = (float)to_d;
            out.a64[l] = to_d;
            out.dinv[l] = (float)(1.0 / diag);
            if (out.b) out.b[l] = (float)bsum;
        }
    }
    badT = __syncthreads_or(badT);
    badC = __syncthreads_or(badC);
    badP = __syncthreads_or(badP);
    anyC = __syncthreads_or(anyC);
    if (threadIdx.x == 0) {
        if (badT) atomicOr(&out.flags[0], 1);
        if (badC) atomicOr(&out.flags[1], 1);
        if (badP) atomicOr(&out.flags[2], 1);
        if (anyC) atomicOr(&out.flags[4], 1);
    }
}

// number of Dirichlet cells (exact count, one atomic per block)
__global__ __launch_bounds__(kThreads) void count_dirichlet(int64_t n, const uint8_t* dmask, int* out) {
    __shared__ int red[kThreads / kWave];
    int c = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) c += dmask[e] ? 1 : 0;
    const int tot = block_sum(c, red);
    if (threadIdx.x == 0 && tot) atomicAdd(out, tot);
}

// Right-hand side of one backward-Euler step of the pressure equation with
// wells: the storage term carries the previous pressure, a well perforation
// adds its index times the bottom-hole pressure (the index itself belongs to
// the operator's diagonal), a source adds its rate, and Dirichlet rows keep
// their value:
//   rhs_K = b_K + c_K p_K^n + WI_K pw_K + q_K   (K not Dirichlet)
//   rhs_K = b_K = p_K^D                           (K Dirichlet)
// evaluated left to right in FP32.
__global__ __launch_bounds__(kThreads) void step_rhs_kernel(int64_t n, StepRhsIn in, float* __restrict__ rhs) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) {
        float v = in.b[e];
        if (!in.dmask[e]) {
            v += (in.c ? in.c[e] : in.c_scalar) * in.p_old[e];
            if (in.wi) v += in.wi[e] * in.pw[e];
            if (in.q) v += in.q[e];
        }
        rhs[e] = v;
    }
}

// The same, four cells per thread (n % 4 == 0, 16-byte aligned arrays).
__global__ __launch_bounds__(kThreads) void step_rhs_v4(int64_t n4, StepRhsIn in, float4* __restrict__ rhs) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n4; e += stride) {
        const float4 b = reinterpret_cast<const float4*>(in.b)[e];
        const uchar4 d = reinterpret_cast<const uchar4*>(in.dmask)[e];
        const float4 p = reinterpret_cast<const float4*>(in.p_old)[e];
        const float4 c = in.c ? reinterpret_cast<const float4*>(in.c)[e] : make_float4(in.c_scalar, in.c_scalar,
                                                                                        in.c_scalar, in.c_scalar);
        float4 w = make_float4(0.f, 0.f, 0.f, 0.f), pw = w, q = w;
        if (in.wi) {
            w = reinterpret_cast<const float4*>(in.wi)[e];
            pw = reinterpret_cast<const float4*>(in.pw)[e];
        }
        if (in.q) q = reinterpret_cast<const float4*>(in.q)[e];
        auto cell = [&](float bv, unsigned char dv, float pv, float cv, float wv, float pwv, float qv) {
            float v = bv;
            if (!dv) {
                v += cv * pv;
                if (in.wi) v += wv * pwv;
                if (in.q) v += qv;
            }
            return v;
        };
        rhs[e] = make_float4(cell(b.x, d.x, p.x, c.x, w.x, pw.x, q.x), cell(b.y, d.y, p.y, c.y, w.y, pw.y, q.y),
                             cell(b.z, d.z, p.z, c.z, w.z, pw.z, q.z), cell(b.w, d.w, p.w, c.w, w.w, pw.w, q.w));
    }
}

int grid_for(int64_t n, int per_thread = 1, int cap = 8192) {
    int64_t b = (n / per_thread + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

}  // namespace

hipError_t launch_phase_b_f32(int mode, int64_t n, const VecIO<float>& io, int nb, hipStream_t s) {
    switch (mode) {
        case kBInit: hipLaunchKernelGGL((phase_b<float, kBInit>), dim3(nb), dim3(kThreads), 0, s, n, io); break;
        case kBPlain: hipLaunchKernelGGL((phase_b<float, kBPlain>), dim3(nb), dim3(kThreads), 0, s, n, io); break;
        case kBJacobi: hipLaunchKernelGGL((phase_b<float, kBJacobi>), dim3(nb), dim3(kThreads), 0, s, n, io); break;
        default: hipLaunchKernelGGL((phase_b<float, kBFlex>), dim3(nb), dim3(kThreads), 0, s, n, io); break;
    }
    return hipGetLastError();
}

hipError_t launch_phase_b_f64(int mode, int64_t n, const VecIO<double>& io, int nb, hipStream_t s) {
    switch (mode) {
        case kBInit: hipLaunchKernelGGL((phase_b<double, kBInit>), dim3(nb), dim3(kThreads), 0, s, n, io); break;
        case kBPlain: hipLaunchKernelGGL((phase_b<double, kBPlain>), dim3(nb), dim3(kThreads), 0, s, n, io); break;
        case kBJacobi: hipLaunchKernelGGL((phase_b<double, kBJacobi>), dim3(nb), dim3(kThreads), 0, s, n, io); break;
        default: hipLaunchKernelGGL((phase_b<double, kBFlex>), dim3(nb), dim3(kThreads), 0, s, n, io); break;
    }
    return hipGetLastError();
}

hipError_t launch_flex_dots_f32(int64_t n, const VecIO<float>& io, int nb, hipStream_t s) {
    hipLaunchKernelGGL((flex_dots<float>), dim3(nb), dim3(kThreads), 0, s, n, io);
    return hipGetLastError();
}

hipError_t launch_finalize_f32(int64_t n, float* x, const float* p0, const float* p1,
                               const CgState<float>* st, hipStream_t s) {
    hipLaunchKernelGGL((finalize<float>), dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, x, p0, p1, st);
    return hipGetLastError();
}

hipError_t launch_finalize_f64(int64_t n, double* x, const double* p0, const double* p1,
                               const CgState<double>* st, hipStream_t s) {
    hipLaunchKernelGGL((finalize<double>), dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, x, p0, p1, st);
    return hipGetLastError();
}

hipError_t launch_harvest(int64_t n, const float* r, const float* x, const double* xstar,
                          const float* dinv, const uint8_t* dmask, float* part, float n_u,
                          float* r_hat, float* target, float* s_out, hipStream_t s) {
    const int nb = grid_for(n, 1, 1024);
    hipLaunchKernelGGL(dinv_sq_partials, dim3(nb), dim3(kThreads), 0, s, n, r, dinv, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(harvest_scale, dim3(nb), dim3(kThreads), 0, s, n, r, x, xstar, dinv, dmask,
                       (const float*)part, nb, n_u, r_hat, target, s_out);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double* parts, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kThreads), 0, s, parts, n, out);
    return hipGetLastError();
}

hipError_t launch_copy_dirichlet_f32(int64_t n, const uint8_t* dmask, const float* b, float* x,
                                     hipStream_t s) {
    hipLaunchKernelGGL((copy_dirichlet<float, float>), dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, dmask, b, x);
    return hipGetLastError();
}

hipError_t launch_copy_dirichlet_f64(int64_t n, const uint8_t* dmask, const void* b, int b_f64,
                                     double* x, hipStream_t s) {
    if (b_f64)
        hipLaunchKernelGGL((copy_dirichlet<double, double>), dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, dmask,
                           static_cast<const double*>(b), x);
    else
        hipLaunchKernelGGL((copy_dirichlet<double, float>), dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, dmask,
                           static_cast<const float*>(b), x);
    return hipGetLastError();
}

hipError_t launch_masked_norm2(int64_t n, const uint8_t* dmask, const void* v, int v_f64,
                               double* partials, double* out, int nb, hipStream_t s) {
    if (v_f64)
        hipLaunchKernelGGL((masked_norm2<double>), dim3(nb), dim3(kThreads), 0, s, n, dmask,
                           static_cast<const double*>(v), partials);
    else
        hipLaunchKernelGGL((masked_norm2<float>), dim3(nb), dim3(kThreads), 0, s, n, dmask,
                           static_cast<const float*>(v), partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_sum_partials(partials, nb, out, s);
}

hipError_t launch_scale_to_f32(int64_t n, const double* r64, const double* norm2, float* r32,
                               hipStream_t s) {
    hipLaunchKernelGGL(scale_to_f32, dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, r64, norm2, r32);
    return hipGetLastError();
}

hipError_t launch_axpy_f64_from_f32(int64_t n, const double* norm2, const float* d, double* x,
                                    hipStream_t s) {
    hipLaunchKernelGGL(axpy_f64_from_f32, dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, norm2, d, x);
    return hipGetLastError();
}

hipError_t launch_convert_f32_to_f64(int64_t n, const float* a, double* b, hipStream_t s) {
    hipLaunchKernelGGL((convert<float, double>), dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, a, b);
    return hipGetLastError();
}

hipError_t launch_convert_f64_to_f32(int64_t n, const double* a, float* b, hipStream_t s) {
    hipLaunchKernelGGL((convert<double, float>), dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, a, b);
    return hipGetLastError();
}

hipError_t launch_fill_f32(int64_t n, float* a, float v, hipStream_t s) {
    hipLaunchKernelGGL(fill_f32, dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, a, v);
    return hipGetLastError();
}

hipError_t launch_jacobi_z(int64_t n, const float* r, const float* dinv, const uint8_t* dmask, float* z,
                           hipStream_t s) {
    hipLaunchKernelGGL(jacobi_z, dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, r, dinv, dmask, z);
    return hipGetLastError();
}

hipError_t launch_scale_dsqrt(int64_t n, const float* v, const float* dinv, const uint8_t* dmask, int power,
                              float* out, hipStream_t s) {
    hipLaunchKernelGGL(scale_dsqrt, dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, v, dinv, dmask, power, out);
    return hipGetLastError();
}

hipError_t launch_merged_init(MergedState* ms, float tol2, int max_iter, hipStream_t s) {
    hipLaunchKernelGGL(merged_init, dim3(1), dim3(kWave), 0, s, ms, tol2, max_iter);
    return hipGetLastError();
}

hipError_t launch_differ(int64_t n, const float* a, const float* b, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(differ, dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n,
                       reinterpret_cast<const uint32_t*>(a), reinterpret_cast<const uint32_t*>(b), flag);
    return hipGetLastError();
}

hipError_t launch_stream_probe(int64_t n, const StreamProbeIO& io, hipStream_t s) {
    const int64_t n4 = n / 4;
    // one float4 of every array per thread, one block per 256 of them (as the copy probe)
    hipLaunchKernelGGL(stream_probe, dim3(grid_for(n4, 1, 1 << 24)), dim3(kThreads), 0, s, n4, io);
    return hipGetLastError();
}

hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const int64_t n16 = (int64_t)(bytes / 16);
    hipLaunchKernelGGL(copy_probe, dim3(grid_for(n16, 1, 1 << 24)), dim3(kThreads), 0, s,
                       static_cast<const pu4*>(src), static_cast<pu4*>(dst), n16);
    return hipGetLastError();
}

hipError_t launch_perm_to_trans(const Geom& g, const double* k, double kz_ratio, float* tx,
                                float* ty, float* tz, hipStream_t s) {
    hipLaunchKernelGGL(perm_to_trans, dim3(grid_for(g.n, 4)), dim3(kThreads), 0, s, g, k, kz_ratio, tx, ty, tz);
    return hipGetLastError();
}

hipError_t launch_csr_setup(int64_t n, const CsrSetupIn& in, const SetupOut& out, float* val,
                            hipStream_t s) {
    hipLaunchKernelGGL(csr_setup_kernel, dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, in, out, val);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(count_dirichlet, dim3(grid_for(n, 16, 4096)), dim3(kThreads), 0, s, n,
                       (const uint8_t*)out.dmask, out.flags + 3);
    return hipGetLastError();
}

hipError_t launch_step_rhs(int64_t n, const StepRhsIn& in, float* rhs, hipStream_t s) {
    auto a16 = [](const void* p) { return ((uintptr_t)p % 16) == 0; };
    const bool v4 = n % 4 == 0 && a16(in.b) && a16(in.p_old) && a16(rhs) && (uintptr_t)in.dmask % 4 == 0 &&
                    (!in.c || a16(in.c)) && (!in.wi || (a16(in.wi) && a16(in.pw))) && (!in.q || a16(in.q));
    if (v4) {
        const int64_t n4 = n / 4;
        hipLaunchKernelGGL(step_rhs_v4, dim3(grid_for(n4, 4)), dim3(kThreads), 0, s, n4, in,
                           reinterpret_cast<float4*>(rhs));
    } else {
        hipLaunchKernelGGL(step_rhs_kernel, dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, in, rhs);
    }
    return hipGetLastError();
}

hipError_t launch_setup(const Geom& g, const SetupIn& in, const SetupOut& out, hipStream_t s) {
    hipLaunchKernelGGL(setup_kernel, dim3(grid_for(g.n, 4)), dim3(kThreads), 0, s, g, in, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(count_dirichlet, dim3(grid_for(g.n, 16, 4096)), dim3(kThreads), 0, s, g.n,
                       (const uint8_t*)out.dmask, out.flags + 3);
    return hipGetLastError();
}

}  // namespace mffv
