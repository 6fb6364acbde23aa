// Internal definitions shared by the HIP translation units of libmffv.
//
// Grid layout: flat index l = (i*ny + j)*nz + k, z fastest. A "plane" is all
// cells with one i (ny*nz cells, contiguous); stencil kernels march through
// planes along x and keep the i-1, i, i+1 values of a cell in registers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mffv {

constexpr int kThreads = 256;      // threads per block of every kernel
constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kNumXcd = 8;         // MI355X: 8 accelerator complex dies, own L2 each

struct Geom {
    int nx, ny, nz;
    int64_t n;      // nx*ny*nz
    int64_t plane;  // ny*nz (x stride)
};

// Operator coefficients held by a grid handle (device pointers, FP32, n each).
//  a   : identity coefficient; 1 on Dirichlet cells, c + sum of the faces that
//        touch Dirichlet cells on unknown cells (those faces are zeroed below).
//  tx/ty/tz : faces to the +x/+y/+z neighbour, zero beyond the domain and on
//        every face that touches a Dirichlet cell.
// With this form y = a x + sum_f T_f (x - x_nbr) is the eliminated operator
// on unknown cells and the identity on Dirichlet cells, with no branch.
// a64 holds the same identity coefficient in FP64 (c + the Dirichlet faces
// summed without rounding), read by the FP64 kernels so that their operator is
// exactly the one defined by the FP32 inputs.
struct Coef {
    const float* a;
    const float* tx;
    const float* ty;
    const float* tz;
    const double* a64;
    // a_uniform: a (and a64) equal a_const on the planes 2 <= i < nx - 2, so the
    // kernels read the arrays only on the two planes at each end (a scalar
    // accumulation with the x-plane Dirichlet set: away from those planes the
    // identity coefficient is the accumulation alone)
    int a_uniform;
    float a_const;
    // face-list (unstructured) operator, NULL on a Cartesian grid: each cell's
    // faces as neighbour cells and transmissibilities, zero on every face that
    // touches a Dirichlet cell (the role of tx, ty, tz above). Sliced layout:
    // the cells in slices of kWave consecutive cells; slice s holds entries
    // [sp[s], sp[s+1]), column-major, so entry j of cell K sits at
    // sp[K / kWave] + j * kWave + K % kWave and a wave reads each entry column
    // of its slice in one coalesced access. Padding entries carry T = 0.
    const int* sp;     // slice pointers, ceil(n / kWave) + 1
    const int* col;    // neighbour cell of each entry
    const float* val;  // T of each entry
};

__device__ __forceinline__ bool coef_plane_uniform(const Coef& c, int i, int nx) {
    return c.a_uniform && i >= 2 && i < nx - 2;
}

// Scalars of one CG run, resident on the device between kernels so that the
// host never sits between two iterations. No kernel reduces its own partial
// sums: every block of the consuming kernel sums the producer's per-block
// partials in the same fixed order, so all blocks reach the same scalars
// without atomics or cross-XCD fences, and block 0 records them here for the
// kernels and the host that come later. Fields written while other blocks of
// the same kernel read the state are double-buffered by iteration parity.
template <class real>
struct CgState {
    real rho[2];      // rho[k&1] = r_k.z_k (r_k.r_k for plain CG), written by phase A_k
    real alpha[2];    // alpha[k&1] = step of iteration k, written by phase B_k
    real pq[2];       // pq[k&1] = p_k.A p_k, written by phase B_k
    real rr;          // r.r at the last convergence check
    real beta;        // last direction update (for inspection)
    real thresh2;     // (tol * ||b_U||)^2, fixed by phase A_0
    real bnorm2;      // ||b_U||^2, fixed by phase A_0
    real tol2;        // tol^2, set by the init kernel
    int iterA;        // index k of the next phase A (written by phase B)
    int iterB;        // index k of the next phase B (written by phase A)
    int done;         // 1 once converged, broken down or out of iterations
    int status;       // 0 ok, 1 not converged, -4 breakdown
    int iters;        // completed iterations at exit
    int tail;         // steps x lacks at exit: 1 (alpha_{iters-1} p_{iters-1}) or 2 (and alpha_{iters-2} p_{iters-2})
    int max_iter;
    int fallback;     // flexible CG: iteration iterA uses the Jacobi z
    int fallbacks;    // flexible CG: count of such iterations
    int pad[3];
};

// Scalars of the single-reduction CG (one kernel per iteration). Kernel K
// reads slot K & 1 and writes slot (K + 1) & 1, so no block reads a field that
// another block of the same kernel writes; once a kernel finds the run over it
// marks both slots done.
struct MergedSlot {
    int k;            // index K of the kernel that reads this slot
    int done;         // 1 once converged, broken down or out of iterations
    int status;       // 0 ok, 1 not converged, -4 breakdown
    int iters;        // completed iterations at exit
    float rr;         // r.r of the last completed iteration (exact)
    float thresh2;    // (tol * ||b_U||)^2
    float bnorm2;     // ||b_U||^2
    float beta;       // last direction update (for inspection)
};
struct MergedState {
    MergedSlot s[2];
    float tol2;
    int max_iter;
    int pad[2];
};

// One cell of the eliminated operator in difference form:
//   a x + sum over the six faces of T (x - x_nbr).
template <class real, class creal>
__device__ __forceinline__ real cell_op(creal a, real x, creal txp, real xxp, creal txm, real xxm,
                                        creal typ, real xyp, creal tym, real xym, creal tzp,
                                        real xzp, creal tzm, real xzm) {
    real y = (real)a * x;
    y += (real)txp * (x - xxp);
    y += (real)txm * (x - xxm);
    y += (real)typ * (x - xyp);
    y += (real)tym * (x - xym);
    y += (real)tzp * (x - xzp);
    y += (real)tzm * (x - xzm);
    return y;
}

// Map the hardware block index to a logical work index so that each XCD gets
// a contiguous range of work. Blocks are dispatched round-robin over the XCDs
// (block b runs on XCD b % 8); neighbouring logical tiles then share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb / kNumXcd, rem = nb % kNumXcd;
    const int x = b % kNumXcd, s = b / kNumXcd;
    return x * q + (x < rem ? x : rem) + s;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Deterministic block sum: wave butterfly, then the waves in index order.
template <class T>
__device__ __forceinline__ T block_sum(T v, T* lds /* kThreads/kWave entries */) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    T s = T(0);
#pragma unroll
    for (int i = 0; i < kThreads / kWave; ++i) s += lds[i];
    return s;
}

// Partial values a thread loads before adding them: the loads of a batch are
// in flight together (one memory latency per batch instead of one per value).
constexpr int kPartBatch = 4;

// Sum nparts partial values written by an earlier kernel, in a fixed order
// (strided per thread, then the block tree): every block that calls it gets
// the same bits, and the result is reproducible for a given launch shape.
// A thread adds its values in index order whatever the batching of the loads.
template <class T>
__device__ __forceinline__ T sum_partials(const T* parts, int nparts, T* lds) {
    T s = T(0);
    for (int i = threadIdx.x; i < nparts; i += kPartBatch * kThreads) {
        T v[kPartBatch];
#pragma unroll
        for (int k = 0; k < kPartBatch; ++k) v[k] = i + k * kThreads < nparts ? parts[i + k * kThreads] : T(0);
#pragma unroll
        for (int k = 0; k < kPartBatch; ++k)
            if (i + k * kThreads < nparts) s += v[k];
    }
    return block_sum(s, lds);
}

// The first batch of sum_partials_n's loads of thread threadIdx.x (values at
// or past a count read as 0). Issued on its own, these loads can be in flight
// together with a kernel's other start-up reads: one memory round trip
// instead of several in a row.
// Indexes past the count are clamped to the last entry (an array with count 0
// is not read): every load is unconditional within the block-uniform test, so
// the compiler does not fold a load into the add that consumes it.
template <class T, int N>
__device__ __forceinline__ void load_partials_first(const T* const (&parts)[N], const int (&counts)[N],
                                                    T (&v)[N][kPartBatch]) {
    const int i = threadIdx.x;
#pragma unroll
    for (int j = 0; j < N; ++j) {
#pragma unroll
        for (int k = 0; k < kPartBatch; ++k) v[j][k] = T(0);
        if (counts[j] > 0) {
#pragma unroll
            for (int k = 0; k < kPartBatch; ++k) {
                const int e = i + k * kThreads;
                v[j][k] = parts[j][e < counts[j] ? e : counts[j] - 1];
            }
        }
    }
}

// A relaxed load of a value that no block changes during the kernel (or whose
// change every block would reach by itself): the compiler keeps it where it is
// written, neither moving it past a barrier nor into a branch, so it overlaps
// the loads issued next to it.
template <class T>
__device__ __forceinline__ T early_load(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait for every load the wave has issued: a kernel that returns early after
// such early loads ends with none of them in flight.
__device__ __forceinline__ void drain_loads() { __builtin_amdgcn_s_waitcnt(0); }

// N sums of partials at once, each in sum_partials' order (so each result
// has the same bits as sum_partials of that array), with one pass over the
// arrays and one block tree: the loads of all arrays are in flight together.
// first: the thread's first batch, loaded by load_partials_first with counts
// at least these (a larger load count reads entries that are then not added).
// An array with count 0 sums to 0. lds: N * kThreads / kWave entries.
template <class T, int N>
__device__ __forceinline__ void sum_partials_n_rest(const T* const (&parts)[N], const int (&counts)[N],
                                                    const T (&first)[N][kPartBatch], T* lds, T (&out)[N]) {
    T s[N];
    int mx = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        s[j] = T(0);
        mx = counts[j] > mx ? counts[j] : mx;
    }
    const int i0 = threadIdx.x;
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int k = 0; k < kPartBatch; ++k) {
            // the value enters here and no earlier: the compiler cannot start
            // the adds (and wait for the loads) ahead of a barrier before this
            T v = first[j][k];
            asm volatile("" : "+v"(v));
            if (i0 + k * kThreads < counts[j]) s[j] += v;
        }
    for (int i = i0 + kPartBatch * kThreads; i < mx; i += kPartBatch * kThreads) {
        T v[N][kPartBatch];
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int k = 0; k < kPartBatch; ++k)
                v[j][k] = i + k * kThreads < counts[j] ? parts[j][i + k * kThreads] : T(0);
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int k = 0; k < kPartBatch; ++k)
                if (i + k * kThreads < counts[j]) s[j] += v[j][k];
    }
    constexpr int NW = kThreads / kWave;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
    for (int j = 0; j < N; ++j) s[j] = wave_sum(s[j]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) lds[j * NW + w] = s[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < N; ++j) {
        T t = T(0);
#pragma unroll
        for (int i = 0; i < NW; ++i) t += lds[j * NW + i];
        out[j] = t;
    }
}

template <class T, int N>
__device__ __forceinline__ void sum_partials_n(const T* const (&parts)[N], const int (&counts)[N], T* lds,
                                               T (&out)[N]) {
    T first[N][kPartBatch];
    load_partials_first(parts, counts, first);
    sum_partials_n_rest(parts, counts, first, lds, out);
}

__device__ __forceinline__ bool first_thread() { return blockIdx.x == 0 && threadIdx.x == 0; }

// Thread 0's copy of a flag that every thread has read (so that the read can
// be in flight with other loads), shared through LDS: all waves of the block
// take the same branch even if another block of the same kernel sets the
// flag meanwhile.
__device__ __forceinline__ bool block_uniform(int v) {
    __shared__ int s;
    if (threadIdx.x == 0) s = v;
    __syncthreads();
    const bool r = s != 0;
    __syncthreads();
    return r;
}

// Read a flag once per block (thread 0) and share it through LDS, so that all
// waves of the block take the same branch even if another block of the same
// kernel sets the flag meanwhile.
__device__ __forceinline__ bool block_flag(const int* flag) {
    __shared__ int v;
    if (threadIdx.x == 0) v = *flag;
    __syncthreads();
    const bool r = v != 0;
    __syncthreads();
    return r;
}

}  // namespace mffv
