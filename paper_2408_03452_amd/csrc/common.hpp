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
};

// Scalars of one CG run, resident on the device between kernels so that the
// host never sits between two iterations.
template <class real>
struct CgState {
    real rho;         // r.z of the current residual (r.r for plain CG)
    real rr;          // r.r of the current residual
    real alpha;       // step of the current iteration
    real alpha_prev;  // step of the previous iteration (deferred x update)
    real beta;        // direction update of the current iteration
    real pq;          // p.Ap of the current iteration
    real thresh2;     // (tol * ||b_U||)^2
    real zq;          // flexible CG: z_{k+1}.q_k
    real bnorm2;      // ||b_U||^2
    int iter;         // completed iterations
    int done;         // 1 once converged, broken down or out of iterations
    int status;       // 0 ok, 1 not converged, -4 breakdown
    int pending;      // 1 while x still lacks alpha_prev * p_prev
    int max_iter;
    int fallback;     // flexible CG: this iteration uses the Jacobi z
    int fallbacks;    // flexible CG: count of such iterations
    int pad;
    unsigned cnt[4];  // arrival counters of the last-block reductions
};

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

// Publish one value per block; returns true in exactly one block, the last to
// arrive, after which every block's value is visible to it. Partial values go
// through agent-scope atomics so that they are coherent across the XCD L2s.
template <class T>
__device__ __forceinline__ void store_partial(T* slot, T v) {
    __hip_atomic_store(slot, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T load_partial(const T* slot) {
    return __hip_atomic_load(const_cast<T*>(slot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool arrive_last(unsigned* counter, unsigned nblocks, int* flag_lds) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT);
        *flag_lds = (prev == nblocks - 1) ? 1 : 0;
    }
    __syncthreads();
    const bool last = *flag_lds != 0;
    if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return last;
}

// Sum nparts partial values in a fixed order (strided per thread, then the
// block tree): the result is bitwise reproducible for a given launch shape.
template <class T>
__device__ __forceinline__ T sum_partials(const T* parts, int nparts, T* lds) {
    T s = T(0);
    for (int i = threadIdx.x; i < nparts; i += kThreads) s += load_partial(parts + i);
    return block_sum(s, lds);
}

__device__ __forceinline__ void reset_counter(unsigned* counter) {
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace mffv
