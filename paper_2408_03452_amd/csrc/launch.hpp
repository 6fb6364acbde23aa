// Host-side launchers of the kernels of libmffv (internal interface between
// the C ABI in api.hip and the kernel translation units).
#pragma once

#include "common.hpp"

namespace mffv {

// Work decomposition of a stencil kernel: a block owns a contiguous chunk of
// kThreads*vec cells of a plane and marches through ci consecutive planes.
struct March {
    int vec;     // cells per thread along z: 4 (float4 path) or 1
    int ci;      // planes per block
    int nchunk;  // chunks per plane
    int nich;    // plane groups along x
    int remap;   // 1: XCD-aware block order
    int blocks() const { return nchunk * nich; }
};

March plan_march(const Geom& g, int vec, int ci, int remap);

// Vectors and scalars a stencil kernel works on.
template <class real>
struct StencilIO {
    const real* src = nullptr;   // apply/residual: x; fused CG: r (or z when preconditioned)
    real* p0 = nullptr;          // fused CG: direction buffers, chosen by iteration parity
    real* p1 = nullptr;
    real* out = nullptr;         // apply: y; fused CG: q = A p; residual: r = b - A x
    real* xsol = nullptr;        // fused CG: solution, receives the deferred update
    const void* rhs = nullptr;   // residual: b
    int rhs_f64 = 0;             // residual: b is FP64
    real* partials = nullptr;    // per-block partial dot products
    CgState<real>* st = nullptr; // fused CG: device scalars
    real* sum_out = nullptr;     // residual: ||r||^2 written by the last block (may be null)
    unsigned* counter = nullptr; // residual: arrival counter
};

enum StencilMode { kApply = 0, kFusedCg = 1, kResidual = 2 };

hipError_t launch_stencil_f32(int mode, const Geom& g, const Coef& c, const StencilIO<float>& io,
                              const March& m, hipStream_t s);
hipError_t launch_stencil_f64(int mode, const Geom& g, const Coef& c, const StencilIO<double>& io,
                              const March& m, hipStream_t s);

// Phase B of an iteration: r -= alpha q, dot products, scalar updates.
enum PhaseBMode { kBInit = 0, kBPlain = 1, kBJacobi = 2, kBFlex = 3 };

template <class real>
struct VecIO {
    real* r = nullptr;
    const real* q = nullptr;
    real* z = nullptr;             // Jacobi: written; flexible: read
    const float* dinv = nullptr;   // inverse of diag(A)
    const uint8_t* dmask = nullptr;
    const void* b = nullptr;       // init: right-hand side (for ||b_U||)
    int b_f64 = 0;
    real* partials = nullptr;      // [3][nblocks]
    CgState<real>* st = nullptr;
    real tol2 = 0;                 // init: tol^2
    int max_iter = 0;              // init: iteration cap
};

hipError_t launch_phase_b_f32(int mode, int64_t n, const VecIO<float>& io, int nblocks, hipStream_t s);
hipError_t launch_phase_b_f64(int mode, int64_t n, const VecIO<double>& io, int nblocks, hipStream_t s);
// Flexible CG: dots z.r and z.q of the new z, beta, and the Jacobi safeguard.
hipError_t launch_flex_dots_f32(int64_t n, const VecIO<float>& io, int nblocks, hipStream_t s);
// x += alpha_prev * p_prev once the loop has stopped.
hipError_t launch_finalize_f32(int64_t n, float* x, float* p0, float* p1, CgState<float>* st,
                               hipStream_t s);
hipError_t launch_finalize_f64(int64_t n, double* x, double* p0, double* p1, CgState<double>* st,
                               hipStream_t s);

// Elementwise helpers.
hipError_t launch_copy_dirichlet_f32(int64_t n, const uint8_t* dmask, const float* b, float* x,
                                     hipStream_t s);
hipError_t launch_copy_dirichlet_f64(int64_t n, const uint8_t* dmask, const void* b, int b_f64,
                                     double* x, hipStream_t s);
hipError_t launch_masked_norm2(int64_t n, const uint8_t* dmask, const void* v, int v_f64,
                               double* partials, unsigned* counter, double* out, int nblocks,
                               hipStream_t s);
hipError_t launch_scale_to_f32(int64_t n, const double* r64, const double* scale, float* r32,
                               hipStream_t s);
hipError_t launch_axpy_f64_from_f32(int64_t n, const double* scale, const float* d, double* x,
                                    hipStream_t s);
hipError_t launch_convert_f32_to_f64(int64_t n, const float* a, double* b, hipStream_t s);
hipError_t launch_convert_f64_to_f32(int64_t n, const double* a, float* b, hipStream_t s);
hipError_t launch_fill_f32(int64_t n, float* a, float v, hipStream_t s);
hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, hipStream_t s);

// Operator set-up.
hipError_t launch_perm_to_trans(const Geom& g, const double* k, double kz_ratio, float* tx,
                                float* ty, float* tz, hipStream_t s);
struct SetupIn {
    const float* tx; const float* ty; const float* tz;
    const float* accum; float accum_scalar;
    const uint8_t* dmask; const float* pd;
};
struct SetupOut {
    float* a; double* a64; float* tx; float* ty; float* tz; float* dinv; uint8_t* dmask; float* b;
    int* flags;  // [0] bad T, [1] bad c, [2] bad pD, [3] #Dirichlet cells, [4] any c > 0
};
hipError_t launch_setup(const Geom& g, const SetupIn& in, const SetupOut& out, hipStream_t s);

}  // namespace mffv
