// Host-side launchers of the kernels of libmffv (internal interface between
// the C ABI in api.hip and the kernel translation units).
#pragma once

#include "common.hpp"

#include <string>

namespace mffv {

// Work decomposition of a stencil kernel: a block owns a contiguous chunk of
// kThreads*vec cells of a plane and marches through ci consecutive planes.
struct March {
    int vec;     // cells per thread along z: 4 (float4 path) or 1
    int ci;      // planes per block
    int nchunk;  // chunks per plane
    int nich;    // plane groups along x
    int remap;   // 1: XCD-aware block order
    int nseg;    // float4 path, row-segment chunks: segments per row (nz / seg); 0: flat
                 // chunks of kThreads * 4 consecutive cells of the plane
    int seg;     // cells per row segment (a power of two, 16..1024, dividing nz)
    int tps_log2;  // log2 of the threads per row segment (seg / 4); a chunk holds
                   // kThreads >> tps_log2 rows
    int blocks() const { return nchunk * nich; }
};

// seg: 0 = the library's default chunk shape for the grid, -1 = flat chunks,
// > 0 = row segments of seg cells (the caller has checked march_seg_ok).
March plan_march(const Geom& g, int vec, int ci, int remap, int seg = 0);
bool march_seg_ok(const Geom& g, int vec, int seg);

// Record the message returned by mffv_last_error() on this thread; returns code.
int set_error(int code, const std::string& msg);

// Vectors and scalars a stencil kernel works on.
template <class real>
struct StencilIO {
    const real* src = nullptr;   // apply/residual: x; fused CG: r (z when preconditioned)
    real* p0 = nullptr;          // fused CG: direction buffers, p_k in p0 for even k, p1 for odd k
    real* p1 = nullptr;
    real* out = nullptr;         // apply: y; fused CG: q = A p; residual: r = b - A x
    real* xsol = nullptr;        // fused CG: solution, receives the deferred update
    const void* rhs = nullptr;   // residual: b
    int rhs_f64 = 0;             // residual: b is FP64
    real* partials = nullptr;    // per-block partial sums written by this kernel (p.q, or r.r)
    CgState<real>* st = nullptr; // fused CG: device scalars
    const real* pb = nullptr;    // fused CG: partials of the previous phase B, [3][nb_b]
    int nb_b = 0;
    const real* pf = nullptr;    // flexible CG: partials of the preconditioner dots, [4][nb_f]
    int nb_f = 0;
    int precond = 0;             // 0 none, 1 Jacobi, 2 flexible
    const float* dinv = nullptr; // flexible CG: Jacobi fallback z = dinv * r
    const real* rres = nullptr;  // flexible CG: r (for the fallback)
    // single-reduction CG: previous r, q, p (read), new r, p, q (written), the
    // scalars, the launch's parity and the dot partials [4][nb] of this kernel
    // (partials) and of the previous one (pf, nb_f)
    const real* qin = nullptr;
    const real* pin = nullptr;
    real* rout = nullptr;
    real* pout = nullptr;
    MergedState* ms = nullptr;
    int parity = 0;
    float omega = 0.f;           // kSweep1 / kSweep2: the sweeps' weight
    float* sw_j = nullptr;             // kSweep1: written; kSweep2: read (see above)
    const float* sw_sq = nullptr;      // kSweep2: sqrt(dinv), 0 on Dirichlet cells
    const float* sw_scale = nullptr;   //   the network's scale s (device scalar)
    float* sw_flex = nullptr;          //   optional: per-block partials [4][blocks] of the
                                       //   flexible-CG dots z.r, z.q, dinv r.r, dinv r.q
    const float* sw_q = nullptr;       //   q for those dots (NULL: the z.q and r.q sums are 0)
    uint32_t* nn_x0 = nullptr;         // kSweep1, optional: the network's BF16 input pairs
    const float* nn_feat = nullptr;    //   (sqrt(dinv) r1, sqrt(dinv) r1 feat), unscaled
    const int* done = nullptr;         // kSweep1 / kSweep2: the CG loop's done flag; once it is
                                       //   set the pass returns at once (iterations after the end)
};

// kSweep1 / kSweep2: the damped Jacobi sweeps around the learned
// preconditioner (FP32, Cartesian grids), each one pass over the operator:
//   kSweep1: out = src - A (omega dinv src), per-block partials of dinv out^2,
//            and (sw_j) omega dinv src + dinv out;
//   kSweep2: out = z2 + omega dinv (rres - A z2), where z2 = sw_j + s sw_sq src
//            is formed at every stencil point from the network's output src
//            (s = *sw_scale; sw_sq: sqrt(dinv), 0 on Dirichlet cells).
enum StencilMode { kApply = 0, kFusedCg = 1, kResidual = 2, kMergedCg = 3, kSweep1 = 4, kSweep2 = 5 };

hipError_t launch_stencil_f32(int mode, const Geom& g, const Coef& c, const StencilIO<float>& io,
                              const March& m, hipStream_t s);
hipError_t launch_stencil_f64(int mode, const Geom& g, const Coef& c, const StencilIO<double>& io,
                              const March& m, hipStream_t s);

// Phase B of an iteration: alpha from the phase-A partials, r -= alpha q,
// per-block partial dots for the next phase A.
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
    real* partials = nullptr;      // this kernel's partials: [3][nblocks] (init/B) or [4][nblocks] (flex)
    const real* pa = nullptr;      // partials of the phase A before (p.q), nb_a of them
    int nb_a = 0;
    const real* pb = nullptr;      // flexible dots: partials of the phase B before (r.r)
    int nb_b = 0;
    CgState<real>* st = nullptr;
    real tol2 = 0;                 // init: tol^2
    int max_iter = 0;              // init: iteration cap
    int jacobi = 0;                // init: also form z = dinv r and r.z
    int dinv_dot = 0;              // flexible CG: r.(dinv r) into the second partial slot
};

hipError_t launch_phase_b_f32(int mode, int64_t n, const VecIO<float>& io, int nblocks, hipStream_t s);
hipError_t launch_phase_b_f64(int mode, int64_t n, const VecIO<double>& io, int nblocks, hipStream_t s);
// Flexible CG: partial dots z.r, z.q and their Jacobi counterparts of the new z.
hipError_t launch_flex_dots_f32(int64_t n, const VecIO<float>& io, int nblocks, hipStream_t s);
// x += alpha_{k-1} p_{k-1} once the loop has stopped, if still owed.
hipError_t launch_finalize_f32(int64_t n, float* x, const float* p0, const float* p1,
                               const CgState<float>* st, hipStream_t s);
hipError_t launch_finalize_f64(int64_t n, double* x, const double* p0, const double* p1,
                               const CgState<double>* st, hipStream_t s);
// Learned-preconditioner training pair from the residual r of an iterate x
// and a reference solution xstar (part: scratch of 1024 floats).
hipError_t launch_harvest(int64_t n, const float* r, const float* x, const double* xstar,
                          const float* dinv, const uint8_t* dmask, float* part, float n_u,
                          float* r_hat, float* target, float* s_out, hipStream_t s);
// out[0] = sum of n partials (one block, fixed order).
hipError_t launch_sum_partials(const double* parts, int n, double* out, hipStream_t s);

// Elementwise helpers.
hipError_t launch_copy_dirichlet_f32(int64_t n, const uint8_t* dmask, const float* b, float* x,
                                     hipStream_t s);
hipError_t launch_copy_dirichlet_f64(int64_t n, const uint8_t* dmask, const void* b, int b_f64,
                                     double* x, hipStream_t s);
// ||v_U||^2 into *out (per-block partials, then one summing block).
hipError_t launch_masked_norm2(int64_t n, const uint8_t* dmask, const void* v, int v_f64,
                               double* partials, double* out, int nblocks, hipStream_t s);
hipError_t launch_scale_to_f32(int64_t n, const double* r64, const double* scale, float* r32,
                               hipStream_t s);
hipError_t launch_axpy_f64_from_f32(int64_t n, const double* scale, const float* d, double* x,
                                    hipStream_t s);
hipError_t launch_convert_f32_to_f64(int64_t n, const float* a, double* b, hipStream_t s);

// Backward-Euler step right-hand side (optional arrays may be NULL; wi and pw
// come together).
struct StepRhsIn {
    const uint8_t* dmask;
    const float* b;
    const float* c;  // NULL: c_scalar everywhere
    float c_scalar;
    const float* p_old;
    const float* wi;
    const float* pw;
    const float* q;
};
hipError_t launch_step_rhs(int64_t n, const StepRhsIn& in, float* rhs, hipStream_t s);
hipError_t launch_convert_f64_to_f32(int64_t n, const double* a, float* b, hipStream_t s);
hipError_t launch_fill_f32(int64_t n, float* a, float v, hipStream_t s);
hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, hipStream_t s);
constexpr int kStreamProbeIn = 8, kStreamProbeOut = 4;
struct StreamProbeIO {
    const float* in[kStreamProbeIn];
    float* out[kStreamProbeOut];
    int nin, nout;
};
// n FP32 cells (a multiple of 4), 16-byte aligned arrays
hipError_t launch_stream_probe(int64_t n, const StreamProbeIO& io, hipStream_t s);
hipError_t launch_merged_init(MergedState* ms, float tol2, int max_iter, hipStream_t s);
hipError_t launch_jacobi_z(int64_t n, const float* r, const float* dinv, const uint8_t* dmask, float* z,
                           hipStream_t s);
// out = D^(power/2) v on unknown cells (power +1 or -1, D = diag(A)), 0 on Dirichlet cells.
hipError_t launch_scale_dsqrt(int64_t n, const float* v, const float* dinv, const uint8_t* dmask, int power,
                              float* out, hipStream_t s);
// flag[0] = 1 if a and b (n floats) differ in any bit; flag[0] must be 0 before.
hipError_t launch_differ(int64_t n, const float* a, const float* b, int* flag, hipStream_t s);

// Batched persistent CG.
struct BatchResult {
    int iters;      // CG iterations over all passes
    int status;     // 0 converged, 1 iteration or refinement cap, -4 breakdown
    int passes;     // CG passes: 1 + refinement corrections
    float rr;       // recursive r.r of the last pass at exit
    float bnorm2;   // ||b_U||^2 (FP32)
    int pad;
    double rr64;    // ||b - A x||^2 over the unknown cells, FP64, at exit
    double bb64;    // ||b_U||^2, FP64
};

// The scalar part of a grid's operator that may change when its coefficients
// are set again (Coef::a_uniform, Coef::a_const), in device memory owned by the
// grid, so that a batched plan or a captured graph never holds stale copies.
struct CoefScalars {
    int a_uniform;
    float a_const;
};

struct BatchSys {
    Geom g;
    Coef c;                      // a_uniform and a_const are read from cs at launch
    const CoefScalars* cs;
    const float* dinv;
    const uint8_t* dmask;
    const float* b;
    float* x;
    float *r, *p0, *p1, *q, *z;  // workspace of the system's grid handle
    float* dx;                   // refinement: the correction of a pass (grid workspace)
    float *r2, *q2;              // second r and q buffers (single-reduction form only)
    float* part;                 // 2 sets of 4 * nblk partial sums
    double* part64;              // 2 * nblk FP64 partial sums of the residual pass
    unsigned* bar;               // barrier: arrival count, generation
    unsigned long long* xch;     // per block of the system: (tag << 32) | bits of its p.q partial
    BatchResult* res;
    int blk0, nblk;              // the system's blocks in the launch
    int nchunk, nich, ci;        // work items: plane chunks x plane groups
};

struct BatchRun {
    float tol2;
    int max_iter;
    int precond;            // 0 none, 1 Jacobi
    int merged;             // 1: single-reduction iteration (plain CG only)
    uint64_t limit_ticks;   // barrier watchdog, in wall-clock ticks
    int* err;               // set to 1 when a barrier wait expires
    int max_outer;          // 0: one FP32 pass, its FP64 true residual reported;
                            // > 0: up to this many FP32 correction passes, each
                            // started from the FP64 true residual, until that
                            // residual meets tol
    double tol;             // target of the true residual (max_outer > 0)
    double inner_tol;       // smallest relative reduction asked of one correction pass
};

int batched_blocks_per_cu();
hipError_t launch_batched_cg(const BatchSys* systems, const int* block_sys, int nblocks,
                             unsigned* bars, int nbars, int* err, const BatchRun& run, hipStream_t s);

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
// Face-list grids: every cell's faces in the sliced layout of Coef (entry e:
// neighbour col[e], face ef[e] of the caller's face array T, -1 for padding).
struct CsrSetupIn {
    const int* sp; const int* col; const int* ef; const float* T;
    const float* accum; float accum_scalar;
    const uint8_t* dmask; const float* pd;
};
hipError_t launch_csr_setup(int64_t n, const CsrSetupIn& in, const SetupOut& out, float* val, hipStream_t s);

}  // namespace mffv
