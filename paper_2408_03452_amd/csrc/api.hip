// C ABI of libmffv: grid handles, operator set-up, apply, CG solves.
//
// The CG loop (Alg. 1) runs as two fused kernels per iteration with every
// scalar kept on the device: phase A forms the new direction, applies the
// operator to it, adds the previous step to the solution and reduces p.Ap;
// phase B updates the residual and reduces r.r (and r.z). The host only
// enqueues chunks of iterations (optionally as a replayed HIP graph) and polls
// a convergence flag copied to pinned memory once per chunk, one chunk behind,
// so the device never waits for the host.
#include "mffv.h"
#include "launch.hpp"
#include "nn.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace mffv;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

}  // namespace

namespace mffv {
int set_error(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace mffv

namespace {

int hip_fail(hipError_t e, const char* what) {
    return fail(MFFV_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

template <class T>
int dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) return MFFV_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(MFFV_ENOMEM, std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) +
                                     " bytes failed: " + hipGetErrorString(e));
    }
    return MFFV_OK;
}

template <class T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

}  // namespace

struct CgGraph {
    hipGraphExec_t exec = nullptr;
    int chunk = 0;
    const void* net = nullptr;  // learned preconditioner the graph was captured with
    float omega = 0.f;          // and the weight of its Jacobi sweeps
    int64_t net_gen = 0;        // and the token of its workspace (unique per network and allocation)
};

constexpr int kTimedIters = 32;

struct mffv_grid {
    Geom g{};
    hipStream_t stream = nullptr;
    int device = 0;
    // operator
    float *a = nullptr, *tx = nullptr, *ty = nullptr, *tz = nullptr, *dinv = nullptr;
    double* a64 = nullptr;
    uint8_t* dmask = nullptr;
    int* flags = nullptr;
    CoefScalars* cdev = nullptr;  // a_uniform and a_const in device memory (read by batched solves)
    bool has_coef = false;
    int64_t n_unknown = 0;
    float* feat = nullptr;     // learned preconditioner input feature (lazy)
    float* sqd = nullptr;      // sqrt(dinv) on unknown cells, 0 on Dirichlet cells (with feat)
    const float* flex_part = nullptr;  // flexible-CG dot partials of the last preconditioner step
    int flex_nb = 0;                   //   when the network's second sweep formed them
    bool feat_valid = false;
    // FP32 workspace
    float *r = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr, *z = nullptr, *xw = nullptr,
          *bw = nullptr;
    float* step_rhs = nullptr;  // right-hand side of the time steps
    // face-list grid: every cell's faces in the sliced layout of Coef (slice
    // pointers; entry -> neighbour, face, masked T); NULL on a Cartesian grid
    bool faces = false;
    int nfaces = 0;
    int *csr_sp = nullptr, *csr_col = nullptr, *csr_ef = nullptr;
    float* csr_val = nullptr;
    CgState<float>* st32 = nullptr;
    // single-reduction CG: second r and q buffers, scalars, partials [2][4][max_blocks]
    float *r2 = nullptr, *q2 = nullptr, *partM = nullptr;
    MergedState* ms = nullptr;
    int mpar = 0;              // parity of the next single-reduction launch
    int flex_count = 0;        // flexible CG: iterations enqueued since the run started
    CgGraph graphM;
    // FP64 workspace
    double *r64 = nullptr, *p064 = nullptr, *p164 = nullptr, *q64 = nullptr, *x64 = nullptr,
           *b64 = nullptr, *rres = nullptr;
    CgState<double>* st64 = nullptr;
    // per-block partial sums (stored as doubles, used as floats by FP32 kernels)
    double* partA = nullptr;  // phase A: p.q, max_blocks
    double* partB = nullptr;  // phase B / init: r.r, r.z, ||b_U||^2, 3 * nb_vec
    double* partF = nullptr;  // flexible CG dots, 4 * nb_vec
    double* partR = nullptr;  // residual and norm reductions, max_blocks
    int max_blocks = 0;
    double* dscal = nullptr;  // [0] ||b_U||^2, [1] ||r||^2
    // pinned host mirror of the loop state, double-buffered
    char* hstate = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t t0 = nullptr, t1 = nullptr;
    bool a_uniform = false;  // see Coef::a_uniform
    float a_const = 0.f;
    // per-kernel timing of the first kTimedIters FP32 iterations (opts.timing)
    hipEvent_t tev[kTimedIters][4] = {};
    hipEvent_t tnev[kTimedIters][5] = {};   // the network's layers (learned preconditioner)
    bool tnev_used[kTimedIters] = {};
    bool tev_made = false;
    bool timing = false;
    int timed = 0;
    int timed_real = -1;  // iterations of the first timed CG run that did work
    // launch shapes: FP32 CG kernels, the FP32 apply (tuned on its own), FP64
    March m32{}, m_apply{}, m64{};
    int nb_vec = 0;
    // captured iteration chunks: [precond 0..2]
    CgGraph graph32[3];
    CgGraph graph64[2];
};

namespace {

Coef coef_of(const mffv_grid* G) {
    return Coef{G->a,           G->tx,      G->ty,       G->tz,     G->a64, G->a_uniform ? 1 : 0,
                G->a_const,     G->csr_sp,  G->csr_col,  G->csr_val};
}

// Entry points that need the Cartesian structure (launch shapes, the network,
// the batched kernel) refuse face-list grids.
int check_cartesian(const mffv_grid* G, const char* what) {
    if (G && G->faces) return fail(MFFV_EINVAL, std::string(what) + " needs a Cartesian grid");
    return MFFV_OK;
}

int check_grid(const mffv_grid* G, bool need_coef) {
    if (!G) return fail(MFFV_EINVAL, "grid handle is NULL");
    if (need_coef && !G->has_coef)
        return fail(MFFV_ESTATE, "operator coefficients not set (call mffv_set_transmissibility)");
    return MFFV_OK;
}

int set_device(const mffv_grid* G) {
    HIP_TRY(hipSetDevice(G->device));
    return MFFV_OK;
}

int ensure_ws32(mffv_grid* G) {
    if (G->r) return MFFV_OK;
    const size_t n = (size_t)G->g.n;
    int rc;
    if ((rc = dalloc(&G->r, n)) || (rc = dalloc(&G->p0, n)) || (rc = dalloc(&G->p1, n)) ||
        (rc = dalloc(&G->q, n)) || (rc = dalloc(&G->z, n)) || (rc = dalloc(&G->xw, n)) ||
        (rc = dalloc(&G->bw, n)) || (rc = dalloc(&G->st32, 1))) {
        dfree(G->r); dfree(G->p0); dfree(G->p1); dfree(G->q); dfree(G->z); dfree(G->xw);
        dfree(G->bw); dfree(G->st32);
        return rc;
    }
    HIP_TRY(hipMemsetAsync(G->st32, 0, sizeof(CgState<float>), G->stream));
    return MFFV_OK;
}

int ensure_x64(mffv_grid* G) {
    if (G->x64) return MFFV_OK;
    const size_t n = (size_t)G->g.n;
    int rc;
    if ((rc = dalloc(&G->x64, n)) || (rc = dalloc(&G->rres, n))) {
        dfree(G->x64); dfree(G->rres);
        return rc;
    }
    return MFFV_OK;
}

int ensure_ws64(mffv_grid* G) {
    int rc = ensure_x64(G);
    if (rc) return rc;
    if (G->r64) return MFFV_OK;
    const size_t n = (size_t)G->g.n;
    if ((rc = dalloc(&G->r64, n)) || (rc = dalloc(&G->p064, n)) || (rc = dalloc(&G->p164, n)) ||
        (rc = dalloc(&G->q64, n)) || (rc = dalloc(&G->b64, n)) || (rc = dalloc(&G->st64, 1))) {
        dfree(G->r64); dfree(G->p064); dfree(G->p164); dfree(G->q64); dfree(G->b64);
        dfree(G->st64);
        return rc;
    }
    HIP_TRY(hipMemsetAsync(G->st64, 0, sizeof(CgState<double>), G->stream));
    return MFFV_OK;
}

int ensure_feature(mffv_grid* G) {
    if (G->feat_valid) return MFFV_OK;
    int rc;
    if (!G->feat && (rc = dalloc(&G->feat, (size_t)G->g.n))) return rc;
    if (!G->sqd && (rc = dalloc(&G->sqd, (size_t)G->g.n))) return rc;
    if ((rc = nn_feature(G->g, G->dinv, G->dmask, (float)G->n_unknown,
                         reinterpret_cast<float*>(G->partR), G->feat, G->sqd, G->stream)))
        return rc;
    G->feat_valid = true;
    return MFFV_OK;
}

// Copy the operator's scalars to the grid's device struct; the batched kernel
// reads them there at every launch (stream-ordered after earlier solves).
int store_coef_scalars(mffv_grid* G) {
    const CoefScalars cs{G->a_uniform ? 1 : 0, G->a_const};
    HIP_TRY(hipMemcpyAsync(G->cdev, &cs, sizeof(cs), hipMemcpyHostToDevice, G->stream));
    HIP_TRY(hipStreamSynchronize(G->stream));
    return MFFV_OK;
}

void drop_graphs(mffv_grid* G) {
    for (auto& gr : G->graph32)
        if (gr.exec) { (void)hipGraphExecDestroy(gr.exec); gr.exec = nullptr; }
    for (auto& gr : G->graph64)
        if (gr.exec) { (void)hipGraphExecDestroy(gr.exec); gr.exec = nullptr; }
    if (G->graphM.exec) { (void)hipGraphExecDestroy(G->graphM.exec); G->graphM.exec = nullptr; }
}

// Residual r = b - A x in FP64; ||r||^2 into out[1] and ||b_U||^2 into out[0]
// (device doubles; by default the grid's dscal).
int true_residual_f64(mffv_grid* G, const void* b, int b_f64, const double* x, double* r,
                      double* out = nullptr) {
    if (!out) out = G->dscal;
    StencilIO<double> io;
    io.src = x;
    io.out = r;
    io.rhs = b;
    io.rhs_f64 = b_f64;
    io.partials = G->partR;
    HIP_TRY(launch_stencil_f64(kResidual, G->g, coef_of(G), io, G->m64, G->stream));
    HIP_TRY(launch_sum_partials(G->partR, G->m64.blocks(), out + 1, G->stream));
    HIP_TRY(launch_masked_norm2(G->g.n, G->dmask, b, b_f64, G->partR, out + 0, G->nb_vec,
                                G->stream));
    return MFFV_OK;
}

int read_rel(mffv_grid* G, double* rel, double* rn2_out = nullptr) {
    double h[2];
    HIP_TRY(hipMemcpyAsync(h, G->dscal, sizeof(h), hipMemcpyDeviceToHost, G->stream));
    HIP_TRY(hipStreamSynchronize(G->stream));
    if (rn2_out) *rn2_out = h[1];
    *rel = h[0] > 0 ? std::sqrt(h[1] / h[0]) : std::sqrt(h[1]);
    return MFFV_OK;
}

struct LoopResult {
    int iters = 0;
    int status = 0;
    int fallbacks = 0;
    double rel_rec = 0;
    bool merged = false;  // ran the single-reduction loop
};

// Enqueue one CG iteration (phase A, phase B, and for flexible CG the
// preconditioner and its dots).
int enqueue_iter32(mffv_grid* G, int precond, const mffv_net* net, int nn_every = 1, float omega = 0.f) {
    // flexible CG: the network preconditions every nn_every-th iteration, Jacobi
    // the others (the position in the loop is counted per enqueued iteration)
    const bool use_nn = (++G->flex_count % nn_every) == 0;
    hipEvent_t* ev = nullptr;
    hipEvent_t* nev = nullptr;
    if (G->timing && G->timed < kTimedIters) {
        G->tnev_used[G->timed] = precond == MFFV_PRECOND_LEARNED && use_nn;
        if (G->tnev_used[G->timed]) nev = G->tnev[G->timed];
        ev = G->tev[G->timed++];
    }
    if (ev) HIP_TRY(hipEventRecord(ev[0], G->stream));
    float* pa = reinterpret_cast<float*>(G->partA);
    float* pb = reinterpret_cast<float*>(G->partB);
    float* pf = reinterpret_cast<float*>(G->partF);
    StencilIO<float> a;
    a.src = (precond == MFFV_PRECOND_NONE) ? G->r : G->z;
    a.p0 = G->p0;
    a.p1 = G->p1;
    a.out = G->q;
    a.xsol = G->xw;
    a.partials = pa;
    a.st = G->st32;
    a.pb = pb;
    a.nb_b = G->nb_vec;
    // the flexible-CG dots of the previous preconditioner step: from the
    // fused second sweep (network-owned partials) or from flex_dots
    a.pf = G->flex_part ? G->flex_part : pf;
    a.nb_f = G->flex_part ? G->flex_nb : G->nb_vec;
    a.precond = precond;
    a.dinv = G->dinv;
    a.rres = G->r;
    HIP_TRY(launch_stencil_f32(kFusedCg, G->g, coef_of(G), a, G->m32, G->stream));
    if (ev) HIP_TRY(hipEventRecord(ev[1], G->stream));
    VecIO<float> v;
    v.r = G->r;
    v.q = G->q;
    v.z = G->z;
    v.dinv = G->dinv;
    v.dmask = G->dmask;
    v.partials = pb;
    v.pa = pa;
    v.nb_a = G->m32.blocks();
    v.st = G->st32;
    v.dinv_dot = precond == MFFV_PRECOND_LEARNED ? 1 : 0;
    const int mode = precond == MFFV_PRECOND_NONE ? kBPlain
                     : precond == MFFV_PRECOND_JACOBI ? kBJacobi : kBFlex;
    HIP_TRY(launch_phase_b_f32(mode, G->g.n, v, G->nb_vec, G->stream));
    if (ev) HIP_TRY(hipEventRecord(ev[2], G->stream));
    if (precond == MFFV_PRECOND_LEARNED) {
        if (use_nn) {
            const float* fp = nullptr;
            int nbf = 0;
            int rc = nn_precondition(net, G->g, coef_of(G), G->m32, omega, G->r, G->dinv, G->dmask, G->sqd,
                                     G->z, pb + G->nb_vec, G->nb_vec, G->feat, (float)G->n_unknown, G->stream,
                                     G->q, &fp, &nbf, nev, &G->st32->done);
            if (rc) return rc;
            G->flex_part = fp;
            G->flex_nb = nbf;
        } else {
            HIP_TRY(launch_jacobi_z(G->g.n, G->r, G->dinv, G->dmask, G->z, G->stream));
            G->flex_part = nullptr;
        }
        if (!G->flex_part) {
            VecIO<float> f = v;
            f.partials = pf;
            HIP_TRY(launch_flex_dots_f32(G->g.n, f, G->nb_vec, G->stream));
        }
    }
    if (ev) HIP_TRY(hipEventRecord(ev[3], G->stream));
    return MFFV_OK;
}

// Start per-kernel timing for the next solve (events are created once per grid).
int timing_begin(mffv_grid* G, bool on) {
    G->timing = on;
    G->timed = 0;
    G->timed_real = -1;
    for (bool& u : G->tnev_used) u = false;
    if (!on || G->tev_made) return MFFV_OK;
    for (auto& row : G->tev)
        for (auto& e : row) HIP_TRY(hipEventCreate(&e));
    for (auto& row : G->tnev)
        for (auto& e : row) HIP_TRY(hipEventCreate(&e));
    G->tev_made = true;
    return MFFV_OK;
}

// Mean durations (us) of phase A, phase B and the preconditioner over the
// iterations that were timed; the stream must be synchronized.
int timing_end(mffv_grid* G, mffv_info* inf) {
    if (!G->timing) return MFFV_OK;
    // launches after convergence return at once: time only iterations that did work
    const int nt = G->timed_real >= 0 ? std::min(G->timed, G->timed_real) : G->timed;
    double sum[3] = {0, 0, 0};
    for (int t = 0; t < nt; ++t) {
        for (int k = 0; k < 3; ++k) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, G->tev[t][k], G->tev[t][k + 1]));
            sum[k] += ms;
        }
    }
    if (nt > 0) {
        inf->phase_a_us = 1e3 * sum[0] / nt;
        inf->phase_b_us = 1e3 * sum[1] / nt;
        inf->precond_us = 1e3 * sum[2] / nt;
    }
    inf->timed_iters = nt;
    double lsum[4] = {0, 0, 0, 0};
    int nn_t = 0;
    for (int t = 0; t < nt; ++t) {
        if (!G->tnev_used[t]) continue;
        for (int k = 0; k < 4; ++k) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, G->tnev[t][k], G->tnev[t][k + 1]));
            lsum[k] += ms;
        }
        ++nn_t;
    }
    for (int k = 0; k < 4; ++k) inf->nn_layer_us[k] = nn_t > 0 ? 1e3 * lsum[k] / nn_t : 0.0;
    inf->nn_timed = nn_t;
    G->timing = false;
    return MFFV_OK;
}

int enqueue_iter64(mffv_grid* G, int precond) {
    if (precond != MFFV_PRECOND_NONE) return fail(MFFV_EINVAL, "FP64 CG supports precond NONE only");
    StencilIO<double> a;
    a.src = G->r64;
    a.p0 = G->p064;
    a.p1 = G->p164;
    a.out = G->q64;
    a.xsol = G->x64;
    a.partials = G->partA;
    a.st = G->st64;
    a.pb = G->partB;
    a.nb_b = G->nb_vec;
    HIP_TRY(launch_stencil_f64(kFusedCg, G->g, coef_of(G), a, G->m64, G->stream));
    VecIO<double> v;
    v.r = G->r64;
    v.q = G->q64;
    v.dmask = G->dmask;
    v.partials = G->partB;
    v.pa = G->partA;
    v.nb_a = G->m64.blocks();
    v.st = G->st64;
    HIP_TRY(launch_phase_b_f64(kBPlain, G->g.n, v, G->nb_vec, G->stream));
    return MFFV_OK;
}

template <class F>
int enqueue_chunk(mffv_grid* G, CgGraph& graph, int chunk, bool use_graph, F&& one_iter,
                  const void* net = nullptr, int64_t net_gen = 0, float omega = 0.f) {
    if (use_graph) {
        if (graph.exec && (graph.chunk != chunk || graph.net != net || graph.net_gen != net_gen ||
                           graph.omega != omega)) {
            (void)hipGraphExecDestroy(graph.exec);
            graph.exec = nullptr;
        }
        if (!graph.exec) {
            HIP_TRY(hipStreamBeginCapture(G->stream, hipStreamCaptureModeThreadLocal));
            int rc = MFFV_OK;
            for (int t = 0; t < chunk && rc == MFFV_OK; ++t) rc = one_iter();
            hipGraph_t gr = nullptr;
            hipError_t e = hipStreamEndCapture(G->stream, &gr);
            if (rc) {
                if (gr) (void)hipGraphDestroy(gr);
                return rc;
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&graph.exec, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
            graph.chunk = chunk;
            graph.net = net;
            graph.net_gen = net_gen;
            graph.omega = omega;
        }
        HIP_TRY(hipGraphLaunch(graph.exec, G->stream));
        return MFFV_OK;
    }
    for (int t = 0; t < chunk; ++t) {
        int rc = one_iter();
        if (rc) return rc;
    }
    return MFFV_OK;
}

template <class real>
bool state_done(const CgState<real>& st) { return st.done != 0; }
bool state_done(const MergedState& st) { return st.s[0].done || st.s[1].done; }

// Run the CG loop until the device flag says stop: enqueue chunk c, copy the
// state to pinned memory behind it, then wait for the copy of chunk c-1.
template <class State, class F>
int drive_loop(mffv_grid* G, State* st, int max_iter, int chunk, CgGraph& graph, bool use_graph,
               F&& one_iter, const void* net = nullptr, int64_t net_gen = 0, float omega = 0.f) {
    static_assert(sizeof(State) <= 256, "state mirror too small");
    const int max_chunks = max_iter / chunk + 3;
    bool stop = false;
    for (int c = 0; c < max_chunks && !stop; ++c) {
        int rc = enqueue_chunk(G, graph, chunk, use_graph, one_iter, net, net_gen, omega);
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(G->hstate + 256 * (c & 1), st, sizeof(State),
                               hipMemcpyDeviceToHost, G->stream));
        HIP_TRY(hipEventRecord(G->ev[c & 1], G->stream));
        if (c >= 1) {
            HIP_TRY(hipEventSynchronize(G->ev[(c - 1) & 1]));
            const State* hs = reinterpret_cast<const State*>(G->hstate + 256 * ((c - 1) & 1));
            if (state_done(*hs)) stop = true;
        }
    }
    HIP_TRY(hipStreamSynchronize(G->stream));
    return MFFV_OK;
}

int ensure_merged(mffv_grid* G) {
    if (G->ms) return MFFV_OK;
    const size_t n = (size_t)G->g.n;
    int rc;
    if ((rc = dalloc(&G->r2, n)) || (rc = dalloc(&G->q2, n)) ||
        (rc = dalloc(&G->partM, 8 * (size_t)G->max_blocks)) || (rc = dalloc(&G->ms, 1))) {
        dfree(G->r2); dfree(G->q2); dfree(G->partM); dfree(G->ms);
        return rc;
    }
    return MFFV_OK;
}

// The single-reduction loop applies to plain FP32 CG on the float4 path.
bool merged_applies(const mffv_grid* G, int precond, const mffv_opts& o) {
    return o.single_reduction && precond == MFFV_PRECOND_NONE && G->m32.vec == 4;
}

// Enqueue kernel K of the single-reduction CG; K's parity is G->mpar. Buffers
// R[0] = r2, R[1] = r (r_0 from the initial residual), Q[0] = q2, Q[1] = q,
// P[0] = p0, P[1] = p1: kernel K reads index (K + 1) & 1 and writes K & 1.
int enqueue_merged(mffv_grid* G) {
    const int par = G->mpar;
    hipEvent_t* ev = nullptr;
    if (G->timing && G->timed < kTimedIters) ev = G->tev[G->timed++];
    if (ev) HIP_TRY(hipEventRecord(ev[0], G->stream));
    float* R[2] = {G->r2, G->r};
    float* Q[2] = {G->q2, G->q};
    float* Pv[2] = {G->p0, G->p1};
    const int nb = G->m32.blocks();
    float* part = reinterpret_cast<float*>(G->partM);
    StencilIO<float> a;
    a.src = R[par ^ 1];
    a.qin = Q[par ^ 1];
    a.pin = Pv[par ^ 1];
    a.rout = R[par];
    a.pout = Pv[par];
    a.out = Q[par];
    a.xsol = G->xw;
    a.partials = part + (size_t)par * 4 * nb;
    a.pf = part + (size_t)(par ^ 1) * 4 * nb;
    a.nb_f = nb;
    a.pb = reinterpret_cast<float*>(G->partB);
    a.nb_b = G->nb_vec;
    a.ms = G->ms;
    a.parity = par;
    HIP_TRY(launch_stencil_f32(kMergedCg, G->g, coef_of(G), a, G->m32, G->stream));
    if (ev) {
        HIP_TRY(hipEventRecord(ev[1], G->stream));
        HIP_TRY(hipEventRecord(ev[2], G->stream));
        HIP_TRY(hipEventRecord(ev[3], G->stream));
    }
    G->mpar ^= 1;
    return MFFV_OK;
}

// FP32 CG on the workspace: solves A xw = bw from the xw given.
int cg32(mffv_grid* G, double tol, int max_iter, int precond, const mffv_opts& o, LoopResult* out) {
    const mffv_net* net = o.net;
    if (precond == MFFV_PRECOND_LEARNED && !net)
        return fail(MFFV_EINVAL, "precond LEARNED needs opts.net");
    int net_gen = 0;
    if (precond == MFFV_PRECOND_LEARNED) {
        int rc = ensure_feature(G);
        if (rc) return rc;
        net_gen = nn_prepare(net, G->g.n);
        if (net_gen < 0) return net_gen;
    }
    HIP_TRY(launch_copy_dirichlet_f32(G->g.n, G->dmask, G->bw, G->xw, G->stream));
    {
        StencilIO<float> io;
        io.src = G->xw;
        io.out = G->r;
        io.rhs = G->bw;
        HIP_TRY(launch_stencil_f32(kResidual, G->g, coef_of(G), io, G->m32, G->stream));
    }
    float* pb = reinterpret_cast<float*>(G->partB);
    VecIO<float> v;
    v.r = G->r;
    v.z = G->z;
    v.dinv = G->dinv;
    v.jacobi = precond == MFFV_PRECOND_JACOBI ? 1 : 0;
    v.dinv_dot = precond == MFFV_PRECOND_LEARNED ? 1 : 0;
    v.dmask = G->dmask;
    v.b = G->bw;
    v.partials = pb;
    v.st = G->st32;
    v.tol2 = (float)(tol * tol);
    v.max_iter = max_iter;
    HIP_TRY(launch_phase_b_f32(kBInit, G->g.n, v, G->nb_vec, G->stream));
    if (merged_applies(G, precond, o)) {
        int rc = ensure_merged(G);
        if (rc) return rc;
        HIP_TRY(launch_merged_init(G->ms, (float)(tol * tol), max_iter, G->stream));
        G->mpar = 0;
        // an even chunk keeps every captured launch's parity right on replay
        const int chunk = std::max(2, (o.check_every + 1) & ~1);
        const bool use_graph = o.use_graph && !o.timing && G->stream != nullptr;
        rc = drive_loop(G, G->ms, max_iter + 1, chunk, G->graphM, use_graph,
                        [&]() { return enqueue_merged(G); });
        if (rc) return rc;
        MergedState hs;
        HIP_TRY(hipMemcpyAsync(&hs, G->ms, sizeof(hs), hipMemcpyDeviceToHost, G->stream));
        HIP_TRY(hipStreamSynchronize(G->stream));
        const MergedSlot& sl = hs.s[0].done ? hs.s[0] : hs.s[1];
        out->iters = sl.iters;
        out->status = (hs.s[0].done || hs.s[1].done) ? sl.status : MFFV_NOT_CONVERGED;
        out->fallbacks = 0;
        out->rel_rec = sl.bnorm2 > 0 ? std::sqrt((double)sl.rr / (double)sl.bnorm2) : 0.0;
        out->merged = true;
        if (G->timing && G->timed_real < 0) G->timed_real = sl.iters;
        return MFFV_OK;
    }
    if (precond == MFFV_PRECOND_LEARNED) {
        const float* fp = nullptr;
        int nbf = 0;
        int rc = nn_precondition(net, G->g, coef_of(G), G->m32, (float)o.nn_smooth, G->r, G->dinv, G->dmask,
                                 G->sqd, G->z, pb + G->nb_vec, G->nb_vec, G->feat, (float)G->n_unknown, G->stream,
                                 nullptr, &fp, &nbf);
        if (rc) return rc;
        G->flex_part = fp;
        G->flex_nb = nbf;
        if (!fp) {
            VecIO<float> f = v;
            f.partials = reinterpret_cast<float*>(G->partF);
            HIP_TRY(launch_flex_dots_f32(G->g.n, f, G->nb_vec, G->stream));
        }
    }
    const int nn_every = precond == MFFV_PRECOND_LEARNED ? std::max(1, o.nn_every) : 1;
    const float omega = precond == MFFV_PRECOND_LEARNED ? (float)o.nn_smooth : 0.f;
    // a chunk holding whole network periods keeps the captured pattern right on replay
    const int chunk = (std::max(1, o.check_every) + nn_every - 1) / nn_every * nn_every;
    const bool use_graph = o.use_graph && !o.timing && G->stream != nullptr;
    G->flex_count = 0;
    int rc = drive_loop(G, G->st32, max_iter, chunk, G->graph32[precond], use_graph,
                        [&]() { return enqueue_iter32(G, precond, net, nn_every, omega); },
                        precond == MFFV_PRECOND_LEARNED ? (const void*)net : nullptr,
                        (int64_t)net_gen * 64 + nn_every, omega);
    if (rc) return rc;
    HIP_TRY(launch_finalize_f32(G->g.n, G->xw, G->p0, G->p1, G->st32, G->stream));
    CgState<float> hs;
    HIP_TRY(hipMemcpyAsync(&hs, G->st32, sizeof(hs), hipMemcpyDeviceToHost, G->stream));
    HIP_TRY(hipStreamSynchronize(G->stream));
    out->iters = hs.iters;
    out->status = hs.done ? hs.status : MFFV_NOT_CONVERGED;
    out->fallbacks = hs.fallbacks;
    if (G->timing && G->timed_real < 0) G->timed_real = hs.iters;
    out->rel_rec = hs.bnorm2 > 0 ? std::sqrt((double)hs.rr / (double)hs.bnorm2) : 0.0;
    return MFFV_OK;
}

// FP64 CG on x64 with right-hand side b64.
int cg64(mffv_grid* G, double tol, int max_iter, const mffv_opts& o, LoopResult* out) {
    HIP_TRY(launch_copy_dirichlet_f64(G->g.n, G->dmask, G->b64, 1, G->x64, G->stream));
    {
        StencilIO<double> io;
        io.src = G->x64;
        io.out = G->r64;
        io.rhs = G->b64;
        io.rhs_f64 = 1;
        HIP_TRY(launch_stencil_f64(kResidual, G->g, coef_of(G), io, G->m64, G->stream));
    }
    VecIO<double> v;
    v.r = G->r64;
    v.dmask = G->dmask;
    v.b = G->b64;
    v.b_f64 = 1;
    v.partials = G->partB;
    v.st = G->st64;
    v.tol2 = tol * tol;
    v.max_iter = max_iter;
    HIP_TRY(launch_phase_b_f64(kBInit, G->g.n, v, G->nb_vec, G->stream));
    const int chunk = std::max(1, o.check_every);
    const bool use_graph = o.use_graph && G->stream != nullptr;
    int rc = drive_loop(G, G->st64, max_iter, chunk, G->graph64[0], use_graph,
                        [&]() { return enqueue_iter64(G, MFFV_PRECOND_NONE); });
    if (rc) return rc;
    HIP_TRY(launch_finalize_f64(G->g.n, G->x64, G->p064, G->p164, G->st64, G->stream));
    CgState<double> hs;
    HIP_TRY(hipMemcpyAsync(&hs, G->st64, sizeof(hs), hipMemcpyDeviceToHost, G->stream));
    HIP_TRY(hipStreamSynchronize(G->stream));
    out->iters = hs.iters;
    out->status = hs.done ? hs.status : MFFV_NOT_CONVERGED;
    out->rel_rec = hs.bnorm2 > 0 ? std::sqrt(hs.rr / hs.bnorm2) : 0.0;
    return MFFV_OK;
}

int status_code(int s) {
    if (s == 0) return MFFV_OK;
    if (s == 1) return MFFV_NOT_CONVERGED;
    if (s == -4) return fail(MFFV_EBREAKDOWN, "CG breakdown: p.Ap <= 0 or a non-finite scalar");
    return s;
}

mffv_opts resolve_opts(const mffv_opts* o) {
    mffv_opts r;
    mffv_default_opts(&r);
    if (o) {
        r = *o;
        if (!(r.tol > 0)) r.tol = 1e-6;
        if (r.max_iter <= 0) r.max_iter = 100000;
        if (!(r.inner_tol > 0)) r.inner_tol = 1e-6;
        if (r.max_outer <= 0) r.max_outer = 10;
        if (r.check_every <= 0) r.check_every = 16;
    }
    return r;
}

int validate_opts(const mffv_opts& o) {
    if (!std::isfinite(o.tol) || o.tol >= 1.0)
        return fail(MFFV_EINVAL, "opts.tol must be in (0, 1)");
    if (o.precision < MFFV_FP32 || o.precision > MFFV_FP32_IR)
        return fail(MFFV_EINVAL, "opts.precision must be MFFV_FP32, MFFV_FP64 or MFFV_FP32_IR");
    if (o.precond < MFFV_PRECOND_NONE || o.precond > MFFV_PRECOND_LEARNED)
        return fail(MFFV_EINVAL, "opts.precond out of range");
    if (o.precond == MFFV_PRECOND_LEARNED && !o.net)
        return fail(MFFV_EINVAL, "precond LEARNED needs opts.net");
    if (o.precision == MFFV_FP64 && o.precond != MFFV_PRECOND_NONE)
        return fail(MFFV_EINVAL, "FP64 CG supports precond NONE only");
    if (o.single_reduction != 0 && o.single_reduction != 1)
        return fail(MFFV_EINVAL, "opts.single_reduction must be 0 or 1");
    if (o.async != 0 && o.async != 1) return fail(MFFV_EINVAL, "opts.async must be 0 or 1");
    if (o.nn_every < 1 || o.nn_every > 64)
        return fail(MFFV_EINVAL, "opts.nn_every must be in [1, 64]");
    if (!(o.nn_smooth >= 0.0 && o.nn_smooth < 2.0))
        return fail(MFFV_EINVAL, "opts.nn_smooth must be in [0, 2)");
    return MFFV_OK;
}

// Refinement (Sec. precision policy): FP64 iterate G->x64 and right-hand side
// b; FP32 corrections. Fills info; leaves the refined field in x64.
int solve_ir(mffv_grid* G, const void* b, int b_f64, const mffv_opts& o, mffv_info* info) {
    int rc;
    if ((rc = ensure_ws32(G)) || (rc = ensure_x64(G))) return rc;
    HIP_TRY(launch_copy_dirichlet_f64(G->g.n, G->dmask, b, b_f64, G->x64, G->stream));
    int total = 0, steps = 0, fallbacks = 0;
    bool merged = false;
    double rel = 0, rec = 0;
    int status = MFFV_NOT_CONVERGED;
    for (int outer = 0;; ++outer) {
        if ((rc = true_residual_f64(G, b, b_f64, G->x64, G->rres))) return rc;
        double rn2 = 0;
        if ((rc = read_rel(G, &rel, &rn2))) return rc;
        if (!std::isfinite(rel)) {
            status = fail(MFFV_EBREAKDOWN, "non-finite residual in refinement");
            break;
        }
        if (rel <= o.tol) {
            status = MFFV_OK;
            break;
        }
        if (outer >= o.max_outer || total >= o.max_iter) break;
        // FP32 correction: A d = r / ||r||, to the reduction still needed
        const double inner = std::min(0.5, std::max(o.tol / rel, o.inner_tol));
        HIP_TRY(launch_scale_to_f32(G->g.n, G->rres, G->dscal + 1, G->bw, G->stream));
        HIP_TRY(launch_fill_f32(G->g.n, G->xw, 0.f, G->stream));
        LoopResult lr;
        if ((rc = cg32(G, inner, o.max_iter - total, o.precond, o, &lr))) return rc;
        total += lr.iters;
        fallbacks += lr.fallbacks;
        merged = merged || lr.merged;
        steps += 1;
        rec = lr.rel_rec * rel;
        if (lr.status < 0) {
            status = status_code(lr.status);
            break;
        }
        HIP_TRY(launch_axpy_f64_from_f32(G->g.n, G->dscal + 1, G->xw, G->x64, G->stream));
    }
    if (info) {
        info->iters = total;
        info->ir_steps = steps;
        info->fallbacks = fallbacks;
        info->rel_res_true = rel;
        info->rel_res_recursive = rec;
        info->single_reduction = merged ? 1 : 0;
    }
    return status;
}


// ---------------------------------------------------------------------------
// Batched solves: a plan per distinct argument set, holding the device-side
// descriptors and the captured graph [clear barriers -> persistent CG ->
// per-system FP64 true residuals]; later calls with the same arguments replay
// the graph. Plans are dropped when one of their grids is destroyed.
// ---------------------------------------------------------------------------
struct BatchPlan {
    std::vector<mffv_grid*> grids;
    std::vector<const float*> b;
    std::vector<float*> x;
    int precond = 0, max_iter = 0, blocks_per_cu = 0, items_per_block = 4;
    int merged = 0;  // single-reduction iteration
    int max_outer = 0;  // refinement passes (MFFV_FP32_IR), 0 for MFFV_FP32
    double inner_tol = 0;
    double watchdog_s = 2.0;
    double tol = 0;
    void* dbuf = nullptr;
    BatchSys* dsys = nullptr;
    int* dblock_sys = nullptr;
    unsigned* dbars = nullptr;
    BatchResult* dres = nullptr;
    int* derr = nullptr;
    int nblocks = 0;
    BatchRun run{};
    hipGraphExec_t exec = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<int> blocks;   // per system
    size_t o_part = 0, o_p64 = 0;  // offsets of the partial-sum arrays in dbuf
};

std::mutex g_plans_mu;
int g_batch_bpc = 0;  // blocks per CU of the batched kernel (0 = occupancy limit)
int g_batch_ipb = 4;  // work items per block of the batched kernel
double g_batch_watchdog_s = 2.0;  // limit of one per-system wait of the batched kernel
int g_batch_rebalance = 1;         // block shares follow the previous solve's iteration counts

int batch_blocks_per_cu_override() { return g_batch_bpc; }
std::vector<BatchPlan*> g_plans;

void free_plan(BatchPlan* P) {
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->dbuf) (void)hipFree(P->dbuf);
    if (P->e0) (void)hipEventDestroy(P->e0);
    if (P->e1) (void)hipEventDestroy(P->e1);
    delete P;
}

void drop_plans_with(const mffv_grid* G) {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    for (auto it = g_plans.begin(); it != g_plans.end();) {
        if (std::find((*it)->grids.begin(), (*it)->grids.end(), G) != (*it)->grids.end()) {
            free_plan(*it);
            it = g_plans.erase(it);
        } else {
            ++it;
        }
    }
}

// Blocks per system in proportion to its work, estimated as cells times the
// grid's extent (CG iterations grow with the extent).
// Blocks of each system in proportion to its expected work w[s] (at least
// one each; the remainder goes, block by block, to the system with the most
// work per block).
std::vector<int> share_blocks(const std::vector<double>& w, int total) {
    const int ns = (int)w.size();
    double sw = 0;
    for (double v : w) sw += v;
    std::vector<int> B(ns);
    int sum = 0;
    for (int s = 0; s < ns; ++s) {
        B[s] = std::max(1, (int)std::floor(total * w[s] / sw));
        sum += B[s];
    }
    while (sum > total) {
        int j = -1;
        for (int s = 0; s < ns; ++s)
            if (B[s] > 1 && (j < 0 || w[s] / B[s] < w[j] / B[j])) j = s;
        if (j < 0) break;
        --B[j];
        --sum;
    }
    while (sum < total) {
        int j = 0;
        for (int s = 1; s < ns; ++s)
            if (w[s] / B[s] > w[j] / B[j]) j = s;
        ++B[j];
        ++sum;
    }
    return B;
}

// Expected work of each system before any solve: cells x (nx + ny + nz), CG
// iterations growing with the grid's extent.
std::vector<double> size_weights(const std::vector<mffv_grid*>& grids) {
    std::vector<double> w;
    for (mffv_grid* G : grids) w.push_back((double)G->g.n * (double)(G->g.nx + G->g.ny + G->g.nz));
    return w;
}

// The per-system descriptors and the block map for block shares following
// the work weights w (the device buffer of the plan is already allocated; its
// size depends only on the total block count).
int fill_plan(BatchPlan* P, const std::vector<double>& w) {
    const int ns = (int)P->grids.size();
    const int total = P->nblocks;
    P->blocks = share_blocks(w, total);
    char* base = static_cast<char*>(P->dbuf);
    float* dpart = reinterpret_cast<float*>(base + P->o_part);
    double* dpart64 = reinterpret_cast<double*>(base + P->o_p64);
    std::vector<BatchSys> hs(ns);
    std::vector<int> map(total);
    int b0 = 0;
    for (int s = 0; s < ns; ++s) {
        mffv_grid* G = P->grids[s];
        BatchSys& S = hs[s];
        S.g = G->g;
        S.c = coef_of(G);
        S.cs = G->cdev;
        S.dinv = G->dinv;
        S.dmask = G->dmask;
        S.b = P->b[s];
        S.x = P->x[s];
        S.r = G->r;
        S.p0 = G->p0;
        S.p1 = G->p1;
        S.q = G->q;
        S.z = G->z;
        S.dx = G->xw;
        S.r2 = P->merged ? G->r2 : nullptr;
        S.q2 = P->merged ? G->q2 : nullptr;
        S.part = dpart + 8 * b0;
        S.part64 = dpart64 + 2 * b0;
        S.bar = P->dbars + 2 * s;
        S.xch = reinterpret_cast<unsigned long long*>(P->dbars + 2 * ns) + b0;
        S.res = P->dres + s;
        S.blk0 = b0;
        S.nblk = P->blocks[s];
        S.nchunk = (int)((G->g.plane + kThreads - 1) / kThreads);
        const int64_t ipb = std::max(1, P->items_per_block);
        const int64_t want = ((int64_t)S.nchunk * G->g.nx + ipb * S.nblk - 1) / (ipb * (int64_t)S.nblk);
        S.ci = (int)std::max<int64_t>(1, std::min<int64_t>(G->g.nx, want));
        S.nich = (G->g.nx + S.ci - 1) / S.ci;
        for (int t = 0; t < S.nblk; ++t) map[b0 + t] = s;
        b0 += S.nblk;
    }
    HIP_TRY(hipMemcpy(P->dsys, hs.data(), sizeof(BatchSys) * ns, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(P->dblock_sys, map.data(), sizeof(int) * total, hipMemcpyHostToDevice));
    return MFFV_OK;
}

int build_plan(BatchPlan* P, hipStream_t stream) {
    const int ns = (int)P->grids.size();
    int rc;
    // the batched kernel addresses a system's vectors with 32-bit byte offsets
    for (mffv_grid* G : P->grids)
        if (G->g.n >= (int64_t(1) << 30)) return fail(MFFV_EINVAL, "batched systems must have fewer than 2^30 cells");
    for (mffv_grid* G : P->grids) {
        if ((rc = ensure_ws32(G))) return rc;
        if (P->merged && (rc = ensure_merged(G))) return rc;
    }
    int dev = 0, cus = 0, rate_khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
    const int occ = batched_blocks_per_cu();
    if (occ <= 0) return fail(MFFV_EHIP, "occupancy query of the batched kernel failed");
    const int per_cu = P->blocks_per_cu > 0 ? std::min(P->blocks_per_cu, occ) : occ;
    const int total = per_cu * cus;
    if (ns > total)
        return fail(MFFV_EINVAL, "more systems than co-resident blocks (" + std::to_string(total) + ")");
    P->nblocks = total;
    // device buffer: descriptors, block map, partials, barriers, results
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~size_t(255); return o; };
    const size_t o_sys = take(sizeof(BatchSys) * ns), o_map = take(sizeof(int) * total),
                 o_part = take(sizeof(float) * 8 * total), o_bar = take(sizeof(unsigned) * (2 * (size_t)ns + 2 * (size_t)total)),
                 o_res = take(sizeof(BatchResult) * ns), o_p64 = take(sizeof(double) * 2 * total),
                 o_err = take(sizeof(int));
    HIP_TRY(hipMalloc(&P->dbuf, off));
    char* base = static_cast<char*>(P->dbuf);
    P->dsys = reinterpret_cast<BatchSys*>(base + o_sys);
    P->dblock_sys = reinterpret_cast<int*>(base + o_map);
    P->o_part = o_part;
    P->o_p64 = o_p64;
    P->dbars = reinterpret_cast<unsigned*>(base + o_bar);
    P->dres = reinterpret_cast<BatchResult*>(base + o_res);
    P->derr = reinterpret_cast<int*>(base + o_err);
    if ((rc = fill_plan(P, size_weights(P->grids)))) return rc;
    HIP_TRY(hipMemset(P->derr, 0, sizeof(int)));
    P->run.tol2 = (float)(P->tol * P->tol);
    P->run.max_iter = P->max_iter;
    P->run.precond = P->precond;
    P->run.merged = P->merged;
    P->run.max_outer = P->max_outer;
    P->run.tol = P->tol;
    P->run.inner_tol = P->inner_tol;
    // limit of one per-system wait, in wall-clock ticks (0: a wait not satisfied
    // at once fails)
    P->run.limit_ticks = (uint64_t)((double)rate_khz * 1000.0 * P->watchdog_s);
    P->run.err = P->derr;
    HIP_TRY(hipEventCreate(&P->e0));
    HIP_TRY(hipEventCreate(&P->e1));
    (void)stream;
    return MFFV_OK;
}

// Per-system results of an asynchronous batched solve, written into the
// caller's device array of mffv_info (the same fields the synchronous call
// fills on the host, without the timing).
__global__ void batch_info(int ns, const BatchResult* res, const int* err, int merged, mffv_info* out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    const BatchResult R = res[s];
    mffv_info I{};
    I.status = *err ? MFFV_EHIP
                    : (R.status == 0 ? MFFV_OK : (R.status == 1 ? MFFV_NOT_CONVERGED : MFFV_EBREAKDOWN));
    I.iters = R.iters;
    I.ir_steps = R.passes;
    I.rel_res_recursive = R.bnorm2 > 0.f ? sqrt((double)R.rr / (double)R.bnorm2) : 0.0;
    I.rel_res_true = R.bb64 > 0 ? sqrt(R.rr64 / R.bb64) : sqrt(R.rr64);
    I.single_reduction = merged;
    out[s] = I;
}

// Enqueue the whole batch: the persistent kernel, which also forms every
// system's FP64 true residual (and refines with MFFV_FP32_IR).
int enqueue_batch(BatchPlan* P, hipStream_t stream) {
    // barrier words of every system, then the 64-bit exchange slot of every block
    HIP_TRY(launch_batched_cg(P->dsys, P->dblock_sys, P->nblocks, P->dbars,
                              2 * (int)P->grids.size() + 2 * P->nblocks, P->derr, P->run, stream));
    return MFFV_OK;
}


// ---------------------------------------------------------------------------
// Autotuning of launch shapes. The single-system stencil kernels are tuned by
// timing the apply for every march plan (planes per block x XCD-aware order)
// on the grid itself; every candidate's output must equal the default plan's
// bit for bit (each cell's arithmetic does not depend on the tiling). The
// choice is cached in a JSON file keyed by device architecture and shape.
// ---------------------------------------------------------------------------
std::string tune_key(const mffv_grid* G) {
    hipDeviceProp_t prop;
    std::string arch = "gfx";
    if (hipGetDeviceProperties(&prop, G->device) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    return arch + "/" + std::to_string(G->g.nx) + "x" + std::to_string(G->g.ny) + "x" +
           std::to_string(G->g.nz) + "/v" + std::to_string(G->m32.vec);
}

// A tuned launch: the shape of the CG kernels (chosen on the fused phase A)
// and the shape of the apply (chosen on the apply itself).
struct TuneRec {
    int ci = 0, remap = 1, seg = 0;
    int aci = 0, aremap = 1, aseg = 0;
    double apply_us = 0, pa_us = 0;
};

bool cache_lookup(const char* path, const std::string& key, TuneRec* t) {
    if (!path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    const std::string pat = "\"" + key + "\": {";
    while (std::fgets(line, sizeof(line), f)) {
        const char* p = std::strstr(line, pat.c_str());
        if (!p) continue;
        TuneRec r;
        if (std::sscanf(p + pat.size(),
                        " \"ci\": %d, \"remap\": %d, \"seg\": %d, \"apply_ci\": %d, \"apply_remap\": %d, "
                        "\"apply_seg\": %d, \"apply_us\": %lf, \"phase_a_us\": %lf",
                        &r.ci, &r.remap, &r.seg, &r.aci, &r.aremap, &r.aseg, &r.apply_us, &r.pa_us) == 8) {
            *t = r;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& key, const TuneRec& t) {
    if (!path) return;
    std::vector<std::string> lines;
    if (FILE* f = std::fopen(path, "r")) {
        char line[512];
        while (std::fgets(line, sizeof(line), f)) {
            std::string l(line);
            if (l.find("\": {") != std::string::npos && l.find("\"" + key + "\"") == std::string::npos) {
                while (!l.empty() && (l.back() == '\n' || l.back() == ',')) l.pop_back();
                lines.push_back(l);
            }
        }
        std::fclose(f);
    }
    char buf[512];
    std::snprintf(buf, sizeof(buf),
                  "  \"%s\": {\"ci\": %d, \"remap\": %d, \"seg\": %d, \"apply_ci\": %d, \"apply_remap\": %d, "
                  "\"apply_seg\": %d, \"apply_us\": %.3f, \"phase_a_us\": %.3f}",
                  key.c_str(), t.ci, t.remap, t.seg, t.aci, t.aremap, t.aseg, t.apply_us, t.pa_us);
    lines.push_back(buf);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    for (size_t i = 0; i < lines.size(); ++i)
        std::fprintf(f, "%s%s\n", lines[i].c_str(), i + 1 < lines.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

}  // namespace

extern "C" {

const char* mffv_version(void) { return "mffv 1.0 gfx950"; }

const char* mffv_last_error(void) { return g_last_error.c_str(); }

void mffv_default_opts(mffv_opts* o) {
    if (!o) return;
    o->tol = 1e-6;
    o->max_iter = 100000;
    o->precision = MFFV_FP32;
    o->precond = MFFV_PRECOND_NONE;
    o->inner_tol = 1e-6;
    o->max_outer = 10;
    o->check_every = 16;
    o->use_graph = 1;
    o->net = nullptr;
    o->timing = 0;
    o->async = 0;
    o->single_reduction = 0;
    o->nn_every = 1;
    o->nn_smooth = 0.5;
}

namespace {
// Coefficient arrays, partial sums, events and the pinned state mirror of a
// grid whose sizes (g, max_blocks, nb_vec) are set; cartesian: also the face
// arrays of the stencil kernels.
int alloc_grid(mffv_grid* G, bool cartesian) {
    const size_t n = (size_t)G->g.n;
    int rc;
    if ((rc = dalloc(&G->a, n)) || (rc = dalloc(&G->a64, n)) ||
        (cartesian && ((rc = dalloc(&G->tx, n)) || (rc = dalloc(&G->ty, n)) || (rc = dalloc(&G->tz, n)))) ||
        (rc = dalloc(&G->dinv, n)) || (rc = dalloc(&G->dmask, n)) ||
        (rc = dalloc(&G->flags, 8)) || (rc = dalloc(&G->cdev, 1)) ||
        (rc = dalloc(&G->partA, (size_t)G->max_blocks)) ||
        (rc = dalloc(&G->partB, 3 * (size_t)G->nb_vec)) ||
        (rc = dalloc(&G->partF, 4 * (size_t)G->nb_vec)) ||
        (rc = dalloc(&G->partR, (size_t)std::max(G->max_blocks, 1024))) || (rc = dalloc(&G->dscal, 8)))
        return rc;
    hipError_t e;
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&G->hstate), 512, 0)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&G->ev[0], hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&G->ev[1], hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreate(&G->t0)) != hipSuccess || (e = hipEventCreate(&G->t1)) != hipSuccess ||
        (e = hipStreamSynchronize(G->stream)) != hipSuccess)
        return hip_fail(e, "grid set-up");
    return MFFV_OK;
}
}  // namespace

int mffv_create_grid(int nx, int ny, int nz, void* stream, mffv_grid** out) {
    if (!out) return fail(MFFV_EINVAL, "out is NULL");
    if (nx < 3 || ny < 1 || nz < 1)
        return fail(MFFV_EINVAL, "grid needs nx >= 3, ny >= 1, nz >= 1");
    const int64_t n = (int64_t)nx * ny * nz;
    if (n >= (int64_t(1) << 31)) return fail(MFFV_EINVAL, "grid has 2^31 cells or more");
    mffv_grid* G = new (std::nothrow) mffv_grid();
    if (!G) return fail(MFFV_ENOMEM, "host allocation failed");
    G->g = Geom{nx, ny, nz, n, (int64_t)ny * nz};
    G->stream = static_cast<hipStream_t>(stream);
    int rc = MFFV_OK;
    hipError_t e = hipGetDevice(&G->device);
    if (e != hipSuccess) {
        delete G;
        return hip_fail(e, "hipGetDevice");
    }
    const int vec = (nz % 4 == 0) ? 4 : 1;
    G->m32 = plan_march(G->g, vec, 0, 1);
    G->m_apply = G->m32;
    G->m64 = plan_march(G->g, 1, 0, 1);
    G->nb_vec = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n / 4 + kThreads - 1) / kThreads));
    // partial sums for any launch shape mffv_set_launch accepts, up to 2^18 blocks
    int64_t worst = 0;
    for (int sg = -1; sg <= kThreads * 4; sg = sg < 16 ? 16 : 2 * sg) {
        if (sg > 0 && !march_seg_ok(G->g, vec, sg)) continue;
        const March m1 = plan_march(G->g, vec, 1, 1, sg);
        worst = std::max<int64_t>(worst, (int64_t)m1.nchunk * m1.nich);
    }
    const March m1 = plan_march(G->g, 1, 1, 1);
    worst = std::max<int64_t>(worst, (int64_t)m1.nchunk * m1.nich);
    G->max_blocks = std::max({G->m32.blocks(), G->m64.blocks(), G->nb_vec,
                              (int)std::min<int64_t>(worst, 1 << 18)});
    if ((rc = alloc_grid(G, !G->faces))) {
        mffv_destroy_grid(G);
        return rc;
    }
    *out = G;
    return MFFV_OK;
}

int mffv_face_order(int n, int nfaces, const int* face_k, const int* face_l, int* new_index) {
    if (n < 1 || nfaces < 0 || !new_index) return fail(MFFV_EINVAL, "face order needs n >= 1, nfaces >= 0, new_index");
    if (nfaces > 0 && (!face_k || !face_l)) return fail(MFFV_EINVAL, "face_k and face_l must be host arrays");
    if ((int64_t)nfaces * 2 >= (int64_t(1) << 31)) return fail(MFFV_EINVAL, "2^30 faces or more");
    // adjacency of the cell graph
    std::vector<int> rp((size_t)n + 1, 0);
    for (int f = 0; f < nfaces; ++f) {
        const int k = face_k[f], l = face_l[f];
        if (k < 0 || k >= n || l < 0 || l >= n || k == l)
            return fail(MFFV_EINVAL, "face " + std::to_string(f) + " must join two different cells in [0, n)");
        ++rp[(size_t)k + 1];
        ++rp[(size_t)l + 1];
    }
    for (int i = 0; i < n; ++i) rp[(size_t)i + 1] += rp[i];
    std::vector<int> adj((size_t)2 * nfaces), fill(rp.begin(), rp.end() - 1);
    for (int f = 0; f < nfaces; ++f) {
        adj[fill[face_k[f]]++] = face_l[f];
        adj[fill[face_l[f]]++] = face_k[f];
    }
    std::vector<int> dg((size_t)n);
    for (int v = 0; v < n; ++v) dg[v] = rp[(size_t)v + 1] - rp[v];
    // each cell's neighbours by increasing degree (ties by index), as
    // Cuthill-McKee visits them
    for (int v = 0; v < n; ++v)
        std::sort(adj.begin() + rp[v], adj.begin() + rp[(size_t)v + 1], [&](int a, int b) {
            return dg[a] != dg[b] ? dg[a] < dg[b] : a < b;
        });
    std::vector<int> order;
    order.reserve((size_t)n);
    // per cell: the breadth-first sweep that last reached it and its level
    // there; numbered cells (earlier components) are never reached again
    std::vector<int> stamp((size_t)n, 0), level((size_t)n, 0);
    int sweep_id = 0;
    std::vector<int> sweep;
    auto bfs = [&](int root) {
        ++sweep_id;
        sweep.clear();
        sweep.push_back(root);
        stamp[root] = sweep_id;
        level[root] = 0;
        for (size_t h = 0; h < sweep.size(); ++h) {
            const int v = sweep[h];
            for (int e = rp[v]; e < rp[(size_t)v + 1]; ++e) {
                const int w = adj[e];
                if (stamp[w] == sweep_id) continue;
                stamp[w] = sweep_id;
                level[w] = level[v] + 1;
                sweep.push_back(w);
            }
        }
    };
    auto better = [&](int a, int b) { return dg[a] != dg[b] ? dg[a] < dg[b] : a < b; };
    std::vector<char> numbered((size_t)n, 0);
    for (int s0 = 0; s0 < n; ++s0) {
        if (numbered[s0]) continue;
        // start: the component's cell of minimum degree, moved once to a
        // minimum-degree cell of the last breadth-first level from it (a
        // pseudo-peripheral cell); the sweep from there is the order
        bfs(s0);
        int root = s0;
        for (int v : sweep)
            if (better(v, root)) root = v;
        bfs(root);
        int far = sweep.back();
        const int last = level[far];
        for (size_t h = sweep.size(); h-- > 0 && level[sweep[h]] == last;)
            if (better(sweep[h], far)) far = sweep[h];
        bfs(far);
        for (int v : sweep) {
            numbered[v] = 1;
            order.push_back(v);
        }
    }
    // reversed Cuthill-McKee order: the last visited cell gets index 0
    for (int i = 0; i < n; ++i) new_index[order[(size_t)n - 1 - i]] = i;
    return MFFV_OK;
}

int mffv_create_grid_faces(int n, int nfaces, const int* face_k, const int* face_l, void* stream,
                           mffv_grid** out) {
    if (!out) return fail(MFFV_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || nfaces < 0) return fail(MFFV_EINVAL, "a face-list grid needs n >= 1 and nfaces >= 0");
    if (nfaces > 0 && (!face_k || !face_l)) return fail(MFFV_EINVAL, "face_k and face_l must be host arrays");
    if ((int64_t)nfaces * 2 >= (int64_t(1) << 31)) return fail(MFFV_EINVAL, "2^30 faces or more");
    // rows on the host: each face appears in the rows of both its cells
    std::vector<int> rp((size_t)n + 1, 0);
    for (int f = 0; f < nfaces; ++f) {
        const int k = face_k[f], l = face_l[f];
        if (k < 0 || k >= n || l < 0 || l >= n || k == l)
            return fail(MFFV_EINVAL, "face " + std::to_string(f) + " must join two different cells in [0, n)");
        ++rp[(size_t)k + 1];
        ++rp[(size_t)l + 1];
    }
    for (int i = 0; i < n; ++i) rp[(size_t)i + 1] += rp[i];
    std::vector<int> rcol((size_t)2 * nfaces), ref((size_t)2 * nfaces), fill(rp.begin(), rp.end() - 1);
    for (int f = 0; f < nfaces; ++f) {
        const int k = face_k[f], l = face_l[f];
        rcol[fill[k]] = l;
        ref[fill[k]++] = f;
        rcol[fill[l]] = k;
        ref[fill[l]++] = f;
    }
    // sliced layout: kWave consecutive cells per slice, each slice as wide as
    // its longest row, entries column-major; padding points at the cell itself
    const int ns = (n + kWave - 1) / kWave;
    std::vector<int> sp((size_t)ns + 1, 0);
    for (int sl = 0; sl < ns; ++sl) {
        int w = 0;
        for (int K = sl * kWave; K < std::min(n, (sl + 1) * kWave); ++K) w = std::max(w, rp[K + 1] - rp[K]);
        if ((int64_t)sp[sl] + (int64_t)w * kWave >= (int64_t(1) << 31))
            return fail(MFFV_EINVAL, "face-list grid: too many entries after slicing (2^31)");
        sp[(size_t)sl + 1] = sp[sl] + w * kWave;
    }
    const size_t ne = (size_t)sp[ns];
    std::vector<int> col(ne), ef(ne, -1);
    for (int K = 0; K < n; ++K) {
        const int sl = K / kWave, lane = K % kWave;
        const int w = (sp[(size_t)sl + 1] - sp[sl]) / kWave;
        for (int j = 0; j < w; ++j) {
            const size_t e = (size_t)sp[sl] + (size_t)j * kWave + lane;
            const bool real = j < rp[K + 1] - rp[K];
            col[e] = real ? rcol[(size_t)rp[K] + j] : K;
            ef[e] = real ? ref[(size_t)rp[K] + j] : -1;
        }
    }
    mffv_grid* G = new (std::nothrow) mffv_grid();
    if (!G) return fail(MFFV_ENOMEM, "host allocation failed");
    G->faces = true;
    G->nfaces = nfaces;
    G->g = Geom{n, 1, 1, n, 1};
    G->stream = static_cast<hipStream_t>(stream);
    hipError_t e = hipGetDevice(&G->device);
    if (e != hipSuccess) {
        delete G;
        return hip_fail(e, "hipGetDevice");
    }
    // one thread per cell in a grid-stride loop
    const int nb = (int)std::min<int64_t>(8192, ((int64_t)n + kThreads - 1) / kThreads);
    G->m32 = March{1, 1, nb, 1, 0, 0, 0, 0};
    G->m_apply = G->m32;
    G->m64 = G->m32;
    G->nb_vec = (int)std::min<int64_t>(1024, std::max<int64_t>(1, ((int64_t)n / 4 + kThreads - 1) / kThreads));
    G->max_blocks = std::max(nb, G->nb_vec);
    int rc;
    if ((rc = alloc_grid(G, false)) || (rc = dalloc(&G->csr_sp, (size_t)ns + 1)) ||
        (ne && ((rc = dalloc(&G->csr_col, ne)) || (rc = dalloc(&G->csr_ef, ne)) || (rc = dalloc(&G->csr_val, ne))))) {
        mffv_destroy_grid(G);
        return rc;
    }
    if ((e = hipMemcpy(G->csr_sp, sp.data(), sp.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess ||
        (ne && (e = hipMemcpy(G->csr_col, col.data(), ne * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess) ||
        (ne && (e = hipMemcpy(G->csr_ef, ef.data(), ne * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)) {
        mffv_destroy_grid(G);
        return hip_fail(e, "face-list upload");
    }
    if (!G->csr_col) {
        // a grid without faces: the slice pointers are all 0 and no entry is read,
        // but the operator form needs non-NULL entry arrays
        if ((rc = dalloc(&G->csr_col, 1)) || (rc = dalloc(&G->csr_ef, 1)) || (rc = dalloc(&G->csr_val, 1))) {
            mffv_destroy_grid(G);
            return rc;
        }
    }
    *out = G;
    return MFFV_OK;
}

void mffv_destroy_grid(mffv_grid* G) {
    if (!G) return;
    drop_plans_with(G);
    (void)hipSetDevice(G->device);
    (void)hipStreamSynchronize(G->stream);
    drop_graphs(G);
    dfree(G->a); dfree(G->a64); dfree(G->tx); dfree(G->ty); dfree(G->tz); dfree(G->dinv); dfree(G->dmask);
    dfree(G->feat);
    dfree(G->sqd);
    dfree(G->flags); dfree(G->cdev); dfree(G->partA); dfree(G->partB); dfree(G->partF); dfree(G->partR);
    dfree(G->dscal);
    dfree(G->r); dfree(G->p0); dfree(G->p1); dfree(G->q); dfree(G->z); dfree(G->xw);
    dfree(G->bw); dfree(G->st32); dfree(G->step_rhs);
    dfree(G->csr_sp); dfree(G->csr_col); dfree(G->csr_ef); dfree(G->csr_val);
    dfree(G->r2); dfree(G->q2); dfree(G->partM); dfree(G->ms);
    dfree(G->r64); dfree(G->p064); dfree(G->p164); dfree(G->q64); dfree(G->x64); dfree(G->b64);
    dfree(G->rres); dfree(G->st64);
    if (G->hstate) (void)hipHostFree(G->hstate);
    for (auto& e : G->ev)
        if (e) (void)hipEventDestroy(e);
    if (G->t0) (void)hipEventDestroy(G->t0);
    if (G->t1) (void)hipEventDestroy(G->t1);
    for (auto& row : G->tev)
        for (auto& e : row)
            if (e) (void)hipEventDestroy(e);
    for (auto& row : G->tnev)
        for (auto& e : row)
            if (e) (void)hipEventDestroy(e);
    delete G;
}

int mffv_perm_to_trans(int nx, int ny, int nz, const double* k, double kz_ratio, float* tx,
                       float* ty, float* tz, void* stream) {
    if (!k || !tx || !ty || !tz) return fail(MFFV_EINVAL, "NULL array");
    if (nx < 1 || ny < 1 || nz < 1) return fail(MFFV_EINVAL, "bad grid shape");
    const int64_t n = (int64_t)nx * ny * nz;
    if (n >= (int64_t(1) << 31)) return fail(MFFV_EINVAL, "grid has 2^31 cells or more");
    if (!(kz_ratio > 0) || !std::isfinite(kz_ratio)) return fail(MFFV_EINVAL, "kz_ratio must be > 0");
    Geom g{nx, ny, nz, n, (int64_t)ny * nz};
    HIP_TRY(launch_perm_to_trans(g, k, kz_ratio, tx, ty, tz, static_cast<hipStream_t>(stream)));
    return MFFV_OK;
}

int mffv_set_transmissibility(mffv_grid* G, const float* tx, const float* ty, const float* tz,
                              const float* accum, float accum_scalar, const uint8_t* dmask,
                              const float* pD, float* b_out) {
    int rc = check_grid(G, false);
    if (rc || (rc = check_cartesian(G, "mffv_set_transmissibility (use mffv_set_face_transmissibility)")))
        return rc;
    if (!tx || !ty || !tz) return fail(MFFV_EINVAL, "tx, ty and tz must be device arrays");
    if (!accum && (!(accum_scalar >= 0.f) || !std::isfinite(accum_scalar)))
        return fail(MFFV_EINVAL, "accumulation must be finite and >= 0");
    if ((rc = set_device(G))) return rc;
    drop_graphs(G);
    G->has_coef = false;
    HIP_TRY(hipMemsetAsync(G->flags, 0, 8 * sizeof(int), G->stream));
    SetupIn in{tx, ty, tz, accum, accum_scalar, dmask, pD};
    SetupOut out{G->a, G->a64, G->tx, G->ty, G->tz, G->dinv, G->dmask, b_out, G->flags};
    HIP_TRY(launch_setup(G->g, in, out, G->stream));
    int h[8];
    HIP_TRY(hipMemcpyAsync(h, G->flags, sizeof(h), hipMemcpyDeviceToHost, G->stream));
    HIP_TRY(hipStreamSynchronize(G->stream));
    if (h[0]) return fail(MFFV_EINVAL, "transmissibility negative or not finite");
    if (h[1]) return fail(MFFV_EINVAL, "accumulation negative or not finite");
    if (h[2]) return fail(MFFV_EINVAL, "Dirichlet pressure not finite");
    if (h[3] == 0 && !h[4])
        return fail(MFFV_EINVAL, "singular operator: no Dirichlet cell and zero accumulation");
    if (h[3] == G->g.n) return fail(MFFV_EINVAL, "every cell is a Dirichlet cell");
    G->n_unknown = G->g.n - h[3];
    G->feat_valid = false;
    // a scalar accumulation with the default x-plane Dirichlet set: the identity
    // coefficient is the accumulation itself on every plane not next to D
    G->a_uniform = accum == nullptr && dmask == nullptr;
    G->a_const = accum_scalar;
    if ((rc = store_coef_scalars(G))) return rc;
    G->has_coef = true;
    return MFFV_OK;
}

int mffv_set_face_transmissibility(mffv_grid* G, const float* T, const float* accum, float accum_scalar,
                                   const uint8_t* dmask, const float* pD, float* b_out) {
    int rc = check_grid(G, false);
    if (rc) return rc;
    if (!G->faces) return fail(MFFV_EINVAL, "mffv_set_face_transmissibility needs a face-list grid");
    if (!T && G->nfaces > 0) return fail(MFFV_EINVAL, "T must be a device array");
    if (!accum && (!(accum_scalar >= 0.f) || !std::isfinite(accum_scalar)))
        return fail(MFFV_EINVAL, "accumulation must be finite and >= 0");
    if ((rc = set_device(G))) return rc;
    drop_graphs(G);
    G->has_coef = false;
    HIP_TRY(hipMemsetAsync(G->flags, 0, 8 * sizeof(int), G->stream));
    CsrSetupIn in{G->csr_sp, G->csr_col, G->csr_ef, T, accum, accum_scalar, dmask, pD};
    SetupOut out{G->a, G->a64, nullptr, nullptr, nullptr, G->dinv, G->dmask, b_out, G->flags};
    HIP_TRY(launch_csr_setup(G->g.n, in, out, G->csr_val, G->stream));
    int h[8];
    HIP_TRY(hipMemcpyAsync(h, G->flags, sizeof(h), hipMemcpyDeviceToHost, G->stream));
    HIP_TRY(hipStreamSynchronize(G->stream));
    if (h[0]) return fail(MFFV_EINVAL, "transmissibility negative or not finite");
    if (h[1]) return fail(MFFV_EINVAL, "accumulation negative or not finite");
    if (h[2]) return fail(MFFV_EINVAL, "Dirichlet pressure not finite");
    if (h[3] == 0 && !h[4])
        return fail(MFFV_EINVAL, "singular operator: no Dirichlet cell and zero accumulation");
    if (h[3] == G->g.n) return fail(MFFV_EINVAL, "every cell is a Dirichlet cell");
    G->n_unknown = G->g.n - h[3];
    G->feat_valid = false;
    G->a_uniform = false;
    G->a_const = 0.f;
    if ((rc = store_coef_scalars(G))) return rc;
    G->has_coef = true;
    return MFFV_OK;
}

int mffv_apply(mffv_grid* G, const float* x, float* y) {
    int rc = check_grid(G, true);
    if (rc) return rc;
    if (!x || !y) return fail(MFFV_EINVAL, "NULL vector");
    if (x == y) return fail(MFFV_EINVAL, "x and y must not alias");
    if ((rc = set_device(G))) return rc;
    StencilIO<float> io;
    io.src = x;
    io.out = y;
    March m = G->m_apply;
    const bool aligned = ((uintptr_t)x % 16 == 0) && ((uintptr_t)y % 16 == 0);
    if (m.vec == 4 && !aligned) m = plan_march(G->g, 1, 0, 1);
    HIP_TRY(launch_stencil_f32(kApply, G->g, coef_of(G), io, m, G->stream));
    return MFFV_OK;
}

int mffv_apply_f64(mffv_grid* G, const double* x, double* y) {
    int rc = check_grid(G, true);
    if (rc) return rc;
    if (!x || !y) return fail(MFFV_EINVAL, "NULL vector");
    if (x == y) return fail(MFFV_EINVAL, "x and y must not alias");
    if ((rc = set_device(G))) return rc;
    StencilIO<double> io;
    io.src = x;
    io.out = y;
    HIP_TRY(launch_stencil_f64(kApply, G->g, coef_of(G), io, G->m64, G->stream));
    return MFFV_OK;
}

int mffv_true_residual(mffv_grid* G, const float* b, const double* x, double* r_out,
                       double* rel_out) {
    int rc = check_grid(G, true);
    if (rc) return rc;
    if (!b || !x || !rel_out) return fail(MFFV_EINVAL, "NULL argument");
    if ((rc = set_device(G)) || (rc = ensure_x64(G))) return rc;
    double* r = r_out ? r_out : G->rres;
    if ((rc = true_residual_f64(G, b, 0, x, r))) return rc;
    return read_rel(G, rel_out);
}

// ---------------------------------------------------------------------------
// The true residual without allocation: the two result norms and the
// per-block partial sums of its reductions live in a static device array
// (one per GPU, held until the process ends) instead of grid-owned memory.
// The array's host-side name is not a device address; its address on each
// device comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address is handed to kernels.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {
constexpr int kScratchHead = 32;                  // [0] ||b_U||^2, [1] ||r||^2, rest unused
constexpr int kScratchParts = 1 << 18;            // partial sums (one per block of a launch)
constexpr size_t kScratchDoubles = kScratchHead + kScratchParts;   // 2 MiB + 256 B
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (taken on the first call on it).
int scratch_on(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return fail(MFFV_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(MFFV_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[device] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[device];
    return MFFV_OK;
}
}  // namespace

extern "C" {

int mffv_true_residual_noalloc(mffv_grid* G, const float* b, const double* x, double* r_out,
                               double* rel_out) {
    int rc = check_grid(G, true);
    if (rc) return rc;
    if (!b || !x || !r_out || !rel_out) return fail(MFFV_EINVAL, "NULL argument (r_out is required)");
    if ((const void*)r_out == (const void*)x || (const void*)r_out == (const void*)b)
        return fail(MFFV_EINVAL, "r_out must not alias b or x");
    const int parts = std::max(G->m64.blocks(), G->nb_vec);
    if (parts > kScratchParts)
        return fail(MFFV_EINVAL, "grid needs " + std::to_string(parts) + " partial sums, more than the " +
                                     std::to_string(kScratchParts) + " of the no-allocation scratch");
    if ((rc = set_device(G))) return rc;
    double* sp = nullptr;
    if ((rc = scratch_on(G->device, &sp))) return rc;
    double* head = sp;
    double* part = sp + kScratchHead;
    StencilIO<double> io;
    io.src = x;
    io.out = r_out;
    io.rhs = b;
    io.rhs_f64 = 0;
    io.partials = part;
    HIP_TRY(launch_stencil_f64(kResidual, G->g, coef_of(G), io, G->m64, G->stream));
    HIP_TRY(launch_sum_partials(part, G->m64.blocks(), head + 1, G->stream));
    HIP_TRY(launch_masked_norm2(G->g.n, G->dmask, b, 0, part, head + 0, G->nb_vec, G->stream));
    double h[2];
    HIP_TRY(hipMemcpyAsync(h, head, sizeof(h), hipMemcpyDeviceToHost, G->stream));
    HIP_TRY(hipStreamSynchronize(G->stream));
    *rel_out = h[0] > 0 ? std::sqrt(h[1] / h[0]) : std::sqrt(h[1]);
    return MFFV_OK;
}

int mffv_cg_solve(mffv_grid* G, const float* b, float* x, const mffv_opts* opts, mffv_info* info) {
    int rc = check_grid(G, true);
    if (rc) return rc;
    if (!b || !x) return fail(MFFV_EINVAL, "NULL vector");
    if (b == x) return fail(MFFV_EINVAL, "b and x must not alias");
    mffv_opts o = resolve_opts(opts);
    if ((rc = validate_opts(o))) return rc;
    if (o.precond == MFFV_PRECOND_LEARNED && (rc = check_cartesian(G, "the learned preconditioner")))
        return rc;
    if (o.async) {
        // no host synchronisation: the whole solve runs in the persistent kernel
        if ((o.precision != MFFV_FP32 && o.precision != MFFV_FP32_IR) || o.precond == MFFV_PRECOND_LEARNED)
            return fail(MFFV_EINVAL, "opts.async needs precision MFFV_FP32 or MFFV_FP32_IR and precond NONE or "
                                     "JACOBI");
        mffv_grid* const gs[1] = {G};
        const float* const bs[1] = {b};
        float* const xs[1] = {x};
        return mffv_cg_solve_batched(gs, 1, bs, xs, &o, info);
    }
    if ((rc = set_device(G)) || (rc = ensure_ws32(G))) return rc;
    mffv_info inf{};
    const int64_t n = G->g.n;
    if ((rc = timing_begin(G, o.timing != 0 && o.precision != MFFV_FP64))) return rc;
    HIP_TRY(hipEventRecord(G->t0, G->stream));
    int status = MFFV_OK;
    if (o.precision == MFFV_FP32) {
        HIP_TRY(hipMemcpyAsync(G->bw, b, n * sizeof(float), hipMemcpyDeviceToDevice, G->stream));
        HIP_TRY(hipMemcpyAsync(G->xw, x, n * sizeof(float), hipMemcpyDeviceToDevice, G->stream));
        LoopResult lr;
        if ((rc = cg32(G, o.tol, o.max_iter, o.precond, o, &lr))) return rc;
        HIP_TRY(hipMemcpyAsync(x, G->xw, n * sizeof(float), hipMemcpyDeviceToDevice, G->stream));
        if ((rc = ensure_x64(G))) return rc;
        HIP_TRY(launch_convert_f32_to_f64(n, G->xw, G->x64, G->stream));
        if ((rc = true_residual_f64(G, b, 0, G->x64, G->rres))) return rc;
        if ((rc = read_rel(G, &inf.rel_res_true))) return rc;
        inf.iters = lr.iters;
        inf.ir_steps = 1;
        inf.fallbacks = lr.fallbacks;
        inf.rel_res_recursive = lr.rel_rec;
        inf.single_reduction = lr.merged ? 1 : 0;
        status = lr.status;
    } else if (o.precision == MFFV_FP32_IR) {
        if ((rc = ensure_x64(G))) return rc;
        HIP_TRY(launch_convert_f32_to_f64(n, x, G->x64, G->stream));
        status = solve_ir(G, b, 0, o, &inf);
        // a breakdown still reports its info (x: the last iterate); other errors return at once
        if (status < 0 && status != MFFV_EBREAKDOWN) return status;
        HIP_TRY(launch_convert_f64_to_f32(n, G->x64, x, G->stream));
    } else {
        if ((rc = ensure_ws64(G))) return rc;
        HIP_TRY(launch_convert_f32_to_f64(n, b, G->b64, G->stream));
        HIP_TRY(launch_convert_f32_to_f64(n, x, G->x64, G->stream));
        LoopResult lr;
        if ((rc = cg64(G, o.tol, o.max_iter, o, &lr))) return rc;
        HIP_TRY(launch_convert_f64_to_f32(n, G->x64, x, G->stream));
        if ((rc = true_residual_f64(G, G->b64, 1, G->x64, G->rres))) return rc;
        if ((rc = read_rel(G, &inf.rel_res_true))) return rc;
        inf.iters = lr.iters;
        inf.ir_steps = 1;
        inf.rel_res_recursive = lr.rel_rec;
        status = lr.status;
    }
    HIP_TRY(hipEventRecord(G->t1, G->stream));
    HIP_TRY(hipEventSynchronize(G->t1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, G->t0, G->t1));
    inf.ms = ms;
    if ((rc = timing_end(G, &inf))) return rc;
    status = status_code(status);
    inf.status = status;
    if (info) *info = inf;
    return status;
}

int mffv_cg_solve_f64(mffv_grid* G, const double* b, double* x, const mffv_opts* opts,
                      mffv_info* info) {
    int rc = check_grid(G, true);
    if (rc) return rc;
    if (!b || !x) return fail(MFFV_EINVAL, "NULL vector");
    if (b == x) return fail(MFFV_EINVAL, "b and x must not alias");
    mffv_opts o = resolve_opts(opts);
    if ((rc = validate_opts(o))) return rc;
    if (o.precision == MFFV_FP32)
        return fail(MFFV_EINVAL, "mffv_cg_solve_f64 needs precision MFFV_FP64 or MFFV_FP32_IR");
    if ((rc = set_device(G))) return rc;
    mffv_info inf{};
    const int64_t n = G->g.n;
    HIP_TRY(hipEventRecord(G->t0, G->stream));
    int status;
    if (o.precision == MFFV_FP32_IR) {
        if ((rc = ensure_x64(G))) return rc;
        HIP_TRY(hipMemcpyAsync(G->x64, x, n * sizeof(double), hipMemcpyDeviceToDevice, G->stream));
        status = solve_ir(G, b, 1, o, &inf);
        // a breakdown still reports its info (x: the last iterate); other errors return at once
        if (status < 0 && status != MFFV_EBREAKDOWN) return status;
        HIP_TRY(hipMemcpyAsync(x, G->x64, n * sizeof(double), hipMemcpyDeviceToDevice, G->stream));
    } else {
        if ((rc = ensure_ws64(G))) return rc;
        HIP_TRY(hipMemcpyAsync(G->b64, b, n * sizeof(double), hipMemcpyDeviceToDevice, G->stream));
        HIP_TRY(hipMemcpyAsync(G->x64, x, n * sizeof(double), hipMemcpyDeviceToDevice, G->stream));
        LoopResult lr;
        if ((rc = cg64(G, o.tol, o.max_iter, o, &lr))) return rc;
        HIP_TRY(hipMemcpyAsync(x, G->x64, n * sizeof(double), hipMemcpyDeviceToDevice, G->stream));
        if ((rc = true_residual_f64(G, b, 1, G->x64, G->rres))) return rc;
        if ((rc = read_rel(G, &inf.rel_res_true))) return rc;
        inf.iters = lr.iters;
        inf.ir_steps = 1;
        inf.rel_res_recursive = lr.rel_rec;
        status = lr.status;
    }
    HIP_TRY(hipEventRecord(G->t1, G->stream));
    HIP_TRY(hipEventSynchronize(G->t1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, G->t0, G->t1));
    inf.ms = ms;
    status = status_code(status);
    inf.status = status;
    if (info) *info = inf;
    return status;
}

int mffv_cg_solve_batched(mffv_grid* const* grids, int nsys, const float* const* b,
                          float* const* x, const mffv_opts* opts, mffv_info* info) {
    if (!grids || !b || !x || nsys <= 0) return fail(MFFV_EINVAL, "grids, b, x must be non-NULL and nsys > 0");
    for (int s = 0; s < nsys; ++s) {
        int rc = check_grid(grids[s], true);
        if (rc) return rc;
        if (!b[s] || !x[s]) return fail(MFFV_EINVAL, "NULL vector of system " + std::to_string(s));
        if ((const void*)b[s] == (const void*)x[s]) return fail(MFFV_EINVAL, "b and x must not alias");
        if ((rc = check_cartesian(grids[s], "mffv_cg_solve_batched"))) return rc;
        if (grids[s]->device != grids[0]->device || grids[s]->stream != grids[0]->stream)
            return fail(MFFV_EINVAL, "all grids of a batch must share device and stream");
        for (int t = 0; t < s; ++t)
            if (grids[t] == grids[s]) return fail(MFFV_EINVAL, "a grid appears twice in the batch");
    }
    mffv_opts o = resolve_opts(opts);
    int rc = validate_opts(o);
    if (rc) return rc;
    if (o.precision != MFFV_FP32 && o.precision != MFFV_FP32_IR)
        return fail(MFFV_EINVAL, "batched solves run in MFFV_FP32 or MFFV_FP32_IR");
    const int max_outer = o.precision == MFFV_FP32_IR ? std::max(1, o.max_outer) : 0;
    if (o.precond == MFFV_PRECOND_LEARNED)
        return fail(MFFV_EINVAL, "batched solves support precond NONE or JACOBI");
    if ((rc = set_device(grids[0]))) return rc;
    hipStream_t stream = grids[0]->stream;
    const int bpc = batch_blocks_per_cu_override();
    // the single-reduction iteration applies to plain CG
    const int merged = (o.single_reduction && o.precond == MFFV_PRECOND_NONE) ? 1 : 0;
    std::lock_guard<std::mutex> lk(g_plans_mu);
    BatchPlan* P = nullptr;
    for (BatchPlan* c : g_plans) {
        if ((int)c->grids.size() != nsys || c->precond != o.precond || c->tol != o.tol || c->merged != merged ||
            c->max_iter != o.max_iter || c->blocks_per_cu != bpc || c->items_per_block != g_batch_ipb ||
            c->watchdog_s != g_batch_watchdog_s || c->max_outer != max_outer || c->inner_tol != o.inner_tol)
            continue;
        bool same = true;
        for (int s = 0; s < nsys && same; ++s)
            same = c->grids[s] == grids[s] && c->b[s] == b[s] && c->x[s] == x[s];
        if (same) { P = c; break; }
    }
    if (!P) {
        // building a plan allocates, which stream capture does not allow
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (o.async && stream && hipStreamIsCapturing(stream, &cs) == hipSuccess &&
            cs != hipStreamCaptureStatusNone)
            return fail(MFFV_EINVAL, "the first batched solve with these arguments allocates its plan: make it "
                                     "outside stream capture");
        P = new BatchPlan();
        P->grids.assign(grids, grids + nsys);
        P->b.assign(b, b + nsys);
        P->x.assign(x, x + nsys);
        P->precond = o.precond;
        P->merged = merged;
        P->tol = o.tol;
        P->max_iter = o.max_iter;
        P->max_outer = max_outer;
        P->inner_tol = o.inner_tol;
        P->blocks_per_cu = bpc;
        P->items_per_block = g_batch_ipb;
        P->watchdog_s = g_batch_watchdog_s;
        if ((rc = build_plan(P, stream))) {
            free_plan(P);
            return rc;
        }
        if (g_plans.size() >= 4) {
            free_plan(g_plans.front());
            g_plans.erase(g_plans.begin());
        }
        g_plans.push_back(P);
    }
    if (o.async) {
        // capture-safe: kernels only, no host synchronisation; info is device memory
        if ((rc = enqueue_batch(P, stream))) return rc;
        if (info) {
            hipLaunchKernelGGL(batch_info, dim3((nsys + 255) / 256), dim3(256), 0, stream, nsys, P->dres,
                               P->derr, P->merged, info);
            HIP_TRY(hipGetLastError());
        }
        return MFFV_OK;
    }
    const bool use_graph = o.use_graph && stream != nullptr;
    if (use_graph && !P->exec) {
        HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        int erc = enqueue_batch(P, stream);
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(stream, &gr);
        if (erc) {
            if (gr) (void)hipGraphDestroy(gr);
            return erc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&P->exec, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    }
    HIP_TRY(hipEventRecord(P->e0, stream));
    if (use_graph) {
        HIP_TRY(hipGraphLaunch(P->exec, stream));
    } else if ((rc = enqueue_batch(P, stream))) {
        return rc;
    }
    HIP_TRY(hipEventRecord(P->e1, stream));
    HIP_TRY(hipEventSynchronize(P->e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, P->e0, P->e1));
    std::vector<BatchResult> res(nsys);
    int err = 0;
    HIP_TRY(hipMemcpy(res.data(), P->dres, sizeof(BatchResult) * nsys, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&err, P->derr, sizeof(int), hipMemcpyDeviceToHost));
    if (err) {
        HIP_TRY(hipMemset(P->derr, 0, sizeof(int)));
        return fail(MFFV_EHIP, "batched CG: a per-system wait (barrier or partial-sum exchange) exceeded the "
                                "watchdog limit (blocks not co-resident?)");
    }
    if (g_batch_rebalance) {
        // The systems' blocks advance together only within a system, so the
        // launch lasts as long as the slowest system: cells x iterations / blocks.
        // When shares in proportion to this solve's cells x iterations would
        // shorten that by more than 5 %, the next solve of the batch takes them
        // (its graph is captured again).
        std::vector<double> w(nsys);
        for (int s = 0; s < nsys; ++s) w[s] = (double)P->grids[s]->g.n * std::max(1, res[s].iters);
        auto span = [&](const std::vector<int>& B) {
            double m = 0;
            for (int s = 0; s < nsys; ++s) m = std::max(m, w[s] / B[s]);
            return m;
        };
        const std::vector<int> Bn = share_blocks(w, P->nblocks);
        if (span(Bn) < 0.95 * span(P->blocks)) {
            if ((rc = fill_plan(P, w))) return rc;
            if (P->exec) {
                (void)hipGraphExecDestroy(P->exec);
                P->exec = nullptr;
            }
        }
    }
    int status = MFFV_OK;
    for (int s = 0; s < nsys; ++s) {
        const BatchResult& R = res[s];
        const int st = R.status == 0 ? MFFV_OK : (R.status == 1 ? MFFV_NOT_CONVERGED : MFFV_EBREAKDOWN);
        if (st == MFFV_EBREAKDOWN) status = MFFV_EBREAKDOWN;
        else if (st == MFFV_NOT_CONVERGED && status == MFFV_OK) status = MFFV_NOT_CONVERGED;
        if (info) {
            mffv_info& I = info[s];
            I = mffv_info{};
            I.status = st;
            I.iters = R.iters;
            I.ir_steps = R.passes;
            I.rel_res_recursive = R.bnorm2 > 0 ? std::sqrt((double)R.rr / (double)R.bnorm2) : 0.0;
            I.rel_res_true = R.bb64 > 0 ? std::sqrt(R.rr64 / R.bb64) : std::sqrt(R.rr64);
            I.ms = ms;
            I.single_reduction = P->merged;
        }
    }
    if (status == MFFV_EBREAKDOWN) return fail(MFFV_EBREAKDOWN, "batched CG: breakdown in a system");
    return status;
}

// ---------------------------------------------------------------------------
// Backward-Euler time stepping with wells: each step forms its right-hand side
// from the previous pressure and solves with the previous pressure as the
// initial guess (for this linear residual, one Newton step; with
// MFFV_FP32_IR the FP64 refinement steps are the further Newton steps).
// ---------------------------------------------------------------------------
namespace {
int check_step_args(const float* b, const float* c, float c_scalar, const float* wi, const float* pw) {
    if (!b) return fail(MFFV_EINVAL, "b must be a device array");
    if (!wi != !pw) return fail(MFFV_EINVAL, "wi and pw must be given together");
    if (!c && (!(c_scalar >= 0.f) || !std::isfinite(c_scalar)))
        return fail(MFFV_EINVAL, "c_scalar must be finite and >= 0");
    return MFFV_OK;
}
StepRhsIn step_in(const mffv_grid* G, const float* b, const float* c, float c_scalar, const float* p_old,
                  const float* wi, const float* pw, const float* q) {
    return StepRhsIn{G->dmask, b, c, c_scalar, p_old, wi, pw, q};
}
}  // namespace

int mffv_step_rhs(mffv_grid* G, const float* b, const float* c, float c_scalar, const float* p_old,
                  const float* wi, const float* pw, const float* q, float* rhs) {
    int rc = check_grid(G, true);
    if (rc || (rc = check_step_args(b, c, c_scalar, wi, pw))) return rc;
    if (!p_old || !rhs) return fail(MFFV_EINVAL, "p_old and rhs must be device arrays");
    for (const float* in : {b, c, p_old, wi, pw, q})
        if (in == rhs) return fail(MFFV_EINVAL, "rhs must not alias an input");
    if ((rc = set_device(G))) return rc;
    HIP_TRY(launch_step_rhs(G->g.n, step_in(G, b, c, c_scalar, p_old, wi, pw, q), rhs, G->stream));
    return MFFV_OK;
}

int mffv_time_steps(mffv_grid* G, int nsteps, const float* b, const float* c, float c_scalar,
                    const float* wi, const float* pw, const float* q, float* p, const mffv_opts* opts,
                    mffv_info* info) {
    int rc = check_grid(G, true);
    if (rc || (rc = check_step_args(b, c, c_scalar, wi, pw))) return rc;
    if (!p) return fail(MFFV_EINVAL, "p must be a device array");
    if (nsteps < 0) return fail(MFFV_EINVAL, "nsteps must be >= 0");
    for (const float* in : {b, c, wi, pw, q})
        if (in == p) return fail(MFFV_EINVAL, "p must not alias an input");
    mffv_opts o = resolve_opts(opts);
    if ((rc = validate_opts(o))) return rc;
    if (o.async) return fail(MFFV_EINVAL, "time steps run synchronously (opts.async must be 0)");
    if (o.precision == MFFV_FP64) return fail(MFFV_EINVAL, "time steps solve in MFFV_FP32 or MFFV_FP32_IR");
    if ((rc = set_device(G))) return rc;
    if (!G->step_rhs && (rc = dalloc(&G->step_rhs, (size_t)G->g.n))) return rc;
    int status = MFFV_OK;
    for (int s = 0; s < nsteps; ++s) {
        HIP_TRY(launch_step_rhs(G->g.n, step_in(G, b, c, c_scalar, p, wi, pw, q), G->step_rhs, G->stream));
        mffv_info one{};
        rc = mffv_cg_solve(G, G->step_rhs, p, &o, &one);
        if (info) info[s] = one;
        if (rc < 0) return rc;
        if (rc == MFFV_NOT_CONVERGED) status = MFFV_NOT_CONVERGED;
    }
    return status;
}

int mffv_harvest_pair(mffv_grid* G, const float* b, const float* x, const double* x_star,
                      float* r_hat, float* target, float* scale) {
    int rc = check_grid(G, true);
    if (rc || (rc = check_cartesian(G, "mffv_harvest_pair"))) return rc;
    if (!b || !x || !x_star || !r_hat || !target) return fail(MFFV_EINVAL, "NULL array");
    if ((rc = set_device(G)) || (rc = ensure_ws32(G))) return rc;
    StencilIO<float> io;
    io.src = x;
    io.out = G->r;
    io.rhs = b;
    March m = G->m32;
    if (m.vec == 4 && (((uintptr_t)x | (uintptr_t)b) % 16)) m = plan_march(G->g, 1, 0, 1);
    HIP_TRY(launch_stencil_f32(kResidual, G->g, coef_of(G), io, m, G->stream));
    float* sdev = reinterpret_cast<float*>(G->dscal + 2);
    HIP_TRY(launch_harvest(G->g.n, G->r, x, x_star, G->dinv, G->dmask,
                           reinterpret_cast<float*>(G->partR), (float)G->n_unknown, r_hat, target,
                           sdev, G->stream));
    if (scale) {
        float h = 0.f;
        HIP_TRY(hipMemcpyAsync(&h, sdev, sizeof(float), hipMemcpyDeviceToHost, G->stream));
        HIP_TRY(hipStreamSynchronize(G->stream));
        *scale = h;
    }
    return MFFV_OK;
}

int mffv_nn_smooth_sample(mffv_grid* G, double omega, const float* r_hat, float* out) {
    int rc = check_grid(G, true);
    if (rc || (rc = check_cartesian(G, "mffv_nn_smooth_sample"))) return rc;
    if (!r_hat || !out) return fail(MFFV_EINVAL, "NULL array");
    if (!(omega >= 0.0 && omega < 2.0)) return fail(MFFV_EINVAL, "omega must lie in [0, 2)");
    if ((rc = set_device(G)) || (rc = ensure_ws32(G))) return rc;
    // r = D^1/2 r_hat, r1 = r - A (omega D^-1 r) (the first sweep's pass), out = D^-1/2 r1
    HIP_TRY(launch_scale_dsqrt(G->g.n, r_hat, G->dinv, G->dmask, +1, G->z, G->stream));
    StencilIO<float> io;
    io.src = G->z;
    io.dinv = G->dinv;
    io.omega = (float)omega;
    io.out = G->r;
    io.partials = reinterpret_cast<float*>(G->partR);
    HIP_TRY(launch_stencil_f32(kSweep1, G->g, coef_of(G), io, G->m_apply, G->stream));
    HIP_TRY(launch_scale_dsqrt(G->g.n, G->r, G->dinv, G->dmask, -1, out, G->stream));
    return MFFV_OK;
}

int mffv_nn_loss_grad(mffv_net* net, mffv_grid* G, const float* r_hat, const float* target,
                      double* loss) {
    int rc = check_grid(G, true);
    if (rc || (rc = check_cartesian(G, "the network"))) return rc;
    if (!net) return fail(MFFV_EINVAL, "network handle is NULL");
    if (!r_hat) return fail(MFFV_EINVAL, "r_hat is NULL");
    if ((rc = set_device(G)) || (rc = ensure_feature(G))) return rc;
    if ((rc = nn_loss(net, G->g, coef_of(G), G->m32, G->dinv, G->dmask, G->feat, r_hat, target, true,
                      G->stream)))
        return rc;
    if (loss) {
        HIP_TRY(hipMemcpyAsync(loss, nn_loss_ptr(net), sizeof(double), hipMemcpyDeviceToHost, G->stream));
        HIP_TRY(hipStreamSynchronize(G->stream));
    }
    return MFFV_OK;
}

int mffv_nn_train_step(mffv_net* net, mffv_grid* G, const float* r_hat, const float* target,
                       float lr, double* loss) {
    if (!(lr > 0.f) || !std::isfinite(lr)) return fail(MFFV_EINVAL, "learning rate must be > 0");
    int rc = mffv_nn_loss_grad(net, G, r_hat, target, nullptr);
    if (rc) return rc;
    if ((rc = nn_adam(net, lr, G->stream))) return rc;
    if (loss) {
        HIP_TRY(hipMemcpyAsync(loss, nn_loss_ptr(net), sizeof(double), hipMemcpyDeviceToHost, G->stream));
        HIP_TRY(hipStreamSynchronize(G->stream));
    }
    return MFFV_OK;
}

int mffv_grid_feature(mffv_grid* G, float* feat) {
    int rc = check_grid(G, true);
    if (rc || (rc = check_cartesian(G, "mffv_grid_feature"))) return rc;
    if (!feat) return fail(MFFV_EINVAL, "feat is NULL");
    if ((rc = set_device(G)) || (rc = ensure_feature(G))) return rc;
    HIP_TRY(hipMemcpyAsync(feat, G->feat, G->g.n * sizeof(float), hipMemcpyDeviceToDevice, G->stream));
    return MFFV_OK;
}

int mffv_set_launch(mffv_grid* G, int ci, int remap, int seg) {
    int rc = check_grid(G, false);
    if (rc || (rc = check_cartesian(G, "mffv_set_launch"))) return rc;
    if (ci < 0 || ci > 4096 || (remap != 0 && remap != 1))
        return fail(MFFV_EINVAL, "ci must be in [0, 4096] (0 = default) and remap 0 or 1");
    if (seg < -1 || (seg > 0 && !march_seg_ok(G->g, G->m32.vec, seg)))
        return fail(MFFV_EINVAL,
                    "seg must be 0 (default), -1 (flat chunks) or a power of two in [16, 1024] dividing nz "
                    "(float4 path only)");
    if ((rc = set_device(G))) return rc;
    HIP_TRY(hipStreamSynchronize(G->stream));
    const March m = plan_march(G->g, G->m32.vec, ci, remap, seg);
    if (m.blocks() > G->max_blocks)
        return fail(MFFV_EINVAL, "launch plan needs more blocks than the grid's partial buffers");
    drop_graphs(G);
    G->m32 = m;
    G->m_apply = m;
    return MFFV_OK;
}

}  // extern "C"

namespace {
// Apply a tuned record: the CG kernels' shape, then the apply's own.
int set_launches(mffv_grid* G, const TuneRec& t) {
    int rc = mffv_set_launch(G, t.ci, t.remap, t.seg);
    if (rc) return rc;
    if (t.aseg < -1 || (t.aseg > 0 && !march_seg_ok(G->g, G->m32.vec, t.aseg)) || t.aci < 1 || t.aci > 4096)
        return fail(MFFV_EINVAL, "autotune cache: invalid apply shape");
    const March m = plan_march(G->g, G->m32.vec, t.aci, t.aremap, t.aseg);
    if (m.blocks() > G->max_blocks) return fail(MFFV_EINVAL, "autotune cache: apply shape needs too many blocks");
    G->m_apply = m;
    return MFFV_OK;
}
}  // namespace

extern "C" {

int mffv_autotune(mffv_grid* G, const char* cache_path, mffv_tune_result* out) {
    int rc = check_grid(G, true);
    if (rc || (rc = check_cartesian(G, "mffv_autotune"))) return rc;
    if ((rc = set_device(G)) || (rc = ensure_ws32(G))) return rc;
    const std::string key = tune_key(G);
    TuneRec rec;
    int tried = 0;
    if (cache_lookup(cache_path, key, &rec)) {
        if ((rc = set_launches(G, rec))) return rc;
    } else {
        // input: the inverse diagonal (a varied, bounded field); reference output in
        // z, which the unpreconditioned timing solves below leave alone
        StencilIO<float> io;
        io.src = G->dinv;
        io.out = G->z;
        const March base = plan_march(G->g, G->m32.vec, 0, 1);
        HIP_TRY(launch_stencil_f32(kApply, G->g, coef_of(G), io, base, G->stream));
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        const March keep = G->m32;
        // time one shape: its apply (reps launches) and phase A over the first 32
        // iterations of a solve of A x = dinv; returns an error code
        auto time_shape = [&](const March& m, int reps, double* apply_us, double* pa_us, double* it_us) -> int {
            HIP_TRY(hipEventRecord(e0, G->stream));
            for (int t = 0; t < reps; ++t)
                HIP_TRY(launch_stencil_f32(kApply, G->g, coef_of(G), io, m, G->stream));
            HIP_TRY(hipEventRecord(e1, G->stream));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            *apply_us = 1e3 * ms / reps;
            G->m32 = m;
            HIP_TRY(hipMemcpyAsync(G->bw, G->dinv, G->g.n * sizeof(float), hipMemcpyDeviceToDevice,
                                   G->stream));
            HIP_TRY(hipMemsetAsync(G->xw, 0, G->g.n * sizeof(float), G->stream));
            mffv_opts o;
            mffv_default_opts(&o);
            o.use_graph = 0;
            o.timing = 1;
            int r = timing_begin(G, true);
            if (r) return r;
            LoopResult lr;
            r = cg32(G, 1e-30, 40, MFFV_PRECOND_NONE, o, &lr);
            G->m32 = keep;
            if (r) return r;
            mffv_info inf{};
            if ((r = timing_end(G, &inf))) return r;
            *pa_us = inf.timed_iters > 0 ? inf.phase_a_us : *apply_us;
            // the whole iteration: phase B's prologue sums one partial per
            // phase-A block, so the shape changes its cost too
            *it_us = inf.timed_iters > 0 ? inf.phase_a_us + inf.phase_b_us : *apply_us;
            return MFFV_OK;
        };
        struct Cand {
            March m;
            double apply_us, pa_us, it_us;
        };
        std::vector<Cand> cands;
        const int cis[] = {1, 2, 4, 8, 16, 32, 64};
        // chunk shapes: flat, and row segments of 32..256 cells (16..4 rows a
        // chunk) shorter than a row (a whole-row segment is the flat chunk)
        std::vector<int> segs{-1};
        for (int sg = 32; sg <= 256 && sg < G->g.nz; sg *= 2)
            if (march_seg_ok(G->g, G->m32.vec, sg)) segs.push_back(sg);
        for (int sg : segs)
        for (int c : cis) {
            if (c > G->g.nx) continue;
            for (int rm = 0; rm <= 1; ++rm) {
                const March m = plan_march(G->g, G->m32.vec, c, rm, sg);
                if (m.blocks() > G->max_blocks) continue;
                io.out = G->p0;
                HIP_TRY(launch_stencil_f32(kApply, G->g, coef_of(G), io, m, G->stream));
                // bitwise probe against the default shape's output, on the device
                HIP_TRY(hipMemsetAsync(G->flags + 5, 0, sizeof(int), G->stream));
                HIP_TRY(launch_differ(G->g.n, G->p0, G->z, G->flags + 5, G->stream));
                int differs = 0;
                HIP_TRY(hipMemcpyAsync(&differs, G->flags + 5, sizeof(int), hipMemcpyDeviceToHost, G->stream));
                HIP_TRY(hipStreamSynchronize(G->stream));
                if (differs) continue;
                Cand cd{m, 0, 0, 0};
                if ((rc = time_shape(m, 10, &cd.apply_us, &cd.pa_us, &cd.it_us))) return rc;
                cands.push_back(cd);
                ++tried;
            }
        }
        // timings of one pass move by a few per cent: the best few of each kind
        // are timed twice more and ranked by their fastest time
        auto refine = [&](bool by_apply) -> int {
            std::vector<size_t> idx(cands.size());
            for (size_t t = 0; t < idx.size(); ++t) idx[t] = t;
            std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
                return by_apply ? cands[x].apply_us < cands[y].apply_us : cands[x].it_us < cands[y].it_us;
            });
            idx.resize(std::min<size_t>(idx.size(), 4));
            double best = 1e30;
            for (size_t t : idx) {
                for (int rep = 0; rep < 2; ++rep) {
                    double a = 0, pa = 0, it = 0;
                    int r = time_shape(cands[t].m, 50, &a, &pa, &it);
                    if (r) return r;
                    cands[t].apply_us = std::min(cands[t].apply_us, a);
                    if (it < cands[t].it_us) {  // phase A of the fastest iteration
                        cands[t].it_us = it;
                        cands[t].pa_us = pa;
                    }
                }
                const double v = by_apply ? cands[t].apply_us : cands[t].it_us;
                if (v < best) {
                    best = v;
                    const March& m = cands[t].m;
                    const int sgv = m.seg > 0 ? m.seg : -1;
                    if (by_apply) {
                        rec.aci = m.ci;
                        rec.aremap = m.remap;
                        rec.aseg = sgv;
                        rec.apply_us = v;
                    } else {
                        rec.ci = m.ci;
                        rec.remap = m.remap;
                        rec.seg = sgv;
                        rec.pa_us = cands[t].pa_us;
                    }
                }
            }
            return MFFV_OK;
        };
        if (!cands.empty() && ((rc = refine(false)) || (rc = refine(true)))) return rc;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (!tried) return fail(MFFV_EHIP, "autotune: no candidate reproduced the reference apply");
        if ((rc = set_launches(G, rec))) return rc;
        cache_store(cache_path, key, rec);
    }
    if (out) {
        out->ci = G->m32.ci;
        out->remap = G->m32.remap;
        out->seg = G->m32.seg > 0 ? G->m32.seg : -1;
        out->vec = G->m32.vec;
        out->blocks = G->m32.blocks();
        out->apply_us = rec.apply_us;
        out->candidates = tried;
        out->phase_a_us = rec.pa_us;
        out->apply_ci = G->m_apply.ci;
        out->apply_remap = G->m_apply.remap;
        out->apply_seg = G->m_apply.seg > 0 ? G->m_apply.seg : -1;
        out->apply_blocks = G->m_apply.blocks();
    }
    return MFFV_OK;
}

int mffv_autotune_batched(mffv_grid* const* grids, int nsys, const float* const* b,
                          float* const* x, const mffv_opts* opts, int* blocks_per_cu,
                          int* items_per_block, double* best_ms) {
    if (!grids || !b || !x || nsys <= 0) return fail(MFFV_EINVAL, "grids, b, x must be non-NULL and nsys > 0");
    for (int s = 0; s < nsys; ++s) {
        int rc = check_grid(grids[s], true);
        if (!rc) rc = check_cartesian(grids[s], "mffv_autotune_batched");
        if (rc) return rc;
        if (!x[s]) return fail(MFFV_EINVAL, "NULL vector");
    }
    int rc = set_device(grids[0]);
    if (rc) return rc;
    hipStream_t stream = grids[0]->stream;
    // every timed solve starts from the caller's initial guess
    std::vector<float*> x0((size_t)nsys, nullptr);
    auto release = [&]() {
        for (float*& p : x0) dfree(p);
    };
    for (int s = 0; s < nsys; ++s) {
        if ((rc = dalloc(&x0[s], (size_t)grids[s]->g.n))) {
            release();
            return rc;
        }
        if (hipMemcpyAsync(x0[s], x[s], grids[s]->g.n * sizeof(float), hipMemcpyDeviceToDevice, stream) !=
            hipSuccess) {
            release();
            return fail(MFFV_EHIP, "autotune: saving the initial guess failed");
        }
    }
    auto restore = [&]() -> int {
        for (int s = 0; s < nsys; ++s)
            if (hipMemcpyAsync(x[s], x0[s], grids[s]->g.n * sizeof(float), hipMemcpyDeviceToDevice,
                               stream) != hipSuccess)
                return fail(MFFV_EHIP, "autotune: restoring the initial guess failed");
        return MFFV_OK;
    };
    const int bpcs[] = {1, 2, 3, 4, 0};
    const int ipbs[] = {1, 2, 4, 8, 16};
    double best = 1e30;
    int bb = 0, bi = 4;
    std::vector<mffv_info> info((size_t)nsys);
    for (int bpc : bpcs) {
        for (int ipb : ipbs) {
            if ((rc = mffv_set_batched_launch(bpc, ipb)) || (rc = restore())) break;
            rc = mffv_cg_solve_batched(grids, nsys, b, x, opts, info.data());  // builds the plan
            if (rc < 0 || (rc = restore())) break;
            rc = mffv_cg_solve_batched(grids, nsys, b, x, opts, info.data());  // timed
            if (rc < 0) break;
            rc = MFFV_OK;
            if (info[0].ms < best) {
                best = info[0].ms;
                bb = bpc;
                bi = ipb;
            }
        }
        if (rc < 0) break;
    }
    const int rrc = restore();
    (void)hipStreamSynchronize(stream);
    release();
    if (rc < 0) return rc;
    if (rrc) return rrc;
    if ((rc = mffv_set_batched_launch(bb, bi))) return rc;
    if (blocks_per_cu) *blocks_per_cu = bb;
    if (items_per_block) *items_per_block = bi;
    if (best_ms) *best_ms = best;
    return MFFV_OK;
}

int mffv_set_batched_launch(int blocks_per_cu, int items_per_block) {
    if (blocks_per_cu < 0 || blocks_per_cu > 64 || items_per_block < 1 || items_per_block > 64)
        return fail(MFFV_EINVAL, "blocks_per_cu in [0, 64] (0 = occupancy limit), items_per_block in [1, 64]");
    std::lock_guard<std::mutex> lk(g_plans_mu);
    g_batch_bpc = blocks_per_cu;
    g_batch_ipb = items_per_block;
    return MFFV_OK;
}

int mffv_set_batched_rebalance(int on) {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    g_batch_rebalance = on ? 1 : 0;
    return MFFV_OK;
}

int mffv_set_batched_watchdog(double seconds) {
    if (!(seconds >= 0.0 && seconds <= 3600.0))
        return fail(MFFV_EINVAL, "the batched watchdog limit must be in [0, 3600] seconds");
    std::lock_guard<std::mutex> lk(g_plans_mu);
    g_batch_watchdog_s = seconds;
    return MFFV_OK;
}

int mffv_stream_probe(const float* const* in, int nin, float* const* out, int nout, int64_t n,
                      void* stream) {
    if (!in || !out || nin < 1 || nin > kStreamProbeIn || nout < 1 || nout > kStreamProbeOut)
        return fail(MFFV_EINVAL, "stream probe: 1..8 input and 1..4 output arrays");
    if (n < 0 || n % 4) return fail(MFFV_EINVAL, "stream probe: n must be a multiple of 4");
    StreamProbeIO io{};
    io.nin = nin;
    io.nout = nout;
    for (int k = 0; k < nin; ++k) {
        if (!in[k] || (uintptr_t)in[k] % 16) return fail(MFFV_EINVAL, "stream probe: 16-byte aligned inputs");
        io.in[k] = in[k];
    }
    for (int j = 0; j < nout; ++j) {
        if (!out[j] || (uintptr_t)out[j] % 16) return fail(MFFV_EINVAL, "stream probe: 16-byte aligned outputs");
        for (int k = 0; k < nin; ++k)
            if ((const float*)out[j] == in[k]) return fail(MFFV_EINVAL, "stream probe: an output aliases an input");
        io.out[j] = out[j];
    }
    HIP_TRY(launch_stream_probe(n, io, static_cast<hipStream_t>(stream)));
    return MFFV_OK;
}

int mffv_copy_probe(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src) return fail(MFFV_EINVAL, "NULL pointer");
    if (bytes % 16 || (uintptr_t)dst % 16 || (uintptr_t)src % 16)
        return fail(MFFV_EINVAL, "copy probe needs 16-byte aligned pointers and sizes");
    HIP_TRY(launch_copy_probe(src, dst, bytes, static_cast<hipStream_t>(stream)));
    return MFFV_OK;
}

}  // extern "C"
