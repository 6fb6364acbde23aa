/*
 * mffv.h -- matrix-free finite-volume conjugate gradient on AMD MI355X (gfx950).
 *
 * The library solves the linear system of an implicit single-phase TPFA
 * finite-volume discretisation on a 3D Cartesian grid of unit cells
 * (Sai et al., "Matrix-Free Finite Volume Kernels on a Dataflow Architecture",
 * Sec. II-A, Eq. 3, 4 and 6, Alg. 1 and Alg. 2). The operator is never
 * assembled: each application reads the face transmissibilities and forms
 * T_KL (x_K - x_L) on the six face neighbours of every cell. The same
 * operator runs on face-list (unstructured) meshes (mffv_create_grid_faces),
 * and backward-Euler time steps with wells are solved one after another
 * (mffv_time_steps). Conventions below are stated for the Cartesian grid; a
 * face-list grid has n cells numbered by the caller and its faces in place of
 * tx, ty, tz.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Grid nx x ny x nz, cell (i, j, k), flat index l = (i*ny + j)*nz + k
 *   (z fastest, x slowest). n = nx*ny*nz cells.
 * - Face arrays have n entries: tx[l] is the face between (i,j,k) and
 *   (i+1,j,k), ty[l] between (i,j,k) and (i,j+1,k), tz[l] between (i,j,k) and
 *   (i,j,k+1). Entries on the last plane/row/column are ignored (no-flow).
 * - T = Upsilon * lambda (transmissibility times the constant mobility, Eq. 4).
 * - Dirichlet cells D (Eq. 3) are eliminated symmetrically: the solved operator
 *   on the unknown cells U is
 *       (A x)_K = c_K x_K + sum_{L adj K} T_KL (x_K - x_L),  x_L := 0 for L in D,
 *   i.e. minus the Jacobian of Eq. 6 plus an accumulation diagonal c >= 0;
 *   on D cells A is the identity. This full-grid operator is symmetric
 *   positive definite whenever D is non-empty or c > 0 somewhere.
 * - Right-hand side b: b_K = sum_{L in D} T_KL p^D_L on U and p^D_K on D.
 * - Relative residuals and all norms are taken over U only.
 * - Pointers named as device pointers must be device memory of the current
 *   HIP device (e.g. torch tensors); vectors are FP32 unless the name says
 *   f64. The caller owns every vector it passes. Inputs and outputs of one call
 *   must not alias unless stated.
 * - All GPU work is enqueued on the stream given to mffv_create_grid, in
 *   stream order. Calls that return results on the host synchronize that
 *   stream before returning.
 * - Return codes: MFFV_OK (0), MFFV_NOT_CONVERGED (1, a result: x holds the last
 *   iterate and info is filled) or a negative error. Argument errors are found
 *   before any GPU work is enqueued. No C++ exception crosses this interface.
 *   The message of the last error of the calling thread is returned by
 *   mffv_last_error(). A grid handle must not be used from two threads at once;
 *   distinct handles are independent.
 */
#ifndef MFFV_H
#define MFFV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MFFV_OK             0
#define MFFV_NOT_CONVERGED  1
#define MFFV_EINVAL        (-1)  /* bad argument: null, shape, non-finite or negative coefficient */
#define MFFV_ENOMEM        (-2)  /* device allocation failed */
#define MFFV_EHIP          (-3)  /* a HIP runtime call failed; message from hipGetErrorString */
#define MFFV_EBREAKDOWN    (-4)  /* p.Ap <= 0 or non-finite scalar inside CG */
#define MFFV_ESTATE        (-5)  /* call out of order, e.g. solve before coefficients are set */

typedef struct mffv_grid mffv_grid;

/* Arithmetic of a solve. */
enum {
    MFFV_FP32 = 0,     /* FP32 vectors, apply and dots; FP64 true residual reported  */
    MFFV_FP64 = 1,     /* FP64 vectors, apply and dots (coefficients upcast from FP32) */
    MFFV_FP32_IR = 2   /* FP32 CG corrections inside FP64 iterative refinement        */
};

/* Preconditioner of a solve. */
enum {
    MFFV_PRECOND_NONE = 0,     /* plain CG (Alg. 1)                                  */
    MFFV_PRECOND_JACOBI = 1,   /* z = r / diag(A)                                    */
    MFFV_PRECOND_LEARNED = 2   /* flexible CG with the 3D-conv network of opts.net   */
};

typedef struct mffv_net mffv_net;

typedef struct {
    double tol;          /* target relative residual ||b - A x|| / ||b|| over U (default 1e-6) */
    int max_iter;        /* cap on CG iterations summed over refinement steps (<= 0: 100000) */
    int precision;       /* MFFV_FP32 | MFFV_FP64 | MFFV_FP32_IR                              */
    int precond;         /* MFFV_PRECOND_*                                                    */
    double inner_tol;    /* FP32_IR: smallest relative reduction asked of one FP32 solve (1e-6) */
    int max_outer;       /* FP32_IR: cap on refinement steps (default 10)                     */
    int check_every;     /* iterations enqueued between host polls of the convergence flag (16) */
    int use_graph;       /* 1: replay a captured HIP graph of check_every iterations          */
    const mffv_net* net; /* network for MFFV_PRECOND_LEARNED                                  */
    int single_reduction; /* 1: plain FP32 CG on the four-cells-per-thread path (nz % 4 == 0,
                            16-byte aligned vectors) runs one kernel per iteration with a
                            single reduction phase (r.r of the next iteration from a
                            one-step recurrence on the exact r.r), and a batched plain-CG
                            solve runs one barrier per iteration; 0 (default): the
                            two-phase iteration, faster on one GPU                      */
    int nn_every;        /* MFFV_PRECOND_LEARNED: apply the network every nn_every-th
                            iteration (1 = every one, the default) and the Jacobi step
                            z = r / diag(A) in between; flexible CG accepts the varying
                            preconditioner (1..64)                                     */
    int timing;          /* 1 (mffv_cg_solve, FP32 or FP32_IR): time each kernel of the first
                            32 FP32 CG iterations with HIP events (no graph replay, same
                            arithmetic); means returned in mffv_info                      */
    int async;           /* 1: capture-safe, no host synchronisation. mffv_cg_solve_batched
                            (and mffv_cg_solve, which then runs the persistent solver on its
                            one system; precision MFFV_FP32 or MFFV_FP32_IR, precond NONE
                            or JACOBI) only
                            enqueue work on the stream; info, if not NULL, is a DEVICE
                            array (one mffv_info per system) written when the stream
                            reaches it, with status MFFV_EHIP if a wait of the persistent
                            kernel expired. The first call with a given set of arguments
                            allocates the solver's plan: under stream capture it returns
                            MFFV_EINVAL, so make it once outside capture.               */
    double nn_smooth;    /* MFFV_PRECOND_LEARNED: weight w of the damped Jacobi sweeps around
                            the network (default 0.5). For w > 0 the preconditioned residual
                            of r is z1 = w D^-1 r, r1 = r - A z1, z2 = z1 + D^-1 r1 + C(r1),
                            z = z2 + w D^-1 (r - A z2), where C is the network's correction
                            (see mffv_net_create); with the zero network this is a fixed SPD
                            polynomial preconditioner (for every w in (0, 4): the spectrum of
                            D^-1/2 A D^-1/2 lies in (0, 2)). 0: z = D^-1 r + C(r). In [0, 2). */
} mffv_opts;

typedef struct {
    int status;                /* MFFV_OK, MFFV_NOT_CONVERGED or a negative error            */
    int iters;                 /* CG iterations, summed over refinement steps                */
    int ir_steps;              /* FP32 correction solves in FP32_IR (1 = no refinement needed) */
    int fallbacks;             /* learned preconditioner: iterations that used Jacobi instead */
    double rel_res_recursive;  /* recursively updated residual at exit, relative            */
    double rel_res_true;       /* ||b - A x|| / ||b|| recomputed in FP64 on the GPU          */
    double ms;                 /* device time of the solve (HIP events on the grid's stream) */
    /* opts.timing: mean duration per launch, in microseconds, over timed_iters FP32
       iterations that did work (HIP events on the grid's stream): the fused phase A (direction
       update, apply, deferred solution update, p.Ap partials), phase B (residual
       update and its dots) and, for flexible CG, the network and its dots. */
    double phase_a_us;
    double phase_b_us;
    double precond_us;
    int timed_iters;
    int single_reduction;      /* 1 if the FP32 iterations ran the single-reduction loop
                                  (then phase_a_us is that one kernel, phase_b_us ~ 0) */
    /* opts.timing with the learned preconditioner: mean duration per launch, in
       microseconds, of each of the network's four convolution layers (HIP events
       on the grid's stream around each layer's launch) over the timed iterations
       that applied the network, and their count. */
    double nn_layer_us[4];
    int nn_timed;
} mffv_info;

/* Library version string, e.g. "mffv 1.0 gfx950". Never NULL. */
const char* mffv_version(void);

/* Message of the last error returned on the calling thread ("" if none). */
const char* mffv_last_error(void);

/* Fill *opts with the defaults listed in mffv_opts. */
void mffv_default_opts(mffv_opts* opts);

/*
 * Create a grid handle for an nx x ny x nz mesh (Sec. II-A, the 7-point
 * stencil of the TPFA scheme). Requires nx >= 3 (two Dirichlet planes and at
 * least one unknown plane), ny >= 1, nz >= 1 and n < 2^31. `stream` is a
 * hipStream_t (NULL = the default stream) on which all later work of this
 * handle is enqueued; the current HIP device at creation is the handle's
 * device. Allocates the coefficient arrays (about 21 bytes per cell); solver
 * workspace is allocated on first use. *out is set only on success.
 */
int mffv_create_grid(int nx, int ny, int nz, void* stream, mffv_grid** out);

/* Release the handle and all device memory it owns. NULL is a no-op. */
void mffv_destroy_grid(mffv_grid* grid);

/*
 * Face transmissibilities of unit cells from a cell permeability field
 * (Eq. 4: Upsilon accounts for geometry and permeability). Each face takes the
 * harmonic average of its two cells, 2 k_K k_L / (k_K + k_L), computed in FP64
 * and rounded once to FP32; z faces use kz_ratio * k. Faces beyond the domain
 * are written as 0. `k` (FP64, n entries) and tx/ty/tz (FP32, n entries each)
 * are device pointers in the flat layout. Enqueued on `stream`; does not
 * synchronize. Requires k > 0 and finite (not checked on the device).
 */
int mffv_perm_to_trans(int nx, int ny, int nz, const double* k, double kz_ratio,
                       float* tx, float* ty, float* tz, void* stream);

/*
 * Set the operator of a grid (Eq. 3, 4 and 6 with the accumulation diagonal).
 *   tx, ty, tz   device FP32 face transmissibilities, n each, >= 0 and finite.
 *   accum        device FP32 per-cell accumulation c (n entries, >= 0), or NULL
 *                to use accum_scalar for every cell.
 *   dmask        device uint8 Dirichlet mask (n entries, nonzero = Dirichlet),
 *                or NULL for the planes i = 0 and i = nx-1.
 *   pD           device FP32 Dirichlet pressures (n entries, read on D only),
 *                or NULL for 1 on i = 0 and 0 on i = nx-1.
 *   b_out        device FP32 (n entries) receiving the right-hand side b, or NULL.
 * The library copies what it needs into memory owned by the handle (faces that
 * touch a Dirichlet cell are zeroed in that copy); the caller may free its
 * arrays afterwards. Validates the inputs on the device and synchronizes the
 * stream: returns MFFV_EINVAL for negative or non-finite T or c, non-finite
 * pD, or a singular operator (no Dirichlet cell and c = 0 everywhere).
 */
int mffv_set_transmissibility(mffv_grid* grid, const float* tx, const float* ty, const float* tz,
                              const float* accum, float accum_scalar, const uint8_t* dmask,
                              const float* pD, float* b_out);

/*
 * Face-list (unstructured) grids: the TPFA operator of Eq. 3-4 on any mesh
 * given as cells and faces, the generalisation the paper names as future
 * work (Sec. VI). Face f joins cells face_k[f] and face_l[f]; the operator on
 * an unknown cell K is c_K p_K + sum over K's faces of T_f (p_K - p_L), with
 * the same Dirichlet elimination as on the Cartesian grid.
 *
 * mffv_create_grid_faces: n >= 1 cells (n < 2^31), nfaces >= 0 faces (fewer
 * than 2^30) as HOST int arrays (copied; two different cells in [0, n) per
 * face; repeated pairs add up). The handle works with mffv_apply,
 * mffv_apply_f64, mffv_true_residual, mffv_cg_solve (FP32, FP32_IR; precond
 * NONE or JACOBI; the two-phase iteration), mffv_cg_solve_f64 and the time
 * steps. The entry points that need the Cartesian structure (launch shapes,
 * the network, batched solves) return MFFV_EINVAL for it.
 *
 * mffv_set_face_transmissibility: T is a device FP32 array of nfaces
 * (T_f = Upsilon_f lambda_f >= 0, finite), accum/accum_scalar the
 * accumulation as in mffv_set_transmissibility, dmask a device uint8 array of
 * n (NULL: no Dirichlet cell), pD device FP32 Dirichlet values (NULL: 0), b_out
 * (device, may be NULL) receives the right-hand side. Synchronizes the stream.
 * Errors as mffv_set_transmissibility; MFFV_EINVAL on a Cartesian handle.
 */
int mffv_create_grid_faces(int n, int nfaces, const int* face_k, const int* face_l, void* stream,
                           mffv_grid** out);

/*
 * A locality-preserving numbering of a face-list mesh (host only, no device
 * work): reverse Cuthill-McKee (breadth-first from a pseudo-peripheral cell
 * of each connected component, neighbours by increasing degree, the whole
 * order reversed). new_index (host, n ints) receives the new number of every
 * cell, a permutation of [0, n). Renumbering the mesh with it before
 * mffv_create_grid_faces keeps neighbouring cells close in memory, which the
 * face-list kernels' neighbour gathers need. Faces as for
 * mffv_create_grid_faces. Errors: MFFV_EINVAL.
 */
int mffv_face_order(int n, int nfaces, const int* face_k, const int* face_l, int* new_index);
int mffv_set_face_transmissibility(mffv_grid* grid, const float* T, const float* accum,
                                   float accum_scalar, const uint8_t* dmask, const float* pD,
                                   float* b_out);

/*
 * y = A x on the full grid (Eq. 6 / Alg. 2 with the sign of the Jacobian flipped
 * and the accumulation added; identity on Dirichlet cells). x and y are device
 * FP32 vectors of n entries and must not alias. Enqueued; does not synchronize.
 */
int mffv_apply(mffv_grid* grid, const float* x, float* y);

/* As mffv_apply with FP64 vectors; the FP32 coefficients are upcast exactly. */
int mffv_apply_f64(mffv_grid* grid, const double* x, double* y);

/*
 * FP64 true residual r = b - A x over U (0 on D) and its relative norm
 * ||r|| / ||b_U|| (Eq. 3 evaluated at x, sign flipped). b (FP32) and x (FP64)
 * are device vectors; r_out (FP64 device, n entries) may be NULL.
 * Synchronizes the stream to return *rel_out.
 */
int mffv_true_residual(mffv_grid* grid, const float* b, const double* x, double* r_out,
                       double* rel_out);

/*
 * For callers that cannot allocate device memory (serving loops, harnesses
 * that forbid allocation once set up): mffv_true_residual without any
 * allocation. r_out (FP64 device, n entries) is required here. The two norms
 * and the per-block partial sums of the reductions live in a static device
 * array of 2 MiB + 256 B that each GPU holds until the process ends (taken on
 * the first call on that GPU); a grid whose residual launch needs more than
 * 2^18 partial sums returns MFFV_EINVAL. Every call on one GPU shares that
 * array, so calls that overlap on one GPU (other streams or threads) race.
 * Same result bits as mffv_true_residual. Synchronizes the grid's stream to
 * return *rel_out. Errors: MFFV_EINVAL (NULL argument, aliasing, too many
 * partial sums), MFFV_ESTATE (coefficients not set), MFFV_EHIP.
 */
int mffv_true_residual_noalloc(mffv_grid* grid, const float* b, const double* x, double* r_out,
                               double* rel_out);

/*
 * Solve A x = b with conjugate gradient (Alg. 1), the apply fused with the
 * vector updates and the device-wide dot products.
 *   b     device FP32 right-hand side (n entries); its D entries are the
 *         Dirichlet values, which are copied into x.
 *   x     device FP32; in: initial guess on U; out: the solution.
 *   opts  NULL for the defaults. precision MFFV_FP32 runs FP32 CG and then
 *         reports the FP64 true residual; MFFV_FP32_IR refines in an FP64
 *         iterate held by the library and returns it rounded to FP32;
 *         MFFV_FP64 runs CG in FP64 throughout.
 *   info  may be NULL.
 * Synchronizes the stream. Returns MFFV_OK when the target was met (on the
 * recursive residual for MFFV_FP32 and MFFV_FP64, on the FP64 true residual
 * for MFFV_FP32_IR), MFFV_NOT_CONVERGED when max_iter was reached, or an error.
 * With opts->async = 1 (MFFV_FP32, precond NONE or JACOBI) the solve runs in
 * the persistent kernel of mffv_cg_solve_batched on this one system: nothing
 * is synchronized and info is a device pointer (see mffv_opts).
 */
int mffv_cg_solve(mffv_grid* grid, const float* b, float* x, const mffv_opts* opts,
                  mffv_info* info);

/*
 * As mffv_cg_solve with an FP64 right-hand side and an FP64 solution vector,
 * so that MFFV_FP32_IR can return a field refined beyond FP32 resolution
 * (relative residuals down to ~1e-12). precision must be MFFV_FP64 or
 * MFFV_FP32_IR.
 */
int mffv_cg_solve_f64(mffv_grid* grid, const double* b, double* x, const mffv_opts* opts,
                      mffv_info* info);

/*
 * Solve nsys independent systems (each its own grid handle with coefficients
 * set, any sizes below 2^30 cells; larger ones return MFFV_EINVAL) in one
 * persistent FP32 CG launch (Alg. 1 per system). grids, b and x are host
 * arrays of nsys pointers; b[s] and x[s] are device FP32 vectors of grid s
 * (x: initial guess in, solution out). All handles must share the device and
 * stream of grids[0]. info (host, nsys entries) may be NULL. opts->precond
 * may be NONE or JACOBI. Each system's starting residual is formed in FP64.
 *   precision MFFV_FP32: one FP32 CG pass per system, stopped on the
 *     recursive residual; rel_res_true is the FP64 true residual of the
 *     returned x.
 *   precision MFFV_FP32_IR: after a pass, a system whose FP64 true residual
 *     still exceeds opts->tol runs another FP32 pass on A dx = r from that
 *     residual (to a reduction min(0.5, max(tol / rel, inner_tol))) and adds
 *     dx to x, up to opts->max_outer corrections, all inside the same launch;
 *     the status is MFFV_OK when the true residual of the returned FP32 x
 *     meets tol. (Rounding x to FP32 alone leaves a true residual of a few
 *     1e-7 on grids of ~100 planes, which bounds what FP32 x can reach.)
 * A plan made by an earlier call (same grids, vectors and options) is reused;
 * it holds no copy of the coefficients, so setting a grid's coefficients again
 * needs no new plan. Synchronizes the stream. Returns MFFV_OK if every system
 * converged, MFFV_NOT_CONVERGED if any did not, or an error. With
 * opts->async = 1 it only enqueues the solve (capture-safe once the plan
 * exists, see mffv_opts), info is a device array, and the return value only
 * reports argument errors.
 */
int mffv_cg_solve_batched(mffv_grid* const* grids, int nsys, const float* const* b,
                          float* const* x, const mffv_opts* opts, mffv_info* info);

/*
 * Backward-Euler time stepping with wells (Sec. II-A: the pressure system
 * comes from an implicit backward-Euler discretisation in time with TPFA
 * fluxes in space, Eq. 3-4, and each time step is solved by Newton steps
 * J dp = -r, Eq. 5). Per step n -> n+1 and unknown cell K:
 *   c_K (p_K^{n+1} - p_K^n) + sum_L T_KL (p_K^{n+1} - p_L^{n+1})
 *                           + WI_K (p_K^{n+1} - pw_K) = q_K,
 * and p_K^{n+1} = p_K^D on Dirichlet cells. c is the storage coefficient
 * (porosity x total compressibility x cell volume / time step; 0 gives the
 * paper's incompressible model), WI >= 0 the well index of a perforated cell
 * (Peaceman form, 0 elsewhere), pw its bottom-hole pressure and q a source
 * rate (positive = injection). The residual is linear in p, so one Newton
 * step from p^n solves the step; MFFV_FP32_IR's FP64 refinement steps are the
 * further Newton steps.
 *
 * The operator must carry c + WI as its accumulation: call
 * mffv_set_transmissibility with accum = c + WI (per cell, or the scalar c
 * when there are no wells), and keep its b_out as b here.
 *
 * mffv_step_rhs writes the right-hand side of one step,
 *   rhs_K = b_K + c_K p_K^n + WI_K pw_K + q_K on unknown cells, b_K on
 * Dirichlet cells, in FP32 evaluated left to right. b, p_old, rhs: device FP32
 * arrays of n cells; c (NULL: c_scalar everywhere), wi and pw (both or
 * neither), q: device FP32 arrays or NULL. rhs must not alias an input.
 * Enqueued on the grid's stream. Errors: MFFV_EINVAL (NULL b, p_old or rhs,
 * wi without pw, c_scalar negative or not finite, aliasing), MFFV_ESTATE
 * (coefficients not set).
 *
 * mffv_time_steps runs nsteps >= 0 steps in place on p (in: p^n, out:
 * p^{n+nsteps}): each forms its right-hand side in grid-owned memory
 * (allocated by the first call) and solves with mffv_cg_solve from p^n as
 * the initial guess. opts as for mffv_cg_solve, with precision MFFV_FP32 or
 * MFFV_FP32_IR and async 0. info (host, nsteps entries) may be NULL.
 * Synchronizes the stream. Returns MFFV_OK, MFFV_NOT_CONVERGED if a step
 * missed the tolerance (its info says which; the later steps still run), or
 * the first error (p then holds the last completed step, or the failed
 * step's iterate).
 */
int mffv_step_rhs(mffv_grid* grid, const float* b, const float* c, float c_scalar,
                  const float* p_old, const float* wi, const float* pw, const float* q,
                  float* rhs);
int mffv_time_steps(mffv_grid* grid, int nsteps, const float* b, const float* c, float c_scalar,
                    const float* wi, const float* pw, const float* q, float* p,
                    const mffv_opts* opts, mffv_info* info);

/*
 * Learned preconditioner (flexible CG with opts.precond = MFFV_PRECOND_LEARNED).
 *
 * The network works on the Jacobi-scaled system A~ = D^-1/2 A D^-1/2,
 * D = diag(A). Its two input channels per cell are the scaled residual
 * r_hat = D^-1/2 r / s, s the power of two nearest the D^-1-weighted RMS of r
 * (2^round(log2 rms), rms^2 = r' D^-1 r / n_U; dividing by it is exact), and
 * r_hat times the log-diagonal feature of mffv_grid_feature; four 3x3x3 convolutions with
 * 2 -> 16 -> 16 -> 16 -> 1 channels and a ReLU after each of the first three
 * (zero padding at the grid boundary; y[K, o] = b[o] + sum_tap sum_c
 * W[tap, c, o] x[K + offset(tap), c] with tap = 9 (dx+1) + 3 (dy+1) + (dz+1))
 * map them to N. Inside flexible CG the preconditioned residual is
 * z = D^-1 r + s D^-1/2 N on unknown cells and 0 on Dirichlet cells: Jacobi
 * when N = 0. Training keeps the biases at zero, so N vanishes with r.
 * Weights and activations are BF16 in the matrix-core products, accumulation
 * is FP32, the master weights and Adam state are FP32. Parameter vector (FP32,
 * mffv_net_num_params() entries): for each layer W[27][cin][cout] in C order,
 * then b[cout]. Network calls use the current HIP device.
 */

/* Number of FP32 parameters of the network (15169). */
int mffv_net_num_params(void);

/* Create a network from host parameters (NULL: all zero). Synchronizes. */
int mffv_net_create(const float* params, mffv_net** out);

/* Release a network. NULL is a no-op. */
void mffv_net_destroy(mffv_net* net);

/* Activation of the three hidden layers: 1 = ReLU (default), 0 = identity
 * (the network is then a learned linear operator of its input channels).
 * Synchronizes the device. */
int mffv_net_set_activation(mffv_net* net, int relu);

/* Training loss: 0 = energy norm of the prediction error (the energy functional
 * when no target is given; default), 1 = residual space
 * ||A~ z - r_hat||^2 / ||r_hat||^2 (the sparse-approximate-inverse objective,
 * which weights smooth error modes by their squared eigenvalue; the target is
 * not used). */
int mffv_net_set_loss(mffv_net* net, int kind);

/* Launch shape of the network's convolutions, process-wide: each block of a
 * convolution marches through `run` consecutive x planes (clamped to nx),
 * keeping the planes it needs in a ring of LDS slots; 0 (the default) picks the
 * shortest run for which all blocks are resident at once. Every run gives the
 * same result; callers use it to pin a march length (e.g. tests). Applies to
 * later launches: HIP graphs that a solve has already captured keep theirs.
 * Errors: MFFV_EINVAL for run < 0. */
int mffv_set_nn_run(int run);

/* Copy the FP32 parameters and/or the last computed gradient to host arrays
 * of mffv_net_num_params() floats (either may be NULL). Synchronizes. */
int mffv_net_get_params(const mffv_net* net, float* params, float* grads);

/* Replace the parameters from a host array and reset the Adam state. */
int mffv_net_set_params(mffv_net* net, const float* params);

/*
 * Network output y = N(r_hat, feat) on an nx x ny x nz grid (flat layout of
 * mffv.h), input channels (r_hat, r_hat * feat). r_hat, feat, out: device
 * FP32 arrays of n cells. Enqueued on `stream`.
 */
int mffv_nn_forward(mffv_net* net, int nx, int ny, int nz, const float* r_hat, const float* feat,
                    float* out, void* stream);

/*
 * Measurement of the network's kernels (Sec. II-B's preconditioner as
 * realised here): one forward pass as mffv_nn_forward (into the network's own
 * workspace), then for each of the four layers `reps` back-to-back launches
 * between two HIP events on `stream`. us[4] (host) receives the mean
 * microseconds per launch of layers 1..4. Synchronizes the stream.
 * Errors: MFFV_EINVAL for NULL arrays or reps < 1.
 */
int mffv_nn_time_layers(mffv_net* net, int nx, int ny, int nz, const float* r_hat, const float* feat,
                        int reps, double* us, void* stream);

/*
 * Loss and parameter gradient of one training pair on the grid's operator
 * (the gradient stays in the network; read it with mffv_net_get_params).
 * r_hat is the scaled residual and target the scaled error of
 * mffv_harvest_pair, so that A~ target = r_hat. With z = r_hat + N(r_hat, f):
 *   loss = (z - target)' A~ (z - target) / (target' r_hat)
 * over the unknown cells: the energy norm of the prediction error relative to
 * that of the error (1 for z = 0; the Jacobi value for N = 0). With target
 * NULL the loss is the energy functional (z' A~ z - 2 z' r_hat) / (r_hat' r_hat),
 * minimal at z = A~^-1 r_hat, so any residual can serve as a training input.
 * r_hat is taken as 0 on Dirichlet cells. Enqueued on the grid's stream;
 * *loss (host, may be NULL) synchronizes it.
 */
int mffv_nn_loss_grad(mffv_net* net, mffv_grid* grid, const float* r_hat, const float* target,
                      double* loss);

/* mffv_nn_loss_grad followed by one Adam step (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected, biases fixed) with learning rate lr. */
int mffv_nn_train_step(mffv_net* net, mffv_grid* grid, const float* r_hat, const float* target,
                       float lr, double* loss);

/* The network's second input channel for a grid: log(d) minus its mean over
 * the unknown cells, d = diag(A); 0 on Dirichlet cells. feat: device FP32, n. */
int mffv_grid_feature(mffv_grid* grid, float* feat);

/*
 * One training pair of the learned preconditioner from an iterate x of a solve
 * of A x = b and a reference solution x_star, in the Jacobi-scaled space:
 * r = b - A x (x must hold the Dirichlet values of b), s^2 = r' D^-1 r / n_U,
 * r_hat = D^-1/2 r / s and target = D^1/2 (x_star - x) / s (so that
 * A~ target = r_hat), both zero on Dirichlet cells. b, x: device FP32;
 * x_star: device FP64; outputs device FP32 (n cells each). *scale (host, may
 * be NULL) receives s and synchronizes the grid's stream.
 */
int mffv_harvest_pair(mffv_grid* grid, const float* b, const float* x, const double* x_star,
                      float* r_hat, float* target, float* scale);

/*
 * A training residual as the network sees it between the Jacobi sweeps (an
 * addition of this library: its preconditioner applies the network to the
 * residual left by a damped Jacobi step). For a Jacobi-scaled residual r_hat
 * (mffv_harvest_pair's space), out = (I - omega A~) r_hat on the unknown cells
 * and 0 on Dirichlet cells, A~ = D^-1/2 A D^-1/2, D = diag(A). r_hat, out:
 * device FP32, n cells, may not alias. Enqueued on the grid's stream.
 * Errors: MFFV_EINVAL for NULL arrays or omega outside [0, 2).
 */
int mffv_nn_smooth_sample(mffv_grid* grid, double omega, const float* r_hat, float* out);

/* Launch shape chosen for a grid's stencil kernels. */
typedef struct {
    int ci;          /* planes a block marches through along x */
    int remap;       /* 1: XCD-aware block order */
    int vec;         /* cells per thread along z (4 or 1) */
    int blocks;      /* blocks per launch */
    double apply_us; /* measured apply time of the chosen shape (microseconds) */
    int candidates;  /* shapes timed (0 when read from the cache) */
    double phase_a_us; /* measured time of the fused CG phase A of the chosen shape */
    int seg;         /* chunk shape: row segments of seg cells, -1 = flat chunks */
    /* the apply's own shape (mffv_apply), chosen on the apply's time */
    int apply_ci, apply_remap, apply_seg, apply_blocks;
} mffv_tune_result;

/*
 * Set the launch shape of the grid's FP32 stencil kernels (the CG kernels and
 * the apply) by hand: ci planes per
 * block (0 = the library's default for the shape), remap 0/1, and the shape of
 * a block's chunk of a plane: seg = 0 (the library's default), -1 (flat: 1024
 * consecutive cells of the plane) or a power of two in [16, 1024] that divides
 * nz (row segments: 4096/seg rows of seg cells, the float4 path only).
 * Invalid values return MFFV_EINVAL. Synchronizes.
 */
int mffv_set_launch(mffv_grid* grid, int ci, int remap, int seg);

/*
 * Autotune the grid's FP32 stencil launch shape (the operator must be set):
 * every candidate (ci in 1..64 planes per block, XCD-aware order on or off,
 * flat chunks or row segments of 32..256 cells)
 * must reproduce the default shape's apply bit for bit; it is then timed on
 * the grid's own operator with HIP events, as an apply and as the CG iteration
 * (fused phase A, the solver's hot kernel, plus phase B, whose prologue sums
 * one partial per phase-A block) over the first 32 iterations of a solve. The
 * shape with the fastest iteration is applied to the CG kernels and the one
 * with the fastest apply to mffv_apply. With a cache_path (may be NULL), a
 * previous result for the same device architecture and shape is reused, and a
 * new one is written to that JSON file. Uses the grid's workspace (overwrites
 * the solver's work vectors); synchronizes.
 */
int mffv_autotune(mffv_grid* grid, const char* cache_path, mffv_tune_result* out);

/*
 * Launch shape of later batched solves: blocks per CU of the persistent
 * kernel (0 = as many as fit) and work items (plane chunk x plane group) per
 * block. Process-wide.
 */
int mffv_set_batched_launch(int blocks_per_cu, int items_per_block);

/*
 * Limit of one per-system wait (barrier or partial-sum exchange) of the
 * persistent batched kernel, in seconds (default 2; process-wide, applies to
 * later batched solves). A block whose wait exceeds it records an error and
 * leaves, and the solve returns MFFV_EHIP, so a launch whose blocks cannot all
 * be resident ends instead of hanging. 0 makes every wait that is not
 * satisfied at once fail: for callers that test that failure path. Values
 * outside [0, 3600] return MFFV_EINVAL.
 */
int mffv_set_batched_watchdog(double seconds);

/*
 * Block shares of repeated batched solves (process-wide, default on). The
 * systems of a batch get the persistent kernel's blocks in proportion to their
 * expected work, first cells x (nx + ny + nz). A system's blocks advance
 * together and the launch lasts as long as its slowest system, so after each
 * synchronous solve the plan compares those shares with shares in proportion
 * to the cells x iterations it has just seen; if the latter would shorten the
 * slowest system's time by more than 5 %, the next solve of the same batch
 * (same grids, vectors and options) uses them, and captures its graph again.
 * Results do not depend on the shares beyond FP32 rounding of the dot
 * products. Asynchronous solves neither take nor change shares. on = 0 keeps
 * the size-based shares.
 */
int mffv_set_batched_rebalance(int on);

/*
 * Autotune the batched launch shape: solves the batch (as mffv_cg_solve_batched)
 * for every candidate (1, 2, 3, 4 or all-fitting blocks per CU x 1, 2, 4, 8, 16 work
 * items per block), each from the initial guess held in x, times each with HIP
 * events and applies the fastest (results returned through the pointers, any
 * may be NULL). x holds the initial guess again on return. Allocates a copy of
 * the initial guesses for the duration of the call. Synchronizes.
 */
int mffv_autotune_batched(mffv_grid* const* grids, int nsys, const float* const* b,
                          float* const* x, const mffv_opts* opts, int* blocks_per_cu,
                          int* items_per_block, double* best_ms);

/*
 * Streaming copy dst[i] = src[i] of `bytes` bytes (a multiple of 16) with the
 * library's own vector kernel: the achievable HBM ceiling the stencil kernels
 * are compared with. Device pointers, 16-byte aligned. Enqueued on `stream`.
 */
int mffv_copy_probe(void* dst, const void* src, size_t bytes, void* stream);

/*
 * Streaming probe: out[j][i] = sum_k in[k][i] for i < n, j < nout, four
 * cells per thread with the nontemporal stores of the stencil kernels. With
 * the numbers of arrays a stencil kernel reads and writes (e.g. 4 in / 1 out
 * for the apply), its rate is the achievable ceiling for that kernel's mix of
 * reads and writes, without its arithmetic or neighbour accesses. in and out
 * are host arrays of nin (1..8) and nout (1..4) device FP32 pointers, 16-byte
 * aligned; n a multiple of 4; no output may alias an input. Enqueued on
 * `stream`. Errors: MFFV_EINVAL.
 */
int mffv_stream_probe(const float* const* in, int nin, float* const* out, int nout, int64_t n,
                      void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MFFV_H */
