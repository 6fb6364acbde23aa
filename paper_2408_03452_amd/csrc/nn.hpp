// Learned preconditioner: internal interface used by the CG loop.
#pragma once

#include "launch.hpp"
#include "mffv.h"

namespace mffv {

// The preconditioned residual z of r for flexible CG (0 on Dirichlet cells).
// The network's correction of a residual v is C(v) = s D^-1/2 N(v_hat, feat),
// v_hat = D^-1/2 v / s, s^2 = v' D^-1 v / n_u. omega = 0: z = D^-1 r + C(r),
// with r' D^-1 r the sum of the nb_b phase-B partials pb. omega > 0: the
// network between two damped Jacobi sweeps on the operator (g, c), applied
// with launch shape m: z1 = omega D^-1 r, r1 = r - A z1,
// z2 = z1 + D^-1 r1 + C(r1), z = z2 + omega D^-1 (r - A z2) (sqd: sqrt(dinv),
// 0 on Dirichlet cells, from nn_feature). Enqueued on s;
// allocates nothing if nn_prepare ran. layer_ev (optional): 5 events, recorded
// before the first convolution and after each of the four.
// With the sweeps fused into the operator passes, the second one also forms
// the per-block partials of the flexible-CG dots (z.r, z.q, dinv r.r, dinv r.q;
// q may be NULL, then those of q are 0): *flex_part and *nb_flex receive them
// (network-owned, [4][nb_flex]); otherwise *flex_part is NULL and the caller
// forms the dots itself. done (optional): the CG loop's done flag; every
// kernel of the preconditioner returns at once once it is set, so the
// iterations a chunk holds past the loop's end cost no network passes.
int nn_precondition(const mffv_net* net, const Geom& g, const Coef& c, const March& m, float omega,
                    const float* r, const float* dinv, const uint8_t* dmask, const float* sqd, float* z,
                    const float* pb, int nb_b, const float* feat, float n_u, hipStream_t s,
                    const float* q, const float** flex_part, int* nb_flex, hipEvent_t* layer_ev = nullptr,
                    const int* done = nullptr);

// Make sure the network's inference workspace holds n cells; returns the
// workspace generation (changes whenever the workspace is reallocated), or a
// negative error code.
int nn_prepare(const mffv_net* net, int64_t n);

// Forward pass, energy-norm loss and (if grads) the parameter gradient for a
// training pair (r_hat: Jacobi-scaled residual, target: scaled error) on the
// operator (g, c) with march plan m. The loss is left on the device at
// nn_loss_ptr(net).
int nn_loss(mffv_net* net, const Geom& g, const Coef& c, const March& m, const float* dinv,
            const uint8_t* dmask, const float* feat, const float* r_hat, const float* target,
            bool grads, hipStream_t s);
int nn_adam(mffv_net* net, float lr, hipStream_t s);
const double* nn_loss_ptr(const mffv_net* net);

// Log-diagonal input feature of a grid: log(d) - mean over unknown cells of
// log(d), d = 1 / dinv; 0 on Dirichlet cells. Also sqd = sqrt(dinv) on unknown
// cells, 0 on Dirichlet cells. part: scratch of 1024 floats.
int nn_feature(const Geom& g, const float* dinv, const uint8_t* dmask, float n_u, float* part,
               float* feat, float* sqd, hipStream_t s);

}  // namespace mffv
