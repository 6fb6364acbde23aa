// Learned preconditioner: internal interface used by the CG loop.
#pragma once

#include "launch.hpp"
#include "mffv.h"

namespace mffv {

// z = dinv r + s N([r / s, feat]) on unknown cells (0 on Dirichlet cells) for
// flexible CG, with s = ||r|| / sqrt(n_u) and ||r||^2 the sum of the nb_b
// phase-B partials pb. Enqueued on s; allocates nothing if nn_prepare ran.
// layer_ev (optional): 5 events, recorded before the first convolution and
// after each of the four.
int nn_precondition(const mffv_net* net, const Geom& g, const float* r, const float* dinv,
                    const uint8_t* dmask, float* z, const float* pb, int nb_b, const float* feat,
                    float n_u, hipStream_t s, hipEvent_t* layer_ev = nullptr);

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
// log(d), d = 1 / dinv; 0 on Dirichlet cells. part: scratch of 1024 floats.
int nn_feature(const Geom& g, const float* dinv, const uint8_t* dmask, float n_u, float* part,
               float* feat, hipStream_t s);

}  // namespace mffv
