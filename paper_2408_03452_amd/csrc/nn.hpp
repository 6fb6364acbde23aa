// Learned preconditioner: internal interface used by the CG loop.
#pragma once

#include "common.hpp"
#include "mffv.h"

namespace mffv {

// z = M(r) for flexible CG; ||r||^2 is the sum of the nb_b phase-B partials
// pb[0..nb_b). Enqueued on s.
int nn_precondition(const mffv_net* net, const Geom& g, const float* r, const float* dinv,
                    const uint8_t* dmask, float* z, const float* pb, int nb_b,
                    CgState<float>* st, hipStream_t s);

}  // namespace mffv
