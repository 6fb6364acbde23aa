// Learned preconditioner: internal interface used by the CG loop.
#pragma once

#include "common.hpp"
#include "mffv.h"

namespace mffv {

// z = M(r) for flexible CG; reads ||r||^2 from st->rr. Enqueued on s.
int nn_precondition(const mffv_net* net, const Geom& g, const float* r, const float* dinv,
                    const uint8_t* dmask, float* z, CgState<float>* st, hipStream_t s);

}  // namespace mffv
