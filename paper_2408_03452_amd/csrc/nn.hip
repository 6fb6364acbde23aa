#include "nn.hpp"

namespace mffv {

int nn_precondition(const mffv_net*, const Geom&, const float*, const float*, const uint8_t*,
                    float*, const float*, int, CgState<float>*, hipStream_t) {
    return MFFV_EINVAL;
}

}  // namespace mffv
