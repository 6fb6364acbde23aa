#include "mffv.h"
#include "launch.hpp"

extern "C" int mffv_cg_solve_batched(mffv_grid* const* grids, int nsys, const float* const* b,
                                     float* const* x, const mffv_opts*, mffv_info*) {
    if (!grids || !b || !x || nsys <= 0) return MFFV_EINVAL;
    return MFFV_ESTATE;
}
