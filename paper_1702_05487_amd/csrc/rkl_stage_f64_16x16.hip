// rkl_stage_f64_16x16.hip -- the one-stage kernels of the 16 x 16 tile, FP64.
#include "rkl_stage.h"

namespace rkl {

template hipError_t launch_shape<double, 16, 16>(RKL_SHAPE_ARGS);
template hipError_t launch_fixed<double>(RKL_SHAPE_ARGS);

}  // namespace rkl
