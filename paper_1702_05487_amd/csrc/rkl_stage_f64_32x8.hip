// rkl_stage_f64_32x8.hip -- the one-stage kernels of the 32 x 8 tile, FP64.
#include "rkl_stage.h"

namespace rkl {

template hipError_t launch_shape<double, 32, 8>(RKL_SHAPE_ARGS);

}  // namespace rkl
