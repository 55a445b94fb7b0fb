// rkl_stage_f64_64x4.hip -- the one-stage kernels of the 64 x 4 tile, FP64.
#include "rkl_stage.h"

namespace rkl {

template hipError_t launch_shape<double, 64, 4>(RKL_SHAPE_ARGS);

}  // namespace rkl
