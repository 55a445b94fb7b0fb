// rkl_stage_f32_32x8.hip -- the one-stage kernels of the 32 x 8 tile, flux precision FP32 (mixed).
#include "rkl_stage.h"

namespace rkl {

template hipError_t launch_shape<float, 32, 8>(RKL_SHAPE_ARGS);

}  // namespace rkl
