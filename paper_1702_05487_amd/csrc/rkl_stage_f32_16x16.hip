// rkl_stage_f32_16x16.hip -- the one-stage kernels of the 16 x 16 tile, flux precision FP32 (mixed).
#include "rkl_stage.h"

namespace rkl {

template hipError_t launch_shape<float, 16, 16>(RKL_SHAPE_ARGS);
template hipError_t launch_fixed<float>(RKL_SHAPE_ARGS);

}  // namespace rkl
