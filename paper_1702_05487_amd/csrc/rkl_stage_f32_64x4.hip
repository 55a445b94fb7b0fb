// rkl_stage_f32_64x4.hip -- the one-stage kernels of the 64 x 4 tile, flux precision FP32 (mixed).
#include "rkl_stage.h"

namespace rkl {

template hipError_t launch_shape<float, 64, 4>(RKL_SHAPE_ARGS);

}  // namespace rkl
