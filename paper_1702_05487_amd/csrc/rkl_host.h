// rkl_host.h -- host-side helpers of librkl shared by its C-ABI sources.
#pragma once
#include <string>

#include "../../include/rkl.h"
#include "rkl_internal.h"

namespace rkl {

// record `msg` as the calling thread's last error (rkl_last_error) and
// return `st`
rkl_status fail(rkl_status st, const std::string& msg);
// RKL_EDEVICE with the HIP error's text
rkl_status hipfail(hipError_t e, const char* what);
// descriptor checks of rkl_plan (false with the reason in `why`)
bool validate(const rkl_grid_desc& g, std::string& why);
// per-grid device constants of a descriptor
GridConst make_const(const rkl_grid_desc& g, int scheme);

}  // namespace rkl
