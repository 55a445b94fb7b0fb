// rkl_batch.h -- the batched (many-grid) super-step of librkl.
#pragma once
#include <string>
#include <utility>
#include <vector>

#include "../../include/rkl.h"
#include "rkl_internal.h"

namespace rkl {

struct BatchPlan;

struct BatchBuffers {
    double* T;             // packed temperatures (updated in place)
    const void* b;         // packed unit vectors, 3 x cells per grid
    const double* dt_hyp;  // device, ngrids
    int32_t* s_out;        // device, ngrids, may be NULL
    double* Ya;            // packed stage buffers (plan scratch)
    double* Yb;
    void* MY0;
    const double* coef;    // RKL2 table
    GridState* state;      // ngrids
};

// policy: index into the batched tile policies (batch_policy_count())
rkl_status batch_create(const std::vector<rkl_grid_desc>& desc, const std::vector<GridConst>& gc,
                        const std::vector<int64_t>& off, int precision, int smax, int policy,
                        BatchPlan** out, std::string& why);
int batch_policy_count();
void batch_policy_info(int policy, int* half_rows, int* bz);
void batch_free(BatchPlan* bp);
// Enqueue one super-step of every grid (no host synchronisation).  mode 0:
// one launch per stage; mode 1: the persistent launch (batch_persist_init
// first).  With `events` non-NULL, a pair of HIP events (created here, owned
// by the caller) is recorded around each launch of stages j >= 2 (mode 0) or
// around the persistent launch (mode 1).
hipError_t batch_launch(BatchPlan* bp, const BatchBuffers& buf, hipStream_t st,
                        std::vector<std::pair<hipEvent_t, hipEvent_t>>* events = nullptr, int mode = 0);
// Buffers and launch size of the persistent mode (once per plan).
rkl_status batch_persist_init(BatchPlan* bp, std::string& why);
// Whether the last persistent launch gave up a wait (synchronous read).
hipError_t batch_aborted(const BatchPlan* bp, bool* aborted);

}  // namespace rkl
