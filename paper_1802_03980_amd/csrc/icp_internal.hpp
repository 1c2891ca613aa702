// Library-internal entry points shared by the C-ABI implementation and the
// frame server (not exported).
#pragma once
#include <hip/hip_runtime.h>

#include "icp.h"

namespace icpi {

// Stage and launch a batched registration on stream s and queue the copy of
// the n results into h_res (pinned host memory); nothing waits for the GPU.
int register_batch_async(icp_ctx* ctx, int n, const icp_problem* probs, const icp_params* params, icp_result* h_res,
                         hipStream_t s);
// Grow the context's workspace to at least `bytes` now (may synchronise the device).
int reserve_workspace(icp_ctx* ctx, size_t bytes);
// ICP_OK or ICP_EINVAL with the context's message set.
int validate_params(icp_ctx* ctx, const icp_params* params);
// The context's last error message.
const char* error(icp_ctx* ctx);

}  // namespace icpi
