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
// Grow the context's workspace to exactly `bytes` now if it holds less (may
// synchronise the device).
int reserve_workspace(icp_ctx* ctx, size_t bytes);
// Workspace bytes that suffice for any batch of some or all of these n
// problems: planned with the given tile sizes (tile_px[l] > 0) or otherwise
// the smallest tile, which gives the most tiles and hence the most partials.
size_t workspace_bound(int n, const int32_t* W, const int32_t* H, int levels, const int32_t* tile_px);
// ICP_OK or ICP_EINVAL with the context's message set.
int validate_params(icp_ctx* ctx, const icp_params* params);
// The context's last error message.
const char* error(icp_ctx* ctx);

// For its lifetime, this thread's allocation and free calls run in relaxed
// stream-capture mode, so that they cannot invalidate a graph another thread
// is capturing (a frame server captures on its scheduler thread while clients
// submit frames and open streams).
struct RelaxedCaptureScope {
    hipStreamCaptureMode prev = hipStreamCaptureModeRelaxed;
    RelaxedCaptureScope() { (void)hipThreadExchangeStreamCaptureMode(&prev); }
    ~RelaxedCaptureScope() { (void)hipThreadExchangeStreamCaptureMode(&prev); }
    RelaxedCaptureScope(const RelaxedCaptureScope&) = delete;
    RelaxedCaptureScope& operator=(const RelaxedCaptureScope&) = delete;
};

// Largest |(R^T R - I)_ij| a rotation passed to the library may show.
constexpr double kRotTol = 1e-6;

// True when the 3x3 block R (row i at R + i * stride) is a rotation: finite,
// R^T R = I within kRotTol entry by entry, det R > 0.
inline bool is_rotation(const double* R, int stride) {
    double M[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            M[i][j] = R[i * stride + j];
            if (!(M[i][j] == M[i][j]) || M[i][j] > 1e300 || M[i][j] < -1e300) return false;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double g = M[0][i] * M[0][j] + M[1][i] * M[1][j] + M[2][i] * M[2][j] - (i == j ? 1.0 : 0.0);
            if (!(g <= kRotTol && g >= -kRotTol)) return false;
        }
    const double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                       M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                       M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    return det > 0.0;
}

}  // namespace icpi
