// Host-side launchers of the gfx950 kernels (defined in icp_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "icp_common.hpp"

namespace icpk {

struct PoseArg {
    double v[12];  // 3x4 row-major [R | t]
};

struct MomArg {
    double m[ICP_NMOM];
};

// centroid of every level's valid live vertices (split-precision reduction):
// per-tile FP64 sums over the level's flat tiles (owner[l], tiles[l]), then
// per problem in tile order; uses the pass-2 partials as scratch
hipError_t launch_centroid(const ProbDesc* probs, int n, int levels, const int* const* owner, const int* tiles,
                           hipStream_t s);
// interleaved vertex / normal maps of n depth images (grid: max_blocks x n)
hipError_t launch_depth_to_maps(const MapsDesc* jobs, int n, int max_blocks, hipStream_t s);
// live-map work-groups of a W x H level (one per 64 x 4 pixels)
int live_vn_blocks(int W, int H);
// depth- and model-pyramid threads of a W x H level (one per 2 x 2 block)
int model_blocks(int W, int H);
// Start of every problem's registration: its initial state (pose seeded by
// the IMU rotation or the initial pose; histograms, tickets, flags and
// statistics cleared; the batch's pass-2 flag cleared), then the front end:
// optional bilateral filter of the caller's depth into the level-0 workspace
// plane, depth pyramid, back-projection quotient tables (box normals only),
// live normal planes (forward differences or box gradients), model pyramid
// (two levels per launch), and (with_live_maps) the live vertex planes, which
// only the stage-access calls read (the pixel passes rebuild the vertices from
// depth).  Raw depth with forward-difference normals over two or three levels
// takes two launches.
hipError_t launch_prepare(const ProbDesc* probs, int n, int levels, const int* max_vn_blocks,
                          const int* max_model_blocks, const int* max_quot, bool with_live_maps, const FrontEnd& fe,
                          int use_imu_seed, int32_t* need2, hipStream_t s);
// one ICP iteration at ctl.level: pass 1 over `tiles` flat tiles of all
// problems, the per-problem band, pass 2 over the tiles, the per-problem solve
hipError_t launch_pass1(const ProbDesc* probs, const int* owner, int tiles, IterCtl ctl, const KParams& kp, int fused,
                        hipStream_t s);
hipError_t launch_band(const ProbDesc* probs, int n, IterCtl ctl, const KParams& kp, int fused, hipStream_t s);
hipError_t launch_pass2(const ProbDesc* probs, const int* owner, int tiles, IterCtl ctl, const KParams& kp,
                        hipStream_t s);
hipError_t launch_solve(const ProbDesc* probs, int n, IterCtl ctl, const KParams& kp, hipStream_t s);
// one problem, single pass, FP32 reduction: band, pass 2 and solve in one launch
hipError_t launch_band_pass2(const ProbDesc* probs, int tiles, IterCtl ctl, const KParams& kp, hipStream_t s);
// write one problem descriptor (a kernel argument) to dst; fill n ints with v
hipError_t launch_put_desc(const ProbDesc& d, ProbDesc* dst, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t s);
// pose and statistics of every problem into results[n]
hipError_t launch_finalize(const ProbDesc* probs, int n, icp_result* results, hipStream_t s);

// stage access (problem 0 of `probs`)
hipError_t launch_stage_set(const ProbDesc* probs, PoseArg pose, int k_lo, int k_hi, int level, int pred_hi,
                            int pred_hw, hipStream_t s);
// the single-pass iteration's pass 1 (band-edge window partials) and band
// kernel (moments from the partials when the edge fell in the window), with
// the window's (h0, width) written to window[2] (device)
hipError_t launch_stage_single(const ProbDesc* probs, const int* owner, int tiles, IterCtl ctl, const KParams& kp,
                               int32_t* window, hipStream_t s);
hipError_t launch_stage_pass1(const ProbDesc* probs, const int* owner, int tiles, IterCtl ctl, const KParams& kp,
                              uint8_t* code, int32_t* bin, uint32_t* hist, hipStream_t s);
hipError_t launch_stage_pass2(const ProbDesc* probs, const int* owner, int tiles, IterCtl ctl, const KParams& kp,
                              hipStream_t s);
hipError_t launch_stage_solve(MomArg M, int64_t n, PoseArg pose, const KParams& kp, double* out, hipStream_t s);

// TSDF volume (icp_tsdf.hip): clear every voxel to (0, 0); fuse one depth image
// taken from camera-to-world pose T (3x4); ray-cast interleaved vertex / normal
// maps in the camera of T.  K = fx, fy, cx, cy.  With a brick buffer the fill
// and the fusion keep its counts and flags current and the ray cast uses them.
hipError_t launch_tsdf_fill(const TsdfDesc& d, hipStream_t s);
// bytes of the brick buffer of a dim^3 volume (counts, then flags), and of its counts part
size_t tsdf_brick_bytes(int dim);
size_t tsdf_count_bytes(size_t nb3);
hipError_t launch_tsdf_integrate(const TsdfDesc& d, const float* depth, int W, int H, const double* K, PoseArg T,
                                 hipStream_t s);
hipError_t launch_tsdf_raycast(const TsdfDesc& d, double tmin, double tmax, int W, int H, const double* K, PoseArg T,
                               float* vtx, float* nrm, hipStream_t s);

}  // namespace icpk
