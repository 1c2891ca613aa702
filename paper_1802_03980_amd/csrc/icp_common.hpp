// Internal layout shared by the kernels and the host side of libicp_mi355x.
//
// HBM layout per problem (all float32, level l has W_l x H_l = (W>>l) x (H>>l)):
//   live depth D_l (level 0 is the caller's buffer), live vertex LV_l and
//   normal LN_l as three planes (x plane, y plane, z plane) of W_l*H_l floats,
//   consecutive planes `ps` floats apart (W_l*H_l rounded up to 64, so every
//   plane starts on a 256-byte boundary and a thread reads four consecutive
//   pixels as one 16-byte load); model vertex MV_l and normal MN_l interleaved
//   (x, y, z per pixel: a projective lookup gathers 12 contiguous bytes per
//   map), level 0 being the caller's buffers.  Invalid entries are NaN (maps)
//   or 0 (depth).  Per level a problem also owns its tile partials.  The small
//   per-problem state (pose, histogram, band, statistics) lives in one
//   ProbState.
#pragma once

#include <stdint.h>

#include "icp.h"

#define ICP_WG 256              // threads per work-group (four wave64)
#define ICP_WAVES (ICP_WG / 64)
#define ICP_PART_STRIDE 32      // floats per tile partial: 28 moments, count, pad
#define ICP_NMOM 28
#ifndef ICP_PX_PER_THREAD
#define ICP_PX_PER_THREAD 4
#endif
#define ICP_PASS1_PX 1          // pixels per thread and round in the single-pass kernel
#define ICP_TILE_QUANTUM (ICP_WG * ICP_PX_PER_THREAD)
#define ICP_PLANE_ALIGN 64      // floats
#define ICP_WIN 48              // bins of the predicted band-edge window (single-pass mode)
#define ICP_WIN_SLOTS (ICP_WIN + 1)  // slot 0: rows below the window; slots 1..: one per window bin

struct LevelDesc {
    int32_t W, H, npx;          // size of the level, npx = W*H
    int32_t ps;                 // plane stride in floats (npx rounded up to ICP_PLANE_ALIGN)
    int32_t tile_px;            // pixels per tile (multiple of ICP_TILE_QUANTUM)
    int32_t n_tiles;            // ceil(npx / tile_px)
    int32_t tile_base;          // first flat tile of this problem at this level
    double fx, fy, cx, cy;      // intrinsics of the level
    double rfx, rfy;            // 1/fx, 1/fy (IEEE FP64 divisions)
    double umax, vmax;          // W - 1, H - 1
    const float* D;             // depth (level 0: caller input)
    float* Dw;                  // writable depth (levels >= 1), same as D there
    float* LV;                  // live vertex, 3 planes
    float* LN;                  // live normal, 3 planes
    const float* MV;            // model vertex, interleaved (level 0: caller's buffer)
    const float* MN;            // model normal, interleaved
    float* MVw;                 // writable model maps (levels >= 1), same as MV/MN there
    float* MNw;
    double* XQ;                 // back-projection quotients (u - cx)/fx, u = 0..W
    double* YQ;                 // (v - cy)/fy, v = 0..H
    float* part;                // pass-2 partials: n_tiles * ICP_PART_STRIDE
    float* part1;               // single-pass partials: n_tiles * ICP_WIN_SLOTS * ICP_PART_STRIDE
};

// Front-end options of a batch: the bilateral filter's spatial weights (row-major
// over the (2r+1)^2 window, computed on the host) and range cut-off, and the
// normal mode.
#define ICP_FILTER_MAX_R 7
struct FrontEnd {
    int32_t depth_filter, filter_radius, normal_mode, normal_radius;
    double sigma_m;
    double inv_sigma_m;         // 1 / sigma_m, correctly rounded (an IEEE division on the host)
    double ws[(2 * ICP_FILTER_MAX_R + 1) * (2 * ICP_FILTER_MAX_R + 1)];
};

// One depth image turned into interleaved vertex / normal maps.
struct MapsDesc {
    const float* depth;
    float* mv;
    float* mn;
    int32_t W, H;
    double fx, fy, cx, cy;
};

// A TSDF volume as the kernels see it (the caller's icp_tsdf).
struct TsdfDesc {
    float* voxels;              // dim^3 (tsdf, weight) pairs, x fastest
    int32_t dim;
    double size, origin[3], mu, max_weight;
    void* bricks;               // per-brick counts and flags (NULL: no brick skipping)
};

struct ProbState {
    double R[9];                // current pose, row-major rotation
    double t[3];
    double M[ICP_NMOM];         // last reduced moments (FP64 sums of tile partials)
    double x[6];                // last increment
    int64_t n_last;             // kept pairs of the last reduction
    uint32_t hist[2][ICP_HIST_BINS];  // distance histogram; IterCtl::par selects the one in use
    uint32_t N;                 // gated pairs of the current iteration
    int32_t k_med, k_lo, k_hi;  // median bin and kept band of the current iteration
    int32_t pred_hi[2];         // band upper edge predicted for an iteration (-1: none), by IterCtl::par
    int32_t pred_hw[2];         // half-width of the window around it, in bins (at most ICP_WIN / 2)
    int32_t fused_done;         // this iteration was completed from the single-pass partials
    int32_t level_done;         // the current level has ended (status or convergence)
    int32_t settled;            // successive iterations with an unchanged median
    int32_t last_kmed;
    int32_t last_status;        // status of the last solve
    int32_t ticket;             // work-groups of k_band_pass2 finished this iteration
    icp_stats stats;
    double cen[ICP_MAX_LEVELS][3];  // centroid of each level's valid live vertices
    double cur_c[3];            // centring point of the current iteration (model frame)
};

struct ProbDesc {
    LevelDesc lv[ICP_MAX_LEVELS];
    double imu_R[9];            // IMU rotation prior, row-major
    double init[12];            // initial pose, 3x4 row-major [R | t]
    ProbState* st;
    const float* depth_in;      // the caller's level-0 depth (lv[0].D is its filtered copy when filtering)
};

// Scalars of a launch that are the same for every problem in it.
struct IterCtl {
    int32_t level;
    int32_t iter;               // iteration index within the level
    int32_t last_of_level;      // this is the level's last scheduled iteration
    int32_t no_update;          // stage calls: reduce only, keep the pose
    int32_t par;                // histogram and window prediction in use (0, or the global iteration's
                                //   parity where k_band_pass2 runs: its launch reads one and writes the other)
};

struct KParams {
    double d2max;               // dist_max^2
    double cos_max;
    double band_beta;
    double lambda_c;
    double ill_cond_eps;
    int32_t lambda_mode;
    int32_t use_filter;
    int32_t min_corr;
    int32_t converge_window;
    int32_t reduce_mode;        // 0: FP32 rows; 1: FP16 hi+lo split MFMA on centred rows
    int32_t* need2;             // batch flag: some problem needs pass 2 this iteration (NULL: always run it)
    int32_t anchor_to_imu;      // the damping acts on the deviation from the IMU rotation
    int32_t fold_solve;         // one problem, single pass, FP32 reduction: band, pass 2 and solve in one
                                //   launch per iteration (k_band_pass2)
};
