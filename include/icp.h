/*
 * icp.h -- C ABI of the MI355X (gfx950) tracking hot path of IMU-seeded,
 * median-filtered, rotation-regularised KinectFusion ICP
 * (Giancola, Schneider, Wonka, Ghanem, "Integration of Absolute Orientation
 * Measurements in the KinectFusion Reconstruction pipeline", 2018).
 *
 * Problem statement (paper Sec. 1 and Sec. 3, Eq. (1)): find the rigid motion
 * M = (R, t) in SE(3) that maps the live depth frame onto the model so that the
 * point-to-plane distances of matched points are minimal.  Here M maps
 * live-camera coordinates to model-camera coordinates: X_model = R X_live + t.
 *
 * Conventions shared by every entry point
 *   - Images are row-major: pixel (u, v) (column u, row v) is element v*W + u.
 *   - live_depth: H*W float32 metres on the device; a pixel is valid iff its
 *     value is finite and > 0.
 *   - model_vtx, model_nrm: H*W*3 float32 (x, y, z interleaved) on the device,
 *     in the model camera frame (the predicted maps KinectFusion ray-casts from
 *     its model); a pixel is valid iff all six values are finite.  Normals are
 *     unit length and face the camera.
 *   - Poses are row-major doubles: 4x4 (16 values) in the public calls, 3x4
 *     [R | t] (12 values) in the stage calls.  imu_R is 3x3 row-major.
 *     Every rotation the library takes (imu_R; the rotation of init_pose when
 *     the IMU seed is off; the rotation of a TSDF camera pose T_wc; the server's
 *     imu_rel_R) must be a rotation: finite, |(R^T R - I)_ij| <= 1e-6 for every
 *     entry and det R > 0, else the call returns ICP_EINVAL (the pose is an
 *     element of SE(3), paper Sec. 3).  A caller that chains estimated poses
 *     should project them back onto SO(3): rounding errors in a prior built
 *     from an estimated pose otherwise grow from frame to frame.
 *   - W and H must be divisible by 2^(levels-1); 1 <= levels <= ICP_MAX_LEVELS;
 *     W, H <= ICP_MAX_DIM.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Device buffers handed to a call must stay alive until the stream work
 *     that uses them has completed.
 *   - Return value: ICP_OK (0) or a negative ICP_E* code; icp_strerror() names
 *     it and icp_last_error() gives the context's last message.  Numerical
 *     outcomes (too few correspondences, an ill-conditioned system) are not
 *     errors: they are reported per level in icp_stats and the pose keeps its
 *     last good value.  No C++ exception crosses this interface.
 *   - A context is used by one host thread at a time.  It owns all device
 *     workspace (pyramids, histograms, partial sums, per-problem state).
 *     Its calls may name different streams: since they share that workspace,
 *     each call's stream first waits for the work the context's previous call
 *     queued, so calls on one context never overlap on the device (concurrent
 *     work takes one context per stream).  The TSDF calls use no context
 *     memory and are ordered by their streams alone.
 */
#ifndef ICP_MI355X_H
#define ICP_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ICP_ABI_VERSION 5
#define ICP_MAX_LEVELS 4
#define ICP_MAX_DIM 8192
#define ICP_HIST_BINS 1024 /* distance histogram: bins of 2^-13 m over [0, 0.125) m */

/* return codes */
#define ICP_OK 0
#define ICP_EINVAL (-1)   /* null pointer, bad size or bad parameter */
#define ICP_ENOMEM (-2)   /* workspace would exceed the context's HBM budget, or allocation failed */
#define ICP_EDEVICE (-3)  /* a HIP runtime error; icp_last_error() has its text */
#define ICP_ETIMEOUT (-4) /* reserved for a device-side wait that gives up; no call returns it at present */

/* per-level numerical status (icp_level_stats.status) */
#define ICP_LEVEL_OK 0
#define ICP_TOO_FEW_CORR 1 /* fewer than min_corr pairs kept: the level ends, pose unchanged */
#define ICP_ILL_COND 2     /* an LDL^T pivot <= ill_cond_eps * max diagonal: level ends */
#define ICP_NONFINITE 3    /* the increment was not finite: level ends */

/* lambda as a function of the kept-pair count n (paper Sec. 3.1, Table 4) */
#define ICP_LAMBDA_CONST 0
#define ICP_LAMBDA_C_OVER_SQRT_N 1
#define ICP_LAMBDA_C_OVER_N 2
#define ICP_LAMBDA_C_OVER_N2 3

/* per-pixel association codes written by icp_stage_associate */
#define ICP_PX_INVALID_LIVE 0
#define ICP_PX_BEHIND 1
#define ICP_PX_OUTSIDE 2
#define ICP_PX_INVALID_MODEL 3
#define ICP_PX_FAR 4
#define ICP_PX_ANGLE 5
#define ICP_PX_GATED 6

typedef struct icp_ctx icp_ctx;

typedef struct {
    double fx, fy, cx, cy; /* level-0 pinhole intrinsics, pixels */
} icp_intrinsics;

typedef struct {
    int32_t levels;                 /* pyramid levels (coarse-to-fine, Sec. 3) */
    int32_t iters[ICP_MAX_LEVELS];  /* ICP iterations per level, level 0 (finest) first;
                                       KinectFusion's cadence (4,5,10) coarse to fine is
                                       {10,5,4}, the IMU-seeded one (2,2,3) is {3,2,2} (Sec. 4.4) */
    double dist_max;                /* pair gate: point-to-point distance < dist_max metres (<= 0.125) */
    double cos_angle_max;           /* pair gate: (R n_live) . n_model >= this */
    double band_beta;               /* median filter band (Sec. 3.3): bins
                                       [floor((1-b) k_med), ceil((1+b)(k_med+1)) - 1]; b >= 0 */
    int32_t use_median_filter;      /* 0 keeps every gated pair */
    int32_t use_imu_seed;           /* 1: the initial rotation is imu_R (Sec. 3) */
    int32_t lambda_mode;            /* ICP_LAMBDA_* */
    double lambda_c;                /* c >= 0 (Eq. (4)/(5)) */
    int32_t min_corr;               /* minimum kept pairs for a solve (>= 1) */
    double ill_cond_eps;            /* LDL^T pivot threshold relative to the max diagonal */
    int32_t converge_window;        /* 0: fixed cadence; k >= 1: a level stops once the median
                                       bin is unchanged on k successive iterations (Sec. 3.4) */
    int32_t reduce_mode;            /* 0: FP32 moment reduction; 1: rows centred on the live
                                       centroid moved by the pose, split into FP16 hi + lo and
                                       reduced with MFMA (FP32 accumulation), un-centred in FP64;
                                       in single-pass mode the rows inside the band-edge window
                                       are summed per bin in FP32 (the same centred rows) */
    int32_t pass_mode;              /* 0: single pass over the maps when the band edge falls in a
                                       window around the previous iteration's edge (two passes
                                       otherwise; needs band_beta >= 1 or no median filter);
                                       1: always two passes */
    int32_t tile_px[ICP_MAX_LEVELS];/* pixels per work-group tile per level (multiple of 1024,
                                       at most 65536); 0 = chosen by the library (about 8192
                                       tiles over the batch, 1024..16384 pixels, and at least
                                       4096 at a level whose batch still gives every pass-1
                                       work-group slot of the GPU such a tile) */
    /* live front end (Sec. 3.3: normals by an integral-image method on smoothed depth) */
    int32_t depth_filter;           /* 1: bilateral smoothing of the level-0 depth before the pyramid:
                                       weights exp(-(du^2+dv^2)/(2 s^2)) (s = filter_sigma_px) times
                                       (1-(dz/c)^2)^2 for |dz| < c = filter_sigma_m, over the
                                       (2 filter_radius + 1)^2 window; default 0 */
    int32_t filter_radius;          /* 1..7 (default 3) */
    double filter_sigma_px;         /* > 0 (default 4.5) */
    double filter_sigma_m;          /* > 0 (default 0.05) */
    int32_t normal_mode;            /* 0: forward-difference normals (default); 1: average 3D
                                       gradients over a (2 normal_radius + 1)^2 box (mean of the
                                       valid vertices of the right half minus the left half,
                                       lower minus upper); needs a valid pixel, the box inside the
                                       image and half of each half box valid */
    int32_t normal_radius;          /* 1..7 (default 2) */
    /* regulariser (Eq. (5)) */
    int32_t anchor_to_imu;          /* 0 (default): damp the angles w of each increment, as Eq. (5)
                                       reads; 1: damp the rotation's deviation from the IMU prior
                                       after the update, w + Log(R imu_R^T): the right-hand side
                                       becomes A^T b - 2 lambda n [Log(R imu_R^T); 0] (not for
                                       icp_stage_solve, which has no IMU prior) */
    int32_t reserved;               /* 0 */
} icp_params;

typedef struct {
    int32_t iters_run;
    int32_t status;    /* ICP_LEVEL_* of the last iteration run */
    int64_t n_gated;   /* N: gated pairs (histogram total) of the last iteration run */
    int64_t n_kept;    /* n: pairs kept by the median band in the last iteration run */
    int32_t k_med;     /* median bin of the last iteration run (-1: none) */
    int32_t pad;
    double rmse;       /* sqrt(b^T b / n) of the last iteration run, metres */
} icp_level_stats;

typedef struct {
    icp_level_stats level[ICP_MAX_LEVELS];
    int32_t status;      /* first non-OK level status, coarse to fine, else ICP_LEVEL_OK */
    int32_t iters_total; /* iterations run over all levels */
} icp_stats;

/* one problem of a batch; every pointer is a device pointer except as noted */
typedef struct {
    const float* live_depth;
    const float* model_vtx;
    const float* model_nrm;
    int32_t W, H;
    icp_intrinsics K;
    double imu_R[9];      /* host values */
    double init_pose[16]; /* host values */
} icp_problem;

/* pose (4x4 row-major) and statistics of one registration */
typedef struct {
    double pose[16];
    icp_stats stats;
} icp_result;

/* ---------------------------------------------------------------- context */

/* ABI version of the loaded library (ICP_ABI_VERSION). */
int icp_abi_version(void);

/* Text of a return code (static storage). */
const char* icp_strerror(int code);

/* Last error message of a context (valid until the next call on it). */
const char* icp_last_error(const icp_ctx* ctx);

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
   workspace it may hold (0 = no cap).  *out receives the context. */
int icp_ctx_create(int device, size_t hbm_budget_bytes, icp_ctx** out);

/* Release a context and its device workspace (synchronises the device first).
   NULL is ignored. */
void icp_ctx_destroy(icp_ctx* ctx);

/* Replay registrations as HIP graphs (1, the default) or launch every kernel
   eagerly (0).  With graphs, the launches of a registration are captured
   once per combination of problem sizes, parameters and workspace and
   replayed on later calls (a context keeps the eight most recently used
   graphs); calls with kernel timing enabled launch eagerly. */
int icp_ctx_set_graphs(icp_ctx* ctx, int enable);

/* Bytes of device workspace the context currently holds. */
size_t icp_ctx_workspace_bytes(const icp_ctx* ctx);

/* Bytes of workspace a batch of problems of these sizes needs (W, H arrays of
   length n, host pointers). */
size_t icp_workspace_bytes(int n, const int32_t* W, const int32_t* H, int levels);

/* Fill *p with the defaults: 3 levels, iterations {10,5,4}, dist_max 0.10 m,
   20 degree normal gate, band beta 1, median filter on, IMU seed on,
   lambda = 5 constant (the value of the paper's Freiburg runs, Sec. 5.2),
   min_corr 6, ill_cond_eps 1e-12, no convergence stop, FP32 reduction,
   single-pass mode, tiles chosen by the library. */
void icp_params_default(icp_params* p);

/* Check one problem and the parameters the way icp_register_batch checks
   them, on the host only (no context, no device: the problem's pointers are
   compared with NULL, never read): ICP_OK or ICP_EINVAL, with the reason in
   msg (msg_len bytes, may be NULL/0). */
int icp_validate_problem(const icp_problem* problem, const icp_params* params, char* msg, size_t msg_len);

/* -------------------------------------------------------------- hot path */

/* Register one live depth frame against the model maps (Sec. 3): build the
   live and model pyramids, seed the pose with the IMU rotation, then per
   level (coarse to fine) and per iteration run projective association with
   gates, the distance histogram and median band (Sec. 3.2-3.3), the
   point-to-plane moment reduction (Eq. (3)), the regularised 6x6 solve
   (Eq. (5)) and the SE(3) pose update, all on the device.
   live_depth/model_vtx/model_nrm: device pointers as in the conventions;
   K, imu_R (3x3), init_pose (4x4), params: host pointers.
   pose_out (4x4) and stats_out (may be NULL): host pointers, valid on return
   (the call synchronises `stream`). */
int icp_register(icp_ctx* ctx, const float* live_depth, int W, int H, const float* model_vtx,
                 const float* model_nrm, const icp_intrinsics* K, const double* imu_R,
                 const double* init_pose, const icp_params* params, double* pose_out,
                 icp_stats* stats_out, void* stream);

/* Same as icp_register but asynchronous: result_dev is a device pointer to
   one icp_result, written by the stream; nothing is synchronised. */
int icp_register_async(icp_ctx* ctx, const float* live_depth, int W, int H, const float* model_vtx,
                       const float* model_nrm, const icp_intrinsics* K, const double* imu_R,
                       const double* init_pose, const icp_params* params, icp_result* result_dev,
                       void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the
   registration of icp_register_async with no context and no allocation.  Its
   workspace is one static device array of 32 MiB (ICP_NOALLOC_BYTES) that
   every GPU the library runs on holds from the first call until the process
   ends.  A problem fits when icp_workspace_bytes(1, &W, &H, levels) is at
   most that with tile_px 0 (640x480 and 848x480 do at 3 or 4 levels,
   1280x720 does not); a larger one returns ICP_ENOMEM before anything is
   queued.  Arguments are checked as icp_register checks them (ICP_EINVAL).
   The launches are queued on `stream` (the current device's) and the call
   returns; result_dev, a device pointer to one icp_result, is written by the
   stream.  Every call on one GPU uses that GPU's array and leaves its
   contents behind: calls that overlap on one GPU (different streams, several
   threads) race, so the caller orders them (one stream, or events).  The
   problem descriptor is written by a kernel from its launch arguments, so the
   launches read no host memory. */
#define ICP_NOALLOC_BYTES ((size_t)32 << 20)
int icp_register_noalloc(const float* live_depth, int W, int H, const float* model_vtx, const float* model_nrm,
                         const icp_intrinsics* K, const double* imu_R, const double* init_pose,
                         const icp_params* params, icp_result* result_dev, void* stream);

/* Register n independent problems (possibly of different sizes) with shared
   params in one set of launches: every kernel covers the tiles of all
   problems.  probs: host array of n problems; results: host array of n,
   valid on return (synchronises `stream`). */
int icp_register_batch(icp_ctx* ctx, int n, const icp_problem* probs, const icp_params* params,
                       icp_result* results, void* stream);

/* Same as icp_register_batch but asynchronous: results_dev is a device array
   of n icp_result written by the stream; nothing is synchronised.  The call
   returns once the batch's launches are queued (it waits only until the
   previous call's descriptors have left the context's staging memory), so a
   caller can prepare the next batch while this one runs; calls on one context
   still run one after another on the device. */
int icp_register_batch_async(icp_ctx* ctx, int n, const icp_problem* probs, const icp_params* params,
                             icp_result* results_dev, void* stream);

/* Tile-size autotuner for a batch: for each level, coarsest first, time the
   whole batched registration (HIP events on `stream`, `reps` runs each, the
   median) for every tile size in {1024, 2048, 4096, 8192, 16384} with the
   other levels at their best so far, and keep the fastest.  tile_px_out
   (ICP_MAX_LEVELS entries; unused levels 0) can be copied into
   icp_params.tile_px; *best_ms (may be NULL) receives the time of one
   registration of the batch with them.  The tile size sets how many pixels
   one work-group reduces into one partial sum (it changes the FP32 rounding
   of the moments, not which pixels are used).  Synchronises. */
int icp_autotune_tiles(icp_ctx* ctx, int n, const icp_problem* probs, const icp_params* params, int reps,
                       int32_t* tile_px_out, double* best_ms, void* stream);

/* ------------------------------------------------------ kernel timing
   Tracing for measurement: while enabled, every registration call records
   HIP events on its own stream around each launch of the front end and of
   the four launches of every iteration; durations are accumulated per kind
   once the recorded work has completed (icp_ctx_get_timing waits for it). */

#define ICP_TIME_FRONT_END 0 /* pyramids and vertex/normal maps */
#define ICP_TIME_PASS1 1     /* association, gates, histogram (and single-pass moments) */
#define ICP_TIME_BAND 2      /* per-problem median band (and single-pass solve) */
#define ICP_TIME_PASS2 3     /* band filter and moment reduction */
#define ICP_TIME_SOLVE 4     /* per-problem FP64 sum of partials, solve, update */
#define ICP_TIME_KINDS 5

typedef struct {
    double total_ms;  /* summed launch durations */
    int64_t launches; /* launches recorded */
    int64_t pixels;   /* pixels the recorded launches covered (level pixels) */
} icp_kernel_time;

/* Switch tracing on (1) or off (0); both reset the accumulated times. */
int icp_ctx_set_timing(icp_ctx* ctx, int enable);

/* Accumulated times per kind into out[ICP_TIME_KINDS] (host). */
int icp_ctx_get_timing(icp_ctx* ctx, icp_kernel_time* out);

/* ------------------------------------------------------ stage access
   For parity testing of each step against an independent implementation.
   They use the same kernels and launch configuration as icp_register on one
   problem held in the context. */

/* Build the live and model pyramids of one problem into the context, with
   the front end of params (depth_filter, normal_mode and their constants; NULL:
   defaults).  The later stage calls read the caller's level-0 model maps, which
   must stay alive until the next icp_stage_prepare or registration call. */
int icp_stage_prepare(icp_ctx* ctx, const float* live_depth, int W, int H, const float* model_vtx,
                      const float* model_nrm, const icp_intrinsics* K, int levels, const icp_params* params,
                      void* stream);

/* Copy level `level` of the prepared pyramids to device buffers (any may be
   NULL): depth (H_l*W_l), live vertex/normal as three planes of H_l*W_l
   floats (x plane, y plane, z plane), model vertex/normal interleaved
   (H_l*W_l*3; level 0 is the caller's input).  Synchronises. */
int icp_stage_level(icp_ctx* ctx, int level, float* depth, float* live_vtx, float* live_nrm,
                    float* model_vtx, float* model_nrm, void* stream);

/* One association pass (projective lookup, gates, histogram, median band) at
   `level` for the 3x4 pose12 (host).  code (uint8, H_l*W_l, ICP_PX_* values)
   and bin (int32, -1 unless gated) are device buffers or NULL; hist (host,
   ICP_HIST_BINS) and band (host, {N, k_med, k_lo, k_hi}) may be NULL.
   Synchronises. */
int icp_stage_associate(icp_ctx* ctx, int level, const double* pose12, const icp_params* params,
                        uint8_t* code, int32_t* bin, uint32_t* hist, int64_t* band, void* stream);

/* One filter+reduce pass at `level` for pose12 keeping gated pairs with bins
   in [k_lo, k_hi].  moments (host, 28 doubles: upper triangle of the 7x7
   [a | b]^T [a | b], row-major) and n (host) receive the reduction.
   Synchronises. */
int icp_stage_moments(icp_ctx* ctx, int level, const double* pose12, const icp_params* params,
                      int k_lo, int k_hi, double* moments, int64_t* n, void* stream);

/* One iteration of the single-pass reduction that icp_register runs by
   default (reduce_mode 0, pass_mode 0; paper Eq. (3) over the pairs the median
   band of Sec. 3.3 keeps), at `level` for pose12 (host): pass 1 associates,
   histograms and reduces the rows into per-tile partials -- rows whose bin lies
   below a window of bins around the predicted band edge pred_hi into one sum,
   rows inside the window per bin -- then the band kernel finds the band and,
   when its lower edge is bin 0 and its upper edge lies in the window or just
   below it, sums the partials up to the edge into the moments.  iter = 0 takes
   the full 48-bin window (a level's first iteration); iter > 0 a window of
   2 pred_hw bins (pred_hw 1..24).  pred_hi = -1: no prediction, no window.
   With reduce_mode 1 the rows below the window are reduced by the split
   FP16 hi + lo MFMA, and the moments are returned un-centred.
   The window is [pred_hi - hw, pred_hi + hw) clamped into 0..1023.
   Outputs (host): band {N, k_med, k_lo, k_hi}; window {h0, width} (h0 = -1:
   none); *hit = 1 when the moments came from the partials, else 0 (the
   registration would then run pass 2), with moments and *n zeroed; moments
   (28 doubles, as icp_stage_moments) and *n otherwise.  Needs a prepared stage
   problem and band_beta >= 1 or no median filter (else ICP_EINVAL).
   Synchronises. */
int icp_stage_single_pass(icp_ctx* ctx, int level, const double* pose12, const icp_params* params, int iter,
                          int pred_hi, int pred_hw, int64_t* band, int32_t* window, int* hit, double* moments,
                          int64_t* n, void* stream);

/* The device solve and update on given moments: pose12_out = Exp(x) pose12_in
   with x solving Eq. (5).  All pointers host.  *status receives ICP_LEVEL_*.
   Synchronises. */
int icp_stage_solve(icp_ctx* ctx, const double* moments, int64_t n, const double* pose12_in,
                    const icp_params* params, double* pose12_out, double* x_out, int* status,
                    void* stream);

/* ---------------------------------------------------------------- model maps */

/* Vertex and normal maps of one depth image at full resolution, written
   interleaved (H*W*3 float32 each, device): the same back-projection and
   forward-difference normals (facing the camera, NaN where invalid) that the
   registration computes for its live frame at level 0 (paper Sec. 3, the
   KinectFusion surface measurement).  With them the previous frame of a
   stream serves as the model of the next one (frame-to-frame tracking).
   depth: H*W float32 on the device.  Asynchronous on `stream`. */
int icp_live_maps(icp_ctx* ctx, const float* depth, int W, int H, const icp_intrinsics* K, float* vtx,
                  float* nrm, void* stream);

/* ---------------------------------------------------------------- TSDF model */

/* KinectFusion's reconstruction: a truncated signed distance volume, fused
   from the tracked depth frames and ray-cast into the model maps that the next
   frame registers against (the frame-to-model loop whose tracking the paper
   improves; Sec. 4.3 shows its weights overwritten after a failed alignment,
   Sec. 5.2 sizes it at 512^3 voxels over at most 6 m).  The caller owns the
   voxel memory: icp_tsdf_bytes(dim) bytes on the device, 8 per voxel, a pair
   (tsdf, weight) of float32 for voxel (i, j, k) at pair index
   (k * dim + j) * dim + i (x fastest).  Voxel (i, j, k) is the cube of edge
   side = size / dim whose centre is origin + (i + 1/2, j + 1/2, k + 1/2) side
   in world coordinates.  weight 0 = never observed.  All arithmetic is FP64
   and rounds as written, so results are reproducible bit for bit.
   T_wc: 16 doubles, row-major 4x4 camera-to-world pose, host memory (only
   the top 3x4 is read; its rotation must pass the rotation check of the
   conventions above).  Calls are asynchronous on `stream` and return
   ICP_EINVAL for NULL pointers, dim outside [2, 1024], size, mu or max_weight
   not finite and positive (max_weight >= 1), W, H outside [1, ICP_MAX_DIM],
   bad intrinsics or a T_wc that is not a rigid motion. */
typedef struct {
    float* voxels;        /* device, icp_tsdf_bytes(dim) bytes, 256-byte aligned */
    int32_t dim;          /* voxels per edge */
    int32_t pad_;
    double size;          /* edge of the cube, metres */
    double origin[3];     /* world position of the cube's minimum corner */
    double mu;            /* truncation distance, metres */
    double max_weight;    /* cap of the running-average weight */
    void* bricks;         /* optional device buffer of icp_tsdf_brick_bytes(dim) bytes, 256-byte
                             aligned, or NULL.  Per 8^3 brick it counts the observed voxels with
                             tsdf <= 0 so that the ray cast can jump over bricks that hold none
                             (free or unobserved space); results are identical with and without
                             it.  Its contents are valid only if every change to the voxels went
                             through icp_tsdf_reset / icp_tsdf_integrate with this same buffer
                             attached (attach it before the first reset). */
} icp_tsdf;

size_t icp_tsdf_bytes(int dim);
size_t icp_tsdf_brick_bytes(int dim);

/* Every voxel to (0, 0): nothing observed. */
int icp_tsdf_reset(icp_ctx* ctx, const icp_tsdf* vol, void* stream);

/* Fuse one depth image (H*W float32 metres, device) taken from T_wc.  Each
   voxel centre is moved into the camera; if it is in front (z > 0) and its
   nearest pixel (floor(f x/z + c + 1/2), as in the association) has valid
   depth D, the projective distance sdf = D - z counts unless sdf < -mu:
   f = min(1, sdf / mu), tsdf <- (tsdf w + f) / (w + 1), w <- min(w + 1,
   max_weight).  Voxels not seen keep their values. */
int icp_tsdf_integrate(icp_ctx* ctx, const icp_tsdf* vol, const float* depth, int W, int H,
                       const icp_intrinsics* K, const double* T_wc, void* stream);

/* Predicted maps of a W x H camera with intrinsics K at T_wc, written as
   model maps for icp_register (H*W*3 float32 each, interleaved, camera frame
   of T_wc, NaN where no surface).  The ray of pixel (u, v) is z (x_u, y_v, 1),
   x_u = (u - cx) / fx, sampled at z = tmin + s side / 2 (s = 0, 1, ...) while
   z <= tmax; a sample interpolates the 8 surrounding voxels trilinearly and
   is missing if any of them has weight 0.  The first step from a positive to
   a non-positive sample marks the surface (depth interpolated linearly
   between them); a step from negative to non-negative ends the ray with no
   surface.  The normal is the normalised central difference of samples one
   voxel away along each axis (no normal, and no vertex, if one is missing),
   turned to face the camera.  Requires 0 < tmin < tmax and at most 2^24
   steps. */
int icp_tsdf_raycast(icp_ctx* ctx, const icp_tsdf* vol, int W, int H, const icp_intrinsics* K, const double* T_wc,
                     double tmin, double tmax, float* vtx, float* nrm, void* stream);

/* ---------------------------------------------------------------- serving */

/* A frame server tracks many camera streams frame to frame on one GPU with
   continuous batching.  Each open stream keeps on the device its depth slot
   and its model maps (the vertex / normal maps of its previous frame, built
   with icp_live_maps' arithmetic).  Frames are submitted with the IMU rotation
   of the frame relative to the stream's previous frame (the registration's
   imu_R, paper Sec. 3: the prior that seeds the rotation); init_pose is the
   identity.  A scheduler thread launches one batched registration for every
   stream with waiting frames and no batch on the GPU (oldest request first,
   up to frames_in_flight consecutive frames per stream, at most max_batch),
   on one of `slots` HIP streams, so frames that arrive while a batch runs go
   into the next batch as soon as a slot is free.  The first frame of a
   stream only builds its model maps (pose = identity).

   Admission: icp_server_open_stream fails with ICP_ENOMEM when the resident
   state of every open stream plus, per slot, a workspace that any batch the
   open streams can form fits in would exceed hbm_budget_bytes (0: no limit).
   A stream's resident state is (frames_in_flight + 1) x 28 bytes per pixel;
   the workspace bound counts frames_in_flight frames of every stream (largest
   first, at most max_batch) at the smallest tile size (or params.tile_px),
   and a slot reserves exactly that bound before launching a batch.  The server uses the default front end (params.depth_filter and
   params.normal_mode 0; other values are rejected at creation).  All calls may come from any host thread; results are taken with
   icp_server_poll.  A HIP failure inside the scheduler makes every later call
   return it. */
typedef struct icp_server icp_server;

typedef struct {
    int32_t device;
    int32_t max_batch;          /* most frames per batch, 1..4096 (default 64) */
    int32_t slots;              /* batches in flight at once, 1..4 (default 2) */
    int32_t use_graphs;         /* replay repeated batch shapes as HIP graphs (default 1) */
    int32_t frames_in_flight;   /* most consecutive frames of one stream in one batch, 1..7 (default 2);
                                   a stream holds frames_in_flight + 1 frame slots on the device */
    int32_t pad;
    size_t hbm_budget_bytes;    /* admission budget; 0 = unlimited */
    icp_params params;          /* registration parameters of every stream */
} icp_server_config;

typedef struct {
    int32_t stream_id;
    int32_t status;             /* ICP_OK, or the error that stopped this frame */
    uint64_t frame;             /* 0-based index of the frame in its stream */
    uint64_t tag;               /* the caller's tag */
    double pose_rel[16];        /* the frame's camera in the previous frame's camera (4x4) */
    double pose_world[16];      /* chained: the frame's camera in the stream's first camera */
    icp_stats stats;
    double t_submit;            /* icp_server_clock() seconds: request arrival */
    double t_start;             /* its batch was launched */
    double t_done;              /* its batch was seen complete */
    int32_t batch_size;         /* frames in its batch */
    int32_t pad;
} icp_server_result;

typedef struct {
    uint64_t batches;
    uint64_t frames;            /* results published */
    uint64_t registrations;     /* frames that were registered (not first frames) */
    double busy_s;              /* sum over batches of launch-to-completion time */
    size_t resident_bytes;      /* device state of the open streams */
    size_t workspace_bytes;     /* per-slot batch workspace accounted by admission, all slots */
    int32_t streams_open;
    int32_t pad;
    size_t workspace_held_bytes; /* device workspace the slots hold now (<= workspace_bytes) */
} icp_server_counters;

void icp_server_config_default(icp_server_config* cfg);
/* The server clock (seconds, monotonic) used for t_submit / t_start / t_done. */
double icp_server_clock(void);
int icp_server_create(const icp_server_config* cfg, icp_server** out);
/* Waits for batches on the GPU, then frees everything (pending frames are dropped). */
void icp_server_destroy(icp_server* srv);
const char* icp_server_last_error(icp_server* srv);
/* Admit a W x H stream with intrinsics K; *stream_id receives its id. */
int icp_server_open_stream(icp_server* srv, int W, int H, const icp_intrinsics* K, int* stream_id);
/* Frames already submitted are still served; the state is freed after the last. */
int icp_server_close_stream(icp_server* srv, int stream_id);
/* Queue the stream's next frame: depth_host (H*W float32, host memory, copied
   before the call returns), imu_rel_R (3x3 row-major, host), a caller tag and
   the arrival time on icp_server_clock() (<= 0: now). */
int icp_server_submit(icp_server* srv, int stream_id, const float* depth_host, const double* imu_rel_R,
                      uint64_t tag, double t_submit);
/* Move up to max finished results into out; waits up to timeout_ms for the
   first (0: no wait, < 0: forever).  Returns the count (>= 0) or an error. */
int icp_server_poll(icp_server* srv, icp_server_result* out, int max, int timeout_ms);
int icp_server_get_counters(icp_server* srv, icp_server_counters* out);

#ifdef __cplusplus
}
#endif
#endif
