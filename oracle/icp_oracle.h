/*
 * icp_oracle.h -- plain FP64 CPU oracle of the IMU-seeded, median-filtered,
 * regularised point-to-plane ICP of Giancola, Schneider, Wonka and Ghanem,
 * "Integration of Absolute Orientation Measurements in the KinectFusion
 * Reconstruction pipeline" (2018).
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library; the GPU library never links, loads or
 * calls it and the two share no code, header, table or constant.
 *
 * Parity unpinned: the width of the median band (or_band).  The paper gives
 * no formula or printed values for it; the band is pinned only to its own
 * definition (hand-worked fixtures) and to the paper's one illustration of
 * the filter (about three quarters of the pairs kept).  Every other function
 * is pinned by the tests to closed forms, worked fixtures or invariants.
 *
 * Every array is a host pointer.  Maps are row-major, pixel (u, v) at index
 * v*W + u.  "SoA" maps hold three planes of W*H floats (x plane, y plane,
 * z plane).  Poses are 3x4 row-major [R | t] (12 doubles) unless stated.
 */
#ifndef ICP_ORACLE_H
#define ICP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_LEVELS 4
#define OR_BINS 1024

/* per-pixel association outcome: the first test a pixel fails, or GATED */
enum {
    OR_INVALID_LIVE = 0,  /* live vertex or normal invalid */
    OR_BEHIND = 1,        /* transformed point not in front of the model camera */
    OR_OUTSIDE = 2,       /* projects outside the model image */
    OR_INVALID_MODEL = 3, /* model pixel invalid */
    OR_FAR = 4,           /* point-to-point distance not below d_max */
    OR_ANGLE = 5,         /* normals disagree by more than the angle gate */
    OR_GATED = 6          /* matched pair, enters the distance histogram */
};

/* level status */
enum { OR_LEVEL_OK = 0, OR_TOO_FEW_CORR = 1, OR_ILL_COND = 2, OR_NONFINITE = 3 };

/* lambda as a function of the number n of kept pairs (Table 4's forms) */
enum { OR_LAMBDA_CONST = 0, OR_LAMBDA_C_OVER_SQRT_N = 1, OR_LAMBDA_C_OVER_N = 2,
       OR_LAMBDA_C_OVER_N2 = 3 };

typedef struct {
    int levels;                 /* pyramid levels, 1..4 */
    int iters[OR_MAX_LEVELS];   /* iterations per level, finest (level 0) first */
    double dist_max;            /* gate on the point-to-point distance, metres (<= 0.125) */
    double cos_angle_max;       /* gate: cosine between normals must be >= this */
    double band_beta;           /* median band half-width factor (dyadic) */
    int use_median_filter;      /* 0: keep every gated pair */
    int use_imu_seed;           /* 1: initial rotation := IMU rotation */
    int lambda_mode;            /* OR_LAMBDA_* */
    double lambda_c;            /* the constant c of the lambda form */
    int min_corr;               /* fewer kept pairs end the level */
    double ill_cond_eps;        /* LDLT pivot threshold relative to max diagonal */
    int converge_window;        /* 0: fixed cadence; k: stop a level once the median
                                   bin was equal on k successive iterations */
    int depth_filter;           /* 1: bilateral smoothing of the level-0 depth first */
    int filter_radius;          /* its window is (2r+1)^2 pixels */
    double filter_sigma_px;     /* spatial Gaussian sigma, pixels */
    double filter_sigma_m;      /* range kernel cut-off, metres */
    int normal_mode;            /* 0: forward differences; 1: box-average 3D gradients */
    int normal_radius;          /* the boxes of normal_mode 1 span (2r+1) pixels */
    int anchor_to_imu;          /* 0: Eq. (5) damps each increment's angles (literal);
                                   1: it damps the deviation from the IMU rotation */
} or_params;

typedef struct {
    int32_t iters_run;
    int32_t status;
    int64_t n_gated;   /* N of the last iteration run */
    int64_t n_kept;    /* n of the last iteration run */
    int32_t k_med;     /* median bin of the last iteration run */
    int32_t pad;
    double rmse;       /* sqrt(b^T b / n) of the last iteration run */
} or_level_stats;

typedef struct {
    int32_t level, iter, status, k_med, k_lo, k_hi;
    int64_t n_gated, n_kept;
    double x[6];       /* increment (alpha, beta, gamma, tx, ty, tz) */
    double pose[12];   /* pose after the iteration */
} or_iter_trace;

void or_params_default(or_params* p);
/* threads the per-pixel loops use (OpenMP) */
int or_num_threads(void);
void or_set_num_threads(int n); /* OpenMP threads of later calls (timing only) */
void or_level_intrinsics(const double K0[4], int level, double Kl[4]);

/* live front end */
void or_depth_down(const float* D, int W, int H, float* Dn);
void or_live_vn(const float* D, int W, int H, const double K[4], float* V, float* N);
/* bilateral smoothing of a depth image (see the definition in icp_oracle.c) */
void or_bilateral(const float* D, int W, int H, int r, double sigma_px, double sigma_m, float* out);
/* vertex map and box-average 3D-gradient normals (normal_mode 1) */
void or_live_vn_box(const float* D, int W, int H, const double K[4], int r, float* V, float* N);
/* model maps */
void or_model_l0(const float* vtx_aos, const float* nrm_aos, int W, int H, float* V, float* N);
void or_model_down(const float* V, const float* N, int W, int H, float* Vn, float* Nn);

/* one association pass at one level; code/bin/margin per pixel (any may be NULL),
   hist (OR_BINS counts, overwritten) may be NULL */
void or_associate(const float* LV, const float* LN, const float* MV, const float* MN, int W, int H,
                  const double K[4], const double T[12], double dist_max, double cos_max,
                  uint8_t* code, int32_t* bin, double* margin, uint32_t* hist);
/* the histogram bin of a squared distance */
int or_bin_of(double d2);
/* code, bin and (GATED pixels only) p', q, n_q as (H*W, 3) arrays */
void or_pairs(const float* LV, const float* LN, const float* MV, const float* MN, int W, int H,
              const double K[4], const double T[12], double dist_max, double cos_max, uint8_t* code,
              int32_t* bin, double* pp, double* q, double* nq);
/* out = {N, k_med, k_lo, k_hi} */
void or_band(const uint32_t* hist, int use_filter, double beta, int64_t out[4]);
/* 28 moments of the kept rows [a | b]: upper triangle of the 7x7 matrix, row-major */
void or_moments(const float* LV, const float* LN, const float* MV, const float* MN, int W, int H,
                const double K[4], const double T[12], double dist_max, double cos_max,
                int k_lo, int k_hi, double M[28], int64_t* n);
/* regularised solve and pose update; returns level status */
int or_solve_update(const double M[28], int64_t n, const double T_in[12], int lambda_mode,
                    double lambda_c, int min_corr, double eps, double T_out[12], double x[6]);
void or_se3_exp(const double w[3], const double tau[3], double R[9], double t[3]);
/* rotation vector of a rotation matrix (angle in [0, pi)) */
void or_so3_log(const double R[9], double w[3]);
/* or_solve_update with the damping anchored to the IMU rotation imu_R */
int or_solve_update_anchor(const double M[28], int64_t n, const double T_in[12], int lambda_mode,
                           double lambda_c, int min_corr, double eps, const double imu_R[9],
                           double T_out[12], double x[6]);

/* TSDF volume (the model the tracking aligns to, Sec. 5.2: a 512^3 cube of at
   most 6 m).  dim^3 voxels of side size/dim, voxel (i, j, k) (i fastest) centred
   at origin + (i + 1/2, j + 1/2, k + 1/2) * side; tsdf and weight arrays of
   dim^3 floats.  T_wc: camera-to-world pose, 4x4 row-major. */
void or_tsdf_integrate(float* tsdf, float* weight, int dim, double size, const double origin[3], double mu,
                       double max_weight, const float* depth, int W, int H, const double K[4],
                       const double T_wc[16]);
/* model maps (H*W*3, camera frame of T_wc, NaN where no surface) by ray casting */
void or_tsdf_raycast(const float* tsdf, const float* weight, int dim, double size, const double origin[3],
                     double tmin, double tmax, int W, int H, const double K[4], const double T_wc[16], float* vtx,
                     float* nrm);

/* whole registration; pose_out is 4x4 row-major; trace may be NULL.
   Returns the number of trace records written (or would have written). */
int or_icp_register(const float* depth, int W, int H, const float* model_vtx, const float* model_nrm,
                    const double K[4], const double imu_R[9], const double init_pose[16],
                    const or_params* p, double pose_out[16], or_level_stats* stats,
                    or_iter_trace* trace, int trace_cap);

#ifdef __cplusplus
}
#endif
#endif
