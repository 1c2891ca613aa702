/*
 * icp_oracle.c -- plain FP64 CPU oracle of the IMU-seeded, median-filtered,
 * regularised point-to-plane ICP (Giancola, Schneider, Wonka, Ghanem 2018).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg.  The GPU library shares no code with it.
 *
 * Arithmetic is FP64.  The maps the method keeps between steps (depth
 * pyramid, vertex and normal maps) are stored as FP32, like its FP32 inputs;
 * every such rounding point is marked "stored FP32".  Build with
 * -ffp-contract=off -fno-fast-math so that each expression is evaluated
 * exactly as written, in the order written.
 *
 * Paper map (section / equation of the paper):
 *   Sec. 3, Eq. (1)  point-to-plane objective over matched pairs
 *   Sec. 3           IMU pre-orientation of the live points (seed)
 *   Sec. 3, Eq. (2)  small-angle transform, increment x = (alpha,beta,gamma,t)
 *   Sec. 3, Eq. (3)  linear least squares in x; A^T A, A^T b reduced on the GPU
 *   Sec. 3.1, Eq. (4), (5)  rotation-regularised normal equations
 *   Sec. 3.2         histogram (PDF) and cumulative (CDF) of pair distances
 *   Sec. 3.3         median from the CDF, pairs far from it rejected
 *   Sec. 3.4         a level converges when the median stays put 3 iterations
 *   Sec. 4.4         coarse-to-fine cadence (4,5,10) iterations
 * Where the paper is silent (A and b of Eq. (3), bins, the band, gates,
 * pyramid, normals) the reading taken is stated beside the code.
 *
 * Parity unpinned: the median band's width (or_band), which the paper does
 * not define beyond one illustration; see icp_oracle.h.
 */
#include "icp_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Histogram of Sec. 3.2: OR_BINS bins of width 2^-13 m over [0, 0.125) m. */
static const double BIN_W = 1.0 / 8192.0;

static float f_nan(void) { return (float)NAN; }

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void or_params_default(or_params* p) {
    memset(p, 0, sizeof(*p));
    p->levels = 3;
    p->iters[0] = 10;  /* cadence (4,5,10) coarse to fine, Sec. 4.4 */
    p->iters[1] = 5;
    p->iters[2] = 4;
    p->dist_max = 0.10;
    p->cos_angle_max = cos(20.0 * M_PI / 180.0);
    p->band_beta = 1.0;
    p->use_median_filter = 1;
    p->use_imu_seed = 1;
    p->lambda_mode = OR_LAMBDA_CONST;
    p->lambda_c = 5.0;  /* lambda = 5 in the Freiburg evaluation, Sec. 5.2 */
    p->min_corr = 6;
    p->ill_cond_eps = 1e-12;
    p->converge_window = 0;
    p->depth_filter = 0;
    p->filter_radius = 3;
    p->filter_sigma_px = 4.5;
    p->filter_sigma_m = 0.05;
    p->normal_mode = 0;
    p->normal_radius = 2;
    p->anchor_to_imu = 0;
}

/* Level l pixel (u, v) averages level-(l-1) pixels 2u..2u+1, 2v..2v+1; its
   centre is at 2u + 1/2 in the finer grid, which gives these intrinsics. */
void or_level_intrinsics(const double K0[4], int level, double Kl[4]) {
    double s = ldexp(1.0, -level);
    Kl[0] = K0[0] * s;
    Kl[1] = K0[1] * s;
    Kl[2] = (K0[2] + 0.5) * s - 0.5;
    Kl[3] = (K0[3] + 0.5) * s - 0.5;
}

static int depth_ok(float z) { return isfinite(z) && z > 0.0f; }

/* ---------------------------------------------------------------------------
 * Live front end.  The paper reuses KinectFusion's pyramid and vertex/normal
 * maps (Sec. 3).  Reading taken: 2x2 mean of the four children when all four
 * are valid; back-projected vertices; normals from the forward-difference
 * cross product, flipped to face the camera.
 * ------------------------------------------------------------------------- */
void or_depth_down(const float* D, int W, int H, float* Dn) {
    int Wn = W / 2, Hn = H / 2;
    for (int v = 0; v < Hn; ++v) {
        for (int u = 0; u < Wn; ++u) {
            float a = D[(2 * v) * W + 2 * u];
            float b = D[(2 * v) * W + 2 * u + 1];
            float c = D[(2 * v + 1) * W + 2 * u];
            float d = D[(2 * v + 1) * W + 2 * u + 1];
            float out = 0.0f;
            if (depth_ok(a) && depth_ok(b) && depth_ok(c) && depth_ok(d)) {
                double s = (((double)a + (double)b) + (double)c) + (double)d;
                out = (float)(s * 0.25); /* stored FP32 */
            }
            Dn[v * Wn + u] = out;
        }
    }
}

/* vertex of pixel (u, v): z * ((u - cx)/fx, (v - cy)/fy, 1), stored FP32 */
static int live_vertex(const float* D, int W, int u, int v, const double K[4], float out[3]) {
    float z = D[v * W + u];
    if (!depth_ok(z)) {
        out[0] = out[1] = out[2] = f_nan();
        return 0;
    }
    double zd = (double)z;
    out[0] = (float)(zd * (((double)u - K[2]) / K[0]));
    out[1] = (float)(zd * (((double)v - K[3]) / K[1]));
    out[2] = z;
    return 1;
}

void or_live_vn(const float* D, int W, int H, const double K[4], float* V, float* N) {
    size_t S = (size_t)W * H;
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            size_t i = (size_t)v * W + u;
            float p[3], pr[3], pd[3];
            int ok = live_vertex(D, W, u, v, K, p);
            V[i] = p[0];
            V[S + i] = p[1];
            V[2 * S + i] = p[2];
            N[i] = N[S + i] = N[2 * S + i] = f_nan();
            if (!ok || u + 1 >= W || v + 1 >= H) continue;
            if (!live_vertex(D, W, u + 1, v, K, pr) || !live_vertex(D, W, u, v + 1, K, pd)) continue;
            double e1[3], e2[3], c[3];
            for (int k = 0; k < 3; ++k) {
                e1[k] = (double)pr[k] - (double)p[k];
                e2[k] = (double)pd[k] - (double)p[k];
            }
            c[0] = e1[1] * e2[2] - e1[2] * e2[1];
            c[1] = e1[2] * e2[0] - e1[0] * e2[2];
            c[2] = e1[0] * e2[1] - e1[1] * e2[0];
            double len2 = (c[0] * c[0] + c[1] * c[1]) + c[2] * c[2];
            if (!(len2 > 0.0) || !isfinite(len2)) continue;
            double len = sqrt(len2);
            double n[3] = {c[0] / len, c[1] / len, c[2] / len};
            double side = (n[0] * (double)p[0] + n[1] * (double)p[1]) + n[2] * (double)p[2];
            if (side > 0.0) {
                n[0] = -n[0];
                n[1] = -n[1];
                n[2] = -n[2];
            }
            N[i] = (float)n[0]; /* stored FP32 */
            N[S + i] = (float)n[1];
            N[2 * S + i] = (float)n[2];
        }
    }
}

/* ---------------------------------------------------------------------------
 * The paper's front end (Sec. 3.3: normals by an integral-image method, on
 * KinectFusion's smoothed depth).  Readings taken:
 *  - Smoothing is a bilateral filter over the (2r+1)^2 window: weight of a
 *    valid neighbour q of a valid pixel p = exp(-(du^2 + dv^2) / (2 s^2))
 *    (spatial Gaussian, s in pixels) times (1 - (dz/c)^2)^2 for
 *    |dz| = |z_q - z_p| < c, else 0 (a biweight range kernel: polynomial, so
 *    any implementation reproduces it exactly); out = sum(w z) / sum(w),
 *    sums in FP64 in row-major window order; invalid pixels stay invalid.
 *  - Normals: the average 3D gradient of the integral-image method with a
 *    fixed smoothing box: the horizontal tangent is the mean of the valid
 *    vertices in the right half of the (2r+1)^2 box minus the mean over the
 *    left half (rows v-r..v+r, columns u+1..u+r and u-r..u-1), the vertical
 *    one the lower half minus the upper half; n = normalise(h x g), flipped to
 *    face the camera.  Like the method's valid-count integral images, the
 *    means run over the valid pixels only; the pixel needs a valid vertex, a
 *    box inside the image and at least half of each half box valid.  The box
 *    sums are written out directly (an integral image gives the same sums
 *    faster), in row-major order.
 * ------------------------------------------------------------------------- */
void or_bilateral(const float* D, int W, int H, int r, double sigma_px, double sigma_m, float* out) {
    int n = 2 * r + 1;
    double* ws = (double*)malloc((size_t)n * n * sizeof(double));
    for (int dv = -r; dv <= r; ++dv)
        for (int du = -r; du <= r; ++du)
            ws[(dv + r) * n + (du + r)] = exp(-(double)(du * du + dv * dv) / (2.0 * sigma_px * sigma_px));
#pragma omp parallel for schedule(static)
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            size_t i = (size_t)v * W + u;
            float z = D[i];
            if (!depth_ok(z)) {
                out[i] = 0.0f;
                continue;
            }
            double sw = 0.0, swz = 0.0;
            for (int dv = -r; dv <= r; ++dv) {
                int y = v + dv;
                if (y < 0 || y >= H) continue;
                for (int du = -r; du <= r; ++du) {
                    int x = u + du;
                    if (x < 0 || x >= W) continue;
                    float zq = D[(size_t)y * W + x];
                    if (!depth_ok(zq)) continue;
                    double dz = (double)zq - (double)z;
                    if (!(fabs(dz) < sigma_m)) continue;
                    double t = dz / sigma_m;
                    double a = 1.0 - t * t;
                    double w = ws[(dv + r) * n + (du + r)] * (a * a);
                    sw += w;
                    swz += w * (double)zq;
                }
            }
            out[i] = (float)(swz / sw);
        }
    }
    free(ws);
}

void or_live_vn_box(const float* D, int W, int H, const double K[4], int r, float* V, float* N) {
    size_t S = (size_t)W * H;
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            size_t i = (size_t)v * W + u;
            float p[3];
            live_vertex(D, W, u, v, K, p);
            V[i] = p[0];
            V[S + i] = p[1];
            V[2 * S + i] = p[2];
        }
#pragma omp parallel for schedule(static)
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            size_t i = (size_t)v * W + u;
            N[i] = N[S + i] = N[2 * S + i] = f_nan();
            if (u - r < 0 || u + r >= W || v - r < 0 || v + r >= H) continue;
            if (!isfinite(V[2 * S + i])) continue;
            /* valid pixels of each half box, and the vertex sums over them */
            int nr = 0, nl = 0, nd = 0, nu = 0;
            double sr[3] = {0, 0, 0}, sl[3] = {0, 0, 0}, sd[3] = {0, 0, 0}, su[3] = {0, 0, 0};
            for (int dv = -r; dv <= r; ++dv)
                for (int du = -r; du <= r; ++du) {
                    size_t j = (size_t)(v + dv) * W + (u + du);
                    if (!isfinite(V[2 * S + j])) continue;
                    for (int k = 0; k < 3; ++k) {
                        double x = (double)V[(size_t)k * S + j];
                        if (du > 0) sr[k] += x;
                        if (du < 0) sl[k] += x;
                        if (dv > 0) sd[k] += x;
                        if (dv < 0) su[k] += x;
                    }
                    nr += du > 0;
                    nl += du < 0;
                    nd += dv > 0;
                    nu += dv < 0;
                }
            int need = (r * (2 * r + 1) + 1) / 2;
            if (nr < need || nl < need || nd < need || nu < need) continue;
            double h[3], g[3];
            for (int k = 0; k < 3; ++k) {
                h[k] = sr[k] / nr - sl[k] / nl;
                g[k] = sd[k] / nd - su[k] / nu;
            }
            double c[3];
            c[0] = h[1] * g[2] - h[2] * g[1];
            c[1] = h[2] * g[0] - h[0] * g[2];
            c[2] = h[0] * g[1] - h[1] * g[0];
            double len2 = (c[0] * c[0] + c[1] * c[1]) + c[2] * c[2];
            if (!(len2 > 0.0) || !isfinite(len2)) continue;
            double len = sqrt(len2);
            double nn[3] = {c[0] / len, c[1] / len, c[2] / len};
            double side = (nn[0] * (double)V[i] + nn[1] * (double)V[S + i]) + nn[2] * (double)V[2 * S + i];
            if (side > 0.0) {
                nn[0] = -nn[0];
                nn[1] = -nn[1];
                nn[2] = -nn[2];
            }
            N[i] = (float)nn[0];
            N[S + i] = (float)nn[1];
            N[2 * S + i] = (float)nn[2];
        }
    }
}

/* ---------------------------------------------------------------------------
 * TSDF volume (KinectFusion's model; Sec. 5.2 sizes it 512^3 over at most
 * 6 m).  Readings taken (the paper defers to KinectFusion):
 *  - integration, per voxel centre x_w: x_c = R^T (x_w - t) in the camera of
 *    T_wc = [R | t]; skip unless x_c.z > 0 and the projection (rounded as in
 *    the association) lands on a valid depth z; sdf = z - x_c.z (projective,
 *    along z); skip if sdf < -mu; f = min(1, sdf / mu); running average
 *    tsdf = (tsdf w + f) / (w + 1), w = min(w + 1, max_weight); FP64 math,
 *    FP32 storage;
 *  - ray casting, per pixel: the ray z (x_u, y_v, 1) in the camera, sampled at
 *    z = tmin + s * side / 2 (s = 0, 1, ...) up to tmax, marched in grid
 *    coordinates (voxel units, voxel centres at integers); a sample is the
 *    trilinear interpolation of the 8 voxels around the point (all observed,
 *    weight > 0, else the sample is missing); the first change from > 0 to
 *    <= 0 between consecutive samples is the surface, at the linearly
 *    interpolated depth; a change from < 0 to >= 0 (a back face) ends the ray
 *    without a surface; vertex = z* (x_u, y_v, 1); normal = the normalised
 *    central-difference gradient (one voxel on each side, six samples) turned
 *    into the camera frame and facing the camera.
 * ------------------------------------------------------------------------- */
void or_tsdf_integrate(float* tsdf, float* weight, int dim, double size, const double origin[3], double mu,
                       double max_weight, const float* depth, int W, int H, const double K[4],
                       const double T_wc[16]) {
    double side = size / dim;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < dim; ++k) {
        for (int j = 0; j < dim; ++j) {
            for (int i = 0; i < dim; ++i) {
                double xw[3] = {origin[0] + ((double)i + 0.5) * side, origin[1] + ((double)j + 0.5) * side,
                                origin[2] + ((double)k + 0.5) * side};
                double dx[3] = {xw[0] - T_wc[3], xw[1] - T_wc[7], xw[2] - T_wc[11]};
                double xc[3];
                for (int a = 0; a < 3; ++a)
                    xc[a] = (T_wc[a] * dx[0] + T_wc[4 + a] * dx[1]) + T_wc[8 + a] * dx[2];
                if (!(xc[2] > 0.0)) continue;
                double uu = floor(K[0] * (xc[0] / xc[2]) + K[2] + 0.5);
                double vv = floor(K[1] * (xc[1] / xc[2]) + K[3] + 0.5);
                if (!(uu >= 0.0 && uu <= (double)(W - 1) && vv >= 0.0 && vv <= (double)(H - 1))) continue;
                float z = depth[(size_t)vv * W + (size_t)uu];
                if (!depth_ok(z)) continue;
                double sdf = (double)z - xc[2];
                if (sdf < -mu) continue;
                double f = sdf / mu;
                if (f > 1.0) f = 1.0;
                size_t idx = ((size_t)k * dim + j) * dim + i;
                double w = (double)weight[idx];
                tsdf[idx] = (float)(((double)tsdf[idx] * w + f) / (w + 1.0));
                double wn = w + 1.0;
                weight[idx] = (float)(wn < max_weight ? wn : max_weight);
            }
        }
    }
}

/* trilinear TSDF at grid point g (voxel (i, j, k) has its centre at grid
   point (i, j, k)); returns 0 when a corner voxel is unobserved or g is out of
   the interior */
static int tsdf_sample(const float* tsdf, const float* weight, int dim, const double g[3], double* out) {
    double fr[3];
    int i0[3];
    for (int a = 0; a < 3; ++a) {
        double fl = floor(g[a]);
        if (!(fl >= 0.0 && fl < (double)(dim - 1))) return 0;
        i0[a] = (int)fl;
        fr[a] = g[a] - fl;
    }
    double c[8];
    for (int n = 0; n < 8; ++n) {
        int ii = i0[0] + (n & 1), jj = i0[1] + ((n >> 1) & 1), kk = i0[2] + ((n >> 2) & 1);
        size_t idx = ((size_t)kk * dim + jj) * dim + ii;
        if (!(weight[idx] > 0.0f)) return 0;
        c[n] = (double)tsdf[idx];
    }
    double c00 = c[0] * (1.0 - fr[0]) + c[1] * fr[0];
    double c10 = c[2] * (1.0 - fr[0]) + c[3] * fr[0];
    double c01 = c[4] * (1.0 - fr[0]) + c[5] * fr[0];
    double c11 = c[6] * (1.0 - fr[0]) + c[7] * fr[0];
    double c0 = c00 * (1.0 - fr[1]) + c10 * fr[1];
    double c1 = c01 * (1.0 - fr[1]) + c11 * fr[1];
    *out = c0 * (1.0 - fr[2]) + c1 * fr[2];
    return 1;
}

/* The ray is marched in grid coordinates: with inv = 1/side (rounded once),
   the camera centre sits at gc = (t_wc - origin) inv - 1/2 and the ray
   direction is gd = d_w inv, so the step at depth z is the grid point
   gc + z gd. */
void or_tsdf_raycast(const float* tsdf, const float* weight, int dim, double size, const double origin[3],
                     double tmin, double tmax, int W, int H, const double K[4], const double T_wc[16], float* vtx,
                     float* nrm) {
    double side = size / dim;
    double inv = 1.0 / side;
    double dz = 0.5 * side;
    double gc[3];
    for (int a = 0; a < 3; ++a) gc[a] = (T_wc[4 * a + 3] - origin[a]) * inv - 0.5;
#pragma omp parallel for schedule(dynamic, 4)
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            size_t i = (size_t)v * W + u;
            for (int a = 0; a < 3; ++a) vtx[3 * i + a] = nrm[3 * i + a] = f_nan();
            double dc[3] = {((double)u - K[2]) / K[0], ((double)v - K[3]) / K[1], 1.0};
            double gd[3];
            for (int a = 0; a < 3; ++a) gd[a] = ((T_wc[4 * a] * dc[0] + T_wc[4 * a + 1] * dc[1]) + T_wc[4 * a + 2]) * inv;
            int have_prev = 0;
            double t_prev = 0.0, f_prev = 0.0, t_hit = -1.0;
            for (int s_ = 0;; ++s_) {
                double t = tmin + (double)s_ * dz;
                if (t > tmax) break;
                double g[3] = {gc[0] + t * gd[0], gc[1] + t * gd[1], gc[2] + t * gd[2]};
                double f;
                if (!tsdf_sample(tsdf, weight, dim, g, &f)) {
                    have_prev = 0;
                    continue;
                }
                if (have_prev && f_prev > 0.0 && f <= 0.0) {
                    t_hit = t_prev + (t - t_prev) * (f_prev / (f_prev - f));
                    break;
                }
                if (have_prev && f_prev < 0.0 && f >= 0.0) break;
                have_prev = 1;
                t_prev = t;
                f_prev = f;
            }
            if (!(t_hit > 0.0)) continue;
            double gh[3] = {gc[0] + t_hit * gd[0], gc[1] + t_hit * gd[1], gc[2] + t_hit * gd[2]};
            double gw[3];
            int ok = 1;
            for (int a = 0; a < 3 && ok; ++a) {
                double q1[3] = {gh[0], gh[1], gh[2]}, q0[3] = {gh[0], gh[1], gh[2]};
                q1[a] += 1.0;
                q0[a] -= 1.0;
                double f1, f0;
                ok = tsdf_sample(tsdf, weight, dim, q1, &f1) && tsdf_sample(tsdf, weight, dim, q0, &f0);
                gw[a] = f1 - f0;
            }
            if (!ok) continue;
            double len2 = (gw[0] * gw[0] + gw[1] * gw[1]) + gw[2] * gw[2];
            if (!(len2 > 0.0)) continue;
            double len = sqrt(len2);
            double nw[3] = {gw[0] / len, gw[1] / len, gw[2] / len};
            double nc[3], pc[3];
            for (int a = 0; a < 3; ++a) {
                nc[a] = (T_wc[a] * nw[0] + T_wc[4 + a] * nw[1]) + T_wc[8 + a] * nw[2];
                pc[a] = t_hit * dc[a];
            }
            double sd = (nc[0] * pc[0] + nc[1] * pc[1]) + nc[2] * pc[2];
            if (sd > 0.0)
                for (int a = 0; a < 3; ++a) nc[a] = -nc[a];
            for (int a = 0; a < 3; ++a) {
                vtx[3 * i + a] = (float)pc[a];
                nrm[3 * i + a] = (float)nc[a];
            }
        }
    }
}

/* ---------------------------------------------------------------------------
 * Model maps (the raycast prediction of Sec. 3's frame-to-model alignment;
 * an input here).  A pixel is valid iff all six components are finite.
 * ------------------------------------------------------------------------- */
void or_model_l0(const float* vtx, const float* nrm, int W, int H, float* V, float* N) {
    size_t S = (size_t)W * H;
    for (size_t i = 0; i < S; ++i) {
        int ok = 1;
        for (int k = 0; k < 3; ++k) ok = ok && isfinite(vtx[3 * i + k]) && isfinite(nrm[3 * i + k]);
        for (int k = 0; k < 3; ++k) {
            V[k * S + i] = ok ? vtx[3 * i + k] : f_nan();
            N[k * S + i] = ok ? nrm[3 * i + k] : f_nan();
        }
    }
}

static int model_ok(const float* V, const float* N, size_t S, size_t i) {
    for (int k = 0; k < 3; ++k)
        if (!isfinite(V[k * S + i]) || !isfinite(N[k * S + i])) return 0;
    return 1;
}

void or_model_down(const float* V, const float* N, int W, int H, float* Vn, float* Nn) {
    size_t S = (size_t)W * H;
    int Wn = W / 2, Hn = H / 2;
    size_t Sn = (size_t)Wn * Hn;
    for (int v = 0; v < Hn; ++v) {
        for (int u = 0; u < Wn; ++u) {
            size_t o = (size_t)v * Wn + u;
            size_t ch[4] = {(size_t)(2 * v) * W + 2 * u, (size_t)(2 * v) * W + 2 * u + 1,
                            (size_t)(2 * v + 1) * W + 2 * u, (size_t)(2 * v + 1) * W + 2 * u + 1};
            int ok = 1;
            for (int j = 0; j < 4; ++j) ok = ok && model_ok(V, N, S, ch[j]);
            for (int k = 0; k < 3; ++k) Vn[k * Sn + o] = Nn[k * Sn + o] = f_nan();
            if (!ok) continue;
            double s[3];
            for (int k = 0; k < 3; ++k) {
                double m = (((double)V[k * S + ch[0]] + (double)V[k * S + ch[1]]) + (double)V[k * S + ch[2]]) +
                           (double)V[k * S + ch[3]];
                s[k] = (((double)N[k * S + ch[0]] + (double)N[k * S + ch[1]]) + (double)N[k * S + ch[2]]) +
                       (double)N[k * S + ch[3]];
                Vn[k * Sn + o] = (float)(m * 0.25); /* stored FP32 */
            }
            double len2 = (s[0] * s[0] + s[1] * s[1]) + s[2] * s[2];
            if (!(len2 > 0.0)) {
                for (int k = 0; k < 3; ++k) Vn[k * Sn + o] = f_nan();
                continue;
            }
            double len = sqrt(len2);
            for (int k = 0; k < 3; ++k) Nn[k * Sn + o] = (float)(s[k] / len); /* stored FP32 */
        }
    }
}

/* ---------------------------------------------------------------------------
 * Projective association (the closest-point step of Sec. 3; KinectFusion's
 * projective lookup is used for the paper's normal shooting).  The live point
 * p is moved by the current pose T = [R | t] (which starts at the IMU
 * rotation, Sec. 3), projected into the model image, rounded to the nearest
 * pixel and paired with that pixel's model point q and normal n_q.
 * ------------------------------------------------------------------------- */
typedef struct {
    int code;
    int bin;
    double pp[3];  /* p' = R p + t */
    double q[3];
    double nq[3];
    double d2;
    double margin; /* smallest distance (metres) of a deciding quantity to its threshold */
} px_assoc;

/* bin k of a squared distance: the unique k with (k w)^2 <= d2 < ((k+1) w)^2.
   With w = 2^-13 the squares are exact in FP64, so k depends on d2 only. */
static int bin_of(double d2) {
    int k = (int)floor(sqrt(d2) / BIN_W);
    while (k > 0 && ((double)k * BIN_W) * ((double)k * BIN_W) > d2) --k;
    while (((double)(k + 1) * BIN_W) * ((double)(k + 1) * BIN_W) <= d2) ++k;
    return k;
}

static double dmin(double a, double b) { return a < b ? a : b; }

static void associate_px(const float* LV, const float* LN, const float* MV, const float* MN, int W, int H,
                         size_t i, const double K[4], const double T[12], double dist_max, double cos_max,
                         px_assoc* r) {
    size_t S = (size_t)W * H;
    r->code = OR_INVALID_LIVE;
    r->bin = -1;
    r->margin = INFINITY;
    r->d2 = NAN;
    double p[3], n[3];
    int ok = 1;
    for (int k = 0; k < 3; ++k) {
        p[k] = LV[k * S + i];
        n[k] = LN[k * S + i];
        ok = ok && isfinite(p[k]) && isfinite(n[k]);
    }
    if (!ok) return;
    for (int k = 0; k < 3; ++k)
        r->pp[k] = ((T[4 * k + 0] * p[0] + T[4 * k + 1] * p[1]) + T[4 * k + 2] * p[2]) + T[4 * k + 3];
    r->margin = fabs(r->pp[2]);
    if (!(r->pp[2] > 0.0)) {
        r->code = OR_BEHIND;
        return;
    }
    double uf = K[0] * (r->pp[0] / r->pp[2]) + K[2];
    double vf = K[1] * (r->pp[1] / r->pp[2]) + K[3];
    double uu = floor(uf + 0.5), vv = floor(vf + 0.5);
    /* lateral metres from the rounding edge (a half-integer pixel coordinate) */
    r->margin = dmin(r->margin, (0.5 - fabs(uf - uu)) * r->pp[2] / K[0]);
    r->margin = dmin(r->margin, (0.5 - fabs(vf - vv)) * r->pp[2] / K[1]);
    if (!(uu >= 0.0 && uu <= (double)(W - 1) && vv >= 0.0 && vv <= (double)(H - 1))) {
        r->code = OR_OUTSIDE;
        return;
    }
    size_t j = (size_t)vv * W + (size_t)uu;
    if (!model_ok(MV, MN, S, j)) {
        r->code = OR_INVALID_MODEL;
        return;
    }
    for (int k = 0; k < 3; ++k) {
        r->q[k] = MV[k * S + j];
        r->nq[k] = MN[k * S + j];
    }
    double d[3] = {r->q[0] - r->pp[0], r->q[1] - r->pp[1], r->q[2] - r->pp[2]};
    r->d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    double dist = sqrt(r->d2);
    r->margin = dmin(r->margin, fabs(dist - dist_max));
    if (!(r->d2 < dist_max * dist_max)) {
        r->code = OR_FAR;
        return;
    }
    double rn[3];
    for (int k = 0; k < 3; ++k) rn[k] = (T[4 * k + 0] * n[0] + T[4 * k + 1] * n[1]) + T[4 * k + 2] * n[2];
    double cosv = (rn[0] * r->nq[0] + rn[1] * r->nq[1]) + rn[2] * r->nq[2];
    r->margin = dmin(r->margin, fabs(cosv - cos_max));
    if (!(cosv >= cos_max)) {
        r->code = OR_ANGLE;
        return;
    }
    r->bin = bin_of(r->d2);
    r->margin = dmin(r->margin, dmin(dist - r->bin * BIN_W, (r->bin + 1) * BIN_W - dist));
    r->code = OR_GATED;
}

void or_associate(const float* LV, const float* LN, const float* MV, const float* MN, int W, int H,
                  const double K[4], const double T[12], double dist_max, double cos_max, uint8_t* code,
                  int32_t* bin, double* margin, uint32_t* hist) {
    size_t S = (size_t)W * H;
    uint8_t* c = code ? code : (uint8_t*)malloc(S);
    int32_t* b = bin ? bin : (int32_t*)malloc(S * sizeof(int32_t));
#pragma omp parallel for schedule(static)
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            size_t i = (size_t)v * W + u;
            px_assoc r;
            associate_px(LV, LN, MV, MN, W, H, i, K, T, dist_max, cos_max, &r);
            c[i] = (uint8_t)r.code;
            b[i] = r.bin;
            if (margin) margin[i] = r.margin;
        }
    }
    if (hist) {
        memset(hist, 0, OR_BINS * sizeof(uint32_t));
        for (size_t i = 0; i < S; ++i)
            if (c[i] == OR_GATED) hist[b[i]]++;
    }
    if (!code) free(c);
    if (!bin) free(b);
}

int or_bin_of(double d2) { return bin_of(d2); }

/* per-pixel pairs of one association pass: code, bin and, for GATED pixels,
   p', q, n_q as (H*W, 3) row arrays (other pixels left untouched) */
void or_pairs(const float* LV, const float* LN, const float* MV, const float* MN, int W, int H,
              const double K[4], const double T[12], double dist_max, double cos_max, uint8_t* code,
              int32_t* bin, double* pp, double* q, double* nq) {
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            size_t i = (size_t)v * W + u;
            px_assoc r;
            associate_px(LV, LN, MV, MN, W, H, i, K, T, dist_max, cos_max, &r);
            code[i] = (uint8_t)r.code;
            bin[i] = r.bin;
            if (r.code != OR_GATED) continue;
            for (int k = 0; k < 3; ++k) {
                pp[3 * i + k] = r.pp[k];
                q[3 * i + k] = r.q[k];
                nq[3 * i + k] = r.nq[k];
            }
        }
    }
}

/* Median from the CDF (Sec. 3.3) at bin resolution: the lower median bin
   k_med = min{k : C_k >= ceil(N/2)}.  Band kept around it (reading taken; the
   paper keeps the pairs that gather around the median and gives no formula):
   [max(0, floor((1-beta) k_med)), ceil((1+beta)(k_med+1)) - 1].  Parity
   unpinned for the band's width beyond the paper's one illustration (about
   75% of the pairs kept, which beta = 1 reproduces on the room frames). */
void or_band(const uint32_t* hist, int use_filter, double beta, int64_t out[4]) {
    int64_t N = 0;
    for (int k = 0; k < OR_BINS; ++k) N += hist[k];
    int64_t kmed = -1, klo = 0, khi = -1;
    if (N > 0) {
        int64_t target = (N + 1) / 2, C = 0;
        for (int k = 0; k < OR_BINS; ++k) {
            C += hist[k];
            if (C >= target) {
                kmed = k;
                break;
            }
        }
        if (use_filter) {
            double lo = floor((1.0 - beta) * (double)kmed);
            double hi = ceil((1.0 + beta) * (double)(kmed + 1)) - 1.0;
            klo = lo < 0.0 ? 0 : (int64_t)lo;
            khi = hi > OR_BINS - 1 ? OR_BINS - 1 : (int64_t)hi;
        } else {
            klo = 0;
            khi = OR_BINS - 1;
        }
    }
    out[0] = N;
    out[1] = kmed;
    out[2] = klo;
    out[3] = khi;
}

/* index of entry (i, j), i <= j, of the 7x7 upper triangle, row-major */
static int tri(int i, int j) { return i * 7 - i * (i - 1) / 2 + (j - i); }

/* Rows of Eq. (3).  With the small-angle transform of Eq. (2) applied to the
   current point p', M^ p' = p' + w x p' + tau, so the residual of Eq. (1) is
   n_q . (p' + w x p' + tau - q) = a . x - b with
   a = [(p' x n_q)^T, n_q^T] and b = n_q . (q - p')  (the rows the paper takes
   from Low's report). */
void or_moments(const float* LV, const float* LN, const float* MV, const float* MN, int W, int H,
                const double K[4], const double T[12], double dist_max, double cos_max, int k_lo, int k_hi,
                double M[28], int64_t* n) {
    double* rows = (double*)calloc((size_t)H * 28, sizeof(double));
    int64_t* cnt = (int64_t*)calloc((size_t)H, sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int v = 0; v < H; ++v) {
        double* Mr = rows + (size_t)v * 28;
        for (int u = 0; u < W; ++u) {
            px_assoc r;
            associate_px(LV, LN, MV, MN, W, H, (size_t)v * W + u, K, T, dist_max, cos_max, &r);
            if (r.code != OR_GATED || r.bin < k_lo || r.bin > k_hi) continue;
            double a[7];
            a[0] = r.pp[1] * r.nq[2] - r.pp[2] * r.nq[1];
            a[1] = r.pp[2] * r.nq[0] - r.pp[0] * r.nq[2];
            a[2] = r.pp[0] * r.nq[1] - r.pp[1] * r.nq[0];
            a[3] = r.nq[0];
            a[4] = r.nq[1];
            a[5] = r.nq[2];
            a[6] = (r.nq[0] * (r.q[0] - r.pp[0]) + r.nq[1] * (r.q[1] - r.pp[1])) + r.nq[2] * (r.q[2] - r.pp[2]);
            for (int i = 0; i < 7; ++i)
                for (int j = i; j < 7; ++j) Mr[tri(i, j)] += a[i] * a[j];
            cnt[v]++;
        }
    }
    for (int k = 0; k < 28; ++k) M[k] = 0.0;
    *n = 0;
    for (int v = 0; v < H; ++v) { /* rows summed in row order */
        for (int k = 0; k < 28; ++k) M[k] += rows[(size_t)v * 28 + k];
        *n += cnt[v];
    }
    free(rows);
    free(cnt);
}

/* SE(3) exponential of the twist (w, tau):
   R = I + (sin th / th) [w]x + ((1 - cos th) / th^2) [w]x^2,
   t = (I + ((1 - cos th) / th^2) [w]x + ((th - sin th) / th^3) [w]x^2) tau.
   Its first-order term is the small-angle transform of Eq. (2). */
void or_se3_exp(const double w[3], const double tau[3], double R[9], double t[3]) {
    double th2 = (w[0] * w[0] + w[1] * w[1]) + w[2] * w[2];
    double th = sqrt(th2);
    double A, B, C;
    if (th < 1e-6) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
        C = 1.0 / 6.0 - th2 / 120.0;
    } else {
        double sh = sin(0.5 * th);
        A = sin(th) / th;
        B = 2.0 * sh * sh / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    double Wx[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
    double W2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            W2[3 * i + j] = (Wx[3 * i + 0] * Wx[0 + j] + Wx[3 * i + 1] * Wx[3 + j]) + Wx[3 * i + 2] * Wx[6 + j];
    double V[9];
    for (int k = 0; k < 9; ++k) {
        double I = (k % 4 == 0) ? 1.0 : 0.0;
        R[k] = (I + A * Wx[k]) + B * W2[k];
        V[k] = (I + B * Wx[k]) + C * W2[k];
    }
    for (int i = 0; i < 3; ++i) t[i] = (V[3 * i] * tau[0] + V[3 * i + 1] * tau[1]) + V[3 * i + 2] * tau[2];
}

/* Rotation vector w of R (|w| in [0, pi)): with v = (R32 - R23, R13 - R31,
   R21 - R12) = 2 sin(th) u and trace(R) = 1 + 2 cos(th), th = atan2(|v| / 2,
   (trace - 1) / 2) and w = th u; below |v| = 1e-12 the first-order w = v / 2. */
void or_so3_log(const double R[9], double w[3]) {
    double v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
    double s = 0.5 * sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    double c = 0.5 * (((R[0] + R[4]) + R[8]) - 1.0);
    if (s < 0.5e-12) {
        for (int i = 0; i < 3; ++i) w[i] = 0.5 * v[i];
        return;
    }
    double th = atan2(s, c);
    for (int i = 0; i < 3; ++i) w[i] = v[i] * (th / (2.0 * s));
}

static double lambda_of(int mode, double c, int64_t n) {
    double nd = (double)n;
    switch (mode) {
        case OR_LAMBDA_C_OVER_SQRT_N: return c / sqrt(nd);
        case OR_LAMBDA_C_OVER_N: return c / nd;
        case OR_LAMBDA_C_OVER_N2: return c / (nd * nd);
        default: return c;
    }
}

/* Eq. (4)/(5): minimise (1/2n)|Ax - b|^2 + lambda |Px|^2 with P = [I3 | 0],
   i.e. solve (A^T A + 2 lambda n P^T P) x = A^T b.  The paper solves the 6x6
   system by SVD on the host; for this symmetric positive definite system an
   LDL^T factorisation gives the same x and flags a singular system by its
   pivots.  The increment is then composed on the left of the pose.
   Anchored to the IMU (imu_R not NULL): the damped quantity is the rotation's
   deviation after the update, w + d with d = Log(R_in imu_R^T) (first order in
   w, since R_new = Exp(w) R_in), so the right-hand side becomes
   A^T b - 2 lambda n P^T d; lambda = 0 leaves plain ICP in both forms. */
static int solve_update_core(const double M[28], int64_t n, const double T_in[12], int lambda_mode,
                             double lambda_c, int min_corr, double eps, const double* imu_R, double T_out[12],
                             double x[6]);

int or_solve_update(const double M[28], int64_t n, const double T_in[12], int lambda_mode, double lambda_c,
                    int min_corr, double eps, double T_out[12], double x[6]) {
    return solve_update_core(M, n, T_in, lambda_mode, lambda_c, min_corr, eps, NULL, T_out, x);
}

int or_solve_update_anchor(const double M[28], int64_t n, const double T_in[12], int lambda_mode,
                           double lambda_c, int min_corr, double eps, const double imu_R[9], double T_out[12],
                           double x[6]) {
    return solve_update_core(M, n, T_in, lambda_mode, lambda_c, min_corr, eps, imu_R, T_out, x);
}

static int solve_update_core(const double M[28], int64_t n, const double T_in[12], int lambda_mode,
                             double lambda_c, int min_corr, double eps, const double* imu_R, double T_out[12],
                             double x[6]) {
    memcpy(T_out, T_in, 12 * sizeof(double));
    for (int k = 0; k < 6; ++k) x[k] = 0.0;
    if (n < min_corr) return OR_TOO_FEW_CORR;
    double Hm[6][6], g[6];
    for (int i = 0; i < 6; ++i) {
        for (int j = 0; j < 6; ++j) Hm[i][j] = i <= j ? M[tri(i, j)] : M[tri(j, i)];
        g[i] = M[tri(i, 6)];
    }
    double lam = lambda_of(lambda_mode, lambda_c, n);
    for (int i = 0; i < 3; ++i) Hm[i][i] += 2.0 * lam * (double)n;
    if (imu_R) {
        double Dv[9], dw[3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) /* R_in imu_R^T */
                Dv[3 * i + j] = (T_in[4 * i] * imu_R[3 * j] + T_in[4 * i + 1] * imu_R[3 * j + 1]) +
                                T_in[4 * i + 2] * imu_R[3 * j + 2];
        or_so3_log(Dv, dw);
        for (int i = 0; i < 3; ++i) g[i] -= 2.0 * lam * (double)n * dw[i];
    }
    double maxdiag = 0.0;
    for (int i = 0; i < 6; ++i) maxdiag = Hm[i][i] > maxdiag ? Hm[i][i] : maxdiag;
    double L[6][6] = {{0}}, d[6];
    for (int j = 0; j < 6; ++j) {
        double s = Hm[j][j];
        for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k] * d[k];
        d[j] = s;
        if (!(d[j] > eps * maxdiag)) return OR_ILL_COND;
        L[j][j] = 1.0;
        for (int i = j + 1; i < 6; ++i) {
            double t = Hm[i][j];
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k] * d[k];
            L[i][j] = t / d[j];
        }
    }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double s = g[i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s;
    }
    for (int i = 0; i < 6; ++i) y[i] /= d[i];
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 6; ++k) s -= L[k][i] * x[k];
        x[i] = s;
    }
    for (int i = 0; i < 6; ++i)
        if (!isfinite(x[i])) {
            for (int k = 0; k < 6; ++k) x[k] = 0.0;
            return OR_NONFINITE;
        }
    double dR[9], dt[3];
    or_se3_exp(x, x + 3, dR, dt);
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            T_out[4 * i + j] = (dR[3 * i] * T_in[j] + dR[3 * i + 1] * T_in[4 + j]) + dR[3 * i + 2] * T_in[8 + j];
        T_out[4 * i + 3] = ((dR[3 * i] * T_in[3] + dR[3 * i + 1] * T_in[7]) + dR[3 * i + 2] * T_in[11]) + dt[i];
    }
    return OR_LEVEL_OK;
}

/* ---------------------------------------------------------------------------
 * Whole registration: coarse-to-fine levels, a fixed number of iterations per
 * level (Sec. 4.4), optional early stop on a settled median (Sec. 3.4).
 * ------------------------------------------------------------------------- */
int or_icp_register(const float* depth, int W, int H, const float* model_vtx, const float* model_nrm,
                    const double K[4], const double imu_R[9], const double init_pose[16], const or_params* p,
                    double pose_out[16], or_level_stats* stats, or_iter_trace* trace, int trace_cap) {
    int L = p->levels;
    float *D[OR_MAX_LEVELS] = {0}, *LV[OR_MAX_LEVELS] = {0}, *LN[OR_MAX_LEVELS] = {0};
    float *MV[OR_MAX_LEVELS] = {0}, *MN[OR_MAX_LEVELS] = {0};
    int Wl[OR_MAX_LEVELS], Hl[OR_MAX_LEVELS];
    double Kl[OR_MAX_LEVELS][4];
    for (int l = 0; l < L; ++l) {
        Wl[l] = W >> l;
        Hl[l] = H >> l;
        size_t S = (size_t)Wl[l] * Hl[l];
        D[l] = (float*)malloc(S * sizeof(float));
        LV[l] = (float*)malloc(3 * S * sizeof(float));
        LN[l] = (float*)malloc(3 * S * sizeof(float));
        MV[l] = (float*)malloc(3 * S * sizeof(float));
        MN[l] = (float*)malloc(3 * S * sizeof(float));
        or_level_intrinsics(K, l, Kl[l]);
    }
    if (p->depth_filter)
        or_bilateral(depth, W, H, p->filter_radius, p->filter_sigma_px, p->filter_sigma_m, D[0]);
    else
        memcpy(D[0], depth, (size_t)W * H * sizeof(float));
    for (int l = 1; l < L; ++l) or_depth_down(D[l - 1], Wl[l - 1], Hl[l - 1], D[l]);
    for (int l = 0; l < L; ++l) {
        if (p->normal_mode == 1)
            or_live_vn_box(D[l], Wl[l], Hl[l], Kl[l], p->normal_radius, LV[l], LN[l]);
        else
            or_live_vn(D[l], Wl[l], Hl[l], Kl[l], LV[l], LN[l]);
    }
    or_model_l0(model_vtx, model_nrm, W, H, MV[0], MN[0]);
    for (int l = 1; l < L; ++l) or_model_down(MV[l - 1], MN[l - 1], Wl[l - 1], Hl[l - 1], MV[l], MN[l]);

    /* IMU seed (Sec. 3): the live points are pre-oriented by the IMU rotation */
    double T[12];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) T[4 * i + j] = p->use_imu_seed ? imu_R[3 * i + j] : init_pose[4 * i + j];
        T[4 * i + 3] = init_pose[4 * i + 3];
    }
    int ntrace = 0;
    uint32_t hist[OR_BINS];
    for (int l = L - 1; l >= 0; --l) {
        or_level_stats* st = &stats[l];
        memset(st, 0, sizeof(*st));
        st->k_med = -1;
        int settled = 0;
        int32_t last_kmed = -2;
        for (int it = 0; it < p->iters[l]; ++it) {
            or_associate(LV[l], LN[l], MV[l], MN[l], Wl[l], Hl[l], Kl[l], T, p->dist_max, p->cos_angle_max, NULL,
                         NULL, NULL, hist);
            int64_t band[4];
            or_band(hist, p->use_median_filter, p->band_beta, band);
            double M[28], x[6], Tn[12];
            int64_t n = 0;
            if (band[0] > 0)
                or_moments(LV[l], LN[l], MV[l], MN[l], Wl[l], Hl[l], Kl[l], T, p->dist_max, p->cos_angle_max,
                           (int)band[2], (int)band[3], M, &n);
            else
                memset(M, 0, sizeof(M));
            int status = solve_update_core(M, n, T, p->lambda_mode, p->lambda_c, p->min_corr, p->ill_cond_eps,
                                           p->anchor_to_imu ? imu_R : NULL, Tn, x);
            st->iters_run = it + 1;
            st->status = status;
            st->n_gated = band[0];
            st->n_kept = n;
            st->k_med = (int32_t)band[1];
            st->rmse = n > 0 ? sqrt(M[27] / (double)n) : 0.0;
            if (status == OR_LEVEL_OK) memcpy(T, Tn, sizeof(T));
            if (trace && ntrace < trace_cap) {
                or_iter_trace* tr = &trace[ntrace];
                tr->level = l;
                tr->iter = it;
                tr->status = status;
                tr->k_med = (int32_t)band[1];
                tr->k_lo = (int32_t)band[2];
                tr->k_hi = (int32_t)band[3];
                tr->n_gated = band[0];
                tr->n_kept = n;
                memcpy(tr->x, x, sizeof(x));
                memcpy(tr->pose, T, sizeof(T));
            }
            ++ntrace;
            if (status != OR_LEVEL_OK) break;
            /* Sec. 3.4: converged once the median bin is unchanged for
               converge_window successive iterations */
            settled = ((int32_t)band[1] == last_kmed) ? settled + 1 : 1;
            last_kmed = (int32_t)band[1];
            if (p->converge_window > 0 && settled >= p->converge_window) break;
        }
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 4; ++j) pose_out[4 * i + j] = T[4 * i + j];
    pose_out[12] = pose_out[13] = pose_out[14] = 0.0;
    pose_out[15] = 1.0;
    for (int l = 0; l < L; ++l) {
        free(D[l]);
        free(LV[l]);
        free(LN[l]);
        free(MV[l]);
        free(MN[l]);
    }
    return ntrace;
}
