// TSDF model of the reconstruction (KinectFusion's volume, the one the paper's
// tracking feeds: Sec. 4.3 describes its weights being overwritten by a bad
// alignment, Sec. 5.2 sizes it at 512^3 voxels over at most 6 m).
//
// Arithmetic is FP64 with -ffp-contract=off: every voxel update and every ray
// step rounds exactly as written, so the volume and the ray-cast maps depend
// on nothing but the inputs.  Storage is FP32 pairs (tsdf, weight), 8 bytes
// per voxel, x fastest: a work-group of integration touches 64 consecutive
// voxels of 4 rows, and the 8 corners of a trilinear sample are 4 pairs of
// adjacent voxels.
//
// Integration: one thread per 16 voxels along z.  The voxel centre goes into the camera,
// is projected with the pixel rounding of the association (nearest pixel),
// and the projective signed distance sdf = z(pixel) - z(voxel) is truncated
// at mu: voxels more than mu behind the surface stay untouched, the others
// take f = min(1, sdf / mu) into a running average whose weight saturates at
// max_weight.  Only voxels that are updated are read or written, and an FP32
// frustum pre-test (conservative by a wide margin) spares the FP64 arithmetic
// for voxels outside the camera's view.
//
// Ray casting: one thread per pixel of a 16 x 16 tile.  The ray z (x_u, y_v, 1)
// is sampled at z = tmin + s * side / 2; a sample is the trilinear value of the
// 8 voxels around the point and is missing when any of them is unobserved.  The
// first step from a positive to a non-positive sample is the surface (depth
// interpolated linearly between the two samples), a step from negative to
// non-negative (the back of a surface) ends the ray.  The normal is the
// central-difference gradient one voxel to each side, in the camera frame,
// turned to face the camera.  Samples outside the volume's interior are all
// missing, so each ray walks only the steps of its interval inside the
// interior box, widened by two steps at each end: the skipped samples could
// only have reset the walk.
#include <hip/hip_runtime.h>

#include "icp_launch.hpp"

namespace icpk {
namespace {

struct Geo {
    float2* vox;
    int dim;
    double side;                // size / dim
    double o[3];                // corner of voxel (0, 0, 0)
};

__device__ __forceinline__ bool depth_valid(float z) { return __builtin_isfinite(z) && z > 0.0f; }

__global__ void __launch_bounds__(256) k_tsdf_fill(float2* vox, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        vox[i] = make_float2(0.0f, 0.0f);
}

// FP32 copy of the camera for a conservative pre-test: a voxel whose FP32
// camera coordinates lie more than `margin` outside the viewing frustum
// (behind the camera, or beyond the outer edges of the border pixels) fails
// the exact FP64 test too.  margin is ~100x the FP32 rounding of coordinates
// of the volume's magnitude, so the pre-test only saves work.
struct Cull {
    float o[3], side, t[3], R[9];
    float a_lo, a_hi, b_lo, b_hi;  // x/z and y/z over the image, half a pixel beyond the border centres
    float margin;
};

constexpr int kIntegrateZ = 16;  // voxels along z per thread

// One voxel: pre-test, then the exact FP64 update.
__device__ __forceinline__ void integrate_voxel(const Geo& g, const Cull& c, double mu, double maxw,
                                                const float* __restrict__ depth, int W, int H, double fx, double fy,
                                                double cx, double cy, const double* P, int i, int j, int k) {
    {
        const float e0 = c.o[0] + ((float)i + 0.5f) * c.side - c.t[0];
        const float e1 = c.o[1] + ((float)j + 0.5f) * c.side - c.t[1];
        const float e2 = c.o[2] + ((float)k + 0.5f) * c.side - c.t[2];
        const float z = c.R[2] * e0 + c.R[5] * e1 + c.R[8] * e2;
        const float x = c.R[0] * e0 + c.R[3] * e1 + c.R[6] * e2;
        const float y = c.R[1] * e0 + c.R[4] * e1 + c.R[7] * e2;
        const float m = c.margin;
        if (!(z > -m) || x < c.a_lo * z - m * (1.0f + fabsf(c.a_lo)) || x > c.a_hi * z + m * (1.0f + fabsf(c.a_hi)) ||
            y < c.b_lo * z - m * (1.0f + fabsf(c.b_lo)) || y > c.b_hi * z + m * (1.0f + fabsf(c.b_hi)))
            return;
    }
    const double xw0 = g.o[0] + ((double)i + 0.5) * g.side;
    const double xw1 = g.o[1] + ((double)j + 0.5) * g.side;
    const double xw2 = g.o[2] + ((double)k + 0.5) * g.side;
    const double d0 = xw0 - P[3], d1 = xw1 - P[7], d2 = xw2 - P[11];
    // x_c = R^T (x_w - t): component a is column a of R dotted with d
    const double xc0 = (P[0] * d0 + P[4] * d1) + P[8] * d2;
    const double xc1 = (P[1] * d0 + P[5] * d1) + P[9] * d2;
    const double xc2 = (P[2] * d0 + P[6] * d1) + P[10] * d2;
    if (!(xc2 > 0.0)) return;
    const double uu = floor(fx * (xc0 / xc2) + cx + 0.5);
    const double vv = floor(fy * (xc1 / xc2) + cy + 0.5);
    if (!(uu >= 0.0 && uu <= (double)(W - 1) && vv >= 0.0 && vv <= (double)(H - 1))) return;
    const float z = depth[(size_t)vv * W + (size_t)uu];
    if (!depth_valid(z)) return;
    const double sdf = (double)z - xc2;
    if (sdf < -mu) return;
    double f = sdf / mu;
    if (f > 1.0) f = 1.0;
    float2* p = g.vox + (((size_t)k * g.dim + j) * g.dim + i);
    const float2 cur = *p;
    const double w = (double)cur.y;
    const double wn = w + 1.0;
    *p = make_float2((float)(((double)cur.x * w + f) / wn), (float)(wn < maxw ? wn : maxw));
}

// grid (ceil(dim/64), ceil(dim/4), ceil(dim/kIntegrateZ)), block 64 x 4; a
// thread takes kIntegrateZ voxels along z (fewer, longer work-groups: one
// voxel per thread left the launch rate, not the arithmetic, as the limit)
__global__ void __launch_bounds__(256) k_tsdf_integrate(Geo g, Cull c, double mu, double maxw,
                                                        const float* __restrict__ depth, int W, int H, double fx,
                                                        double fy, double cx, double cy, PoseArg T) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    if (i >= g.dim || j >= g.dim) return;
    const int k0 = blockIdx.z * kIntegrateZ;
    const int k1 = min(k0 + kIntegrateZ, g.dim);
    for (int k = k0; k < k1; ++k) integrate_voxel(g, c, mu, maxw, depth, W, H, fx, fy, cx, cy, T.v, i, j, k);
}

// Trilinear TSDF at world point (p0, p1, p2); false when a corner is unobserved
// or the point is outside the interior box of voxel centres.
__device__ __forceinline__ bool sample(const Geo& g, double p0, double p1, double p2, double& out) {
    const double g0 = (p0 - g.o[0]) / g.side - 0.5;
    const double g1 = (p1 - g.o[1]) / g.side - 0.5;
    const double g2 = (p2 - g.o[2]) / g.side - 0.5;
    const double f0 = floor(g0), f1 = floor(g1), f2 = floor(g2);
    const double lim = (double)(g.dim - 1);
    if (!(f0 >= 0.0 && f0 < lim && f1 >= 0.0 && f1 < lim && f2 >= 0.0 && f2 < lim)) return false;
    const double r0 = g0 - f0, r1 = g1 - f1, r2 = g2 - f2;
    const size_t dim = (size_t)g.dim;
    const float2* b = g.vox + (((size_t)f2 * dim + (size_t)f1) * dim + (size_t)f0);
    const float2 c000 = b[0], c100 = b[1];
    const float2 c010 = b[dim], c110 = b[dim + 1];
    const float2 c001 = b[dim * dim], c101 = b[dim * dim + 1];
    const float2 c011 = b[dim * dim + dim], c111 = b[dim * dim + dim + 1];
    const bool seen = c000.y > 0.0f && c100.y > 0.0f && c010.y > 0.0f && c110.y > 0.0f && c001.y > 0.0f &&
                      c101.y > 0.0f && c011.y > 0.0f && c111.y > 0.0f;
    if (!seen) return false;
    const double a00 = (double)c000.x * (1.0 - r0) + (double)c100.x * r0;
    const double a10 = (double)c010.x * (1.0 - r0) + (double)c110.x * r0;
    const double a01 = (double)c001.x * (1.0 - r0) + (double)c101.x * r0;
    const double a11 = (double)c011.x * (1.0 - r0) + (double)c111.x * r0;
    const double b0 = a00 * (1.0 - r1) + a10 * r1;
    const double b1 = a01 * (1.0 - r1) + a11 * r1;
    out = b0 * (1.0 - r2) + b1 * r2;
    return true;
}

// Narrows [t0, t1] to the ray parameters where o + t d lies in [lo, hi] along
// one axis (an empty interval when the ray runs parallel outside the slab).
__device__ __forceinline__ void slab(double o, double d, double lo, double hi, double& t0, double& t1) {
    if (fabs(d) < 1e-300) {
        if (!(o >= lo && o <= hi)) {
            t0 = 1e300;
            t1 = -1e300;
        }
        return;
    }
    double a = (lo - o) / d, b = (hi - o) / d;
    if (a > b) {
        const double c = a;
        a = b;
        b = c;
    }
    t0 = fmax(t0, a);
    t1 = fmin(t1, b);
}

// grid (ceil(W/16), ceil(H/16)), block 16 x 16
__global__ void __launch_bounds__(256) k_tsdf_raycast(Geo g, double tmin, double tmax, int W, int H, double fx,
                                                      double fy, double cx, double cy, PoseArg T,
                                                      float* __restrict__ vtx, float* __restrict__ nrm) {
    const int u = blockIdx.x * 16 + threadIdx.x;
    const int v = blockIdx.y * 16 + threadIdx.y;
    if (u >= W || v >= H) return;
    const double* P = T.v;
    const size_t px = (size_t)v * W + u;
    const float qnan = __builtin_nanf("");
    float pv[3] = {qnan, qnan, qnan}, pn[3] = {qnan, qnan, qnan};
    const double dc0 = ((double)u - cx) / fx, dc1 = ((double)v - cy) / fy;
    const double dw0 = (P[0] * dc0 + P[1] * dc1) + P[2];
    const double dw1 = (P[4] * dc0 + P[5] * dc1) + P[6];
    const double dw2 = (P[8] * dc0 + P[9] * dc1) + P[10];
    const double dz = 0.5 * g.side;

    // interval of the walk inside the interior box (widened by two steps)
    double t0 = -1e300, t1 = 1e300;
    for (int a = 0; a < 3; ++a) {
        const double o = a == 0 ? P[3] : (a == 1 ? P[7] : P[11]);
        const double d = a == 0 ? dw0 : (a == 1 ? dw1 : dw2);
        slab(o, d, g.o[a] + 0.5 * g.side, g.o[a] + ((double)g.dim - 0.5) * g.side, t0, t1);
    }
    const double n_steps = floor((tmax - tmin) / dz) + 1.0;  // s with tmin + s dz <= tmax, plus one
    double s_lo = floor((t0 - tmin) / dz) - 2.0, s_hi = ceil((t1 - tmin) / dz) + 2.0;
    s_lo = fmax(s_lo, 0.0);
    s_hi = fmin(s_hi, n_steps);

    double t_hit = -1.0;
    if (s_lo <= s_hi) {  // the two-step margins also cover rounding in the interval
        bool have_prev = false;
        double t_prev = 0.0, f_prev = 0.0;
        const int s_end = (int)s_hi;
        for (int s = (int)s_lo; s <= s_end; ++s) {
            const double t = tmin + (double)s * dz;
            if (t > tmax) break;
            double f;
            if (!sample(g, P[3] + t * dw0, P[7] + t * dw1, P[11] + t * dw2, f)) {
                have_prev = false;
                continue;
            }
            if (have_prev && f_prev > 0.0 && f <= 0.0) {
                t_hit = t_prev + (t - t_prev) * (f_prev / (f_prev - f));
                break;
            }
            if (have_prev && f_prev < 0.0 && f >= 0.0) break;
            have_prev = true;
            t_prev = t;
            f_prev = f;
        }
    }
    if (t_hit > 0.0) {
        const double h0 = P[3] + t_hit * dw0, h1 = P[7] + t_hit * dw1, h2 = P[11] + t_hit * dw2;
        // six samples one voxel away along +x, -x, +y, -y, +z, -z, taken one
        // at a time (unrolled, their loads would all be live at once)
        double gx0 = 0.0, gx1 = 0.0, gy0 = 0.0, gy1 = 0.0, gz0 = 0.0, gz1 = 0.0;
        bool ok = true;
#pragma unroll 1
        for (int q = 0; q < 6; ++q) {
            const double sg = (q & 1) ? -g.side : g.side;  // h - side == h + (-side) exactly
            const int a = q >> 1;
            double v;
            if (!sample(g, a == 0 ? h0 + sg : h0, a == 1 ? h1 + sg : h1, a == 2 ? h2 + sg : h2, v)) {
                ok = false;
                break;
            }
            gx1 = q == 0 ? v : gx1;
            gx0 = q == 1 ? v : gx0;
            gy1 = q == 2 ? v : gy1;
            gy0 = q == 3 ? v : gy0;
            gz1 = q == 4 ? v : gz1;
            gz0 = q == 5 ? v : gz0;
        }
        if (ok) {
            const double gw0 = gx1 - gx0, gw1 = gy1 - gy0, gw2 = gz1 - gz0;
            const double len2 = (gw0 * gw0 + gw1 * gw1) + gw2 * gw2;
            if (len2 > 0.0) {
                const double len = sqrt(len2);
                const double nw0 = gw0 / len, nw1 = gw1 / len, nw2 = gw2 / len;
                double nc0 = (P[0] * nw0 + P[4] * nw1) + P[8] * nw2;
                double nc1 = (P[1] * nw0 + P[5] * nw1) + P[9] * nw2;
                double nc2 = (P[2] * nw0 + P[6] * nw1) + P[10] * nw2;
                const double pc0 = t_hit * dc0, pc1 = t_hit * dc1, pc2 = t_hit * 1.0;
                const double sd = (nc0 * pc0 + nc1 * pc1) + nc2 * pc2;
                if (sd > 0.0) {
                    nc0 = -nc0;
                    nc1 = -nc1;
                    nc2 = -nc2;
                }
                pv[0] = (float)pc0;
                pv[1] = (float)pc1;
                pv[2] = (float)pc2;
                pn[0] = (float)nc0;
                pn[1] = (float)nc1;
                pn[2] = (float)nc2;
            }
        }
    }
    for (int a = 0; a < 3; ++a) {
        vtx[3 * px + a] = pv[a];
        nrm[3 * px + a] = pn[a];
    }
}

Geo make_geo(const TsdfDesc& d) {
    Geo g;
    g.vox = reinterpret_cast<float2*>(d.voxels);
    g.dim = d.dim;
    g.side = d.size / (double)d.dim;
    for (int a = 0; a < 3; ++a) g.o[a] = d.origin[a];
    return g;
}

}  // namespace

hipError_t launch_tsdf_fill(const TsdfDesc& d, hipStream_t s) {
    const int64_t n = (int64_t)d.dim * d.dim * d.dim;
    const int64_t blocks = (n + 255) / 256;
    const unsigned grid = (unsigned)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(k_tsdf_fill, dim3(grid), dim3(256), 0, s, reinterpret_cast<float2*>(d.voxels), n);
    return hipGetLastError();
}

hipError_t launch_tsdf_integrate(const TsdfDesc& d, const float* depth, int W, int H, const double* K, PoseArg T,
                                 hipStream_t s) {
    Cull c;
    double extent = d.size;
    for (int a = 0; a < 3; ++a) {
        c.o[a] = (float)d.origin[a];
        c.t[a] = (float)T.v[4 * a + 3];
        extent += fabs(d.origin[a]) + fabs(T.v[4 * a + 3]);
        for (int b = 0; b < 3; ++b) c.R[3 * a + b] = (float)T.v[4 * a + b];
    }
    c.side = (float)(d.size / (double)d.dim);
    c.a_lo = (float)((-0.5 - K[2]) / K[0]);
    c.a_hi = (float)(((double)W - 0.5 - K[2]) / K[0]);
    c.b_lo = (float)((-0.5 - K[3]) / K[1]);
    c.b_hi = (float)(((double)H - 0.5 - K[3]) / K[1]);
    c.margin = (float)(1e-4 * (1.0 + extent));
    dim3 grid((unsigned)((d.dim + 63) / 64), (unsigned)((d.dim + 3) / 4),
              (unsigned)((d.dim + kIntegrateZ - 1) / kIntegrateZ));
    hipLaunchKernelGGL(k_tsdf_integrate, grid, dim3(64, 4), 0, s, make_geo(d), c, d.mu, d.max_weight, depth, W, H,
                       K[0], K[1], K[2], K[3], T);
    return hipGetLastError();
}

hipError_t launch_tsdf_raycast(const TsdfDesc& d, double tmin, double tmax, int W, int H, const double* K, PoseArg T,
                               float* vtx, float* nrm, hipStream_t s) {
    dim3 grid((unsigned)((W + 15) / 16), (unsigned)((H + 15) / 16));
    hipLaunchKernelGGL(k_tsdf_raycast, grid, dim3(16, 16), 0, s, make_geo(d), tmin, tmax, W, H, K[0], K[1], K[2],
                       K[3], T, vtx, nrm);
    return hipGetLastError();
}

}  // namespace icpk
