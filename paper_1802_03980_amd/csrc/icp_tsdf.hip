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
// Integration: one thread per 16 voxels along z.  The voxel centre goes into
// the camera, is projected with the pixel rounding of the association
// (nearest pixel), and the projective signed distance sdf = z(pixel) -
// z(voxel) is truncated at mu: voxels more than mu behind the surface stay
// untouched, the others take f = min(1, sdf / mu) into a running average whose
// weight saturates at max_weight.  Only voxels that are updated are read or
// written, and an FP32 frustum pre-test (conservative by a wide margin) spares
// the FP64 arithmetic for voxels outside the camera's view, first for a
// thread's whole run of 16 voxels (from its two ends), then voxel by voxel.
//
// Ray casting: kRayLanes (4) lanes per pixel, each taking every fourth step
// of the walk (four lanes per ray measured faster than one, two or eight).
// The ray z (x_u, y_v, 1) is sampled at z = tmin + s * side / 2, in grid
// coordinates (voxel centres at integers); a sample is the trilinear value
// of the 8 voxels around the point and is missing when any of them is
// unobserved.  The first step from a positive to a non-positive sample is the
// surface (depth interpolated linearly between the two samples), a step from
// negative to non-negative (the back of a surface) ends the ray.  The normal
// is the central-difference gradient one voxel to each side, in the camera
// frame, turned to face the camera.  Samples outside the volume's interior
// are all missing, so each ray walks only the steps of its interval inside
// the interior box, widened by two steps at each end: the skipped samples
// could only have reset the walk.
//
// Brick skipping (optional, same results): integration keeps per 8^3 brick
// the number of observed voxels with tsdf <= 0, and a small kernel marks a
// brick skippable when it and its +x/+y/+z neighbours hold none.  Every
// sample whose cell starts in such a brick is then either missing or > 0 (its
// corners are observed and positive), so no step from + to <= 0 or from - to
// >= 0 can happen among them: a ray whose step falls in a skippable brick
// jumps to the last step still in the brick, which is where the full walk
// would have arrived in the same state.  The jump is not taken right after a
// negative sample (the full walk may end there).  Its length is estimated
// from the brick's faces and then checked: the grid coordinates of a step are
// monotone in the step index (each rounded operation is monotone), so if the
// landing step's cell is still in the brick, so is every step in between.
// The landing step itself can hold no event either, so the walk restarts
// there as if its predecessor were missing.
#include <hip/hip_runtime.h>

#include "icp_launch.hpp"

namespace icpk {
namespace {

struct Geo {
    float2* vox;
    int dim;
    double side;                // size / dim
    double inv;                 // 1 / side (rounded once)
    double o[3];                // corner of voxel (0, 0, 0)
    int nb;                     // bricks per edge, ceil(dim / 8)
    int* cnt;                   // per brick: observed voxels with tsdf <= 0 (NULL: no bricks)
    uint8_t* flags;             // per brick: 1 = skippable
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

// The pre-test's five constraints at voxel (i, j, k), each >= 0 (the first
// > 0) where the voxel may lie in the frustum: in front of the camera, right
// of the left edge, left of the right edge, below the top, above the bottom.
// Each is, up to FP32 rounding far below the margin, a linear function of the
// voxel centre, so a constraint negative at both ends of a run of voxels
// along z is negative (the exact test fails) all along it.
__device__ __forceinline__ void frustum_terms(const Cull& c, int i, int j, int k, float (&q)[5]) {
    const float e0 = c.o[0] + ((float)i + 0.5f) * c.side - c.t[0];
    const float e1 = c.o[1] + ((float)j + 0.5f) * c.side - c.t[1];
    const float e2 = c.o[2] + ((float)k + 0.5f) * c.side - c.t[2];
    const float z = c.R[2] * e0 + c.R[5] * e1 + c.R[8] * e2;
    const float x = c.R[0] * e0 + c.R[3] * e1 + c.R[6] * e2;
    const float y = c.R[1] * e0 + c.R[4] * e1 + c.R[7] * e2;
    const float m = c.margin;
    q[0] = z + m;
    q[1] = x - (c.a_lo * z - m * (1.0f + fabsf(c.a_lo)));
    q[2] = (c.a_hi * z + m * (1.0f + fabsf(c.a_hi))) - x;
    q[3] = y - (c.b_lo * z - m * (1.0f + fabsf(c.b_lo)));
    q[4] = (c.b_hi * z + m * (1.0f + fabsf(c.b_hi))) - y;
}

// a / b rounded correctly from y = RN(1/b): q = RN(a y) lies within an ulp
// of a / b, so the remainder a - b q is exact in one FMA, and one more FMA
// with y gives the correctly rounded quotient (Markstein's theorem; it needs
// no underflow or overflow in a y and the remainder, which the callers'
// ranges guarantee: moderate a, and b at least 2^-900).
__device__ __forceinline__ double div_by_recip(double a, double b, double y) {
    const double q = a * y;
    return __builtin_fma(__builtin_fma(-q, b, a), y, q);
}

constexpr double kRecipMinDivisor = 0x1p-900;

// 1/k for the running average's integer weight counts k = 1..kMaxCount,
// each correctly rounded (IEEE divisions at compile time).
constexpr int kMaxCount = 256;
struct CountRecip {
    double v[kMaxCount + 1];
};
constexpr CountRecip make_count_recips() {
    CountRecip t{};
    for (int k = 1; k <= kMaxCount; ++k) t.v[k] = 1.0 / (double)k;
    return t;
}
__constant__ CountRecip kCountRecip = make_count_recips();

// One voxel: pre-test, then the exact FP64 update.  The quotients are the
// IEEE quotients of the definition, formed from correctly rounded
// reciprocals: one division for both projection quotients (a shared
// divisor), 1/mu from the host, and a table for the weight count (an IEEE
// division for counts that are not small integers).
__device__ __forceinline__ void integrate_voxel(const Geo& g, const Cull& c, double mu, double inv_mu, double maxw,
                                                const float* __restrict__ depth, int W, int H, double fx, double fy,
                                                double cx, double cy, const double* P, int i, int j, int k,
                                                int& d_neg) {
    {
        float q[5];
        frustum_terms(c, i, j, k, q);
        if (!(q[0] > 0.0f) || q[1] < 0.0f || q[2] < 0.0f || q[3] < 0.0f || q[4] < 0.0f) return;
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
    double q0, q1;
    if (xc2 >= kRecipMinDivisor) {
        const double y = 1.0 / xc2;
        q0 = div_by_recip(xc0, xc2, y);
        q1 = div_by_recip(xc1, xc2, y);
    } else {
        q0 = xc0 / xc2;
        q1 = xc1 / xc2;
    }
    const double uu = floor(fx * q0 + cx + 0.5);
    const double vv = floor(fy * q1 + cy + 0.5);
    if (!(uu >= 0.0 && uu <= (double)(W - 1) && vv >= 0.0 && vv <= (double)(H - 1))) return;
    const float z = depth[(size_t)vv * W + (size_t)uu];
    if (!depth_valid(z)) return;
    const double sdf = (double)z - xc2;
    if (sdf < -mu) return;
    double f = mu >= kRecipMinDivisor ? div_by_recip(sdf, mu, inv_mu) : sdf / mu;
    if (f > 1.0) f = 1.0;
    float2* p = g.vox + (((size_t)k * g.dim + j) * g.dim + i);
    const float2 cur = *p;
    const double w = (double)cur.y;
    const double wn = w + 1.0;
    const double a = (double)cur.x * w + f;
    double avg;
    if (wn >= 1.0 && wn <= (double)kMaxCount && wn == floor(wn))
        avg = div_by_recip(a, wn, kCountRecip.v[(int)wn]);
    else
        avg = a / wn;
    const float tn = (float)avg;
    *p = make_float2(tn, (float)(wn < maxw ? wn : maxw));
    d_neg += (tn <= 0.0f ? 1 : 0) - (cur.y > 0.0f && cur.x <= 0.0f ? 1 : 0);
}

// grid (ceil(dim/64), ceil(dim/4), ceil(dim/kIntegrateZ)), block 64 x 4; a
// thread takes kIntegrateZ voxels along z (fewer, longer work-groups: one
// voxel per thread left the launch rate, not the arithmetic, as the limit)
__global__ void __launch_bounds__(256) k_tsdf_integrate(Geo g, Cull c, double mu, double inv_mu, double maxw,
                                                        const float* __restrict__ depth, int W, int H, double fx,
                                                        double fy, double cx, double cy, PoseArg T) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;  // the same for the whole wave
    if (j >= g.dim) return;
    const int k0 = blockIdx.z * kIntegrateZ;
    const int k1 = min(k0 + kIntegrateZ, g.dim);
    const bool inside = i < g.dim;
    bool active = inside;
    if (active) {  // the whole run outside one side of the frustum?
        float qa[5], qb[5];
        frustum_terms(c, i, j, k0, qa);
        frustum_terms(c, i, j, k1 - 1, qb);
        const bool out = (!(qa[0] > 0.0f) && !(qb[0] > 0.0f)) || (qa[1] < 0.0f && qb[1] < 0.0f) ||
                         (qa[2] < 0.0f && qb[2] < 0.0f) || (qa[3] < 0.0f && qb[3] < 0.0f) ||
                         (qa[4] < 0.0f && qb[4] < 0.0f);
        active = !out;
    }
    if (__ballot(active) == 0) return;  // nothing to update or count in this wave
    int a_neg = 0;
    for (int k = k0; k < k1; ++k) {
        if (active) integrate_voxel(g, c, mu, inv_mu, maxw, depth, W, H, fx, fy, cx, cy, T.v, i, j, k, a_neg);
        if (g.cnt && ((k & 7) == 7 || k + 1 == k1)) {
            // the 8 lanes sharing i >> 3 cover one brick row: one atomic per brick and row
#pragma unroll
            for (int off = 1; off < 8; off <<= 1) a_neg += __shfl_xor(a_neg, off, 64);
            if (inside && (threadIdx.x & 7) == 0 && a_neg != 0)  // the group's first lane, culled or not
                atomicAdd(g.cnt + (((size_t)(k >> 3) * g.nb) + (j >> 3)) * g.nb + (i >> 3), a_neg);
            a_neg = 0;
        }
    }
}

// One thread per brick: skippable when it and its +1 neighbours (those inside
// the volume) hold no observed voxel with tsdf <= 0.
__global__ void __launch_bounds__(256) k_tsdf_flags(const int* __restrict__ cnt, uint8_t* __restrict__ flags, int nb) {
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= (int64_t)nb * nb * nb) return;
    const int bx = (int)(b % nb), by = (int)((b / nb) % nb), bz = (int)(b / ((int64_t)nb * nb));
    bool skip = true;
    for (int q = 0; q < 8; ++q) {
        const int x = bx + (q & 1), y = by + ((q >> 1) & 1), z = bz + (q >> 2);
        if (x < nb && y < nb && z < nb) skip = skip && cnt[((size_t)z * nb + y) * nb + x] == 0;
    }
    flags[b] = skip ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_tsdf_zero_counts(int* cnt, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) cnt[i] = 0;
}

// Corner pairs (tsdf, weight) of voxels x and x + 1, read as one 16-byte load
// (8-byte aligned).
typedef float pair2_t __attribute__((ext_vector_type(4), aligned(8)));

// Trilinear TSDF at grid point (g0, g1, g2) (voxel centres at integers) whose
// cell (f0, f1, f2) = floor(g) is inside [0, dim - 2]^3; false when a corner
// is unobserved.
__device__ __forceinline__ bool sample_cell(const Geo& g, double g0, double g1, double g2, double f0, double f1,
                                            double f2, double& out) {
    const double r0 = g0 - f0, r1 = g1 - f1, r2 = g2 - f2;
    const uint32_t dim = (uint32_t)g.dim;
    const uint32_t idx = ((uint32_t)f2 * dim + (uint32_t)f1) * dim + (uint32_t)f0;  // < 2^30
    const float2* b = g.vox + idx;
    const pair2_t x00 = *reinterpret_cast<const pair2_t*>(b);                  // (i, j, k), (i+1, j, k)
    const pair2_t x10 = *reinterpret_cast<const pair2_t*>(b + dim);            // j + 1
    const pair2_t x01 = *reinterpret_cast<const pair2_t*>(b + dim * dim);      // k + 1
    const pair2_t x11 = *reinterpret_cast<const pair2_t*>(b + dim * dim + dim);
    // weights are +0 or >= 1, so their bit patterns order like their values
    const uint32_t wmin = min(min(min(__float_as_uint(x00.y), __float_as_uint(x00.w)),
                                  min(__float_as_uint(x10.y), __float_as_uint(x10.w))),
                              min(min(__float_as_uint(x01.y), __float_as_uint(x01.w)),
                                  min(__float_as_uint(x11.y), __float_as_uint(x11.w))));
    if (wmin == 0u) return false;
    const double q0 = 1.0 - r0, q1 = 1.0 - r1, q2 = 1.0 - r2;
    const double a00 = (double)x00.x * q0 + (double)x00.z * r0;
    const double a10 = (double)x10.x * q0 + (double)x10.z * r0;
    const double a01 = (double)x01.x * q0 + (double)x01.z * r0;
    const double a11 = (double)x11.x * q0 + (double)x11.z * r0;
    const double b0 = a00 * q1 + a10 * r1;
    const double b1 = a01 * q1 + a11 * r1;
    out = b0 * q2 + b1 * r2;
    return true;
}

__device__ __forceinline__ bool in_range(const Geo& g, double f0, double f1, double f2) {
    const double lim = (double)(g.dim - 1);
    return f0 >= 0.0 && f0 < lim && f1 >= 0.0 && f1 < lim && f2 >= 0.0 && f2 < lim;
}

// Trilinear TSDF at grid point (g0, g1, g2); false when a corner is
// unobserved or the point's cell is outside [0, dim - 2]^3.
__device__ __forceinline__ bool sample(const Geo& g, double g0, double g1, double g2, double& out) {
    const double f0 = floor(g0), f1 = floor(g1), f2 = floor(g2);
    if (!in_range(g, f0, f1, f2)) return false;
    return sample_cell(g, g0, g1, g2, f0, f1, f2, out);
}

// Brick of a cell packed into one int (10 bits per axis; bricks per edge <= 128).
__device__ __forceinline__ int pack_brick(double f0, double f1, double f2) {
    return ((int)f0 >> 3) | (((int)f1 >> 3) << 10) | (((int)f2 >> 3) << 20);
}

// Ray parameter at which the cell along one axis leaves brick b, from the
// reciprocal rg = 1/gd (an estimate; callers verify).
__device__ __forceinline__ double brick_exit(double gc, double gd, double rg, int b) {
    if (gd > 1e-300) return (8.0 * b + 8.0 - gc) * rg;
    if (gd < -1e-300) return (8.0 * b - gc) * rg;
    return 1e300;
}

// Narrows [t0, t1] to the ray parameters where gc + t gd lies in [lo, hi]
// along one axis (an empty interval when the ray runs parallel outside).
__device__ __forceinline__ void slab(double gc, double gd, double lo, double hi, double& t0, double& t1) {
    if (fabs(gd) < 1e-300) {
        if (!(gc >= lo && gc <= hi)) {
            t0 = 1e300;
            t1 = -1e300;
        }
        return;
    }
    double a = (lo - gc) / gd, b = (hi - gc) / gd;
    if (a > b) {
        const double c = a;
        a = b;
        b = c;
    }
    t0 = fmax(t0, a);
    t1 = fmin(t1, b);
}

#ifndef ICP_RAY_LANES
#define ICP_RAY_LANES 4
#endif
constexpr int kRayLanes = ICP_RAY_LANES;  // lanes per ray: one step each per round

// kRayLanes lanes per ray.  Each round the ray's lanes take the samples of
// kRayLanes consecutive steps at once; the walk's rule is then applied to
// them in step order with shuffles (a lane sees its predecessor's sample, NaN
// when missing; lane 0 sees the step before the round) and a ballot picks the
// first step where the walk stops.  The hop over a skippable brick starts
// from the round's last step, whose brick flag is loaded with the round's
// samples.  Every lane of a ray takes the same control decisions (from
// shuffled or identically computed values), so a ray's lanes stay together.
// gc: camera centre in grid coordinates minus 1/2 (host-computed).
__global__ void __launch_bounds__(256) k_tsdf_raycast(Geo g, double gc0, double gc1, double gc2, double tmin,
                                                      double tmax, double inv_dz, int W, int H, double fx, double fy,
                                                      double cx, double cy, PoseArg T, float* __restrict__ vtx,
                                                      float* __restrict__ nrm) {
    constexpr uint32_t kMask = (kRayLanes == 32) ? 0xffffffffu : ((1u << kRayLanes) - 1);
    const int j = threadIdx.x & (kRayLanes - 1);
    const int gshift = threadIdx.x & 63 & ~(kRayLanes - 1);  // first lane of this ray in the wave
    const int64_t ray = (int64_t)blockIdx.x * (256 / kRayLanes) + (threadIdx.x / kRayLanes);
    if (ray >= (int64_t)W * H) return;  // all lanes of a ray leave together
    const int u = (int)(ray % W), v = (int)(ray / W);
    const double* P = T.v;
    const double dc0 = ((double)u - cx) / fx, dc1 = ((double)v - cy) / fy;
    const double gd0 = ((P[0] * dc0 + P[1] * dc1) + P[2]) * g.inv;
    const double gd1 = ((P[4] * dc0 + P[5] * dc1) + P[6]) * g.inv;
    const double gd2 = ((P[8] * dc0 + P[9] * dc1) + P[10]) * g.inv;
    const double dz = 0.5 * g.side;

    // interval of the walk inside the sampling box (widened by two steps)
    double t0 = -1e300, t1 = 1e300;
    const double hi = (double)(g.dim - 1);
    slab(gc0, gd0, 0.0, hi, t0, t1);
    slab(gc1, gd1, 0.0, hi, t0, t1);
    slab(gc2, gd2, 0.0, hi, t0, t1);
    const double n_steps = floor((tmax - tmin) / dz) + 1.0;  // s with tmin + s dz <= tmax, plus one
    double s_lo = floor((t0 - tmin) / dz) - 2.0, s_hi = ceil((t1 - tmin) / dz) + 2.0;
    s_lo = fmax(s_lo, 0.0);
    s_hi = fmin(s_hi, n_steps);

    double t_hit = -1.0;
    if (s_lo <= s_hi) {  // the two-step margins also cover rounding in the interval
        const double qnan = __builtin_nan("");
        const int s_end = (int)s_hi;
        // reciprocals for the hop estimates only (not part of any sample)
        const double rg0 = fabs(gd0) > 1e-300 ? 1.0 / gd0 : 0.0;
        const double rg1 = fabs(gd1) > 1e-300 ? 1.0 / gd1 : 0.0;
        const double rg2 = fabs(gd2) > 1e-300 ? 1.0 / gd2 : 0.0;
        int s = (int)s_lo;
        double c_f = qnan;  // sample of the step before the round (NaN: missing)
        for (;;) {
            const int sj = s + j;
            const double tj = tmin + (double)sj * dz;
            const bool beyond = sj > s_end || tj > tmax;
            const double x0 = gc0 + tj * gd0, x1 = gc1 + tj * gd1, x2 = gc2 + tj * gd2;
            const double f0 = floor(x0), f1 = floor(x1), f2 = floor(x2);
            const bool inr = !beyond && in_range(g, f0, f1, f2);
            double fj = qnan;
            if (inr) {
                double f;
                if (sample_cell(g, x0, x1, x2, f0, f1, f2, f)) fj = f;
            }
            // brick of the round's last step (-1: beyond the walk or outside the range)
            const int bq = __shfl(inr ? pack_brick(f0, f1, f2) : -1, kRayLanes - 1, kRayLanes);
            const bool hop = g.flags && bq >= 0 &&
                             g.flags[(((uint32_t)bq >> 20) * (uint32_t)g.nb + (((uint32_t)bq >> 10) & 1023u)) *
                                         (uint32_t)g.nb + ((uint32_t)bq & 1023u)] != 0;
            // the walk's rule in step order
            double pf = __shfl_up(fj, 1, kRayLanes);
            if (j == 0) pf = c_f;
            int ev = 0;  // 1: surface between the previous step and this one; 2: back of a surface
            if (!__builtin_isnan(fj) && !__builtin_isnan(pf)) {
                if (pf > 0.0 && fj <= 0.0)
                    ev = 1;
                else if (pf < 0.0 && fj >= 0.0)
                    ev = 2;
            }
            const uint32_t evm = (uint32_t)(__ballot(ev != 0) >> gshift) & kMask;
            if (evm) {
                const int first = __ffs((int)evm) - 1;
                const double tp = tmin + (double)(sj - 1) * dz;  // the previous step's depth, as the walk had it
                const double th = ev == 1 ? tp + (tj - tp) * (pf / (pf - fj)) : -1.0;
                t_hit = __shfl(th, first, kRayLanes);
                break;
            }
            if ((uint32_t)(__ballot(beyond) >> gshift) & kMask) break;  // walked past the end
            c_f = __shfl(fj, kRayLanes - 1, kRayLanes);
            const int sq = s + kRayLanes - 1;
            s += kRayLanes;
            // hop from the round's last step (in a skippable brick, so its
            // sample is missing or > 0) to the last step still in the brick;
            // the round then starts there with no previous sample (the
            // skipped steps hold no event and that step cannot be one)
            if (hop) {
                const int b0 = bq & 1023, b1 = (bq >> 10) & 1023, b2 = bq >> 20;
                const double tq = tmin + (double)sq * dz;
                const double te = fmin(fmin(brick_exit(gc0, gd0, rg0, b0), brick_exit(gc1, gd1, rg1, b1)),
                                       brick_exit(gc2, gd2, rg2, b2));
                const double jump = fmin(floor((te - tq) * inv_dz) - 1.0, (double)(s_end - sq));
                if (jump >= 2.0) {
                    const int sl = sq + (int)jump;
                    const double tl = tmin + (double)sl * dz;
                    const double l0 = floor(gc0 + tl * gd0), l1 = floor(gc1 + tl * gd1), l2 = floor(gc2 + tl * gd2);
                    if (!(tl > tmax) && in_range(g, l0, l1, l2) && pack_brick(l0, l1, l2) == bq) {
                        s = sl;
                        c_f = qnan;
                    }
                }
            }
        }
    }
    float pv3[3], pn3[3];
    const float fnan = __builtin_nanf("");
    for (int a = 0; a < 3; ++a) pv3[a] = pn3[a] = fnan;
    if (t_hit > 0.0) {
        // the six samples one voxel away along +x, -x, +y, -y, +z, -z, spread
        // over the ray's lanes (two rounds with four lanes)
        const double h0 = gc0 + t_hit * gd0, h1 = gc1 + t_hit * gd1, h2 = gc2 + t_hit * gd2;
        double gq[6];
        bool ok = true;
#pragma unroll 1
        for (int q0 = 0; q0 < 6; q0 += kRayLanes) {
            const int q = q0 + j;
            const double sg = (q & 1) ? -1.0 : 1.0;  // h - 1 == h + (-1) exactly
            const int a = q >> 1;
            double gv = 0.0;
            const bool okq = q >= 6 || sample(g, a == 0 ? h0 + sg : h0, a == 1 ? h1 + sg : h1, a == 2 ? h2 + sg : h2, gv);
            ok = ok && ((uint32_t)(__ballot(!okq) >> gshift) & kMask) == 0;
#pragma unroll
            for (int r = 0; r < 6; ++r)
                if (r >= q0 && r < q0 + kRayLanes) gq[r] = __shfl(gv, r - q0, kRayLanes);
        }
        if (ok) {
            const double gw0 = gq[0] - gq[1], gw1 = gq[2] - gq[3], gw2 = gq[4] - gq[5];
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
                pv3[0] = (float)pc0;
                pv3[1] = (float)pc1;
                pv3[2] = (float)pc2;
                pn3[0] = (float)nc0;
                pn3[1] = (float)nc1;
                pn3[2] = (float)nc2;
            }
        }
    }
    for (int a = j; a < 3; a += kRayLanes) {
        vtx[3 * (size_t)ray + a] = pv3[a];
        nrm[3 * (size_t)ray + a] = pn3[a];
    }
}

Geo make_geo(const TsdfDesc& d) {
    Geo g;
    g.vox = reinterpret_cast<float2*>(d.voxels);
    g.dim = d.dim;
    g.side = d.size / (double)d.dim;
    g.inv = 1.0 / g.side;
    for (int a = 0; a < 3; ++a) g.o[a] = d.origin[a];
    g.nb = (d.dim + 7) / 8;
    const size_t nb3 = (size_t)g.nb * g.nb * g.nb;
    char* br = static_cast<char*>(d.bricks);
    g.cnt = br ? reinterpret_cast<int*>(br) : nullptr;  // one count per brick
    g.flags = br ? reinterpret_cast<uint8_t*>(br + tsdf_count_bytes(nb3)) : nullptr;
    return g;
}

unsigned stride_grid(int64_t n) {
    const int64_t blocks = (n + 255) / 256;
    return (unsigned)(blocks < 65536 ? blocks : 65536);
}

hipError_t launch_flags(const Geo& g, hipStream_t s) {
    const int64_t nb3 = (int64_t)g.nb * g.nb * g.nb;
    hipLaunchKernelGGL(k_tsdf_flags, dim3((unsigned)((nb3 + 255) / 256)), dim3(256), 0, s, g.cnt, g.flags, g.nb);
    return hipGetLastError();
}

}  // namespace

size_t tsdf_count_bytes(size_t nb3) { return (nb3 * 4 + 255) / 256 * 256; }

size_t tsdf_brick_bytes(int dim) {
    const size_t nb = (size_t)(dim + 7) / 8, nb3 = nb * nb * nb;
    return tsdf_count_bytes(nb3) + (nb3 + 255) / 256 * 256;
}

hipError_t launch_tsdf_fill(const TsdfDesc& d, hipStream_t s) {
    const int64_t n = (int64_t)d.dim * d.dim * d.dim;
    hipLaunchKernelGGL(k_tsdf_fill, dim3(stride_grid(n)), dim3(256), 0, s, reinterpret_cast<float2*>(d.voxels), n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !d.bricks) return e;
    const Geo g = make_geo(d);
    const int64_t nc = (int64_t)g.nb * g.nb * g.nb;
    hipLaunchKernelGGL(k_tsdf_zero_counts, dim3(stride_grid(nc)), dim3(256), 0, s, g.cnt, nc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_flags(g, s);
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
    const Geo g = make_geo(d);
    const double inv_mu = 1.0 / d.mu;  // correctly rounded (IEEE division)
    hipLaunchKernelGGL(k_tsdf_integrate, grid, dim3(64, 4), 0, s, g, c, d.mu, inv_mu, d.max_weight, depth, W, H, K[0],
                       K[1], K[2], K[3], T);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !d.bricks) return e;
    return launch_flags(g, s);
}

hipError_t launch_tsdf_raycast(const TsdfDesc& d, double tmin, double tmax, int W, int H, const double* K, PoseArg T,
                               float* vtx, float* nrm, hipStream_t s) {
    const Geo g = make_geo(d);
    double gc[3];  // camera centre in grid coordinates, minus half a voxel
    for (int a = 0; a < 3; ++a) gc[a] = (T.v[4 * a + 3] - d.origin[a]) * g.inv - 0.5;
    const int64_t rays = (int64_t)W * H;
    const int per_block = 256 / kRayLanes;
    const double inv_dz = 1.0 / (0.5 * g.side);
    hipLaunchKernelGGL(k_tsdf_raycast, dim3((unsigned)((rays + per_block - 1) / per_block)), dim3(256), 0, s, g,
                       gc[0], gc[1], gc[2], tmin, tmax, inv_dz, W, H, K[0], K[1], K[2], K[3], T, vtx, nrm);
    return hipGetLastError();
}

}  // namespace icpk
