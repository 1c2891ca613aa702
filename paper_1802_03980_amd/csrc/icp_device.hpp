// Device-side steps of one ICP iteration for gfx950.
//
// Every match decision (transform, projection, pixel rounding, gates, bin) is
// FP64 and the translation units that include this header are compiled with
// -ffp-contract=off: each product and sum is rounded exactly as written, so
// the decisions do not depend on instruction selection.  The rows [a | b] and
// their moments are FP32 (explicit fmaf).
#pragma once

#include <hip/hip_runtime.h>

#include "icp_common.hpp"

namespace icpk {

constexpr double kBinW = 1.0 / 8192.0;  // histogram bin width, 2^-13 m

enum : int {
    kInvalidLive = ICP_PX_INVALID_LIVE,
    kBehind = ICP_PX_BEHIND,
    kOutside = ICP_PX_OUTSIDE,
    kInvalidModel = ICP_PX_INVALID_MODEL,
    kFar = ICP_PX_FAR,
    kAngle = ICP_PX_ANGLE,
    kGated = ICP_PX_GATED,
};

__device__ __forceinline__ bool fin(float a) { return __builtin_isfinite(a); }

// Bin of a squared distance: the unique k with (k w)^2 <= d2 < ((k+1) w)^2.
// With w = 2^-13, (k w)^2 = k^2 2^-26 exactly, and k^2 is an integer, so k is
// the integer square root of floor(d2 2^26) (below 2^20 for any gated pair,
// hence exact in FP32).  The FP32 square root of that integer lands within
// one of the root; two integer checks settle it.
__device__ __forceinline__ int dist_bin(double d2) {
    const double D = d2 * 67108864.0;  // times 2^26, exact
    if (!(D < 1048576.0)) return ICP_HIST_BINS - 1;
    const int n = (int)D;
    int k = (int)__builtin_amdgcn_sqrtf((float)n);  // hardware square root, 1 ulp
    k -= (int)__umul24(k, k) > n ? 1 : 0;
    k += (int)__umul24(k + 1, k + 1) <= n ? 1 : 0;
    return k;
}

// floor(f a/b + c + 1/2) with a/b rounded as an IEEE FP64 division rounds it.
// The quotient comes from a refined reciprocal (error a few FP64 ulps); when
// f a/b + c + 1/2 lies more than 1e-6 from an integer no rounding of the
// quotient can move the floor, otherwise the correctly rounded division
// decides.  `look` false skips the check (the result is not used).
__device__ __forceinline__ void project_round(double a, double b, double f, double c, double a2, double f2,
                                              double c2, bool look, double& uu, double& vv) {
    double r = __builtin_amdgcn_rcp(b);
    r = __builtin_fma(r, __builtin_fma(-b, r, 1.0), r);
    r = __builtin_fma(r, __builtin_fma(-b, r, 1.0), r);
    const double uf = f * (a * r) + c + 0.5;
    const double vf = f2 * (a2 * r) + c2 + 0.5;
    uu = floor(uf);
    vv = floor(vf);
    const double tu = uf - uu, tv = vf - vv;
    const bool safe = tu > 1e-6 && tu < 1.0 - 1e-6 && tv > 1e-6 && tv < 1.0 - 1e-6;
    if (look && !safe) {
        uu = floor(f * (a / b) + c + 0.5);
        vv = floor(f2 * (a2 / b) + c2 + 0.5);
    }
}

#define ICP_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ const ICP_GLOBAL T* gconst(const T* p) {
    return (const ICP_GLOBAL T*)p;
}

template <typename T>
__device__ __forceinline__ ICP_GLOBAL T* gmut(T* p) {
    return (ICP_GLOBAL T*)p;
}

// A value that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ double uniform(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

struct Pose {
    double r[9];
    double t[3];
};

__device__ __forceinline__ Pose load_pose(const ProbState* st) {
    Pose T;
    const ICP_GLOBAL double* R = gconst(st->R);
    const ICP_GLOBAL double* t = gconst(st->t);
#pragma unroll
    for (int k = 0; k < 9; ++k) T.r[k] = uniform(R[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) T.t[k] = uniform(t[k]);
    return T;
}

// The maps and geometry of one level held in registers for a pass.
struct Lvl {
    const ICP_GLOBAL float* D;    // live depth of the level
    const ICP_GLOBAL float* LN;   // live normal planes
    const ICP_GLOBAL double* XQ;  // (u - cx) / fx, u = 0..W
    const ICP_GLOBAL double* YQ;  // (v - cy) / fy, v = 0..H
    const ICP_GLOBAL float* MV;
    const ICP_GLOBAL float* MN;
    int W, H, npx, ps;
    float invW;
    double fx, fy, cx, cy, umax, vmax;
    double rfx, rfy;  // RN(1/fx), RN(1/fy)
};

__device__ __forceinline__ Lvl load_level(const LevelDesc& L) {
    Lvl v;
    v.D = gconst(L.D);
    v.LN = gconst(L.LN);
    v.ps = L.ps;
    v.XQ = gconst(L.XQ);
    v.YQ = gconst(L.YQ);
    v.MV = gconst(L.MV);
    v.MN = gconst(L.MN);
    v.W = L.W;
    v.H = L.H;
    v.npx = L.npx;
    v.invW = 1.0f / (float)L.W;
    v.fx = L.fx;
    v.fy = L.fy;
    v.cx = L.cx;
    v.cy = L.cy;
    v.umax = L.umax;
    v.vmax = L.vmax;
    v.rfx = L.rfx;
    v.rfy = L.rfy;
    return v;
}

// a/b rounded as the IEEE FP64 division rounds it, given y = RN(1/b): q =
// RN(a y) is within an ulp of a/b, and one correction RN(q + RN(a - b q) y)
// (the remainder exact by FMA) is the correctly rounded quotient (Markstein's
// theorem for division by a correctly rounded reciprocal; no operand here
// comes near the underflow or overflow range).
__device__ __forceinline__ double div_rn(double a, double b, double y) {
    const double q = a * y;
    return __builtin_fma(__builtin_fma(-q, b, a), y, q);
}

// The back-projection quotient (t - c)/f of the front end's tables, without
// a division (y = RN(1/f) from the descriptor): saves the pixel passes a
// dependent table load per pixel.
__device__ __forceinline__ double bp_quot(int t, double c, double f, double y) {
    return div_rn((double)t - c, f, y);
}

// Association result of one pixel handed to the caller: the code, the bin
// (gated pixels) and the FP32 inputs of its row (p', q - p', n_q).
struct PixelOut {
    int code;
    int bin;
    float p[3];
    float d[3];
    float n[3];
};

// The association (paper Sec. 3) is written as straight-line code: every
// quantity is computed for every pixel (NaN inputs propagate and fail every
// comparison) and the code is selected at the end in the order the checks
// are defined, so a wavefront runs one path.  The live maps store an invalid
// pixel as NaN in all three components, so one component decides their
// validity.  The live vertex of each pixel is rebuilt from the level's depth
// with the front end's arithmetic and its normal is read from the stored
// normal planes: 16 bytes of live data per pixel instead of 24.
typedef float vf4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bool depth_ok(float z) { return __builtin_isfinite(z) && z > 0.0f; }

// Live vertex p and forward-difference normal n (flipped to face the camera)
// of a pixel with depth z, from its right and lower neighbours' depths and the
// back-projection quotients x0 = (u - cx)/fx, x1 = (u + 1 - cx)/fx,
// y0 = (v - cy)/fy, y1 = (v + 1 - cy)/fy; NaN where invalid.  The one
// arithmetic of the live maps: the front-end kernels and the pixel passes
// both call it, so the maps they see are the same bits.
__device__ __forceinline__ void live_vertex(float z, double x0, double y0, float (&p)[3]) {
    const float qnan = __builtin_nanf("");
    const bool ok = depth_ok(z);
    const double zd = (double)z;
    p[0] = ok ? (float)(zd * x0) : qnan;
    p[1] = ok ? (float)(zd * y0) : qnan;
    p[2] = ok ? z : qnan;
}

__device__ __forceinline__ void live_from_depth(float z, float zr, float zb, bool has_r, bool has_b, double x0,
                                                double x1, double y0, double y1, float (&p)[3], float (&n)[3]) {
    const float qnan = __builtin_nanf("");
    for (int k = 0; k < 3; ++k) n[k] = qnan;
    live_vertex(z, x0, y0, p);
    const bool ok = depth_ok(z);
    if (ok && has_r && has_b && depth_ok(zr) && depth_ok(zb)) {
        const double zrd = (double)zr, zbd = (double)zb;
        const float pr[3] = {(float)(zrd * x1), (float)(zrd * y0), zr};
        const float pd[3] = {(float)(zbd * x0), (float)(zbd * y1), zb};
        double e1[3], e2[3];
        for (int k = 0; k < 3; ++k) {
            e1[k] = (double)pr[k] - (double)p[k];
            e2[k] = (double)pd[k] - (double)p[k];
        }
        const double c0 = e1[1] * e2[2] - e1[2] * e2[1];
        const double c1 = e1[2] * e2[0] - e1[0] * e2[2];
        const double c2 = e1[0] * e2[1] - e1[1] * e2[0];
        const double len2 = (c0 * c0 + c1 * c1) + c2 * c2;
        if (len2 > 0.0 && __builtin_isfinite(len2)) {
            const double len = sqrt(len2);
            const double y = 1.0 / len;  // one division, then c / len for each component
            double m0 = div_rn(c0, len, y), m1 = div_rn(c1, len, y), m2 = div_rn(c2, len, y);
            const double side = (m0 * (double)p[0] + m1 * (double)p[1]) + m2 * (double)p[2];
            if (side > 0.0) {
                m0 = -m0;
                m1 = -m1;
                m2 = -m2;
            }
            n[0] = (float)m0;
            n[1] = (float)m1;
            n[2] = (float)m2;
        }
    }
}

// Row and column of pixel i (an FP32 estimate of i / W, corrected by one).
__device__ __forceinline__ void pixel_uv(const Lvl& L, int i, int& u, int& v) {
    v = (int)((float)i * L.invW);
    v -= v * L.W > i ? 1 : 0;
    v += (v + 1) * L.W <= i ? 1 : 0;
    u = i - v * L.W;
}

// What a pixel's live vertex comes from: its depth (the vertex is rebuilt
// from it with the front end's arithmetic).  Its normal is read from the
// stored normal planes with the model gather (the normal needs two
// neighbours, a square root and three divisions: cheaper to read than to
// rebuild every iteration).  A loop loads the depths rounds ahead.
template <int NPX>
struct LiveIn {
    float z[NPX];
};

template <int NPX>
__device__ __forceinline__ LiveIn<NPX> load_live(const Lvl& L, int i) {
    LiveIn<NPX> q;
#pragma unroll
    for (int k = 0; k < NPX; ++k) q.z[k] = L.D[min(i + k, L.npx - 1)];  // past the end: the last pixel (invalid)
    return q;
}

// The association of a pixel in three phases, so that a loop can issue one
// round's model gathers before it decides the previous round's pixels:
// projection (live point moved by the pose, projected and rounded to a model
// pixel), gather (the model point and normal there), decision (gates, bin and
// the row's inputs).
template <int NPX>
struct Proj {
    double P[NPX][3];  // p' = R p + t
    int j[NPX];        // model pixel gathered (0 when nothing is looked up)
    bool vok[NPX], front[NPX], inside[NPX];
};

template <int NPX>
struct Gath {
    float Q[NPX][3], M[NPX][3];  // model point and normal at the projection
    float N[NPX][3];             // live normal (rotated at the decision)
};

// Pixels at or beyond `lim` count as invalid live pixels (their planes may
// be any in-bounds data).
template <int NPX>
__device__ __forceinline__ Proj<NPX> assoc_project(const Lvl& L, int i, int lim, const LiveIn<NPX>& lq,
                                                   const Pose& T) {
    Proj<NPX> a;
#pragma unroll
    for (int k = 0; k < NPX; ++k) {
        int u, v;
        pixel_uv(L, min(i + k, L.npx - 1), u, v);
        float V[3];
        live_vertex(lq.z[k], bp_quot(u, L.cx, L.fx, L.rfx), bp_quot(v, L.cy, L.fy, L.rfy), V);
        a.vok[k] = (i + k < lim) && fin(V[2]);
        const double px = V[0], py = V[1], pz = V[2];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            a.P[k][c] = ((T.r[3 * c] * px + T.r[3 * c + 1] * py) + T.r[3 * c + 2] * pz) + T.t[c];
        a.front[k] = a.P[k][2] > 0.0;
        double uu, vv;
        project_round(a.P[k][0], a.P[k][2], L.fx, L.cx, a.P[k][1], L.fy, L.cy, a.vok[k] && a.front[k], uu, vv);
        a.inside[k] = uu >= 0.0 && uu <= L.umax && vv >= 0.0 && vv <= L.vmax;
        const bool look = a.vok[k] && a.front[k] && a.inside[k];
        a.j[k] = look ? (int)vv * L.W + (int)uu : 0;
    }
    return a;
}

template <int NPX>
__device__ __forceinline__ Gath<NPX> assoc_gather(const Lvl& L, int i, const Proj<NPX>& a) {
    Gath<NPX> g;
#pragma unroll
    for (int k = 0; k < NPX; ++k) {
        const int li = min(i + k, L.npx - 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            g.Q[k][c] = L.MV[3 * a.j[k] + c];
            g.M[k][c] = L.MN[3 * a.j[k] + c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) g.N[k][c] = L.LN[c * L.ps + li];
    }
    return g;
}

template <int NPX, class Emit>
__device__ __forceinline__ void assoc_decide(const Proj<NPX>& a, const Gath<NPX>& g, const Pose& T, double d2max,
                                             double cos_max, Emit&& emit) {
#pragma unroll
    for (int k = 0; k < NPX; ++k) {
        const float(&Q)[3] = g.Q[k];
        const float(&M)[3] = g.M[k];
        const double(&P)[3] = a.P[k];
        const bool nok = fin(g.N[k][2]);
        // the caller's level-0 model maps may be partly NaN: all six decide
        const bool mok = fin(Q[0]) && fin(Q[1]) && fin(Q[2]) && fin(M[0]) && fin(M[1]) && fin(M[2]);
        const double d0 = (double)Q[0] - P[0];
        const double d1 = (double)Q[1] - P[1];
        const double d2 = (double)Q[2] - P[2];
        const double dd = (d0 * d0 + d1 * d1) + d2 * d2;
        const bool near = dd < d2max;
        const double nxd = g.N[k][0], nyd = g.N[k][1], nzd = g.N[k][2];
        const double r0 = (T.r[0] * nxd + T.r[1] * nyd) + T.r[2] * nzd;
        const double r1 = (T.r[3] * nxd + T.r[4] * nyd) + T.r[5] * nzd;
        const double r2 = (T.r[6] * nxd + T.r[7] * nyd) + T.r[8] * nzd;
        const double cv = (r0 * (double)M[0] + r1 * (double)M[1]) + r2 * (double)M[2];
        const bool agree = cv >= cos_max;
        int code = kGated;
        code = agree ? code : kAngle;
        code = near ? code : kFar;
        code = mok ? code : kInvalidModel;
        code = a.inside[k] ? code : kOutside;
        code = a.front[k] ? code : kBehind;
        code = (a.vok[k] && nok) ? code : kInvalidLive;
        PixelOut o;
        o.code = code;
        o.bin = code == kGated ? dist_bin(dd) : -1;
        o.p[0] = (float)P[0];
        o.p[1] = (float)P[1];
        o.p[2] = (float)P[2];
        o.d[0] = (float)d0;
        o.d[1] = (float)d1;
        o.d[2] = (float)d2;
        o.n[0] = M[0];
        o.n[1] = M[1];
        o.n[2] = M[2];
        emit(k, o);
    }
}

// Projective association of live pixels i..i+NPX-1 (paper Sec. 3): move each
// live point by the current pose, project it into the model image, round to
// the nearest pixel, fetch the model point and normal there, then gate on
// validity, distance and normal agreement.
template <int NPX, class Emit>
__device__ __forceinline__ void associate_px(const Lvl& L, int i, int lim, const LiveIn<NPX>& lq, const Pose& T,
                                             double d2max, double cos_max, Emit&& emit) {
    const Proj<NPX> a = assoc_project<NPX>(L, i, lim, lq, T);
    assoc_decide<NPX>(a, assoc_gather<NPX>(L, i, a), T, d2max, cos_max, emit);
}

// Four pixels i..i+3 of one level, every pixel below npx valid.
template <class Emit>
__device__ __forceinline__ void associate4(const Lvl& L, int i, const Pose& T, double d2max, double cos_max,
                                           Emit&& emit) {
    associate_px<4>(L, i, L.npx, load_live<4>(L, i), T, d2max, cos_max, emit);
}

// The row r = [a | b] of Eq. (3) for a kept pair (see accumulate_row).
__device__ __forceinline__ void make_row(const float (&p)[3], const float (&d)[3], const float (&n)[3],
                                         float (&r)[7]) {
    r[0] = p[1] * n[2] - p[2] * n[1];
    r[1] = p[2] * n[0] - p[0] * n[2];
    r[2] = p[0] * n[1] - p[1] * n[0];
    r[3] = n[0];
    r[4] = n[1];
    r[5] = n[2];
    r[6] = __builtin_fmaf(n[2], d[2], __builtin_fmaf(n[1], d[1], n[0] * d[0]));
}

// The row of Eq. (3) for a kept pair and its 28 products.  With the
// small-angle transform of Eq. (2) applied to p', the residual of Eq. (1) is
// n . (p' + w x p' + tau - q) = a . x - b, a = [p' x n, n], b = n . (q - p').
__device__ __forceinline__ void accumulate_row(const float (&p)[3], const float (&d)[3], const float (&n)[3],
                                               float (&acc)[ICP_NMOM]) {
    float r[7];
    r[0] = p[1] * n[2] - p[2] * n[1];
    r[1] = p[2] * n[0] - p[0] * n[2];
    r[2] = p[0] * n[1] - p[1] * n[0];
    r[3] = n[0];
    r[4] = n[1];
    r[5] = n[2];
    r[6] = __builtin_fmaf(n[2], d[2], __builtin_fmaf(n[1], d[1], n[0] * d[0]));
    int k = 0;
#pragma unroll
    for (int a = 0; a < 7; ++a) {
#pragma unroll
        for (int b = a; b < 7; ++b) {
            acc[k] = __builtin_fmaf(r[a], r[b], acc[k]);
            ++k;
        }
    }
}

// ---------------------------------------------------------------- solve

__device__ __forceinline__ int tri7(int i, int j) { return i * 7 - i * (i - 1) / 2 + (j - i); }

// Regularised normal equations of Eq. (5): (A^T A + 2 lambda n P^T P) x = A^T b,
// P = [I3 | 0], solved by LDL^T (the system is symmetric positive definite
// whenever it is solvable).  Returns an ICP_LEVEL_* status.
// Rotation vector of a rotation matrix (angle in [0, pi)): v = (R32 - R23,
// R13 - R31, R21 - R12) has length 2 sin(th) and trace(R) = 1 + 2 cos(th),
// so th = atan2(|v| / 2, (trace - 1) / 2) and the vector is v th / (2 sin th)
// (v / 2 when |v| is below 1e-12).
__device__ inline void rotation_vector(const double* R, double* w) {
    const double v0 = R[7] - R[5], v1 = R[2] - R[6], v2 = R[3] - R[1];
    const double s = 0.5 * sqrt((v0 * v0 + v1 * v1) + v2 * v2);
    const double c = 0.5 * (((R[0] + R[4]) + R[8]) - 1.0);
    const double f = s < 0.5e-12 ? 0.5 : atan2(s, c) / (2.0 * s);
    w[0] = v0 * f;
    w[1] = v1 * f;
    w[2] = v2 * f;
}

// Eq. (4)/(5): (A^T A + 2 lambda n P^T P) x = A^T b, LDL^T in FP64.  With the
// damping anchored to the IMU prior (kp.anchor_to_imu, imu_R given), the
// damped angles are those of the deviation after the update, w + d with
// d = Log(R imu_R^T), R the rotation before it: the right-hand side loses
// 2 lambda n d in its rotation rows.
__device__ inline int solve_regularised(const double* M, int64_t n, const KParams& kp, const double* R,
                                        const double* imu_R, double* x) {
    for (int k = 0; k < 6; ++k) x[k] = 0.0;
    if (n < kp.min_corr) return ICP_TOO_FEW_CORR;
    double A[6][6], g[6];
    for (int i = 0; i < 6; ++i) {
        for (int j = i; j < 6; ++j) A[i][j] = A[j][i] = M[tri7(i, j)];
        g[i] = M[tri7(i, 6)];
    }
    const double nd = (double)n;
    double lam = kp.lambda_c;
    if (kp.lambda_mode == ICP_LAMBDA_C_OVER_SQRT_N) lam = kp.lambda_c / sqrt(nd);
    else if (kp.lambda_mode == ICP_LAMBDA_C_OVER_N) lam = kp.lambda_c / nd;
    else if (kp.lambda_mode == ICP_LAMBDA_C_OVER_N2) lam = kp.lambda_c / (nd * nd);
    for (int i = 0; i < 3; ++i) A[i][i] += 2.0 * lam * nd;
    if (kp.anchor_to_imu && imu_R) {
        double Dv[9], d[3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)  // R imu_R^T
                Dv[3 * i + j] = (R[3 * i] * imu_R[3 * j] + R[3 * i + 1] * imu_R[3 * j + 1]) + R[3 * i + 2] * imu_R[3 * j + 2];
        rotation_vector(Dv, d);
        for (int i = 0; i < 3; ++i) g[i] -= 2.0 * lam * nd * d[i];
    }
    double dmax = 0.0;
    for (int i = 0; i < 6; ++i) dmax = A[i][i] > dmax ? A[i][i] : dmax;
    // A = L D L^T, L unit lower triangular (stored below the diagonal of A)
    double D[6];
    for (int j = 0; j < 6; ++j) {
        double dj = A[j][j];
        for (int k = 0; k < j; ++k) dj -= A[j][k] * A[j][k] * D[k];
        if (!(dj > kp.ill_cond_eps * dmax)) return ICP_ILL_COND;
        D[j] = dj;
        for (int i = j + 1; i < 6; ++i) {
            double s = A[i][j];
            for (int k = 0; k < j; ++k) s -= A[i][k] * A[j][k] * D[k];
            A[i][j] = s / dj;
        }
    }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double s = g[i];
        for (int k = 0; k < i; ++k) s -= A[i][k] * y[k];
        y[i] = s;
    }
    for (int i = 0; i < 6; ++i) y[i] = y[i] / D[i];
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 6; ++k) s -= A[k][i] * x[k];
        x[i] = s;
    }
    for (int i = 0; i < 6; ++i)
        if (!__builtin_isfinite(x[i])) {
            for (int k = 0; k < 6; ++k) x[k] = 0.0;
            return ICP_NONFINITE;
        }
    return ICP_LEVEL_OK;
}

// Left-compose Exp(w, tau) in SE(3) onto (R, t).  The rotation is built from
// the unit quaternion (cos(th/2), sin(th/2) w/th); the translation part is
// V tau = tau + B (w x tau) + C (w x (w x tau)) with B = (1 - cos th)/th^2 and
// C = (th - sin th)/th^3 (series below 1e-4 rad).  First order it is the
// small-angle transform of Eq. (2).
__device__ inline void compose_exp(const double* x, double* R, double* t) {
    const double w0 = x[0], w1 = x[1], w2 = x[2];
    const double th2 = (w0 * w0 + w1 * w1) + w2 * w2;
    const double th = sqrt(th2);
    double qs, qw, B, C;
    if (th < 1e-4) {
        qs = 0.5 - th2 / 48.0;
        qw = 1.0 - th2 / 8.0 + th2 * th2 / 384.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        const double sh = sin(0.5 * th);
        qs = sh / th;
        qw = cos(0.5 * th);
        B = 2.0 * sh * sh / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    const double qx = qs * w0, qy = qs * w1, qz = qs * w2;
    double dR[9];
    dR[0] = 1.0 - 2.0 * (qy * qy + qz * qz);
    dR[1] = 2.0 * (qx * qy - qz * qw);
    dR[2] = 2.0 * (qx * qz + qy * qw);
    dR[3] = 2.0 * (qx * qy + qz * qw);
    dR[4] = 1.0 - 2.0 * (qx * qx + qz * qz);
    dR[5] = 2.0 * (qy * qz - qx * qw);
    dR[6] = 2.0 * (qx * qz - qy * qw);
    dR[7] = 2.0 * (qy * qz + qx * qw);
    dR[8] = 1.0 - 2.0 * (qx * qx + qy * qy);
    const double ta = x[3], tb = x[4], tc = x[5];
    const double c1[3] = {w1 * tc - w2 * tb, w2 * ta - w0 * tc, w0 * tb - w1 * ta};
    const double c2[3] = {w1 * c1[2] - w2 * c1[1], w2 * c1[0] - w0 * c1[2], w0 * c1[1] - w1 * c1[0]};
    const double dt[3] = {ta + B * c1[0] + C * c2[0], tb + B * c1[1] + C * c2[1], tc + B * c1[2] + C * c2[2]};
    double Rn[9], tn[3];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) Rn[3 * i + j] = dR[3 * i] * R[j] + dR[3 * i + 1] * R[3 + j] + dR[3 * i + 2] * R[6 + j];
        tn[i] = dR[3 * i] * t[0] + dR[3 * i + 1] * t[1] + dR[3 * i + 2] * t[2] + dt[i];
    }
    for (int k = 0; k < 9; ++k) R[k] = Rn[k];
    for (int k = 0; k < 3; ++k) t[k] = tn[k];
}

// ---------------------------------------------------------------- wave ops

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace icpk
