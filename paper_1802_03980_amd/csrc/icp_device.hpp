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
// k w and its square are exact in FP64 (w = 2^-13, k < 2^13), so the result
// depends on the value of d2 alone; the FP32 square root only seeds the search.
__device__ __forceinline__ int dist_bin(double d2) {
    int k = (int)(__builtin_sqrtf((float)d2) * 8192.0f);
    k = k > ICP_HIST_BINS - 1 ? ICP_HIST_BINS - 1 : k;
    while (k > 0) {
        double e = (double)k * kBinW;
        if (e * e <= d2) break;
        --k;
    }
    while (k < ICP_HIST_BINS - 1) {
        double e = (double)(k + 1) * kBinW;
        if (e * e > d2) break;
        ++k;
    }
    return k;
}

#define ICP_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ const ICP_GLOBAL T* gconst(const T* p) {
    return (const ICP_GLOBAL T*)p;
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
    const ICP_GLOBAL float* LV;
    const ICP_GLOBAL float* LN;
    const ICP_GLOBAL float* MV;
    const ICP_GLOBAL float* MN;
    int W, npx, ps;
    double fx, fy, cx, cy, umax, vmax;
};

__device__ __forceinline__ Lvl load_level(const LevelDesc& L) {
    Lvl v;
    v.LV = gconst(L.LV);
    v.LN = gconst(L.LN);
    v.MV = gconst(L.MV);
    v.MN = gconst(L.MN);
    v.W = L.W;
    v.npx = L.npx;
    v.ps = L.ps;
    v.fx = L.fx;
    v.fy = L.fy;
    v.cx = L.cx;
    v.cy = L.cy;
    v.umax = (double)(L.W - 1);
    v.vmax = (double)(L.H - 1);
    return v;
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

typedef float vf4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ vf4 ld4(const ICP_GLOBAL float* p) { return *(const ICP_GLOBAL vf4*)p; }

// Projective association of live pixels i..i+3 (i a multiple of 4, paper
// Sec. 3): move each live point by the current pose, project it into the
// model image, round to the nearest pixel, fetch the model point and normal
// there, then gate on validity, distance and normal agreement.
//
// Written as straight-line code: every quantity is computed for every pixel
// (NaN inputs propagate and fail every comparison) and the code is selected
// at the end in the order the checks are defined, so a wavefront runs one
// path.  The live maps store an invalid pixel as NaN in all three components,
// so one component decides their validity.  The live vertices arrive as one
// 16-byte load per plane; the model gathers (12 contiguous bytes per map) of
// the four pixels and the live normals are issued together.
template <class Emit>
__device__ __forceinline__ void associate4(const Lvl& L, int i, const Pose& T, double d2max, double cos_max,
                                           Emit&& emit) {
    const int S = L.ps;
    const vf4 vx = ld4(L.LV + i), vy = ld4(L.LV + S + i), vz = ld4(L.LV + 2 * S + i);
    const float V[4][3] = {{vx.x, vy.x, vz.x}, {vx.y, vy.y, vz.y}, {vx.z, vy.z, vz.z}, {vx.w, vy.w, vz.w}};
    double P[4][3];
    int j[4];
    bool vok[4], front[4], inside[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        vok[k] = (i + k < L.npx) && fin(V[k][2]);
        const double px = V[k][0], py = V[k][1], pz = V[k][2];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            P[k][c] = ((T.r[3 * c] * px + T.r[3 * c + 1] * py) + T.r[3 * c + 2] * pz) + T.t[c];
        front[k] = P[k][2] > 0.0;
        const double uf = L.fx * (P[k][0] / P[k][2]) + L.cx;
        const double vf = L.fy * (P[k][1] / P[k][2]) + L.cy;
        const double uu = floor(uf + 0.5), vv = floor(vf + 0.5);
        inside[k] = uu >= 0.0 && uu <= L.umax && vv >= 0.0 && vv <= L.vmax;
        const bool look = vok[k] && front[k] && inside[k];
        j[k] = look ? (int)vv * L.W + (int)uu : 0;
    }
    const vf4 nx = ld4(L.LN + i), ny = ld4(L.LN + S + i), nz = ld4(L.LN + 2 * S + i);
    const float N[4][3] = {{nx.x, ny.x, nz.x}, {nx.y, ny.y, nz.y}, {nx.z, ny.z, nz.z}, {nx.w, ny.w, nz.w}};
    float Q[4][3], M[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Q[k][c] = L.MV[3 * j[k] + c];
            M[k][c] = L.MN[3 * j[k] + c];
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool nok = fin(N[k][2]);
        // the caller's level-0 model maps may be partly NaN: all six decide
        const bool mok = fin(Q[k][0]) && fin(Q[k][1]) && fin(Q[k][2]) && fin(M[k][0]) && fin(M[k][1]) &&
                         fin(M[k][2]);
        const double d0 = (double)Q[k][0] - P[k][0];
        const double d1 = (double)Q[k][1] - P[k][1];
        const double d2 = (double)Q[k][2] - P[k][2];
        const double dd = (d0 * d0 + d1 * d1) + d2 * d2;
        const bool near = dd < d2max;
        const double nxd = N[k][0], nyd = N[k][1], nzd = N[k][2];
        const double r0 = (T.r[0] * nxd + T.r[1] * nyd) + T.r[2] * nzd;
        const double r1 = (T.r[3] * nxd + T.r[4] * nyd) + T.r[5] * nzd;
        const double r2 = (T.r[6] * nxd + T.r[7] * nyd) + T.r[8] * nzd;
        const double cv = (r0 * (double)M[k][0] + r1 * (double)M[k][1]) + r2 * (double)M[k][2];
        const bool agree = cv >= cos_max;
        int code = kGated;
        code = agree ? code : kAngle;
        code = near ? code : kFar;
        code = mok ? code : kInvalidModel;
        code = inside[k] ? code : kOutside;
        code = front[k] ? code : kBehind;
        code = (vok[k] && nok) ? code : kInvalidLive;
        PixelOut o;
        o.code = code;
        o.bin = code == kGated ? dist_bin(dd) : -1;
        o.p[0] = (float)P[k][0];
        o.p[1] = (float)P[k][1];
        o.p[2] = (float)P[k][2];
        o.d[0] = (float)d0;
        o.d[1] = (float)d1;
        o.d[2] = (float)d2;
        o.n[0] = M[k][0];
        o.n[1] = M[k][1];
        o.n[2] = M[k][2];
        emit(k, o);
    }
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
__device__ inline int solve_regularised(const double* M, int64_t n, const KParams& kp, double* x) {
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
