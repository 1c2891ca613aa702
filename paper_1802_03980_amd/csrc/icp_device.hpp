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

struct Pose {
    double r[9];
    double t[3];
};

struct Match {
    double p[3];   // live point moved by the current pose, p' = R p + t
    double d[3];   // q - p'
    float n[3];    // model normal n_q
    int bin;
};

// Projective association of live pixel i (paper Sec. 3): move the live point
// by the current pose, project it into the model image, round to the nearest
// pixel, fetch the model point and normal there, then gate on validity,
// distance and normal agreement.  Returns an ICP_PX_* code.
__device__ __forceinline__ int associate(const LevelDesc& L, int i, const Pose& T, double d2max, double cos_max,
                                         Match& m) {
    const int S = L.npx;
    const float vx = L.LV[i], vy = L.LV[S + i], vz = L.LV[2 * S + i];
    const float nx = L.LN[i], ny = L.LN[S + i], nz = L.LN[2 * S + i];
    if (!(fin(vx) && fin(vy) && fin(vz) && fin(nx) && fin(ny) && fin(nz))) return kInvalidLive;
    const double px = vx, py = vy, pz = vz;
#pragma unroll
    for (int k = 0; k < 3; ++k) m.p[k] = ((T.r[3 * k] * px + T.r[3 * k + 1] * py) + T.r[3 * k + 2] * pz) + T.t[k];
    if (!(m.p[2] > 0.0)) return kBehind;
    const double uf = L.fx * (m.p[0] / m.p[2]) + L.cx;
    const double vf = L.fy * (m.p[1] / m.p[2]) + L.cy;
    const double uu = floor(uf + 0.5), vv = floor(vf + 0.5);
    if (!(uu >= 0.0 && uu <= (double)(L.W - 1) && vv >= 0.0 && vv <= (double)(L.H - 1))) return kOutside;
    const int j = (int)vv * L.W + (int)uu;
    const float qx = L.MV[j], qy = L.MV[S + j], qz = L.MV[2 * S + j];
    const float mx = L.MN[j], my = L.MN[S + j], mz = L.MN[2 * S + j];
    if (!(fin(qx) && fin(qy) && fin(qz) && fin(mx) && fin(my) && fin(mz))) return kInvalidModel;
    m.d[0] = (double)qx - m.p[0];
    m.d[1] = (double)qy - m.p[1];
    m.d[2] = (double)qz - m.p[2];
    const double d2 = (m.d[0] * m.d[0] + m.d[1] * m.d[1]) + m.d[2] * m.d[2];
    if (!(d2 < d2max)) return kFar;
    const double nxd = nx, nyd = ny, nzd = nz;
    double c = 0.0;
    {
        const double r0 = (T.r[0] * nxd + T.r[1] * nyd) + T.r[2] * nzd;
        const double r1 = (T.r[3] * nxd + T.r[4] * nyd) + T.r[5] * nzd;
        const double r2 = (T.r[6] * nxd + T.r[7] * nyd) + T.r[8] * nzd;
        c = (r0 * (double)mx + r1 * (double)my) + r2 * (double)mz;
    }
    if (!(c >= cos_max)) return kAngle;
    m.n[0] = mx;
    m.n[1] = my;
    m.n[2] = mz;
    m.bin = dist_bin(d2);
    return kGated;
}

// The row of Eq. (3) for a kept pair and its 28 products.  With the
// small-angle transform of Eq. (2) applied to p', the residual of Eq. (1) is
// n . (p' + w x p' + tau - q) = a . x - b, a = [p' x n, n], b = n . (q - p').
__device__ __forceinline__ void accumulate_row(const Match& m, float (&acc)[ICP_NMOM]) {
    const float px = (float)m.p[0], py = (float)m.p[1], pz = (float)m.p[2];
    const float dx = (float)m.d[0], dy = (float)m.d[1], dz = (float)m.d[2];
    const float nx = m.n[0], ny = m.n[1], nz = m.n[2];
    float r[7];
    r[0] = py * nz - pz * ny;
    r[1] = pz * nx - px * nz;
    r[2] = px * ny - py * nx;
    r[3] = nx;
    r[4] = ny;
    r[5] = nz;
    r[6] = __builtin_fmaf(nz, dz, __builtin_fmaf(ny, dy, nx * dx));
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
