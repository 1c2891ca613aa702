/*
 * A plain C client of the icp C ABI (include/icp.h): it renders a corner of
 * four planes analytically (model maps at the identity, the live depth seen
 * from a camera moved by a known rigid motion), uploads them with the HIP
 * runtime API, registers the live frame with icp_register and writes its
 * inputs and the resulting pose to a binary file, which the tests read back
 * and hand to the oracle.
 *
 *   register_planes OUT.bin
 *
 * Exit status: 0 registered; 3 no GPU (after the host-only calls, whose
 * results are printed); 1 any other failure.
 *
 * File layout (little endian): int32 W, H; double K[4] (fx, fy, cx, cy);
 * double imu_R[9]; double init_pose[16]; double T_true[16]; float depth[H*W];
 * float model_vtx[H*W*3]; float model_nrm[H*W*3]; double pose[16];
 * int32 status; int32 iters_total.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "icp.h"

enum { W = 160, H = 120, NPLANES = 4 };

static const double FX = 130.0, FY = 130.0, CX = 79.5, CY = 59.5;

/* planes n . X = n . p0, normals facing the camera at the origin */
static double PN[NPLANES][3] = {{0, 0, -1}, {0, -1, 0}, {1, 0, 0}, {-1, 0, -0.5}};
static const double P0[NPLANES][3] = {{0, 0, 3.0}, {0, 0.8, 0}, {-1.0, 0, 0}, {1.2, 0, 2.5}};

static void rot_axis_angle(const double axis[3], double ang, double R[9]) {
    const double n = sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
    const double x = axis[0] / n, y = axis[1] / n, z = axis[2] / n, c = cos(ang), s = sin(ang), C = 1.0 - c;
    const double r[9] = {c + x * x * C,     x * y * C - z * s, x * z * C + y * s,
                         y * x * C + z * s, c + y * y * C,     y * z * C - x * s,
                         z * x * C - y * s, z * y * C + x * s, c + z * z * C};
    memcpy(R, r, sizeof(r));
}

/* Nearest plane hit along the ray o + s * d (s > 0) in model coordinates;
   returns the plane index or -1, and the ray parameter in *s_out. */
static int hit(const double o[3], const double d[3], double* s_out) {
    int best = -1;
    double bs = 1e30;
    for (int k = 0; k < NPLANES; ++k) {
        const double* n = PN[k];
        const double den = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
        if (den >= -1e-9) continue;
        const double num = n[0] * (P0[k][0] - o[0]) + n[1] * (P0[k][1] - o[1]) + n[2] * (P0[k][2] - o[2]);
        const double s = num / den;
        if (s > 0 && s < bs) {
            bs = s;
            best = k;
        }
    }
    *s_out = bs;
    return best;
}

#define HIP_OK(x)                                                             \
    do {                                                                      \
        hipError_t e_ = (x);                                                  \
        if (e_ != hipSuccess) {                                               \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));           \
            return 1;                                                         \
        }                                                                     \
    } while (0)

int main(int argc, char** argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s OUT.bin\n", argv[0]);
        return 1;
    }
    /* host-only calls */
    icp_params params;
    icp_params_default(&params);
    const int32_t ws_w = W, ws_h = H;
    printf("abi %d levels %d iters %d %d %d workspace %zu strerror '%s'\n", icp_abi_version(), params.levels,
           params.iters[0], params.iters[1], params.iters[2], icp_workspace_bytes(1, &ws_w, &ws_h, params.levels),
           icp_strerror(ICP_EINVAL));
    for (int k = 0; k < NPLANES; ++k) {
        const double n = sqrt(PN[k][0] * PN[k][0] + PN[k][1] * PN[k][1] + PN[k][2] * PN[k][2]);
        for (int i = 0; i < 3; ++i) PN[k][i] /= n;
    }
    /* the live camera: X_model = R X_live + t */
    const double axis[3] = {0.3, 1.0, 0.2};
    double R[9];
    rot_axis_angle(axis, 1.5 * M_PI / 180.0, R);
    const double t[3] = {0.01, -0.005, 0.015};
    double T_true[16] = {0};
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) T_true[4 * i + j] = R[3 * i + j];
        T_true[4 * i + 3] = t[i];
    }
    T_true[15] = 1.0;
    double imu_R[9];
    const double imu_axis[3] = {1.0, -0.4, 0.7};
    double E[9];
    rot_axis_angle(imu_axis, 0.3 * M_PI / 180.0, E);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            imu_R[3 * i + j] = E[3 * i] * R[j] + E[3 * i + 1] * R[3 + j] + E[3 * i + 2] * R[6 + j];
    double init_pose[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};

    static float depth[H * W], mv[H * W * 3], mn[H * W * 3];
    const float qnan = nanf("");
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            const int i = v * W + u;
            const double d[3] = {(u - CX) / FX, (v - CY) / FY, 1.0};
            const double o[3] = {0, 0, 0};
            double s;
            const int k = hit(o, d, &s);
            if (k >= 0 && s > 0.5 && s < 4.0) {
                for (int c = 0; c < 3; ++c) {
                    mv[3 * i + c] = (float)(s * d[c]);
                    mn[3 * i + c] = (float)PN[k][c];
                }
            } else {
                for (int c = 0; c < 3; ++c) mv[3 * i + c] = mn[3 * i + c] = qnan;
            }
            /* live ray in model coordinates: origin t, direction R d */
            const double dm[3] = {R[0] * d[0] + R[1] * d[1] + R[2] * d[2], R[3] * d[0] + R[4] * d[1] + R[5] * d[2],
                                  R[6] * d[0] + R[7] * d[1] + R[8] * d[2]};
            const int kl = hit(t, dm, &s);
            depth[i] = (kl >= 0 && s > 0.5 && s < 4.0) ? (float)s : 0.0f; /* z of the live point = s (d_z = 1) */
        }

    icp_ctx* ctx = NULL;
    int rc = icp_ctx_create(0, 0, &ctx);
    if (rc == ICP_EDEVICE) {
        printf("no GPU: icp_ctx_create returned %d (%s)\n", rc, icp_strerror(rc));
        return 3;
    }
    if (rc != ICP_OK) {
        fprintf(stderr, "icp_ctx_create: %s\n", icp_strerror(rc));
        return 1;
    }
    float *d_depth = NULL, *d_mv = NULL, *d_mn = NULL;
    HIP_OK(hipMalloc((void**)&d_depth, sizeof(depth)));
    HIP_OK(hipMalloc((void**)&d_mv, sizeof(mv)));
    HIP_OK(hipMalloc((void**)&d_mn, sizeof(mn)));
    HIP_OK(hipMemcpy(d_depth, depth, sizeof(depth), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_mv, mv, sizeof(mv), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_mn, mn, sizeof(mn), hipMemcpyHostToDevice));
    const icp_intrinsics K = {FX, FY, CX, CY};
    double pose[16];
    icp_stats stats;
    rc = icp_register(ctx, d_depth, W, H, d_mv, d_mn, &K, imu_R, init_pose, &params, pose, &stats, NULL);
    if (rc != ICP_OK) {
        fprintf(stderr, "icp_register: %s (%s)\n", icp_strerror(rc), icp_last_error(ctx));
        return 1;
    }
    printf("status %d iterations %d translation %.6f %.6f %.6f\n", stats.status, stats.iters_total, pose[3],
           pose[7], pose[11]);
    FILE* f = fopen(argv[1], "wb");
    if (!f) {
        perror(argv[1]);
        return 1;
    }
    const int32_t dims[2] = {W, H};
    const double Kd[4] = {FX, FY, CX, CY};
    const int32_t tail[2] = {stats.status, stats.iters_total};
    int ok = fwrite(dims, sizeof(dims), 1, f) == 1 && fwrite(Kd, sizeof(Kd), 1, f) == 1 &&
             fwrite(imu_R, sizeof(imu_R), 1, f) == 1 && fwrite(init_pose, sizeof(init_pose), 1, f) == 1 &&
             fwrite(T_true, sizeof(T_true), 1, f) == 1 && fwrite(depth, sizeof(depth), 1, f) == 1 &&
             fwrite(mv, sizeof(mv), 1, f) == 1 && fwrite(mn, sizeof(mn), 1, f) == 1 &&
             fwrite(pose, sizeof(pose), 1, f) == 1 && fwrite(tail, sizeof(tail), 1, f) == 1;
    ok = fclose(f) == 0 && ok;
    (void)hipFree(d_depth);
    (void)hipFree(d_mv);
    (void)hipFree(d_mn);
    icp_ctx_destroy(ctx);
    return ok ? 0 : 1;
}
