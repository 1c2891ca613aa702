// gfx950 kernels of the ICP tracking hot path.
//
// Launch shapes: work-groups of 256 threads (four wave64).  Front-end kernels
// use one thread per output pixel with grid.y = problem.  The two pixel passes
// use one work-group per tile of `tile_px` consecutive pixels of one problem
// (four consecutive pixels per thread and round); a flat tile index spans every
// problem of the batch and `owner` maps it to its problem.  The per-problem
// steps (median band; FP64 reduction of the tile partials, solve and pose
// update) run in their own launches with one work-group per problem, so no
// kernel needs a device-scope fence or an arrival counter: data crosses
// work-groups only at kernel boundaries.  One ICP iteration of a whole batch
// is four launches and the pose never leaves the device.
#include <hip/hip_runtime.h>

#include "icp_device.hpp"
#include "icp_launch.hpp"

namespace icpk {

// ------------------------------------------------------------------ helpers

// ------------------------------------------------------------------ init

// The state of problem p at the start of a registration (one work-group).
__device__ __forceinline__ void init_block(const ProbDesc* __restrict__ probs, int p, int use_imu_seed,
                                           int32_t* need2) {
    const ProbDesc& P = probs[p];
    ProbState* st = P.st;
    if (need2 && p == 0 && threadIdx.x == 0) *need2 = 0;
    for (int b = threadIdx.x; b < ICP_HIST_BINS; b += ICP_WG) st->hist[0][b] = st->hist[1][b] = 0u;
    if (threadIdx.x == 0) {
        // Sec. 3: the live points are pre-oriented by the IMU rotation
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) st->R[3 * i + j] = use_imu_seed ? P.imu_R[3 * i + j] : P.init[4 * i + j];
            st->t[i] = P.init[4 * i + 3];
        }
        for (int k = 0; k < ICP_NMOM; ++k) st->M[k] = 0.0;
        for (int k = 0; k < 6; ++k) st->x[k] = 0.0;
        st->n_last = 0;
        st->N = 0;
        st->k_med = -1;
        st->k_lo = 0;
        st->k_hi = -1;
        st->pred_hi[0] = st->pred_hi[1] = -1;
        st->pred_hw[0] = st->pred_hw[1] = ICP_WIN / 2;
        st->fused_done = 0;
        st->ticket = 0;
        st->level_done = 0;
        st->settled = 0;
        st->last_kmed = -2;
        st->last_status = ICP_LEVEL_OK;
        for (int l = 0; l < ICP_MAX_LEVELS; ++l) {
            icp_level_stats& S = st->stats.level[l];
            S.iters_run = 0;
            S.status = ICP_LEVEL_OK;
            S.n_gated = 0;
            S.n_kept = 0;
            S.k_med = -1;
            S.pad = 0;
            S.rmse = 0.0;
        }
        st->stats.status = ICP_LEVEL_OK;
        st->stats.iters_total = 0;
    }
}

__global__ __launch_bounds__(ICP_WG) void k_init(const ProbDesc* __restrict__ probs, int use_imu_seed,
                                                 int32_t* need2) {
    init_block(probs, blockIdx.x, use_imu_seed, need2);
}

// ------------------------------------------------------------------ front end
// Depth pyramid: 2x2 mean of the four children when all four are valid.
// Level l and, with also_next, level l + 1 in one launch: one thread per
// 2 x 2 block of level-l pixels reads the 4 x 2 children of each of the
// block's rows (one 16-byte load when the rows allow it), writes the level-l
// depths and forms the level-(l+1) depth from the four it kept.  Only a block
// at the right or bottom edge of an odd-sized level is partial, and such a
// block has no level-(l+1) pixel.
__device__ __forceinline__ float depth_px(float a, float b, float c, float d) {
    if (!(depth_ok(a) && depth_ok(b) && depth_ok(c) && depth_ok(d))) return 0.0f;
    return (float)(((((double)a + (double)b) + (double)c) + (double)d) * 0.25);
}

// (bx: the work-group's index within the launch's range for this step)
__device__ __forceinline__ void depth_down_block(const ProbDesc* __restrict__ probs, int level, int also_next,
                                                 int bx) {
    const ProbDesc& P = probs[blockIdx.y];
    const LevelDesc& F = P.lv[level - 1];
    const LevelDesc& C = P.lv[level];
    const int qw = (C.W + 1) >> 1;  // blocks per row
    const int t = bx * ICP_WG + threadIdx.x;
    if (t >= qw * ((C.H + 1) >> 1)) return;
    const int vb = t / qw, u = 2 * (t % qw);
    const bool two = u + 1 < C.W;
    const int rows = 2 * vb + 1 < C.H ? 2 : 1;
    const ICP_GLOBAL float* D = gconst(F.D);
    const bool vec = two && (F.W & 3) == 0 && (reinterpret_cast<uintptr_t>(F.D) & 15) == 0;
    ICP_GLOBAL float* Do = gmut(C.Dw);
    float kept[4];
    for (int b = 0; b < rows; ++b) {
        const int v = 2 * vb + b;
        float r[2][4];
        for (int q = 0; q < 2; ++q) {
            const int base = (2 * v + q) * F.W + 2 * u;
            if (vec) {
                const vf4 x = *(const ICP_GLOBAL vf4*)(D + base);
                for (int c = 0; c < 4; ++c) r[q][c] = x[c];
            } else {
                for (int c = 0; c < 4; ++c) r[q][c] = c < (two ? 4 : 2) ? D[base + c] : 0.0f;
            }
        }
        for (int o = 0; o < (two ? 2 : 1); ++o) {
            const float z = depth_px(r[0][2 * o], r[0][2 * o + 1], r[1][2 * o], r[1][2 * o + 1]);
            Do[v * C.W + u + o] = z;
            kept[2 * b + o] = z;
        }
    }
    if (!also_next || !two || rows != 2) return;
    const LevelDesc& N = P.lv[level + 1];  // C.W >> 1 by C.H >> 1
    gmut(N.Dw)[vb * N.W + (u >> 1)] = depth_px(kept[0], kept[1], kept[2], kept[3]);
}

__global__ __launch_bounds__(ICP_WG) void k_depth_down(const ProbDesc* __restrict__ probs, int level,
                                                       int also_next) {
    depth_down_block(probs, level, also_next, blockIdx.x);
}

// Live vertex map and forward-difference normal map (flipped to face the
// camera).  A work-group covers FE_TX x FE_TY pixels; the back-projection
// quotients (u - cx)/fx and (v - cy)/fy of its columns and rows (one beyond,
// for the neighbours) are computed once into LDS, so every vertex, own or
// neighbour's, is z times the same two FP64 quotients.
#define FE_TX 64
#define FE_TY 16  // rows per work-group: each thread takes every fourth row

__device__ __forceinline__ void fe_quotients(double* sx, double* sy, int u0, int v0, double fx, double fy, double cx,
                                             double cy) {
    const int t = threadIdx.x;
    if (t <= FE_TX)
        sx[t] = ((double)(u0 + t) - cx) / fx;
    else if (t <= FE_TX + 1 + FE_TY)
        sy[t - FE_TX - 1] = ((double)(v0 + t - FE_TX - 1) - cy) / fy;
}

// Vertex p and normal n of pixel (u, v) = (u0 + du, v0 + dv); NaN when invalid.
__device__ __forceinline__ void live_px(const ICP_GLOBAL float* D, int W, int H, const double* sx, const double* sy,
                                        int du, int dv, int u, int v, float (&p)[3], float (&n)[3]) {
    const int i = v * W + u;
    const bool has_r = u + 1 < W, has_b = v + 1 < H;
    const float z = D[i];
    const float zr = has_r ? D[i + 1] : 0.0f;
    const float zb = has_b ? D[i + W] : 0.0f;
    live_from_depth(z, zr, zb, has_r, has_b, sx[du], sx[du + 1], sy[dv], sy[dv + 1], p, n);
}

// Bilateral smoothing of the level-0 depth into the level's workspace plane:
// over the (2r+1)^2 window in row-major order, valid neighbours within the
// range cut-off add ws * (1 - (dz/c)^2)^2 to the weight sum and that times z
// to the weighted sum (FP64); out = sum(w z) / sum(w); invalid pixels stay 0.
// The quotient dz/c is the correctly rounded one without a division: with
// y = RN(1/c) (from the host), q = RN(dz y) is within an ulp of dz/c, and one
// correction RN(q + RN(dz - c q) y) (the remainder exact by FMA) rounds
// correctly -- Markstein's theorem for division by a correctly rounded
// reciprocal.
// A work-group takes an FE_TX x FE_TY tile whose depth and R-pixel halo are
// staged in LDS (0, an invalid depth, outside the image).
constexpr int kBoxW = FE_TX + 2 * ICP_FILTER_MAX_R, kBoxH = FE_TY + 2 * ICP_FILTER_MAX_R;

template <int R>
__global__ __launch_bounds__(ICP_WG) void k_bilateral(const ProbDesc* __restrict__ probs, FrontEnd fe) {
    static_assert(R >= 1 && R <= ICP_FILTER_MAX_R, "filter radius");
    constexpr int HW = FE_TX + 2 * R, HH = FE_TY + 2 * R, N = 2 * R + 1;
    __shared__ double sz[kBoxH][kBoxW];  // (as FP64: no conversion per tap)
    const ProbDesc& P = probs[blockIdx.y];
    const LevelDesc& L = P.lv[0];
    const int tiles_x = (L.W + FE_TX - 1) / FE_TX;
    const int bx = blockIdx.x % tiles_x, by = blockIdx.x / tiles_x;
    const int u0 = bx * FE_TX, v0 = by * FE_TY;
    if (v0 >= L.H) return;  // uniform: grids cover the largest frame of the batch
    const ICP_GLOBAL float* D = gconst(P.depth_in);
    for (int t = threadIdx.x; t < HW * HH; t += ICP_WG) {
        const int ly = t / HW, lx = t - ly * HW;
        const int x = u0 - R + lx, y = v0 - R + ly;
        sz[ly][lx] = (x >= 0 && x < L.W && y >= 0 && y < L.H) ? (double)D[y * L.W + x] : 0.0;
    }
    __syncthreads();
    const int tx = threadIdx.x % FE_TX;
    const int u = u0 + tx;
    if (u >= L.W) return;
    ICP_GLOBAL float* out_plane = gmut(L.Dw);
    for (int ty = threadIdx.x / FE_TX; ty < FE_TY; ty += ICP_WG / FE_TX) {
        const int v = v0 + ty;
        if (v >= L.H) break;
        const double z = sz[ty + R][tx + R];
        float out = 0.0f;
        if (__builtin_isfinite(z) && z > 0.0) {
            double sw = 0.0, swz = 0.0;
#pragma unroll
            for (int dv = -R; dv <= R; ++dv)
#pragma unroll
                for (int du = -R; du <= R; ++du) {
                    const double zq = sz[ty + R + dv][tx + R + du];
                    if (!(__builtin_isfinite(zq) && zq > 0.0)) continue;
                    const double dz = zq - z;
                    if (!(fabs(dz) < fe.sigma_m)) continue;
                    const double q = dz * fe.inv_sigma_m;
                    const double t = __builtin_fma(__builtin_fma(-q, fe.sigma_m, dz), fe.inv_sigma_m, q);
                    const double a = 1.0 - t * t;
                    // the host's table is exp(-(du^2 + dv^2) / (2 s^2)): one entry per
                    // distinct (max(|du|, |dv|), min(|du|, |dv|)) holds every value, so the
                    // unrolled taps name only those (a few scalar registers, no spills)
                    const int ea = (du < 0 ? -du : du) > (dv < 0 ? -dv : dv) ? (du < 0 ? -du : du) : (dv < 0 ? -dv : dv);
                    const int eb = (du < 0 ? -du : du) > (dv < 0 ? -dv : dv) ? (dv < 0 ? -dv : dv) : (du < 0 ? -du : du);
                    const double w = fe.ws[(ea + R) * N + (eb + R)] * (a * a);
                    sw += w;
                    swz += w * zq;
                }
            out = (float)(swz / sw);
        }
        out_plane[v * L.W + u] = out;
    }
}

// Box-average 3D-gradient normals (normal_mode 1): for the (2r+1)^2 box around
// the pixel, the tangents are (mean over the right half - mean over the left
// half) and (lower - upper) of the valid vertices, each half sum a row-major
// FP64 sum of the FP32 vertices; n = normalise(h x g), flipped to face the
// camera; the pixel needs a valid vertex, a box inside the image and at least
// half of each half box valid.
//
// A work-group takes an FE_TX x FE_TY tile: the live vertices of the tile and
// an R-pixel halo are formed once into LDS (the same live_vertex of the same
// depth and quotients, NaN outside the image), then every pixel sums its box
// from LDS in row-major order.
// Correctly rounded reciprocals 1/k of the box counts k = 1 .. r (2r + 1)
// (constant evaluation rounds to nearest, as an IEEE division does), and s / k
// from them with Markstein's correction (as in the bilateral filter): the
// IEEE quotient without a division.
constexpr int kMaxBoxCount = ICP_FILTER_MAX_R * (2 * ICP_FILTER_MAX_R + 1);
struct RecipTable {
    double v[kMaxBoxCount + 1];
};
constexpr RecipTable make_recips() {
    RecipTable t{};
    for (int k = 1; k <= kMaxBoxCount; ++k) t.v[k] = 1.0 / (double)k;
    return t;
}
__constant__ RecipTable kBoxRecip = make_recips();

__device__ __forceinline__ double div_count(double s, int k) {
    const double y = kBoxRecip.v[k];
    const double q = s * y;
    return __builtin_fma(__builtin_fma(-q, (double)k, s), y, q);
}

template <int R>
__global__ __launch_bounds__(ICP_WG) void k_live_n_box(const ProbDesc* __restrict__ probs, int level) {
    static_assert(R >= 1 && R <= ICP_FILTER_MAX_R, "box radius");
    constexpr int HW = FE_TX + 2 * R, HH = FE_TY + 2 * R;
    __shared__ float sv[3][kBoxH][kBoxW];
    const LevelDesc& L = probs[blockIdx.y].lv[level];
    const int tiles_x = (L.W + FE_TX - 1) / FE_TX;
    const int bx = blockIdx.x % tiles_x, by = blockIdx.x / tiles_x;
    const int u0 = bx * FE_TX, v0 = by * FE_TY;
    if (v0 >= L.H) return;  // uniform: grids cover the largest level of the batch
    const ICP_GLOBAL float* D = gconst(L.D);
    const ICP_GLOBAL double* XQ = gconst(L.XQ);
    const ICP_GLOBAL double* YQ = gconst(L.YQ);
    const float qnan = __builtin_nanf("");
    for (int t = threadIdx.x; t < HW * HH; t += ICP_WG) {
        const int ly = t / HW, lx = t - ly * HW;
        const int x = u0 - R + lx, y = v0 - R + ly;
        float p[3] = {qnan, qnan, qnan};
        if (x >= 0 && x < L.W && y >= 0 && y < L.H) live_vertex(D[y * L.W + x], XQ[x], YQ[y], p);
        sv[0][ly][lx] = p[0];
        sv[1][ly][lx] = p[1];
        sv[2][ly][lx] = p[2];
    }
    __syncthreads();
    const int tx = threadIdx.x % FE_TX;
    const int u = u0 + tx;
    if (u >= L.W) return;
    ICP_GLOBAL float* LN = gmut(L.LN);
    constexpr int need = (R * (2 * R + 1) + 1) / 2;
    for (int ty = threadIdx.x / FE_TX; ty < FE_TY; ty += ICP_WG / FE_TX) {
        const int v = v0 + ty;
        if (v >= L.H) break;
        float n[3] = {qnan, qnan, qnan};
        const float p[3] = {sv[0][ty + R][tx + R], sv[1][ty + R][tx + R], sv[2][ty + R][tx + R]};
        if (u - R >= 0 && u + R < L.W && v - R >= 0 && v + R < L.H && fin(p[2])) {
            double sr[3] = {0, 0, 0}, sl[3] = {0, 0, 0}, sd[3] = {0, 0, 0}, su[3] = {0, 0, 0};
            int nr = 0, nl = 0, nd = 0, nu = 0;
#pragma unroll
            for (int dv = -R; dv <= R; ++dv)
#pragma unroll
                for (int du = -R; du <= R; ++du) {
                    const int yy = ty + R + dv, xx = tx + R + du;
                    const float q[3] = {sv[0][yy][xx], sv[1][yy][xx], sv[2][yy][xx]};
                    if (!fin(q[2])) continue;
                    for (int k = 0; k < 3; ++k) {
                        const double x = (double)q[k];
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
            if (nr >= need && nl >= need && nd >= need && nu >= need) {
                double h[3], g[3];
                for (int k = 0; k < 3; ++k) {
                    h[k] = div_count(sr[k], nr) - div_count(sl[k], nl);
                    g[k] = div_count(sd[k], nd) - div_count(su[k], nu);
                }
                const double c0 = h[1] * g[2] - h[2] * g[1];
                const double c1 = h[2] * g[0] - h[0] * g[2];
                const double c2 = h[0] * g[1] - h[1] * g[0];
                const double len2 = (c0 * c0 + c1 * c1) + c2 * c2;
                if (len2 > 0.0 && __builtin_isfinite(len2)) {
                    const double len = sqrt(len2), y = 1.0 / len;  // one division, then c / len per component
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
        const int i = v * L.W + u;
        LN[i] = n[0];
        LN[L.ps + i] = n[1];
        LN[2 * L.ps + i] = n[2];
    }
}

// Back-projection quotient tables of a level: XQ[u] = (u - cx)/fx for
// u = 0..W and YQ[v] = (v - cy)/fy for v = 0..H (the same FP64 divisions as
// fe_quotients), read by the pixel passes.
__global__ __launch_bounds__(ICP_WG) void k_quotients(const ProbDesc* __restrict__ probs, int level) {
    const LevelDesc& L = probs[blockIdx.y].lv[level];
    const int t = blockIdx.x * ICP_WG + threadIdx.x;
    if (t <= L.W)
        gmut(L.XQ)[t] = ((double)t - L.cx) / L.fx;
    else if (t <= L.W + 1 + L.H)
        gmut(L.YQ)[t - L.W - 1] = ((double)(t - L.W - 1) - L.cy) / L.fy;
}

__device__ __forceinline__ void live_vn_block(const ProbDesc* __restrict__ probs, int level, int with_vertex,
                                              int blk) {
    __shared__ double sx[FE_TX + 1], sy[FE_TY + 1];
    const LevelDesc& L = probs[blockIdx.y].lv[level];
    const int tiles_x = (L.W + FE_TX - 1) / FE_TX;
    const int bx = blk % tiles_x, by = blk / tiles_x;
    const int u0 = bx * FE_TX, v0 = by * FE_TY;
    if (v0 >= L.H) return;  // uniform: grids cover the largest level of the batch
    fe_quotients(sx, sy, u0, v0, L.fx, L.fy, L.cx, L.cy);
    __syncthreads();
    const int du = threadIdx.x % FE_TX;
    const int u = u0 + du;
    if (u >= L.W) return;
    const int S = L.ps;
    ICP_GLOBAL float* LV = gmut(L.LV);
    ICP_GLOBAL float* LN = gmut(L.LN);
    // every row's depth, right and lower neighbour are loaded before any row
    // is computed and stored (rows past the image read row v0 and are unused)
    constexpr int kStep = ICP_WG / FE_TX, kRows = FE_TY / kStep;
    const ICP_GLOBAL float* D = gconst(L.D);
    const int r0 = threadIdx.x / FE_TX;
    const bool has_r = u + 1 < L.W;
    float zc[kRows], zr[kRows], zb[kRows];
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
        const int v = v0 + r0 + q * kStep;
        const bool in = v < L.H;
        const int i = (in ? v : v0) * L.W + u;
        zc[q] = D[i];
        zr[q] = has_r ? D[i + 1] : 0.0f;
        zb[q] = in && v + 1 < L.H ? D[i + L.W] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
        const int dv = r0 + q * kStep;
        const int v = v0 + dv;
        if (v >= L.H) break;
        float p[3], n[3];
        live_from_depth(zc[q], zr[q], zb[q], has_r, v + 1 < L.H, sx[du], sx[du + 1], sy[dv], sy[dv + 1], p, n);
        const int i = v * L.W + u;
        if (with_vertex) {
            LV[i] = p[0];
            LV[S + i] = p[1];
            LV[2 * S + i] = p[2];
        }
        LN[i] = n[0];
        LN[S + i] = n[1];
        LN[2 * S + i] = n[2];
    }
}

__global__ __launch_bounds__(ICP_WG) void k_live_vn(const ProbDesc* __restrict__ probs, int level, int with_vertex) {
    live_vn_block(probs, level, with_vertex, blockIdx.x);
}

// The same vertex and normal maps of full-resolution depth images, written
// interleaved (H x W x 3): the model maps of frame-to-frame tracking.
__global__ __launch_bounds__(ICP_WG) void k_depth_to_maps(const MapsDesc* __restrict__ jobs) {
    __shared__ double sx[FE_TX + 1], sy[FE_TY + 1];
    const MapsDesc& J = jobs[blockIdx.y];
    const int tiles_x = (J.W + FE_TX - 1) / FE_TX;
    const int bx = blockIdx.x % tiles_x, by = blockIdx.x / tiles_x;
    const int u0 = bx * FE_TX, v0 = by * FE_TY;
    if (v0 >= J.H) return;
    fe_quotients(sx, sy, u0, v0, J.fx, J.fy, J.cx, J.cy);
    __syncthreads();
    const int du = threadIdx.x % FE_TX;
    const int u = u0 + du;
    if (u >= J.W) return;
    ICP_GLOBAL float* MV = gmut(J.mv);
    ICP_GLOBAL float* MN = gmut(J.mn);
    for (int dv = threadIdx.x / FE_TX; dv < FE_TY; dv += ICP_WG / FE_TX) {
        const int v = v0 + dv;
        if (v >= J.H) break;
        float p[3], n[3];
        live_px(gconst(J.depth), J.W, J.H, sx, sy, du, dv, u, v, p, n);
        const int i = v * J.W + u;
        for (int k = 0; k < 3; ++k) {
            MV[3 * i + k] = p[k];
            MN[3 * i + k] = n[k];
        }
    }
}

// Model level l from l-1 (interleaved maps): vertex = mean of the four
// children, normal = their normalised sum, valid iff all four children have
// six finite values; invalid pixels are NaN in all six.
__device__ __forceinline__ void model_px(const float (&cv)[4][3], const float (&cn)[4][3], float (&vo)[3],
                                         float (&no)[3]) {
    const float qnan = __builtin_nanf("");
    bool ok = true;
    for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 3; ++k) ok = ok && fin(cv[j][k]) && fin(cn[j][k]);
    for (int k = 0; k < 3; ++k) vo[k] = no[k] = qnan;
    if (!ok) return;
    double s[3];
    for (int k = 0; k < 3; ++k) {
        const double m = (((double)cv[0][k] + (double)cv[1][k]) + (double)cv[2][k]) + (double)cv[3][k];
        s[k] = (((double)cn[0][k] + (double)cn[1][k]) + (double)cn[2][k]) + (double)cn[3][k];
        vo[k] = (float)(m * 0.25);
    }
    const double len2 = (s[0] * s[0] + s[1] * s[1]) + s[2] * s[2];
    if (len2 > 0.0) {
        const double len = sqrt(len2), y = 1.0 / len;  // one division, then s / len per component
        for (int k = 0; k < 3; ++k) no[k] = (float)div_rn(s[k], len, y);
    } else {
        vo[0] = vo[1] = vo[2] = qnan;
    }
}

// Model level l from l - 1 and, with also_next, level l + 1 in the same
// launch: one thread per level-l pixel, the four lanes of a quad holding the
// pixels of one 2 x 2 block.  Each thread reads its four children (two rows of
// six consecutive floats per map), writes its level-l pixel and keeps it; the
// quad's first lane gathers the block's four pixels from its neighbours (DPP
// broadcasts within the quad) and forms the level-(l+1) pixel, so level l is
// never read back.  A block is partial only at the right or bottom edge of an
// odd-sized level, and then it has no level-(l+1) pixel (each level halves
// the size, rounding down).
template <int K>
__device__ __forceinline__ float quad_bcast(float x) {
    // quad_perm(K, K, K, K): every lane of a quad takes lane K's value
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x55 * K, 0xF, 0xF, false));
}

__device__ __forceinline__ void model_down_block(const ProbDesc* __restrict__ probs, int level, int also_next,
                                                 int bx) {
    const ProbDesc& P = probs[blockIdx.y];
    const LevelDesc& F = P.lv[level - 1];
    const LevelDesc& C = P.lv[level];
    const int qw = (C.W + 1) >> 1, qh = (C.H + 1) >> 1;  // blocks per row, block rows
    const int t = bx * ICP_WG + threadIdx.x;
    const int blk = t >> 2, q = t & 3;
    if (blk >= qw * qh) return;  // (whole quads)
    const int bv = blk / qw, bu = blk - bv * qw;
    const int u = 2 * bu + (q & 1), v = 2 * bv + (q >> 1);
    const bool inside = u < C.W && v < C.H;
    const ICP_GLOBAL float* MV = gconst(F.MV);
    const ICP_GLOBAL float* MN = gconst(F.MN);
    // children (2u, 2v), (2u+1, 2v), (2u, 2v+1), (2u+1, 2v+1), row-major
    float cv[4][3], cn[4][3];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int base = inside ? 3 * ((2 * v + r) * F.W + 2 * u) : 0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            cv[2 * r + k / 3][k % 3] = MV[base + k];
            cn[2 * r + k / 3][k % 3] = MN[base + k];
        }
    }
    float vo[3], no[3];
    model_px(cv, cn, vo, no);
    if (inside) {
        ICP_GLOBAL float* MVo = gmut(C.MVw);
        ICP_GLOBAL float* MNo = gmut(C.MNw);
        const int i = v * C.W + u;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            MVo[3 * i + k] = vo[k];
            MNo[3 * i + k] = no[k];
        }
    }
    if (!also_next) return;  // (uniform)
    // every lane of the quad takes part in the broadcasts
    float kv[4][3], kn[4][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        kv[0][k] = quad_bcast<0>(vo[k]);
        kv[1][k] = quad_bcast<1>(vo[k]);
        kv[2][k] = quad_bcast<2>(vo[k]);
        kv[3][k] = quad_bcast<3>(vo[k]);
        kn[0][k] = quad_bcast<0>(no[k]);
        kn[1][k] = quad_bcast<1>(no[k]);
        kn[2][k] = quad_bcast<2>(no[k]);
        kn[3][k] = quad_bcast<3>(no[k]);
    }
    if (q != 0 || 2 * bu + 1 >= C.W || 2 * bv + 1 >= C.H) return;
    // a whole block: level l+1 (C.W >> 1 by C.H >> 1) has its pixel (bu, bv)
    const LevelDesc& N = P.lv[level + 1];
    model_px(kv, kn, vo, no);
    const int i = bv * N.W + bu;
    ICP_GLOBAL float* NVo = gmut(N.MVw);
    ICP_GLOBAL float* NNo = gmut(N.MNw);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        NVo[3 * i + k] = vo[k];
        NNo[3 * i + k] = no[k];
    }
}

__global__ __launch_bounds__(ICP_WG) void k_model_down(const ProbDesc* __restrict__ probs, int level,
                                                       int also_next) {
    model_down_block(probs, level, also_next, blockIdx.x);
}

// The raw-depth front end of two or three levels in two launches.  The model
// pyramid, the depth pyramid, level 0's live maps and the problem's initial
// state depend only on the inputs, so one launch does all four, each on its
// own range of the grid's work-groups (the model pyramid's memory traffic then
// overlaps the normals' FP64 arithmetic); the coarser levels' live maps, which
// need the depth pyramid, follow in a second launch.
__global__ __launch_bounds__(ICP_WG) void k_front_inputs(const ProbDesc* __restrict__ probs, int nb_model,
                                                         int nb_depth, int nb_vn, int also_next, int with_vertex,
                                                         int use_imu_seed, int32_t* need2) {
    const int b = blockIdx.x;  // (each range is whole work-groups: the branches are uniform)
    if (b < nb_model)
        model_down_block(probs, 1, also_next, b);
    else if (b < nb_model + nb_depth)
        depth_down_block(probs, 1, also_next, b - nb_model);
    else if (b < nb_model + nb_depth + nb_vn)
        live_vn_block(probs, 0, with_vertex, b - nb_model - nb_depth);
    else
        init_block(probs, blockIdx.y, use_imu_seed, need2);
}

__global__ __launch_bounds__(ICP_WG) void k_front_coarse(const ProbDesc* __restrict__ probs, int nb_level1,
                                                         int with_vertex) {
    const int b = blockIdx.x;
    if (b < nb_level1)
        live_vn_block(probs, 1, with_vertex, b);
    else
        live_vn_block(probs, 2, with_vertex, b - nb_level1);
}

// Centroid of the valid live vertices of one level: the centring point of the
// split-precision reduction.  Each tile of the level sums its valid vertices
// (x = z (u - cx)/fx, y likewise, rounded to FP32 as the vertex map stores
// them) in FP64 into its pass-2 partial slot (free during the front end); one
// work-group per problem then adds the tiles in tile order.  Deterministic.
__global__ __launch_bounds__(ICP_WG) void k_centroid_tiles(const ProbDesc* __restrict__ probs,
                                                           const int* __restrict__ owner, int level) {
    __shared__ double sh[ICP_WG][4];
    const int g = blockIdx.x;
    const ProbDesc& P = probs[owner[g]];
    const LevelDesc& L = P.lv[level];
    const int tile = g - L.tile_base;
    const int tid = threadIdx.x;
    const int base = tile * L.tile_px, end = min(base + L.tile_px, L.npx);
    double sx = 0.0, sy = 0.0, sz = 0.0, n = 0.0;
    const ICP_GLOBAL float* D = gconst(L.D);
    const Lvl Lv = load_level(L);
    // four of the thread's pixels per step, their depths loaded together; the
    // vertices use the pixel passes' quotients (the table values), and the
    // sums take the pixels in the same order as one at a time
    constexpr int kStep = 4;
    for (int i0 = base + tid; i0 < end; i0 += kStep * ICP_WG) {
        float z[kStep];
#pragma unroll
        for (int k = 0; k < kStep; ++k) {
            const int i = i0 + k * ICP_WG;
            z[k] = D[i < end ? i : i0];
        }
#pragma unroll
        for (int k = 0; k < kStep; ++k) {
            const int i = i0 + k * ICP_WG;
            if (i < end && depth_ok(z[k])) {
                int u, v;
                pixel_uv(Lv, i, u, v);
                sx += (double)(float)((double)z[k] * bp_quot(u, Lv.cx, Lv.fx, Lv.rfx));
                sy += (double)(float)((double)z[k] * bp_quot(v, Lv.cy, Lv.fy, Lv.rfy));
                sz += (double)z[k];
                n += 1.0;
            }
        }
    }
    sh[tid][0] = sx;
    sh[tid][1] = sy;
    sh[tid][2] = sz;
    sh[tid][3] = n;
    __syncthreads();
    for (int w = ICP_WG / 2; w > 0; w >>= 1) {
        if (tid < w)
            for (int k = 0; k < 4; ++k) sh[tid][k] += sh[tid + w][k];
        __syncthreads();
    }
    if (tid < 4) reinterpret_cast<double*>(L.part + (size_t)tile * ICP_PART_STRIDE)[tid] = sh[0][tid];
}

__global__ __launch_bounds__(64) void k_centroid_sum(const ProbDesc* __restrict__ probs) {
    __shared__ double sh[64];
    const ProbDesc& P = probs[blockIdx.x];
    const int level = blockIdx.y;
    const LevelDesc& L = P.lv[level];
    const int tid = threadIdx.x, k = tid & 3, c = tid >> 2;  // component k, chunk c of 16
    const int per = (L.n_tiles + 15) / 16, t0 = c * per, t1 = min(t0 + per, L.n_tiles);
    double s = 0.0;
    for (int t = t0; t < t1; ++t) s += reinterpret_cast<const double*>(L.part + (size_t)t * ICP_PART_STRIDE)[k];
    sh[tid] = s;
    __syncthreads();
    if (tid < 4) {
        double tot = 0.0;
        for (int q = 0; q < 16; ++q) tot += sh[4 * q + tid];
        sh[tid] = tot;  // chunk 0's slot: read again by thread 0 below after the barrier
    }
    __syncthreads();
    if (tid == 0) {
        ProbState* st = P.st;
        for (int a = 0; a < 3; ++a) st->cen[level][a] = sh[3] > 0.0 ? sh[a] / sh[3] : 0.0;
    }
}

// ------------------------------------------------------------------ pass 1
// Association, gates and the distance histogram (Sec. 3.2).  In single-pass
// mode the rows are also reduced: rows whose bin lies below a window around
// the band edge predicted from the previous iteration go to per-thread
// accumulators, rows inside the window to per-bin LDS sums, so that once the
// band is known the kept rows' moments are a prefix of the tile partials.

// The window of an iteration: bins [h0, h0 + w), 2 hw of them around the
// predicted edge.  The first iteration of a level, whose prediction comes
// from the coarser level, takes the full ICP_WIN bins; later iterations take
// the half-width the band kernel derived from how far the edge last moved.
// h0 = -1: no prediction, no window.
struct Win {
    int h0, w;
};

__device__ __forceinline__ Win band_window(int pred_hi, int pred_hw, int iter) {
    if (pred_hi < 0) return Win{-1, 0};
    const int hw = iter == 0 ? ICP_WIN / 2 : pred_hw;
    const int h0 = pred_hi - hw, hmax = ICP_HIST_BINS - 2 * hw;
    return Win{h0 < 0 ? 0 : (h0 > hmax ? hmax : h0), 2 * hw};
}

// Half-width of the next iteration's window: twice the edge's last move plus
// four bins, at least six and at most ICP_WIN / 2 (the full window when the
// move is unknown: the first iteration of a level, or no prediction).
__device__ __forceinline__ int next_half_width(int k_hi, int pred_hi, int iter) {
    if (iter == 0 || pred_hi < 0) return ICP_WIN / 2;
    const int hw = 2 * abs(k_hi - pred_hi) + 4;
    return hw < 6 ? 6 : (hw > ICP_WIN / 2 ? ICP_WIN / 2 : hw);
}

// Rows of the histogram whose CDF is `cdf` that a window of half-width hw
// around k_hi (placed as band_window places it) would hold.
__device__ __forceinline__ uint32_t window_rows(const uint32_t* cdf, int k_hi, int hw) {
    int h0 = k_hi - hw;
    const int hmax = ICP_HIST_BINS - 2 * hw;
    h0 = h0 < 0 ? 0 : (h0 > hmax ? hmax : h0);
    return cdf[h0 + 2 * hw - 1] - (h0 > 0 ? cdf[h0 - 1] : 0u);
}

// Rows inside the window take the slow per-bin path (staged through LDS, one
// moment per lane), at several times the cost of a pixel's whole pass; a
// missed window costs one more pass over the problem's pixels.  So where the
// pairs are dense around the edge (smoothed depth: most pixels are gated in)
// the window is narrowed, down to six bins either side, until this
// iteration's histogram puts at most 1/ICP_WIN_ROW_CAP of the level's pixels
// in it.
#ifndef ICP_WIN_ROW_CAP
#define ICP_WIN_ROW_CAP 40
#endif
__device__ __forceinline__ int capped_half_width(const uint32_t* cdf, int k_hi, int hw, int npx) {
    const uint32_t cap = (uint32_t)(npx / ICP_WIN_ROW_CAP);
    while (hw > 6 && window_rows(cdf, k_hi, hw) > cap) --hw;
    return hw;
}

// Sum the 28 accumulators and the count over the work-group into `out`
// (29 floats); every thread calls it.
__device__ __forceinline__ void block_reduce_row(float (&acc)[ICP_NMOM], float cnt, float (*sh_red)[ICP_PART_STRIDE],
                                                 ICP_GLOBAL float* out) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int k = 0; k < ICP_NMOM; ++k) acc[k] = wave_sum(acc[k]);
    cnt = wave_sum(cnt);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < ICP_NMOM; ++k) sh_red[wave][k] = acc[k];
        sh_red[wave][ICP_NMOM] = cnt;
    }
    __syncthreads();
    if (tid <= ICP_NMOM) out[tid] = (sh_red[0][tid] + sh_red[1][tid]) + (sh_red[2][tid] + sh_red[3][tid]);
}

#define ICP_STAGE 8  // window rows a wave stages at a time

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The (a, b) entry of the 7x7 upper triangle that moment m holds (row-major).
__device__ __forceinline__ void moment_pair(int m, int& a, int& b) {
    a = 0;
    int rem = m;
    while (rem >= 7 - a) {
        rem -= 7 - a;
        ++a;
    }
    b = a + rem;
}

// Add the window rows of this wave's lanes (those with `inwin`) to the wave's
// own window sums, in lane order: the rows r = [a | b] are staged in LDS in
// lane order, then lane m < 28 adds product m of each staged row in turn (lane
// 28 the count), so the sums do not depend on timing.
__device__ __forceinline__ void window_add(bool inwin, int bin_off, const float (&p)[3], const float (&d)[3],
                                           const float (&n)[3], float (*win)[ICP_NMOM + 1], float (*stage)[8]) {
    const int lane = threadIdx.x & 63;
    uint64_t m = __ballot(inwin);
    if (!m) return;
    int ma, mb;
    moment_pair(min(lane, ICP_NMOM - 1), ma, mb);
    while (m) {
        // the lowest ICP_STAGE pending lanes
        uint64_t c = m, keep = 0;
        for (int q = 0; q < ICP_STAGE && c; ++q) {
            const uint64_t low = c & (~c + 1);
            keep |= low;
            c &= c - 1;
        }
        if ((keep >> lane) & 1ull) {
            const int slot = __popcll(keep & ((1ull << lane) - 1ull));
            float r[7];
            make_row(p, d, n, r);
#pragma unroll
            for (int t = 0; t < 7; ++t) stage[slot][t] = r[t];
            stage[slot][7] = __int_as_float(bin_off);
        }
        wave_sync();
        const int nst = __popcll(keep);
        if (lane <= ICP_NMOM) {
            for (int j = 0; j < nst; ++j) {
                const int b = __float_as_int(stage[j][7]);
                win[b][lane] += lane < ICP_NMOM ? stage[j][ma] * stage[j][mb] : 1.0f;
            }
        }
        wave_sync();
        m &= ~keep;
    }
}

// Split-precision reduction (reduce_mode 1): a row r = [(p' - c) x n, n, b, 1]
// (centred on the pose-moved live centroid c), scaled per column by a power of
// two, is split into FP16 hi = fp16(r) and lo = fp16(r - hi); X = [hi | lo]
// (rows x 16) goes through v_mfma_f32_16x16x32_f16 as X^T X with FP32
// accumulation, whose four 8 x 8 blocks sum to the rows' Gram matrix.
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr float kScaleRot = 8.0f;     // |(p' - c) x n| stays well inside FP16 range
constexpr float kScaleB = 1024.0f;    // |b| < dist_max <= 0.125 m; lifts b's lo part out of FP16 subnormals

// The 8 split-precision columns of a kept row (zeros for a row not kept).
__device__ __forceinline__ void split_row(bool keep, const float (&pc)[3], const float (&d)[3], const float (&n)[3],
                                          _Float16 (&hi)[8], _Float16 (&lo)[8]) {
    float r[7];
    make_row(pc, d, n, r);
    const float v[8] = {r[0] * kScaleRot, r[1] * kScaleRot, r[2] * kScaleRot, r[3], r[4], r[5], r[6] * kScaleB, 1.0f};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const _Float16 h = (_Float16)v[c];
        hi[c] = keep ? h : (_Float16)0.0f;
        lo[c] = keep ? (_Float16)(v[c] - (float)h) : (_Float16)0.0f;
    }
}

// Add the kept rows of this round (one per lane) to the wave's MFMA
// accumulator: each half of the wave stages its 32 rows column-major in the
// wave's 16 x 32 FP16 area (zeros where a lane keeps nothing), then one
// 16x16x32 MFMA takes X^T X of them.  Halves without a kept row are skipped
// (uniform).
__device__ __forceinline__ void mfma_rows(bool keep, const float (&pc)[3], const float (&d)[3], const float (&n)[3],
                                          _Float16 (*sx)[32], f4v& acc) {
    const uint64_t m = __ballot(keep);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    _Float16 hi[8], lo[8];
    split_row(keep, pc, d, n, hi, lo);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (!((m >> (32 * h)) & 0xffffffffull)) continue;
        if ((lane >> 5) == h) {
            const int row = lane & 31;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                sx[c][row] = hi[c];
                sx[8 + c][row] = lo[c];
            }
        }
        wave_sync();
        const h8v a = *(const h8v*)&sx[lane & 15][8 * (lane >> 4)];
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, a, acc, 0, 0, 0);
        wave_sync();
    }
}

// The 28 moments (and the count) of a wave's MFMA accumulator, unscaled, in
// lane 0 (zeros elsewhere): D[4 (l / 16) + t][l % 16] is written to the wave's
// staging area (16 x 16 floats, exactly its size), then the four 8 x 8 blocks
// hi'hi + hi'lo + lo'hi + lo'lo are added.
__device__ __forceinline__ void mfma_moments(const f4v& acc, _Float16 (*sx)[32], float (&mom)[ICP_NMOM], float& cnt) {
    const int lane = threadIdx.x & 63;
    float* sd = reinterpret_cast<float*>(&sx[0][0]);
    wave_sync();
#pragma unroll
    for (int t = 0; t < 4; ++t) sd[(4 * (lane >> 4) + t) * 16 + (lane & 15)] = acc[t];
    wave_sync();
    int k = 0;
    for (int a = 0; a < 7; ++a)
        for (int b = a; b < 7; ++b) {
            const float g = (sd[a * 16 + b] + sd[a * 16 + 8 + b]) + (sd[(8 + a) * 16 + b] + sd[(8 + a) * 16 + 8 + b]);
            const float sa = a < 3 ? kScaleRot : (a == 6 ? kScaleB : 1.0f);
            const float sb = b < 3 ? kScaleRot : (b == 6 ? kScaleB : 1.0f);
            mom[k++] = lane == 0 ? g / (sa * sb) : 0.0f;
        }
    cnt = lane == 0 ? (sd[7 * 16 + 7] + sd[7 * 16 + 15]) + (sd[15 * 16 + 7] + sd[15 * 16 + 15]) : 0.0f;
}

#ifndef ICP_PASS1_WAVES
#define ICP_PASS1_WAVES 5
#endif
template <bool kDebug, bool kFused, bool kSplit>
__global__ __launch_bounds__(ICP_WG) __attribute__((amdgpu_waves_per_eu(ICP_PASS1_WAVES))) void k_pass1(const ProbDesc* __restrict__ probs, const int* __restrict__ owner,
                                                  IterCtl ctl, KParams kp, uint8_t* __restrict__ dbg_code,
                                                  int32_t* __restrict__ dbg_bin) {
    __shared__ __attribute__((aligned(16))) uint32_t sh_hist[ICP_HIST_BINS];
    __shared__ float sh_win[kFused ? ICP_WAVES : 1][kFused ? ICP_WIN : 1][ICP_NMOM + 1];
    __shared__ float sh_stage[kFused ? ICP_WAVES : 1][kFused ? ICP_STAGE : 1][8];
    __shared__ float sh_red[ICP_WAVES][ICP_PART_STRIDE];
    __shared__ _Float16 sh_x[kSplit ? ICP_WAVES : 1][16][32];  // split precision: a half-wave's rows, column-major
    const int g = blockIdx.x;
    const ProbDesc& P = probs[owner[g]];
    const LevelDesc& L = P.lv[ctl.level];
    const ProbState* st = P.st;
    const int tid = threadIdx.x;
    const int tile = g - L.tile_base;
    const Lvl Lv = load_level(L);
    const int base = tile * L.tile_px;
    const int end = min(base + L.tile_px, L.npx);
    // Every lane of the block runs the same rounds (the queue and window
    // steps work across the wave); a lane past the tile's end loads the
    // round's first pixels and treats its own as invalid.
    constexpr int kRound = ICP_WG * ICP_PASS1_PX;  // pixels per round
    auto ld_index = [&](int r) {
        const int i = r + ICP_PASS1_PX * tid;
        return i < end ? i : r;
    };
    // The first round's live data depend on the level alone: they are loaded
    // before the problem's state, so that their latency overlaps the state's
    // and the pose's (a work-group of a coarse level runs only a few rounds).
    // (The state is read through a global pointer, as scalar loads, so that
    // waiting for it does not also wait for the live loads.)
    LiveIn<ICP_PASS1_PX> cur;
    if (base < end) cur = load_live<ICP_PASS1_PX>(Lv, ld_index(base));
    const ICP_GLOBAL ProbState* gst = gconst(st);
    if (gst->level_done) return;  // uniform: the level has ended for this problem
    const Win win = kFused ? band_window(gst->pred_hi[ctl.par], gst->pred_hw[ctl.par], ctl.iter) : Win{-1, 0};
    const int h0 = win.h0;
    const Pose T = load_pose(st);
    static_assert(ICP_HIST_BINS == 4 * ICP_WG, "four histogram bins per thread");
    typedef uint32_t u4v __attribute__((ext_vector_type(4)));
    reinterpret_cast<u4v*>(sh_hist)[tid] = u4v{0u, 0u, 0u, 0u};
    if (kFused && h0 >= 0)
        // only the window's w bins of each wave's sums are cleared (and later read)
        for (int wv = 0; wv < ICP_WAVES; ++wv)
            for (int b = tid; b < win.w * (ICP_NMOM + 1); b += ICP_WG) (&sh_win[wv][0][0])[b] = 0.0f;
    __syncthreads();
    const int wave = tid >> 6;
    float acc[ICP_NMOM];
#pragma unroll
    for (int k = 0; k < ICP_NMOM; ++k) acc[k] = 0.0f;
    float cnt = 0.0f;
    f4v macc = {0.0f, 0.0f, 0.0f, 0.0f};  // split precision: the wave's X^T X
    {
        // split precision: rows are centred on the level's live centroid moved
        // by the pose of this iteration (the centring point of the two-pass
        // variant, formed with the same FP64 expression, then rounded)
        float cc[3] = {0.0f, 0.0f, 0.0f};
        if (kSplit) {
            const ICP_GLOBAL double* cen = gconst(st->cen[ctl.level]);
            const double e0 = uniform(cen[0]), e1 = uniform(cen[1]), e2 = uniform(cen[2]);
#pragma unroll
            for (int i = 0; i < 3; ++i)
                cc[i] = (float)(((T.r[3 * i] * e0 + T.r[3 * i + 1] * e1) + T.r[3 * i + 2] * e2) + T.t[i]);
        }
        // Software pipeline over the rounds: while a round's pixels are
        // decided, the next round's model gathers and the live planes of the
        // round after it are in flight.  Past the tile's end every lane's
        // projection is invalid (a gather of model pixel 0) and the live loads
        // repeat the last round's pixels (no branch: the waits stay exact).
        auto next_r = [&](int r) { return r + kRound < end ? r + kRound : r; };
        Proj<ICP_PASS1_PX> pa = assoc_project<ICP_PASS1_PX>(Lv, base + ICP_PASS1_PX * tid, end, cur, T);
        Gath<ICP_PASS1_PX> ga = assoc_gather<ICP_PASS1_PX>(Lv, base + ICP_PASS1_PX * tid, pa);
        LiveIn<ICP_PASS1_PX> nxt = load_live<ICP_PASS1_PX>(Lv, ld_index(next_r(base)));
        for (int r = base; r < end; r += kRound) {
            const int i = r + ICP_PASS1_PX * tid;
            const LiveIn<ICP_PASS1_PX> nn = load_live<ICP_PASS1_PX>(Lv, ld_index(next_r(next_r(r))));
            const Proj<ICP_PASS1_PX> pb = assoc_project<ICP_PASS1_PX>(Lv, r + kRound + ICP_PASS1_PX * tid, end, nxt, T);
            const Gath<ICP_PASS1_PX> gb = assoc_gather<ICP_PASS1_PX>(Lv, r + kRound + ICP_PASS1_PX * tid, pb);
            assoc_decide<ICP_PASS1_PX>(pa, ga, T, kp.d2max, kp.cos_max, [&](int k, const PixelOut& q) {
                if (kDebug && i + k < end) {
                    if (dbg_code) dbg_code[i + k] = (uint8_t)q.code;
                    if (dbg_bin) dbg_bin[i + k] = q.bin;
                }
                const bool gated = q.code == kGated;
                if (gated) atomicAdd(&sh_hist[q.bin], 1u);
                if (kFused && h0 >= 0) {
                    const bool inwin = gated && q.bin >= h0 && q.bin < h0 + win.w;
                    if (kSplit) {
                        const float pc[3] = {q.p[0] - cc[0], q.p[1] - cc[1], q.p[2] - cc[2]};
                        mfma_rows(gated && q.bin < h0, pc, q.d, q.n, sh_x[wave], macc);
                        window_add(inwin, q.bin - h0, pc, q.d, q.n, sh_win[wave], sh_stage[wave]);
                    } else {
                        if (gated && q.bin < h0) {
                            accumulate_row(q.p, q.d, q.n, acc);
                            cnt += 1.0f;
                        }
                        window_add(inwin, q.bin - h0, q.p, q.d, q.n, sh_win[wave], sh_stage[wave]);
                    }
                }
            });
            pa = pb;
            ga = gb;
            nxt = nn;
        }
    }
    __syncthreads();
    // (Partials are stored and the histogram added through global pointers:
    // a generic-pointer store or atomic also counts as an LDS access, so each
    // later LDS wait would wait for it to reach memory.)
    if (kFused && h0 >= 0) {
        ICP_GLOBAL float* part = gmut(L.part1) + (size_t)tile * ICP_WIN_SLOTS * ICP_PART_STRIDE;
        if (kSplit) mfma_moments(macc, sh_x[wave], acc, cnt);
        block_reduce_row(acc, cnt, sh_red, part);
        // slot b+1 holds the prefix sum over window bins 0..b (b < w), so the
        // band kernel needs two slots per tile whatever the band edge.  The 48 bins
        // are scanned as 8 chunks of 6 by 8 x 29 threads: each sums its chunk
        // (waves, then bins in order), the chunk totals go through LDS, and
        // each thread adds the totals of the chunks before its own.
        constexpr int kChunks = 8, kPer = ICP_WIN / kChunks;
        static_assert(kChunks * kPer == ICP_WIN && kChunks * (ICP_NMOM + 1) <= ICP_WAVES * ICP_STAGE * 8,
                      "window scan layout");
        float* sh_tot = &sh_stage[0][0][0];  // reused: [chunk][moment]
        __syncthreads();
        const int cj = tid / (ICP_NMOM + 1), mj = tid - cj * (ICP_NMOM + 1);
        float pre[kPer];
        if (cj < kChunks) {
            float run = 0.0f;
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int b = cj * kPer + q;
                if (b < win.w) run += (sh_win[0][b][mj] + sh_win[1][b][mj]) + (sh_win[2][b][mj] + sh_win[3][b][mj]);
                pre[q] = run;
            }
            sh_tot[cj * (ICP_NMOM + 1) + mj] = run;
        }
        __syncthreads();
        if (cj < kChunks) {
            float off = 0.0f;
            for (int c2 = 0; c2 < cj; ++c2) off += sh_tot[c2 * (ICP_NMOM + 1) + mj];
#pragma unroll
            for (int q = 0; q < kPer; ++q)
                if (cj * kPer + q < win.w) part[(cj * kPer + q + 1) * ICP_PART_STRIDE + mj] = off + pre[q];
        }
    }
    // the tile's histogram, last: nothing after it waits for the adds
    ICP_GLOBAL unsigned int* hist = gmut(P.st->hist[ctl.par]);
    // (lane-consecutive bins: each atomic instruction of a wave covers 256
    // contiguous bytes; four bins per thread would spread it over four times
    // as many cache lines, which a one-problem registration's 300 work-groups,
    // all adding into one histogram, pay in latency)
    for (int b = tid; b < ICP_HIST_BINS; b += ICP_WG) {
        const uint32_t c = sh_hist[b];
        if (c) __hip_atomic_fetch_add(hist + b, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------------ epilogues

// After a level's last scheduled iteration: the next level starts afresh.
__device__ __forceinline__ void level_reset(ProbState* st) {
    st->level_done = 0;
    st->settled = 0;
    st->last_kmed = -2;
}

// The state a solve starts from.  Loaded before the work that precedes the
// solve (with the kernel's other loads), so that the solve itself waits for
// no memory.
struct EpiIn {
    double R[9], t[3];
    int32_t done, last_kmed, settled, iters_total, first_status;
};

__device__ __forceinline__ EpiIn load_epi(const ProbState* st_in) {
    const ICP_GLOBAL ProbState* st = gconst(st_in);
    EpiIn e;
#pragma unroll
    for (int k = 0; k < 9; ++k) e.R[k] = st->R[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) e.t[k] = st->t[k];
    e.done = st->level_done;
    e.last_kmed = st->last_kmed;
    e.settled = st->settled;
    e.iters_total = st->stats.iters_total;
    e.first_status = st->stats.status;
    return e;
}

// Regularised solve (Eq. (5)), pose update and per-level bookkeeping of one
// problem; thread 0 only.  It starts from e (load_epi) and the iteration's
// gated count N and median bin k_med, and stores every field it writes
// through a global pointer, after all of its arithmetic.
__device__ void solve_epilogue(ProbState* st_in, const EpiIn& e, uint32_t N, int32_t k_med, const double* M,
                               int64_t n, const IterCtl& ctl, const KParams& kp, const double* imu_R) {
    ICP_GLOBAL ProbState* st = gmut(st_in);
    const int32_t done = e.done;
    double R[9], t[3];
    for (int k = 0; k < 9; ++k) R[k] = e.R[k];
    for (int k = 0; k < 3; ++k) t[k] = e.t[k];
    const int32_t last_kmed = e.last_kmed, settled = e.settled;
    const int32_t iters_total = e.iters_total, first_status = e.first_status;
    if (done) return;
    if (ctl.no_update) {
        for (int k = 0; k < ICP_NMOM; ++k) st->M[k] = M[k];
        st->n_last = n;
        return;
    }
    double x[6];
    const int status = solve_regularised(M, n, kp, R, imu_R, x);
    if (status == ICP_LEVEL_OK) compose_exp(x, R, t);
    int32_t level_done = 0, new_settled = settled, new_last = last_kmed, total_status = first_status;
    if (status != ICP_LEVEL_OK) {
        level_done = 1;
        if (first_status == ICP_LEVEL_OK) total_status = status;
    } else if (kp.converge_window > 0) {
        // Sec. 3.4: a level has converged once its median bin stays put
        new_settled = (k_med == last_kmed) ? settled + 1 : 1;
        new_last = k_med;
        if (new_settled >= kp.converge_window) level_done = 1;
    }
    for (int k = 0; k < ICP_NMOM; ++k) st->M[k] = M[k];
    st->n_last = n;
    if (status == ICP_LEVEL_OK) {
        for (int k = 0; k < 9; ++k) st->R[k] = R[k];
        for (int k = 0; k < 3; ++k) st->t[k] = t[k];
    }
    for (int k = 0; k < 6; ++k) st->x[k] = x[k];
    st->last_status = status;
    ICP_GLOBAL icp_level_stats& S = st->stats.level[ctl.level];
    S.iters_run = ctl.iter + 1;
    S.status = status;
    S.n_gated = N;
    S.n_kept = n;
    S.k_med = k_med;
    S.rmse = n > 0 ? sqrt(M[ICP_NMOM - 1] / (double)n) : 0.0;
    st->stats.iters_total = iters_total + 1;
    st->stats.status = total_status;
    st->settled = new_settled;
    st->last_kmed = new_last;
    if (level_done) st->level_done = 1;
}

// The tile partials a thread of a summing work-group adds: thread (g, c)
// takes entries 4g .. 4g + 3 (one 16-byte load per tile) of tiles
// t0 .. t1 - 1, the c-th of kRuns equal runs of consecutive tiles.  Eight
// lanes cover one tile's 32 floats, so a wave reads eight whole partials per
// load instruction.
constexpr int kGroups = ICP_PART_STRIDE / 4;
constexpr int kRuns = ICP_WG / kGroups;
static_assert(kGroups * 4 == ICP_PART_STRIDE && kGroups * kRuns == ICP_WG && ICP_NMOM < ICP_PART_STRIDE,
              "partial sum layout");
struct TileRun {
    int g, t0, t1;
};

__device__ __forceinline__ TileRun tile_run(int n_tiles) {
    const int tid = threadIdx.x;
    TileRun r;
    r.g = tid % kGroups;
    const int c = tid / kGroups;
    const int per = (n_tiles + kRuns - 1) / kRuns;
    r.t0 = c * per;
    r.t1 = min(r.t0 + per, n_tiles);
    return r;
}

typedef float pf4 __attribute__((ext_vector_type(4)));

// Slot 0 of the first kSumBatch tiles of the thread's run (loaded before the
// band is known: it does not depend on it).  Past the run's end a valid tile
// is loaded and not added, so no branch separates the loads.
constexpr int kSumBatch = 12;
__device__ __forceinline__ void load_slot0(const float* part_in, int tile_stride, const TileRun& r,
                                           pf4 (&a)[kSumBatch]) {
    const ICP_GLOBAL float* part = gconst(part_in);
#pragma unroll
    for (int u = 0; u < kSumBatch; ++u) {
        const int tt = max(0, min(r.t0 + u, r.t1 - 1));
        a[u] = *reinterpret_cast<const ICP_GLOBAL pf4*>(part + (size_t)tt * tile_stride + 4 * r.g);
    }
}

// Deterministic FP64 sums over the tiles of slot 0 plus, if slot2 > 0, slot
// `slot2` of every tile partial into sh_out[0..28]; whole work-group.  Each
// run adds its tiles in order and the runs are added in order.  a0 holds slot
// 0 of the first kSumBatch tiles of each thread's run (load_slot0).
__device__ void sum_partials(const float* part_in, int n_tiles, int tile_stride, int slot2, const pf4 (&a0)[kSumBatch],
                             double* sh_out) {
    const ICP_GLOBAL float* part = gconst(part_in);
    __shared__ double sh_sum[ICP_PART_STRIDE][kRuns + 1];
    const int tid = threadIdx.x;
    const TileRun r = tile_run(n_tiles);
    // kSumBatch tiles' loads are issued before their adds (the adds stay in
    // tile order): one memory latency per batch, not per tile.  The second
    // slot is always loaded (slot 0 again when unused) and selected.
    const bool two = slot2 > 0;
    const size_t off2 = two ? (size_t)slot2 * ICP_PART_STRIDE : 0;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    auto add = [&](const pf4& x, const pf4& y) {
        s[0] += two ? (double)x.x + (double)y.x : (double)x.x;
        s[1] += two ? (double)x.y + (double)y.y : (double)x.y;
        s[2] += two ? (double)x.z + (double)y.z : (double)x.z;
        s[3] += two ? (double)x.w + (double)y.w : (double)x.w;
    };
    {  // the first batch: slot 0 is already in a0
        pf4 b[kSumBatch];
#pragma unroll
        for (int u = 0; u < kSumBatch; ++u) {
            const int tt = max(0, min(r.t0 + u, r.t1 - 1));
            b[u] = *reinterpret_cast<const ICP_GLOBAL pf4*>(part + (size_t)tt * tile_stride + 4 * r.g + off2);
        }
#pragma unroll
        for (int u = 0; u < kSumBatch; ++u)
            if (r.t0 + u < r.t1) add(a0[u], b[u]);
    }
    for (int t = r.t0 + kSumBatch; t < r.t1; t += kSumBatch) {
        pf4 a[kSumBatch], b[kSumBatch];
#pragma unroll
        for (int u = 0; u < kSumBatch; ++u) {
            const int tt = min(t + u, r.t1 - 1);
            const ICP_GLOBAL float* q = part + (size_t)tt * tile_stride + 4 * r.g;
            a[u] = *reinterpret_cast<const ICP_GLOBAL pf4*>(q);
            b[u] = *reinterpret_cast<const ICP_GLOBAL pf4*>(q + off2);
        }
#pragma unroll
        for (int u = 0; u < kSumBatch; ++u)
            if (t + u < r.t1) add(a[u], b[u]);
    }
    const int c = tid / kGroups;
#pragma unroll
    for (int k = 0; k < 4; ++k) sh_sum[4 * r.g + k][c] = s[k];
    __syncthreads();
    if (tid <= ICP_NMOM) {
        double v = 0.0;
        for (int q = 0; q < kRuns; ++q) v += sh_sum[tid][q];
        sh_out[tid] = v;
    }
    __syncthreads();
}

__device__ __forceinline__ void sum_partials(const float* part, int n_tiles, int tile_stride, int slot2,
                                             double* sh_out) {
    pf4 a0[kSumBatch];
    load_slot0(part, tile_stride, tile_run(n_tiles), a0);
    sum_partials(part, n_tiles, tile_stride, slot2, a0, sh_out);
}

struct Band {
    uint32_t N;
    int32_t k_med, k_lo, k_hi;
};

// The histogram entries 4 tid .. 4 tid + 3 a thread of the band kernel owns
// (loaded together with the rest of the state the kernel starts from).
__device__ __forceinline__ void load_hist4(const ProbState* st, int par, uint32_t (&h)[4]) {
    const ICP_GLOBAL uint32_t* hist = gconst(st->hist[par]);
#pragma unroll
    for (int k = 0; k < 4; ++k) h[k] = hist[4 * threadIdx.x + k];
}

// Cleared for the next iteration, through a global pointer so that no later
// LDS wait waits for the stores.
__device__ __forceinline__ void clear_hist4(ProbState* st, int par) {
    ICP_GLOBAL uint32_t* hist = gmut(st->hist[par]);
#pragma unroll
    for (int k = 0; k < 4; ++k) hist[4 * threadIdx.x + k] = 0u;
}

// Median bin k_med = min{k : C_k >= ceil(N/2)} of the CDF of the histogram
// h (each thread's four entries) and the kept band (Sec. 3.3), returned to
// every thread through LDS; the CDF is left in sh_cdf (ICP_HIST_BINS
// entries; set when N > 0).  Whole work-group; it writes no state.
__device__ Band find_band(const uint32_t (&h)[4], const KParams& kp, uint32_t* dbg_hist, uint32_t* sh_cdf) {
    __shared__ uint32_t sh_wsum[ICP_WAVES];
    __shared__ int32_t sh_kmed;
    __shared__ Band sh_band;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (dbg_hist)
        for (int k = 0; k < 4; ++k) dbg_hist[4 * tid + k] = h[k];
    const uint32_t own = (h[0] + h[1]) + (h[2] + h[3]);
    uint32_t incl = own;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) sh_wsum[wave] = incl;
    if (tid == 0) sh_kmed = -1;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < ICP_WAVES; ++w) {
        if (w < wave) before += sh_wsum[w];
        total += sh_wsum[w];
    }
    const uint32_t target = (total + 1u) / 2u;
    uint32_t c = before + incl - own;  // CDF just before this thread's first bin
    if (total > 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t prev = c;
            c += h[k];
            sh_cdf[4 * tid + k] = c;
            if (prev < target && c >= target) sh_kmed = 4 * tid + k;
        }
    }
    __syncthreads();
    if (tid == 0) {
        const int32_t km = sh_kmed;
        int32_t lo = 0, hi = -1;
        if (total > 0) {
            if (kp.use_filter) {
                const double flo = floor((1.0 - kp.band_beta) * (double)km);
                const double fhi = ceil((1.0 + kp.band_beta) * (double)(km + 1)) - 1.0;
                lo = flo < 0.0 ? 0 : (int32_t)flo;
                hi = fhi > (double)(ICP_HIST_BINS - 1) ? ICP_HIST_BINS - 1 : (int32_t)fhi;
            } else {
                hi = ICP_HIST_BINS - 1;
            }
        }
        sh_band = Band{total, km, lo, hi};
    }
    __syncthreads();
    return sh_band;
}

// The band of the iteration into the problem's state (one thread), through a
// global pointer: no later barrier or LDS wait waits for the stores.
__device__ __forceinline__ void store_band(ProbState* st, const Band& b) {
    ICP_GLOBAL ProbState* gw = gmut(st);
    gw->N = b.N;
    gw->k_med = b.k_med;
    gw->k_lo = b.k_lo;
    gw->k_hi = b.k_hi;
}

// Centring point of the split-precision reduction: the level's live centroid
// moved by the current pose.
__device__ __forceinline__ void set_centre(ProbState* st_in, int level) {
    ICP_GLOBAL ProbState* st = gmut(st_in);
    const double R[9] = {st->R[0], st->R[1], st->R[2], st->R[3], st->R[4], st->R[5], st->R[6], st->R[7], st->R[8]};
    const double t[3] = {st->t[0], st->t[1], st->t[2]};
    const double c[3] = {st->cen[level][0], st->cen[level][1], st->cen[level][2]};
    for (int i = 0; i < 3; ++i) st->cur_c[i] = ((R[3 * i] * c[0] + R[3 * i + 1] * c[1]) + R[3 * i + 2] * c[2]) + t[i];
}

// Back from centred rows: with a = [ (p' - c) x n + c x n, n ] = J a~,
// J = [[I, [c]x], [0, I]], the moments are J M~ J^T and J g~ (FP64).
__device__ void uncentre(double* M, const double* c) {
    double A[6][6], g[6];
    for (int i = 0; i < 6; ++i) {
        for (int j = i; j < 6; ++j) A[i][j] = A[j][i] = M[tri7(i, j)];
        g[i] = M[tri7(i, 6)];
    }
    const double C[3][3] = {{0.0, -c[2], c[1]}, {c[2], 0.0, -c[0]}, {-c[1], c[0], 0.0}};
    double J[6][6] = {};
    for (int i = 0; i < 6; ++i) J[i][i] = 1.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) J[i][3 + j] = C[i][j];
    double T[6][6], B[6][6], h[6];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += J[i][k] * A[k][j];
            T[i][j] = s;
        }
    for (int i = 0; i < 6; ++i) {
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += T[i][k] * J[j][k];
            B[i][j] = s;
        }
        double s = 0.0;
        for (int k = 0; k < 6; ++k) s += J[i][k] * g[k];
        h[i] = s;
    }
    for (int i = 0; i < 6; ++i) {
        for (int j = i; j < 6; ++j) M[tri7(i, j)] = B[i][j];
        M[tri7(i, 6)] = h[i];
    }
}

// One work-group per problem: the band; in single-pass mode, when the band
// edge fell inside the predicted window, the kept rows' moments are summed
// from the pass-1 partials and the iteration is completed here.
__global__ __launch_bounds__(ICP_WG) void k_band(const ProbDesc* __restrict__ probs, IterCtl ctl, KParams kp,
                                                 int fused, uint32_t* dbg_hist) {
    __shared__ double sh_M[ICP_NMOM + 1];
    const ProbDesc& P = probs[blockIdx.x];
    const LevelDesc& L = P.lv[ctl.level];
    ProbState* st = P.st;
    // the state the kernel starts from, loaded together: one wait, not three
    const ICP_GLOBAL ProbState* gst = gconst(st);
    uint32_t h[4];
    load_hist4(st, ctl.par, h);
    const int done = gst->level_done, pred = gst->pred_hi[ctl.par], pred_hw = gst->pred_hw[ctl.par];
    const EpiIn epi = load_epi(st);
    // (an empty statement that takes the loaded values, so that the compiler
    // issues every load above before the early return and waits once)
    __asm__ volatile("" ::"v"(h[0]), "v"(h[1]), "v"(h[2]), "v"(h[3]), "s"(pred), "s"(pred_hw), "v"(epi.R[0]),
                     "v"(epi.t[2]), "v"(epi.iters_total), "v"(epi.first_status));
    if (done) return;  // (pass 1 added nothing: the histogram is still clear)
    // slot 0 of the tile partials does not depend on the band: its loads are
    // in flight while the band is found
    pf4 a0[kSumBatch];
    if (fused) load_slot0(L.part1, ICP_WIN_SLOTS * ICP_PART_STRIDE, tile_run(L.n_tiles), a0);
    const Win win = fused ? band_window(pred, pred_hw, ctl.iter) : Win{-1, 0};
    const int h0 = win.h0;
    // split precision: the centring point of this iteration (before any update)
    if (kp.reduce_mode == 1 && threadIdx.x == 0) set_centre(st, ctl.level);
    __shared__ uint32_t sh_cdf[ICP_HIST_BINS];
    const Band b = find_band(h, kp, dbg_hist, sh_cdf);
    if (threadIdx.x == 0) store_band(st, b);
    clear_hist4(st, ctl.par);
    const bool hit = h0 >= 0 && b.N > 0 && b.k_lo == 0 && b.k_hi >= h0 - 1 && b.k_hi <= h0 + win.w - 1;
    if (hit) {
        sum_partials(L.part1, L.n_tiles, ICP_WIN_SLOTS * ICP_PART_STRIDE, b.k_hi - h0 + 1, a0, sh_M);
        if (threadIdx.x == 0) {
            if (kp.reduce_mode == 1) uncentre(sh_M, st->cur_c);
            solve_epilogue(st, epi, b.N, b.k_med, sh_M, (int64_t)sh_M[ICP_NMOM], ctl, kp, P.imu_R);
        }
    }
    if (threadIdx.x == 0) {
        st->fused_done = hit ? 1 : 0;
        if (!hit && kp.need2) atomicExch(kp.need2, 1);  // pass 2 has work this iteration
        if (b.N > 0) {
            st->pred_hw[ctl.par] = capped_half_width(sh_cdf, b.k_hi, next_half_width(b.k_hi, pred, ctl.iter), L.npx);
            st->pred_hi[ctl.par] = b.k_hi;
        }
    }
}

// ------------------------------------------------------------------ pass 2
// Filter (kept iff gated and its bin lies in the band) and the 28-moment
// reduction of the kept rows into one partial per tile.

#ifndef ICP_PASS2_WAVES
#define ICP_PASS2_WAVES 5
#endif

// Pass 2 over one tile: the rows kept by the band [klo, khi] reduced into
// acc and cnt (one pixel per lane and round, software-pipelined as in pass 1:
// the next round's gathers are in flight while a round is decided).
__device__ __forceinline__ void pass2_tile(const LevelDesc& L, const ProbState* st, int tile, int klo, int khi,
                                           const KParams& kp, float (&acc)[ICP_NMOM], float& cnt) {
    const int tid = threadIdx.x;
    const Pose T = load_pose(st);
    const Lvl Lv = load_level(L);
    const int base = tile * L.tile_px;
    const int end = min(base + L.tile_px, L.npx);
    constexpr int kRound = ICP_WG;
    auto ld_index = [&](int r) {
        const int i = r + tid;
        return i < end ? i : r;
    };
    auto next_r = [&](int r) { return r + kRound < end ? r + kRound : r; };
    Proj<1> pa = assoc_project<1>(Lv, base + tid, end, load_live<1>(Lv, ld_index(base)), T);
    Gath<1> ga = assoc_gather<1>(Lv, base + tid, pa);
    LiveIn<1> nxt = load_live<1>(Lv, ld_index(next_r(base)));
    for (int r = base; r < end; r += kRound) {
        const LiveIn<1> nn = load_live<1>(Lv, ld_index(next_r(next_r(r))));
        const Proj<1> pb = assoc_project<1>(Lv, r + kRound + tid, end, nxt, T);
        const Gath<1> gb = assoc_gather<1>(Lv, r + kRound + tid, pb);
        assoc_decide<1>(pa, ga, T, kp.d2max, kp.cos_max, [&](int, const PixelOut& q) {
            if (q.code == kGated && q.bin >= klo && q.bin <= khi) {
                accumulate_row(q.p, q.d, q.n, acc);
                cnt += 1.0f;
            }
        });
        pa = pb;
        ga = gb;
        nxt = nn;
    }
}

__global__ __launch_bounds__(ICP_WG) __attribute__((amdgpu_waves_per_eu(ICP_PASS2_WAVES))) void k_pass2(
    const ProbDesc* __restrict__ probs, const int* __restrict__ owner, IterCtl ctl, KParams kp) {
    // every problem of the batch finished its iteration in the band kernel
    if (kp.need2 && __builtin_amdgcn_readfirstlane(*kp.need2) == 0) return;
    __shared__ float sh_red[ICP_WAVES][ICP_PART_STRIDE];
    const int g = blockIdx.x;
    const ProbDesc& P = probs[owner[g]];
    const LevelDesc& L = P.lv[ctl.level];
    const ProbState* st = P.st;
    const int tile = g - L.tile_base;
    if (st->level_done || st->fused_done) return;  // uniform
    float acc[ICP_NMOM];
#pragma unroll
    for (int k = 0; k < ICP_NMOM; ++k) acc[k] = 0.0f;
    float cnt = 0.0f;
    pass2_tile(L, st, tile, __builtin_amdgcn_readfirstlane(st->k_lo), __builtin_amdgcn_readfirstlane(st->k_hi), kp,
               acc, cnt);
    block_reduce_row(acc, cnt, sh_red, gmut(L.part) + (size_t)tile * ICP_PART_STRIDE);
}

// One problem in single-pass mode (FP32 reduction): the band kernel, pass 2
// and the solve in one launch over the problem's tiles.  Every work-group
// finds the band from the histogram pass 1 left (the same arithmetic on the
// same counts, so the same band in each).  When the band edge fell inside the
// predicted window (or nothing was gated, or the level has ended) no pixel is
// revisited, and work-group 0 completes the iteration alone: the window's
// sums, the solve, the level's books.  Otherwise each work-group filters and
// reduces its own tile as pass 2 does, publishes its partial and takes a
// ticket; the one that takes the last completes the iteration from pass 2's
// partials.
//
// What a work-group decides from (histogram, window prediction, level_done)
// is never changed in a way that changes a decision while the launch runs:
// the histogram and the prediction in use are the ones IterCtl::par selects,
// and the iteration's writes go to the others (the next iteration's
// prediction, and the clear of the histogram the previous launch read, which
// the next pass 1 fills); level_done changes only where the band was a hit
// or the level had ended, where every work-group has nothing to do whatever
// it reads (a level reset leaves the histogram in use clear: N = 0).
// (Occupancy does not matter for one problem: the registers are not limited.)
__device__ __forceinline__ void band_pass2_finish(ProbState* st, const ProbDesc& P, const LevelDesc& L,
                                                  const IterCtl& ctl, const KParams& kp, const EpiIn& epi,
                                                  const Band& b, bool done, int pred, int pred_hw,
                                                  const double* sh_M, const uint32_t* sh_cdf) {
    const int par = ctl.par;
    if (threadIdx.x == 0) {
        ICP_GLOBAL ProbState* sw = gmut(st);
        if (!done) {
            store_band(st, b);
            solve_epilogue(st, epi, b.N, b.k_med, sh_M, (int64_t)sh_M[ICP_NMOM], ctl, kp, P.imu_R);
        }
        const bool upd = !done && b.N > 0;
        sw->pred_hw[1 - par] =
            upd ? capped_half_width(sh_cdf, b.k_hi, next_half_width(b.k_hi, pred, ctl.iter), L.npx) : pred_hw;
        sw->pred_hi[1 - par] = upd ? b.k_hi : pred;
        if (ctl.last_of_level) level_reset(st);
    }
    clear_hist4(st, 1 - par);
}

__global__ __launch_bounds__(ICP_WG) void k_band_pass2(const ProbDesc* __restrict__ probs, IterCtl ctl, KParams kp) {
    __shared__ double sh_M[ICP_NMOM + 1];
    __shared__ uint32_t sh_cdf[ICP_HIST_BINS];
    __shared__ float sh_red[ICP_WAVES][ICP_PART_STRIDE];
    __shared__ int sh_last;
    const ProbDesc& P = probs[0];
    const LevelDesc& L = P.lv[ctl.level];
    ProbState* st = P.st;
    const ICP_GLOBAL ProbState* gst = gconst(st);
    const int tid = threadIdx.x, tile = blockIdx.x;
    uint32_t h[4];
    load_hist4(st, ctl.par, h);
    const int done = gst->level_done, pred = gst->pred_hi[ctl.par], pred_hw = gst->pred_hw[ctl.par];
    // work-group 0 completes most iterations: its solve state and slot 0 of
    // the window partials are loaded with the histogram
    EpiIn epi;
    pf4 a0[kSumBatch];
    if (tile == 0) {
        epi = load_epi(st);
        load_slot0(L.part1, ICP_WIN_SLOTS * ICP_PART_STRIDE, tile_run(L.n_tiles), a0);
    }
    __asm__ volatile("" ::"v"(h[0]), "v"(h[1]), "v"(h[2]), "v"(h[3]), "s"(done), "s"(pred), "s"(pred_hw));
    const Win win = band_window(pred, pred_hw, ctl.iter);
    Band b{0u, -1, 0, -1};
    bool hit = false, need2 = false;
    if (!done) {  // uniform; when done, pass 1 added nothing
        b = find_band(h, kp, nullptr, sh_cdf);
        hit = win.h0 >= 0 && b.N > 0 && b.k_lo == 0 && b.k_hi >= win.h0 - 1 && b.k_hi <= win.h0 + win.w - 1;
        need2 = b.N > 0 && !hit;
    }
    if (!need2) {
        if (tile != 0) return;
        if (hit) {
            sum_partials(L.part1, L.n_tiles, ICP_WIN_SLOTS * ICP_PART_STRIDE, b.k_hi - win.h0 + 1, a0, sh_M);
        } else {  // nothing gated (or the level has ended): every moment is zero
            if (tid <= ICP_NMOM) sh_M[tid] = 0.0;
            __syncthreads();
        }
        band_pass2_finish(st, P, L, ctl, kp, epi, b, done, pred, pred_hw, sh_M, sh_cdf);
        return;
    }
    {
        float acc[ICP_NMOM];
#pragma unroll
        for (int k = 0; k < ICP_NMOM; ++k) acc[k] = 0.0f;
        float cnt = 0.0f;
        pass2_tile(L, st, tile, b.k_lo, b.k_hi, kp, acc, cnt);
        block_reduce_row(acc, cnt, sh_red, gmut(L.part) + (size_t)tile * ICP_PART_STRIDE);
    }
    __threadfence();  // the partial is visible device-wide before the ticket
    __syncthreads();
    if (tid == 0) sh_last = atomicAdd(&st->ticket, 1) == L.n_tiles - 1;
    __syncthreads();
    if (!sh_last) return;
    __threadfence();
    epi = load_epi(st);
    sum_partials(L.part, L.n_tiles, ICP_PART_STRIDE, 0, sh_M);
    band_pass2_finish(st, P, L, ctl, kp, epi, b, false, pred, pred_hw, sh_M, sh_cdf);
    if (tid == 0) gmut(st)->ticket = 0;
}

// Split-precision variant of pass 2 (reduce_mode 1): each kept row
// r = [(p' - c) x n, n, b, 1], scaled per column by a power of two, is split
// into FP16 hi = fp16(r) and lo = fp16(r - hi).  Thirty-two rows of
// X = [hi | lo] (32 x 16) go through one v_mfma_f32_16x16x32_f16 as
// X^T X with FP32 accumulation; the four 8x8 blocks hi'hi + hi'lo + lo'hi +
// lo'lo sum to the Gram matrix of the rows.  Lane l supplies column l % 16
// of eight rows to both operands, so the product does not depend on how the
// hardware orders the k slots.  Rows are staged through LDS: each round a
// wave's 256 pixels form eight groups of 32.

__global__ __launch_bounds__(ICP_WG) __attribute__((amdgpu_waves_per_eu(6))) void k_pass2_mfma(
    const ProbDesc* __restrict__ probs, const int* __restrict__ owner, IterCtl ctl, KParams kp) {
    if (kp.need2 && __builtin_amdgcn_readfirstlane(*kp.need2) == 0) return;  // nothing to do (see k_pass2)
    __shared__ _Float16 sh_x[ICP_WAVES][16][32];  // a half-wave's rows, column-major
    __shared__ float sh_red[ICP_WAVES][ICP_PART_STRIDE];
    const int g = blockIdx.x;
    const ProbDesc& P = probs[owner[g]];
    const LevelDesc& L = P.lv[ctl.level];
    const ProbState* st = P.st;
    const int tid = threadIdx.x, wave = tid >> 6;
    const int tile = g - L.tile_base;
    if (st->level_done || st->fused_done) return;  // uniform
    const float c0 = (float)st->cur_c[0], c1 = (float)st->cur_c[1], c2 = (float)st->cur_c[2];
    f4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
    {
        const Pose T = load_pose(st);
        const Lvl Lv = load_level(L);
        const int klo = __builtin_amdgcn_readfirstlane(st->k_lo);
        const int khi = __builtin_amdgcn_readfirstlane(st->k_hi);
        const int base = tile * L.tile_px;
        const int end = min(base + L.tile_px, L.npx);
        // pass 2's software pipeline; every lane of the work-group runs the
        // same rounds (the MFMA staging works across the wave)
        constexpr int kRound = ICP_WG;
        auto ld_index = [&](int r) {
            const int i = r + tid;
            return i < end ? i : r;
        };
        auto next_r = [&](int r) { return r + kRound < end ? r + kRound : r; };
        Proj<1> pa = assoc_project<1>(Lv, base + tid, end, load_live<1>(Lv, ld_index(base)), T);
        Gath<1> ga = assoc_gather<1>(Lv, base + tid, pa);
        LiveIn<1> nxt = load_live<1>(Lv, ld_index(next_r(base)));
        for (int r = base; r < end; r += kRound) {
            const LiveIn<1> nn = load_live<1>(Lv, ld_index(next_r(next_r(r))));
            const Proj<1> pb = assoc_project<1>(Lv, r + kRound + tid, end, nxt, T);
            const Gath<1> gb = assoc_gather<1>(Lv, r + kRound + tid, pb);
            assoc_decide<1>(pa, ga, T, kp.d2max, kp.cos_max, [&](int, const PixelOut& q) {
                const bool keep = q.code == kGated && q.bin >= klo && q.bin <= khi;
                const float pc[3] = {q.p[0] - c0, q.p[1] - c1, q.p[2] - c2};
                mfma_rows(keep, pc, q.d, q.n, sh_x[wave], acc);
            });
            pa = pb;
            ga = gb;
            nxt = nn;
        }
    }
    float mom[ICP_NMOM];
    float cnt = 0.0f;
    mfma_moments(acc, sh_x[wave], mom, cnt);
    block_reduce_row(mom, cnt, sh_red, gmut(L.part) + (size_t)tile * ICP_PART_STRIDE);
}

// One work-group per problem: FP64 sum of the pass-2 partials in tile order,
// solve, update; then the end-of-level bookkeeping.
__global__ __launch_bounds__(ICP_WG) void k_solve(const ProbDesc* __restrict__ probs, IterCtl ctl, KParams kp) {
    __shared__ double sh_M[ICP_NMOM + 1];
    const ProbDesc& P = probs[blockIdx.x];
    const LevelDesc& L = P.lv[ctl.level];
    ProbState* st = P.st;
    const ICP_GLOBAL ProbState* gst = gconst(st);
    const int32_t fused_done = gst->fused_done, done = gst->level_done;  // loaded together
    if (!fused_done && !done) {
        const EpiIn epi = load_epi(st);
        const uint32_t N = gst->N;
        const int32_t k_med = gst->k_med;
        sum_partials(L.part, L.n_tiles, ICP_PART_STRIDE, 0, sh_M);
        if (threadIdx.x == 0) {
            if (kp.reduce_mode == 1) uncentre(sh_M, st->cur_c);
            solve_epilogue(st, epi, N, k_med, sh_M, (int64_t)sh_M[ICP_NMOM], ctl, kp, P.imu_R);
        }
    }
    if (threadIdx.x == 0) {
        st->fused_done = 0;
        if (kp.need2 && blockIdx.x == 0) *kp.need2 = 0;  // pass 2 of this iteration has run
        if (ctl.last_of_level) level_reset(st);
    }
}

// ------------------------------------------------------------------ results

__global__ void k_finalize(const ProbDesc* __restrict__ probs, int n, icp_result* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const ProbState* st = probs[p].st;
    icp_result& r = out[p];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) r.pose[4 * i + j] = st->R[3 * i + j];
        r.pose[4 * i + 3] = st->t[i];
    }
    r.pose[12] = r.pose[13] = r.pose[14] = 0.0;
    r.pose[15] = 1.0;
    r.stats = st->stats;
}

// ------------------------------------------------------------------ stage access

__global__ void k_stage_set(const ProbDesc* __restrict__ probs, PoseArg pose, int k_lo, int k_hi, int level,
                            int pred_hi, int pred_hw) {
    ProbState* st = probs[0].st;
    for (int b = threadIdx.x; b < ICP_HIST_BINS; b += blockDim.x) st->hist[0][b] = 0u;  // (stage calls use par 0)
    if (threadIdx.x == 0) {
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) st->R[3 * i + j] = pose.v[4 * i + j];
            st->t[i] = pose.v[4 * i + 3];
        }
        st->k_lo = k_lo;
        st->k_hi = k_hi;
        st->pred_hi[0] = pred_hi;
        st->pred_hw[0] = pred_hw;
        st->fused_done = 0;
        st->level_done = 0;
        set_centre(st, level);
    }
}

// The band-edge window that pass 1 used for problem 0 (h0, width), read before
// the band kernel replaces the prediction.
__global__ void k_stage_window(const ProbDesc* __restrict__ probs, IterCtl ctl, int32_t* out) {
    if (threadIdx.x != 0) return;
    const ProbState* st = probs[0].st;
    const Win w = band_window(st->pred_hi[ctl.par], st->pred_hw[ctl.par], ctl.iter);
    out[0] = w.h0;
    out[1] = w.w;
}

__global__ void k_stage_solve(MomArg M, int64_t n, PoseArg pose, KParams kp, double* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double R[9], t[3], x[6];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) R[3 * i + j] = pose.v[4 * i + j];
        t[i] = pose.v[4 * i + 3];
    }
    const int status = solve_regularised(M.m, n, kp, R, nullptr, x);
    if (status == ICP_LEVEL_OK) compose_exp(x, R, t);
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) out[4 * i + j] = R[3 * i + j];
        out[4 * i + 3] = t[i];
    }
    for (int k = 0; k < 6; ++k) out[12 + k] = x[k];
    out[18] = (double)status;
}

// ------------------------------------------------------------------ descriptor upload
// A problem descriptor passed by value (a kernel argument) written to device
// memory, and a fill of an int array: set-up without host-to-device copies.
__global__ void k_put_desc(ProbDesc d, ProbDesc* dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = d;
}

__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ launchers

static inline unsigned blocks_for(int n) { return (unsigned)((n + ICP_WG - 1) / ICP_WG); }

hipError_t launch_centroid(const ProbDesc* probs, int n, int levels, const int* const* owner, const int* tiles,
                           hipStream_t s) {
    for (int l = 0; l < levels; ++l)
        hipLaunchKernelGGL(k_centroid_tiles, dim3(tiles[l]), dim3(ICP_WG), 0, s, probs, owner[l], l);
    hipLaunchKernelGGL(k_centroid_sum, dim3(n, levels), dim3(64), 0, s, probs);
    return hipGetLastError();
}

int live_vn_blocks(int W, int H) { return ((W + FE_TX - 1) / FE_TX) * ((H + FE_TY - 1) / FE_TY); }

int model_blocks(int W, int H) { return ((W + 1) / 2) * ((H + 1) / 2); }

hipError_t launch_prepare(const ProbDesc* probs, int n, int levels, const int* max_vn_blocks,
                          const int* max_model_blocks, const int* max_quot, bool with_live_maps, const FrontEnd& fe,
                          int use_imu_seed, int32_t* need2, hipStream_t s) {
    if (fe.depth_filter) {
        const dim3 grid(max_vn_blocks[0], n);
        switch (fe.filter_radius) {
            case 1: hipLaunchKernelGGL(k_bilateral<1>, grid, dim3(ICP_WG), 0, s, probs, fe); break;
            case 2: hipLaunchKernelGGL(k_bilateral<2>, grid, dim3(ICP_WG), 0, s, probs, fe); break;
            case 3: hipLaunchKernelGGL(k_bilateral<3>, grid, dim3(ICP_WG), 0, s, probs, fe); break;
            case 4: hipLaunchKernelGGL(k_bilateral<4>, grid, dim3(ICP_WG), 0, s, probs, fe); break;
            case 5: hipLaunchKernelGGL(k_bilateral<5>, grid, dim3(ICP_WG), 0, s, probs, fe); break;
            case 6: hipLaunchKernelGGL(k_bilateral<6>, grid, dim3(ICP_WG), 0, s, probs, fe); break;
            case 7: hipLaunchKernelGGL(k_bilateral<7>, grid, dim3(ICP_WG), 0, s, probs, fe); break;
            default: return hipErrorInvalidValue;
        }
    }
    if (!fe.depth_filter && fe.normal_mode == 0 && (levels == 2 || levels == 3)) {
        const int nb_model = (int)blocks_for(4 * max_model_blocks[1]), nb_depth = (int)blocks_for(max_model_blocks[1]);
        const int next = levels == 3 ? 1 : 0, wv = with_live_maps ? 1 : 0;
        hipLaunchKernelGGL(k_front_inputs, dim3(nb_model + nb_depth + max_vn_blocks[0] + 1, n), dim3(ICP_WG), 0, s,
                           probs, nb_model, nb_depth, max_vn_blocks[0], next, wv, use_imu_seed, need2);
        if (levels == 3)
            hipLaunchKernelGGL(k_front_coarse, dim3(max_vn_blocks[1] + max_vn_blocks[2], n), dim3(ICP_WG), 0, s,
                               probs, max_vn_blocks[1], wv);
        else
            hipLaunchKernelGGL(k_live_vn, dim3(max_vn_blocks[1], n), dim3(ICP_WG), 0, s, probs, 1, wv);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_init, dim3(n), dim3(ICP_WG), 0, s, probs, use_imu_seed, need2);
    for (int l = 1; l < levels; l += 2)  // two levels per launch, as for the model maps
        hipLaunchKernelGGL(k_depth_down, dim3(blocks_for(max_model_blocks[l]), n), dim3(ICP_WG), 0, s, probs, l,
                           l + 1 < levels ? 1 : 0);
    if (fe.normal_mode == 1)  // (the quotient tables are read by the box normals only)
        for (int l = 0; l < levels; ++l)
            hipLaunchKernelGGL(k_quotients, dim3(blocks_for(max_quot[l]), n), dim3(ICP_WG), 0, s, probs, l);
    for (int l = 0; l < levels; ++l) {
        // live vertex planes (stage access) and forward-difference normals
        if (with_live_maps || fe.normal_mode == 0)
            hipLaunchKernelGGL(k_live_vn, dim3(max_vn_blocks[l], n), dim3(ICP_WG), 0, s, probs, l,
                               with_live_maps ? 1 : 0);
        if (fe.normal_mode == 1) {
            const dim3 grid(max_vn_blocks[l], n);
            switch (fe.normal_radius) {
                case 1: hipLaunchKernelGGL(k_live_n_box<1>, grid, dim3(ICP_WG), 0, s, probs, l); break;
                case 2: hipLaunchKernelGGL(k_live_n_box<2>, grid, dim3(ICP_WG), 0, s, probs, l); break;
                case 3: hipLaunchKernelGGL(k_live_n_box<3>, grid, dim3(ICP_WG), 0, s, probs, l); break;
                case 4: hipLaunchKernelGGL(k_live_n_box<4>, grid, dim3(ICP_WG), 0, s, probs, l); break;
                case 5: hipLaunchKernelGGL(k_live_n_box<5>, grid, dim3(ICP_WG), 0, s, probs, l); break;
                case 6: hipLaunchKernelGGL(k_live_n_box<6>, grid, dim3(ICP_WG), 0, s, probs, l); break;
                case 7: hipLaunchKernelGGL(k_live_n_box<7>, grid, dim3(ICP_WG), 0, s, probs, l); break;
                default: return hipErrorInvalidValue;
            }
        }
    }
    for (int l = 1; l < levels; l += 2)
        hipLaunchKernelGGL(k_model_down, dim3(blocks_for(4 * max_model_blocks[l]), n), dim3(ICP_WG), 0, s, probs, l,
                           l + 1 < levels ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_depth_to_maps(const MapsDesc* jobs, int n, int max_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_depth_to_maps, dim3(max_blocks, n), dim3(ICP_WG), 0, s, jobs);
    return hipGetLastError();
}

hipError_t launch_pass1(const ProbDesc* probs, const int* owner, int tiles, IterCtl ctl, const KParams& kp, int fused,
                        hipStream_t s) {
    if (fused && kp.reduce_mode == 1)
        hipLaunchKernelGGL((k_pass1<false, true, true>), dim3(tiles), dim3(ICP_WG), 0, s, probs, owner, ctl, kp,
                           nullptr, nullptr);
    else if (fused)
        hipLaunchKernelGGL((k_pass1<false, true, false>), dim3(tiles), dim3(ICP_WG), 0, s, probs, owner, ctl, kp,
                           nullptr, nullptr);
    else
        hipLaunchKernelGGL((k_pass1<false, false, false>), dim3(tiles), dim3(ICP_WG), 0, s, probs, owner, ctl, kp,
                           nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_band(const ProbDesc* probs, int n, IterCtl ctl, const KParams& kp, int fused, hipStream_t s) {
    hipLaunchKernelGGL(k_band, dim3(n), dim3(ICP_WG), 0, s, probs, ctl, kp, fused, nullptr);
    return hipGetLastError();
}

hipError_t launch_pass2(const ProbDesc* probs, const int* owner, int tiles, IterCtl ctl, const KParams& kp,
                        hipStream_t s) {
    if (kp.reduce_mode == 1)
        hipLaunchKernelGGL(k_pass2_mfma, dim3(tiles), dim3(ICP_WG), 0, s, probs, owner, ctl, kp);
    else
        hipLaunchKernelGGL(k_pass2, dim3(tiles), dim3(ICP_WG), 0, s, probs, owner, ctl, kp);
    return hipGetLastError();
}

hipError_t launch_band_pass2(const ProbDesc* probs, int tiles, IterCtl ctl, const KParams& kp, hipStream_t s) {
    hipLaunchKernelGGL(k_band_pass2, dim3(tiles), dim3(ICP_WG), 0, s, probs, ctl, kp);
    return hipGetLastError();
}

hipError_t launch_solve(const ProbDesc* probs, int n, IterCtl ctl, const KParams& kp, hipStream_t s) {
    hipLaunchKernelGGL(k_solve, dim3(n), dim3(ICP_WG), 0, s, probs, ctl, kp);
    return hipGetLastError();
}

hipError_t launch_put_desc(const ProbDesc& d, ProbDesc* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, d, dst);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n)), dim3(ICP_WG), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_finalize(const ProbDesc* probs, int n, icp_result* results, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3((n + 63) / 64), dim3(64), 0, s, probs, n, results);
    return hipGetLastError();
}

hipError_t launch_stage_set(const ProbDesc* probs, PoseArg pose, int k_lo, int k_hi, int level, int pred_hi,
                            int pred_hw, hipStream_t s) {
    hipLaunchKernelGGL(k_stage_set, dim3(1), dim3(ICP_WG), 0, s, probs, pose, k_lo, k_hi, level, pred_hi, pred_hw);
    return hipGetLastError();
}

hipError_t launch_stage_single(const ProbDesc* probs, const int* owner, int tiles, IterCtl ctl, const KParams& kp,
                               int32_t* window, hipStream_t s) {
    if (kp.reduce_mode == 1)
        hipLaunchKernelGGL((k_pass1<false, true, true>), dim3(tiles), dim3(ICP_WG), 0, s, probs, owner, ctl, kp,
                           nullptr, nullptr);
    else
        hipLaunchKernelGGL((k_pass1<false, true, false>), dim3(tiles), dim3(ICP_WG), 0, s, probs, owner, ctl, kp,
                           nullptr, nullptr);
    hipLaunchKernelGGL(k_stage_window, dim3(1), dim3(64), 0, s, probs, ctl, window);
    hipLaunchKernelGGL(k_band, dim3(1), dim3(ICP_WG), 0, s, probs, ctl, kp, 1, nullptr);
    return hipGetLastError();
}

hipError_t launch_stage_pass1(const ProbDesc* probs, const int* owner, int tiles, IterCtl ctl, const KParams& kp,
                              uint8_t* code, int32_t* bin, uint32_t* hist, hipStream_t s) {
    hipLaunchKernelGGL((k_pass1<true, false, false>), dim3(tiles), dim3(ICP_WG), 0, s, probs, owner, ctl, kp, code,
                       bin);
    hipLaunchKernelGGL(k_band, dim3(1), dim3(ICP_WG), 0, s, probs, ctl, kp, 0, hist);
    return hipGetLastError();
}

hipError_t launch_stage_pass2(const ProbDesc* probs, const int* owner, int tiles, IterCtl ctl, const KParams& kp,
                              hipStream_t s) {
    if (kp.reduce_mode == 1)
        hipLaunchKernelGGL(k_pass2_mfma, dim3(tiles), dim3(ICP_WG), 0, s, probs, owner, ctl, kp);
    else
        hipLaunchKernelGGL(k_pass2, dim3(tiles), dim3(ICP_WG), 0, s, probs, owner, ctl, kp);
    hipLaunchKernelGGL(k_solve, dim3(1), dim3(ICP_WG), 0, s, probs, ctl, kp);
    return hipGetLastError();
}

hipError_t launch_stage_solve(MomArg M, int64_t n, PoseArg pose, const KParams& kp, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_stage_solve, dim3(1), dim3(64), 0, s, M, n, pose, kp, out);
    return hipGetLastError();
}

}  // namespace icpk
