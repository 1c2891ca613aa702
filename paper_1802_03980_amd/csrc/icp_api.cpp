// Host side of the C ABI declared in include/icp.h: context, workspace
// planning, the per-level iteration driver and the stage-access calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "icp.h"
#include "icp_common.hpp"
#include "icp_internal.hpp"
#include "icp_launch.hpp"

struct icp_ctx {
    int device = 0;
    size_t budget = 0;
    void* ws = nullptr;  // device workspace
    size_t ws_cap = 0;
    void* hstage = nullptr;  // pinned upload staging
    size_t hstage_cap = 0;
    hipEvent_t ev_upload = nullptr;  // upload of the staging buffer finished
    bool ev_pending = false;
    hipEvent_t ev_done = nullptr;       // end of the work the last call queued
    hipStream_t done_stream = nullptr;  // the stream it was queued on
    bool done_valid = false;
    std::string err;
    // stage-access problem (problem 0 of the last icp_stage_prepare)
    bool stage_ready = false;
    int stage_levels = 0;
    ProbDesc stage_desc{};
    ProbDesc* d_desc = nullptr;
    int* d_owner[ICP_MAX_LEVELS] = {};
    int tiles[ICP_MAX_LEVELS] = {};
    ProbState* d_state = nullptr;
    double* d_scratch = nullptr;
    // kernel timing
    struct EvRec {
        int kind;
        hipEvent_t a, b;
        int64_t px;
    };
    bool timing = false;
    std::vector<EvRec> pending;
    std::vector<hipEvent_t> ev_pool;
    icp_kernel_time times[ICP_TIME_KINDS] = {};
    // plan and graph caches (valid for the current workspace allocation)
    std::vector<int64_t> plan_key;      // shapes + tiling of the cached plan
    std::vector<int64_t> owners_key;    // plan whose tile owners are in device memory
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;   // private stream used only for capture
    struct GraphEntry {
        std::vector<int64_t> key;       // plan, workspace and parameters it was captured with
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        uint64_t used = 0;              // last use (for least-recently-used eviction)
    };
    std::vector<GraphEntry> graphs;     // at most kGraphCache
    uint64_t graph_clock = 0;
    void* plan_mem = nullptr;  // the cached Plan (see ctx_plan)
    MapsDesc* d_jobs = nullptr;  // icp_live_maps job descriptor (device)
};

// Device memory of icp_register_noalloc: one file-scope array.  Every GPU the
// library runs on holds its own copy, at its own address, until the process
// ends; the host-side name is only a handle (see static_scratch).
constexpr size_t kStaticScratchBytes = ICP_NOALLOC_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kScratchBytes = 4096 + 8 * 64;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int fail(icp_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int hip_fail(icp_ctx* ctx, hipError_t e, const char* where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(ctx, ICP_EDEVICE, m);
}

#define HIP_TRY(ctx, expr)                                  \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

int check_params(icp_ctx* ctx, const icp_params* p) {
    if (!p) return fail(ctx, ICP_EINVAL, "params is NULL");
    if (p->levels < 1 || p->levels > ICP_MAX_LEVELS) return fail(ctx, ICP_EINVAL, "levels must be in 1..4");
    for (int l = 0; l < p->levels; ++l) {
        if (p->iters[l] < 0 || p->iters[l] > 100000) return fail(ctx, ICP_EINVAL, "iters out of range");
        const int t = p->tile_px[l];
        if (t != 0 && (t < ICP_TILE_QUANTUM || t > 65536 || t % ICP_TILE_QUANTUM != 0))
            return fail(ctx, ICP_EINVAL, "tile_px must be 0 or a multiple of 1024 in [1024, 65536]");
    }
    if (!(p->dist_max > 0.0 && p->dist_max <= 0.125)) return fail(ctx, ICP_EINVAL, "dist_max must be in (0, 0.125]");
    if (!(p->cos_angle_max >= -1.0 && p->cos_angle_max <= 1.0))
        return fail(ctx, ICP_EINVAL, "cos_angle_max must be in [-1, 1]");
    if (!(p->band_beta >= 0.0 && std::isfinite(p->band_beta))) return fail(ctx, ICP_EINVAL, "band_beta must be >= 0");
    if (p->lambda_mode < ICP_LAMBDA_CONST || p->lambda_mode > ICP_LAMBDA_C_OVER_N2)
        return fail(ctx, ICP_EINVAL, "unknown lambda_mode");
    if (!(p->lambda_c >= 0.0 && std::isfinite(p->lambda_c))) return fail(ctx, ICP_EINVAL, "lambda_c must be >= 0");
    if (p->min_corr < 1) return fail(ctx, ICP_EINVAL, "min_corr must be >= 1");
    if (!(p->ill_cond_eps >= 0.0)) return fail(ctx, ICP_EINVAL, "ill_cond_eps must be >= 0");
    if (p->converge_window < 0) return fail(ctx, ICP_EINVAL, "converge_window must be >= 0");
    if (p->reduce_mode != 0 && p->reduce_mode != 1) return fail(ctx, ICP_EINVAL, "reduce_mode must be 0 or 1");
    if (p->pass_mode != 0 && p->pass_mode != 1) return fail(ctx, ICP_EINVAL, "pass_mode must be 0 or 1");
    if (p->depth_filter != 0 && p->depth_filter != 1) return fail(ctx, ICP_EINVAL, "depth_filter must be 0 or 1");
    if (p->depth_filter &&
        (p->filter_radius < 1 || p->filter_radius > ICP_FILTER_MAX_R || !(p->filter_sigma_px > 0.0) ||
         !std::isfinite(p->filter_sigma_px) || !(p->filter_sigma_m > 0.0) || !std::isfinite(p->filter_sigma_m)))
        return fail(ctx, ICP_EINVAL, "filter_radius must be in 1..7 and the filter sigmas > 0");
    if (p->normal_mode != 0 && p->normal_mode != 1) return fail(ctx, ICP_EINVAL, "normal_mode must be 0 or 1");
    if (p->normal_mode == 1 && (p->normal_radius < 1 || p->normal_radius > ICP_FILTER_MAX_R))
        return fail(ctx, ICP_EINVAL, "normal_radius must be in 1..7");
    if (p->anchor_to_imu != 0 && p->anchor_to_imu != 1) return fail(ctx, ICP_EINVAL, "anchor_to_imu must be 0 or 1");
    return ICP_OK;
}

int check_problem(icp_ctx* ctx, const icp_problem& q, int levels, int use_imu_seed) {
    if (!q.live_depth || !q.model_vtx || !q.model_nrm) return fail(ctx, ICP_EINVAL, "input pointer is NULL");
    const int div = 1 << (levels - 1);
    if (q.W < 1 || q.H < 1 || q.W > ICP_MAX_DIM || q.H > ICP_MAX_DIM)
        return fail(ctx, ICP_EINVAL, "W and H must be in 1..8192");
    if (q.W % div || q.H % div) return fail(ctx, ICP_EINVAL, "W and H must be divisible by 2^(levels-1)");
    const icp_intrinsics& K = q.K;
    if (!(K.fx > 0 && K.fy > 0 && std::isfinite(K.fx) && std::isfinite(K.fy) && std::isfinite(K.cx) &&
          std::isfinite(K.cy)))
        return fail(ctx, ICP_EINVAL, "intrinsics must be finite with fx, fy > 0");
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(q.imu_R[k])) return fail(ctx, ICP_EINVAL, "imu_R not finite");
    for (int k = 0; k < 12; ++k)
        if (!std::isfinite(q.init_pose[k])) return fail(ctx, ICP_EINVAL, "init_pose not finite");
    // the pose lives in SE(3): the rotation the registration starts from must be one
    if (!icpi::is_rotation(q.imu_R, 3))
        return fail(ctx, ICP_EINVAL, "imu_R is not a rotation (|R^T R - I| > 1e-6 or det R <= 0)");
    if (!use_imu_seed && !icpi::is_rotation(q.init_pose, 4))
        return fail(ctx, ICP_EINVAL, "init_pose's rotation is not a rotation (|R^T R - I| > 1e-6 or det R <= 0)");
    return ICP_OK;
}

// Tile size: aim for ~8192 work-groups per pass over the batch (32 per CU).
// Pass-1 work-groups the GPU holds at once: five 256-thread work-groups per
// compute unit (96 VGPRs, 28 KB of LDS each) on 256 compute units.
constexpr int64_t kPass1Slots = 1280;

// Tile of a level: about 8192 tiles over the batch (at least one 1024-pixel
// quantum, at most 16384 pixels).  A work-group spends about four rounds'
// time starting up (first loads, the pipeline's first gathers, LDS clears)
// and finishing (tile sums, window scan, histogram merge), so a level whose
// tiles would run fewer than 16 rounds takes 4096-pixel tiles instead while
// that still gives every work-group slot a tile (the coarse levels of large
// batches).  `level_px` is the batch's pixel count at the level.
int pick_tile(int npx, int nprob, int req, int64_t level_px) {
    if (req > 0) return req;
    const long target = std::max(1L, 8192L / std::max(1, nprob));
    long t = (npx + target - 1) / target;
    t = (t + ICP_TILE_QUANTUM - 1) / ICP_TILE_QUANTUM * ICP_TILE_QUANTUM;
    t = std::min(16384L, std::max((long)ICP_TILE_QUANTUM, t));
    if (t < 4096 && level_px / 4096 >= kPass1Slots) t = 4096;
    return (int)t;
}

// Workspace layout of a batch; offsets are relative to the workspace base.
struct Plan {
    size_t off_desc = 0, off_state = 0, off_res = 0, off_scratch = 0, off_flags = 0, off_owner[ICP_MAX_LEVELS] = {};
    int tiles[ICP_MAX_LEVELS] = {};
    int max_vn[ICP_MAX_LEVELS] = {};  // live-map work-groups of the largest level
    int max_mp[ICP_MAX_LEVELS] = {};  // pyramid threads (2 x 2 blocks) of the largest level
    int max_q[ICP_MAX_LEVELS] = {};   // quotient-table entries (W + H + 2) of the largest level
    std::vector<ProbDesc> desc;  // pointers hold offsets until rebased
    std::vector<int> owner[ICP_MAX_LEVELS];
    size_t total = 0;
};

// Level sizes, tiles and level buffers of one problem of an n-problem batch:
// the buffers' offsets come from take(bytes), its tiles are appended to the
// flat tile ranges tiles[l], and the largest launch sizes are kept.
template <class Take>
void lay_out_problem(ProbDesc& d, int32_t W, int32_t H, int levels, const int32_t* tile_req, int nprob,
                     const int64_t* level_px, int* tiles, int* max_vn, int* max_mp, int* max_q, Take&& take) {
    for (int l = 0; l < levels; ++l) {
        LevelDesc& L = d.lv[l];
        L.W = W >> l;
        L.H = H >> l;
        L.npx = L.W * L.H;
        L.ps = (L.npx + ICP_PLANE_ALIGN - 1) / ICP_PLANE_ALIGN * ICP_PLANE_ALIGN;
        L.tile_px = pick_tile(L.npx, nprob, tile_req ? tile_req[l] : 0, level_px[l]);
        L.n_tiles = (L.npx + L.tile_px - 1) / L.tile_px;
        L.tile_base = tiles[l];
        tiles[l] += L.n_tiles;
        max_vn[l] = std::max(max_vn[l], icpk::live_vn_blocks(L.W, L.H));
        max_mp[l] = std::max(max_mp[l], icpk::model_blocks(L.W, L.H));
        max_q[l] = std::max(max_q[l], L.W + L.H + 2);
        const size_t S = (size_t)L.ps * sizeof(float);
        L.Dw = reinterpret_cast<float*>(take(S));  // level 0: the filtered depth, when filtering
        L.LV = reinterpret_cast<float*>(take(3 * S));
        L.LN = reinterpret_cast<float*>(take(3 * S));
        const size_t A = (size_t)L.npx * 3 * sizeof(float);
        L.MVw = l > 0 ? reinterpret_cast<float*>(take(A)) : nullptr;
        L.MNw = l > 0 ? reinterpret_cast<float*>(take(A)) : nullptr;
        L.XQ = reinterpret_cast<double*>(take((size_t)(L.W + 1) * sizeof(double)));
        L.YQ = reinterpret_cast<double*>(take((size_t)(L.H + 1) * sizeof(double)));
        L.part = reinterpret_cast<float*>(take((size_t)L.n_tiles * ICP_PART_STRIDE * sizeof(float)));
        L.part1 = reinterpret_cast<float*>(take((size_t)L.n_tiles * ICP_WIN_SLOTS * ICP_PART_STRIDE * sizeof(float)));
    }
}

void make_plan(int n, const int32_t* W, const int32_t* H, int levels, const int32_t* tile_req, Plan& P) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    P.desc.assign(n, ProbDesc{});
    P.off_desc = take(sizeof(ProbDesc) * n);
    P.off_state = take(sizeof(ProbState) * n);
    P.off_res = take(sizeof(icp_result) * n);
    P.off_scratch = take(kScratchBytes);
    P.off_flags = take(sizeof(int32_t));
    for (int l = 0; l < levels; ++l) {
        P.tiles[l] = 0;
        P.max_vn[l] = 0;
        P.max_mp[l] = 0;
        P.max_q[l] = 0;
        P.owner[l].clear();
    }
    int64_t level_px[ICP_MAX_LEVELS] = {};
    for (int p = 0; p < n; ++p)
        for (int l = 0; l < levels; ++l) level_px[l] += (int64_t)(W[p] >> l) * (H[p] >> l);
    for (int p = 0; p < n; ++p) {
        ProbDesc& d = P.desc[p];
        d.st = reinterpret_cast<ProbState*>(P.off_state + sizeof(ProbState) * p);
        lay_out_problem(d, W[p], H[p], levels, tile_req, n, level_px, P.tiles, P.max_vn, P.max_mp, P.max_q, take);
        for (int l = 0; l < levels; ++l)
            for (int t = 0; t < d.lv[l].n_tiles; ++t) P.owner[l].push_back(p);
    }
    for (int l = 0; l < levels; ++l) P.off_owner[l] = take(sizeof(int) * std::max(1, P.tiles[l]));
    P.total = off;
}

Plan& ctx_plan(icp_ctx* ctx) {
    if (!ctx->plan_mem) ctx->plan_mem = new Plan();
    return *static_cast<Plan*>(ctx->plan_mem);
}

std::vector<int64_t> plan_signature(int n, const icp_problem* probs, int levels, const int32_t* tile_req) {
    std::vector<int64_t> k;
    k.reserve(6 + 2 * (size_t)n);
    k.push_back(n);
    k.push_back(levels);
    for (int l = 0; l < ICP_MAX_LEVELS; ++l) k.push_back(tile_req ? tile_req[l] : 0);
    for (int p = 0; p < n; ++p) {
        k.push_back(probs[p].W);
        k.push_back(probs[p].H);
    }
    return k;
}

void destroy_graph(icp_ctx::GraphEntry& g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g.exec = nullptr;
    g.graph = nullptr;
}

void drop_graphs(icp_ctx* ctx) {
    for (auto& g : ctx->graphs) destroy_graph(g);
    ctx->graphs.clear();
}

template <typename T>
T* rebase(T* off, char* base) {
    return reinterpret_cast<T*>(base + reinterpret_cast<size_t>(off));
}

int ensure_workspace(icp_ctx* ctx, size_t bytes, bool exact = false) {
    if (ctx->budget && bytes > ctx->budget)
        return fail(ctx, ICP_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes exceeds the HBM budget");
    if (bytes <= ctx->ws_cap) return ICP_OK;
    const icpi::RelaxedCaptureScope relaxed;
    if (ctx->ws) {
        // the old workspace is free once this context's last call has ended
        // (each call waits for the one before); no device-wide wait, which
        // would also wait on a graph another thread may be capturing
        if (ctx->done_valid) HIP_TRY(ctx, hipEventSynchronize(ctx->ev_done));
        HIP_TRY(ctx, hipFree(ctx->ws));
        ctx->ws = nullptr;
        ctx->ws_cap = 0;
        ctx->stage_ready = false;
    }
    ctx->owners_key.clear();
    drop_graphs(ctx);
    // growth margin so that slightly larger batches reuse the allocation; none
    // when the caller sized the request itself
    size_t want = exact ? bytes : bytes + bytes / 4;
    if (ctx->budget) want = std::min(want, ctx->budget);
    hipError_t e = hipMalloc(&ctx->ws, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ctx->ws = nullptr;
        return fail(ctx, ICP_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    ctx->ws_cap = want;
    return ICP_OK;
}

// Calls may come on different streams, while the workspace, descriptors and
// staging memory of a context are shared: a call first orders its stream
// after the work the previous call queued, and on its way out (on every path,
// errors included) records where its own work ends.
class StreamTurn {
  public:
    int enter(icp_ctx* ctx, hipStream_t s) {
        if (ctx->done_valid && s != ctx->done_stream) HIP_TRY(ctx, hipStreamWaitEvent(s, ctx->ev_done, 0));
        ctx_ = ctx;
        s_ = s;
        return ICP_OK;
    }
    ~StreamTurn() {
        if (!ctx_) return;
        if (hipEventRecord(ctx_->ev_done, s_) == hipSuccess) {
            ctx_->done_stream = s_;
            ctx_->done_valid = true;
        } else {
            (void)hipGetLastError();
        }
    }

  private:
    icp_ctx* ctx_ = nullptr;
    hipStream_t s_ = nullptr;
};

int ensure_stage(icp_ctx* ctx, size_t bytes) {
    if (ctx->ev_pending) {
        HIP_TRY(ctx, hipEventSynchronize(ctx->ev_upload));
        ctx->ev_pending = false;
    }
    if (bytes <= ctx->hstage_cap) return ICP_OK;
    const icpi::RelaxedCaptureScope relaxed;
    if (ctx->hstage) HIP_TRY(ctx, hipHostFree(ctx->hstage));
    ctx->hstage = nullptr;
    ctx->hstage_cap = 0;
    HIP_TRY(ctx, hipHostMalloc(&ctx->hstage, bytes));
    ctx->hstage_cap = bytes;
    return ICP_OK;
}

// The bilateral filter's spatial weights exp(-(du^2 + dv^2) / (2 s^2)) in
// row-major window order, evaluated on the host once per call.
FrontEnd front_end(const icp_params* p) {
    FrontEnd fe{};
    fe.depth_filter = p->depth_filter;
    fe.filter_radius = p->filter_radius;
    fe.normal_mode = p->normal_mode;
    fe.normal_radius = p->normal_radius;
    fe.sigma_m = p->filter_sigma_m;
    fe.inv_sigma_m = 1.0 / p->filter_sigma_m;
    if (p->depth_filter) {
        const int r = p->filter_radius, n = 2 * r + 1;
        const double sp = p->filter_sigma_px;
        for (int dv = -r; dv <= r; ++dv)
            for (int du = -r; du <= r; ++du)
                fe.ws[(dv + r) * n + (du + r)] = std::exp(-(double)(du * du + dv * dv) / (2.0 * sp * sp));
    }
    return fe;
}

KParams kparams(const icp_params* p) {
    KParams k{};
    k.d2max = p->dist_max * p->dist_max;
    k.cos_max = p->cos_angle_max;
    k.band_beta = p->band_beta;
    k.lambda_c = p->lambda_c;
    k.ill_cond_eps = p->ill_cond_eps;
    k.lambda_mode = p->lambda_mode;
    k.use_filter = p->use_median_filter;
    k.min_corr = p->min_corr;
    k.converge_window = p->converge_window;
    k.reduce_mode = p->reduce_mode;
    k.anchor_to_imu = p->anchor_to_imu;
    return k;
}

// A laid-out descriptor (pointers holding workspace offsets) made absolute
// against the workspace base, with the problem's inputs, level intrinsics
// (the pixel centre of a level-(l+1) pixel is the mean of its children's:
// f / 2^l, (c + 1/2) / 2^l - 1/2), IMU prior and initial pose.
void bind_problem(ProbDesc& d, const icp_problem& q, int levels, int depth_filter, char* base) {
    d.st = rebase(d.st, base);
    for (int l = 0; l < levels; ++l) {
        LevelDesc& L = d.lv[l];
        const double s2 = std::ldexp(1.0, -l);
        L.fx = q.K.fx * s2;
        L.fy = q.K.fy * s2;
        L.cx = (q.K.cx + 0.5) * s2 - 0.5;
        L.cy = (q.K.cy + 0.5) * s2 - 0.5;
        L.rfx = 1.0 / L.fx;
        L.rfy = 1.0 / L.fy;
        L.umax = (double)(L.W - 1);
        L.vmax = (double)(L.H - 1);
        L.Dw = rebase(L.Dw, base);
        L.D = (l > 0 || depth_filter) ? L.Dw : q.live_depth;
        L.LV = rebase(L.LV, base);
        L.LN = rebase(L.LN, base);
        L.MVw = l > 0 ? rebase(L.MVw, base) : nullptr;
        L.MNw = l > 0 ? rebase(L.MNw, base) : nullptr;
        L.MV = l > 0 ? L.MVw : q.model_vtx;
        L.MN = l > 0 ? L.MNw : q.model_nrm;
        L.XQ = rebase(L.XQ, base);
        L.YQ = rebase(L.YQ, base);
        L.part = rebase(L.part, base);
        L.part1 = rebase(L.part1, base);
    }
    d.depth_in = q.live_depth;
    std::memcpy(d.imu_R, q.imu_R, sizeof(d.imu_R));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 4; ++j) d.init[4 * i + j] = q.init_pose[4 * i + j];
}

// Plan, place and upload a batch; leaves device descriptors ready.
int stage_batch(icp_ctx* ctx, int n, const icp_problem* probs, int levels, const int32_t* tile_req,
                int depth_filter, Plan& P, hipStream_t s) {
    std::vector<int64_t> key = plan_signature(n, probs, levels, tile_req);
    if (key != ctx->plan_key || P.desc.size() != (size_t)n) {
        std::vector<int32_t> W(n), H(n);
        for (int p = 0; p < n; ++p) {
            W[p] = probs[p].W;
            H[p] = probs[p].H;
        }
        make_plan(n, W.data(), H.data(), levels, tile_req, P);
        ctx->plan_key = key;
    } else {
        // same shapes: reset the descriptors' device pointers to offsets
        std::vector<int32_t> W(n), H(n);
        for (int p = 0; p < n; ++p) {
            W[p] = probs[p].W;
            H[p] = probs[p].H;
        }
        Plan fresh;
        make_plan(n, W.data(), H.data(), levels, tile_req, fresh);
        P.desc.swap(fresh.desc);
    }
    int rc = ensure_workspace(ctx, P.total);
    if (rc) return rc;
    char* base = static_cast<char*>(ctx->ws);
    for (int p = 0; p < n; ++p) bind_problem(P.desc[p], probs[p], levels, depth_filter, base);
    const size_t up = sizeof(ProbDesc) * n;
    const bool owners = ctx->owners_key != key;
    size_t owner_bytes = 0;
    if (owners)
        for (int l = 0; l < levels; ++l) owner_bytes += sizeof(int) * P.owner[l].size();
    rc = ensure_stage(ctx, up + owner_bytes);
    if (rc) return rc;
    char* h = static_cast<char*>(ctx->hstage);
    std::memcpy(h, P.desc.data(), up);
    HIP_TRY(ctx, hipMemcpyAsync(base + P.off_desc, h, up, hipMemcpyHostToDevice, s));
    if (owners) {
        size_t ho = up;
        for (int l = 0; l < levels; ++l) {
            const size_t b = sizeof(int) * P.owner[l].size();
            std::memcpy(h + ho, P.owner[l].data(), b);
            HIP_TRY(ctx, hipMemcpyAsync(base + P.off_owner[l], h + ho, b, hipMemcpyHostToDevice, s));
            ho += b;
        }
        ctx->owners_key = key;
    }
    HIP_TRY(ctx, hipEventRecord(ctx->ev_upload, s));
    ctx->ev_pending = true;
    return ICP_OK;
}

hipEvent_t take_event(icp_ctx* ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Start a timed region on stream s (no-op unless timing is on).
int time_begin(icp_ctx* ctx, hipStream_t s, icp_ctx::EvRec& r, int kind, int64_t px) {
    r.kind = -1;
    if (!ctx->timing) return ICP_OK;
    r.a = take_event(ctx);
    r.b = take_event(ctx);
    if (!r.a || !r.b) return fail(ctx, ICP_EDEVICE, "hipEventCreate failed");
    HIP_TRY(ctx, hipEventRecord(r.a, s));
    r.kind = kind;
    r.px = px;
    return ICP_OK;
}

int time_end(icp_ctx* ctx, hipStream_t s, icp_ctx::EvRec& r) {
    if (r.kind < 0) return ICP_OK;
    HIP_TRY(ctx, hipEventRecord(r.b, s));
    ctx->pending.push_back(r);
    return ICP_OK;
}

int resolve_timing(icp_ctx* ctx) {
    for (auto& r : ctx->pending) {
        HIP_TRY(ctx, hipEventSynchronize(r.b));
        float ms = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, r.a, r.b));
        icp_kernel_time& t = ctx->times[r.kind];
        t.total_ms += ms;
        t.launches += 1;
        t.pixels += r.px;
        ctx->ev_pool.push_back(r.a);
        ctx->ev_pool.push_back(r.b);
    }
    ctx->pending.clear();
    return ICP_OK;
}

// Where the launches of a registration find their device data.
struct Launches {
    const ProbDesc* d_desc;
    int32_t* need2;                        // batch flag: some problem needs pass 2
    const int* owner[ICP_MAX_LEVELS];      // problem of every flat tile, per level
    int tiles[ICP_MAX_LEVELS];
    const int* max_vn;                     // largest launch sizes per level
    const int* max_mp;
    const int* max_q;
    int64_t px[ICP_MAX_LEVELS];            // pixels of all problems per level (kernel timing)
};

// Every launch of a registration of n problems on s, results into `res_dev`
// (device).  ctx may be NULL (no kernel timing, no error message).
int launch_registration(icp_ctx* ctx, int n, const icp_params* prm, const Launches& G, icp_result* res_dev,
                        hipStream_t s) {
    const ProbDesc* d_desc = G.d_desc;
    KParams kp = kparams(prm);
    kp.need2 = G.need2;
    int rc;
    icp_ctx::EvRec r;
    const bool timed = ctx && ctx->timing;
    auto begin = [&](int kind, int64_t px) { return timed ? time_begin(ctx, s, r, kind, px) : ICP_OK; };
    auto end = [&]() { return timed ? time_end(ctx, s, r) : ICP_OK; };
    if ((rc = begin(ICP_TIME_FRONT_END, G.px[0]))) return rc;
    HIP_TRY(ctx, icpk::launch_prepare(d_desc, n, prm->levels, G.max_vn, G.max_mp, G.max_q, false, front_end(prm),
                                      prm->use_imu_seed, kp.need2, s));
    if (prm->reduce_mode == 1) HIP_TRY(ctx, icpk::launch_centroid(d_desc, n, prm->levels, G.owner, G.tiles, s));
    if ((rc = end())) return rc;
    // single pass needs the band's lower edge at bin 0
    const int fused = prm->pass_mode == 0 && (!prm->use_median_filter || prm->band_beta >= 1.0) ? 1 : 0;
    // one problem in single-pass mode with the FP32 reduction: the band, pass 2
    // and the solve are one launch (k_band_pass2), two launches per iteration
    kp.fold_solve = fused && n == 1 && prm->reduce_mode == 0 ? 1 : 0;
    int gidx = 0;  // iterations so far, over all levels
    for (int l = prm->levels - 1; l >= 0; --l) {
        const int* owner = G.owner[l];
        const int64_t px = G.px[l];
        for (int it = 0; it < prm->iters[l]; ++it, ++gidx) {
            // (k_band_pass2 alternates the histogram and the window prediction)
            IterCtl ctl{l, it, it == prm->iters[l] - 1 ? 1 : 0, 0, kp.fold_solve ? gidx & 1 : 0};
            if ((rc = begin(ICP_TIME_PASS1, px))) return rc;
            HIP_TRY(ctx, icpk::launch_pass1(d_desc, owner, G.tiles[l], ctl, kp, fused, s));
            if ((rc = end())) return rc;
            if (kp.fold_solve) {
                if ((rc = begin(ICP_TIME_PASS2, px))) return rc;
                HIP_TRY(ctx, icpk::launch_band_pass2(d_desc, G.tiles[l], ctl, kp, s));
                if ((rc = end())) return rc;
                continue;
            }
            if ((rc = begin(ICP_TIME_BAND, 0))) return rc;
            HIP_TRY(ctx, icpk::launch_band(d_desc, n, ctl, kp, fused, s));
            if ((rc = end())) return rc;
            if ((rc = begin(ICP_TIME_PASS2, px))) return rc;
            HIP_TRY(ctx, icpk::launch_pass2(d_desc, owner, G.tiles[l], ctl, kp, s));
            if ((rc = end())) return rc;
            if ((rc = begin(ICP_TIME_SOLVE, 0))) return rc;
            HIP_TRY(ctx, icpk::launch_solve(d_desc, n, ctl, kp, s));
            if ((rc = end())) return rc;
        }
    }
    HIP_TRY(ctx, icpk::launch_finalize(d_desc, n, res_dev, s));
    return ICP_OK;
}

// Whole registration of a staged batch; results into `res_dev` (device).
int run_batch(icp_ctx* ctx, int n, const icp_params* prm, Plan& P, icp_result* res_dev, hipStream_t s) {
    char* base = static_cast<char*>(ctx->ws);
    Launches G{};
    G.d_desc = reinterpret_cast<const ProbDesc*>(base + P.off_desc);
    G.need2 = reinterpret_cast<int32_t*>(base + P.off_flags);
    for (int l = 0; l < prm->levels; ++l) {
        G.owner[l] = reinterpret_cast<const int*>(base + P.off_owner[l]);
        G.tiles[l] = P.tiles[l];
        for (int p = 0; p < n; ++p) G.px[l] += P.desc[p].lv[l].npx;
    }
    G.max_vn = P.max_vn;
    G.max_mp = P.max_mp;
    G.max_q = P.max_q;
    return launch_registration(ctx, n, prm, G, res_dev, s);
}

// Launch the whole registration of a staged batch on s, results into the
// workspace's result array.  Without timing, the launches are captured once
// per (plan, parameters, workspace) into a HIP graph and replayed; the context
// keeps the kGraphCache most recently used graphs (a frame server's batches
// cycle through a few shapes).
constexpr size_t kGraphCache = 8;

int execute(icp_ctx* ctx, int n, const icp_params* prm, Plan& P, hipStream_t s) {
    char* base = static_cast<char*>(ctx->ws);
    icp_result* d_res = reinterpret_cast<icp_result*>(base + P.off_res);
    if (!ctx->use_graphs || ctx->timing) return run_batch(ctx, n, prm, P, d_res, s);
    std::vector<int64_t> key = ctx->plan_key;
    key.push_back(reinterpret_cast<int64_t>(ctx->ws));
    const int64_t* pw = reinterpret_cast<const int64_t*>(prm);
    for (size_t k = 0; k < sizeof(icp_params) / sizeof(int64_t); ++k) key.push_back(pw[k]);
    icp_ctx::GraphEntry* hit = nullptr;
    for (auto& g : ctx->graphs)
        if (g.key == key) {
            hit = &g;
            break;
        }
    if (!hit) {
        if (ctx->graphs.size() >= kGraphCache) {
            // an asynchronous call may still be running the evicted graph: it
            // is destroyed only after the previous call's work has finished
            // (every earlier call's work is ordered before that)
            if (ctx->done_valid) HIP_TRY(ctx, hipEventSynchronize(ctx->ev_done));
            auto lru = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                        [](const auto& a, const auto& b) { return a.used < b.used; });
            destroy_graph(*lru);
            ctx->graphs.erase(lru);
        }
        if (!ctx->cap_stream) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        // (relaxed: allocations that other threads make meanwhile, such as a
        // frame server's clients, must not invalidate the capture; this
        // thread makes none until it ends)
        HIP_TRY(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
        int rc = run_batch(ctx, n, prm, P, d_res, ctx->cap_stream);
        icp_ctx::GraphEntry g;
        hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g.graph);
        if (rc || e != hipSuccess) {
            destroy_graph(g);
            // A device-wide call that another thread makes meanwhile (a
            // synchronisation, a free) can spoil a capture in progress.  This
            // call's launches then go straight to its stream (a genuine error
            // shows there again); the next call with this shape captures anew.
            (void)hipGetLastError();
            ctx->err.clear();
            return run_batch(ctx, n, prm, P, d_res, s);
        }
        e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            g.exec = nullptr;
            destroy_graph(g);
            return hip_fail(ctx, e, "hipGraphInstantiate");
        }
        g.key = std::move(key);
        ctx->graphs.push_back(std::move(g));
        hit = &ctx->graphs.back();
    }
    hit->used = ++ctx->graph_clock;
    HIP_TRY(ctx, hipGraphLaunch(hit->exec, s));
    return ICP_OK;
}

icp_problem one_problem(const float* depth, int W, int H, const float* mv, const float* mn, const icp_intrinsics* K,
                        const double* imu_R, const double* init_pose) {
    icp_problem q{};
    q.live_depth = depth;
    q.model_vtx = mv;
    q.model_nrm = mn;
    q.W = W;
    q.H = H;
    if (K) q.K = *K;
    for (int k = 0; k < 9; ++k) q.imu_R[k] = imu_R ? imu_R[k] : (k % 4 == 0 ? 1.0 : 0.0);
    for (int k = 0; k < 16; ++k) q.init_pose[k] = init_pose ? init_pose[k] : (k % 5 == 0 ? 1.0 : 0.0);
    return q;
}

// The device address of `scratch` on device `dev` (the current device): looked
// up with hipGetSymbolAddress once per device, with that device current, and
// kept.  Kernels take this address, never the array's host-side name.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) return ICP_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return ICP_EDEVICE;
        }
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return ICP_OK;
}

}  // namespace

extern "C" {

int icp_abi_version(void) { return ICP_ABI_VERSION; }

const char* icp_strerror(int code) {
    switch (code) {
        case ICP_OK: return "ok";
        case ICP_EINVAL: return "invalid argument";
        case ICP_ENOMEM: return "out of device memory or over the HBM budget";
        case ICP_EDEVICE: return "HIP runtime error";
        case ICP_ETIMEOUT: return "device-side wait timed out";
        default: return "unknown error";
    }
}

const char* icp_last_error(const icp_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

void icp_params_default(icp_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->levels = 3;
    p->iters[0] = 10;
    p->iters[1] = 5;
    p->iters[2] = 4;
    p->dist_max = 0.10;
    p->cos_angle_max = std::cos(20.0 * M_PI / 180.0);
    p->band_beta = 1.0;
    p->use_median_filter = 1;
    p->use_imu_seed = 1;
    p->lambda_mode = ICP_LAMBDA_CONST;
    p->lambda_c = 5.0;
    p->min_corr = 6;
    p->ill_cond_eps = 1e-12;
    p->converge_window = 0;
    p->reduce_mode = 0;
    p->depth_filter = 0;
    p->filter_radius = 3;
    p->filter_sigma_px = 4.5;
    p->filter_sigma_m = 0.05;
    p->normal_mode = 0;
    p->normal_radius = 2;
    p->anchor_to_imu = 0;
    p->reserved = 0;
}

int icp_validate_problem(const icp_problem* problem, const icp_params* params, char* msg, size_t msg_len) {
    icp_ctx tmp;  // holds the message only: no device state is touched
    int rc = problem ? check_params(&tmp, params) : fail(&tmp, ICP_EINVAL, "problem is NULL");
    if (rc == ICP_OK) rc = check_problem(&tmp, *problem, params->levels, params->use_imu_seed);
    if (msg && msg_len > 0) {
        const size_t n = std::min(msg_len - 1, tmp.err.size());
        std::memcpy(msg, tmp.err.data(), n);
        msg[n] = '\0';
    }
    return rc;
}

int icp_ctx_create(int device, size_t hbm_budget_bytes, icp_ctx** out) {
    if (!out) return ICP_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return ICP_EDEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return ICP_EDEVICE;
    icp_ctx* ctx = new icp_ctx();
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    if (hipEventCreateWithFlags(&ctx->ev_upload, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_done, hipEventDisableTiming) != hipSuccess) {
        if (ctx->ev_upload) (void)hipEventDestroy(ctx->ev_upload);
        delete ctx;
        return ICP_EDEVICE;
    }
    *out = ctx;
    return ICP_OK;
}

void icp_ctx_destroy(icp_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    const icpi::RelaxedCaptureScope relaxed;
    // this context's work has ended once its last call's event has (see
    // ensure_workspace); a context may die while another thread captures
    if (ctx->done_valid) (void)hipEventSynchronize(ctx->ev_done);
    if (ctx->ev_pending) (void)hipEventSynchronize(ctx->ev_upload);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->hstage) (void)hipHostFree(ctx->hstage);
    if (ctx->ev_upload) (void)hipEventDestroy(ctx->ev_upload);
    if (ctx->ev_done) (void)hipEventDestroy(ctx->ev_done);
    for (auto& r : ctx->pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    drop_graphs(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete static_cast<Plan*>(ctx->plan_mem);
    if (ctx->d_jobs) (void)hipFree(ctx->d_jobs);
    delete ctx;
}

int icp_ctx_set_graphs(icp_ctx* ctx, int enable) {
    if (!ctx) return ICP_EINVAL;
    ctx->use_graphs = enable != 0;
    return ICP_OK;
}

int icp_ctx_set_timing(icp_ctx* ctx, int enable) {
    if (!ctx) return ICP_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    int rc = resolve_timing(ctx);
    if (rc) return rc;
    ctx->timing = enable != 0;
    for (auto& t : ctx->times) t = icp_kernel_time{};
    return ICP_OK;
}

int icp_ctx_get_timing(icp_ctx* ctx, icp_kernel_time* out) {
    if (!ctx || !out) return ICP_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    int rc = resolve_timing(ctx);
    if (rc) return rc;
    for (int k = 0; k < ICP_TIME_KINDS; ++k) out[k] = ctx->times[k];
    return ICP_OK;
}

size_t icp_ctx_workspace_bytes(const icp_ctx* ctx) { return ctx ? ctx->ws_cap : 0; }

size_t icp_workspace_bytes(int n, const int32_t* W, const int32_t* H, int levels) {
    if (n < 1 || !W || !H || levels < 1 || levels > ICP_MAX_LEVELS) return 0;
    Plan P;
    make_plan(n, W, H, levels, nullptr, P);
    return P.total;
}

namespace {

// A batched registration queued on s, its n results copied to `results`
// (host memory when to_host, else device memory) by the stream; nothing waits.
int batch_submit(icp_ctx* ctx, int n, const icp_problem* probs, const icp_params* params, icp_result* results,
                 bool to_host, hipStream_t s) {
    if (n < 1 || !probs || !results) return fail(ctx, ICP_EINVAL, "empty batch or NULL array");
    if (n > 65535) return fail(ctx, ICP_EINVAL, "at most 65535 problems per batch");
    int rc = check_params(ctx, params);
    if (rc) return rc;
    for (int p = 0; p < n; ++p)
        if ((rc = check_problem(ctx, probs[p], params->levels, params->use_imu_seed))) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    StreamTurn turn;
    if (const int trc = turn.enter(ctx, s)) return trc;
    Plan& P = ctx_plan(ctx);
    if ((rc = stage_batch(ctx, n, probs, params->levels, params->tile_px, params->depth_filter, P, s))) return rc;
    ctx->stage_ready = false;
    if ((rc = execute(ctx, n, params, P, s))) return rc;
    icp_result* d_res = reinterpret_cast<icp_result*>(static_cast<char*>(ctx->ws) + P.off_res);
    HIP_TRY(ctx, hipMemcpyAsync(results, d_res, sizeof(icp_result) * n,
                                to_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
    return ICP_OK;
}

}  // namespace

int icp_register_batch(icp_ctx* ctx, int n, const icp_problem* probs, const icp_params* params, icp_result* results,
                       void* stream) {
    if (!ctx) return ICP_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = batch_submit(ctx, n, probs, params, results, true, s);
    if (rc) return rc;
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return resolve_timing(ctx);
}

int icp_register_batch_async(icp_ctx* ctx, int n, const icp_problem* probs, const icp_params* params,
                             icp_result* results_dev, void* stream) {
    if (!ctx) return ICP_EINVAL;
    return batch_submit(ctx, n, probs, params, results_dev, false, static_cast<hipStream_t>(stream));
}

int icp_autotune_tiles(icp_ctx* ctx, int n, const icp_problem* probs, const icp_params* params, int reps,
                       int32_t* tile_px_out, double* best_ms, void* stream) {
    if (!ctx) return ICP_EINVAL;
    if (n < 1 || !probs || !tile_px_out || reps < 1 || reps > 100)
        return fail(ctx, ICP_EINVAL, "autotune: empty batch, NULL output or reps outside 1..100");
    int rc = check_params(ctx, params);
    if (rc) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamTurn turn;
    if (const int trc = turn.enter(ctx, s)) return trc;
    std::vector<icp_result> res(n);
    icp_params p = *params;
    for (int l = 0; l < ICP_MAX_LEVELS; ++l)
        if (l >= p.levels) p.tile_px[l] = 0;
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(ctx, hipEventCreate(&a));
    HIP_TRY(ctx, hipEventCreate(&b));
    auto time_once = [&](const icp_params& q, double& ms) -> int {
        std::vector<double> t;
        int r = icp_register_batch(ctx, n, probs, &q, res.data(), stream);  // warm: plan, workspace, graph
        for (int k = 0; k < reps && r == ICP_OK; ++k) {
            if (hipEventRecord(a, s) != hipSuccess) return fail(ctx, ICP_EDEVICE, "hipEventRecord");
            r = icp_register_batch(ctx, n, probs, &q, res.data(), stream);
            if (r) break;
            if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess)
                return fail(ctx, ICP_EDEVICE, "hipEventSynchronize");
            float f = 0.0f;
            (void)hipEventElapsedTime(&f, a, b);
            t.push_back(f);
        }
        if (r) return r;
        std::sort(t.begin(), t.end());
        ms = t[t.size() / 2];
        return ICP_OK;
    };
    static const int kCand[] = {1024, 2048, 4096, 8192, 16384};
    double best = 0.0;
    for (int l = 0; l < p.levels && rc == ICP_OK; ++l) p.tile_px[l] = p.tile_px[l] ? p.tile_px[l] : 4096;
    for (int l = p.levels - 1; l >= 0 && rc == ICP_OK; --l) {
        int pick = p.tile_px[l];
        double pick_ms = 1e300;
        for (int c : kCand) {
            icp_params q = p;
            q.tile_px[l] = c;
            double ms = 0.0;
            if ((rc = time_once(q, ms))) break;
            if (ms < pick_ms) {
                pick_ms = ms;
                pick = c;
            }
        }
        p.tile_px[l] = pick;
        best = pick_ms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    for (int l = 0; l < ICP_MAX_LEVELS; ++l) tile_px_out[l] = l < p.levels ? p.tile_px[l] : 0;
    if (best_ms) *best_ms = best;
    return ICP_OK;
}

int icp_register(icp_ctx* ctx, const float* live_depth, int W, int H, const float* model_vtx,
                 const float* model_nrm, const icp_intrinsics* K, const double* imu_R, const double* init_pose,
                 const icp_params* params, double* pose_out, icp_stats* stats_out, void* stream) {
    if (!ctx) return ICP_EINVAL;
    if (!K || !imu_R || !init_pose || !pose_out) return fail(ctx, ICP_EINVAL, "NULL host argument");
    icp_problem q = one_problem(live_depth, W, H, model_vtx, model_nrm, K, imu_R, init_pose);
    icp_result r;
    int rc = icp_register_batch(ctx, 1, &q, params, &r, stream);
    if (rc) return rc;
    std::memcpy(pose_out, r.pose, sizeof(r.pose));
    if (stats_out) *stats_out = r.stats;
    return ICP_OK;
}

int icp_live_maps(icp_ctx* ctx, const float* depth, int W, int H, const icp_intrinsics* K, float* vtx, float* nrm,
                  void* stream) {
    if (!ctx) return ICP_EINVAL;
    if (!depth || !K || !vtx || !nrm) return fail(ctx, ICP_EINVAL, "NULL argument");
    if (W < 1 || H < 1 || W > ICP_MAX_DIM || H > ICP_MAX_DIM) return fail(ctx, ICP_EINVAL, "W and H must be in 1..8192");
    if (!(K->fx > 0 && K->fy > 0 && std::isfinite(K->fx) && std::isfinite(K->fy) && std::isfinite(K->cx) &&
          std::isfinite(K->cy)))
        return fail(ctx, ICP_EINVAL, "intrinsics must be finite with fx, fy > 0");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamTurn turn;
    if (const int trc = turn.enter(ctx, s)) return trc;
    if (!ctx->d_jobs) HIP_TRY(ctx, hipMalloc(&ctx->d_jobs, sizeof(MapsDesc)));
    int rc = ensure_stage(ctx, sizeof(MapsDesc));
    if (rc) return rc;
    MapsDesc* J = static_cast<MapsDesc*>(ctx->hstage);
    *J = MapsDesc{depth, vtx, nrm, W, H, K->fx, K->fy, K->cx, K->cy};
    HIP_TRY(ctx, hipMemcpyAsync(ctx->d_jobs, J, sizeof(MapsDesc), hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipEventRecord(ctx->ev_upload, s));
    ctx->ev_pending = true;
    HIP_TRY(ctx, icpk::launch_depth_to_maps(ctx->d_jobs, 1, icpk::live_vn_blocks(W, H), s));
    return ICP_OK;
}

namespace {

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_tsdf(icp_ctx* ctx, const icp_tsdf* vol, TsdfDesc* out) {
    if (!vol || !vol->voxels) return fail(ctx, ICP_EINVAL, "TSDF volume or its voxels is NULL");
    if (vol->dim < 2 || vol->dim > 1024) return fail(ctx, ICP_EINVAL, "TSDF dim must be in 2..1024");
    if (!finite_pos(vol->size) || !finite_pos(vol->mu) || !(std::isfinite(vol->max_weight) && vol->max_weight >= 1.0))
        return fail(ctx, ICP_EINVAL, "TSDF size and mu must be finite and > 0, max_weight finite and >= 1");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(vol->origin[a])) return fail(ctx, ICP_EINVAL, "TSDF origin must be finite");
    *out = TsdfDesc{vol->voxels, vol->dim, vol->size, {vol->origin[0], vol->origin[1], vol->origin[2]}, vol->mu,
                    vol->max_weight, vol->bricks};
    return ICP_OK;
}

int check_camera(icp_ctx* ctx, int W, int H, const icp_intrinsics* K, const double* T_wc, icpk::PoseArg* T) {
    if (!K || !T_wc) return fail(ctx, ICP_EINVAL, "NULL argument");
    if (W < 1 || H < 1 || W > ICP_MAX_DIM || H > ICP_MAX_DIM) return fail(ctx, ICP_EINVAL, "W and H must be in 1..8192");
    if (!(finite_pos(K->fx) && finite_pos(K->fy) && std::isfinite(K->cx) && std::isfinite(K->cy)))
        return fail(ctx, ICP_EINVAL, "intrinsics must be finite with fx, fy > 0");
    for (int i = 0; i < 12; ++i) {
        if (!std::isfinite(T_wc[i])) return fail(ctx, ICP_EINVAL, "T_wc must be finite");
        T->v[i] = T_wc[i];
    }
    if (!icpi::is_rotation(T_wc, 4))
        return fail(ctx, ICP_EINVAL, "T_wc's rotation is not a rotation (|R^T R - I| > 1e-6 or det R <= 0)");
    return ICP_OK;
}

}  // namespace

size_t icp_tsdf_bytes(int dim) {
    if (dim < 2 || dim > 1024) return 0;
    return (size_t)dim * dim * dim * 8;
}

size_t icp_tsdf_brick_bytes(int dim) {
    if (dim < 2 || dim > 1024) return 0;
    return icpk::tsdf_brick_bytes(dim);
}

int icp_tsdf_reset(icp_ctx* ctx, const icp_tsdf* vol, void* stream) {
    if (!ctx) return ICP_EINVAL;
    TsdfDesc d;
    int rc = check_tsdf(ctx, vol, &d);
    if (rc) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, icpk::launch_tsdf_fill(d, static_cast<hipStream_t>(stream)));
    return ICP_OK;
}

int icp_tsdf_integrate(icp_ctx* ctx, const icp_tsdf* vol, const float* depth, int W, int H, const icp_intrinsics* K,
                       const double* T_wc, void* stream) {
    if (!ctx) return ICP_EINVAL;
    TsdfDesc d;
    icpk::PoseArg T;
    int rc = check_tsdf(ctx, vol, &d);
    if (rc) return rc;
    if (!depth) return fail(ctx, ICP_EINVAL, "depth is NULL");
    rc = check_camera(ctx, W, H, K, T_wc, &T);
    if (rc) return rc;
    const double Kv[4] = {K->fx, K->fy, K->cx, K->cy};
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, icpk::launch_tsdf_integrate(d, depth, W, H, Kv, T, static_cast<hipStream_t>(stream)));
    return ICP_OK;
}

int icp_tsdf_raycast(icp_ctx* ctx, const icp_tsdf* vol, int W, int H, const icp_intrinsics* K, const double* T_wc,
                     double tmin, double tmax, float* vtx, float* nrm, void* stream) {
    if (!ctx) return ICP_EINVAL;
    TsdfDesc d;
    icpk::PoseArg T;
    int rc = check_tsdf(ctx, vol, &d);
    if (rc) return rc;
    if (!vtx || !nrm) return fail(ctx, ICP_EINVAL, "output map is NULL");
    rc = check_camera(ctx, W, H, K, T_wc, &T);
    if (rc) return rc;
    const double side = vol->size / (double)vol->dim;
    if (!(finite_pos(tmin) && std::isfinite(tmax) && tmax > tmin && (tmax - tmin) / (0.5 * side) <= 16777216.0))
        return fail(ctx, ICP_EINVAL, "need 0 < tmin < tmax and at most 2^24 ray steps");
    const double Kv[4] = {K->fx, K->fy, K->cx, K->cy};
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, icpk::launch_tsdf_raycast(d, tmin, tmax, W, H, Kv, T, vtx, nrm, static_cast<hipStream_t>(stream)));
    return ICP_OK;
}

int icp_register_async(icp_ctx* ctx, const float* live_depth, int W, int H, const float* model_vtx,
                       const float* model_nrm, const icp_intrinsics* K, const double* imu_R, const double* init_pose,
                       const icp_params* params, icp_result* result_dev, void* stream) {
    if (!ctx) return ICP_EINVAL;
    if (!K || !imu_R || !init_pose || !result_dev) return fail(ctx, ICP_EINVAL, "NULL argument");
    int rc = check_params(ctx, params);
    if (rc) return rc;
    icp_problem q = one_problem(live_depth, W, H, model_vtx, model_nrm, K, imu_R, init_pose);
    if ((rc = check_problem(ctx, q, params->levels, params->use_imu_seed))) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamTurn turn;
    if (const int trc = turn.enter(ctx, s)) return trc;
    Plan& P = ctx_plan(ctx);
    if ((rc = stage_batch(ctx, 1, &q, params->levels, params->tile_px, params->depth_filter, P, s))) return rc;
    ctx->stage_ready = false;
    if ((rc = execute(ctx, 1, params, P, s))) return rc;
    icp_result* d_res = reinterpret_cast<icp_result*>(static_cast<char*>(ctx->ws) + P.off_res);
    HIP_TRY(ctx, hipMemcpyAsync(result_dev, d_res, sizeof(icp_result), hipMemcpyDeviceToDevice, s));
    return ICP_OK;
}

int icp_register_noalloc(const float* live_depth, int W, int H, const float* model_vtx, const float* model_nrm,
                         const icp_intrinsics* K, const double* imu_R, const double* init_pose,
                         const icp_params* params, icp_result* result_dev, void* stream) {
    if (!K || !imu_R || !init_pose || !result_dev) return ICP_EINVAL;
    int rc = check_params(nullptr, params);
    if (rc) return rc;
    const icp_problem q = one_problem(live_depth, W, H, model_vtx, model_nrm, K, imu_R, init_pose);
    if ((rc = check_problem(nullptr, q, params->levels, params->use_imu_seed))) return rc;
    // layout in the static array (as a one-problem batch in a context's
    // workspace): descriptor, state, batch flag, level buffers, tile owners
    const int levels = params->levels;
    ProbDesc d{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const size_t off_desc = take(sizeof(ProbDesc));
    d.st = reinterpret_cast<ProbState*>(take(sizeof(ProbState)));
    const size_t off_flags = take(sizeof(int32_t));
    int tiles[ICP_MAX_LEVELS] = {}, max_vn[ICP_MAX_LEVELS] = {}, max_mp[ICP_MAX_LEVELS] = {},
        max_q[ICP_MAX_LEVELS] = {};
    int64_t level_px[ICP_MAX_LEVELS] = {};
    for (int l = 0; l < levels; ++l) level_px[l] = (int64_t)(W >> l) * (H >> l);
    lay_out_problem(d, W, H, levels, params->tile_px, 1, level_px, tiles, max_vn, max_mp, max_q, take);
    int max_tiles = 1;
    for (int l = 0; l < levels; ++l) max_tiles = std::max(max_tiles, tiles[l]);
    const size_t off_owner = take(sizeof(int32_t) * max_tiles);  // every tile belongs to problem 0
    if (off > kStaticScratchBytes) return ICP_ENOMEM;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return ICP_EDEVICE;
    }
    char* base = nullptr;
    if ((rc = static_scratch(dev, &base))) return rc;
    bind_problem(d, q, levels, params->depth_filter, base);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t* owner = reinterpret_cast<int32_t*>(base + off_owner);
    HIP_TRY(nullptr, icpk::launch_put_desc(d, reinterpret_cast<ProbDesc*>(base + off_desc), s));
    HIP_TRY(nullptr, icpk::launch_fill_i32(owner, max_tiles, 0, s));
    Launches G{};
    G.d_desc = reinterpret_cast<const ProbDesc*>(base + off_desc);
    G.need2 = reinterpret_cast<int32_t*>(base + off_flags);
    for (int l = 0; l < levels; ++l) {
        G.owner[l] = owner;
        G.tiles[l] = tiles[l];
        G.px[l] = d.lv[l].npx;
    }
    G.max_vn = max_vn;
    G.max_mp = max_mp;
    G.max_q = max_q;
    return launch_registration(nullptr, 1, params, G, result_dev, s);
}

// ------------------------------------------------------------------ stages

int icp_stage_prepare(icp_ctx* ctx, const float* live_depth, int W, int H, const float* model_vtx,
                      const float* model_nrm, const icp_intrinsics* K, int levels, const icp_params* params,
                      void* stream) {
    if (!ctx) return ICP_EINVAL;
    if (!K) return fail(ctx, ICP_EINVAL, "K is NULL");
    if (levels < 1 || levels > ICP_MAX_LEVELS) return fail(ctx, ICP_EINVAL, "levels must be in 1..4");
    icp_params dflt;
    icp_params_default(&dflt);
    const icp_params* prm = params ? params : &dflt;
    int rc = check_params(ctx, prm);
    if (rc) return rc;
    icp_problem q = one_problem(live_depth, W, H, model_vtx, model_nrm, K, nullptr, nullptr);
    if ((rc = check_problem(ctx, q, levels, 1))) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamTurn turn;
    if (const int trc = turn.enter(ctx, s)) return trc;
    Plan& P = ctx_plan(ctx);
    if ((rc = stage_batch(ctx, 1, &q, levels, nullptr, prm->depth_filter, P, s))) return rc;
    char* base = static_cast<char*>(ctx->ws);
    ctx->d_desc = reinterpret_cast<ProbDesc*>(base + P.off_desc);
    for (int l = 0; l < levels; ++l) {
        ctx->d_owner[l] = reinterpret_cast<int*>(base + P.off_owner[l]);
        ctx->tiles[l] = P.tiles[l];
    }
    ctx->d_state = reinterpret_cast<ProbState*>(base + P.off_state);
    ctx->d_scratch = reinterpret_cast<double*>(base + P.off_scratch);
    ctx->stage_desc = P.desc[0];
    ctx->stage_levels = levels;
    HIP_TRY(ctx, icpk::launch_prepare(ctx->d_desc, 1, levels, P.max_vn, P.max_mp, P.max_q, true,
                                      front_end(prm), 0, nullptr, s));
    HIP_TRY(ctx, icpk::launch_centroid(ctx->d_desc, 1, levels, ctx->d_owner, ctx->tiles, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    ctx->stage_ready = true;
    return ICP_OK;
}

static int stage_check(icp_ctx* ctx, int level) {
    if (!ctx) return ICP_EINVAL;
    if (!ctx->stage_ready) return fail(ctx, ICP_EINVAL, "no prepared stage problem (call icp_stage_prepare)");
    if (level < 0 || level >= ctx->stage_levels) return fail(ctx, ICP_EINVAL, "level out of range");
    return ICP_OK;
}

int icp_stage_level(icp_ctx* ctx, int level, float* depth, float* live_vtx, float* live_nrm, float* model_vtx,
                    float* model_nrm, void* stream) {
    int rc = stage_check(ctx, level);
    if (rc) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamTurn turn;
    if (const int trc = turn.enter(ctx, s)) return trc;
    const LevelDesc& L = ctx->stage_desc.lv[level];
    const size_t S = (size_t)L.npx * sizeof(float);
    if (depth) HIP_TRY(ctx, hipMemcpyAsync(depth, L.D, S, hipMemcpyDeviceToDevice, s));
    float* dst[2] = {live_vtx, live_nrm};
    const float* src[2] = {L.LV, L.LN};
    for (int m = 0; m < 2; ++m) {
        if (!dst[m]) continue;
        for (int c = 0; c < 3; ++c)  // planes are ps floats apart in the workspace, packed in the output
            HIP_TRY(ctx, hipMemcpyAsync(dst[m] + (size_t)c * L.npx, src[m] + (size_t)c * L.ps, S,
                                        hipMemcpyDeviceToDevice, s));
    }
    if (model_vtx) HIP_TRY(ctx, hipMemcpyAsync(model_vtx, L.MV, 3 * S, hipMemcpyDeviceToDevice, s));
    if (model_nrm) HIP_TRY(ctx, hipMemcpyAsync(model_nrm, L.MN, 3 * S, hipMemcpyDeviceToDevice, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return ICP_OK;
}

static icpk::PoseArg pose_arg(const double* pose12) {
    icpk::PoseArg a;
    std::memcpy(a.v, pose12, sizeof(a.v));
    return a;
}

int icp_stage_associate(icp_ctx* ctx, int level, const double* pose12, const icp_params* params, uint8_t* code,
                        int32_t* bin, uint32_t* hist, int64_t* band, void* stream) {
    int rc = stage_check(ctx, level);
    if (rc) return rc;
    if (!pose12) return fail(ctx, ICP_EINVAL, "pose12 is NULL");
    if ((rc = check_params(ctx, params))) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamTurn turn;
    if (const int trc = turn.enter(ctx, s)) return trc;
    const KParams kp = kparams(params);
    uint32_t* d_hist = reinterpret_cast<uint32_t*>(ctx->d_scratch);
    HIP_TRY(ctx, icpk::launch_stage_set(ctx->d_desc, pose_arg(pose12), 0, -1, level, -1, ICP_WIN / 2, s));
    IterCtl ctl{level, 0, 0, 0};
    HIP_TRY(ctx, icpk::launch_stage_pass1(ctx->d_desc, ctx->d_owner[level], ctx->tiles[level], ctl, kp, code, bin,
                                          d_hist, s));
    uint32_t hh[ICP_HIST_BINS];
    int32_t bandv[4];
    HIP_TRY(ctx, hipMemcpyAsync(hh, d_hist, sizeof(hh), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(bandv, &ctx->d_state->N, sizeof(bandv), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (hist) std::memcpy(hist, hh, sizeof(hh));
    if (band) {
        band[0] = (int64_t)(uint32_t)bandv[0];
        band[1] = bandv[1];
        band[2] = bandv[2];
        band[3] = bandv[3];
    }
    return ICP_OK;
}

int icp_stage_moments(icp_ctx* ctx, int level, const double* pose12, const icp_params* params, int k_lo, int k_hi,
                      double* moments, int64_t* n, void* stream) {
    int rc = stage_check(ctx, level);
    if (rc) return rc;
    if (!pose12 || !moments || !n) return fail(ctx, ICP_EINVAL, "NULL argument");
    if ((rc = check_params(ctx, params))) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamTurn turn;
    if (const int trc = turn.enter(ctx, s)) return trc;
    const KParams kp = kparams(params);
    HIP_TRY(ctx, icpk::launch_stage_set(ctx->d_desc, pose_arg(pose12), k_lo, k_hi, level, -1, ICP_WIN / 2, s));
    IterCtl ctl{level, 0, 0, 1};
    HIP_TRY(ctx, icpk::launch_stage_pass2(ctx->d_desc, ctx->d_owner[level], ctx->tiles[level], ctl, kp, s));
    HIP_TRY(ctx, hipMemcpyAsync(moments, ctx->d_state->M, sizeof(double) * ICP_NMOM, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(n, &ctx->d_state->n_last, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return ICP_OK;
}

int icp_stage_single_pass(icp_ctx* ctx, int level, const double* pose12, const icp_params* params, int iter,
                          int pred_hi, int pred_hw, int64_t* band, int32_t* window, int* hit, double* moments,
                          int64_t* n, void* stream) {
    int rc = stage_check(ctx, level);
    if (rc) return rc;
    if (!pose12 || !band || !window || !hit || !moments || !n) return fail(ctx, ICP_EINVAL, "NULL argument");
    if ((rc = check_params(ctx, params))) return rc;
    if (params->use_median_filter && params->band_beta < 1.0)
        return fail(ctx, ICP_EINVAL, "the single pass needs band_beta >= 1 (or no median filter)");
    if (iter < 0 || pred_hi < -1 || pred_hi >= ICP_HIST_BINS || (iter > 0 && (pred_hw < 1 || pred_hw > ICP_WIN / 2)))
        return fail(ctx, ICP_EINVAL, "iter >= 0, pred_hi in -1..1023 and (iter > 0) pred_hw in 1..24");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamTurn turn;
    if (const int trc = turn.enter(ctx, s)) return trc;
    const KParams kp = kparams(params);
    int32_t* d_win = reinterpret_cast<int32_t*>(ctx->d_scratch);
    HIP_TRY(ctx, icpk::launch_stage_set(ctx->d_desc, pose_arg(pose12), 0, -1, level, pred_hi,
                                        iter > 0 ? pred_hw : ICP_WIN / 2, s));
    IterCtl ctl{level, iter, 0, 1};
    HIP_TRY(ctx, icpk::launch_stage_single(ctx->d_desc, ctx->d_owner[level], ctx->tiles[level], ctl, kp, d_win, s));
    int32_t bandv[4], win[2], fused = 0;
    HIP_TRY(ctx, hipMemcpyAsync(bandv, &ctx->d_state->N, sizeof(bandv), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(win, d_win, sizeof(win), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(&fused, &ctx->d_state->fused_done, sizeof(fused), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(moments, ctx->d_state->M, sizeof(double) * ICP_NMOM, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(n, &ctx->d_state->n_last, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    band[0] = (int64_t)(uint32_t)bandv[0];
    band[1] = bandv[1];
    band[2] = bandv[2];
    band[3] = bandv[3];
    window[0] = win[0];
    window[1] = win[1];
    *hit = fused;
    if (!fused) {
        for (int k = 0; k < ICP_NMOM; ++k) moments[k] = 0.0;
        *n = 0;
    }
    return ICP_OK;
}

int icp_stage_solve(icp_ctx* ctx, const double* moments, int64_t n, const double* pose12_in, const icp_params* params,
                    double* pose12_out, double* x_out, int* status, void* stream) {
    if (!ctx) return ICP_EINVAL;
    if (!moments || !pose12_in || !pose12_out) return fail(ctx, ICP_EINVAL, "NULL argument");
    int rc = check_params(ctx, params);
    if (rc) return rc;
    if (params->anchor_to_imu) return fail(ctx, ICP_EINVAL, "the stage solve has no IMU prior: anchor_to_imu must be 0");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamTurn turn;
    if (const int trc = turn.enter(ctx, s)) return trc;
    if (!ctx->ws || ctx->ws_cap < kScratchBytes) {
        if ((rc = ensure_workspace(ctx, kScratchBytes))) return rc;
        ctx->stage_ready = false;
        ctx->d_scratch = static_cast<double*>(ctx->ws);
    }
    if (!ctx->stage_ready) ctx->d_scratch = static_cast<double*>(ctx->ws);
    icpk::MomArg M;
    std::memcpy(M.m, moments, sizeof(M.m));
    HIP_TRY(ctx, icpk::launch_stage_solve(M, n, pose_arg(pose12_in), kparams(params), ctx->d_scratch, s));
    double out[19];
    HIP_TRY(ctx, hipMemcpyAsync(out, ctx->d_scratch, sizeof(out), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    std::memcpy(pose12_out, out, 12 * sizeof(double));
    if (x_out) std::memcpy(x_out, out + 12, 6 * sizeof(double));
    if (status) *status = (int)out[18];
    return ICP_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ library-internal

namespace icpi {

int register_batch_async(icp_ctx* ctx, int n, const icp_problem* probs, const icp_params* params, icp_result* h_res,
                         hipStream_t s) {
    if (!ctx) return ICP_EINVAL;
    if (n < 1 || !probs || !h_res) return fail(ctx, ICP_EINVAL, "empty batch or NULL array");
    int rc = check_params(ctx, params);
    if (rc) return rc;
    for (int p = 0; p < n; ++p)
        if ((rc = check_problem(ctx, probs[p], params->levels, params->use_imu_seed))) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    Plan& P = ctx_plan(ctx);
    if ((rc = stage_batch(ctx, n, probs, params->levels, params->tile_px, params->depth_filter, P, s))) return rc;
    ctx->stage_ready = false;
    if ((rc = execute(ctx, n, params, P, s))) return rc;
    icp_result* d_res = reinterpret_cast<icp_result*>(static_cast<char*>(ctx->ws) + P.off_res);
    HIP_TRY(ctx, hipMemcpyAsync(h_res, d_res, sizeof(icp_result) * n, hipMemcpyDeviceToHost, s));
    return ICP_OK;
}

int reserve_workspace(icp_ctx* ctx, size_t bytes) {
    if (!ctx) return ICP_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    return ensure_workspace(ctx, bytes, true);
}

size_t workspace_bound(int n, const int32_t* W, const int32_t* H, int levels, const int32_t* tile_px) {
    if (n < 1 || !W || !H || levels < 1 || levels > ICP_MAX_LEVELS) return 0;
    int32_t req[ICP_MAX_LEVELS];
    for (int l = 0; l < ICP_MAX_LEVELS; ++l) req[l] = (tile_px && tile_px[l] > 0) ? tile_px[l] : ICP_TILE_QUANTUM;
    Plan P;
    make_plan(n, W, H, levels, req, P);
    return P.total;
}

int validate_params(icp_ctx* ctx, const icp_params* params) { return check_params(ctx, params); }

const char* error(icp_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

}  // namespace icpi
