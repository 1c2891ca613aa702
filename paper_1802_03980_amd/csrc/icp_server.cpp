// Frame server: frame-to-frame tracking of many camera streams on one GPU with
// continuous batching.
//
// Each open stream keeps its state on the device: a ring of R frame slots,
// each a depth image and its interleaved vertex / normal maps (the model of
// the stream's next frame).  Callers submit frames (host depth + the IMU
// rotation of the frame relative to the previous one); a scheduler thread
// forms a batch from every stream that has waiting frames and no batch on the
// GPU, oldest request first, taking up to R-1 consecutive frames of a stream,
// and launches it on one of `slots` HIP streams, each with its own context
// and workspace.  Frames that arrive while batches run wait for the next free
// slot, so with two slots one batch is staged and launched while the other is
// still on the GPU.  A batch uploads its depths, turns every depth into the
// maps of its ring slot, then registers every frame but a stream's first
// against the maps of the frame before it (in the same batch or an earlier,
// finished one).  Frame k lives in ring slot k mod R: the batch's frames and
// the maps they read occupy at most R distinct slots, and any older frame's
// slot is no longer read.  Results are taken with icp_server_poll.
//
// Streams are admitted against an HBM budget: the resident state of every
// open stream plus, per slot, the workspace of the largest batch the open
// streams can form.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "icp.h"
#include "icp_common.hpp"
#include "icp_internal.hpp"
#include "icp_launch.hpp"

namespace {

double clock_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t frame = 0;
    uint64_t tag = 0;
    double t_submit = 0.0;
    double prior[9] = {};
    float* depth = nullptr;  // pinned copy of the caller's depth, from the stream's pool
};

constexpr int kMaxRing = 8;

struct Stream {
    int id = -1;
    int W = 0, H = 0;
    icp_intrinsics K{};
    int ring = 2;                       // frame slots
    float* d_depth[kMaxRing] = {};      // depth of the frame in each slot, H x W
    float* d_mv[kMaxRing] = {};         // its vertex / normal maps, H x W x 3
    float* d_mn[kMaxRing] = {};
    size_t bytes = 0;                   // device bytes held
    bool in_flight = false;             // a batch with this stream's frames is on the GPU
    bool closing = false;
    uint64_t submitted = 0;
    double world[16] = {};     // pose of the last served frame in the stream's first camera
    std::deque<Request> pending;
    std::vector<float*> pool;  // free pinned depth buffers of this stream's size
};

struct Slot {
    icp_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    double t_start = 0.0;
    std::vector<Stream*> streams;  // batch order
    std::vector<Request> reqs;
    std::vector<int> reg;          // registration index per request, -1 for a stream's first frame
    std::vector<icp_problem> probs;
    icp_result* h_res = nullptr;   // pinned, max_batch entries
    MapsDesc* h_jobs = nullptr;    // pinned, max_batch entries
    MapsDesc* d_jobs = nullptr;
    size_t ws_reserved = 0;
};

void mat4_mul(const double* A, const double* B, double* C) {
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += A[4 * i + k] * B[4 * k + j];
            C[4 * i + j] = s;
        }
}

void eye4(double* T) {
    for (int k = 0; k < 16; ++k) T[k] = (k % 5 == 0) ? 1.0 : 0.0;
}

}  // namespace

struct icp_server {
    icp_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv_work;  // new request, new stream or stop
    std::condition_variable cv_done;  // new results
    std::thread worker;
    bool stop = false;
    int fatal = ICP_OK;  // a HIP failure of the scheduler: every later call reports it
    std::string err;
    std::vector<Stream*> streams;  // by id (nullptr once closed)
    std::vector<Slot> slots;
    std::deque<icp_server_result> done;
    size_t resident = 0;
    size_t ws_need = 0;  // per-slot workspace the open streams can require
    icp_server_counters ctr{};
};

namespace {

int srv_fail(icp_server* s, int code, const std::string& m) {
    s->err = m;
    return code;
}

// Workspace that any batch the given streams can form fits in: a batch holds
// up to frames_in_flight frames of each stream and at most max_batch frames,
// so the largest frames_in_flight copies of every stream, largest first, cut
// at max_batch, planned with the parameters' tiles or the smallest tile
// (a batch of fewer problems picks smaller tiles and so needs more partials).
size_t batch_workspace(const std::vector<Stream*>& ss, const icp_server_config& cfg) {
    std::vector<std::pair<int, int>> wh;
    for (Stream* st : ss)
        if (st && !st->closing)
            for (int f = 0; f < cfg.frames_in_flight; ++f) wh.push_back({st->W, st->H});
    if (wh.empty()) return 0;
    std::sort(wh.begin(), wh.end(), [](auto a, auto b) { return (long)a.first * a.second > (long)b.first * b.second; });
    if ((int)wh.size() > cfg.max_batch) wh.resize(cfg.max_batch);
    std::vector<int32_t> W, H;
    for (auto& p : wh) {
        W.push_back(p.first);
        H.push_back(p.second);
    }
    return icpi::workspace_bound((int)W.size(), W.data(), H.data(), cfg.params.levels, cfg.params.tile_px);
}

size_t stream_bytes(int W, int H, int ring) {
    const size_t px = (size_t)W * H;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    return (size_t)ring * (al(px * 4) + 2 * al(px * 12));
}

void free_stream(Stream* st) {
    const icpi::RelaxedCaptureScope relaxed;
    for (int r = 0; r < kMaxRing; ++r) {
        if (st->d_depth[r]) (void)hipFree(st->d_depth[r]);
        if (st->d_mv[r]) (void)hipFree(st->d_mv[r]);
        if (st->d_mn[r]) (void)hipFree(st->d_mn[r]);
    }
    for (float* p : st->pool) (void)hipHostFree(p);
    for (Request& r : st->pending)
        if (r.depth) (void)hipHostFree(r.depth);
    delete st;
}

// Publish the results of a finished batch (lock held).
void finish_slot(icp_server* S, Slot& sl) {
    const double t_done = clock_s();
    const int nb = (int)sl.reqs.size();
    for (int i = 0; i < nb; ++i) {
        Stream* st = sl.streams[i];
        Request& rq = sl.reqs[i];
        icp_server_result r{};
        r.stream_id = st->id;
        r.status = ICP_OK;
        r.frame = rq.frame;
        r.tag = rq.tag;
        r.t_submit = rq.t_submit;
        r.t_start = sl.t_start;
        r.t_done = t_done;
        r.batch_size = nb;
        if (sl.reg[i] >= 0) {
            const icp_result& g = sl.h_res[sl.reg[i]];
            std::memcpy(r.pose_rel, g.pose, sizeof(r.pose_rel));
            r.stats = g.stats;
            mat4_mul(st->world, r.pose_rel, r.pose_world);
        } else {
            eye4(r.pose_rel);
            eye4(r.pose_world);
        }
        std::memcpy(st->world, r.pose_world, sizeof(st->world));
        st->pool.push_back(rq.depth);
        S->done.push_back(r);
        S->ctr.frames += 1;
        if (sl.reg[i] >= 0) S->ctr.registrations += 1;
    }
    for (int i = 0; i < nb; ++i) {
        Stream* st = sl.streams[i];
        if (!st->in_flight) continue;  // already released (a stream appears once per frame)
        st->in_flight = false;
        if (st->closing && st->pending.empty()) {
            S->resident -= st->bytes;
            S->streams[st->id] = nullptr;
            free_stream(st);
        }
    }
    S->ctr.batches += 1;
    S->ctr.busy_s += t_done - sl.t_start;
    sl.busy = false;
    sl.reqs.clear();
    sl.streams.clear();
    S->cv_done.notify_all();
}

// Stage and launch the batch held in `sl` (lock not held: the streams in the
// batch are in flight, so nobody else touches their device state).
int launch_slot(icp_server* S, Slot& sl) {
    const int nb = (int)sl.reqs.size();
    const icp_params& prm = S->cfg.params;
    sl.probs.clear();
    sl.reg.assign(nb, -1);
    int max_blocks = 0;
    for (int i = 0; i < nb; ++i) {
        Stream* st = sl.streams[i];
        const Request& rq = sl.reqs[i];
        const int cur = (int)(rq.frame % st->ring);
        hipError_t e = hipMemcpyAsync(st->d_depth[cur], rq.depth, sizeof(float) * st->W * st->H,
                                      hipMemcpyHostToDevice, sl.stream);
        if (e != hipSuccess) return srv_fail(S, ICP_EDEVICE, std::string("depth upload: ") + hipGetErrorString(e));
        if (rq.frame > 0) {
            const int prev = (int)((rq.frame - 1) % st->ring);
            icp_problem q{};
            q.live_depth = st->d_depth[cur];
            q.W = st->W;
            q.H = st->H;
            q.model_vtx = st->d_mv[prev];
            q.model_nrm = st->d_mn[prev];
            q.K = st->K;
            std::memcpy(q.imu_R, rq.prior, sizeof(q.imu_R));
            eye4(q.init_pose);
            sl.reg[i] = (int)sl.probs.size();
            sl.probs.push_back(q);
        }
        sl.h_jobs[i] = MapsDesc{st->d_depth[cur], st->d_mv[cur], st->d_mn[cur], st->W, st->H,
                                st->K.fx,         st->K.fy,     st->K.cx,     st->K.cy};
        max_blocks = std::max(max_blocks, icpk::live_vn_blocks(st->W, st->H));
    }
    // the maps of every frame of the batch (the model of the frame after it), before the registrations read them
    hipError_t e = hipMemcpyAsync(sl.d_jobs, sl.h_jobs, sizeof(MapsDesc) * nb, hipMemcpyHostToDevice, sl.stream);
    if (e == hipSuccess) e = icpk::launch_depth_to_maps(sl.d_jobs, nb, max_blocks, sl.stream);
    if (e != hipSuccess) return srv_fail(S, ICP_EDEVICE, std::string("maps: ") + hipGetErrorString(e));
    if (!sl.probs.empty()) {
        int rc = icpi::register_batch_async(sl.ctx, (int)sl.probs.size(), sl.probs.data(), &prm, sl.h_res, sl.stream);
        if (rc) return srv_fail(S, rc, std::string("batch: ") + icpi::error(sl.ctx));
    }
    e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) return srv_fail(S, ICP_EDEVICE, std::string("event: ") + hipGetErrorString(e));
    return ICP_OK;
}

void scheduler(icp_server* S) {
    (void)hipSetDevice(S->cfg.device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // completions
        bool any_busy = false;
        for (Slot& sl : S->slots) {
            if (!sl.busy) continue;
            lk.unlock();
            const hipError_t q = hipEventQuery(sl.done);
            lk.lock();
            if (q == hipSuccess) {
                finish_slot(S, sl);
            } else if (q != hipErrorNotReady) {
                S->fatal = ICP_EDEVICE;
                S->err = std::string("batch failed: ") + hipGetErrorString(q);
                sl.busy = false;
                S->cv_done.notify_all();
            } else {
                any_busy = true;
            }
        }
        if (S->stop && !any_busy) break;
        // launch: one free slot, every stream with a waiting frame and none in flight
        Slot* free_slot = nullptr;
        for (Slot& sl : S->slots)
            if (!sl.busy) {
                free_slot = &sl;
                break;
            }
        std::vector<Stream*> ready;
        if (free_slot && !S->stop && S->fatal == ICP_OK)
            for (Stream* st : S->streams)
                if (st && !st->in_flight && !st->pending.empty()) ready.push_back(st);
        if (!ready.empty()) {
            std::sort(ready.begin(), ready.end(),
                      [](Stream* a, Stream* b) { return a->pending.front().t_submit < b->pending.front().t_submit; });
            if ((int)ready.size() > S->cfg.max_batch) ready.resize(S->cfg.max_batch);
            Slot& sl = *free_slot;
            sl.streams.clear();
            sl.reqs.clear();
            // one frame of every ready stream first, then more frames of the same
            // streams (up to ring-1 consecutive ones) while the batch has room
            for (int take = 0; take < kMaxRing && (int)sl.reqs.size() < S->cfg.max_batch; ++take)
                for (Stream* st : ready) {
                    if ((int)sl.reqs.size() >= S->cfg.max_batch) break;
                    if (take >= st->ring - 1 || st->pending.empty()) continue;
                    sl.streams.push_back(st);
                    sl.reqs.push_back(st->pending.front());
                    st->pending.pop_front();
                    st->in_flight = true;
                }
            // keep each stream's frames consecutive and in order
            std::vector<size_t> ord(sl.reqs.size());
            for (size_t q = 0; q < ord.size(); ++q) ord[q] = q;
            std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
                if (sl.streams[a] != sl.streams[b]) return sl.streams[a]->id < sl.streams[b]->id;
                return sl.reqs[a].frame < sl.reqs[b].frame;
            });
            std::vector<Stream*> s2;
            std::vector<Request> r2;
            for (size_t q : ord) {
                s2.push_back(sl.streams[q]);
                r2.push_back(sl.reqs[q]);
            }
            sl.streams.swap(s2);
            sl.reqs.swap(r2);
            sl.busy = true;
            sl.t_start = clock_s();
            const size_t need = S->ws_need;
            lk.unlock();
            int rc = ICP_OK;
            if (need > sl.ws_reserved) {
                rc = icpi::reserve_workspace(sl.ctx, need);
                if (rc == ICP_OK) sl.ws_reserved = need;
                else srv_fail(S, rc, std::string("workspace: ") + icpi::error(sl.ctx));
            }
            if (rc == ICP_OK) rc = launch_slot(S, sl);
            lk.lock();
            if (rc != ICP_OK) {
                // nothing of this batch reached the GPU in a usable state: report it per frame
                S->fatal = rc;
                const double t = clock_s();
                for (size_t i = 0; i < sl.reqs.size(); ++i) {
                    icp_server_result r{};
                    r.stream_id = sl.streams[i]->id;
                    r.status = rc;
                    r.frame = sl.reqs[i].frame;
                    r.tag = sl.reqs[i].tag;
                    r.t_submit = sl.reqs[i].t_submit;
                    r.t_start = r.t_done = t;
                    S->done.push_back(r);
                }
                lk.unlock();
                (void)hipStreamSynchronize(sl.stream);
                lk.lock();
                for (size_t i = 0; i < sl.reqs.size(); ++i) {
                    sl.streams[i]->in_flight = false;
                    sl.streams[i]->pool.push_back(sl.reqs[i].depth);
                }
                sl.busy = false;
                sl.reqs.clear();
                sl.streams.clear();
                S->cv_done.notify_all();
            }
            continue;
        }
        if (any_busy) {
            // a batch is on the GPU: look again shortly (or when a frame arrives)
            S->cv_work.wait_for(lk, std::chrono::microseconds(20));
        } else {
            S->cv_work.wait(lk);
        }
    }
}

}  // namespace

extern "C" {

void icp_server_config_default(icp_server_config* cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->device = 0;
    cfg->max_batch = 64;
    cfg->slots = 2;
    cfg->use_graphs = 1;
    cfg->frames_in_flight = 2;
    cfg->hbm_budget_bytes = 0;
    icp_params_default(&cfg->params);
}

double icp_server_clock(void) { return clock_s(); }

int icp_server_create(const icp_server_config* cfg, icp_server** out) {
    if (!cfg || !out) return ICP_EINVAL;
    *out = nullptr;
    if (cfg->max_batch < 1 || cfg->max_batch > 4096 || cfg->slots < 1 || cfg->slots > 4 ||
        cfg->frames_in_flight < 1 || cfg->frames_in_flight > kMaxRing - 1)
        return ICP_EINVAL;
    icp_server* S = new icp_server();
    S->cfg = *cfg;
    S->slots.resize(cfg->slots);
    int rc = ICP_OK;
    for (Slot& sl : S->slots) {
        if ((rc = icp_ctx_create(cfg->device, 0, &sl.ctx)) != ICP_OK) break;
        icp_ctx_set_graphs(sl.ctx, cfg->use_graphs);
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(&sl.h_res, sizeof(icp_result) * cfg->max_batch) != hipSuccess ||
            hipHostMalloc(&sl.h_jobs, sizeof(MapsDesc) * cfg->max_batch) != hipSuccess ||
            hipMalloc(&sl.d_jobs, sizeof(MapsDesc) * cfg->max_batch) != hipSuccess) {
            rc = ICP_EDEVICE;
            break;
        }
    }
    if (rc == ICP_OK) rc = icpi::validate_params(S->slots[0].ctx, &cfg->params);
    // the served model maps are built with the default front end, so the live frames must be too
    if (rc == ICP_OK && (cfg->params.depth_filter != 0 || cfg->params.normal_mode != 0)) rc = ICP_EINVAL;
    if (rc != ICP_OK) {
        for (Slot& sl : S->slots) {
            if (sl.ctx) icp_ctx_destroy(sl.ctx);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.h_res) (void)hipHostFree(sl.h_res);
            if (sl.h_jobs) (void)hipHostFree(sl.h_jobs);
            if (sl.d_jobs) (void)hipFree(sl.d_jobs);
        }
        delete S;
        return rc;
    }
    S->worker = std::thread(scheduler, S);
    *out = S;
    return ICP_OK;
}

void icp_server_destroy(icp_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();  // in-flight batches finish first
    (void)hipSetDevice(S->cfg.device);
    for (Slot& sl : S->slots) {
        (void)hipStreamSynchronize(sl.stream);
        icp_ctx_destroy(sl.ctx);
        (void)hipStreamDestroy(sl.stream);
        (void)hipEventDestroy(sl.done);
        (void)hipHostFree(sl.h_res);
        (void)hipHostFree(sl.h_jobs);
        (void)hipFree(sl.d_jobs);
        for (Request& r : sl.reqs)
            if (r.depth) (void)hipHostFree(r.depth);
    }
    for (Stream* st : S->streams)
        if (st) free_stream(st);
    delete S;
}

const char* icp_server_last_error(icp_server* S) { return S ? S->err.c_str() : ""; }

int icp_server_open_stream(icp_server* S, int W, int H, const icp_intrinsics* K, int* stream_id) {
    if (!S || !K || !stream_id) return ICP_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fatal) return S->fatal;
    const int div = 1 << (S->cfg.params.levels - 1);
    if (W < 1 || H < 1 || W > ICP_MAX_DIM || H > ICP_MAX_DIM || W % div || H % div)
        return srv_fail(S, ICP_EINVAL, "W and H must be in 1..8192 and divisible by 2^(levels-1)");
    if (!(K->fx > 0 && K->fy > 0 && std::isfinite(K->fx) && std::isfinite(K->fy) && std::isfinite(K->cx) &&
          std::isfinite(K->cy)))
        return srv_fail(S, ICP_EINVAL, "intrinsics must be finite with fx, fy > 0");
    Stream* st = new Stream();
    st->W = W;
    st->H = H;
    st->K = *K;
    st->ring = S->cfg.frames_in_flight + 1;
    st->bytes = stream_bytes(W, H, st->ring);
    eye4(st->world);
    // admission: resident state of all streams + per-slot workspace of the largest batch
    std::vector<Stream*> with = S->streams;
    with.push_back(st);
    const size_t ws = batch_workspace(with, S->cfg);
    const size_t need = S->resident + st->bytes + ws * S->slots.size();
    if (S->cfg.hbm_budget_bytes && need > S->cfg.hbm_budget_bytes) {
        delete st;
        return srv_fail(S, ICP_ENOMEM,
                        "stream not admitted: " + std::to_string(need) + " bytes needed, budget " +
                            std::to_string(S->cfg.hbm_budget_bytes));
    }
    (void)hipSetDevice(S->cfg.device);
    const icpi::RelaxedCaptureScope relaxed;
    const size_t px = (size_t)W * H;
    for (int r = 0; r < st->ring; ++r)
        if (hipMalloc(&st->d_depth[r], px * 4) != hipSuccess || hipMalloc(&st->d_mv[r], px * 12) != hipSuccess ||
            hipMalloc(&st->d_mn[r], px * 12) != hipSuccess) {
            (void)hipGetLastError();
            free_stream(st);
            return srv_fail(S, ICP_ENOMEM, "device allocation of the stream state failed");
        }
    st->id = (int)S->streams.size();
    S->streams.push_back(st);
    S->resident += st->bytes;
    S->ws_need = std::max(S->ws_need, ws);
    *stream_id = st->id;
    return ICP_OK;
}

int icp_server_close_stream(icp_server* S, int id) {
    if (!S) return ICP_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (id < 0 || id >= (int)S->streams.size() || !S->streams[id]) return srv_fail(S, ICP_EINVAL, "unknown stream");
    Stream* st = S->streams[id];
    st->closing = true;
    if (!st->in_flight && st->pending.empty()) {
        S->resident -= st->bytes;
        S->streams[id] = nullptr;
        free_stream(st);
    }
    // the per-slot workspace already reserved stays; admission counts the streams left
    S->ws_need = batch_workspace(S->streams, S->cfg);
    return ICP_OK;
}

int icp_server_submit(icp_server* S, int id, const float* depth_host, const double* imu_rel_R, uint64_t tag,
                      double t_submit) {
    if (!S || !depth_host || !imu_rel_R) return ICP_EINVAL;
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(imu_rel_R[k])) return srv_fail(S, ICP_EINVAL, "imu_rel_R not finite");
    if (!icpi::is_rotation(imu_rel_R, 3))
        return srv_fail(S, ICP_EINVAL, "imu_rel_R is not a rotation (|R^T R - I| > 1e-6 or det R <= 0)");
    float* buf = nullptr;
    size_t bytes = 0;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->fatal) return S->fatal;
        if (id < 0 || id >= (int)S->streams.size() || !S->streams[id] || S->streams[id]->closing)
            return srv_fail(S, ICP_EINVAL, "unknown or closing stream");
        Stream* st = S->streams[id];
        bytes = sizeof(float) * st->W * st->H;
        if (!st->pool.empty()) {
            buf = st->pool.back();
            st->pool.pop_back();
        }
    }
    if (!buf) {
        (void)hipSetDevice(S->cfg.device);
        const icpi::RelaxedCaptureScope relaxed;
        if (hipHostMalloc(&buf, bytes) != hipSuccess) return srv_fail(S, ICP_ENOMEM, "pinned depth buffer");
    }
    std::memcpy(buf, depth_host, bytes);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        Stream* st = (id < (int)S->streams.size()) ? S->streams[id] : nullptr;
        if (!st || st->closing) {
            const icpi::RelaxedCaptureScope relaxed;
            (void)hipHostFree(buf);
            return srv_fail(S, ICP_EINVAL, "stream closed during submit");
        }
        Request r;
        r.frame = st->submitted++;
        r.tag = tag;
        r.t_submit = t_submit > 0.0 ? t_submit : clock_s();
        std::memcpy(r.prior, imu_rel_R, sizeof(r.prior));
        r.depth = buf;
        st->pending.push_back(r);
    }
    S->cv_work.notify_one();
    return ICP_OK;
}

int icp_server_poll(icp_server* S, icp_server_result* out, int max, int timeout_ms) {
    if (!S || !out || max < 1) return ICP_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->done.empty() && timeout_ms != 0) {
        auto pred = [&] { return !S->done.empty() || S->fatal != ICP_OK; };
        if (timeout_ms < 0) S->cv_done.wait(lk, pred);
        else S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
    }
    int n = 0;
    while (n < max && !S->done.empty()) {
        out[n++] = S->done.front();
        S->done.pop_front();
    }
    if (n == 0 && S->fatal) return S->fatal;
    return n;
}

int icp_server_get_counters(icp_server* S, icp_server_counters* out) {
    if (!S || !out) return ICP_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->ctr;
    out->resident_bytes = S->resident;
    out->workspace_bytes = S->ws_need * S->slots.size();
    out->workspace_held_bytes = 0;
    for (const Slot& sl : S->slots) out->workspace_held_bytes += icp_ctx_workspace_bytes(sl.ctx);
    int open = 0;
    for (Stream* st : S->streams)
        if (st) ++open;
    out->streams_open = open;
    return ICP_OK;
}

}  // extern "C"
