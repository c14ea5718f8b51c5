// Served form: a request loop that admits max-flow solves by HBM budget as
// they arrive and runs them with continuous batching.
//
//  - mf_server_submit copies the request to the host queue and returns a
//    ticket at once.
//  - A worker thread admits requests in arrival order while the device
//    region (one allocation of the budget's size, carved by a best-fit
//    allocator) and the in-flight limit allow, copies the graph to its
//    slice by DMA and publishes it to the queue of its lane count, in
//    coherent host memory.
//  - One persistent kernel per lane count keeps taking published requests
//    (one workgroup per request: residency checks, both phases, outputs)
//    while it runs; a request that arrives while others are on the GPU joins
//    the running kernel as soon as a workgroup is free.  A kernel that finds
//    no work for idle_ms leaves; the worker starts it again when requests
//    arrive.
//  - Finished requests are copied back, their device slice is freed, and
//    mf_server_poll / mf_server_wait return them.
// Graphs and residual state stay in device memory for the whole solve.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mf_host.h"

namespace {

using Clock = std::chrono::steady_clock;

// Best-fit allocator over one device region.
class RegionAllocator {
  public:
    void init(size_t size)
    {
        free_.clear();
        free_[0] = size;
        size_ = size;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = align256(bytes);
        auto best = free_.end();
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes && (best == free_.end() || it->second < best->second)) best = it;
        if (best == free_.end()) return false;
        off = best->first;
        const size_t rest = best->second - bytes;
        free_.erase(best);
        if (rest) free_[off + bytes] = rest;
        used_ += bytes;
        return true;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align256(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

enum ReqState { PENDING, PUBLISHED, COMPLETE };

struct Request {
    uint64_t ticket = 0;
    int32_t n = 0, s = 0, t = 0;
    int64_t S = 0;
    std::vector<int64_t> off, rev;
    std::vector<int32_t> head, cap;
    mf_options opt;
    bool want_flow = false;
    bool canceled = false;
    int G = 4, queue = 0;
    int32_t index = -1;          // position in its queue
    size_t bytes = 0, region_off = 0;
    InstLayout lay;
    ReqState state = PENDING;
    Clock::time_point t_submit, t_done;
    mf_result result;
    std::vector<int32_t> flow;
    std::vector<uint8_t> side;
};

// Slice of one request: the instance layout, then the int64 offsets and
// reverse slots as received, then the five control blocks.
size_t staging_rev(int64_t n) { return align256(8 * (size_t)(n + 1)); }
size_t staging_ctl(int64_t n, int64_t S) { return staging_rev(n) + align256(8 * (size_t)std::max<int64_t>(S, 1)); }

size_t request_bytes(int64_t n, int64_t S, bool want_flow)
{
    InstLayout L = layout_for(0, n, S, want_flow);
    return L.end + staging_ctl(n, S) + align256(5 * sizeof(Ctl));
}

}  // namespace

struct mf_server {
    mf_context *ctx = nullptr;
    mf_server_config cfg;
    uint8_t *region = nullptr;
    RegionAllocator alloc;
    ServeHostQueue *hq[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t *next_d = nullptr;       // [4] device counters
    int32_t published[4] = {0, 0, 0, 0};
    hipStream_t kstream[4] = {nullptr, nullptr, nullptr, nullptr};
    hipStream_t copy = nullptr;
    uint64_t idle_ticks = 0;
    int grid[4] = {0, 0, 0, 0};

    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    std::atomic<bool> stop{false};
    uint64_t next_ticket = 1;
    std::deque<Request *> pending;
    std::unordered_map<uint64_t, Request *> reqs;
    std::vector<Request *> inflight_list;
    std::vector<Request *> slot_owner[4];
    mf_server_stats st;
    std::string err;
};

static void server_loop(mf_server *sv);

extern "C" mf_status mf_server_create(mf_context *ctx, const mf_server_config *cfg, mf_server **out)
{
    if (!ctx || !out) return fail(ctx, MF_EINVAL, "NULL argument");
    *out = nullptr;
    mf_server *sv = new (std::nothrow) mf_server();
    if (!sv) return fail(ctx, MF_ENOMEM, "host allocation failed");
    sv->ctx = ctx;
    memset(&sv->cfg, 0, sizeof sv->cfg);
    if (cfg) sv->cfg = *cfg;
    if (sv->cfg.hbm_budget_bytes == 0) sv->cfg.hbm_budget_bytes = (size_t)64 << 30;
    if (sv->cfg.max_inflight <= 0 || sv->cfg.max_inflight > SERVE_CAP) sv->cfg.max_inflight = SERVE_CAP;
    if (sv->cfg.idle_ms <= 0) sv->cfg.idle_ms = 20;
    memset(&sv->st, 0, sizeof sv->st);
    auto bail = [&](mf_status s, const char *what) {
        mf_server_destroy(sv);
        return fail(ctx, s, "%s", what);
    };
    if (hipSetDevice(ctx->device) != hipSuccess) return bail(MF_EDEVICE, "hipSetDevice failed");
    mf_status ms = dalloc(ctx, (void **)&sv->region, sv->cfg.hbm_budget_bytes);
    if (ms != MF_OK) {
        std::string e = ctx->err;
        mf_server_destroy(sv);
        return fail(ctx, ms, "server region: %s", e.c_str());
    }
    sv->alloc.init(sv->cfg.hbm_budget_bytes);
    for (int q = 0; q < 4; q++) {
        if (hipHostMalloc((void **)&sv->hq[q], sizeof(ServeHostQueue), hipHostMallocCoherent) != hipSuccess)
            return bail(MF_ENOMEM, "pinned queue allocation failed");
        memset(sv->hq[q], 0, sizeof(ServeHostQueue));
        if (hipStreamCreateWithFlags(&sv->kstream[q], hipStreamNonBlocking) != hipSuccess)
            return bail(MF_EDEVICE, "stream creation failed");
        int per_cu = serve_blocks_per_cu(4 << q);
        if (per_cu <= 0) per_cu = 1;
        if (sv->cfg.blocks_per_cu > 0) per_cu = std::min(per_cu, (int)sv->cfg.blocks_per_cu);
        sv->grid[q] = per_cu * ctx->num_cus;
    }
    if (hipStreamCreateWithFlags(&sv->copy, hipStreamNonBlocking) != hipSuccess)
        return bail(MF_EDEVICE, "stream creation failed");
    if (hipMalloc((void **)&sv->next_d, 4 * sizeof(int32_t)) != hipSuccess ||
        hipMemset(sv->next_d, 0, 4 * sizeof(int32_t)) != hipSuccess)
        return bail(MF_EDEVICE, "device counter allocation failed");
    sv->idle_ticks = ctx->wall_hz / 1000ull * (uint64_t)sv->cfg.idle_ms;
    for (int q = 0; q < 4; q++) sv->slot_owner[q].assign(SERVE_CAP, nullptr);
    sv->worker = std::thread(server_loop, sv);
    *out = sv;
    return MF_OK;
}

extern "C" void mf_server_destroy(mf_server *sv)
{
    if (!sv) return;
    if (sv->worker.joinable()) {
        sv->stop = true;
        sv->cv.notify_all();
        sv->worker.join();
    }
    (void)hipSetDevice(sv->ctx->device);
    for (int q = 0; q < 4; q++)
        if (sv->hq[q]) __atomic_store_n(&sv->hq[q]->shutdown, 1, __ATOMIC_RELEASE);
    for (int q = 0; q < 4; q++)
        if (sv->kstream[q]) {
            (void)hipStreamSynchronize(sv->kstream[q]);
            (void)hipStreamDestroy(sv->kstream[q]);
        }
    if (sv->copy) {
        (void)hipStreamSynchronize(sv->copy);
        (void)hipStreamDestroy(sv->copy);
    }
    for (int q = 0; q < 4; q++)
        if (sv->hq[q]) (void)hipHostFree(sv->hq[q]);
    if (sv->next_d) (void)hipFree(sv->next_d);
    if (sv->region) dfree(sv->ctx, sv->region, sv->cfg.hbm_budget_bytes);
    for (auto &kv : sv->reqs) delete kv.second;
    delete sv;
}

extern "C" mf_status mf_server_submit(mf_server *sv, const mf_graph *g, const mf_options *opt, int want_flow,
                                      uint64_t *ticket)
{
    if (!sv || !g || !ticket) return MF_EINVAL;
    mf_options o;
    if (opt) o = *opt; else mf_options_default(&o);
    Request *r = new (std::nothrow) Request();
    if (!r) return MF_ENOMEM;
    r->n = g->n;
    r->s = g->s;
    r->t = g->t;
    r->S = g->slots;
    r->opt = o;
    r->want_flow = want_flow != 0 && !(o.flags & MF_PREFLOW_ONLY);
    memset(&r->result, 0, sizeof r->result);
    const bool shape_ok = g->n >= 2 && g->slots >= 0 && g->slots < 2147483647LL &&
                          (int64_t)g->n + g->slots < 2147483647LL && g->s >= 0 && g->s < g->n && g->t >= 0 &&
                          g->t < g->n && g->s != g->t && g->offsets && (g->slots == 0 || (g->head && g->rev && g->cap)) &&
                          o.gr_freq_den > 0 && o.gr_freq_num >= 0 && o.gr_alpha >= 0 && o.gr_beta >= 0 &&
                          o.gr_round_charge >= 0 && o.max_rounds >= 0;
    if (shape_ok) {
        r->off.assign(g->offsets, g->offsets + g->n + 1);
        r->rev.assign(g->rev, g->rev + g->slots);
        r->head.assign(g->head, g->head + g->slots);
        r->cap.assign(g->cap, g->cap + g->slots);
        r->G = batch_lanes(o.lanes_per_vertex, g->n, g->slots);
        r->queue = r->G == 4 ? 0 : r->G == 8 ? 1 : r->G == 16 ? 2 : 3;
        r->bytes = request_bytes(g->n, g->slots, r->want_flow);
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    r->ticket = sv->next_ticket++;
    r->t_submit = Clock::now();
    sv->reqs[r->ticket] = r;
    sv->st.submitted++;
    if (!shape_ok || r->bytes > sv->cfg.hbm_budget_bytes) {
        r->result.status = shape_ok ? MF_ENOMEM : MF_EINVAL;
        r->state = COMPLETE;
        r->t_done = Clock::now();
        sv->st.rejected++;
    } else {
        sv->pending.push_back(r);
    }
    *ticket = r->ticket;
    sv->cv.notify_all();
    return MF_OK;
}

static void take_outputs(Request *r, mf_result *out, int32_t *flow, uint8_t *side)
{
    if (out) {
        *out = r->result;
        out->ms_latency = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    }
    if (flow && !r->flow.empty()) memcpy(flow, r->flow.data(), 4 * r->flow.size());
    if (side && !r->side.empty()) memcpy(side, r->side.data(), r->side.size());
}

extern "C" mf_status mf_server_poll(mf_server *sv, uint64_t ticket, mf_result *out, int32_t *flow, uint8_t *side)
{
    if (!sv) return MF_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return MF_ENOTFOUND;
    Request *r = it->second;
    if (r->state != COMPLETE) return MF_EAGAIN;
    take_outputs(r, out, flow, side);
    sv->reqs.erase(it);
    delete r;
    return MF_OK;
}

extern "C" mf_status mf_server_wait(mf_server *sv, uint64_t ticket, int64_t timeout_ms, mf_result *out,
                                    int32_t *flow, uint8_t *side)
{
    if (!sv) return MF_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    const auto deadline = Clock::now() + std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms);
    while (true) {
        auto it = sv->reqs.find(ticket);
        if (it == sv->reqs.end()) return MF_ENOTFOUND;
        Request *r = it->second;
        if (r->state == COMPLETE) {
            take_outputs(r, out, flow, side);
            sv->reqs.erase(it);
            delete r;
            return MF_OK;
        }
        if (timeout_ms >= 0 && Clock::now() >= deadline) return MF_EAGAIN;
        if (timeout_ms >= 0)
            sv->cv.wait_until(lk, deadline);
        else
            sv->cv.wait(lk);
    }
}

extern "C" mf_status mf_server_cancel(mf_server *sv, uint64_t ticket)
{
    if (!sv) return MF_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return MF_ENOTFOUND;
    Request *r = it->second;
    if (r->state == COMPLETE) return MF_OK;
    r->canceled = true;
    if (r->state == PENDING) {
        for (auto p = sv->pending.begin(); p != sv->pending.end(); ++p)
            if (*p == r) {
                sv->pending.erase(p);
                break;
            }
        r->result.status = MF_ECANCELED;
        r->state = COMPLETE;
        r->t_done = Clock::now();
        sv->st.canceled++;
        sv->cv.notify_all();
    }
    return MF_OK;
}

extern "C" mf_status mf_server_get_stats(mf_server *sv, mf_server_stats *out)
{
    if (!sv || !out) return MF_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->st;
    out->inflight = (int64_t)sv->inflight_list.size();
    out->queued = (int64_t)sv->pending.size();
    out->bytes_in_use = sv->alloc.used();
    return MF_OK;
}

// ---------------------------------------------------------------------------
// Worker

// Copies the graph to its slice and publishes the request.  Called with the
// lock held; the copies are synchronous on the copy stream.
static bool admit(mf_server *sv, Request *r)
{
    size_t off;
    if ((int)sv->inflight_list.size() >= sv->cfg.max_inflight) return false;
    const int q = r->queue;
    // the ring slot of this queue must be free
    const int32_t index = sv->published[q];
    if (sv->slot_owner[q][index % SERVE_CAP]) return false;
    if (!sv->alloc.alloc(r->bytes, off)) return false;
    r->region_off = off;
    uint8_t *base = sv->region + off;
    r->lay = layout_for(0, r->n, r->S, r->want_flow);
    const InstLayout &L = r->lay;
    int64_t *off64 = (int64_t *)(base + L.end);
    int64_t *rev64 = (int64_t *)(base + L.end + staging_rev(r->n));
    const size_t S = (size_t)r->S, N = (size_t)r->n;
    hipError_t e = hipMemcpyAsync(off64, r->off.data(), 8 * (N + 1), hipMemcpyHostToDevice, sv->copy);
    if (e == hipSuccess && S) e = hipMemcpyAsync(rev64, r->rev.data(), 8 * S, hipMemcpyHostToDevice, sv->copy);
    if (e == hipSuccess && S) e = hipMemcpyAsync(base + L.head, r->head.data(), 4 * S, hipMemcpyHostToDevice, sv->copy);
    if (e == hipSuccess && S) e = hipMemcpyAsync(base + L.cap, r->cap.data(), 4 * S, hipMemcpyHostToDevice, sv->copy);
    if (e == hipSuccess) e = hipStreamSynchronize(sv->copy);
    if (e != hipSuccess) {
        sv->alloc.release(off, r->bytes);
        r->result.status = MF_EDEVICE;
        r->state = COMPLETE;
        r->t_done = Clock::now();
        sv->err = hipGetErrorString(e);
        return true;
    }
    // the host copy of the graph is no longer needed
    std::vector<int64_t>().swap(r->off);
    std::vector<int64_t>().swap(r->rev);
    std::vector<int32_t>().swap(r->head);
    std::vector<int32_t>().swap(r->cap);
    BatchItem it;
    memset(&it, 0, sizeof it);
    it.g.n = r->n;
    it.g.s = r->s;
    it.g.t = r->t;
    it.g.slots = (int32_t)r->S;
    it.g.off = (int32_t *)(base + L.off);
    it.g.head = (int32_t *)(base + L.head);
    it.g.rev = (int32_t *)(base + L.rev);
    it.g.cap = (int32_t *)(base + L.cap);
    it.st.res = (int32_t *)(base + L.res);
    it.st.delta = (int32_t *)(base + L.delta);
    it.st.C = (int32_t *)(base + L.C);
    it.st.d = (int32_t *)(base + L.d);
    it.st.dn = (int32_t *)(base + L.dn);
    it.st.owner = (int32_t *)(base + L.owner);
    it.st.A = (int32_t *)(base + L.A);
    it.st.A2 = (int32_t *)(base + L.A2);
    it.st.Q = (int32_t *)(base + L.Q);
    it.st.Q2 = (int32_t *)(base + L.Q2);
    it.st.H = (int32_t *)(base + L.H);
    it.st.e = (int64_t *)(base + L.e);
    it.st.act = base + L.act;
    it.st.touched = base + L.touched;
    it.ctl = nullptr;
    it.flow = r->want_flow ? (int32_t *)(base + L.flow) : nullptr;
    it.side = base + L.side;
    it.off64 = off64;
    it.rev64 = rev64;
    it.G = r->G;
    it.preflow_only = (r->opt.flags & MF_PREFLOW_ONLY) ? 1 : 0;
    const mf_options &o = r->opt;
    it.p.freq_num = o.gr_freq_num;
    it.p.freq_den = o.gr_freq_den;
    it.p.alpha = o.gr_alpha;
    it.p.beta = o.gr_beta;
    it.p.round_charge = o.gr_round_charge;
    it.p.max_rounds = o.max_rounds;
    it.p.dense_threshold = o.dense_threshold > 0 ? o.dense_threshold : std::max<int64_t>(512, r->n / 16);
    it.p.bu_factor = 8;
    it.p.hubdeg = 64 * r->G;
    it.ctl = (Ctl *)(base + L.end + staging_ctl(r->n, r->S));
    r->index = index;
    sv->slot_owner[q][index % SERVE_CAP] = r;
    ServeHostQueue *hq = sv->hq[q];
    hq->done[index % SERVE_CAP] = 0;
    hq->items[index % SERVE_CAP] = it;
    sv->published[q] = index + 1;
    __atomic_store_n(&hq->count, index + 1, __ATOMIC_RELEASE);
    r->state = PUBLISHED;
    sv->inflight_list.push_back(r);
    sv->st.admitted++;
    sv->st.peak_bytes = std::max<size_t>(sv->st.peak_bytes, sv->alloc.used());
    return true;
}

static void finish(mf_server *sv, Request *r)
{
    const int q = r->queue;
    ServeHostQueue *hq = sv->hq[q];
    const int slot = r->index % SERVE_CAP;
    const BatchResult br = hq->results[slot];
    uint8_t *base = sv->region + r->region_off;
    const InstLayout &L = r->lay;
    mf_result &R = r->result;
    R.lanes_per_vertex = r->G;
    R.status = br.status == 0 ? MF_OK : br.status == 1 ? MF_ETIMEOUT : br.status == 3 ? MF_EINVAL : MF_EDEVICE;
    R.value = br.value;
    R.cut_capacity = br.cut;
    R.rounds = br.rounds;
    R.rounds2 = br.rounds2;
    R.global_relabels = br.grs;
    R.global_relabels2 = br.grs2;
    R.bfs_levels = br.levels;
    R.pushes = br.pushes;
    R.relabels = br.relabels;
    R.ms_start = 0;
    R.ms_end = 1e3 * (double)(br.t_end - br.t_start) / (double)sv->ctx->wall_hz;
    if (!r->canceled && R.status == MF_OK) {
        r->side.resize((size_t)r->n);
        hipError_t e = hipMemcpyAsync(r->side.data(), base + L.side, (size_t)r->n, hipMemcpyDeviceToHost, sv->copy);
        if (e == hipSuccess && r->want_flow && r->S) {
            r->flow.resize((size_t)r->S);
            e = hipMemcpyAsync(r->flow.data(), base + L.flow, 4 * (size_t)r->S, hipMemcpyDeviceToHost, sv->copy);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(sv->copy);
        if (e != hipSuccess) R.status = MF_EDEVICE;
    }
    if (r->canceled) {
        R.status = MF_ECANCELED;
        sv->st.canceled++;
    } else {
        sv->st.completed++;
    }
    sv->alloc.release(r->region_off, r->bytes);
    sv->slot_owner[q][slot] = nullptr;
    r->state = COMPLETE;
    r->t_done = Clock::now();
}

static void server_loop(mf_server *sv)
{
    (void)hipSetDevice(sv->ctx->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    while (!sv->stop) {
        bool progress = false;
        // completions
        for (size_t i = 0; i < sv->inflight_list.size();) {
            Request *r = sv->inflight_list[i];
            ServeHostQueue *hq = sv->hq[r->queue];
            const int d = __atomic_load_n(&hq->done[r->index % SERVE_CAP], __ATOMIC_ACQUIRE);
            if (d == r->index + 1) {
                finish(sv, r);
                sv->inflight_list[i] = sv->inflight_list.back();
                sv->inflight_list.pop_back();
                progress = true;
            } else {
                i++;
            }
        }
        if (progress) sv->cv.notify_all();
        // admission in arrival order
        while (!sv->pending.empty()) {
            Request *r = sv->pending.front();
            if (!admit(sv, r)) break;
            sv->pending.pop_front();
            progress = true;
            if (r->state == COMPLETE) sv->cv.notify_all();
        }
        // keep a serve kernel running for every queue with published work
        for (int q = 0; q < 4; q++) {
            bool has_work = false;
            for (Request *r : sv->inflight_list)
                if (r->queue == q) {
                    has_work = true;
                    break;
                }
            if (!has_work) continue;
            if (hipStreamQuery(sv->kstream[q]) == hipSuccess) {
                int backlog = 0;
                for (Request *r : sv->inflight_list) backlog += r->queue == q;
                // enough workgroups for the work at hand plus room for arrivals
                const int grid = std::max(1, std::min(sv->grid[q], std::max(16, 2 * backlog)));
                if (launch_serve(4 << q, grid, sv->hq[q], sv->next_d + q, sv->idle_ticks, sv->kstream[q]) ==
                    hipSuccess)
                    sv->st.kernel_launches++;
            }
        }
        if (!progress) sv->cv.wait_for(lk, std::chrono::microseconds(100));
    }
}
