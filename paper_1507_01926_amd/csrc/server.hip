// Served form: a request loop that admits max-flow solves by HBM budget as
// they arrive and runs them with continuous batching.
//
//  - mf_server_submit copies the request to the host queue and returns a
//    ticket at once.
//  - A worker thread admits requests in arrival order while the device
//    region (one allocation of the budget's size, carved by a best-fit
//    allocator), the pinned host staging arena and the in-flight limit
//    allow, writes the graph into its staging slice and publishes the
//    request to the queue in coherent host memory.
//  - One persistent kernel, launched with every workgroup the device can
//    hold, keeps taking published requests (one workgroup per request:
//    pulling the graph from host memory into its device slice, residency
//    checks, both phases, outputs sent back to the staging slice, with the
//    request's own lane count) while it runs; a request that arrives while others are on the
//    GPU joins the running kernel as soon as a workgroup is free.  A kernel that finds
//    no work for idle_ms leaves; the worker starts it again when requests
//    arrive.
//  - Finished requests are read from their staging slice, their slices are
//    freed, and mf_server_poll / mf_server_wait return them.
// No runtime copy runs while the serve kernel runs: all transfers are done
// by the kernel's own loads and stores over PCIe, so a kernel that keeps
// every compute unit busy never waits for a copy queued behind it.
// Graphs and residual state stay in device memory for the whole solve.
//
// Grid lane.  A request above the routing size (batch_grid_slots: one
// workgroup would take seconds on it) and every re-solve of a resident graph
// go to a second worker with a context of its own, which solves them one at
// a time with the grid-wide kernels in a slice of the same device region,
// beside the serve kernel.  A resident graph (mf_server_register_graph)
// keeps its arrays and the residuals of its last complete solve in its
// slice; a re-solve with new capacities (mf_server_submit_caps) resumes
// from that flow when every new capacity still holds it (the warm start of
// the plain solver), and starts from zero flow otherwise.
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

enum ReqState { STAGING, PENDING, ADMITTING, PUBLISHED, COMPLETE };
enum ReqKind { SOLVE, REGISTER, RESOLVE };

// A graph kept in the device region for re-solves (grid lane).
struct Resident {
    uint64_t id = 0;
    int32_t n = 0, s = 0, t = 0;
    int64_t S = 0;
    size_t off = 0, bytes = 0;       // slice of the region
    InstLayout lay;                  // graph, state, flow, side
    size_t keep = 0;                 // region offset of the kept residuals (int32[S])
    bool valid = false;              // the graph was uploaded and checked
    bool has_flow = false;           // keep holds the residuals of a complete solve
    int64_t value = 0;               // its flow value
    bool released = false;
    int pending = 0;                 // queued requests that name it
    int32_t maxdeg_inner = 0, deg_s = 0, deg_t = 0;   // degree figures (the structure never changes)
};

struct Request {
    uint64_t ticket = 0;
    ReqKind kind = SOLVE;
    bool grid = false;           // solved by the grid lane
    uint64_t graph_id = 0;       // REGISTER / RESOLVE: the resident graph
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
    size_t host_bytes = 0, host_off = 0;
    bool staged = false;         // graph already in its host staging slice
    InstLayout lay;
    ReqState state = PENDING;
    Clock::time_point t_submit, t_done;
    mf_result result;
    std::vector<int32_t> flow;
    std::vector<uint8_t> side;
};

// Device slice of one request: the instance layout, then the five control
// blocks.
size_t request_bytes(int64_t n, int64_t S, bool want_flow)
{
    InstLayout L = layout_for(0, n, S, want_flow);
    return L.end + align256(5 * sizeof(Ctl));
}

// Host staging slice of one request: int64 offsets, int64 reverse slots,
// int32 heads, int32 capacities as received.  The results reuse it once the
// graph has been pulled: the sink side at the start, the flow at the second
// part (both fit the parts they overwrite).
struct HostLayout {
    size_t rev, head, cap, end;
};
HostLayout host_layout(int64_t n, int64_t S)
{
    HostLayout h;
    h.rev = align256(8 * (size_t)(n + 1));
    h.head = h.rev + align256(8 * (size_t)S);
    h.cap = h.head + align256(4 * (size_t)S);
    h.end = h.cap + align256(4 * (size_t)S);
    return h;
}

// Device slice of a request solved by the grid lane: the instance layout
// (with the packed heads of the top-down search), then int64 staging for the
// offsets and reverse slots during the upload.
struct GridSlice {
    InstLayout lay;
    size_t stage, keep, end;
};
GridSlice grid_slice(int64_t n, int64_t S, bool want_flow, bool resident)
{
    GridSlice g;
    g.lay = layout_for(0, n, S, want_flow || resident, true);
    size_t p = g.lay.end;
    g.keep = 0;
    if (resident) {
        g.keep = p;
        p = align256(p + std::max<size_t>(4 * (size_t)S, 4));
    }
    g.stage = p;
    p = align256(p + 8 * (size_t)(n + 1) + 8 * (size_t)S);
    g.end = p;
    return g;
}

}  // namespace

struct mf_server {
    mf_context *ctx = nullptr;
    mf_server_config cfg;
    uint8_t *region = nullptr;
    RegionAllocator alloc;
    uint8_t *harena = nullptr;       // pinned coherent host staging arena
    size_t harena_bytes = 0;
    RegionAllocator halloc;
    ServeHostQueue *hq[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t *next_d = nullptr;       // [4] device counters
    int32_t published[4] = {0, 0, 0, 0};
    hipStream_t kstream[4] = {nullptr, nullptr, nullptr, nullptr};
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
    int64_t unstaged = 0;            // pending requests whose graph waits in pageable memory
    mf_server_stats st;
    size_t bytes_in_use = 0;
    std::string err;
    // grid lane: worker threads, each with a context of its own (worker 0
    // also takes registrations and re-solves of resident graphs, in order)
    std::vector<mf_context *> gctx;
    std::vector<std::thread> gworkers;
    std::deque<Request *> gpending;
    std::mutex amu;                   // guards `alloc` (both workers carve the region)
    std::condition_variable acv;      // region space freed
    std::unordered_map<uint64_t, Resident *> residents;
    uint64_t next_graph = 1;
    int grid_busy = 0;                // a grid-lane request is being solved
};

static void server_loop(mf_server *sv);
static void grid_loop(mf_server *sv, int wi);

// Gives back what a request that will not be admitted holds on the host
// side (called with the lock held).
static void drop_staging(mf_server *sv, Request *r)
{
    if (r->staged) {
        sv->halloc.release(r->host_off, r->host_bytes);
        r->staged = false;
    } else {
        sv->unstaged--;
    }
    std::vector<int64_t>().swap(r->off);
    std::vector<int64_t>().swap(r->rev);
    std::vector<int32_t>().swap(r->head);
    std::vector<int32_t>().swap(r->cap);
}

static void stage_graph(mf_server *sv, Request *r, const int64_t *off, const int64_t *rev, const int32_t *head,
                        const int32_t *cap);

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
        int per_cu = serve_blocks_per_cu(0);
        if (per_cu <= 0) per_cu = 1;
        if (sv->cfg.blocks_per_cu > 0) per_cu = std::min(per_cu, (int)sv->cfg.blocks_per_cu);
        sv->grid[q] = per_cu * ctx->num_cus;
    }
    sv->harena_bytes = sv->cfg.host_staging_mib > 0 ? (size_t)sv->cfg.host_staging_mib << 20
                                                    : std::min(sv->cfg.hbm_budget_bytes, (size_t)1 << 30);
    sv->harena_bytes = align256(sv->harena_bytes);
    if (hipHostMalloc((void **)&sv->harena, sv->harena_bytes, hipHostMallocCoherent) != hipSuccess)
        return bail(MF_ENOMEM, "pinned staging allocation failed");
    sv->halloc.init(sv->harena_bytes);
    if (hipMalloc((void **)&sv->next_d, 8 * sizeof(int32_t)) != hipSuccess ||
        hipMemset(sv->next_d, 0, 8 * sizeof(int32_t)) != hipSuccess)
        return bail(MF_EDEVICE, "device counter allocation failed");
    sv->idle_ticks = ctx->wall_hz / 1000ull * (uint64_t)sv->cfg.idle_ms;
    for (int q = 0; q < 4; q++) sv->slot_owner[q].assign(SERVE_CAP, nullptr);
    const int nw = sv->cfg.grid_workers > 0 ? std::min(sv->cfg.grid_workers, 32) : 4;
    for (int w = 0; w < nw; w++) {
        mf_context *gc = nullptr;
        if (mf_context_create(ctx->device, 0, &gc) != MF_OK) return bail(MF_EDEVICE, "grid-lane context failed");
        sv->gctx.push_back(gc);
    }
    sv->worker = std::thread(server_loop, sv);
    for (int w = 0; w < nw; w++) sv->gworkers.emplace_back(grid_loop, sv, w);
    *out = sv;
    return MF_OK;
}

extern "C" void mf_server_destroy(mf_server *sv)
{
    if (!sv) return;
    sv->stop = true;
    sv->cv.notify_all();
    sv->acv.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    for (auto &t : sv->gworkers)
        if (t.joinable()) t.join();
    for (auto g : sv->gctx) mf_context_destroy(g);
    for (auto &kv : sv->residents) delete kv.second;
    (void)hipSetDevice(sv->ctx->device);
    for (int q = 0; q < 4; q++)
        if (sv->hq[q]) __atomic_store_n(&sv->hq[q]->shutdown, 1, __ATOMIC_RELEASE);
    for (int q = 0; q < 4; q++)
        if (sv->kstream[q]) {
            (void)hipStreamSynchronize(sv->kstream[q]);
            (void)hipStreamDestroy(sv->kstream[q]);
        }
    for (int q = 0; q < 4; q++)
        if (sv->hq[q]) (void)hipHostFree(sv->hq[q]);
    if (sv->harena) (void)hipHostFree(sv->harena);
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
                          o.gr_round_charge >= 0 && o.gr_level_charge >= 0 && o.max_rounds >= 0 &&
                          !(o.flags & (MF_GAP_RELABEL | MF_CHECK_INVARIANTS));
    if (shape_ok) {
        r->G = batch_lanes(o.lanes_per_vertex, g->n, g->slots);
        r->queue = 0;        // one queue; the serve kernel handles every lane count
        r->grid = g->slots > batch_grid_slots(o);
        if (r->grid) {
            r->bytes = grid_slice(g->n, g->slots, r->want_flow, false).end;
            r->host_bytes = 0;
        } else {
            r->bytes = request_bytes(g->n, g->slots, r->want_flow);
            r->host_bytes = host_layout(g->n, g->slots).end;
        }
    }
    const bool fits = shape_ok && r->bytes <= sv->cfg.hbm_budget_bytes && r->host_bytes <= sv->harena_bytes;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        r->ticket = sv->next_ticket++;
        r->t_submit = Clock::now();
        sv->reqs[r->ticket] = r;
        sv->st.submitted++;
        *ticket = r->ticket;
        if (!fits) {
            r->result.status = shape_ok ? MF_ENOMEM : MF_EINVAL;
            r->state = COMPLETE;
            r->t_done = Clock::now();
            sv->st.rejected++;
            sv->cv.notify_all();
            return MF_OK;
        }
        // The graph goes straight into a staging slice when one is free and
        // no earlier request is still waiting for one; otherwise into
        // pageable memory, and the worker stages it at admission.  Pending
        // requests stay in ticket order, so those holding a slice always
        // precede those waiting for one.  Grid-lane requests keep their copy
        // in pageable memory.
        r->state = STAGING;
        if (r->grid)
            ;
        else if (sv->unstaged == 0 && sv->halloc.alloc(r->host_bytes, r->host_off))
            r->staged = true;
        else
            sv->unstaged++;
    }
    // the copy runs on the caller's thread, without the lock
    if (r->staged) {
        stage_graph(sv, r, g->offsets, g->rev, g->head, g->cap);
    } else {
        r->off.assign(g->offsets, g->offsets + g->n + 1);
        r->rev.assign(g->rev, g->rev + g->slots);
        r->head.assign(g->head, g->head + g->slots);
        r->cap.assign(g->cap, g->cap + g->slots);
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    if (r->canceled) {                     // canceled while its graph was copied
        drop_staging(sv, r);
        r->result.status = MF_ECANCELED;
        r->state = COMPLETE;
        r->t_done = Clock::now();
        sv->st.canceled++;
    } else {
        r->state = PENDING;
        auto &q = r->grid ? sv->gpending : sv->pending;
        auto pos = q.end();
        while (pos != q.begin() && (*(pos - 1))->ticket > r->ticket) --pos;
        q.insert(pos, r);
    }
    sv->cv.notify_all();
    return MF_OK;
}

// Resident graphs (grid lane).  Registration is processed by the grid
// worker in queue order and waited for here.
extern "C" mf_status mf_server_register_graph(mf_server *sv, const mf_graph *g, uint64_t *graph_id)
{
    if (!sv || !g || !graph_id) return MF_EINVAL;
    const bool shape_ok = g->n >= 2 && g->slots >= 0 && g->slots < 2147483647LL &&
                          (int64_t)g->n + g->slots < 2147483647LL && g->s >= 0 && g->s < g->n && g->t >= 0 &&
                          g->t < g->n && g->s != g->t && g->offsets && (g->slots == 0 || (g->head && g->rev && g->cap));
    if (!shape_ok) return MF_EINVAL;
    const size_t bytes = grid_slice(g->n, g->slots, true, true).end;
    if (bytes > sv->cfg.hbm_budget_bytes) return MF_ENOMEM;
    Request *r = new (std::nothrow) Request();
    Resident *res = new (std::nothrow) Resident();
    if (!r || !res) {
        delete r;
        delete res;
        return MF_ENOMEM;
    }
    mf_options_default(&r->opt);
    r->kind = REGISTER;
    r->grid = true;
    r->n = g->n;
    r->s = g->s;
    r->t = g->t;
    r->S = g->slots;
    r->bytes = bytes;
    r->off.assign(g->offsets, g->offsets + g->n + 1);
    r->rev.assign(g->rev, g->rev + g->slots);
    r->head.assign(g->head, g->head + g->slots);
    r->cap.assign(g->cap, g->cap + g->slots);
    memset(&r->result, 0, sizeof r->result);
    res->n = g->n;
    res->s = g->s;
    res->t = g->t;
    res->S = g->slots;
    std::unique_lock<std::mutex> lk(sv->mu);
    res->id = sv->next_graph++;
    r->graph_id = res->id;
    res->pending = 1;
    sv->residents[res->id] = res;
    r->ticket = sv->next_ticket++;
    r->t_submit = Clock::now();
    r->state = PENDING;
    sv->reqs[r->ticket] = r;
    sv->gpending.push_back(r);
    sv->cv.notify_all();
    while (r->state != COMPLETE) sv->cv.wait(lk);
    const mf_status st = (mf_status)r->result.status;
    sv->reqs.erase(r->ticket);
    delete r;
    if (st != MF_OK) {
        sv->residents.erase(res->id);
        delete res;
        return st;
    }
    *graph_id = res->id;
    return MF_OK;
}

extern "C" mf_status mf_server_submit_caps(mf_server *sv, uint64_t graph_id, const int32_t *cap,
                                           const mf_options *opt, int want_flow, uint64_t *ticket)
{
    if (!sv || !ticket) return MF_EINVAL;
    Request *r = new (std::nothrow) Request();
    if (!r) return MF_ENOMEM;
    if (opt) r->opt = *opt; else mf_options_default(&r->opt);
    r->kind = RESOLVE;
    r->grid = true;
    r->graph_id = graph_id;
    r->want_flow = want_flow != 0 && !(r->opt.flags & MF_PREFLOW_ONLY);
    memset(&r->result, 0, sizeof r->result);
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->residents.find(graph_id);
    if (it == sv->residents.end() || it->second->released) {
        delete r;
        return MF_ENOTFOUND;
    }
    Resident *res = it->second;
    if (!cap && res->S > 0) {
        delete r;
        return MF_EINVAL;
    }
    r->n = res->n;
    r->s = res->s;
    r->t = res->t;
    r->S = res->S;
    if (res->S) r->cap.assign(cap, cap + res->S);
    res->pending++;
    r->ticket = sv->next_ticket++;
    r->t_submit = Clock::now();
    r->state = PENDING;
    sv->reqs[r->ticket] = r;
    sv->st.submitted++;
    sv->gpending.push_back(r);
    *ticket = r->ticket;
    sv->cv.notify_all();
    return MF_OK;
}

extern "C" mf_status mf_server_release_graph(mf_server *sv, uint64_t graph_id)
{
    if (!sv) return MF_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->residents.find(graph_id);
    if (it == sv->residents.end() || it->second->released) return MF_ENOTFOUND;
    it->second->released = true;     // the grid worker frees it once no request names it
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
    r->canceled = true;    // STAGING, ADMITTING or PUBLISHED: completes as canceled when that step ends
    if (r->state == PENDING && r->grid) {
        if (r->kind == REGISTER) return MF_OK;     // registration is waited for by its caller
        for (auto p = sv->gpending.begin(); p != sv->gpending.end(); ++p)
            if (*p == r) {
                sv->gpending.erase(p);
                break;
            }
        if (r->kind == RESOLVE) {
            auto it2 = sv->residents.find(r->graph_id);
            if (it2 != sv->residents.end()) it2->second->pending--;
        }
        r->result.status = MF_ECANCELED;
        r->state = COMPLETE;
        r->t_done = Clock::now();
        sv->st.canceled++;
        sv->cv.notify_all();
        return MF_OK;
    }
    if (r->state == PENDING) {
        for (auto p = sv->pending.begin(); p != sv->pending.end(); ++p)
            if (*p == r) {
                sv->pending.erase(p);
                break;
            }
        drop_staging(sv, r);
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
    out->inflight = (int64_t)sv->inflight_list.size() + sv->grid_busy;
    out->queued = (int64_t)sv->pending.size() + (int64_t)sv->gpending.size();
    out->bytes_in_use = sv->bytes_in_use;
    return MF_OK;
}

// ---------------------------------------------------------------------------
// Worker

// The worker owns the device region, the allocator, the queues and the
// in-flight list; the mutex guards what the API threads touch (the pending
// queue, the ticket map, request states and results, the statistics).  Copies
// and kernel launches happen without the mutex.

// Copies a graph into the request's host staging slice.
static void stage_graph(mf_server *sv, Request *r, const int64_t *off, const int64_t *rev, const int32_t *head,
                        const int32_t *cap)
{
    uint8_t *hbase = sv->harena + r->host_off;
    const HostLayout H = host_layout(r->n, r->S);
    const size_t S = (size_t)r->S, N = (size_t)r->n;
    memcpy(hbase, off, 8 * (N + 1));
    if (S) {
        memcpy(hbase + H.rev, rev, 8 * S);
        memcpy(hbase + H.head, head, 4 * S);
        memcpy(hbase + H.cap, cap, 4 * S);
    }
}

// Writes the graph to its staging slice and publishes the request (without
// the mutex; the request is in state ADMITTING).  Returns false if the
// request does not fit now (it stays pending).
static bool admit(mf_server *sv, Request *r)
{
    size_t off;
    if ((int)sv->inflight_list.size() >= sv->cfg.max_inflight) return false;
    const int q = r->queue;
    const int32_t index = sv->published[q];
    if (sv->slot_owner[q][index % SERVE_CAP]) return false;
    {
        std::lock_guard<std::mutex> la(sv->amu);
        if (!sv->alloc.alloc(r->bytes, off)) return false;
    }
    if (!r->staged) {
        bool got;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            got = sv->halloc.alloc(r->host_bytes, r->host_off);
        }
        if (!got) {
            std::lock_guard<std::mutex> la(sv->amu);
            sv->alloc.release(off, r->bytes);
            return false;
        }
        stage_graph(sv, r, r->off.data(), r->rev.data(), r->head.data(), r->cap.data());
        std::vector<int64_t>().swap(r->off);
        std::vector<int64_t>().swap(r->rev);
        std::vector<int32_t>().swap(r->head);
        std::vector<int32_t>().swap(r->cap);
        r->staged = true;
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->unstaged--;
    }
    r->region_off = off;
    uint8_t *base = sv->region + off;
    uint8_t *hbase = sv->harena + r->host_off;
    r->lay = layout_for(0, r->n, r->S, r->want_flow);
    const InstLayout &L = r->lay;
    const HostLayout H = host_layout(r->n, r->S);
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
    it.flow = r->want_flow ? (int32_t *)(base + L.flow) : nullptr;
    it.side = base + L.side;
    it.off64 = (const int64_t *)hbase;
    it.rev64 = (const int64_t *)(hbase + H.rev);
    it.head_h = (const int32_t *)(hbase + H.head);
    it.cap_h = (const int32_t *)(hbase + H.cap);
    it.side_h = hbase;
    it.flow_h = r->want_flow ? (int32_t *)(hbase + H.rev) : nullptr;
    it.G = r->G;
    it.preflow_only = (r->opt.flags & MF_PREFLOW_ONLY) ? 1 : 0;
    const mf_options &o = r->opt;
    it.p.freq_num = o.gr_freq_num;
    it.p.freq_den = o.gr_freq_den;
    it.p.alpha = o.gr_alpha;
    it.p.beta = o.gr_beta;
    it.p.round_charge = o.gr_round_charge;
    it.p.level_charge = o.gr_level_charge;
    it.p.max_rounds = o.max_rounds;
    it.p.dense_threshold = o.dense_threshold > 0 ? o.dense_threshold : std::max<int64_t>(512, r->n / 16);
    it.p.bu_factor = o.bfs_bottom_up_factor > 0 ? o.bfs_bottom_up_factor : 8;
    it.p.hubdeg = 64 * r->G;
    it.p.simple = (o.flags & MF_SIMPLE_ROUNDS) ? 1 : 0;
    it.ctl = (Ctl *)(base + L.end);
    r->index = index;
    sv->slot_owner[q][index % SERVE_CAP] = r;
    ServeHostQueue *hq = sv->hq[q];
    hq->done[index % SERVE_CAP] = 0;
    hq->items[index % SERVE_CAP] = it;
    sv->published[q] = index + 1;
    // the staging copies may use non-temporal stores: a full fence orders
    // them before the publishing store
    std::atomic_thread_fence(std::memory_order_seq_cst);
    __atomic_store_n(&hq->count, index + 1, __ATOMIC_RELEASE);
    sv->inflight_list.push_back(r);
    return true;
}

// Reads the result of a finished request and its outputs from the staging
// slice (without the mutex); frees its slices.
static void finish(mf_server *sv, Request *r, bool canceled)
{
    const int q = r->queue;
    ServeHostQueue *hq = sv->hq[q];
    const int slot = r->index % SERVE_CAP;
    const BatchResult br = hq->results[slot];
    const uint8_t *hbase = sv->harena + r->host_off;
    const HostLayout H = host_layout(r->n, r->S);
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
    R.ms_start = br.t_solve > br.t_start ? 1e3 * (double)(br.t_solve - br.t_start) / (double)sv->ctx->wall_hz : 0;
    R.ms_end = 1e3 * (double)(br.t_end - br.t_start) / (double)sv->ctx->wall_hz;
    if (!canceled && R.status == MF_OK) {
        r->side.assign(hbase, hbase + r->n);
        if (r->want_flow && r->S) {
            const int32_t *f = (const int32_t *)(hbase + H.rev);
            r->flow.assign(f, f + r->S);
        }
    }
    {
        std::lock_guard<std::mutex> la(sv->amu);
        sv->alloc.release(r->region_off, r->bytes);
    }
    sv->acv.notify_all();
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->halloc.release(r->host_off, r->host_bytes);
    sv->slot_owner[q][slot] = nullptr;
}

static void server_loop(mf_server *sv)
{
    (void)hipSetDevice(sv->ctx->device);
    while (!sv->stop) {
        bool progress = false;
        // completions
        for (size_t i = 0; i < sv->inflight_list.size();) {
            Request *r = sv->inflight_list[i];
            ServeHostQueue *hq = sv->hq[r->queue];
            const int d = __atomic_load_n(&hq->done[r->index % SERVE_CAP], __ATOMIC_ACQUIRE);
            if (d != r->index + 1) {
                i++;
                continue;
            }
            bool canceled;
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                canceled = r->canceled;
            }
            finish(sv, r, canceled);
            sv->inflight_list[i] = sv->inflight_list.back();
            sv->inflight_list.pop_back();
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                if (r->canceled) {
                    r->result.status = MF_ECANCELED;
                    sv->st.canceled++;
                } else {
                    sv->st.completed++;
                }
                r->state = COMPLETE;
                r->t_done = Clock::now();
            }
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                std::lock_guard<std::mutex> la(sv->amu);
                sv->bytes_in_use = sv->alloc.used();
            }
            sv->cv.notify_all();
            progress = true;
        }
        // admission in arrival order
        while (true) {
            Request *r = nullptr;
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                if (sv->pending.empty()) break;
                r = sv->pending.front();
                sv->pending.pop_front();
                r->state = ADMITTING;
            }
            const bool done = admit(sv, r);
            std::lock_guard<std::mutex> lk(sv->mu);
            if (!done && r->canceled) {            // canceled while being admitted
                drop_staging(sv, r);
                r->result.status = MF_ECANCELED;
                r->state = COMPLETE;
                r->t_done = Clock::now();
                sv->st.canceled++;
                sv->cv.notify_all();
                progress = true;
                continue;
            }
            if (!done) {
                r->state = PENDING;
                sv->pending.push_front(r);
                break;
            }
            r->state = PUBLISHED;
            sv->st.admitted++;
            {
                std::lock_guard<std::mutex> la(sv->amu);
                sv->bytes_in_use = sv->alloc.used();
            }
            sv->st.peak_bytes = std::max<size_t>(sv->st.peak_bytes, sv->bytes_in_use);
            progress = true;
        }
        // keep the serve kernel running while requests are published
        if (!sv->inflight_list.empty() && hipStreamQuery(sv->kstream[0]) == hipSuccess) {
            const int grid = std::max(2, sv->grid[0]);
            if (launch_serve(0, grid, sv->hq[0], sv->next_d, sv->idle_ticks, (int)sv->st.kernel_launches + 1,
                             sv->kstream[0]) == hipSuccess) {
                std::lock_guard<std::mutex> lk(sv->mu);
                sv->st.kernel_launches++;
            }
        }
        if (!progress) {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->pending.empty() && sv->inflight_list.empty())
                sv->cv.wait_for(lk, std::chrono::milliseconds(2));
            else
                sv->cv.wait_for(lk, std::chrono::microseconds(50));
        }
    }
}

// ---------------------------------------------------------------------------
// Grid lane worker: requests above the routing size, registrations and
// re-solves of resident graphs, one at a time on the lane's own context.

// Carves `bytes` of the region, waiting while the other lane holds the
// space; false if the server is stopping.
static bool carve(mf_server *sv, size_t bytes, size_t &off)
{
    std::unique_lock<std::mutex> la(sv->amu);
    while (!sv->alloc.alloc(bytes, off)) {
        if (sv->stop) return false;
        sv->acv.wait_for(la, std::chrono::milliseconds(1));
    }
    return true;
}

static void uncarve(mf_server *sv, size_t off, size_t bytes)
{
    {
        std::lock_guard<std::mutex> la(sv->amu);
        sv->alloc.release(off, bytes);
    }
    sv->acv.notify_all();
}

static void fill_result(mf_result &R, mf_status st, const mf_stats &ss, double ms_start, double ms_end)
{
    R.status = st;
    R.lanes_per_vertex = 0;
    R.value = ss.value;
    R.cut_capacity = ss.cut_capacity;
    R.rounds = ss.rounds;
    R.rounds2 = ss.rounds2;
    R.global_relabels = ss.global_relabels;
    R.global_relabels2 = ss.global_relabels2;
    R.bfs_levels = ss.bfs_levels;
    R.pushes = ss.pushes;
    R.relabels = ss.relabels;
    R.ms_start = ms_start;
    R.ms_end = ms_end;
}

// Reads the sink side and the flow of a finished solve into the request.
static mf_status take_device_outputs(mf_context *g, Request *r, const uint8_t *side_dev, const int32_t *flow_dev)
{
    r->side.resize((size_t)r->n);
    hipError_t he = hipMemcpyAsync(r->side.data(), side_dev, (size_t)r->n, hipMemcpyDeviceToHost, g->stream);
    if (he == hipSuccess && r->want_flow && r->S) {
        r->flow.resize((size_t)r->S);
        he = hipMemcpyAsync(r->flow.data(), flow_dev, 4 * (size_t)r->S, hipMemcpyDeviceToHost, g->stream);
    }
    if (he == hipSuccess) he = hipStreamSynchronize(g->stream);
    return he == hipSuccess ? MF_OK : MF_EDEVICE;
}

static void grid_solve(mf_server *sv, mf_context *g, Request *r)
{
    const auto t0 = Clock::now();
    const GridSlice G = grid_slice(r->n, r->S, r->want_flow, false);
    size_t off;
    if (!carve(sv, G.end, off)) {
        r->result.status = MF_ECANCELED;
        return;
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->st.admitted++;
        std::lock_guard<std::mutex> la(sv->amu);
        sv->bytes_in_use = sv->alloc.used();
        sv->st.peak_bytes = std::max<size_t>(sv->st.peak_bytes, sv->bytes_in_use);
    }
    uint8_t *base = sv->region + off;
    mf_graph mg{r->n, r->S, r->off.data(), r->head.data(), r->rev.data(), r->cap.data(), r->s, r->t};
    mf_dgraph dg;
    mf_stats ss;
    memset(&ss, 0, sizeof ss);
    mf_status st = upload_graph_into(g, &mg, base, G.lay, (int64_t *)(base + G.stage), &dg);
    const double ms_in = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    if (st == MF_OK) {
        Workspace w = workspace_in(base, G.lay, r->n, r->S);
        mf_options o = r->opt;
        o.flags &= ~(uint32_t)(MF_PROFILE | MF_WARM_START | MF_PERSISTENT);
        int64_t val = 0;
        st = solve_in_workspace(g, &dg, &o, &val, r->want_flow ? (int32_t *)(base + G.lay.flow) : nullptr,
                                base + G.lay.side, &ss, &w, false);
        if (st == MF_OK) st = take_device_outputs(g, r, base + G.lay.side, (int32_t *)(base + G.lay.flow));
    }
    fill_result(r->result, st, ss, ms_in, std::chrono::duration<double, std::milli>(Clock::now() - t0).count());
    uncarve(sv, off, G.end);
}

static void grid_register(mf_server *sv, mf_context *g, Request *r, Resident *res)
{
    const GridSlice G = grid_slice(r->n, r->S, true, true);
    size_t off;
    if (!carve(sv, G.end, off)) {
        r->result.status = MF_ECANCELED;
        return;
    }
    res->off = off;
    res->bytes = G.end;
    res->lay = G.lay;
    res->keep = G.keep;
    uint8_t *base = sv->region + off;
    mf_graph mg{r->n, r->S, r->off.data(), r->head.data(), r->rev.data(), r->cap.data(), r->s, r->t};
    mf_dgraph dg;
    mf_status st = upload_graph_into(g, &mg, base, G.lay, (int64_t *)(base + G.stage), &dg);
    if (st != MF_OK) {
        uncarve(sv, off, G.end);
        res->bytes = 0;
    } else {
        res->valid = true;
        res->maxdeg_inner = dg.maxdeg_inner;
        res->deg_s = dg.deg_s;
        res->deg_t = dg.deg_t;
    }
    r->result.status = st;
}

static void grid_resolve(mf_server *sv, mf_context *g, Request *r, Resident *res)
{
    const auto t0 = Clock::now();
    mf_stats ss;
    memset(&ss, 0, sizeof ss);
    if (!res->valid) {
        r->result.status = MF_EINVAL;
        return;
    }
    uint8_t *base = sv->region + res->off;
    const InstLayout &L = res->lay;
    mf_dgraph dg;
    dg.n = res->n;
    dg.s = res->s;
    dg.t = res->t;
    dg.slots = res->S;
    dg.off = (int32_t *)(base + L.off);
    dg.head = (int32_t *)(base + L.head);
    dg.rev = (int32_t *)(base + L.rev);
    dg.cap = (int32_t *)(base + L.cap);
    dg.maxdeg_inner = res->maxdeg_inner;
    dg.deg_s = res->deg_s;
    dg.deg_t = res->deg_t;
    int32_t *keep = (int32_t *)(base + res->keep);
    bool resumable = false;
    mf_status st = check_caps_into(g, &dg, r->cap.data(), (int32_t *)(base + L.flow), keep, res->has_flow,
                                   &resumable);
    const double ms_in = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    if (st == MF_OK) {
        Workspace w = workspace_in(base, L, res->n, res->S);
        if (resumable) {
            // the kept flow goes back into the workspace, e(t) its value
            hipError_t he = hipSuccess;
            if (res->S) he = hipMemcpyAsync(w.res, keep, 4 * (size_t)res->S, hipMemcpyDeviceToDevice, g->stream);
            if (he == hipSuccess)
                he = hipMemcpyAsync(w.e + res->t, &res->value, sizeof(int64_t), hipMemcpyHostToDevice, g->stream);
            if (he == hipSuccess) he = hipStreamSynchronize(g->stream);
            if (he != hipSuccess) st = MF_EDEVICE;
        }
        mf_options o = r->opt;
        o.flags &= ~(uint32_t)(MF_PROFILE | MF_WARM_START | MF_PERSISTENT | MF_PREFLOW_ONLY);
        int64_t val = 0;
        if (st == MF_OK)
            st = solve_in_workspace(g, &dg, &o, &val, (int32_t *)(base + L.flow), base + L.side, &ss, &w,
                                    resumable);
        if (st == MF_OK) {
            // keep this flow for the next re-solve
            hipError_t he = hipSuccess;
            if (res->S) he = hipMemcpyAsync(keep, w.res, 4 * (size_t)res->S, hipMemcpyDeviceToDevice, g->stream);
            if (he == hipSuccess) he = hipStreamSynchronize(g->stream);
            if (he != hipSuccess) st = MF_EDEVICE;
            res->has_flow = st == MF_OK;
            res->value = val;
        } else {
            res->has_flow = false;
        }
        if (st == MF_OK) st = take_device_outputs(g, r, base + L.side, (int32_t *)(base + L.flow));
    }
    fill_result(r->result, st, ss, ms_in, std::chrono::duration<double, std::milli>(Clock::now() - t0).count());
    r->result.resumed = resumable ? 1 : 0;
}

static void grid_loop(mf_server *sv, int wi)
{
    (void)hipSetDevice(sv->ctx->device);
    mf_context *g = sv->gctx[(size_t)wi];
    while (!sv->stop) {
        Request *r = nullptr;
        Resident *res = nullptr;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            // free released resident graphs that no queued request names
            if (wi == 0)
                for (auto it = sv->residents.begin(); it != sv->residents.end();) {
                    Resident *x = it->second;
                    if (x->released && x->pending == 0) {
                        if (x->bytes) uncarve(sv, x->off, x->bytes);
                        delete x;
                        it = sv->residents.erase(it);
                    } else {
                        ++it;
                    }
                }
            // the first request this worker may take: worker 0 any, the
            // others one-shot solves only (resident graphs stay in order)
            auto pick = sv->gpending.end();
            for (auto it = sv->gpending.begin(); it != sv->gpending.end(); ++it)
                if (wi == 0 || (*it)->kind == SOLVE) {
                    pick = it;
                    break;
                }
            if (pick == sv->gpending.end()) {
                sv->cv.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
            r = *pick;
            sv->gpending.erase(pick);
            r->state = ADMITTING;
            if (r->kind != SOLVE) {
                auto it = sv->residents.find(r->graph_id);
                res = it == sv->residents.end() ? nullptr : it->second;
            }
            sv->grid_busy++;
        }
        if (r->kind == SOLVE)
            grid_solve(sv, g, r);
        else if (!res)
            r->result.status = MF_ENOTFOUND;
        else if (r->kind == REGISTER)
            grid_register(sv, g, r, res);
        else
            grid_resolve(sv, g, r, res);
        std::vector<int64_t>().swap(r->off);
        std::vector<int64_t>().swap(r->rev);
        std::vector<int32_t>().swap(r->head);
        std::vector<int32_t>().swap(r->cap);
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (res) res->pending--;
            sv->grid_busy--;
            if (r->kind != REGISTER) {
                if (r->canceled) {
                    r->result.status = MF_ECANCELED;
                    sv->st.canceled++;
                } else {
                    sv->st.completed++;
                }
            }
            r->state = COMPLETE;
            r->t_done = Clock::now();
            std::lock_guard<std::mutex> la(sv->amu);
            sv->bytes_in_use = sv->alloc.used();
        }
        sv->cv.notify_all();
    }
}
