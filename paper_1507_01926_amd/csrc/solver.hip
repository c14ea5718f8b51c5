// Host side and C ABI of the maximum-flow library.
//
// The host loop runs the synchronous push-relabel loop of Sec. 3.1 (Listing 1):
//   - init and source saturation;
//   - global relabel first (W = infinity) and whenever the relabel work since
//     the last one crosses the threshold of Sec. 3 (freq * W > alpha*n + m);
//     a global relabel rebuilds the working set from every vertex with
//     positive excess and a label below n;
//   - a round = discharge + merge;
//   - the loop ends when a global relabel run at that point finds no active
//     vertex, so the result is a maximum preflow (value = e(t)) and the
//     labels are exact BFS distances: sink_side[v] = d(v) < n.
// Phase 2 (flow reconstruction, Sec. 2.1 / Sec. 3) runs the same loop with s
// as the sink and t excluded, returning every remaining excess to s.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <mutex>
#include <thread>
#include <new>
#include <string>
#include <vector>

#include "../../include/maxflow.h"
#include "mf_device.h"
#include "mf_phase.h"
#include "mf_host.h"

namespace mf {
void launch_discharge_hubs(bool dense, GraphView g, StateView st, RoundParams p, int grid, hipStream_t s,
                           KEv ev = KEv());
void launch_merge_hubs(bool dense, GraphView g, StateView st, int sink, int other, int grid, hipStream_t s,
                       KEv ev = KEv());
void launch_discharge(int G, bool dense, GraphView g, StateView st, RoundParams p, int grid, hipStream_t s,
                      KEv ev = KEv(), bool two = false);
void launch_merge(int G, bool dense, GraphView g, StateView st, int sink, int other, int hubd, int grid,
                  hipStream_t s, KEv ev = KEv());
void launch_gr_td(int G, GraphView g, StateView st, int level, int sink, int other, const int32_t *qin,
                  int32_t *qout, int hubdeg, int flags, int grid, hipStream_t s, KEv ev = KEv());
void launch_gr_hub(GraphView g, StateView st, int level, int sink, int other, int32_t *qout, int track_deg,
                   int grid, hipStream_t s, KEv ev = KEv());
void launch_gr_bu(GraphView g, StateView st, int level, int sink, int other, int grid, hipStream_t s,
                  KEv ev = KEv());
void launch_gr_collect(GraphView g, StateView st, int level, int32_t *qout, int grid, hipStream_t s);
void launch_compact_flags(const uint8_t *flags, int n, int32_t *list, int32_t *count, int maxgrid, hipStream_t s,
                          KEv ev = KEv(), const int32_t *stop = nullptr);
void launch_warm_state(GraphView g, StateView st, int grid, hipStream_t s);
void launch_recap(GraphView g, const int32_t *cap_new, int32_t *res, int warm, Ctl *ctl, int grid, hipStream_t s);
void launch_degree_stats(GraphView g, Ctl *ctl, int grid, hipStream_t s);
void launch_round_begin(Ctl *ctl, int first, hipStream_t s);
void launch_round_close(Ctl *ctl, int first, int64_t W0, int64_t charge, int64_t freq_num, int64_t freq_den,
                        int64_t gr_threshold, int64_t dense_threshold, hipStream_t s, int dense = 0);
void launch_narrow(const int64_t *off64, const int64_t *rev64, int32_t *off, int32_t *rev, int32_t n,
                   int64_t slots, Ctl *ctl, int grid, hipStream_t s);
void launch_validate(GraphView g, Ctl *ctl, int grid, hipStream_t s);
void launch_init_state(GraphView g, StateView st, int grid, hipStream_t s);
void launch_saturate(GraphView g, StateView st, int grid, hipStream_t s);
void launch_gr_init(GraphView g, StateView st, int sink, int grid, hipStream_t s);
void launch_gr_slots(GraphView g, const int32_t *d, int hubdeg, LevelSet lv, int64_t *out, int grid,
                     hipStream_t s);
void launch_gr_rebuild(GraphView g, StateView st, int sink, int other, int grid, hipStream_t s);
void launch_round_reset(Ctl *ctl, bool dense, hipStream_t s);
void launch_round_end(Ctl *ctl, hipStream_t s);
void launch_side(GraphView g, const int32_t *d, uint8_t *side, int grid, hipStream_t s);
void launch_cut(GraphView g, const uint8_t *side, Ctl *ctl, int grid, hipStream_t s);
void launch_flow(GraphView g, const int32_t *res, int32_t *flow, int grid, hipStream_t s);
void launch_read_value(const int64_t *e, int t, Ctl *ctl, hipStream_t s);
void launch_check_state(GraphView g, StateView st, int sink, int other, int after_gr, int grid, hipStream_t s);
void launch_gap_round(GraphView g, StateView st, int sink, int other, int dense, int grid, hipStream_t s);
void launch_gap_recount(GraphView g, StateView st, int sink, int other, int grid, hipStream_t s);
void launch_rounds_block(int G, GraphView g, StateView st, RoundParams p, int other, int64_t W0, int64_t charge,
                         int64_t freq_num, int64_t freq_den, int64_t gr_threshold, int64_t dense_threshold,
                         int small_max, int64_t budget, hipStream_t s, KEv ev);
void launch_bump(int32_t *p, hipStream_t s);


}  // namespace mf

using namespace mf;

thread_local std::string g_global_err;

// ---------------------------------------------------------------------------
// Scratch of the no-allocation entry point (mf_solve_device_noalloc): one
// file-scope device array per GPU, held from the library's first context on
// that GPU until the process ends.  Host code never uses its name as an
// address: mf_context_create looks up the array's device address once per
// device (with that device current) and every use goes through that address.
static __device__ __align__(256) uint8_t scratch[MF_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_addr[MAX_DEVICES] = {};   // device address of `scratch` on each device
}

// Called with `device` current.
static mf_status scratch_lookup(int device, uint8_t **out)
{
    if (device < 0 || device >= MAX_DEVICES) return fail(nullptr, MF_EINVAL, "device %d beyond the table", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, MF_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_addr[device] = (uint8_t *)p;
    }
    *out = g_scratch_addr[device];
    return MF_OK;
}

// ---------------------------------------------------------------------------
// Public helpers

extern "C" {

void mf_options_default(mf_options *o)
{
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->gr_freq_num = 1;
    o->gr_freq_den = 2;
    o->gr_alpha = 6;
    o->gr_beta = 12;
    o->gr_round_charge = 0;
    o->gr_level_charge = 0;
    o->max_rounds = 0;
    o->flags = 0;
    o->lanes_per_vertex = 0;
    o->lanes_per_merge = 0;
    o->lanes_per_bfs = 0;
    o->profile_mask = 0;
    o->bfs_bottom_up_factor = 0;
    o->profile_stride = 0;
}

const char *mf_version(void) { return "mi355x-maxflow 0.1 (gfx950)"; }

const char *mf_status_str(mf_status s)
{
    switch (s) {
    case MF_OK: return "ok";
    case MF_EINVAL: return "invalid argument";
    case MF_ENOMEM: return "out of memory or over budget";
    case MF_EDEVICE: return "device error";
    case MF_ETIMEOUT: return "round limit reached";
    case MF_EAGAIN: return "not ready";
    case MF_ECANCELED: return "canceled";
    case MF_ENOTFOUND: return "not found";
    case MF_EINVARIANT: return "invariant check failed";
    }
    return "unknown status";
}

const char *mf_last_error(const mf_context *ctx)
{
    return ctx ? ctx->err.c_str() : g_global_err.c_str();
}

mf_status mf_context_create(int device, size_t hbm_budget_bytes, mf_context **out)
{
    if (!out) return fail(nullptr, MF_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0)
        return fail(nullptr, MF_EDEVICE, "no HIP device available (%s)",
                    e != hipSuccess ? hipGetErrorString(e) : "count 0");
    if (device < 0 || device >= count)
        return fail(nullptr, MF_EINVAL, "device %d out of range (%d devices)", device, count);
    mf_context *ctx = new (std::nothrow) mf_context();
    if (!ctx) return fail(nullptr, MF_ENOMEM, "host allocation failed");
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    mf_status st = MF_OK;
    do {
        if (hipSetDevice(device) != hipSuccess) { st = fail(nullptr, MF_EDEVICE, "hipSetDevice failed"); break; }
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cus = prop.multiProcessorCount;
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            st = fail(nullptr, MF_EDEVICE, "hipStreamCreate failed");
            break;
        }
        int wall_khz = 0;
        if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, device) == hipSuccess &&
            wall_khz > 0)
            ctx->wall_hz = (uint64_t)wall_khz * 1000ull;
        if (hipMalloc((void **)&ctx->ctl, 5 * sizeof(Ctl)) != hipSuccess ||
            hipMalloc((void **)&ctx->bar, sizeof(GridBar)) != hipSuccess ||
            hipHostMalloc((void **)&ctx->ctl_host, 5 * sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
            st = fail(nullptr, MF_EDEVICE, "control block allocation failed");
            break;
        }
        for (auto &ev : ctx->ev)
            if (hipEventCreate(&ev) != hipSuccess) { st = fail(nullptr, MF_EDEVICE, "hipEventCreate failed"); break; }
        for (auto &ev : ctx->pev)
            if (hipEventCreate(&ev) != hipSuccess) { st = fail(nullptr, MF_EDEVICE, "hipEventCreate failed"); break; }
        for (auto &ev : ctx->sev)
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                st = fail(nullptr, MF_EDEVICE, "hipEventCreate failed");
                break;
            }
        if (st == MF_OK) st = scratch_lookup(device, &ctx->scratch);
    } while (0);
    if (st != MF_OK) {
        mf_context_destroy(ctx);
        return st;
    }
    *out = ctx;
    return MF_OK;
}

void mf_context_destroy(mf_context *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    Workspace &w = ctx->ws;
    void *ptrs[] = {w.res, w.delta, w.d, w.dn, w.owner, w.e, w.act, w.side, w.touched,
                    w.A, w.A2, w.C, w.Q, w.Q2, w.H, w.hr, w.lcount, w.gcand};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (ctx->ctl) (void)hipFree(ctx->ctl);
    if (ctx->bar) (void)hipFree(ctx->bar);
    if (ctx->one) (void)hipFree(ctx->one);
    if (ctx->ctl_host) (void)hipHostFree(ctx->ctl_host);
    for (auto ev : ctx->ev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto ev : ctx->pev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto ev : ctx->bev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto ev : ctx->sev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto ev : ctx->gev)
        if (ev) (void)hipEventDestroy(ev);
    if (ctx->lstream) (void)hipStreamDestroy(ctx->lstream);
    for (auto h : ctx->helpers) mf_context_destroy(h);
    for (auto ev : ctx->lev) (void)hipEventDestroy(ev);
    for (auto bs : ctx->bstream)
        if (bs) (void)hipStreamDestroy(bs);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Graph residency and validation (step a1)

static const char *validation_message(int bits)
{
    if (bits & 1) return "offsets are not a non-decreasing sequence from 0 to slots";
    if (bits & 2) return "a reverse slot index is out of range";
    if (bits & 4) return "a head is out of range";
    if (bits & 8) return "self-loop";
    if (bits & 16) return "rev is not an involution with matching heads";
    if (bits & 32) return "negative capacity";
    if (bits & 64) return "cap[a] + cap[rev[a]] >= 2^31";
    return "invalid graph";
}

static mf_status read_ctl(mf_context *ctx, int count = 1)
{
    HIPCHK(ctx, hipMemcpyAsync(ctx->ctl_host, ctx->ctl, count * sizeof(Ctl), hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return MF_OK;
}

// The library's work on a caller's buffers waits for everything enqueued on
// the caller's stream so far; afterwards the caller's stream waits for the
// library's stream.
static mf_status order_after(mf_context *ctx, mf_stream stream)
{
    HIPCHK(ctx, hipEventRecord(ctx->sev[0], (hipStream_t)stream));
    HIPCHK(ctx, hipStreamWaitEvent(ctx->stream, ctx->sev[0], 0));
    return MF_OK;
}
static mf_status order_before(mf_context *ctx, mf_stream stream)
{
    HIPCHK(ctx, hipEventRecord(ctx->sev[1], ctx->stream));
    HIPCHK(ctx, hipStreamWaitEvent((hipStream_t)stream, ctx->sev[1], 0));
    return MF_OK;
}

static mf_status graph_upload(mf_context *ctx, const mf_graph *g, int on_device, mf_dgraph **out);

extern "C" mf_status mf_graph_upload(mf_context *ctx, const mf_graph *g, int on_device, mf_stream stream,
                                     mf_dgraph **out)
{
    if (!ctx || !g || !out) return fail(ctx, MF_EINVAL, "NULL argument");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    mf_status st = MF_OK;
    if (on_device && (st = order_after(ctx, stream)) != MF_OK) return st;
    st = graph_upload(ctx, g, on_device, out);
    if (on_device) {
        mf_status so = order_before(ctx, stream);
        if (st == MF_OK) st = so;
    }
    return st;
}

static mf_status graph_upload(mf_context *ctx, const mf_graph *g, int on_device, mf_dgraph **out)
{
    if (!ctx || !g || !out) return fail(ctx, MF_EINVAL, "NULL argument");
    *out = nullptr;
    if (g->n < 2) return fail(ctx, MF_EINVAL, "n must be at least 2");
    if (g->slots < 0 || g->slots >= 2147483647LL || (int64_t)g->n + g->slots >= 2147483647LL)
        return fail(ctx, MF_EINVAL, "slots out of the supported range");
    if (g->s < 0 || g->s >= g->n || g->t < 0 || g->t >= g->n || g->s == g->t)
        return fail(ctx, MF_EINVAL, "s and t must be distinct vertices");
    if (!g->offsets || (g->slots > 0 && (!g->head || !g->rev || !g->cap)))
        return fail(ctx, MF_EINVAL, "NULL graph array");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    mf_dgraph *dg = new (std::nothrow) mf_dgraph();
    if (!dg) return fail(ctx, MF_ENOMEM, "host allocation failed");
    dg->n = g->n;
    dg->s = g->s;
    dg->t = g->t;
    dg->slots = g->slots;
    const size_t S = (size_t)g->slots, N = (size_t)g->n;
    dg->bytes = 4 * (N + 1) + 12 * S + 12;
    mf_status st;
    if ((st = dalloc(ctx, (void **)&dg->off, 4 * (N + 1))) != MF_OK ||
        (st = dalloc(ctx, (void **)&dg->head, 4 * S)) != MF_OK ||
        (st = dalloc(ctx, (void **)&dg->rev, 4 * S)) != MF_OK ||
        (st = dalloc(ctx, (void **)&dg->cap, 4 * S)) != MF_OK) {
        mf_graph_free(ctx, dg);
        return st;
    }
    // int64 staging of offsets and rev, narrowed on the device
    int64_t *off64 = nullptr, *rev64 = nullptr;
    bool own64 = false;
    if (on_device) {
        off64 = const_cast<int64_t *>(g->offsets);
        rev64 = const_cast<int64_t *>(g->rev);
    } else {
        own64 = true;
        if ((st = dalloc(ctx, (void **)&off64, 8 * (N + 1))) != MF_OK ||
            (st = dalloc(ctx, (void **)&rev64, 8 * S)) != MF_OK) {
            dfree(ctx, off64, 8 * (N + 1));
            mf_graph_free(ctx, dg);
            return st;
        }
    }
    auto cleanup = [&]() {
        if (own64) {
            dfree(ctx, off64, 8 * (N + 1));
            dfree(ctx, rev64, 8 * S);
        }
    };
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipError_t he = hipSuccess;
    if (!on_device) {
        he = hipMemcpyAsync(off64, g->offsets, 8 * (N + 1), hipMemcpyHostToDevice, ctx->stream);
        if (he == hipSuccess && S) he = hipMemcpyAsync(rev64, g->rev, 8 * S, hipMemcpyHostToDevice, ctx->stream);
    }
    if (he == hipSuccess && S) he = hipMemcpyAsync(dg->head, g->head, 4 * S, kind, ctx->stream);
    if (he == hipSuccess && S) he = hipMemcpyAsync(dg->cap, g->cap, 4 * S, kind, ctx->stream);
    if (he == hipSuccess) he = hipMemsetAsync(ctx->ctl, 0, sizeof(Ctl), ctx->stream);
    if (he != hipSuccess) {
        cleanup();
        mf_graph_free(ctx, dg);
        return fail(ctx, MF_EDEVICE, "graph upload failed: %s", hipGetErrorString(he));
    }
    const int maxg = ctx->num_cus * 8;
    launch_narrow(off64, rev64, dg->off, dg->rev, dg->n, dg->slots, ctx->ctl,
                  grid_for(std::max<int64_t>(dg->slots, N + 1), 256, maxg), ctx->stream);
    if ((st = read_ctl(ctx)) != MF_OK) {
        cleanup();
        mf_graph_free(ctx, dg);
        return st;
    }
    if (ctx->ctl_host->err == 0) {
        launch_validate(dg->view(), ctx->ctl, grid_for(S, 256, maxg), ctx->stream);
        launch_degree_stats(dg->view(), ctx->ctl, grid_for(N, 256, maxg), ctx->stream);
        if ((st = read_ctl(ctx)) != MF_OK) {
            cleanup();
            mf_graph_free(ctx, dg);
            return st;
        }
        dg->maxdeg_inner = ctx->ctl_host->maxdeg_inner;
        dg->deg_s = ctx->ctl_host->deg_s;
        dg->deg_t = ctx->ctl_host->deg_t;
    }
    cleanup();
    if (ctx->ctl_host->err) {
        int bits = ctx->ctl_host->err;
        mf_graph_free(ctx, dg);
        return fail(ctx, MF_EINVAL, "invalid graph: %s", validation_message(bits));
    }
    *out = dg;
    return MF_OK;
}

extern "C" void mf_graph_free(mf_context *ctx, mf_dgraph *dg)
{
    if (!dg) return;
    if (ctx && ctx->warm_dg == dg) ctx->warm_dg = nullptr;
    if (ctx) {
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        const size_t S = (size_t)dg->slots, N = (size_t)dg->n;
        dfree(ctx, dg->off, 4 * (N + 1));
        dfree(ctx, dg->head, 4 * S);
        dfree(ctx, dg->rev, 4 * S);
        dfree(ctx, dg->cap, 4 * S);
    }
    delete dg;
}

static mf_status graph_set_caps(mf_context *ctx, mf_dgraph *dg, const int32_t *cap, int on_device,
                                int *resumable);

extern "C" mf_status mf_graph_set_caps(mf_context *ctx, mf_dgraph *dg, const int32_t *cap, int on_device,
                                       mf_stream stream, int *resumable)
{
    if (resumable) *resumable = 0;
    if (!ctx || !dg || (!cap && dg->slots > 0)) return fail(ctx, MF_EINVAL, "NULL argument");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    mf_status st = MF_OK;
    if (on_device && (st = order_after(ctx, stream)) != MF_OK) return st;
    st = graph_set_caps(ctx, dg, cap, on_device, resumable);
    if (on_device) {
        mf_status so = order_before(ctx, stream);
        if (st == MF_OK) st = so;
    }
    return st;
}

static mf_status graph_set_caps(mf_context *ctx, mf_dgraph *dg, const int32_t *cap, int on_device,
                                int *resumable)
{
    const int64_t S = dg->slots;
    if (S == 0) {
        if (resumable) *resumable = ctx->warm_dg == dg;
        return MF_OK;
    }
    int32_t *tmp = nullptr;
    mf_status st = dalloc(ctx, (void **)&tmp, 4 * S);
    if (st != MF_OK) return st;
    auto release = [&]() {
        (void)hipStreamSynchronize(ctx->stream);
        dfree(ctx, tmp, 4 * S);
    };
    hipError_t he = hipMemcpyAsync(tmp, cap, 4 * S, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                   ctx->stream);
    if (he == hipSuccess) he = hipMemsetAsync(ctx->ctl, 0, sizeof(Ctl), ctx->stream);
    if (he != hipSuccess) {
        release();
        return fail(ctx, MF_EDEVICE, "capacity upload failed: %s", hipGetErrorString(he));
    }
    const int maxg = ctx->num_cus * 8;
    GraphView gv = dg->view();
    gv.cap = tmp;
    launch_validate(gv, ctx->ctl, grid_for(S, 256, maxg), ctx->stream);
    if ((st = read_ctl(ctx)) != MF_OK) {
        release();
        return st;
    }
    if (ctx->ctl_host->err) {
        const int bits = ctx->ctl_host->err;
        release();
        return fail(ctx, MF_EINVAL, "invalid capacities: %s", validation_message(bits));
    }
    // the kept flow moves with the capacities (its residuals change by the
    // same amounts); then the new capacities replace the old ones
    const bool warm = ctx->warm_dg == dg;
    launch_recap(dg->view(), tmp, ctx->ws.res, warm ? 1 : 0, ctx->ctl, grid_for(S, 256, maxg), ctx->stream);
    he = hipMemcpyAsync(dg->cap, tmp, 4 * S, hipMemcpyDeviceToDevice, ctx->stream);
    if (he != hipSuccess) {
        release();
        ctx->warm_dg = nullptr;
        return fail(ctx, MF_EDEVICE, "capacity update failed: %s", hipGetErrorString(he));
    }
    st = read_ctl(ctx);
    release();
    if (st != MF_OK) {
        ctx->warm_dg = nullptr;
        return st;
    }
    if (warm && (ctx->ctl_host->err & 128)) ctx->warm_dg = nullptr;   // a flow above its new capacity
    if (resumable) *resumable = ctx->warm_dg == dg;
    return MF_OK;
}

// ---------------------------------------------------------------------------
// Workspace

static mf_status ensure_workspace(mf_context *ctx, int64_t n, int64_t slots)
{
    Workspace &w = ctx->ws;
    if (w.n_cap >= n && w.s_cap >= slots && w.res) return MF_OK;
    // release the old one
    void *ptrs[] = {w.res, w.delta, w.d, w.dn, w.owner, w.e, w.act, w.side, w.touched,
                    w.A, w.A2, w.C, w.Q, w.Q2, w.H, w.hr, w.lcount, w.gcand};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    ctx->used -= std::min(ctx->used, w.bytes);
    w = Workspace();
    const int64_t N = std::max(n, w.n_cap), S = std::max(slots, (int64_t)1);
    mf_status st;
    size_t before = ctx->used;
    if ((st = dalloc(ctx, (void **)&w.res, 4 * S)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.delta, 4 * S)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.C, 4 * (S + N))) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.d, 4 * N)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.dn, 4 * N)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.owner, 4 * N)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.e, 8 * N)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.act, N)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.side, N)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.A, 4 * N)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.A2, 4 * N)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.Q, 4 * N)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.Q2, 4 * N)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.H, 4 * N)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.touched, N)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.hr, 4 * S)) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.lcount, 4 * (N + 1))) != MF_OK) return st;
    if ((st = dalloc(ctx, (void **)&w.gcand, 4 * N)) != MF_OK) return st;
    w.n_cap = N;
    w.s_cap = S;
    w.bytes = ctx->used - before;
    return MF_OK;
}

// ---------------------------------------------------------------------------
// The solver

struct PhaseStats {
    int64_t rounds = 0, grs = 0, levels = 0;
};

static int pick_lanes(int requested, int64_t n, int64_t slots)
{
    if (requested > 0) {
        int G = 1;
        while (G < requested && G < 64) G <<= 1;
        return G;
    }
    const double avg = n > 0 ? (double)slots / (double)n : 1.0;
    int G = 1;
    while (G < avg && G < 64) G <<= 1;
    return std::max(G, 4);
}

// Automatic lane counts of the host-driven path, from sweeps on the grid,
// layered and R-MAT families: graphs with hub vertices (a vertex other than
// s and t of degree above 64 times the average) discharge and expand with 32
// lanes; otherwise a discharge uses 4 lanes up to an average degree of 12
// (more lanes per vertex mean fewer vertices per wave, and the passes over a
// vertex's slots are short), and a top-down BFS level 8 lanes (4 below an
// average degree of 4).
static void auto_lanes(const mf_dgraph *dg, int &G, int &Gb)
{
    const double avg = dg->n > 0 ? (double)dg->slots / (double)dg->n : 1.0;
    if ((double)dg->maxdeg_inner > 64.0 * std::max(1.0, avg)) {
        G = 32;
        Gb = 32;
        return;
    }
    if (avg <= 12.0) {
        G = 4;
    } else {
        G = 4;
        while (G < avg / 2 && G < 32) G <<= 1;
    }
    Gb = avg <= 4.0 ? 4 : 8;
}

struct Solve {
    mf_context *ctx;
    const mf_dgraph *dg;
    GraphView g;
    StateView st;
    mf_options opt;
    int G, Gm, Gb;             // lanes per vertex: discharge, merge, top-down BFS level
    int hubd;                  // round vertices above this degree go to the hub kernels (a block each)
    bool hub_kernels;          // some vertex other than s and t exceeds hubd
    int hub_grid;
    int maxgrid;
    int rgrid;                 // cap on the grids of the round kernels (discharge, merge, flag compaction)
    int64_t avg_deg_ceil;
    int64_t dense_threshold;   // working sets larger than this run in dense mode
    int64_t bu_factor;         // bottom-up BFS level when frontier * bu_factor > unvisited
    int64_t gr_depth = 0;      // depth of the last global relabel
    int64_t td_slots = 0;      // profiling: slots expanded by top-down levels
    int hubdeg;                // frontier vertices above this degree are expanded by the grid
    bool profile;
    uint32_t pmask;            // kernels (bits of mf_kernel_id) timed with events under MF_PROFILE
    bool persistent;
    bool check;                // MF_CHECK_INVARIANTS: state checks after every round and global relabel
    int block_small_max;       // working sets up to this size run their rounds in one workgroup (0 = never)
    bool gap;                  // MF_GAP_RELABEL: the gap rule after every round
    // the discharge kernels that keep two chunks of slots in registers: used
    // when every vertex other than s and t has more than G and at most 2G
    // slots (the 3D grid at 4 lanes); they cost registers, and occupancy,
    // that other graphs do not repay
    bool two_chunks = false;
    bool fault_done = false;   // the check_fault_round test hook has fired
    // profiling accumulators
    double ms_dis = 0, ms_mer = 0, ms_gr = 0, ms_phase = 0;
    int64_t n_dis = 0, n_mer = 0, n_gr = 0, n_phase = 0;
    int64_t dense_rounds = 0, bu_levels = 0, td_levels = 0, grs = 0;
    double kms[MF_K_COUNT] = {};         // per kernel: event time, launches, algorithmic bytes
    int64_t kn[MF_K_COUNT] = {}, kb[MF_K_COUNT] = {};
    int64_t kt[MF_K_COUNT] = {};         // launches in kms
    int64_t kissue[MF_K_COUNT] = {};     // launches issued, for the sampling stride
    int64_t stride = 1;                  // time every stride-th launch of a timed kernel
    std::vector<hipEvent_t> rec;         // start events of sampled launches not yet read
    Ctl last;                            // counters at the previous readback
};

// ms < 0: the launch was not sampled for timing (only its count and bytes).
static void kernel_record(Solve &S, int k, double ms, int64_t bytes)
{
    if (ms >= 0) {
        S.kms[k] += ms;
        S.kt[k]++;
    }
    S.kn[k]++;
    S.kb[k] += bytes;
}
static double timed_ms(double ms) { return ms > 0 ? ms : 0.0; }

// Algorithmic bytes of the rounds since the last readback: discharge, hub
// discharge, merge, hub merge (the per-unit model of mf_kernel_id).
static void round_bytes(const Solve &S, const Ctl &c, int64_t b[4])
{
    const Ctl &l = S.last;
    const int64_t p = c.pushes - l.pushes, ph = c.dh_pushes - l.dh_pushes;
    b[0] = 40 * (c.dverts - l.dverts) + 13 * (c.dslots - l.dslots) + 16 * (p - ph);
    b[1] = 40 * (c.dh_verts - l.dh_verts) + 13 * (c.dh_slots - l.dh_slots) + 16 * ph;
    b[2] = 41 * (c.mverts - l.mverts) + 4 * (c.mslots - l.mslots) + 12 * p;
    b[3] = 41 * (c.mh_verts - l.mh_verts) + 4 * (c.mh_slots - l.mh_slots);
}

static float elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms;
}

// With MF_PROFILE, launches of the kernels in the profile mask are bracketed
// by HIP events (an event costs device time, so a caller that times a solve
// can restrict them to the kernel it studies); bytes and launch counts are
// kept for every kernel.
static bool timed(const Solve &S, int kind) { return S.profile && ((S.pmask >> kind) & 1u); }
// ev: an event array (read only when the kernel is timed); the launch records
// ev[i] and ev[i+1] from its own dispatch.
// Every stride-th launch of a timed kernel is sampled.
static KEv kev(Solve &S, int kind, const hipEvent_t *ev, int i)
{
    KEv k;
    if (timed(S, kind) && S.kissue[kind]++ % S.stride == 0) {
        k.a = ev[i];
        k.b = ev[i + 1];
        S.rec.push_back(ev[i]);
    }
    return k;
}
// Duration of the launch that recorded ev[a] and ev[b], or -1 if it was not
// sampled.
static double span(Solve &S, int kind, const hipEvent_t *ev, int a, int b)
{
    if (!timed(S, kind)) return -1.0;
    auto it = std::find(S.rec.begin(), S.rec.end(), ev[a]);
    if (it == S.rec.end()) return -1.0;
    S.rec.erase(it);
    return (double)elapsed(ev[a], ev[b]);
}

// Working-set representation for the next round: a list for small sets, the
// activity flags for large ones.  `count` is the size of the new set; when a
// list is needed and the last step left only flags, they are compacted.
static void prepare_working_set(Solve &S, int count, bool have_list, bool &dense)
{
    dense = (int64_t)count > S.dense_threshold;
    if (!dense && !have_list) {
        (void)hipMemsetAsync(&S.ctx->ctl->na, 0, sizeof(int32_t), S.ctx->stream);
        launch_compact_flags(S.st.act, S.g.n, S.st.A, &S.ctx->ctl->na, S.rgrid, S.ctx->stream);
    }
}

// Events for per-kernel times inside a batch of speculative levels.
static mf_status batch_events(mf_context *ctx, size_t count)
{
    while (ctx->lev.size() < count) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return fail(ctx, MF_EDEVICE, "hipEventCreate failed");
        ctx->lev.push_back(e);
    }
    return MF_OK;
}

// Flags of a top-down level (the TD_* flags of the kernel): degree tracking
// on graphs with hubs, and eager reverse-residual reads for frontiers small
// enough that the level is latency-bound.
static int td_flags(bool track_deg, int64_t nq)
{
    constexpr int64_t EAGER_MAX = 16384;
    return (track_deg ? 1 : 0) | (nq <= EAGER_MAX ? 4 : 0);
}

// MF_CHECK_INVARIANTS: checks the state between rounds (k_check_state).
static mf_status check_state(Solve &S, int sink, int other, bool after_gr, int64_t rounds)
{
    mf_context *ctx = S.ctx;
    const bool phase1 = sink == S.dg->t;
    if (phase1 && !S.fault_done && S.opt.check_fault_round > 0 && rounds >= S.opt.check_fault_round &&
        S.g.slots > 0) {
        launch_bump(S.st.res, ctx->stream);      // test hook: break the state once
        S.fault_done = true;
    }
    HIPCHK(ctx, hipMemsetAsync(&ctx->ctl->inv_err, 0, sizeof(int32_t), ctx->stream));
    launch_check_state(S.g, S.st, sink, other, after_gr ? 1 : 0, grid_for(S.g.n, 256, S.maxgrid), ctx->stream);
    mf_status st = read_ctl(ctx);
    if (st != MF_OK) return st;
    const int bits = ctx->ctl_host->inv_err;
    if (!bits) return MF_OK;
    static const char *what[] = {"a residual below 0", "res[a] + res[rev a] != cap[a] + cap[rev a]",
                                 "a push pending between rounds", "an excess != the net inflow of its residuals",
                                 "an excess below 0 off s", "a label out of range or on a terminal",
                                 "d(v) > d(w) + 1 on a residual arc after a global relabel",
                                 "a touched mark left set"};
    int k = 0;
    while (!((bits >> k) & 1)) k++;
    return fail(ctx, MF_EINVARIANT, "invariant broken in phase %d after %lld rounds%s: %s (bits 0x%x)",
                phase1 ? 1 : 2, (long long)rounds, after_gr ? " and a global relabel" : "", what[k], bits);
}

static mf_status global_relabel(Solve &S, int sink, int other, PhaseStats &ps, int &na, bool &dense)
{
    mf_context *ctx = S.ctx;
    const int n = S.g.n;
    launch_gr_init(S.g, S.st, sink, grid_for(std::max<int64_t>(n, S.g.slots), 256, S.maxgrid), ctx->stream);
    int64_t nq = 1;
    int64_t unvisited = n - 2;
    std::vector<int> bu_lv;            // profiling: levels run bottom-up
    int64_t found_before = 0;          // gr_found at the last readback
    int level = 0;
    // Top-down levels launched per readback: 1 while the frontier grows
    // fast (the grid and the choice of a bottom-up level follow its size),
    // doubling up to a cap of 32 to 128 while it stays within a factor 2 of
    // the last one.
    int batch = 1;
    bool have_list = true;
    int32_t *qin = S.st.Q, *qout = S.st.Q2;
    const int groups = 256 / S.Gb;
    // A frontier holds the sink alone at level 0 and only vertices other
    // than s and t later, so the hub expansion runs only where one of them
    // can exceed the hub degree.
    const int deg_sink = sink == S.dg->s ? S.dg->deg_s : S.dg->deg_t;
    const bool hub_first = deg_sink > S.hubdeg;
    const bool hub_later = S.dg->maxdeg_inner > S.hubdeg;
    // Direction choice: a level runs bottom-up when its frontier holds more
    // than 1/bu_factor of the unvisited vertices, or, in graphs with hub
    // vertices, when the frontier's slots exceed 1/14 of the slots of the
    // unvisited vertices (a few frontier vertices of very high degree).
    int64_t fdeg = deg_sink;                       // slots of the current frontier
    int64_t unexplored = S.g.slots - deg_sink;     // slots of the vertices not yet labelled
    while (nq > 0) {
        const bool bottom_up = nq * S.bu_factor > unvisited || (hub_later && fdeg * 14 > unexplored);
        if (!bottom_up && have_list) {
            // A batch of top-down levels with one readback at its end; the
            // levels after the one that empties the frontier return at once.
            const int K = batch;
            const int grid = grid_for(K == 1 ? nq : std::max<int64_t>(4 * nq, 2048), groups, S.maxgrid);
            // launches, with their kinds for the profile; events lev[2i] and
            // lev[2i+1] bracket launch i
            int nl = 0;
            int kinds[2 * 128];
            if (S.profile) {
                mf_status est = batch_events(ctx, 4 * 128);
                if (est != MF_OK) return est;
            }
            const int tdf = td_flags(hub_later, nq);
            for (int j = 0; j < K; j++) {
                const int L = level + j;
                launch_gr_td(S.Gb, S.g, S.st, L, sink, other, qin, qout, S.hubdeg, tdf, grid, ctx->stream,
                       kev(S, MF_K_GR_TOPDOWN, ctx->lev.data(), 2 * nl));
                kinds[nl++] = MF_K_GR_TOPDOWN;
                if (L == 0 ? hub_first : hub_later) {
                    launch_gr_hub(S.g, S.st, L, sink, other, qout, hub_later, ctx->num_cus * 2, ctx->stream,
                           kev(S, MF_K_GR_HUB, ctx->lev.data(), 2 * nl));
                    kinds[nl++] = MF_K_GR_HUB;
                }
                std::swap(qin, qout);
            }
            mf_status st = read_ctl(ctx);
            if (st != MF_OK) return st;
            const Ctl &c = *ctx->ctl_host;
            const bool ended = c.bfs_empty_level < level + K;
            const int ran = ended ? c.bfs_empty_level - level : K;   // levels with a non-empty frontier
            // each level adds its frontier size to gr_found, so the batch
            // labelled the sum of its frontiers less the first plus the next
            const int64_t frontier = c.gr_found - found_before;
            const int64_t nq_next = ended ? 0 : c.nq[(level + K) % 3];
            const int64_t found = frontier - nq + nq_next;
            if (S.profile) {
                // bytes by the model of each kernel (the slots the levels
                // expanded are added once the relabel is done)
                int64_t td_bytes = 12 * frontier + 8 * found;
                int64_t hub_bytes = 12 * (c.hslots - S.last.hslots);
                for (int i = 0; i < nl; i++) {
                    const int k = kinds[i];
                    int64_t b = 0;
                    if (k == MF_K_GR_TOPDOWN) { b = td_bytes; td_bytes = 0; }
                    else { b = hub_bytes; hub_bytes = 0; }
                    const double ms = span(S, k, ctx->lev.data(), 2 * i, 2 * i + 1);
                    kernel_record(S, k, ms, b);
                    S.ms_gr += timed_ms(ms);
                }
                S.n_gr += ran;
                S.last = c;
            }
            S.td_levels += ran;
            unvisited -= found;
            found_before = c.gr_found;
            unexplored = S.g.slots - deg_sink - c.gr_found_deg;
            fdeg = ended ? 0 : c.fdeg[(level + K) % 3];
            level += ran;
            // the cap grows with the depth reached (32 up to level 128, 128 from
            // level 512): a deep search saves readbacks, and a shallow one
            // launches few empty levels after its frontier runs out
            const int cap = (int)std::min<int64_t>(128, std::max<int64_t>(32, level / 4));
            batch = nq_next > 2 * nq ? 1 : std::min(cap, 2 * batch);
            nq = nq_next;
            continue;
        }
        // one level at a time: bottom-up, or top-down after a bottom-up level
        const bool hubs = level == 0 ? hub_first : hub_later;
        if (bottom_up) {
            S.bu_levels++;
            if (S.profile) bu_lv.push_back(level);
            launch_gr_bu(S.g, S.st, level, sink, other, grid_for(n, 256, S.maxgrid), ctx->stream,
                   kev(S, MF_K_GR_BOTTOMUP, ctx->pev, 4));
            have_list = false;
        } else {
            S.td_levels++;
            HIPCHK(ctx, hipMemsetAsync(&ctx->ctl->nq[(level + 2) % 3], 0, sizeof(int32_t), ctx->stream));
            launch_gr_collect(S.g, S.st, level, qin, grid_for(n, 256, S.maxgrid), ctx->stream);
            launch_gr_td(S.Gb, S.g, S.st, level, sink, other, qin, qout, S.hubdeg, td_flags(hub_later, nq),
                         grid_for(nq, groups, S.maxgrid), ctx->stream,
                   kev(S, MF_K_GR_TOPDOWN, ctx->pev, 4));
            if (hubs) {
                launch_gr_hub(S.g, S.st, level, sink, other, qout, hub_later, ctx->num_cus * 2, ctx->stream,
                       kev(S, MF_K_GR_HUB, ctx->pev, 6));
            }
            std::swap(qin, qout);
            have_list = true;
        }
        mf_status st = read_ctl(ctx);
        if (st != MF_OK) return st;
        const Ctl &c = *ctx->ctl_host;
        const int64_t found = c.nq[(level + 1) % 3];
        if (S.profile) {
            S.n_gr++;
            const int64_t gs = c.gslots - S.last.gslots;
            if (bottom_up) {
                const double ms = span(S, MF_K_GR_BOTTOMUP, ctx->pev, 4, 5);
                S.ms_gr += timed_ms(ms);
                kernel_record(S, MF_K_GR_BOTTOMUP, ms, 4 * (int64_t)n + 8 * unvisited + 12 * gs + 8 * found);
            } else {
                const double ms_td = span(S, MF_K_GR_TOPDOWN, ctx->pev, 4, 5);
                S.ms_gr += timed_ms(ms_td);
                kernel_record(S, MF_K_GR_TOPDOWN, ms_td, 12 * nq + 8 * found);
                if (hubs) {
                    const int64_t nh = c.nh[level % 3];
                    const double ms_h = span(S, MF_K_GR_HUB, ctx->pev, 6, 7);
                    S.ms_gr += timed_ms(ms_h);
                    kernel_record(S, MF_K_GR_HUB, ms_h, 12 * nh + 12 * (c.hslots - S.last.hslots));
                }
            }
            S.last = c;
        }
        found_before = c.gr_found;
        unexplored = S.g.slots - deg_sink - c.gr_found_deg;
        fdeg = c.fdeg[(level + 1) % 3];
        nq = found;
        unvisited -= nq;
        level++;
    }
    ps.levels += level - 1;
    S.gr_depth = level - 1;
    ps.grs++;
    S.grs++;
    if (S.profile) {
        // slots expanded by the top-down levels: those of the labelled
        // vertices, less those whose level ran bottom-up
        const int grid = grid_for(n, 256, S.maxgrid);
        HIPCHK(ctx, hipMemsetAsync(&ctx->ctl->td_slots, 0, sizeof(int64_t), ctx->stream));
        LevelSet all{};
        launch_gr_slots(S.g, S.st.d, S.hubdeg, all, &ctx->ctl->td_slots, grid, ctx->stream);
        for (size_t i = 0; i < bu_lv.size(); i += 15) {
            LevelSet part{};
            for (size_t k = i; k < bu_lv.size() && k < i + 15; k++) part.lv[part.count++] = bu_lv[k];
            launch_gr_slots(S.g, S.st.d, S.hubdeg, part, &ctx->ctl->td_slots, grid, ctx->stream);
        }
    }
    launch_gr_rebuild(S.g, S.st, sink, other, grid_for(n, 256, S.maxgrid), ctx->stream);
    if (S.gap) launch_gap_recount(S.g, S.st, sink, other, grid_for(n, 256, S.rgrid), ctx->stream);
    mf_status st = read_ctl(ctx);
    if (st != MF_OK) return st;
    if (S.profile) {
        // a top-down slot reads its packed head (4 B) and, for an open arc,
        // the neighbour's label (4 B): 8 B counted per slot; without packed
        // heads (head, reverse index, reverse residual, label) 16 B
        S.kb[MF_K_GR_TOPDOWN] += (S.st.hr ? 8 : 16) * ctx->ctl_host->td_slots;
        S.td_slots += ctx->ctl_host->td_slots;
        S.last = *ctx->ctl_host;
    }
    na = ctx->ctl_host->na2;
    prepare_working_set(S, na, false, dense);
    return MF_OK;
}

// One phase of the synchronous loop toward `sink`.  Returns MF_ETIMEOUT when
// the round limit stops it.
static mf_status run_phase(Solve &S, int sink, int other, int64_t max_rounds, PhaseStats &ps)
{
    mf_context *ctx = S.ctx;
    const int64_t n = S.g.n, m = S.g.slots;
    const mf_options &o = S.opt;
    const RoundParams rp{o.gr_beta, sink, S.hubd, (o.flags & MF_SIMPLE_ROUNDS) ? 1 : 0};
    bool force = true;
    int64_t W = 0;
    int na = 0;
    bool dense = false;
    int rbatch = 1;              // list rounds per readback: doubles up to 16 while no round stops a batch
    int dbatch = 1;              // dense rounds per readback: doubles up to 8 likewise
    bool list_ready = false;     // the working set is listed in A (else only flagged in act)
    int64_t checked = 0;         // MF_CHECK_INVARIANTS: rounds whose end state was checked
    while (true) {
        if (S.check && ps.rounds > checked) {
            mf_status st = check_state(S, sink, other, false, ps.rounds);
            if (st != MF_OK) return st;
            checked = ps.rounds;
        }
        bool just = false;
        const int64_t gr_thr = o.gr_alpha * n + m + o.gr_level_charge * S.gr_depth;
        if (force || o.gr_freq_num * W > o.gr_freq_den * gr_thr) {
            mf_status st = global_relabel(S, sink, other, ps, na, dense);
            if (st != MF_OK) return st;
            if (S.check && (st = check_state(S, sink, other, true, ps.rounds)) != MF_OK) return st;
            list_ready = !dense;     // a list-mode working set was compacted from the flags
            rbatch = 1;
            W = 0;
            force = false;
            just = true;
        }
        if (na == 0) {
            if (just) return MF_OK;
            force = true;
            continue;
        }
        if (max_rounds > 0 && ps.rounds >= max_rounds) return MF_ETIMEOUT;
        if (!dense && na <= S.block_small_max) {
            // a small working set: its rounds inside one workgroup, until
            // one of them stops it as a stopped batch of list rounds
            // (at most 65,536 rounds per launch: the launch returns at a round
            // boundary and the host goes on from there)
            const int64_t budget = std::min<int64_t>(65536, max_rounds > 0 ? max_rounds - ps.rounds : INT64_MAX);
            if (S.profile) {
                mf_status est = batch_events(ctx, 2);
                if (est != MF_OK) return est;
            }
            launch_rounds_block(S.G, S.g, S.st, rp, other, W, o.gr_round_charge, o.gr_freq_num, o.gr_freq_den,
                                o.gr_alpha * n + m + o.gr_level_charge * S.gr_depth, S.dense_threshold,
                                S.block_small_max, budget, ctx->stream, kev(S, MF_K_BLOCK_ROUNDS, ctx->lev.data(), 0));
            mf_status st = read_ctl(ctx);
            if (st != MF_OK) return st;
            const Ctl &c = *ctx->ctl_host;
            const int r = c.batch_rounds;
            W = c.batch_W;
            ps.rounds += r;
            if ((r - 1) & 1) std::swap(S.st.A, S.st.A2);   // the rounds before the stopping one
            if (S.profile) {
                int64_t b[4];
                round_bytes(S, c, b);
                const double ms = span(S, MF_K_BLOCK_ROUNDS, ctx->lev.data(), 0, 1);
                kernel_record(S, MF_K_BLOCK_ROUNDS, ms, b[0] + b[2]);
                S.ms_dis += timed_ms(ms);
                S.n_dis += r;
                S.n_mer += r;
                S.last = c;
            }
            const int count = c.na2;
            dense = count > S.dense_threshold;
            launch_round_end(ctx->ctl, ctx->stream);   // na = na2
            std::swap(S.st.A, S.st.A2);
            list_ready = true;
            na = count;
            rbatch = 1;
            continue;
        }
        if (!dense) {
            // Speculative list rounds: up to `rbatch` rounds with one readback;
            // the round that must be followed by a global relabel, a dense
            // round or an empty working set stops the rest.
            int K = rbatch;
            if (max_rounds > 0) K = (int)std::min<int64_t>(K, max_rounds - ps.rounds);
            const int groups = 256 / S.G;
            const int dgrid = grid_for(std::min<int64_t>(S.dense_threshold, 4 * (int64_t)na + 2048), groups,
                                       S.rgrid);
            const int mgrid = grid_for(std::min<int64_t>(S.dense_threshold, 4 * (int64_t)na + 2048) *
                                           (1 + S.avg_deg_ceil), 256 / S.Gm, S.rgrid);
            if (S.profile) {
                mf_status est = batch_events(ctx, 8 * 16);
                if (est != MF_OK) return est;
            }
            // events 8j .. 8j+7 bracket the discharge, hub discharge, merge and
            // hub merge of round j (the hub pairs stay empty without hubs)
            StateView sj = S.st;
            for (int j = 0; j < K; j++) {
                const hipEvent_t *e = ctx->lev.data();
                const int q = 8 * j;
                if (j == 0) launch_round_begin(ctx->ctl, 1, ctx->stream);
                launch_discharge(S.G, false, S.g, sj, rp, dgrid, ctx->stream,
                       kev(S, MF_K_DISCHARGE_LIST, e, q + 0), S.two_chunks);
                if (S.hub_kernels) {
                    launch_discharge_hubs(false, S.g, sj, rp, S.hub_grid, ctx->stream,
                           kev(S, MF_K_DISCHARGE_HUB, e, q + 2));
                }
                launch_merge(S.Gm, false, S.g, sj, sink, other, S.hubd, mgrid, ctx->stream,
                       kev(S, MF_K_MERGE_LIST, e, q + 4));
                if (S.hub_kernels) {
                    launch_merge_hubs(false, S.g, sj, sink, other, S.hub_grid, ctx->stream,
                           kev(S, MF_K_MERGE_HUB, e, q + 6));
                }
                if (S.gap) launch_gap_round(S.g, sj, sink, other, 0, S.rgrid, ctx->stream);
                launch_round_close(ctx->ctl, j == 0, W, o.gr_round_charge, o.gr_freq_num, o.gr_freq_den,
                                   o.gr_alpha * n + m + o.gr_level_charge * S.gr_depth, S.dense_threshold,
                                   ctx->stream);
                std::swap(sj.A, sj.A2);
            }
            mf_status st = read_ctl(ctx);
            if (st != MF_OK) return st;
            const Ctl &c = *ctx->ctl_host;
            const int r = c.batch_rounds;
            const bool stopped = c.batch_stop != 0;
            W = c.batch_W;
            ps.rounds += r;
            if ((stopped ? r - 1 : r) & 1) std::swap(S.st.A, S.st.A2);   // rounds the device closed
            if (S.profile) {
                int64_t b[4];
                round_bytes(S, c, b);
                for (int j = 0; j < K; j++) {
                    const hipEvent_t *e = ctx->lev.data();
                    const int q = 8 * j;
                    const double md = span(S, MF_K_DISCHARGE_LIST, e, q, q + 1);
                    const double mm = span(S, MF_K_MERGE_LIST, e, q + 4, q + 5);
                    kernel_record(S, MF_K_DISCHARGE_LIST, md, j == 0 ? b[0] : 0);
                    kernel_record(S, MF_K_MERGE_LIST, mm, j == 0 ? b[2] : 0);
                    S.ms_dis += timed_ms(md);
                    S.ms_mer += timed_ms(mm);
                    if (S.hub_kernels) {
                        const double hd = span(S, MF_K_DISCHARGE_HUB, e, q + 2, q + 3);
                        const double hm = span(S, MF_K_MERGE_HUB, e, q + 6, q + 7);
                        kernel_record(S, MF_K_DISCHARGE_HUB, hd, j == 0 ? b[1] : 0);
                        kernel_record(S, MF_K_MERGE_HUB, hm, j == 0 ? b[3] : 0);
                        S.ms_dis += timed_ms(hd);
                        S.ms_mer += timed_ms(hm);
                    }
                }
                S.n_dis += K;
                S.n_mer += K;
                S.last = c;
            }
            if (!stopped) {
                list_ready = true;
                na = c.na;
                rbatch = S.check ? 1 : std::min(16, 2 * rbatch);
                continue;
            }
            // the round that stopped the batch: its merge listed the next
            // working set in A2
            const int count = c.na2;
            dense = count > S.dense_threshold;
            launch_round_end(ctx->ctl, ctx->stream);   // na = na2
            std::swap(S.st.A, S.st.A2);
            list_ready = true;
            na = count;
            continue;
        }
        // Dense rounds, speculatively batched like the list rounds: up to
        // `dbatch` rounds with one readback.  Each round: the working set as
        // a list (the previous round's merge wrote it; after a global relabel
        // it is listed from the activity flags), discharge of the listed
        // vertices, list of the touched vertices, their merge, and a
        // one-thread close that stops the batch when the next round must not
        // be a dense round (working set at or below the dense threshold) or
        // W calls for a global relabel.  Every kernel of a later round then
        // returns at once.
        rbatch = 1;
        int K = dbatch;
        if (max_rounds > 0) K = (int)std::min<int64_t>(K, max_rounds - ps.rounds);
        launch_round_reset(ctx->ctl, !list_ready, ctx->stream);
        const int groups = 256 / S.G;
        const int64_t na_room = K == 1 ? (int64_t)na : 2 * (int64_t)na;      // later rounds may grow
        const int dgrid = grid_for(na_room, groups, S.rgrid);
        const int mgrid = grid_for(std::min<int64_t>(n, na_room * (1 + S.avg_deg_ceil)), 256 / S.Gm, S.rgrid);
        if (S.profile) {
            mf_status est = batch_events(ctx, 12 * 8);
            if (est != MF_OK) return est;
        }
        // events 12j .. 12j+11 bracket round j's compaction of the working
        // set, discharge, hub discharge, compaction of the touched vertices,
        // merge and hub merge
        const bool compact_first = !list_ready;
        StateView sj = S.st;
        for (int j = 0; j < K; j++) {
            const hipEvent_t *e = ctx->lev.data() + 12 * j;
            if (j == 0 && compact_first) {
                launch_compact_flags(sj.act, (int)n, sj.A, &ctx->ctl->na, S.rgrid, ctx->stream,
                       kev(S, MF_K_COMPACT, e, 0));
            }
            launch_discharge(S.G, true, S.g, sj, rp, dgrid, ctx->stream,
                   kev(S, MF_K_DISCHARGE_DENSE, e, 2), S.two_chunks);
            if (S.hub_kernels) {
                launch_discharge_hubs(true, S.g, sj, rp, S.hub_grid, ctx->stream,
                       kev(S, MF_K_DISCHARGE_HUB, e, 4));
            }
            launch_compact_flags(sj.touched, (int)n, sj.C, &ctx->ctl->nc, S.rgrid, ctx->stream,
                   kev(S, MF_K_COMPACT, e, 6), &ctx->ctl->batch_stop);
            launch_merge(S.Gm, true, S.g, sj, sink, other, S.hubd, mgrid, ctx->stream,
                   kev(S, MF_K_MERGE_DENSE, e, 8));
            if (S.hub_kernels) {
                launch_merge_hubs(true, S.g, sj, sink, other, S.hub_grid, ctx->stream,
                       kev(S, MF_K_MERGE_HUB, e, 10));
            }
            if (S.gap) launch_gap_round(S.g, sj, sink, other, 1, S.rgrid, ctx->stream);
            launch_round_close(ctx->ctl, j == 0, W, o.gr_round_charge, o.gr_freq_num, o.gr_freq_den,
                               o.gr_alpha * n + m + o.gr_level_charge * S.gr_depth, S.dense_threshold,
                               ctx->stream, 1);
            std::swap(sj.A, sj.A2);
        }
        mf_status st = read_ctl(ctx);
        if (st != MF_OK) return st;
        const Ctl &c = *ctx->ctl_host;
        const int r = c.batch_rounds;
        const bool stopped = c.batch_stop != 0;
        W = c.batch_W;
        ps.rounds += r;
        S.dense_rounds += r;
        if (S.profile) {
            int64_t b[4];
            round_bytes(S, c, b);
            for (int j = 0; j < K; j++) {
                const hipEvent_t *e = ctx->lev.data() + 12 * j;
                const bool ran = j < r;       // rounds after the stop returned at once
                const double md = span(S, MF_K_DISCHARGE_DENSE, e, 2, 3);
                const double mm = span(S, MF_K_MERGE_DENSE, e, 8, 9);
                S.ms_dis += timed_ms(md);
                S.ms_mer += timed_ms(mm);
                if (j == 0 && compact_first)
                    kernel_record(S, MF_K_COMPACT, span(S, MF_K_COMPACT, e, 0, 1), n + 4 * (int64_t)na);
                kernel_record(S, MF_K_DISCHARGE_DENSE, md, j == 0 ? b[0] : 0);
                // the touched-list compaction reads n flags per round it ran
                kernel_record(S, MF_K_COMPACT, span(S, MF_K_COMPACT, e, 6, 7), ran ? n : 0);
                kernel_record(S, MF_K_MERGE_DENSE, mm, j == 0 ? b[2] : 0);
                if (S.hub_kernels) {
                    kernel_record(S, MF_K_DISCHARGE_HUB, span(S, MF_K_DISCHARGE_HUB, e, 4, 5), j == 0 ? b[1] : 0);
                    kernel_record(S, MF_K_MERGE_HUB, span(S, MF_K_MERGE_HUB, e, 10, 11), j == 0 ? b[3] : 0);
                }
            }
            S.n_dis += K;
            S.n_mer += K;
            S.last = c;
        }
        // the rounds the device closed each made the next working set current
        if ((stopped ? r - 1 : r) & 1) std::swap(S.st.A, S.st.A2);
        list_ready = true;
        if (!stopped) {
            na = c.na;
            dbatch = S.check ? 1 : std::min(8, 2 * dbatch);
            continue;
        }
        // the round that stopped the batch: its merge listed the next
        // working set in A2
        dbatch = 1;
        const int count = c.na2;
        dense = count > S.dense_threshold;
        launch_round_end(ctx->ctl, ctx->stream);   // na = na2
        std::swap(S.st.A, S.st.A2);
        na = count;
    }
}

// One phase as a single persistent cooperative kernel.
static mf_status run_phase_persistent(Solve &S, int sink, int other, int64_t max_rounds, PhaseStats &ps,
                                      int64_t cum[8])
{
    mf_context *ctx = S.ctx;
    const mf_options &o = S.opt;
    HIPCHK(ctx, hipMemsetAsync(ctx->ctl + 1, 0, 4 * sizeof(Ctl), ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(ctx->bar, 0, sizeof(GridBar), ctx->stream));
    PhaseParams P;
    P.sink = sink;
    P.other = other;
    P.freq_num = o.gr_freq_num;
    P.freq_den = o.gr_freq_den;
    P.alpha = o.gr_alpha;
    P.beta = o.gr_beta;
    P.round_charge = o.gr_round_charge;
    P.level_charge = o.gr_level_charge;
    P.max_rounds = max_rounds;
    P.dense_threshold = S.dense_threshold;
    P.bu_factor = S.bu_factor;
    P.hubdeg = 64 * S.G;          // the phase kernel expands frontier vertices with G lanes
    P.simple = (o.flags & MF_SIMPLE_ROUNDS) ? 1 : 0;
    P.limit_ticks = ctx->wall_hz * 30ull;      // 30 s: far above any single step
    int per_cu = phase_blocks_per_cu(S.G);
    if (per_cu <= 0) return fail(ctx, MF_EDEVICE, "occupancy query for the persistent kernel failed");
    if (o.blocks_per_cu > 0) per_cu = std::min(per_cu, (int)o.blocks_per_cu);
    const int grid = per_cu * ctx->num_cus;
    if (S.profile) HIPCHK(ctx, hipEventRecord(ctx->pev[0], ctx->stream));
    hipError_t e = launch_phase(S.G, grid, S.g, S.st, P, ctx->ctl + 1, ctx->ctl + 4, ctx->bar, ctx->stream);
    if (e != hipSuccess)
        return fail(ctx, MF_EDEVICE, "persistent kernel launch failed: %s", hipGetErrorString(e));
    if (S.profile) HIPCHK(ctx, hipEventRecord(ctx->pev[1], ctx->stream));
    mf_status st = read_ctl(ctx, 5);
    if (st != MF_OK) return st;
    if (S.profile) {
        S.ms_phase += elapsed(ctx->pev[0], ctx->pev[1]);
        S.n_phase++;
    }
    const Ctl *h = ctx->ctl_host;
    const Ctl &gc = h[4];
    if (gc.p_status == 2) return fail(ctx, MF_EDEVICE, "persistent kernel barrier timed out");
    ps.rounds += gc.p_rounds;
    ps.grs += gc.p_grs;
    ps.levels += gc.p_levels;
    S.dense_rounds += gc.p_dense_rounds;
    S.bu_levels += gc.p_bu_levels;
    S.grs += gc.p_grs;
    for (int i = 1; i <= 3; i++) {
        cum[0] += h[i].pushes;
        cum[1] += h[i].relabels;
        cum[2] += h[i].scans;
        cum[3] += h[i].dverts;
        cum[4] += h[i].dslots;
        cum[5] += h[i].mverts;
        cum[6] += h[i].mslots;
    }
    cum[7] += gc.gslots;
    return gc.p_status == 1 ? MF_ETIMEOUT : MF_OK;
}

// Helper contexts of the batched form's grid-wide solves (one per worker
// thread).
static mf_status ensure_helpers(mf_context *ctx, int count)
{
    while ((int)ctx->helpers.size() < count) {
        mf_context *h = nullptr;
        mf_status st = mf_context_create(ctx->device, 0, &h);
        if (st != MF_OK) return fail(ctx, st, "helper context: %s", g_global_err.c_str());
        ctx->helpers.push_back(h);
    }
    return MF_OK;
}

static mf_status ensure_batch_streams(mf_context *ctx)
{
    for (auto &bs : ctx->bstream)
        if (!bs) HIPCHK(ctx, hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
    if (!ctx->lstream) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->lstream, hipStreamNonBlocking));
    for (auto &ev : ctx->gev)
        if (!ev) HIPCHK(ctx, hipEventCreate(&ev));
    for (auto &ev : ctx->bev)
        if (!ev) HIPCHK(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    return MF_OK;
}

static mf_status check_options(mf_context *ctx, const mf_options *o)
{
    if (o->gr_freq_den <= 0 || o->gr_freq_num < 0 || o->gr_alpha < 0 || o->gr_beta < 0 ||
        o->gr_round_charge < 0 || o->gr_level_charge < 0 || o->max_rounds < 0)
        return fail(ctx, MF_EINVAL, "invalid global-relabel schedule");
    if (o->lanes_per_vertex < 0 || o->lanes_per_vertex > 64 || o->lanes_per_merge < 0 ||
        o->lanes_per_merge > 64 || o->lanes_per_bfs < 0 || o->lanes_per_bfs > 64)
        return fail(ctx, MF_EINVAL, "lane counts must be 0..64");
    if (o->profile_stride < 0)
        return fail(ctx, MF_EINVAL, "profile_stride must be >= 0");
    if (o->bfs_bottom_up_factor < 0)
        return fail(ctx, MF_EINVAL, "bfs_bottom_up_factor must be >= 0");
    return MF_OK;
}

// A small graph solved by one workgroup in a single launch: the batched
// form's kernel on one instance, over the context's workspace.  Its rounds
// are those of the grid-wide path (each round is a function of its start
// state), without a host round trip per round or level.
static mf_status solve_small(mf_context *ctx, mf_dgraph *dg, const mf_options &o, int64_t *value,
                             int32_t *flow_dev, uint8_t *side_dev, mf_stats *stats)
{
    const size_t oi = 0, orr = align256(sizeof(BatchItem)), oq = orr + align256(sizeof(BatchResult)),
                 oo = oq + align256(sizeof(BatchQueue)), total = oo + 256;
    if (!ctx->one) {
        mf_status st = dalloc(ctx, (void **)&ctx->one, total);
        if (st != MF_OK) return st;
    }
    Workspace &w = ctx->ws;
    std::vector<uint8_t> host(total, 0);
    BatchItem &it = *(BatchItem *)(host.data() + oi);
    it.g = dg->view();
    StateView &sv = it.st;
    sv.res = w.res;
    sv.delta = w.delta;
    sv.d = w.d;
    sv.dn = w.dn;
    sv.owner = w.owner;
    sv.e = w.e;
    sv.act = w.act;
    sv.touched = w.touched;
    sv.H = w.H;
    sv.A = w.A;
    sv.A2 = w.A2;
    sv.C = w.C;
    sv.Q = w.Q;
    sv.Q2 = w.Q2;
    it.ctl = ctx->ctl;
    it.flow = flow_dev;
    it.side = side_dev ? side_dev : w.side;
    it.G = batch_lanes(o.lanes_per_vertex, dg->n, dg->slots);
    it.preflow_only = (o.flags & MF_PREFLOW_ONLY) ? 1 : 0;
    PhaseParams &P = it.p;
    P.freq_num = o.gr_freq_num;
    P.freq_den = o.gr_freq_den;
    P.alpha = o.gr_alpha;
    P.beta = o.gr_beta;
    P.round_charge = o.gr_round_charge;
    P.level_charge = o.gr_level_charge;
    P.max_rounds = o.max_rounds;
    P.dense_threshold = o.dense_threshold > 0 ? o.dense_threshold : std::max<int64_t>(512, dg->n / 16);
    P.bu_factor = o.bfs_bottom_up_factor > 0 ? o.bfs_bottom_up_factor : 8;
    P.hubdeg = 64 * it.G;
    P.simple = (o.flags & MF_SIMPLE_ROUNDS) ? 1 : 0;
    P.limit_ticks = 0;
    BatchQueue &q = *(BatchQueue *)(host.data() + oq);
    q.next = 0;
    q.count = 1;
    uint8_t *dev = ctx->one;
    HIPCHK(ctx, hipMemcpyAsync(dev, host.data(), total, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipEventRecord(ctx->ev[0], ctx->stream));
    HIPCHK(ctx, launch_batch(it.G, 1, (const BatchItem *)(dev + oi), (const int32_t *)(dev + oo),
                             (BatchResult *)(dev + orr), (BatchQueue *)(dev + oq), ctx->stream));
    HIPCHK(ctx, hipEventRecord(ctx->ev[2], ctx->stream));
    BatchResult r;
    HIPCHK(ctx, hipMemcpyAsync(&r, dev + orr, sizeof r, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (r.status != 0 && r.status != 1) return fail(ctx, MF_EDEVICE, "single-workgroup solve failed (%d)", r.status);
    if (value) *value = r.value;
    if (stats) {
        memset(stats, 0, sizeof *stats);
        stats->value = r.value;
        stats->cut_capacity = r.cut;
        stats->rounds = r.rounds;
        stats->global_relabels = r.grs;
        stats->bfs_levels = r.levels;
        stats->rounds2 = r.rounds2;
        stats->global_relabels2 = r.grs2;
        stats->pushes = r.pushes;
        stats->relabels = r.relabels;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[2]);
        stats->ms_total = ms;
        stats->ms_preflow = 1e3 * (double)(r.t_phase1 - r.t_start) / (double)ctx->wall_hz;
        stats->ms_phase_kernel = ms;
        stats->phase_launches = 1;
        if (o.flags & MF_PROFILE) {
            stats->kernel_ms[MF_K_BLOCK_SOLVE] = ms;
            stats->kernel_timed[MF_K_BLOCK_SOLVE] = 1;
            stats->kernel_launches[MF_K_BLOCK_SOLVE] = 1;
        }
    }
    return r.status == 1 ? fail(ctx, MF_ETIMEOUT, "round limit %lld reached", (long long)o.max_rounds) : MF_OK;
}

static mf_status solve_uploaded(mf_context *ctx, mf_dgraph *dg, const mf_options *opt, int64_t *value,
                                int32_t *flow_dev, uint8_t *side_dev, mf_stats *stats, Workspace *ext = nullptr,
                                bool resume = false);

extern "C" mf_status mf_solve_uploaded(mf_context *ctx, mf_dgraph *dg, mf_stream stream, const mf_options *opt,
                                       int64_t *value, int32_t *flow_dev, uint8_t *side_dev,
                                       mf_stats *stats)
{
    if (!ctx || !dg) return fail(ctx, MF_EINVAL, "NULL context or graph");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    mf_status st = order_after(ctx, stream);
    if (st != MF_OK) return st;
    st = solve_uploaded(ctx, dg, opt, value, flow_dev, side_dev, stats);
    mf_status so = order_before(ctx, stream);
    return st == MF_OK ? so : st;
}

// ext: a workspace carved by the caller (the no-allocation entry point, the
// large instances of the batched and served forms); then nothing is
// allocated, the graph is always solved by the grid-wide kernels, and the
// context's resumable state is left alone.  resume (with ext): the
// workspace holds the residuals of a complete flow of this graph and e(t)
// its value (a resident graph of the server), and the solve continues from
// that flow as MF_WARM_START does.
static mf_status solve_uploaded(mf_context *ctx, mf_dgraph *dg, const mf_options *opt, int64_t *value,
                                int32_t *flow_dev, uint8_t *side_dev, mf_stats *stats, Workspace *ext,
                                bool resume)
{
    if (!ctx || !dg) return fail(ctx, MF_EINVAL, "NULL context or graph");
    mf_options o;
    if (opt)
        o = *opt;
    else
        mf_options_default(&o);
    mf_status st = check_options(ctx, &o);
    if (st != MF_OK) return st;
    const bool preflow_only = (o.flags & MF_PREFLOW_ONLY) != 0;
    if (preflow_only && flow_dev) return fail(ctx, MF_EINVAL, "flow output requires phase 2");
    if (resume) o.flags |= MF_WARM_START;
    const bool warm = (o.flags & MF_WARM_START) != 0;
    if (warm && !resume && ctx->warm_dg != dg)
        return fail(ctx, MF_EINVAL, "no resumable flow of this graph on this context (MF_WARM_START needs a "
                                    "complete solve of it as the context's last solve, and capacities that "
                                    "still hold its flow)");
    if ((o.flags & MF_CHECK_INVARIANTS) && (o.flags & MF_PERSISTENT))
        return fail(ctx, MF_EINVAL, "MF_CHECK_INVARIANTS runs the host-driven rounds: not with MF_PERSISTENT");
    if (ext && ((warm && !resume) || (o.flags & (MF_PROFILE | MF_GAP_RELABEL))))
        return fail(ctx, MF_EINVAL, "MF_WARM_START, MF_PROFILE and MF_GAP_RELABEL are not available without allocation");
    if ((o.flags & MF_GAP_RELABEL) && (o.flags & MF_PERSISTENT))
        return fail(ctx, MF_EINVAL, "MF_GAP_RELABEL runs the host-driven rounds: not with MF_PERSISTENT");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if (!ext) {
        ctx->warm_dg = nullptr;       // the workspace is about to change
        if ((st = ensure_workspace(ctx, dg->n, dg->slots)) != MF_OK) return st;
    }
    if (!ext && !warm && !(o.flags & (MF_PERSISTENT | MF_GRID_PATH | MF_CHECK_INVARIANTS | MF_GAP_RELABEL)) &&
        dg->n <= MF_SMALL_N &&
        dg->slots <= MF_SMALL_SLOTS)
        return solve_small(ctx, dg, o, value, flow_dev, side_dev, stats);

    Solve S;
    memset(&S.last, 0, sizeof S.last);
    S.ctx = ctx;
    S.dg = dg;
    S.g = dg->view();
    Workspace &w = ext ? *ext : ctx->ws;
    S.st.res = w.res;
    S.st.delta = w.delta;
    S.st.d = w.d;
    S.st.dn = w.dn;
    S.st.owner = w.owner;
    S.st.e = w.e;
    S.st.act = w.act;
    S.st.touched = w.touched;
    S.st.H = w.H;
    S.st.A = w.A;
    S.st.A2 = w.A2;
    S.st.C = w.C;
    S.st.Q = w.Q;
    S.st.Q2 = w.Q2;
    S.st.hr = w.hr;
    S.st.ctl = ctx->ctl;
    S.opt = o;
    {
        int Ga = 4, Gba = 8;
        auto_lanes(dg, Ga, Gba);
        S.G = o.lanes_per_vertex > 0 ? pick_lanes(o.lanes_per_vertex, 1, 1) : Ga;
        S.Gb = o.lanes_per_bfs > 0 ? pick_lanes(o.lanes_per_bfs, 1, 1) : Gba;
    }
    S.Gm = o.lanes_per_merge > 0 ? pick_lanes(o.lanes_per_merge, 1, 1) : S.G;
    S.maxgrid = ctx->num_cus * 16;
    // Round kernels end with one atomic per block on a few shared counters,
    // which serialize (about 12 ns each): at most 4 blocks per compute unit,
    // striding over the rest of the work.
    S.rgrid = ctx->num_cus * (!(o.flags & MF_PERSISTENT) && o.blocks_per_cu > 0 ? o.blocks_per_cu : 4);
    S.avg_deg_ceil = (dg->slots + dg->n - 1) / std::max<int64_t>(1, dg->n);
    S.dense_threshold = std::min<int64_t>(65536, std::max<int64_t>(2048, dg->n / 256));
    S.bu_factor = o.bfs_bottom_up_factor > 0 ? o.bfs_bottom_up_factor : 8;
    S.hubdeg = 64 * S.Gb;
    // Rounds discharge and merge vertices other than s and t only (a push
    // into s needs a label of n + 1 in the first phase, and the sink of a
    // phase takes its pushes directly).
    S.hub_kernels = dg->maxdeg_inner > 64 * S.G;
    S.hubd = S.hub_kernels ? 64 * S.G : 0x7fffffff;
    S.hub_grid = ctx->num_cus * 2;
    S.profile = (o.flags & MF_PROFILE) != 0;
    S.pmask = o.profile_mask ? o.profile_mask : 0xffffffffu;
    S.stride = o.profile_stride > 1 ? o.profile_stride : 1;
    S.persistent = (o.flags & MF_PERSISTENT) != 0;
    S.check = (o.flags & MF_CHECK_INVARIANTS) != 0;
    S.gap = (o.flags & MF_GAP_RELABEL) != 0;
    S.st.lcount = S.gap ? w.lcount : nullptr;
    S.st.gcand = S.gap ? w.gcand : nullptr;
    S.block_small_max = (o.block_round_max < 0 || S.check || S.hub_kernels || S.gap) ? 0
                        : (o.block_round_max > 0 ? o.block_round_max : 256);
    S.two_chunks = (S.G == 4 || S.G == 8) && !S.hub_kernels && dg->maxdeg_inner > S.G &&
                   dg->maxdeg_inner <= 2 * S.G;
    if (o.dense_threshold > 0) S.dense_threshold = o.dense_threshold;

    const int n = dg->n;
    HIPCHK(ctx, hipEventRecord(ctx->ev[0], ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(ctx->ctl, 0, sizeof(Ctl), ctx->stream));
    if (warm)
        launch_warm_state(S.g, S.st, grid_for(std::max<int64_t>(dg->slots, n), 256, S.maxgrid), ctx->stream);
    else
        launch_init_state(S.g, S.st, grid_for(std::max<int64_t>(dg->slots, n), 256, S.maxgrid), ctx->stream);
    launch_saturate(S.g, S.st, ctx->num_cus * 4, ctx->stream);
    launch_compact_flags(S.st.touched, n, S.st.C, &ctx->ctl->nc, S.rgrid, ctx->stream);
    launch_merge(S.Gm, true, S.g, S.st, dg->t, dg->s, S.hubd, grid_for(n, 256 / S.Gm, S.rgrid), ctx->stream);
    if (S.hub_kernels) launch_merge_hubs(true, S.g, S.st, dg->t, dg->s, S.hub_grid, ctx->stream);

    PhaseStats p1;
    int64_t cum[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // persistent-mode counters
    mf_status ph = S.persistent ? run_phase_persistent(S, dg->t, dg->s, o.max_rounds, p1, cum)
                                : run_phase(S, dg->t, dg->s, o.max_rounds, p1);
    if (ph != MF_OK && ph != MF_ETIMEOUT) return ph;
    const bool timed_out = ph == MF_ETIMEOUT;
    HIPCHK(ctx, hipEventRecord(ctx->ev[1], ctx->stream));
    if ((st = read_ctl(ctx)) != MF_OK) return st;
    const int64_t pushes = ctx->ctl_host->pushes + cum[0], relabels = ctx->ctl_host->relabels + cum[1],
                  scans = ctx->ctl_host->scans + cum[2];
    const int64_t lifts1 = ctx->ctl_host->gap_lifts;

    // value, sink side and cut capacity of the maximum preflow (the labels are
    // exact distances to t here)
    launch_read_value(w.e, dg->t, ctx->ctl, ctx->stream);
    uint8_t *side = side_dev ? side_dev : w.side;
    launch_side(S.g, w.d, side, grid_for(n, 256, S.maxgrid), ctx->stream);
    HIPCHK(ctx, hipMemsetAsync(&ctx->ctl->cut, 0, sizeof(int64_t), ctx->stream));
    launch_cut(S.g, side, ctx->ctl, grid_for(dg->slots, 256, S.maxgrid), ctx->stream);
    if ((st = read_ctl(ctx)) != MF_OK) return st;
    const int64_t val = ctx->ctl_host->value, cut = ctx->ctl_host->cut;

    PhaseStats p2;
    if (!preflow_only && !timed_out) {
        ph = S.persistent ? run_phase_persistent(S, dg->s, dg->t, 0, p2, cum)
                          : run_phase(S, dg->s, dg->t, 0, p2);
        if (ph != MF_OK) return ph;
    }
    if (flow_dev) launch_flow(S.g, w.res, flow_dev, grid_for(dg->slots, 256, S.maxgrid), ctx->stream);
    HIPCHK(ctx, hipEventRecord(ctx->ev[2], ctx->stream));
    if ((st = read_ctl(ctx)) != MF_OK) return st;
    HIPCHK(ctx, hipGetLastError());
    // a complete flow stays in the workspace for a resumed solve
    if (!ext && !preflow_only && !timed_out) ctx->warm_dg = dg;

    if (value) *value = val;
    if (stats) {
        memset(stats, 0, sizeof *stats);
        stats->value = val;
        stats->cut_capacity = cut;
        stats->rounds = p1.rounds;
        stats->global_relabels = p1.grs;
        stats->bfs_levels = p1.levels;
        stats->rounds2 = p2.rounds;
        stats->global_relabels2 = p2.grs;
        stats->pushes = pushes;
        stats->relabels = relabels;
        stats->arc_scans = scans;
        float ms1 = 0, ms2 = 0;
        (void)hipEventElapsedTime(&ms1, ctx->ev[0], ctx->ev[1]);
        (void)hipEventElapsedTime(&ms2, ctx->ev[0], ctx->ev[2]);
        stats->ms_preflow = ms1;
        stats->ms_total = ms2;
        stats->gap_lifts = lifts1;
        stats->gap_lifts2 = ctx->ctl_host->gap_lifts - lifts1;
        if (S.profile) {
            // Algorithmic bytes per unit of work:
            //  discharge: 40 B per discharged vertex (list entry or flag, two
            //    offsets, label, excess, new label and excess, touched mark),
            //    13 B per slot of a discharged vertex (residual, head, head's
            //    label and activity flag), 16 B per push (reverse slot index,
            //    residual, delta, touched mark or candidate entry), plus the
            //    activity flags of all n vertices in a dense round;
            //  merge: 41 B per merged vertex, 4 B per slot of it (delta), 12 B
            //    per push received (residual update, delta clear), plus n B in
            //    a dense round;
            //  global relabel: 12 B per slot examined (head, reverse index,
            //    residual, label), 9 B per vertex per relabel (labels reset,
            //    working-set rebuild) and 4 B per vertex per bottom-up level.
            Ctl c = *ctx->ctl_host;
            c.pushes += cum[0];
            c.dverts += cum[3];
            c.dslots += cum[4];
            c.mverts += cum[5];
            c.mslots += cum[6];
            c.gslots += cum[7];
            stats->ms_phase_kernel = S.ms_phase;
            stats->phase_launches = S.n_phase;
            stats->ms_discharge = S.ms_dis;
            stats->ms_merge = S.ms_mer;
            stats->ms_global_relabel = S.ms_gr;
            stats->discharge_launches = S.n_dis;
            stats->merge_launches = S.n_mer;
            stats->global_relabel_launches = S.n_gr;
            stats->discharge_bytes = 40 * c.dverts + 13 * c.dslots + 16 * c.pushes + S.dense_rounds * (int64_t)n;
            stats->merge_bytes = 41 * c.mverts + 4 * c.mslots + 12 * c.pushes + S.dense_rounds * (int64_t)n;
            stats->global_relabel_bytes = 12 * (c.gslots + c.hslots) + (S.st.hr ? 8 : 16) * S.td_slots +
                                          S.grs * (9 * (int64_t)n + (S.st.hr ? 16 : 0) * (int64_t)S.g.slots) +
                                          S.bu_levels * 4 * (int64_t)n;
            for (int k = 0; k < MF_K_COUNT; k++) {
                stats->kernel_ms[k] = S.kms[k];
                stats->kernel_timed[k] = S.kt[k];
                stats->kernel_launches[k] = S.kn[k];
                stats->kernel_bytes[k] = S.kb[k];
            }
        }
    }
    return timed_out ? fail(ctx, MF_ETIMEOUT, "round limit %lld reached", (long long)o.max_rounds) : MF_OK;
}

extern "C" mf_status mf_solve_device(mf_context *ctx, const mf_graph *dev_g, mf_stream stream,
                                     const mf_options *opt, int64_t *value, int32_t *flow_dev, uint8_t *side_dev,
                                     mf_stats *stats)
{
    if (!ctx || !dev_g) return fail(ctx, MF_EINVAL, "NULL argument");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    mf_status st = order_after(ctx, stream);
    if (st != MF_OK) return st;
    mf_dgraph *dg = nullptr;
    st = graph_upload(ctx, dev_g, 1, &dg);
    if (st == MF_OK) {
        st = solve_uploaded(ctx, dg, opt, value, flow_dev, side_dev, stats);
        mf_graph_free(ctx, dg);
    }
    mf_status so = order_before(ctx, stream);
    return st == MF_OK ? so : st;
}

extern "C" mf_status mf_solve(mf_context *ctx, const mf_graph *host_g, const mf_options *opt,
                              int64_t *value, int32_t *flow, uint8_t *sink_side, mf_stats *stats)
{
    if (!ctx || !host_g) return fail(ctx, MF_EINVAL, "NULL argument");
    mf_dgraph *dg = nullptr;
    mf_status st = graph_upload(ctx, host_g, 0, &dg);
    if (st != MF_OK) return st;
    int32_t *flow_dev = nullptr;
    uint8_t *side_dev = nullptr;
    const size_t S = (size_t)dg->slots, N = (size_t)dg->n;
    if (flow && (st = dalloc(ctx, (void **)&flow_dev, 4 * S)) != MF_OK) {
        mf_graph_free(ctx, dg);
        return st;
    }
    if (sink_side && (st = dalloc(ctx, (void **)&side_dev, N)) != MF_OK) {
        dfree(ctx, flow_dev, 4 * S);
        mf_graph_free(ctx, dg);
        return st;
    }
    st = solve_uploaded(ctx, dg, opt, value, flow_dev, side_dev, stats);
    if (st == MF_OK || st == MF_ETIMEOUT) {
        hipError_t e = hipSuccess;
        if (flow && S) e = hipMemcpy(flow, flow_dev, 4 * S, hipMemcpyDeviceToHost);
        if (e == hipSuccess && sink_side) e = hipMemcpy(sink_side, side_dev, N, hipMemcpyDeviceToHost);
        if (e != hipSuccess) st = fail(ctx, MF_EDEVICE, "result copy failed: %s", hipGetErrorString(e));
    }
    dfree(ctx, flow_dev, 4 * S);
    dfree(ctx, side_dev, N);
    mf_graph_free(ctx, dg);
    return st;
}

// ---------------------------------------------------------------------------
// Pieces shared with the server's grid lane and the batched form's large
// instances (declared in mf_host.h)

mf_status solve_in_workspace(mf_context *ctx, mf_dgraph *dg, const mf_options *opt, int64_t *value,
                             int32_t *flow_dev, uint8_t *side_dev, mf_stats *stats, Workspace *w, bool resume)
{
    return solve_uploaded(ctx, dg, opt, value, flow_dev, side_dev, stats, w, resume);
}

mf_status upload_graph_into(mf_context *ctx, const mf_graph *g, uint8_t *base, const InstLayout &L,
                            int64_t *stage64, mf_dgraph *dg)
{
    const size_t S = (size_t)g->slots, N = (size_t)g->n;
    dg->n = g->n;
    dg->s = g->s;
    dg->t = g->t;
    dg->slots = g->slots;
    dg->off = (int32_t *)(base + L.off);
    dg->head = (int32_t *)(base + L.head);
    dg->rev = (int32_t *)(base + L.rev);
    dg->cap = (int32_t *)(base + L.cap);
    int64_t *off64 = stage64, *rev64 = stage64 + (N + 1);
    hipError_t he = hipMemcpyAsync(off64, g->offsets, 8 * (N + 1), hipMemcpyHostToDevice, ctx->stream);
    if (he == hipSuccess && S) he = hipMemcpyAsync(rev64, g->rev, 8 * S, hipMemcpyHostToDevice, ctx->stream);
    if (he == hipSuccess && S) he = hipMemcpyAsync(dg->head, g->head, 4 * S, hipMemcpyHostToDevice, ctx->stream);
    if (he == hipSuccess && S) he = hipMemcpyAsync(dg->cap, g->cap, 4 * S, hipMemcpyHostToDevice, ctx->stream);
    if (he == hipSuccess) he = hipMemsetAsync(ctx->ctl, 0, sizeof(Ctl), ctx->stream);
    if (he != hipSuccess) return fail(ctx, MF_EDEVICE, "graph upload failed: %s", hipGetErrorString(he));
    const int maxg = ctx->num_cus * 8;
    launch_narrow(off64, rev64, dg->off, dg->rev, dg->n, dg->slots, ctx->ctl,
                  grid_for(std::max<int64_t>(dg->slots, N + 1), 256, maxg), ctx->stream);
    mf_status st = read_ctl(ctx);
    if (st != MF_OK) return st;
    if (ctx->ctl_host->err == 0) {
        launch_validate(dg->view(), ctx->ctl, grid_for(S, 256, maxg), ctx->stream);
        launch_degree_stats(dg->view(), ctx->ctl, grid_for(N, 256, maxg), ctx->stream);
        if ((st = read_ctl(ctx)) != MF_OK) return st;
    }
    if (ctx->ctl_host->err) return fail(ctx, MF_EINVAL, "invalid graph: %s", validation_message(ctx->ctl_host->err));
    dg->maxdeg_inner = ctx->ctl_host->maxdeg_inner;
    dg->deg_s = ctx->ctl_host->deg_s;
    dg->deg_t = ctx->ctl_host->deg_t;
    return MF_OK;
}

// New capacities for a resident graph (host array): checked as at upload;
// with has_flow the kept residuals move by the changes, and *resumable says
// whether every new capacity still holds the kept flow.  MF_EINVAL leaves
// the graph unchanged.  tmp_dev: int32[slots] device scratch.
mf_status check_caps_into(mf_context *ctx, mf_dgraph *dg, const int32_t *cap_host, int32_t *tmp_dev,
                          int32_t *keep_res, bool has_flow, bool *resumable)
{
    *resumable = false;
    const int64_t S = dg->slots;
    if (S == 0) {
        *resumable = has_flow;
        return MF_OK;
    }
    HIPCHK(ctx, hipMemcpyAsync(tmp_dev, cap_host, 4 * S, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(ctx->ctl, 0, sizeof(Ctl), ctx->stream));
    const int maxg = ctx->num_cus * 8;
    GraphView gv = dg->view();
    gv.cap = tmp_dev;
    launch_validate(gv, ctx->ctl, grid_for(S, 256, maxg), ctx->stream);
    mf_status st = read_ctl(ctx);
    if (st != MF_OK) return st;
    if (ctx->ctl_host->err)
        return fail(ctx, MF_EINVAL, "invalid capacities: %s", validation_message(ctx->ctl_host->err));
    if (has_flow) launch_recap(dg->view(), tmp_dev, keep_res, 1, ctx->ctl, grid_for(S, 256, maxg), ctx->stream);
    HIPCHK(ctx, hipMemcpyAsync(dg->cap, tmp_dev, 4 * S, hipMemcpyDeviceToDevice, ctx->stream));
    if ((st = read_ctl(ctx)) != MF_OK) return st;
    *resumable = has_flow && !(ctx->ctl_host->err & 128);
    return MF_OK;
}

// ---------------------------------------------------------------------------
// The solve of mf_solve_device without device allocation

// Byte offsets of the graph copies and the per-solve state inside the
// scratch array; returns the bytes needed.
struct ScratchLayout {
    size_t off, rev, res, delta, C, d, dn, owner, e, act, side, touched, A, A2, Q, Q2, H, end;
};
static ScratchLayout scratch_layout(int64_t n, int64_t slots)
{
    ScratchLayout L;
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p += align256(bytes ? bytes : 4);
        return at;
    };
    const size_t N = (size_t)n, S = (size_t)std::max<int64_t>(slots, 1);
    L.off = take(4 * (N + 1));
    L.rev = take(4 * S);
    L.res = take(4 * S);
    L.delta = take(4 * S);
    L.C = take(4 * (S + N));
    L.d = take(4 * N);
    L.dn = take(4 * N);
    L.owner = take(4 * N);
    L.e = take(8 * N);
    L.act = take(N);
    L.side = take(N);
    L.touched = take(N);
    L.A = take(4 * N);
    L.A2 = take(4 * N);
    L.Q = take(4 * N);
    L.Q2 = take(4 * N);
    L.H = take(4 * N);
    L.end = p;
    return L;
}

extern "C" mf_status mf_solve_device_noalloc(mf_context *ctx, const mf_graph *g, mf_stream stream,
                                             const mf_options *opt, int64_t *value, int32_t *flow_dev,
                                             uint8_t *side_dev, mf_stats *stats)
{
    if (!ctx || !g) return fail(ctx, MF_EINVAL, "NULL argument");
    if (g->n < 2) return fail(ctx, MF_EINVAL, "n must be at least 2");
    if (g->slots < 0 || g->slots >= 2147483647LL || (int64_t)g->n + g->slots >= 2147483647LL)
        return fail(ctx, MF_EINVAL, "slots out of the supported range");
    if (g->s < 0 || g->s >= g->n || g->t < 0 || g->t >= g->n || g->s == g->t)
        return fail(ctx, MF_EINVAL, "s and t must be distinct vertices");
    if (!g->offsets || (g->slots > 0 && (!g->head || !g->rev || !g->cap)))
        return fail(ctx, MF_EINVAL, "NULL graph array");
    const ScratchLayout L = scratch_layout(g->n, g->slots);
    if (L.end > (size_t)MF_NOALLOC_SCRATCH_BYTES)
        return fail(ctx, MF_ENOMEM, "the graph needs %zu bytes of scratch; the no-allocation entry point has %zu",
                    L.end, (size_t)MF_NOALLOC_SCRATCH_BYTES);
    if (!ctx->scratch) return fail(ctx, MF_EDEVICE, "no scratch address for device %d", ctx->device);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    mf_status st = order_after(ctx, stream);
    if (st != MF_OK) return st;
    uint8_t *base = ctx->scratch;
    // residency step into the scratch: int32 offsets and reverse slots;
    // heads and capacities are read where the caller keeps them
    mf_dgraph dg;
    dg.n = g->n;
    dg.s = g->s;
    dg.t = g->t;
    dg.slots = g->slots;
    dg.off = (int32_t *)(base + L.off);
    dg.rev = (int32_t *)(base + L.rev);
    dg.head = const_cast<int32_t *>(g->head);
    dg.cap = const_cast<int32_t *>(g->cap);
    const int maxg = ctx->num_cus * 8;
    HIPCHK(ctx, hipMemsetAsync(ctx->ctl, 0, sizeof(Ctl), ctx->stream));
    launch_narrow(g->offsets, g->rev, dg.off, dg.rev, dg.n, dg.slots, ctx->ctl,
                  grid_for(std::max<int64_t>(dg.slots, (int64_t)dg.n + 1), 256, maxg), ctx->stream);
    if ((st = read_ctl(ctx)) != MF_OK) return st;
    if (ctx->ctl_host->err == 0) {
        launch_validate(dg.view(), ctx->ctl, grid_for(dg.slots, 256, maxg), ctx->stream);
        launch_degree_stats(dg.view(), ctx->ctl, grid_for(dg.n, 256, maxg), ctx->stream);
        if ((st = read_ctl(ctx)) != MF_OK) return st;
    }
    if (ctx->ctl_host->err) {
        const int bits = ctx->ctl_host->err;
        (void)order_before(ctx, stream);
        return fail(ctx, MF_EINVAL, "invalid graph: %s", validation_message(bits));
    }
    dg.maxdeg_inner = ctx->ctl_host->maxdeg_inner;
    dg.deg_s = ctx->ctl_host->deg_s;
    dg.deg_t = ctx->ctl_host->deg_t;
    Workspace w;
    w.n_cap = g->n;
    w.s_cap = std::max<int64_t>(g->slots, 1);
    w.res = (int32_t *)(base + L.res);
    w.delta = (int32_t *)(base + L.delta);
    w.C = (int32_t *)(base + L.C);
    w.d = (int32_t *)(base + L.d);
    w.dn = (int32_t *)(base + L.dn);
    w.owner = (int32_t *)(base + L.owner);
    w.e = (int64_t *)(base + L.e);
    w.act = base + L.act;
    w.side = base + L.side;
    w.touched = base + L.touched;
    w.A = (int32_t *)(base + L.A);
    w.A2 = (int32_t *)(base + L.A2);
    w.Q = (int32_t *)(base + L.Q);
    w.Q2 = (int32_t *)(base + L.Q2);
    w.H = (int32_t *)(base + L.H);
    st = solve_uploaded(ctx, &dg, opt, value, flow_dev, side_dev, stats, &w);
    mf_status so = order_before(ctx, stream);
    return st == MF_OK ? so : st;
}

// ---------------------------------------------------------------------------
// Batched solver (host side)


extern "C" mf_status mf_batch_solve(mf_context *ctx, int32_t k, const mf_graph *graphs, const mf_options *opts,
                                    int32_t *const *flows, uint8_t *const *sides, mf_result *results,
                                    mf_stats *stats)
{
    if (!ctx || k < 0 || (k > 0 && (!graphs || !results))) return fail(ctx, MF_EINVAL, "NULL argument");
    if (k == 0) return MF_OK;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    memset(results, 0, sizeof(mf_result) * (size_t)k);
    std::vector<mf_options> o((size_t)k);
    std::vector<char> ok((size_t)k, 1);
    std::vector<InstLayout> lay((size_t)k);
    size_t total = 0;
    int64_t max_n = 0, max_S = 0;
    for (int i = 0; i < k; i++) {
        if (opts) o[i] = opts[i]; else mf_options_default(&o[i]);
        const mf_graph &g = graphs[i];
        results[i].status = MF_OK;
        bool good = g.n >= 2 && g.slots >= 0 && g.slots < 2147483647LL && (int64_t)g.n + g.slots < 2147483647LL &&
                    g.s >= 0 && g.s < g.n && g.t >= 0 && g.t < g.n && g.s != g.t && g.offsets &&
                    (g.slots == 0 || (g.head && g.rev && g.cap)) && check_options(ctx, &o[i]) == MF_OK;
        if (good && (o[i].flags & MF_PREFLOW_ONLY) && flows && flows[i]) good = false;
        if (o[i].flags & (MF_GAP_RELABEL | MF_CHECK_INVARIANTS)) good = false;   // host-driven rounds only
        if (!good) {
            ok[i] = 0;
            results[i].status = MF_EINVAL;
            continue;
        }
        lay[i] = layout_for(total, g.n, g.slots, flows && flows[i], g.slots > batch_grid_slots(o[i]));
        total = lay[i].end;
        max_n = std::max<int64_t>(max_n, g.n);
        max_S = std::max<int64_t>(max_S, g.slots);
    }
    // device memory: arena, per-instance control blocks, items, results, queues, staging
    uint8_t *arena = nullptr;
    Ctl *ctls = nullptr;
    BatchItem *items_d = nullptr;
    BatchResult *res_d = nullptr;
    BatchQueue *q_d = nullptr;
    int32_t *order_d = nullptr;
    int64_t *stage64 = nullptr;
    const size_t ctl_bytes = sizeof(Ctl) * 5 * (size_t)k;
    const size_t stage_bytes = 8 * (size_t)(max_n + 1 + max_S);
    mf_status st = MF_OK;
    auto release = [&]() {
        dfree(ctx, arena, total);
        dfree(ctx, ctls, ctl_bytes);
        dfree(ctx, items_d, sizeof(BatchItem) * (size_t)k);
        dfree(ctx, res_d, sizeof(BatchResult) * (size_t)k);
        dfree(ctx, q_d, sizeof(BatchQueue) * 4);
        dfree(ctx, order_d, 4 * (size_t)k);
        dfree(ctx, stage64, stage_bytes);
    };
    if ((st = dalloc(ctx, (void **)&arena, total)) != MF_OK || (st = dalloc(ctx, (void **)&ctls, ctl_bytes)) != MF_OK ||
        (st = dalloc(ctx, (void **)&items_d, sizeof(BatchItem) * (size_t)k)) != MF_OK ||
        (st = dalloc(ctx, (void **)&res_d, sizeof(BatchResult) * (size_t)k)) != MF_OK ||
        (st = dalloc(ctx, (void **)&q_d, sizeof(BatchQueue) * 4)) != MF_OK ||
        (st = dalloc(ctx, (void **)&order_d, 4 * (size_t)k)) != MF_OK ||
        (st = dalloc(ctx, (void **)&stage64, stage_bytes)) != MF_OK) {
        release();
        return st;
    }
    hipStream_t s0 = ctx->stream;
    auto dev_err = [&](hipError_t e, const char *what) {
        release();
        return fail(ctx, MF_EDEVICE, "%s failed: %s", what, hipGetErrorString(e));
    };
    hipError_t he = hipMemsetAsync(ctls, 0, ctl_bytes, s0);
    if (he != hipSuccess) return dev_err(he, "hipMemsetAsync");
    // upload and validate every instance (residency step)
    const int maxg = ctx->num_cus * 8;
    std::vector<BatchItem> items((size_t)k);
    for (int i = 0; i < k; i++) {
        if (!ok[i]) continue;
        const mf_graph &gh = graphs[i];
        const InstLayout &L = lay[i];
        const size_t S = (size_t)gh.slots, N = (size_t)gh.n;
        GraphView gv;
        gv.n = gh.n;
        gv.s = gh.s;
        gv.t = gh.t;
        gv.slots = (int32_t)gh.slots;
        gv.off = (int32_t *)(arena + L.off);
        gv.head = (int32_t *)(arena + L.head);
        gv.rev = (int32_t *)(arena + L.rev);
        gv.cap = (int32_t *)(arena + L.cap);
        int64_t *off64 = stage64, *rev64 = stage64 + (N + 1);
        he = hipMemcpyAsync(off64, gh.offsets, 8 * (N + 1), hipMemcpyHostToDevice, s0);
        if (he == hipSuccess && S) he = hipMemcpyAsync(rev64, gh.rev, 8 * S, hipMemcpyHostToDevice, s0);
        if (he == hipSuccess && S) he = hipMemcpyAsync((void *)gv.head, gh.head, 4 * S, hipMemcpyHostToDevice, s0);
        if (he == hipSuccess && S) he = hipMemcpyAsync((void *)gv.cap, gh.cap, 4 * S, hipMemcpyHostToDevice, s0);
        if (he != hipSuccess) return dev_err(he, "batch upload");
        Ctl *c0 = ctls + 5 * (size_t)i;
        launch_narrow(off64, rev64, (int32_t *)gv.off, (int32_t *)gv.rev, gh.n, gh.slots, c0,
                      grid_for(std::max<int64_t>(S, N + 1), 256, maxg), s0);
        // k_validate relies on valid offsets; it only reads segments inside [0, slots) because k_narrow
        // clamps bad offsets to 0, so run it and report either error.
        launch_validate(gv, c0, grid_for(S, 256, maxg), s0);
        launch_degree_stats(gv, c0, grid_for(N, 256, maxg), s0);
        BatchItem &it = items[i];
        it.g = gv;
        StateView sv;
        memset(&sv, 0, sizeof sv);
        sv.res = (int32_t *)(arena + L.res);
        sv.delta = (int32_t *)(arena + L.delta);
        sv.C = (int32_t *)(arena + L.C);
        sv.d = (int32_t *)(arena + L.d);
        sv.dn = (int32_t *)(arena + L.dn);
        sv.owner = (int32_t *)(arena + L.owner);
        sv.A = (int32_t *)(arena + L.A);
        sv.A2 = (int32_t *)(arena + L.A2);
        sv.Q = (int32_t *)(arena + L.Q);
        sv.Q2 = (int32_t *)(arena + L.Q2);
        sv.H = (int32_t *)(arena + L.H);
        sv.e = (int64_t *)(arena + L.e);
        sv.act = arena + L.act;
        sv.touched = arena + L.touched;
        it.st = sv;
        it.ctl = c0;
        it.flow = L.flow ? (int32_t *)(arena + L.flow) : nullptr;
        it.side = arena + L.side;
        const mf_options &oi = o[i];
        it.G = batch_lanes(oi.lanes_per_vertex, gh.n, gh.slots);
        PhaseParams &P = it.p;
        memset(&P, 0, sizeof P);
        P.freq_num = oi.gr_freq_num;
        P.freq_den = oi.gr_freq_den;
        P.alpha = oi.gr_alpha;
        P.beta = oi.gr_beta;
        P.round_charge = oi.gr_round_charge;
        P.level_charge = oi.gr_level_charge;
        P.max_rounds = oi.max_rounds;
        P.dense_threshold = oi.dense_threshold > 0 ? oi.dense_threshold : std::max<int64_t>(512, gh.n / 16);
        P.bu_factor = oi.bfs_bottom_up_factor > 0 ? oi.bfs_bottom_up_factor : 8;
        P.hubdeg = 64 * it.G;
        P.simple = (oi.flags & MF_SIMPLE_ROUNDS) ? 1 : 0;
        P.limit_ticks = 0;
        it.preflow_only = (oi.flags & MF_PREFLOW_ONLY) ? 1 : 0;
        results[i].lanes_per_vertex = it.G;
    }
    // validation results
    std::vector<Ctl> hc(5 * (size_t)k);
    he = hipMemcpyAsync(hc.data(), ctls, ctl_bytes, hipMemcpyDeviceToHost, s0);
    if (he == hipSuccess) he = hipStreamSynchronize(s0);
    if (he != hipSuccess) return dev_err(he, "validation read-back");
    std::vector<std::vector<int32_t>> bucket(4);
    std::vector<int32_t> large;          // solved by the grid-wide kernels after the batch launch
    for (int i = 0; i < k; i++) {
        if (!ok[i]) continue;
        if (hc[5 * (size_t)i].err) {
            ok[i] = 0;
            results[i].status = MF_EINVAL;
            continue;
        }
        if (graphs[i].slots > batch_grid_slots(o[i])) {
            large.push_back(i);
            continue;
        }
        const int G = items[i].G;
        bucket[G == 4 ? 0 : G == 8 ? 1 : G == 16 ? 2 : 3].push_back(i);
    }
    std::vector<int32_t> order;
    int boff[4], bcnt[4];
    for (int b = 0; b < 4; b++) {
        // largest instances first: the longest solves start earliest
        std::stable_sort(bucket[b].begin(), bucket[b].end(), [&](int32_t x, int32_t y) {
            return graphs[x].n + graphs[x].slots > graphs[y].n + graphs[y].slots;
        });
        boff[b] = (int)order.size();
        bcnt[b] = (int)bucket[b].size();
        order.insert(order.end(), bucket[b].begin(), bucket[b].end());
    }
    he = hipMemcpyAsync(items_d, items.data(), sizeof(BatchItem) * (size_t)k, hipMemcpyHostToDevice, s0);
    if (he == hipSuccess && !order.empty())
        he = hipMemcpyAsync(order_d, order.data(), 4 * order.size(), hipMemcpyHostToDevice, s0);
    if (he == hipSuccess) he = hipMemsetAsync(res_d, 0, sizeof(BatchResult) * (size_t)k, s0);
    if (he == hipSuccess) he = hipStreamSynchronize(s0);
    if (he != hipSuccess) return dev_err(he, "batch descriptors");
    // one graph: fork to one stream per lane-count group, one persistent kernel each, join
    if ((st = ensure_batch_streams(ctx)) != MF_OK) {
        release();
        return st;
    }
    const auto t_launch = std::chrono::steady_clock::now();
    float ms = 0;
    std::vector<BatchResult> hr((size_t)k);
    const bool any_small = !order.empty();
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (any_small) {
    he = hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) return dev_err(he, "hipStreamBeginCapture");
    (void)hipEventRecord(ctx->bev[4], s0);
    for (int b = 0; b < 4; b++) {
        if (!bcnt[b]) continue;
        const int G = 4 << b;
        hipStream_t sb = ctx->bstream[b];
        (void)hipStreamWaitEvent(sb, ctx->bev[4], 0);
        launch_queue_init(q_d + b, bcnt[b], sb);
        int per_cu = batch_blocks_per_cu(G);
        if (per_cu <= 0) per_cu = 1;
        const int grid = std::max(1, std::min(bcnt[b], per_cu * ctx->num_cus));
        (void)launch_batch(G, grid, items_d, order_d + boff[b], res_d, q_d + b, sb);
        (void)hipEventRecord(ctx->bev[b], sb);
        (void)hipStreamWaitEvent(s0, ctx->bev[b], 0);
    }
    he = hipStreamEndCapture(s0, &graph);
    if (he != hipSuccess) return dev_err(he, "hipStreamEndCapture");
    he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (he != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return dev_err(he, "hipGraphInstantiate");
    }
    // the batch runs on its own stream while the large instances below run
    // on the context's stream
    (void)hipEventRecord(ctx->gev[0], ctx->lstream);
    he = hipGraphLaunch(exec, ctx->lstream);
    (void)hipEventRecord(ctx->gev[1], ctx->lstream);
    if (he == hipSuccess)
        he = hipMemcpyAsync(hr.data(), res_d, sizeof(BatchResult) * (size_t)k, hipMemcpyDeviceToHost, ctx->lstream);
    if (he != hipSuccess) {
        (void)hipStreamSynchronize(ctx->lstream);
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return dev_err(he, "batch launch");
    }
    }
    // Instances above the routing size: by the grid-wide kernels while the
    // batch launch runs, grid_workers at a time (each worker a host thread
    // with a helper context: its own stream and control block), each over
    // its own slice of the arena.
    std::vector<char> big((size_t)k, 0);
    for (int i : large) big[i] = 1;
    std::vector<mf_status> lst((size_t)k, MF_OK);
    if (!large.empty()) {
        const int want = opts && opts[0].grid_workers > 0 ? opts[0].grid_workers : 4;
        const int nw = std::max(1, std::min<int>(want, (int)large.size()));
        mf_status hs = ensure_helpers(ctx, nw);
        if (hs != MF_OK) {
            if (any_small) (void)hipStreamSynchronize(ctx->lstream);
            release();
            return hs;
        }
        std::atomic<int> next_large{0};
        auto worker = [&](int wi) {
            mf_context *hx = ctx->helpers[(size_t)wi];
            (void)hipSetDevice(ctx->device);
            while (true) {
                const int q = next_large.fetch_add(1);
                if (q >= (int)large.size()) break;
                const int i = large[(size_t)q];
                const mf_graph &gh = graphs[i];
                const InstLayout &L = lay[i];
                const Ctl &c0 = hc[5 * (size_t)i];
                mf_dgraph dg;
                dg.n = gh.n;
                dg.s = gh.s;
                dg.t = gh.t;
                dg.slots = gh.slots;
                dg.off = (int32_t *)(arena + L.off);
                dg.head = (int32_t *)(arena + L.head);
                dg.rev = (int32_t *)(arena + L.rev);
                dg.cap = (int32_t *)(arena + L.cap);
                dg.maxdeg_inner = c0.maxdeg_inner;
                dg.deg_s = c0.deg_s;
                dg.deg_t = c0.deg_t;
                Workspace w = workspace_in(arena, L, gh.n, gh.slots);
                mf_options oi = o[i];
                oi.flags &= ~(uint32_t)MF_PROFILE;
                mf_stats sst;
                memset(&sst, 0, sizeof sst);
                int64_t val = 0;
                const double t_in =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_launch).count();
                mf_status sr = solve_uploaded(hx, &dg, &oi, &val, L.flow ? (int32_t *)(arena + L.flow) : nullptr,
                                              arena + L.side, &sst, &w);
                const size_t S = (size_t)gh.slots, N = (size_t)gh.n;
                hipError_t e2 = hipSuccess;
                if (sr == MF_OK && flows && flows[i] && S)
                    e2 = hipMemcpyAsync(flows[i], arena + L.flow, 4 * S, hipMemcpyDeviceToHost, hx->stream);
                if (e2 == hipSuccess && sr != MF_EDEVICE && sides && sides[i])
                    e2 = hipMemcpyAsync(sides[i], arena + L.side, N, hipMemcpyDeviceToHost, hx->stream);
                if (e2 == hipSuccess) e2 = hipStreamSynchronize(hx->stream);
                if (e2 != hipSuccess) sr = MF_EDEVICE;
                mf_result &R = results[i];
                R.status = sr;
                R.lanes_per_vertex = 0;
                R.value = sst.value;
                R.cut_capacity = sst.cut_capacity;
                R.rounds = sst.rounds;
                R.rounds2 = sst.rounds2;
                R.global_relabels = sst.global_relabels;
                R.global_relabels2 = sst.global_relabels2;
                R.bfs_levels = sst.bfs_levels;
                R.pushes = sst.pushes;
                R.relabels = sst.relabels;
                R.ms_start = t_in;
                R.ms_end =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_launch).count();
                lst[(size_t)i] = sr;
            }
        };
        std::vector<std::thread> th;
        for (int wi = 1; wi < nw; wi++) th.emplace_back(worker, wi);
        worker(0);
        for (auto &t : th) t.join();
        for (int i : large)
            if (lst[(size_t)i] == MF_EDEVICE) {
                if (any_small) (void)hipStreamSynchronize(ctx->lstream);
                std::string e = ctx->helpers[0]->err;
                release();
                return fail(ctx, MF_EDEVICE, "grid-wide solve of a large batch instance failed: %s", e.c_str());
            }
    }
    if (any_small) {
        he = hipStreamSynchronize(ctx->lstream);
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        if (he != hipSuccess) return dev_err(he, "batch launch");
        (void)hipEventElapsedTime(&ms, ctx->gev[0], ctx->gev[1]);
    }
    int64_t t0 = INT64_MAX;
    for (int i = 0; i < k; i++)
        if (ok[i] && !big[i]) t0 = std::min(t0, hr[i].t_start);
    for (int i = 0; i < k; i++) {
        if (!ok[i] || big[i]) continue;
        const BatchResult &r = hr[i];
        mf_result &R = results[i];
        R.status = r.status == 0 ? MF_OK : r.status == 1 ? MF_ETIMEOUT : MF_EDEVICE;
        R.value = r.value;
        R.cut_capacity = r.cut;
        R.rounds = r.rounds;
        R.rounds2 = r.rounds2;
        R.global_relabels = r.grs;
        R.global_relabels2 = r.grs2;
        R.bfs_levels = r.levels;
        R.pushes = r.pushes;
        R.relabels = r.relabels;
        R.ms_start = 1e3 * (double)(r.t_start - t0) / (double)ctx->wall_hz;
        R.ms_end = 1e3 * (double)(r.t_end - t0) / (double)ctx->wall_hz;
        const size_t S = (size_t)graphs[i].slots, N = (size_t)graphs[i].n;
        if (flows && flows[i] && S && R.status == MF_OK)
            he = hipMemcpy(flows[i], items[i].flow, 4 * S, hipMemcpyDeviceToHost);
        if (he == hipSuccess && sides && sides[i]) he = hipMemcpy(sides[i], items[i].side, N, hipMemcpyDeviceToHost);
        if (he != hipSuccess) return dev_err(he, "batch output copy");
    }
    if (stats) {
        memset(stats, 0, sizeof *stats);
        stats->ms_total = large.empty() ? ms
                                        : std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                                  t_launch).count();
    }
    release();
    return MF_OK;
}
