// Host-side internals shared by the solver, the batch path and the server.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/maxflow.h"
#include "mf_device.h"
#include "mf_phase.h"

using namespace mf;

extern thread_local std::string g_global_err;

struct mf_dgraph {
    int32_t n = 0, s = 0, t = 0;
    int64_t slots = 0;
    int32_t *off = nullptr, *head = nullptr, *rev = nullptr, *cap = nullptr;
    size_t bytes = 0;
    int32_t maxdeg_inner = 0, deg_s = 0, deg_t = 0;   // out-degrees (hub levels of the BFS)
    GraphView view() const
    {
        GraphView g;
        g.n = n;
        g.s = s;
        g.t = t;
        g.slots = (int32_t)slots;
        g.off = off;
        g.head = head;
        g.rev = rev;
        g.cap = cap;
        return g;
    }
};

struct Workspace {
    int64_t n_cap = 0, s_cap = 0;
    int32_t *res = nullptr, *delta = nullptr, *d = nullptr, *dn = nullptr, *owner = nullptr;
    int64_t *e = nullptr;
    uint8_t *act = nullptr, *side = nullptr, *touched = nullptr;
    int32_t *A = nullptr, *A2 = nullptr, *C = nullptr, *Q = nullptr, *Q2 = nullptr, *H = nullptr;
    int32_t *hr = nullptr;   // packed heads of the top-down search (null: gather reverse residuals)
    int32_t *lcount = nullptr, *gcand = nullptr;   // gap rule: label histogram [n+1], candidates [n]
    size_t bytes = 0;
};

struct mf_context {
    int device = 0;
    size_t budget = 0;     // 0 = unbounded
    size_t used = 0;       // bytes held (graphs + workspace)
    hipStream_t stream = nullptr;
    Ctl *ctl = nullptr;        // device: [0] main, [1..3] round ring, [4] global relabel (persistent)
    Ctl *ctl_host = nullptr;   // pinned host mirror of all five
    GridBar *bar = nullptr;    // device: persistent-kernel barrier
    uint64_t wall_hz = 100000000ull;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    hipEvent_t pev[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};   // profiling
    hipStream_t bstream[4] = {nullptr, nullptr, nullptr, nullptr};                 // batch groups
    hipEvent_t bev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hipEvent_t sev[2] = {nullptr, nullptr};   // ordering against a caller's stream (in, out)
    hipStream_t lstream = nullptr;             // the batch launch, beside the grid-wide solves of large instances
    hipEvent_t gev[2] = {nullptr, nullptr};    // start and end of the batch launch
    std::vector<mf_context *> helpers;         // batched form: contexts of the grid-wide solve workers
    std::vector<hipEvent_t> lev;     // profiling of batched levels, created on first use
    Workspace ws;
    uint8_t *one = nullptr;    // device: item, result, queue and order of a single-workgroup solve
    // the graph whose complete flow the workspace holds (residuals, excess
    // of t), from the last grid-path solve; nullptr once anything else has
    // used the workspace
    const mf_dgraph *warm_dg = nullptr;
    uint8_t *scratch = nullptr;   // device address of the no-allocation scratch array on this device
    int num_cus = 256;
    std::string err;
};

// ---------------------------------------------------------------------------
// Error helpers

inline mf_status fail(mf_context *ctx, mf_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_global_err = buf;
    return st;
}

#define HIPCHK(ctx, expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail((ctx), MF_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

inline int grid_for(int64_t items, int per_block, int max_grid)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > max_grid) g = max_grid;
    return (int)g;
}

inline mf_status dalloc(mf_context *ctx, void **p, size_t bytes)
{
    if (bytes == 0) bytes = 4;
    if (ctx->budget && ctx->used + bytes > ctx->budget)
        return fail(ctx, MF_ENOMEM, "HBM budget exceeded: %zu held + %zu requested > %zu", ctx->used,
                    bytes, ctx->budget);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(ctx, MF_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    ctx->used += bytes;
    return MF_OK;
}

inline void dfree(mf_context *ctx, void *p, size_t bytes)
{
    if (!p) return;
    (void)hipFree(p);
    if (bytes == 0) bytes = 4;
    ctx->used -= std::min(ctx->used, bytes);
}


// ---------------------------------------------------------------------------
// Per-instance device layout of the batched and served paths.

struct InstLayout {
    size_t off, head, rev, cap, res, delta, C, d, dn, owner, A, A2, Q, Q2, H, e, act, touched, side, flow;
    size_t hr;         // packed heads of the top-down search (grid-wide kernels only; 0 = none)
    size_t end;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline InstLayout layout_for(size_t base, int64_t n, int64_t S, bool want_flow, bool with_hr = false)
{
    InstLayout L;
    size_t p = base;
    auto take = [&](size_t bytes) {
        size_t at = p;
        p = align256(p + std::max<size_t>(bytes, 4));
        return at;
    };
    L.off = take(4 * (n + 1));
    L.head = take(4 * S);
    L.rev = take(4 * S);
    L.cap = take(4 * S);
    L.res = take(4 * S);
    L.delta = take(4 * S);
    L.C = take(4 * (S + n));
    L.d = take(4 * n);
    L.dn = take(4 * n);
    L.owner = take(4 * n);
    L.A = take(4 * n);
    L.A2 = take(4 * n);
    L.Q = take(4 * n);
    L.Q2 = take(4 * n);
    L.H = take(4 * n);
    L.e = take(8 * n);
    L.act = take(n);
    L.touched = take(n);
    L.side = take(n);
    L.flow = want_flow ? take(4 * S) : 0;
    L.hr = with_hr ? take(4 * S) : 0;
    L.end = p;
    return L;
}

// The per-solve state of the grid-wide kernels over an instance's slice.
inline Workspace workspace_in(uint8_t *base, const InstLayout &L, int64_t n, int64_t S)
{
    Workspace w;
    w.n_cap = n;
    w.s_cap = std::max<int64_t>(S, 1);
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
    w.hr = L.hr ? (int32_t *)(base + L.hr) : nullptr;
    return w;
}

// Batched and served forms: an instance with more slots than this is solved
// by the grid-wide kernels instead of one workgroup.
inline int64_t batch_grid_slots(const mf_options &o)
{
    return o.batch_grid_slots > 0 ? (int64_t)o.batch_grid_slots : (int64_t)MF_BATCH_GRID_SLOTS;
}

// Solver entry points shared with the server (solver.hip).
//  solve_in_workspace: the solve of mf_solve_uploaded over a caller-carved
//    workspace (nothing allocated, grid-wide kernels); with resume, the
//    workspace already holds the residuals of a complete flow of this graph
//    and e(t) its value, and the solve continues from that flow.
//  upload_graph_into: copies a host graph into a caller-carved slice
//    (stage64: device int64 scratch of 8(n+1) + 8 slots bytes), narrows and
//    checks it on the context's stream, and fills *dg.
mf_status solve_in_workspace(mf_context *ctx, mf_dgraph *dg, const mf_options *opt, int64_t *value,
                             int32_t *flow_dev, uint8_t *side_dev, mf_stats *stats, Workspace *w, bool resume);
mf_status upload_graph_into(mf_context *ctx, const mf_graph *host_g, uint8_t *base, const InstLayout &L,
                            int64_t *stage64, mf_dgraph *dg);
mf_status check_caps_into(mf_context *ctx, mf_dgraph *dg, const int32_t *cap_host, int32_t *tmp_dev,
                          int32_t *keep_res, bool has_flow, bool *resumable);

inline int batch_lanes(int requested, int64_t n, int64_t S)
{
    int G = requested;
    if (G <= 0) {
        const double avg = n > 0 ? (double)S / (double)n : 1.0;
        G = 4;
        while (G < avg && G < 32) G <<= 1;
    }
    if (G <= 4) return 4;
    if (G <= 8) return 8;
    if (G <= 16) return 16;
    return 32;
}

