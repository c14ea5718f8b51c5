// Per-vertex steps of a synchronous round, shared by the host-driven kernels
// and the persistent solver kernel.
#pragma once
#include "mf_device.h"

namespace mf {

// One pass over a chunk of up to G slots, in slot order.  Each lane holds one
// slot: r its residual, w its head, dw = d(w), aw = act(w).  Pushes along
// admissible arcs the vertex may use take min(r, e - excl) where excl is the
// total residual of the admissible, usable arcs before it in slot order: the
// result of visiting the arcs one after another.
//
// The sink never discharges and nobody reads its own slots or its excess
// during a round, so a push into the sink updates the reverse slot directly
// (each slot has one pusher) and is added to the sink's excess once per block.
// sg (list rounds of the grid-wide kernels): the candidate appends collect
// in the block's LDS stage (one global atomic per block); null: one atomic
// per wave.
template <int G, bool DENSE>
__device__ __forceinline__ int chunk_pass(const GraphView &g, StateView &st, int v, int dv, int dp,
                                          int gl, int a, int &r, int w, int dw, bool aw,
                                          int64_t &el, bool &lose, int64_t &pushes, int sink,
                                          int64_t &to_sink, bool simple, Stage *sg)
{
    const bool adm = r > 0 && dp == dw + 1;
    const bool win = (dv == dw + 1) || (dv < dw - 1) || (dv == dw && v < w);
    lose = !simple && adm && aw && !win;
    const bool use = adm && !lose;
    const int64_t amt = use ? (int64_t)r : 0;
    const int64_t incl = group_incl_scan<G>(amt, gl);
    const int64_t tot = group_bcast<G>(incl, G - 1);
    const int64_t excl = incl - amt;
    int dl = 0;
    if (use && excl < el) {
        const int64_t rem = el - excl;
        dl = rem < (int64_t)r ? (int)rem : r;
    }
    const bool into_sink = w == sink;
    if (dl > 0) {
        r -= dl;
        pushes++;
        if (into_sink) {
            st.res[g.rev[a]] += dl;
            to_sink += dl;
        } else {
            st.delta[g.rev[a]] = dl;
            if (DENSE) st.touched[w] = 1;
        }
    }
    if (!DENSE) {
        const bool app = dl > 0 && !into_sink;
        if (sg) {
            stage_append_owner(*sg, app, w, st.C, &st.ctl->nc, st.owner);
        } else {
            const int idx = wave_append(app, w, st.C, &st.ctl->nc);
            if (app) st.owner[w] = idx;
        }
    }
    el = tot >= el ? 0 : el - tot;
    return dl;
}

struct DisAcc {
    int64_t work = 0, pushes = 0, relabels = 0, scans = 0, to_sink = 0, dverts = 0, dslots = 0;
};

// Full discharge of one vertex v by a group of G lanes (the loop body of
// Listing 1 for one element of the working set).  TWO: vertices of up to 2G
// slots keep both chunks in registers across passes (more registers per
// lane; the host uses it for graphs whose vertices all fit).
template <int G, bool DENSE, bool TWO = false>
__device__ __forceinline__ void discharge_vertex(const GraphView &g, StateView &st, const RoundParams &p,
                                                 int v, int gl, DisAcc &acc, Stage *sg = nullptr)
{
    const int n = g.n;
    const int beg = g.off[v], end = g.off[v + 1], deg = end - beg;
    if (gl == 0) {
        acc.dverts++;
        acc.dslots += deg;
    }
    const int dv = st.d[v];
    int dp = dv;
    int64_t el = st.e[v];
    if (deg <= G) {
        // The vertex's slots stay in registers across passes.
        const int a = beg + gl;
        int r = 0, w = -1, dw = 0;
        bool aw = false;
        if (gl < deg) {
            r = st.res[a];
            const int h = g.head[a];     // read beside the residual: one link fewer
            if (r > 0) {
                w = h;
                dw = st.d[w];
                aw = st.act[w] != 0;
            }
        }
        bool dirty = false;
        while (el > 0) {
            if (gl == 0) acc.scans += deg;
            bool lose;
            if (chunk_pass<G, DENSE>(g, st, v, dv, dp, gl, a, r, w, dw, aw, el, lose, acc.pushes, p.sink,
                                     acc.to_sink, p.simple, sg) > 0)
                dirty = true;
            if (el == 0) break;
            const int cand = (r > 0 && dw >= dp) ? dw + 1 : n;
            const int nl = group_min<G>(cand);
            if (group_or<G>(lose ? 1 : 0)) break;          // skipped
            dp = nl < n ? nl : n;                            // relabel
            if (gl == 0) {
                acc.work += deg + p.beta;
                acc.relabels++;
            }
            if (dp >= n) break;
            if (p.simple) break;                              // one relabel per round
        }
        if (dirty) st.res[a] = r;
    } else if (TWO && deg <= 2 * G) {
        // Two chunks, both kept in registers across passes (slot a0 of the
        // first, a1 of the second; lanes past the end hold r = 0).  Only v
        // writes these residuals during the round and the labels and
        // activity it reads are the round's snapshot, so the registers stay
        // current; each pass visits the chunks in slot order as the loop
        // below does.
        const int a0 = beg + gl, a1 = beg + G + gl;
        int r0 = st.res[a0], w0 = -1, dw0 = 0;
        int r1 = 0, w1 = -1, dw1 = 0;
        bool aw0 = false, aw1 = false;
        const int h0 = g.head[a0];
        const int h1 = a1 < end ? g.head[a1] : -1;
        if (a1 < end) r1 = st.res[a1];
        if (r0 > 0) {
            w0 = h0;
            dw0 = st.d[w0];
            aw0 = st.act[w0] != 0;
        }
        if (r1 > 0) {
            w1 = h1;
            dw1 = st.d[w1];
            aw1 = st.act[w1] != 0;
        }
        bool dirty0 = false, dirty1 = false;
        while (el > 0) {
            int cand = n;
            bool lose;
            if (gl == 0) acc.scans += G;
            if (chunk_pass<G, DENSE>(g, st, v, dv, dp, gl, a0, r0, w0, dw0, aw0, el, lose, acc.pushes, p.sink,
                                     acc.to_sink, p.simple, sg) > 0)
                dirty0 = true;
            if (el == 0) break;
            if (r0 > 0 && dw0 >= dp) cand = dw0 + 1;
            int sk = lose ? 1 : 0;
            if (gl == 0) acc.scans += deg - G;
            if (chunk_pass<G, DENSE>(g, st, v, dv, dp, gl, a1, r1, w1, dw1, aw1, el, lose, acc.pushes, p.sink,
                                     acc.to_sink, p.simple, sg) > 0)
                dirty1 = true;
            if (el == 0) break;
            if (r1 > 0 && dw1 >= dp && dw1 + 1 < cand) cand = dw1 + 1;
            sk |= lose ? 1 : 0;
            const int nl = group_min<G>(cand);
            if (group_or<G>(sk)) break;
            dp = nl < n ? nl : n;
            if (gl == 0) {
                acc.work += deg + p.beta;
                acc.relabels++;
            }
            if (dp >= n) break;
            if (p.simple) break;
        }
        if (dirty0) st.res[a0] = r0;
        if (dirty1) st.res[a1] = r1;
    } else {
        while (el > 0) {
            int cand = n;
            int sk = 0;
            for (int base = beg; base < end; base += G) {
                const int a = base + gl;
                int r = 0, w = -1, dw = 0;
                bool aw = false;
                if (a < end) {
                    r = st.res[a];
                    const int h = g.head[a];
                    if (r > 0) {
                        w = h;
                        dw = st.d[w];
                        aw = st.act[w] != 0;
                    }
                }
                if (gl == 0) acc.scans += (end - base) < G ? (end - base) : G;
                bool lose;
                if (chunk_pass<G, DENSE>(g, st, v, dv, dp, gl, a, r, w, dw, aw, el, lose, acc.pushes, p.sink,
                                         acc.to_sink, p.simple, sg) > 0)
                    st.res[a] = r;
                if (el == 0) break;
                if (r > 0 && dw >= dp && dw + 1 < cand) cand = dw + 1;
                sk |= lose ? 1 : 0;
            }
            if (el == 0) break;
            const int nl = group_min<G>(cand);
            if (group_or<G>(sk)) break;
            dp = nl < n ? nl : n;
            if (gl == 0) {
                acc.work += deg + p.beta;
                acc.relabels++;
            }
            if (dp >= n) break;
            if (p.simple) break;
        }
    }
    if (gl == 0) {
        st.dn[v] = dp;
        st.e[v] = el;
        if (DENSE) st.touched[v] = 1;
    }
    if (!DENSE) {
        if (sg) {
            stage_append_owner(*sg, gl == 0, v, st.C, &st.ctl->nc, st.owner);
        } else {
            const int idx = wave_append(gl == 0, v, st.C, &st.ctl->nc);
            if (gl == 0) st.owner[v] = idx;
        }
    }
}

__device__ __forceinline__ void discharge_flush(StateView &st, const RoundParams &p, DisAcc &acc)
{
    block_add64(acc.to_sink, &st.e[p.sink]);
    block_add64(acc.work, &st.ctl->work);
    block_add64(acc.pushes, &st.ctl->pushes);
    block_add64(acc.relabels, &st.ctl->relabels);
    block_add64(acc.scans, &st.ctl->scans);
    block_add64(acc.dverts, &st.ctl->dverts);
    block_add64(acc.dslots, &st.ctl->dslots);
}

struct MerAcc {
    int64_t mverts = 0, mslots = 0;
};

template <int G, bool DENSE>
__device__ __forceinline__ void merge_vertex(const GraphView &g, StateView &st, int w, int gl, int sink,
                                             int other, MerAcc &acc, Stage *sg)
{
    const int beg = g.off[w], end = g.off[w + 1];
    if (gl == 0) {
        acc.mverts++;
        acc.mslots += end - beg;
    }
    int64_t sum = 0;
    for (int a = beg + gl; a < end; a += G) {
        const int dl = st.delta[a];
        if (dl != 0) {
            st.res[a] += dl;
            st.delta[a] = 0;
            sum += dl;
        }
    }
    sum = group_sum<G>(sum);
    bool pa = false;
    int dold = 0, dnew = 0;
    if (gl == 0) {
        const int64_t e = st.e[w] + sum;
        st.e[w] = e;
        dnew = st.dn[w];
        dold = st.d[w];
        st.d[w] = dnew;
        pa = w != sink && w != other && e > 0 && dnew < g.n;
        st.act[w] = pa;
        if (DENSE) st.touched[w] = 0;
    }
    if (st.lcount) {
        // gap rule: the next working set is listed after the round's gap
        // has lifted its labels (k_gap_next)
        gap_relabel_count(st, gl == 0 && dnew != dold, dold, dnew, g.n);
        return;
    }
    // the next working set, listed in A2 (each vertex is merged once); with a
    // stage the entries collect in LDS and the caller flushes them
    if (sg)
        stage_append(*sg, pa, w, st.A2, &st.ctl->na2);
    else
        wave_append(pa, w, st.A2, &st.ctl->na2);
}

__device__ __forceinline__ void merge_flush(StateView &st, bool dense, MerAcc &acc)
{
    (void)dense;
    block_add64(acc.mverts, &st.ctl->mverts);
    block_add64(acc.mslots, &st.ctl->mslots);
}

// ---------------------------------------------------------------------------
// Hub vertices: one block of 256 threads discharges (or merges) one vertex of
// very high degree, 256 slots at a time.  The block reproduces the group
// version exactly: the in-order push is a block prefix sum of the usable
// residuals clamped to the excess, the relabel candidate a block minimum and
// "skipped" a block OR, over the chunks a pass scans.

constexpr int HUB_BLOCK = 256;

// Inclusive prefix sum over the block; *total receives the block sum.  All
// threads must call it.  sh: LDS [HUB_BLOCK / 64].
__device__ __forceinline__ int64_t block_incl_scan64(int64_t x, int64_t &total, int64_t *sh)
{
    const int lane = lane_id(), wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, (unsigned)o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    int64_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < HUB_BLOCK / 64; k++) {
        const int64_t t = sh[k];
        if (k < wv) off += t;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return x + off;
}

__device__ __forceinline__ int block_min32(int x, int *sh)
{
    for (int o = 32; o > 0; o >>= 1) {
        const int y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    if (lane_id() == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    int m = sh[0];
#pragma unroll
    for (int k = 1; k < HUB_BLOCK / 64; k++) m = sh[k] < m ? sh[k] : m;
    __syncthreads();
    return m;
}

__device__ __forceinline__ int block_or32(int x, int *sh)
{
    for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
    if (lane_id() == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    int m = 0;
#pragma unroll
    for (int k = 0; k < HUB_BLOCK / 64; k++) m |= sh[k];
    __syncthreads();
    return m;
}

template <bool DENSE>
__device__ __forceinline__ void discharge_hub(const GraphView &g, StateView &st, const RoundParams &p, int v,
                                              DisAcc &acc, int64_t *sh64, int *sh32)
{
    const int n = g.n;
    const int beg = g.off[v], end = g.off[v + 1], deg = end - beg;
    const int tid = threadIdx.x;
    if (tid == 0) {
        acc.dverts++;
        acc.dslots += deg;
    }
    const int dv = st.d[v];
    int dp = dv;
    int64_t el = st.e[v];
    while (el > 0) {
        int cand = n;
        int sk = 0;
        for (int base = beg; base < end; base += HUB_BLOCK) {
            const int a = base + tid;
            int r = 0, w = -1, dw = 0;
            bool aw = false;
            if (a < end) {
                r = st.res[a];
                if (r > 0) {
                    w = g.head[a];
                    dw = st.d[w];
                    aw = st.act[w] != 0;
                }
            }
            if (tid == 0) acc.scans += (end - base) < HUB_BLOCK ? (end - base) : HUB_BLOCK;
            const bool adm = r > 0 && dp == dw + 1;
            const bool win = (dv == dw + 1) || (dv < dw - 1) || (dv == dw && v < w);
            const bool lose = !p.simple && adm && aw && !win;
            const bool use = adm && !lose;
            const int64_t amt = use ? (int64_t)r : 0;
            int64_t tot;
            const int64_t incl = block_incl_scan64(amt, tot, sh64);
            const int64_t excl = incl - amt;
            int dl = 0;
            if (use && excl < el) {
                const int64_t rem = el - excl;
                dl = rem < (int64_t)r ? (int)rem : r;
            }
            const bool into_sink = w == p.sink;
            if (dl > 0) {
                r -= dl;
                acc.pushes++;
                if (into_sink) {
                    st.res[g.rev[a]] += dl;
                    acc.to_sink += dl;
                } else {
                    st.delta[g.rev[a]] = dl;
                    if (DENSE) st.touched[w] = 1;
                }
                st.res[a] = r;
            }
            if (!DENSE) {
                const bool app = dl > 0 && !into_sink;
                const int idx = wave_append(app, w, st.C, &st.ctl->nc);
                if (app) st.owner[w] = idx;
            }
            el = tot >= el ? 0 : el - tot;
            if (el == 0) break;
            if (r > 0 && dw >= dp && dw + 1 < cand) cand = dw + 1;
            sk |= lose ? 1 : 0;
        }
        if (el == 0) break;
        const int nl = block_min32(cand, sh32);
        if (block_or32(sk, sh32)) break;
        dp = nl < n ? nl : n;
        if (tid == 0) {
            acc.work += deg + p.beta;
            acc.relabels++;
        }
        if (dp >= n) break;
        if (p.simple) break;
    }
    if (tid == 0) {
        st.dn[v] = dp;
        st.e[v] = el;
        if (DENSE) st.touched[v] = 1;
    }
    if (!DENSE) {
        const int idx = wave_append(tid == 0, v, st.C, &st.ctl->nc);
        if (tid == 0) st.owner[v] = idx;
    }
}

__device__ __forceinline__ void discharge_flush_hub(StateView &st, const RoundParams &p, DisAcc &acc)
{
    block_add64(acc.to_sink, &st.e[p.sink]);
    block_add64(acc.work, &st.ctl->work);
    block_add64(acc.pushes, &st.ctl->pushes);
    block_add64(acc.pushes, &st.ctl->dh_pushes);
    block_add64(acc.relabels, &st.ctl->relabels);
    block_add64(acc.scans, &st.ctl->scans);
    block_add64(acc.dverts, &st.ctl->dh_verts);
    block_add64(acc.dslots, &st.ctl->dh_slots);
}

__device__ __forceinline__ void merge_flush_hub(StateView &st, MerAcc &acc)
{
    block_add64(acc.mverts, &st.ctl->mh_verts);
    block_add64(acc.mslots, &st.ctl->mh_slots);
}

template <bool DENSE>
__device__ __forceinline__ void merge_hub(const GraphView &g, StateView &st, int w, int sink, int other,
                                          MerAcc &acc, Stage &sg, int64_t *sh64)
{
    const int beg = g.off[w], end = g.off[w + 1];
    const int tid = threadIdx.x;
    if (tid == 0) {
        acc.mverts++;
        acc.mslots += end - beg;
    }
    int64_t sum = 0;
    for (int a = beg + tid; a < end; a += HUB_BLOCK) {
        const int dl = st.delta[a];
        if (dl != 0) {
            st.res[a] += dl;
            st.delta[a] = 0;
            sum += dl;
        }
    }
    int64_t tot;
    (void)block_incl_scan64(sum, tot, sh64);
    bool pa = false;
    int dold = 0, dnew = 0;
    if (tid == 0) {
        const int64_t e = st.e[w] + tot;
        st.e[w] = e;
        dnew = st.dn[w];
        dold = st.d[w];
        st.d[w] = dnew;
        pa = w != sink && w != other && e > 0 && dnew < g.n;
        st.act[w] = pa;
        if (DENSE) st.touched[w] = 0;
    }
    if (st.lcount) {
        if (threadIdx.x < 64) gap_relabel_count(st, tid == 0 && dnew != dold, dold, dnew, g.n);
        return;
    }
    stage_append(sg, pa, w, st.A2, &st.ctl->na2);
}

}  // namespace mf
