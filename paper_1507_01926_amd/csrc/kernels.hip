// HIP kernels of the synchronous push-relabel solver (gfx950, wave64).
//
// One round of the synchronous method (Sec. 3.1) is two kernels:
//   k_discharge  every vertex of the working set is discharged by a group of
//                G lanes against the labels d, the excesses e and the
//                activity flags act of the start of the round, and against
//                its own residual capacities.  A push of delta on slot a
//                (v -> w) lowers res[a] (a slot only v writes during the
//                round) and stores delta at the reverse slot in the separate
//                array delta[], so nobody else's residuals change during the
//                round.  Every pushed-to vertex and v itself are appended
//                to a candidate list, and owner[w] records one entry per
//                vertex (plain stores; the last one wins).
//   k_merge      each candidate entry that owns its vertex w pulls the pushes
//                w received from its own delta segment (coalesced, no
//                atomics), applies them to res and e, applies the new label
//                and decides whether w is active in the next round.
// A global relabel (Sec. 2.1, Sec. 3) is a level-synchronous reverse BFS from
// the sink (k_gr_init, then k_gr_td or k_gr_bu per level, k_gr_rebuild).
#include <hip/hip_ext.h>

#include "mf_device.h"
#include "mf_phase.h"
#include "mf_steps.h"

namespace mf {

// ---------------------------------------------------------------------------
// Residency and validation

__global__ void k_narrow(const int64_t *__restrict__ off64, const int64_t *__restrict__ rev64,
                         int32_t *__restrict__ off, int32_t *__restrict__ rev, int32_t n,
                         int64_t slots, Ctl *ctl)
{
    int err = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t total = slots > (int64_t)n + 1 ? slots : (int64_t)n + 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        if (i <= n) {
            const int64_t o = off64[i];
            if (o < 0 || o > slots) err |= 1;
            if (i == 0 && o != 0) err |= 1;
            if (i == n && o != slots) err |= 1;
            if (i > 0 && o < off64[i - 1]) err |= 1;
            off[i] = (o < 0 || o > slots) ? 0 : (int32_t)o;
        }
        if (i < slots) {
            const int64_t r = rev64[i];
            const bool ok = r >= 0 && r < slots;
            if (!ok) err |= 2;
            rev[i] = ok ? (int32_t)r : (int32_t)i;
        }
    }
    if (err) atomicOr(&ctl->err, err);
}

// Tail of slot a by binary search over the offsets (used before rev is known
// to be consistent).
__device__ __forceinline__ int tail_of(const int32_t *__restrict__ off, int n, int a)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= a) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Requires offsets already checked (k_narrow) so that every segment lies in
// [0, slots).  Reads through rev only after checking it is in range.
__global__ void k_validate(GraphView g, Ctl *ctl)
{
    int err = 0;
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < g.slots; a += gridDim.x * blockDim.x) {
        const int v = tail_of(g.off, g.n, a);
        const int w = g.head[a];
        if (w < 0 || w >= g.n) { err |= 4; continue; }
        if (w == v) err |= 8;
        const int b = g.rev[a];
        if (b < 0 || b >= g.slots) { err |= 2; continue; }
        if (g.rev[b] != a || g.head[b] != v) err |= 16;
        const int64_t c = g.cap[a];
        if (c < 0) err |= 32;
        if (c + (int64_t)g.cap[b] > 2147483647LL) err |= 64;
    }
    if (err) atomicOr(&ctl->err, err);
}

// Degree figures that decide which global-relabel levels can meet a hub
// vertex: the largest out-degree over the vertices other than s and t, and
// the out-degrees of s and t (the BFS roots of the two phases).
__global__ void k_degree_stats(GraphView g, Ctl *ctl)
{
    int mx = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x) {
        const int deg = g.off[v + 1] - g.off[v];
        if (v == g.s) ctl->deg_s = deg;
        else if (v == g.t) ctl->deg_t = deg;
        else mx = max(mx, deg);
    }
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
    if (lane_id() == 0 && mx > 0) atomicMax(&ctl->maxdeg_inner, mx);
}

// ---------------------------------------------------------------------------
// Initialisation (Listing 1: d = 0, e = 0, f = 0, d(s) = n) and source
// saturation (every arc out of s carries its capacity).

__global__ void k_init_state(GraphView g, StateView st)
{
    const int stride = gridDim.x * blockDim.x;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int a = tid; a < g.slots; a += stride) {
        st.res[a] = g.cap[a];
        st.delta[a] = 0;
    }
    for (int v = tid; v < g.n; v += stride) {
        const int lab = v == g.s ? g.n : 0;
        st.d[v] = lab;
        st.dn[v] = lab;
        st.e[v] = 0;
        st.act[v] = 0;
        st.touched[v] = 0;
    }
}

// Saturation of the arcs out of s, written like a dense round: the heads
// receive the capacity in delta[] of the reverse slot and are marked touched;
// an arc into t goes straight to t (see chunk_pass).
// Saturates the arcs out of s: pushes each one's residual (its capacity
// after k_init_state, what the last flow left of it after k_warm_state).
// Start of a solve that resumes from the flow of the last complete solve:
// the residuals stay, and so does e(t) (the value so far); every other
// vertex had zero excess at the end of that solve.  Labels, flags and
// deltas start as in k_init_state.
__global__ void k_warm_state(GraphView g, StateView st)
{
    const int stride = gridDim.x * blockDim.x;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int a = tid; a < g.slots; a += stride) st.delta[a] = 0;
    for (int v = tid; v < g.n; v += stride) {
        const int lab = v == g.s ? g.n : 0;
        st.d[v] = lab;
        st.dn[v] = lab;
        if (v != g.t) st.e[v] = 0;
        st.act[v] = 0;
        st.touched[v] = 0;
    }
}

// New capacities of an uploaded graph; with `warm` the residuals of the kept
// flow move by the same amounts, and a slot whose new capacity is below its
// flow sets bit 128 of ctl->err.
__global__ void k_recap(GraphView g, const int32_t *__restrict__ cap_new, int32_t *res, int warm, Ctl *ctl)
{
    int bad = 0;
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < g.slots; a += gridDim.x * blockDim.x) {
        if (!warm) continue;
        const int64_t r = (int64_t)res[a] + cap_new[a] - g.cap[a];
        if (r < 0) bad = 1;
        res[a] = (int32_t)(r < 0 ? 0 : r);
    }
    if (bad) atomicOr(&ctl->err, 128);
}

__global__ void k_saturate(GraphView g, StateView st)
{
    const int beg = g.off[g.s], end = g.off[g.s + 1];
    int64_t to_sink = 0;
    for (int a = beg + blockIdx.x * blockDim.x + threadIdx.x; a < end; a += gridDim.x * blockDim.x) {
        const int c = st.res[a];
        if (c <= 0) continue;
        const int w = g.head[a];
        st.res[a] = 0;
        if (w == g.t) {
            st.res[g.rev[a]] += c;
            to_sink += c;
        } else {
            st.delta[g.rev[a]] = c;
            st.touched[w] = 1;
        }
    }
    block_add64(to_sink, &st.e[g.t]);
}

// ---------------------------------------------------------------------------
// State checks between rounds (MF_CHECK_INVARIANTS).  One thread per vertex
// walks the vertex's slots; bits of ctl->inv_err:
//   1  a residual below 0 (a flow above its capacity, Eq. 1)
//   2  res[a] + res[rev a] != cap[a] + cap[rev a] (antisymmetry, Eq. 1)
//   4  a push still pending (delta != 0) at a round boundary
//   8  an excess other than that of s differs from the net inflow its
//      residuals give (s's excess is not tracked: it is never read)
//   16 an excess below 0 at a vertex other than s (not a preflow)
//   32 a label outside [0, n], d(sink) != 0 or d(excluded terminal) != n
//   64 after a global relabel: d(v) > d(w) + 1 on a residual arc v -> w
//      (exact distances are valid labels, Sec. 2.1)
//   128 a touched mark left set between rounds
__global__ void k_check_state(GraphView g, StateView st, int sink, int other, int after_gr, Ctl *ctl)
{
    int err = 0;
    const int stride = gridDim.x * blockDim.x;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += stride) {
        const int beg = g.off[v], end = g.off[v + 1];
        const int dv = st.d[v];
        if (dv < 0 || dv > g.n || (v == sink && dv != 0) || (v == other && dv != g.n)) err |= 32;
        if (st.touched[v]) err |= 128;
        int64_t net = 0;
        for (int a = beg; a < end; a++) {
            const int r = st.res[a], b = g.rev[a];
            if (r < 0) err |= 1;
            if ((int64_t)r + st.res[b] != (int64_t)g.cap[a] + g.cap[b]) err |= 2;
            if (st.delta[a] != 0) err |= 4;
            net += (int64_t)r - g.cap[a];
            if (after_gr && r > 0 && v != other) {
                const int w = g.head[a];
                if (w != other && dv > st.d[w] + 1) err |= 64;
            }
        }
        if (v != g.s) {
            if (st.e[v] != net) err |= 8;
            if (st.e[v] < 0) err |= 16;
        }
    }
    if (err) atomicOr(&ctl->inv_err, err);
}

// Test hook of MF_CHECK_INVARIANTS: raises one residual by 1.
__global__ void k_bump(int32_t *p) { *p += 1; }

// ---------------------------------------------------------------------------
// Global relabel (Listing 2): d(v) = n for all v, d(sink) = 0, then one
// breadth-first level at a time.  w gets label L+1 when it has a residual arc
// w -> v into a vertex v of label L (c_f(w,v) > 0: the residual capacity of
// the reverse slot) and w is neither terminal.  A level runs either
//   top-down   over a list of the frontier: each frontier vertex claims its
//              unlabelled neighbours by compare-and-swap (as in Listing 2);
//              frontier vertices of degree above a threshold are put on a
//              hub list and expanded by the whole grid (k_gr_hub), or
//   bottom-up  over all vertices: every unlabelled vertex looks for a
//              neighbour of label L through its own residual slots (no
//              atomics; each vertex writes only its own label).
// Both give the same labels: exact distances are unique.

__global__ void k_gr_init(GraphView g, StateView st, int sink)
{
    const int stride = gridDim.x * blockDim.x;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int v = tid; v < g.n; v += stride) {
        st.d[v] = v == sink ? 0 : g.n;        // dn follows in k_gr_rebuild
    }
    if (st.hr) {
        // the residuals do not change during the relabel: pack "w can send
        // to v" (res of the reverse slot > 0) beside each slot's head
        for (int a = tid; a < g.slots; a += stride) {
            const int w = g.head[a];
            st.hr[a] = st.res[g.rev[a]] > 0 ? (int)((unsigned)w | 0x80000000u) : w;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st.Q[0] = sink;
        st.ctl->nq[0] = 1;
        st.ctl->nq[1] = 0;
        st.ctl->nq[2] = 0;
        st.ctl->nh[0] = 0;
        st.ctl->nh[1] = 0;
        st.ctl->nh[2] = 0;
        st.ctl->na = 0;
        st.ctl->na2 = 0;
        st.ctl->bfs_empty_level = 0x7fffffff;
        st.ctl->gr_found = 0;
        st.ctl->gr_found_deg = 0;
        st.ctl->fdeg[0] = g.off[sink + 1] - g.off[sink];
        st.ctl->fdeg[1] = 0;
        st.ctl->fdeg[2] = 0;
    }
}

// Top-down level.  Levels may be launched several at a time without the host
// reading the frontier sizes in between: a level whose frontier is empty
// records itself in bfs_empty_level and returns (every later level is empty
// too, since it finds nothing to expand).  Each non-empty level adds its
// frontier size to gr_found, from which the host derives the vertices a batch
// of levels labelled.
//
// With packed heads the level claims an open neighbour by compare-and-swap
// straight away, without reading its label first: a failed swap costs what
// the read would, and the chain of dependent loads gets one link shorter.
//
// Flags: TD_TRACK_DEG sums the slots of the claimed vertices (the
// direction choice on graphs with hubs), TD_EAGER reads the reverse residual
// of every slot together with the neighbour's label instead of after it,
// which takes one dependent load off the level's critical path at the cost
// of the reads for labelled neighbours (used for small frontiers, where
// latency bounds the level).  The slots a level expands are not counted here
// (a per-block count cost more than half the level's time); profiling gets
// them from k_gr_slots once the relabel is done.
constexpr int TD_TRACK_DEG = 1, TD_EAGER = 4;

template <int G>
__global__ __launch_bounds__(256) void k_gr_td(GraphView g, StateView st, int level, int sink,
                                               int other, const int32_t *__restrict__ qin,
                                               int32_t *__restrict__ qout, int hubdeg, int flags)
{
    const int nq = st.ctl->nq[level % 3];
    const int gl = threadIdx.x & (G - 1);
    const int groups = blockDim.x / G;
    const int stride = gridDim.x * groups;
    const int next = level + 1;
    int i = blockIdx.x * groups + threadIdx.x / G;
    // The first entry is read together with the frontier size (the queue
    // holds n entries, so the read stays in bounds; entries past the
    // frontier are not used).
    int v = i < g.n ? qin[i] : 0;
    __shared__ unsigned long long s_cdeg;
    if (threadIdx.x == 0) s_cdeg = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st.ctl->nq[(level + 2) % 3] = 0;
        st.ctl->fdeg[(level + 2) % 3] = 0;
        st.ctl->nh[(level + 1) % 3] = 0;
        if (nq == 0) atomicMin(&st.ctl->bfs_empty_level, level);
        else atomicAdd((unsigned long long *)&st.ctl->gr_found, (unsigned long long)nq);
    }
    if (i - threadIdx.x / G >= nq) return;          // no frontier vertex for this block
    MF_STAGE(stage);
    stage_init(stage);
    while (i < nq) {
        const int inext = i + stride;
        const int vnext = inext < nq ? qin[inext] : 0;
        const int beg = g.off[v], end = g.off[v + 1];
        if (end - beg > hubdeg) {
            wave_append(gl == 0, v, st.H, &st.ctl->nh[level % 3]);
        } else {
            for (int base = beg; base < end; base += G) {
                const int a = base + gl;
                bool claim = false;
                int w = 0;
                if (a < end) {
                    bool open;
                    if (st.hr) {
                        const int x = st.hr[a];
                        w = x & 0x7fffffff;
                        open = x < 0;
                    } else if (flags & TD_EAGER) {
                        w = g.head[a];
                        const int r = st.res[g.rev[a]];
                        open = st.d[w] == g.n && r > 0;
                    } else {
                        w = g.head[a];
                        open = st.d[w] == g.n && st.res[g.rev[a]] > 0;
                    }
                    if (open && w != sink && w != other && atomicCAS(&st.d[w], g.n, next) == g.n) {
                        claim = true;
                        if (flags & TD_TRACK_DEG)
                            atomicAdd(&s_cdeg, (unsigned long long)(g.off[w + 1] - g.off[w]));
                    }
                }
                stage_append(stage, claim, w, qout, &st.ctl->nq[next % 3]);
            }
        }
        i = inext;
        v = vnext;
    }
    stage_flush(stage, qout, &st.ctl->nq[next % 3]);
    if (threadIdx.x == 0 && (flags & TD_TRACK_DEG) && s_cdeg) {
        atomicAdd((unsigned long long *)&st.ctl->fdeg[next % 3], s_cdeg);
        atomicAdd((unsigned long long *)&st.ctl->gr_found_deg, s_cdeg);
    }
}

// Profiling: slots of the vertices a finished relabel expanded top-down,
// i.e. labelled vertices of degree at most hubdeg (hubs go to k_gr_hub),
// without those whose level ran bottom-up.  With lv.count == 0 the kernel
// adds the slots of every such labelled vertex to *out; otherwise it
// subtracts those of the vertices whose label is one of lv.
__global__ __launch_bounds__(256) void k_gr_slots(GraphView g, const int32_t *__restrict__ d, int hubdeg,
                                                  LevelSet lv, int64_t *out)
{
    int64_t s = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x) {
        const int L = d[v];
        if (L >= g.n) continue;
        const int deg = g.off[v + 1] - g.off[v];
        if (deg > hubdeg) continue;
        bool take = lv.count == 0;
        for (int k = 0; k < lv.count; k++) take |= L == lv.lv[k];
        if (take) s += deg;
    }
    block_add64(lv.count == 0 ? s : -s, out);
}

// The hub vertices of a top-down level, each expanded by every block.
__global__ __launch_bounds__(256) void k_gr_hub(GraphView g, StateView st, int level, int sink,
                                                int other, int32_t *__restrict__ qout, int track_deg)
{
    const int nh = st.ctl->nh[level % 3];
    const int next = level + 1;
    int64_t gslots = 0, cdeg = 0;
    MF_STAGE(stage);
    stage_init(stage);
    for (int h = 0; h < nh; h++) {
        const int v = st.H[h];
        const int beg = g.off[v], end = g.off[v + 1];
        if (blockIdx.x == 0 && threadIdx.x == 0) gslots += end - beg;
        for (int base = beg + blockIdx.x * blockDim.x; base < end; base += gridDim.x * blockDim.x) {
            const int a = base + threadIdx.x;
            bool claim = false;
            int w = 0;
            if (a < end) {
                bool open;
                if (st.hr) {
                    const int x = st.hr[a];
                    w = x & 0x7fffffff;
                    open = x < 0;
                } else {
                    w = g.head[a];
                    open = st.res[g.rev[a]] > 0;
                }
                if (open && w != sink && w != other && st.d[w] == g.n) {
                    if (atomicCAS(&st.d[w], g.n, next) == g.n) {
                        claim = true;
                        if (track_deg) cdeg += g.off[w + 1] - g.off[w];
                    }
                }
            }
            stage_append(stage, claim, w, qout, &st.ctl->nq[next % 3]);
        }
    }
    stage_flush(stage, qout, &st.ctl->nq[next % 3]);
    block_add64(gslots, &st.ctl->hslots);
    if (track_deg) {
        block_add64(cdeg, &st.ctl->fdeg[next % 3]);
        block_add64(cdeg, &st.ctl->gr_found_deg);
    }
}

__global__ __launch_bounds__(256) void k_gr_bu(GraphView g, StateView st, int level, int sink, int other)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st.ctl->nq[(level + 2) % 3] = 0;
        st.ctl->fdeg[(level + 2) % 3] = 0;
        st.ctl->nh[(level + 1) % 3] = 0;
    }
    const int next = level + 1;
    int found = 0;
    int64_t gslots = 0, cdeg = 0;
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < g.n; w += gridDim.x * blockDim.x) {
        if (st.d[w] != g.n || w == sink || w == other) continue;
        const int beg = g.off[w], end = g.off[w + 1];
        for (int a = beg; a < end; a++) {
            gslots++;
            if (st.res[a] > 0 && st.d[g.head[a]] == level) {
                st.d[w] = next;
                found++;
                cdeg += end - beg;
                break;
            }
        }
    }
    block_add32(found, &st.ctl->nq[next % 3]);
    block_add64(gslots, &st.ctl->gslots);
    block_add64(cdeg, &st.ctl->fdeg[next % 3]);
    block_add64(cdeg, &st.ctl->gr_found_deg);
}

// Frontier list of a level from the labels (after a bottom-up level).
__global__ __launch_bounds__(256) void k_gr_collect(GraphView g, StateView st, int level,
                                                    int32_t *__restrict__ qout)
{
    MF_STAGE(stage);
    stage_init(stage);
    for (int base = blockIdx.x * blockDim.x; base < g.n; base += gridDim.x * blockDim.x) {
        const int v = base + threadIdx.x;
        const bool p = v < g.n && st.d[v] == level;
        stage_append(stage, p, v, qout, &st.ctl->nq[(level + 2) % 3]);
    }
    stage_flush(stage, qout, &st.ctl->nq[(level + 2) % 3]);
}

// Working set after a global relabel: every vertex other than the two
// terminals with positive excess and a label below n (dense flags + count).
// After a global relabel: the round labels dn take the new labels (the
// levels write only d, so the label copies are one coalesced pass here
// instead of a scattered store per claimed vertex), and the working set is
// every vertex other than the terminals with excess and a label below n.
__global__ void k_gr_rebuild(GraphView g, StateView st, int sink, int other)
{
    int cnt = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x) {
        const int dv = st.d[v];
        st.dn[v] = dv;
        const bool p = v != sink && v != other && st.e[v] > 0 && dv < g.n;
        st.act[v] = p;
        cnt += p;
    }
    block_add32(cnt, &st.ctl->na2);
}

// ---------------------------------------------------------------------------
// Discharge (Listing 1, the loop over the working set).
//
// A round runs in one of two modes.  In list mode the working set is the list
// A and every touched vertex is appended to the candidate list C, with
// owner[w] naming one entry per vertex.  In dense mode (large working sets)
// the kernels walk all vertices: the working set is act[], and touched[]
// marks the vertices to merge, which avoids list appends altogether.

// List mode: the working set is A[0 .. na).  In a batch of speculative rounds
// a round after the one that stopped the batch does nothing.
template <int G, bool TWO>
__global__ __launch_bounds__(256) void k_discharge_list(GraphView g, StateView st, RoundParams p)
{
    if (st.ctl->batch_stop) return;
    const int na = st.ctl->na;
    const int gl = threadIdx.x & (G - 1);
    const int groups = blockDim.x / G;
    if (blockIdx.x * groups >= na) return;          // no vertex for this block
    DisAcc acc;
    MF_STAGE(stage);
    stage_init(stage);
    // every wave of the block runs the same number of iterations (the
    // vertices past na do nothing), so the stage's barriers see every wave
    const int span = gridDim.x * groups;
    const int iters = (na - blockIdx.x * groups + span - 1) / span;
    int i = blockIdx.x * groups + threadIdx.x / G;
    for (int it = 0; it < iters; it++, i += span) {
        if (i >= na) continue;
        const int v = st.A[i];
        if (g.off[v + 1] - g.off[v] > p.hubd) {        // left to k_discharge_hubs
            wave_append(gl == 0, v, st.H, &st.ctl->nhd);
            continue;
        }
        discharge_vertex<G, false, TWO>(g, st, p, v, gl, acc, &stage);
    }
    stage_flush_owner(stage, st.C, &st.ctl->nc, st.owner);
    discharge_flush(st, p, acc);
}

// Dense mode: the working set is act[], which k_compact_flags has listed in
// A[0 .. na) (in any order); the groups take the listed vertices in turn, so
// active vertices that cluster in one region of the graph still spread over
// the whole grid.  Pushes mark their heads in touched[] instead of appending
// candidates.
template <int G, bool TWO>
__global__ __launch_bounds__(256) void k_discharge_dense(GraphView g, StateView st, RoundParams p)
{
    if (st.ctl->batch_stop) return;
    const int na = st.ctl->na;
    const int gl = threadIdx.x & (G - 1);
    const int groups = blockDim.x / G;
    if (blockIdx.x * groups >= na) return;          // no vertex for this block
    DisAcc acc;
    for (int i = blockIdx.x * groups + threadIdx.x / G; i < na; i += gridDim.x * groups) {
        const int v = st.A[i];
        if (g.off[v + 1] - g.off[v] > p.hubd) {        // left to k_discharge_hubs
            wave_append(gl == 0, v, st.H, &st.ctl->nhd);
            continue;
        }
        discharge_vertex<G, true, TWO>(g, st, p, v, gl, acc);
    }
    discharge_flush(st, p, acc);
}

// ---------------------------------------------------------------------------
// Merge (Listing 1, the two loops after the discharge): e(w) += pushes
// received, d(w) := d'(w), new working set = touched vertices with e > 0 and
// d < n other than the terminals.  Each touched vertex is merged once: in
// list mode by the candidate entry that owns it, in dense mode by the walk
// over all vertices.

template <int G>
__global__ __launch_bounds__(256) void k_merge_list(GraphView g, StateView st, int sink, int other, int hubd)
{
    if (st.ctl->batch_stop) return;
    const int nc = st.ctl->nc;
    const int gl = threadIdx.x & (G - 1);
    const int groups = blockDim.x / G;
    if (blockIdx.x * groups >= nc) return;          // no vertex for this block
    MerAcc acc;
    MF_STAGE(stage);
    stage_init(stage);
    for (int i = blockIdx.x * groups + threadIdx.x / G; i < nc; i += gridDim.x * groups) {
        const int w = st.C[i];
        if (st.owner[w] != i) continue;
        if (g.off[w + 1] - g.off[w] > hubd) {           // left to k_merge_hubs
            wave_append(gl == 0, w, st.H, &st.ctl->nhm);
            continue;
        }
        merge_vertex<G, false>(g, st, w, gl, sink, other, acc, &stage);
    }
    stage_flush(stage, st.A2, &st.ctl->na2);
    merge_flush(st, false, acc);
}

// Dense mode: the touched vertices, listed in C[0 .. nc) by k_compact_flags.
template <int G>
__global__ __launch_bounds__(256) void k_merge_dense(GraphView g, StateView st, int sink, int other, int hubd)
{
    if (st.ctl->batch_stop) return;
    const int nc = st.ctl->nc;
    const int gl = threadIdx.x & (G - 1);
    const int groups = blockDim.x / G;
    if (blockIdx.x * groups >= nc) return;          // no vertex for this block
    MerAcc acc;
    MF_STAGE(stage);
    stage_init(stage);
    for (int i = blockIdx.x * groups + threadIdx.x / G; i < nc; i += gridDim.x * groups) {
        const int w = st.C[i];
        if (g.off[w + 1] - g.off[w] > hubd) {           // left to k_merge_hubs
            wave_append(gl == 0, w, st.H, &st.ctl->nhm);
            continue;
        }
        merge_vertex<G, true>(g, st, w, gl, sink, other, acc, &stage);
    }
    stage_flush(stage, st.A2, &st.ctl->na2);
    merge_flush(st, true, acc);
}

// Lists the vertices whose flag is set (in any order) and adds their number
// to *count.  Each lane tests 16 flags with one 16-byte load per step; a
// block scan places the step's entries in an LDS buffer that collects the
// block's entries over all its steps, and the block writes the buffer out
// with one atomic on *count when it is full or the block is done (device
// atomics on one counter serialize, so a launch makes as few as it can).
// flags must be 16-byte aligned.
constexpr int COMPACT_CAP = 8192;     // entries; a step adds at most 256 * 16 = 4096

__device__ __forceinline__ void compact_flush(int32_t *list, int32_t *count, int32_t *buf, int &held, int *s_base)
{
    // all threads of the block, held is block-uniform
    if (threadIdx.x == 0) *s_base = held ? atomicAdd(count, held) : 0;
    __syncthreads();
    const int g0 = *s_base;
    for (int j = threadIdx.x; j < held; j += blockDim.x) list[g0 + j] = buf[j];
    __syncthreads();
    held = 0;
}

__global__ __launch_bounds__(256) void k_compact_flags(const uint8_t *__restrict__ flags, int n,
                                                      int32_t *__restrict__ list, int32_t *count,
                                                      const int32_t *stop)
{
    if (stop && *stop) return;          // a later round of a stopped batch
    __shared__ int s_wave[4];
    __shared__ int s_base;
    __shared__ int32_t s_buf[COMPACT_CAP];
    const int nchunks = (n + 15) >> 4;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    int held = 0;                       // entries in s_buf (the same in every thread)
    for (int c0 = blockIdx.x * 256; c0 < nchunks; c0 += gridDim.x * 256) {
        const int c = c0 + threadIdx.x;
        unsigned bits = 0;
        if (c < nchunks) {
            if (16 * c + 16 <= n) {
                const uint4 q = ((const uint4 *)flags)[c];
                const unsigned wds[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                for (int k = 0; k < 4; k++)
#pragma unroll
                    for (int b = 0; b < 4; b++)
                        if ((wds[k] >> (8 * b)) & 0xffu) bits |= 1u << (4 * k + b);
            } else {
                for (int j = 0; 16 * c + j < n; j++)
                    if (flags[16 * c + j]) bits |= 1u << j;
            }
        }
        const int cnt = __popc(bits);
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        if (lane == 63) s_wave[wv] = incl;
        __syncthreads();
        int before = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int t = s_wave[k];
            if (k < wv) before += t;
            tot += t;
        }
        if (held + tot > COMPACT_CAP) compact_flush(list, count, s_buf, held, &s_base);
        int pos = held + before + incl - cnt;
        while (bits) {
            const int j = __ffs(bits) - 1;
            bits &= bits - 1;
            s_buf[pos++] = 16 * c + j;
        }
        held += tot;
        __syncthreads();
    }
    compact_flush(list, count, s_buf, held, &s_base);
}

// Hub vertices of the round, one block each (the vertices the discharge or
// merge kernels above left in H).
template <bool DENSE>
__global__ __launch_bounds__(256) void k_discharge_hubs(GraphView g, StateView st, RoundParams p)
{
    if (st.ctl->batch_stop) return;
    const int nh = st.ctl->nhd;
    if ((int)blockIdx.x >= nh) return;               // no hub for this block
    __shared__ int64_t sh64[HUB_BLOCK / 64];
    __shared__ int sh32[HUB_BLOCK / 64];
    DisAcc acc;
    for (int i = blockIdx.x; i < nh; i += gridDim.x) discharge_hub<DENSE>(g, st, p, st.H[i], acc, sh64, sh32);
    discharge_flush_hub(st, p, acc);
}

template <bool DENSE>
__global__ __launch_bounds__(256) void k_merge_hubs(GraphView g, StateView st, int sink, int other)
{
    if (st.ctl->batch_stop) return;
    const int nh = st.ctl->nhm;
    if ((int)blockIdx.x >= nh) return;               // no hub for this block
    __shared__ int64_t sh64[HUB_BLOCK / 64];
    MF_STAGE(stage);
    stage_init(stage);
    MerAcc acc;
    for (int i = blockIdx.x; i < nh; i += gridDim.x) merge_hub<DENSE>(g, st, st.H[i], sink, other, acc, stage, sh64);
    stage_flush(stage, st.A2, &st.ctl->na2);
    merge_flush_hub(st, acc);
}

__global__ void k_round_reset(Ctl *ctl, int dense)
{
    ctl->nc = 0;
    ctl->na2 = 0;
    ctl->work = 0;
    ctl->batch_stop = 0;
    ctl->nhd = 0;
    ctl->nhm = 0;
    if (dense) ctl->na = 0;        // the dense round lists its working set again
}

__global__ void k_round_end(Ctl *ctl)
{
    ctl->na = ctl->na2;
    ctl->na2 = 0;
}

// Speculative list rounds: the host launches several rounds of list mode
// without reading the counters in between.  k_round_begin opens the first
// round of a batch (and clears the stop flag and the round count);
// k_round_close adds the round's relabel work and charge to W and stops the
// batch when the next round must not run as a list round: its working set
// is empty or above the dense threshold, or W calls for a global relabel
// (the conditions the host checks after a single round).  A round that does
// not stop the batch makes the next working set current (na := na2) and
// opens the next round.
__global__ void k_round_begin(Ctl *ctl, int first)
{
    if (first) {
        ctl->batch_stop = 0;
        ctl->batch_rounds = 0;
    } else if (ctl->batch_stop) {
        return;
    }
    ctl->nc = 0;
    ctl->na2 = 0;
    ctl->work = 0;
    ctl->nhd = 0;
    ctl->nhm = 0;
}

// dense: a batch of dense rounds, which stops instead when the next working
// set is small enough for a list round (or empty).
__global__ void k_round_close(Ctl *ctl, int first, int64_t W0, int64_t charge, int64_t freq_num,
                              int64_t freq_den, int64_t gr_threshold, int64_t dense_threshold, int dense)
{
    if (ctl->batch_stop) return;
    const int64_t W = (first ? W0 : ctl->batch_W) + ctl->work + charge;
    ctl->batch_W = W;
    ctl->batch_rounds = first ? 1 : ctl->batch_rounds + 1;
    const int64_t next = ctl->na2;
    const bool other_kind = dense ? next <= dense_threshold : (next == 0 || next > dense_threshold);
    if (other_kind || freq_num * W > freq_den * gr_threshold) {
        ctl->batch_stop = 1;
        return;
    }
    ctl->na = ctl->na2;
    // open the next round (what k_round_begin does)
    ctl->nc = 0;
    ctl->na2 = 0;
    ctl->work = 0;
    ctl->nhd = 0;
    ctl->nhm = 0;
}

// ---------------------------------------------------------------------------
// Gap rule (Sec. 3 names gap relabeling, after Cherkassky and Goldberg), at
// the end of every round: the smallest label k in (0, n) that no vertex other
// than the terminals holds while some hold larger labels is a gap, and every
// label in (k, n) becomes n.  The merges keep the label histogram lcount and
// list the labels whose count fell to 0 during the round (gcand); since the
// rule leaves no hole behind, a gap can open only there.

// The round's gap: the smallest candidate whose count is still 0 (n: none).
__global__ __launch_bounds__(256) void k_gap_find(GraphView g, StateView st)
{
    Ctl *ctl = st.ctl;
    if (ctl->batch_stop) return;
    const int ngc = ctl->ngc;
    int best = g.n;
    for (int i = threadIdx.x; i < ngc; i += blockDim.x) {
        const int k = st.gcand[i];
        if (k > 0 && k < best && st.lcount[k] == 0) best = k;
    }
    __shared__ int sh[4];
    for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
    if (lane_id() == 0) sh[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        ctl->gap = min(min(sh[0], sh[1]), min(sh[2], sh[3]));
        ctl->ngc = 0;
    }
}

// Lifts every label in (gap, n) to n (vertices other than the terminals);
// they leave the working set.
__global__ __launch_bounds__(256) void k_gap_lift(GraphView g, StateView st, int sink, int other)
{
    Ctl *ctl = st.ctl;
    if (ctl->batch_stop) return;
    const int gap = ctl->gap;
    if (gap >= g.n) return;
    const int stride = gridDim.x * blockDim.x;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    int64_t lifted = 0;
    for (int v = tid; v < g.n; v += stride) {
        const int d = st.d[v];
        if (v != sink && v != other && d > gap && d < g.n) {
            st.d[v] = g.n;
            st.dn[v] = g.n;
            st.act[v] = 0;
            lifted++;
        }
    }
    for (int k = gap + 1 + tid; k < g.n; k += stride) st.lcount[k] = 0;
    block_add64(lifted, &ctl->gap_lifts);
}

// The next working set after the gap rule: the vertices merged this round
// (list rounds: the candidate entries that own their vertex; dense rounds:
// the listed touched vertices) that are active.
__global__ __launch_bounds__(256) void k_gap_next(GraphView g, StateView st, int sink, int other, int dense)
{
    Ctl *ctl = st.ctl;
    if (ctl->batch_stop) return;
    const int nc = ctl->nc;
    if ((int)(blockIdx.x * blockDim.x) >= nc) return;
    MF_STAGE(stage);
    stage_init(stage);
    for (int base = blockIdx.x * blockDim.x; base < nc; base += gridDim.x * blockDim.x) {
        const int i = base + threadIdx.x;
        bool pa = false;
        int w = 0;
        if (i < nc) {
            w = st.C[i];
            if (dense || st.owner[w] == i)
                pa = w != sink && w != other && st.e[w] > 0 && st.d[w] < g.n;
        }
        stage_append(stage, pa, w, st.A2, &ctl->na2);
    }
    stage_flush(stage, st.A2, &ctl->na2);
}

// The histogram after a global relabel (labels are exact distances then).
__global__ __launch_bounds__(256) void k_gap_clear(GraphView g, StateView st)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k <= g.n; k += gridDim.x * blockDim.x) st.lcount[k] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) st.ctl->ngc = 0;
}
__global__ __launch_bounds__(256) void k_gap_recount(GraphView g, StateView st, int sink, int other)
{
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < g.n; base += stride) {
        const int v = base + threadIdx.x;
        const int d = v < g.n ? st.d[v] : g.n;
        int amt;
        (void)wave_count_add(v < g.n && v != sink && v != other && d < g.n, d, 1, st.lcount, &amt);
    }
}

// ---------------------------------------------------------------------------
// Rounds of small working sets in one workgroup.  While the working set stays
// at or below `small_max` vertices, consecutive list rounds (the discharge
// and the merge above, with the same counters) run inside one workgroup of
// 1024 threads with block barriers between the steps, instead of three
// launches and a share of a host read-back per round.  Each round is a
// function of its start state, so the rounds are the ones the grid-wide
// kernels would run.  The kernel stops, as k_round_close stops a batch of
// speculative rounds, after the first round whose next working set is empty,
// larger than small_max or the dense threshold, or after which W calls for a
// global relabel, or when `budget` rounds have run; it leaves batch_rounds,
// batch_W and batch_stop = 1 as a stopped batch does (the next working set
// listed in the A2 of the stopping round).  Graphs with hub vertices do not
// use it (their hubs take a block each in the grid-wide rounds).
constexpr int BLOCK_ROUNDS_THREADS = 1024;

template <int G>
__global__ __launch_bounds__(BLOCK_ROUNDS_THREADS) void k_rounds_block(GraphView g, StateView st,
                                                                      RoundParams p, int other, int64_t W0,
                                                                      int64_t charge, int64_t freq_num,
                                                                      int64_t freq_den, int64_t gr_threshold,
                                                                      int64_t dense_threshold, int small_max,
                                                                      int64_t budget)
{
    Ctl *ctl = st.ctl;
    const int gl = threadIdx.x & (G - 1);
    const int groups = blockDim.x / G;
    MF_STAGE(stage);
    int32_t *A = st.A, *A2 = st.A2;
    int64_t W = W0;
    int rounds = 0;
    int na = ldc32(&ctl->na);
    while (true) {
        if (threadIdx.x == 0) {
            ctl->nc = 0;
            ctl->na2 = 0;
            ctl->work = 0;
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        StateView sr = st;
        sr.A = A;
        sr.A2 = A2;
        DisAcc dacc;
        for (int i = threadIdx.x / G; i < na; i += groups) discharge_vertex<G, false>(g, sr, p, A[i], gl, dacc);
        discharge_flush(sr, p, dacc);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const int nc = ldc32(&ctl->nc);
        MerAcc macc;
        stage_init(stage);
        for (int i = threadIdx.x / G; i < nc; i += groups) {
            const int w = st.C[i];
            if (st.owner[w] != i) continue;
            merge_vertex<G, false>(g, sr, w, gl, p.sink, other, macc, &stage);
        }
        stage_flush(stage, A2, &ctl->na2);
        merge_flush(sr, false, macc);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        W += ldc64(&ctl->work) + charge;
        rounds++;
        const int next = ldc32(&ctl->na2);
        const bool stop = next == 0 || next > small_max || next > dense_threshold ||
                          freq_num * W > freq_den * gr_threshold || rounds >= budget;
        if (stop) break;
        int32_t *t = A;
        A = A2;
        A2 = t;
        na = next;
        __syncthreads();          // every thread has read the counters before they are reset
    }
    if (threadIdx.x == 0) {
        ctl->batch_rounds = rounds;
        ctl->batch_W = W;
        ctl->batch_stop = 1;
        ctl->na = na;
    }
}


// ---------------------------------------------------------------------------
// Outputs.

__global__ void k_side(GraphView g, const int32_t *__restrict__ d, uint8_t *__restrict__ side)
{
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x)
        side[v] = d[v] < g.n ? 1 : 0;
}

// Cut capacity: sum of cap[a] over slots from the source side to the sink
// side; the tail of slot a is head[rev[a]].
__global__ void k_cut(GraphView g, const uint8_t *__restrict__ side, Ctl *ctl)
{
    int64_t sum = 0;
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < g.slots; a += gridDim.x * blockDim.x) {
        if (side[g.head[a]] && !side[g.head[g.rev[a]]]) sum += g.cap[a];
    }
    block_add64(sum, &ctl->cut);
}

__global__ void k_flow(GraphView g, const int32_t *__restrict__ res, int32_t *__restrict__ flow)
{
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < g.slots; a += gridDim.x * blockDim.x)
        flow[a] = g.cap[a] - res[a];
}

__global__ void k_read_value(const int64_t *e, int t, Ctl *ctl) { ctl->value = e[t]; }

// ---------------------------------------------------------------------------
// Launch helpers used by the host driver.

#define MF_DISPATCH_G(G, CALL)                    \
    switch (G) {                                  \
    case 1: CALL(1); break;                       \
    case 2: CALL(2); break;                       \
    case 4: CALL(4); break;                       \
    case 8: CALL(8); break;                       \
    case 16: CALL(16); break;                     \
    case 32: CALL(32); break;                     \
    default: CALL(64); break;                     \
    }

// A launch whose events are set records them from the kernel's dispatch (the
// timestamps of the kernel's own execution).
#define MF_LAUNCH(K, GRID, S, EV, ...)                                                                \
    do {                                                                                              \
        if ((EV).a) hipExtLaunchKernelGGL(K, dim3(GRID), dim3(256), 0, S, (EV).a, (EV).b, 0, __VA_ARGS__); \
        else hipLaunchKernelGGL(K, dim3(GRID), dim3(256), 0, S, __VA_ARGS__);                         \
    } while (0)

#define MF_LAUNCH_T(K, GRID, THREADS, S, EV, ...)                                                 \
    do {                                                                                              \
        if ((EV).a) hipExtLaunchKernelGGL(K, dim3(GRID), dim3(THREADS), 0, S, (EV).a, (EV).b, 0, __VA_ARGS__); \
        else hipLaunchKernelGGL(K, dim3(GRID), dim3(THREADS), 0, S, __VA_ARGS__);                     \
    } while (0)

void launch_gap_round(GraphView g, StateView st, int sink, int other, int dense, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_gap_find, dim3(1), dim3(256), 0, s, g, st);
    hipLaunchKernelGGL(k_gap_lift, dim3(grid), dim3(256), 0, s, g, st, sink, other);
    hipLaunchKernelGGL(k_gap_next, dim3(grid), dim3(256), 0, s, g, st, sink, other, dense);
}
void launch_gap_recount(GraphView g, StateView st, int sink, int other, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_gap_clear, dim3(grid), dim3(256), 0, s, g, st);
    hipLaunchKernelGGL(k_gap_recount, dim3(grid), dim3(256), 0, s, g, st, sink, other);
}

void launch_rounds_block(int G, GraphView g, StateView st, RoundParams p, int other, int64_t W0, int64_t charge,
                         int64_t freq_num, int64_t freq_den, int64_t gr_threshold, int64_t dense_threshold,
                         int small_max, int64_t budget, hipStream_t s, KEv ev)
{
#define C_(X) MF_LAUNCH_T((k_rounds_block<X>), 1, BLOCK_ROUNDS_THREADS, s, ev, g, st, p, other, W0, charge, \
                          freq_num, freq_den, gr_threshold, dense_threshold, small_max, budget)
    MF_DISPATCH_G(G, C_)
#undef C_
}

void launch_discharge(int G, bool dense, GraphView g, StateView st, RoundParams p, int grid, hipStream_t s,
                      KEv ev, bool two)
{
    // the two-chunk variants exist for 4 and 8 lanes
    if (two && G == 4) {
        if (dense) MF_LAUNCH((k_discharge_dense<4, true>), grid, s, ev, g, st, p);
        else MF_LAUNCH((k_discharge_list<4, true>), grid, s, ev, g, st, p);
        return;
    }
    if (two && G == 8) {
        if (dense) MF_LAUNCH((k_discharge_dense<8, true>), grid, s, ev, g, st, p);
        else MF_LAUNCH((k_discharge_list<8, true>), grid, s, ev, g, st, p);
        return;
    }
#define C_(X)                                                             \
    if (dense) MF_LAUNCH((k_discharge_dense<X, false>), grid, s, ev, g, st, p); \
    else MF_LAUNCH((k_discharge_list<X, false>), grid, s, ev, g, st, p)
    MF_DISPATCH_G(G, C_)
#undef C_
}

void launch_merge(int G, bool dense, GraphView g, StateView st, int sink, int other, int hubd, int grid,
                  hipStream_t s, KEv ev)
{
#define C_(X)                                                                     \
    if (dense) MF_LAUNCH((k_merge_dense<X>), grid, s, ev, g, st, sink, other, hubd); \
    else MF_LAUNCH((k_merge_list<X>), grid, s, ev, g, st, sink, other, hubd)
    MF_DISPATCH_G(G, C_)
#undef C_
}

void launch_discharge_hubs(bool dense, GraphView g, StateView st, RoundParams p, int grid, hipStream_t s, KEv ev)
{
    p.hubd = 0x7fffffff;
    if (dense) MF_LAUNCH(k_discharge_hubs<true>, grid, s, ev, g, st, p);
    else MF_LAUNCH(k_discharge_hubs<false>, grid, s, ev, g, st, p);
}

void launch_merge_hubs(bool dense, GraphView g, StateView st, int sink, int other, int grid, hipStream_t s, KEv ev)
{
    if (dense) MF_LAUNCH(k_merge_hubs<true>, grid, s, ev, g, st, sink, other);
    else MF_LAUNCH(k_merge_hubs<false>, grid, s, ev, g, st, sink, other);
}

void launch_gr_td(int G, GraphView g, StateView st, int level, int sink, int other, const int32_t *qin,
                  int32_t *qout, int hubdeg, int flags, int grid, hipStream_t s, KEv ev)
{
#define C_(X) MF_LAUNCH((k_gr_td<X>), grid, s, ev, g, st, level, sink, other, qin, qout, hubdeg, flags)
    MF_DISPATCH_G(G, C_)
#undef C_
}

void launch_gr_hub(GraphView g, StateView st, int level, int sink, int other, int32_t *qout, int track_deg,
                   int grid, hipStream_t s, KEv ev)
{
    MF_LAUNCH(k_gr_hub, grid, s, ev, g, st, level, sink, other, qout, track_deg);
}
void launch_gr_bu(GraphView g, StateView st, int level, int sink, int other, int grid, hipStream_t s, KEv ev)
{
    MF_LAUNCH(k_gr_bu, grid, s, ev, g, st, level, sink, other);
}
void launch_gr_collect(GraphView g, StateView st, int level, int32_t *qout, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_gr_collect, dim3(grid), dim3(256), 0, s, g, st, level, qout);
}
void launch_compact_flags(const uint8_t *flags, int n, int32_t *list, int32_t *count, int maxgrid, hipStream_t s,
                          KEv ev, const int32_t *stop)
{
    const int chunks = (n + 15) / 16;
    int grid = (chunks + 255) / 256;
    if (grid > maxgrid) grid = maxgrid;
    if (grid < 1) grid = 1;
    MF_LAUNCH(k_compact_flags, grid, s, ev, flags, n, list, count, stop);
}
void launch_narrow(const int64_t *off64, const int64_t *rev64, int32_t *off, int32_t *rev, int32_t n,
                   int64_t slots, Ctl *ctl, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_narrow, dim3(grid), dim3(256), 0, s, off64, rev64, off, rev, n, slots, ctl);
}
void launch_validate(GraphView g, Ctl *ctl, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_validate, dim3(grid), dim3(256), 0, s, g, ctl);
}
void launch_degree_stats(GraphView g, Ctl *ctl, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_degree_stats, dim3(grid), dim3(256), 0, s, g, ctl);
}
void launch_init_state(GraphView g, StateView st, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_state, dim3(grid), dim3(256), 0, s, g, st);
}
void launch_saturate(GraphView g, StateView st, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_saturate, dim3(grid), dim3(256), 0, s, g, st);
}
void launch_warm_state(GraphView g, StateView st, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_warm_state, dim3(grid), dim3(256), 0, s, g, st);
}
void launch_recap(GraphView g, const int32_t *cap_new, int32_t *res, int warm, Ctl *ctl, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_recap, dim3(grid), dim3(256), 0, s, g, cap_new, res, warm, ctl);
}
void launch_gr_init(GraphView g, StateView st, int sink, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_gr_init, dim3(grid), dim3(256), 0, s, g, st, sink);
}
void launch_gr_slots(GraphView g, const int32_t *d, int hubdeg, LevelSet lv, int64_t *out, int grid,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_gr_slots, dim3(grid), dim3(256), 0, s, g, d, hubdeg, lv, out);
}
void launch_gr_rebuild(GraphView g, StateView st, int sink, int other, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_gr_rebuild, dim3(grid), dim3(256), 0, s, g, st, sink, other);
}
void launch_round_reset(Ctl *ctl, bool dense, hipStream_t s)
{
    hipLaunchKernelGGL(k_round_reset, dim3(1), dim3(1), 0, s, ctl, dense ? 1 : 0);
}
void launch_round_end(Ctl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k_round_end, dim3(1), dim3(1), 0, s, ctl);
}
void launch_round_begin(Ctl *ctl, int first, hipStream_t s)
{
    hipLaunchKernelGGL(k_round_begin, dim3(1), dim3(1), 0, s, ctl, first);
}
void launch_round_close(Ctl *ctl, int first, int64_t W0, int64_t charge, int64_t freq_num, int64_t freq_den,
                        int64_t gr_threshold, int64_t dense_threshold, hipStream_t s, int dense)
{
    hipLaunchKernelGGL(k_round_close, dim3(1), dim3(1), 0, s, ctl, first, W0, charge, freq_num, freq_den,
                       gr_threshold, dense_threshold, dense);
}
void launch_side(GraphView g, const int32_t *d, uint8_t *side, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_side, dim3(grid), dim3(256), 0, s, g, d, side);
}
void launch_cut(GraphView g, const uint8_t *side, Ctl *ctl, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_cut, dim3(grid), dim3(256), 0, s, g, side, ctl);
}
void launch_flow(GraphView g, const int32_t *res, int32_t *flow, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_flow, dim3(grid), dim3(256), 0, s, g, res, flow);
}
void launch_check_state(GraphView g, StateView st, int sink, int other, int after_gr, int grid, hipStream_t s)
{
    k_check_state<<<grid, 256, 0, s>>>(g, st, sink, other, after_gr, st.ctl);
}

void launch_bump(int32_t *p, hipStream_t s) { k_bump<<<1, 1, 0, s>>>(p); }

void launch_read_value(const int64_t *e, int t, Ctl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k_read_value, dim3(1), dim3(1), 0, s, e, t, ctl);
}

}  // namespace mf
