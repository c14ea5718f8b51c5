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
// the sink (k_gr_init, k_gr_level per level, k_gr_rebuild).
#include "mf_device.h"

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
__global__ void k_saturate(GraphView g, StateView st)
{
    const int beg = g.off[g.s], end = g.off[g.s + 1];
    int64_t to_sink = 0;
    for (int a = beg + blockIdx.x * blockDim.x + threadIdx.x; a < end; a += gridDim.x * blockDim.x) {
        const int c = g.cap[a];
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
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += stride) {
        const int lab = v == sink ? 0 : g.n;
        st.d[v] = lab;
        st.dn[v] = lab;
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
    }
}

template <int G>
__global__ __launch_bounds__(256) void k_gr_td(GraphView g, StateView st, int level, int sink,
                                               int other, const int32_t *__restrict__ qin,
                                               int32_t *__restrict__ qout, int hubdeg)
{
    const int nq = st.ctl->nq[level % 3];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st.ctl->nq[(level + 2) % 3] = 0;
        st.ctl->nh[(level + 1) % 3] = 0;
    }
    const int gl = threadIdx.x & (G - 1);
    const int groups = blockDim.x / G;
    const int next = level + 1;
    int64_t gslots = 0;
    for (int i = blockIdx.x * groups + threadIdx.x / G; i < nq; i += gridDim.x * groups) {
        const int v = qin[i];
        const int beg = g.off[v], end = g.off[v + 1];
        if (end - beg > hubdeg) {
            wave_append(gl == 0, v, st.H, &st.ctl->nh[level % 3]);
            continue;
        }
        if (gl == 0) gslots += end - beg;
        for (int base = beg; base < end; base += G) {
            const int a = base + gl;
            bool claim = false;
            int w = 0;
            if (a < end) {
                w = g.head[a];
                if (w != sink && w != other && st.d[w] == g.n && st.res[g.rev[a]] > 0) {
                    if (atomicCAS(&st.d[w], g.n, next) == g.n) {
                        claim = true;
                        st.dn[w] = next;
                    }
                }
            }
            wave_append(claim, w, qout, &st.ctl->nq[next % 3]);
        }
    }
    block_add64(gslots, &st.ctl->gslots);
}

// The hub vertices of a top-down level, each expanded by every block.
__global__ __launch_bounds__(256) void k_gr_hub(GraphView g, StateView st, int level, int sink,
                                                int other, int32_t *__restrict__ qout)
{
    const int nh = st.ctl->nh[level % 3];
    const int next = level + 1;
    int64_t gslots = 0;
    for (int h = 0; h < nh; h++) {
        const int v = st.H[h];
        const int beg = g.off[v], end = g.off[v + 1];
        if (blockIdx.x == 0 && threadIdx.x == 0) gslots += end - beg;
        for (int base = beg + blockIdx.x * blockDim.x; base < end; base += gridDim.x * blockDim.x) {
            const int a = base + threadIdx.x;
            bool claim = false;
            int w = 0;
            if (a < end) {
                w = g.head[a];
                if (w != sink && w != other && st.d[w] == g.n && st.res[g.rev[a]] > 0) {
                    if (atomicCAS(&st.d[w], g.n, next) == g.n) {
                        claim = true;
                        st.dn[w] = next;
                    }
                }
            }
            wave_append(claim, w, qout, &st.ctl->nq[next % 3]);
        }
    }
    block_add64(gslots, &st.ctl->gslots);
}

__global__ __launch_bounds__(256) void k_gr_bu(GraphView g, StateView st, int level, int sink, int other)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st.ctl->nq[(level + 2) % 3] = 0;
        st.ctl->nh[(level + 1) % 3] = 0;
    }
    const int next = level + 1;
    int found = 0;
    int64_t gslots = 0;
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < g.n; w += gridDim.x * blockDim.x) {
        if (st.d[w] != g.n || w == sink || w == other) continue;
        const int beg = g.off[w], end = g.off[w + 1];
        for (int a = beg; a < end; a++) {
            gslots++;
            if (st.res[a] > 0 && st.d[g.head[a]] == level) {
                st.d[w] = next;
                st.dn[w] = next;
                found++;
                break;
            }
        }
    }
    block_add32(found, &st.ctl->nq[next % 3]);
    block_add64(gslots, &st.ctl->gslots);
}

// Frontier list of a level from the labels (after a bottom-up level).
__global__ void k_gr_collect(GraphView g, StateView st, int level, int32_t *__restrict__ qout)
{
    for (int base = blockIdx.x * blockDim.x; base < g.n; base += gridDim.x * blockDim.x) {
        const int v = base + threadIdx.x;
        const bool p = v < g.n && st.d[v] == level;
        wave_append(p, v, qout, &st.ctl->nq[(level + 2) % 3]);
    }
}

// Working set after a global relabel: every vertex other than the two
// terminals with positive excess and a label below n (dense flags + count).
__global__ void k_gr_rebuild(GraphView g, StateView st, int sink, int other)
{
    int cnt = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x) {
        const bool p = v != sink && v != other && st.e[v] > 0 && st.d[v] < g.n;
        st.act[v] = p;
        cnt += p;
    }
    block_add32(cnt, &st.ctl->na2);
}

// Working-set list from the activity flags.
__global__ void k_compact_act(GraphView g, StateView st)
{
    for (int base = blockIdx.x * blockDim.x; base < g.n; base += gridDim.x * blockDim.x) {
        const int v = base + threadIdx.x;
        const bool p = v < g.n && st.act[v];
        wave_append(p, v, st.A, &st.ctl->na);
    }
}

// ---------------------------------------------------------------------------
// Discharge (Listing 1, the loop over the working set).
//
// A round runs in one of two modes.  In list mode the working set is the list
// A and every touched vertex is appended to the candidate list C, with
// owner[w] naming one entry per vertex.  In dense mode (large working sets)
// the kernels walk all vertices: the working set is act[], and touched[]
// marks the vertices to merge, which avoids list appends altogether.

struct RoundParams {
    int64_t beta;      // work per relabel = outdeg + beta
    int sink;          // pushes into the sink go straight to its reverse slot and excess
};

// One pass over a chunk of up to G slots, in slot order.  Each lane holds one
// slot: r its residual, w its head, dw = d(w), aw = act(w).  Pushes along
// admissible arcs the vertex may use take min(r, e - excl) where excl is the
// total residual of the admissible, usable arcs before it in slot order: the
// result of visiting the arcs one after another.
//
// The sink never discharges and nobody reads its own slots or its excess
// during a round, so a push into the sink updates the reverse slot directly
// (each slot has one pusher) and is added to the sink's excess once per block.
template <int G, bool DENSE>
__device__ __forceinline__ int chunk_pass(const GraphView &g, StateView &st, int v, int dv, int dp,
                                          int gl, int a, int &r, int w, int dw, bool aw,
                                          int64_t &el, bool &lose, int64_t &pushes, int sink,
                                          int64_t &to_sink)
{
    const bool adm = r > 0 && dp == dw + 1;
    const bool win = (dv == dw + 1) || (dv < dw - 1) || (dv == dw && v < w);
    lose = adm && aw && !win;
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
        const int idx = wave_append(app, w, st.C, &st.ctl->nc);
        if (app) st.owner[w] = idx;
    }
    el = tot >= el ? 0 : el - tot;
    return dl;
}

template <int G, bool DENSE>
__global__ __launch_bounds__(256) void k_discharge(GraphView g, StateView st, RoundParams p)
{
    const int limit = DENSE ? g.n : st.ctl->na;
    const int gl = threadIdx.x & (G - 1);
    const int groups = blockDim.x / G;
    const int n = g.n;
    int64_t work = 0, pushes = 0, relabels = 0, scans = 0, to_sink = 0, dverts = 0, dslots = 0;
    for (int i = blockIdx.x * groups + threadIdx.x / G; i < limit; i += gridDim.x * groups) {
        int v;
        if (DENSE) {
            v = i;
            if (!st.act[v]) continue;
        } else {
            v = st.A[i];
        }
        const int beg = g.off[v], end = g.off[v + 1], deg = end - beg;
        if (gl == 0) {
            dverts++;
            dslots += deg;
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
                if (r > 0) {
                    w = g.head[a];
                    dw = st.d[w];
                    aw = st.act[w] != 0;
                }
            }
            bool dirty = false;
            while (el > 0) {
                if (gl == 0) scans += deg;
                bool lose;
                if (chunk_pass<G, DENSE>(g, st, v, dv, dp, gl, a, r, w, dw, aw, el, lose, pushes, p.sink,
                                         to_sink) > 0)
                    dirty = true;
                if (el == 0) break;
                const int cand = (r > 0 && dw >= dp) ? dw + 1 : n;
                const int nl = group_min<G>(cand);
                if (group_or<G>(lose ? 1 : 0)) break;          // skipped
                dp = nl < n ? nl : n;                            // relabel
                if (gl == 0) {
                    work += deg + p.beta;
                    relabels++;
                }
                if (dp >= n) break;
            }
            if (dirty) st.res[a] = r;
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
                        if (r > 0) {
                            w = g.head[a];
                            dw = st.d[w];
                            aw = st.act[w] != 0;
                        }
                    }
                    if (gl == 0) scans += (end - base) < G ? (end - base) : G;
                    bool lose;
                    if (chunk_pass<G, DENSE>(g, st, v, dv, dp, gl, a, r, w, dw, aw, el, lose, pushes,
                                             p.sink, to_sink) > 0)
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
                    work += deg + p.beta;
                    relabels++;
                }
                if (dp >= n) break;
            }
        }
        if (gl == 0) {
            st.dn[v] = dp;
            st.e[v] = el;
            if (DENSE) st.touched[v] = 1;
        }
        if (!DENSE) {
            const int idx = wave_append(gl == 0, v, st.C, &st.ctl->nc);
            if (gl == 0) st.owner[v] = idx;
        }
    }
    block_add64(to_sink, &st.e[p.sink]);
    block_add64(work, &st.ctl->work);
    block_add64(pushes, &st.ctl->pushes);
    block_add64(relabels, &st.ctl->relabels);
    block_add64(scans, &st.ctl->scans);
    block_add64(dverts, &st.ctl->dverts);
    block_add64(dslots, &st.ctl->dslots);
}

// ---------------------------------------------------------------------------
// Merge (Listing 1, the two loops after the discharge): e(w) += pushes
// received, d(w) := d'(w), new working set = touched vertices with e > 0 and
// d < n other than the terminals.  Each touched vertex is merged once: in
// list mode by the candidate entry that owns it, in dense mode by the walk
// over all vertices.

template <int G, bool DENSE>
__global__ __launch_bounds__(256) void k_merge(GraphView g, StateView st, int sink, int other)
{
    const int limit = DENSE ? g.n : st.ctl->nc;
    const int gl = threadIdx.x & (G - 1);
    const int groups = blockDim.x / G;
    int cnt = 0;
    int64_t mverts = 0, mslots = 0;
    for (int i = blockIdx.x * groups + threadIdx.x / G; i < limit; i += gridDim.x * groups) {
        int w;
        if (DENSE) {
            w = i;
            if (!st.touched[w]) continue;
        } else {
            w = st.C[i];
            if (st.owner[w] != i) continue;
        }
        const int beg = g.off[w], end = g.off[w + 1];
        if (gl == 0) {
            mverts++;
            mslots += end - beg;
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
        if (gl == 0) {
            const int64_t e = st.e[w] + sum;
            st.e[w] = e;
            const int dnew = st.dn[w];
            st.d[w] = dnew;
            pa = w != sink && w != other && e > 0 && dnew < g.n;
            st.act[w] = pa;
            if (DENSE) {
                st.touched[w] = 0;
                cnt += pa;
            }
        }
        if (!DENSE) wave_append(pa, w, st.A2, &st.ctl->na2);
    }
    if (DENSE) block_add32(cnt, &st.ctl->na2);
    block_add64(mverts, &st.ctl->mverts);
    block_add64(mslots, &st.ctl->mslots);
}

__global__ void k_round_reset(Ctl *ctl)
{
    ctl->nc = 0;
    ctl->na2 = 0;
    ctl->work = 0;
}

__global__ void k_round_end(Ctl *ctl)
{
    ctl->na = ctl->na2;
    ctl->na2 = 0;
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

void launch_discharge(int G, bool dense, GraphView g, StateView st, int64_t beta, int sink, int grid,
                      hipStream_t s)
{
    RoundParams p{beta, sink};
#define C_(X)                                                                                     \
    if (dense) hipLaunchKernelGGL((k_discharge<X, true>), dim3(grid), dim3(256), 0, s, g, st, p); \
    else hipLaunchKernelGGL((k_discharge<X, false>), dim3(grid), dim3(256), 0, s, g, st, p)
    MF_DISPATCH_G(G, C_)
#undef C_
}

void launch_merge(int G, bool dense, GraphView g, StateView st, int sink, int other, int grid,
                  hipStream_t s)
{
#define C_(X)                                                                                          \
    if (dense) hipLaunchKernelGGL((k_merge<X, true>), dim3(grid), dim3(256), 0, s, g, st, sink, other); \
    else hipLaunchKernelGGL((k_merge<X, false>), dim3(grid), dim3(256), 0, s, g, st, sink, other)
    MF_DISPATCH_G(G, C_)
#undef C_
}

void launch_gr_td(int G, GraphView g, StateView st, int level, int sink, int other, const int32_t *qin,
                  int32_t *qout, int hubdeg, int grid, hipStream_t s)
{
#define C_(X) hipLaunchKernelGGL((k_gr_td<X>), dim3(grid), dim3(256), 0, s, g, st, level, sink, other, qin, qout, hubdeg)
    MF_DISPATCH_G(G, C_)
#undef C_
}

void launch_gr_hub(GraphView g, StateView st, int level, int sink, int other, int32_t *qout, int grid,
                   hipStream_t s)
{
    hipLaunchKernelGGL(k_gr_hub, dim3(grid), dim3(256), 0, s, g, st, level, sink, other, qout);
}
void launch_gr_bu(GraphView g, StateView st, int level, int sink, int other, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_gr_bu, dim3(grid), dim3(256), 0, s, g, st, level, sink, other);
}
void launch_gr_collect(GraphView g, StateView st, int level, int32_t *qout, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_gr_collect, dim3(grid), dim3(256), 0, s, g, st, level, qout);
}
void launch_compact_act(GraphView g, StateView st, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_compact_act, dim3(grid), dim3(256), 0, s, g, st);
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
void launch_init_state(GraphView g, StateView st, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_state, dim3(grid), dim3(256), 0, s, g, st);
}
void launch_saturate(GraphView g, StateView st, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_saturate, dim3(grid), dim3(256), 0, s, g, st);
}
void launch_gr_init(GraphView g, StateView st, int sink, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_gr_init, dim3(grid), dim3(256), 0, s, g, st, sink);
}
void launch_gr_rebuild(GraphView g, StateView st, int sink, int other, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_gr_rebuild, dim3(grid), dim3(256), 0, s, g, st, sink, other);
}
void launch_round_reset(Ctl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k_round_reset, dim3(1), dim3(1), 0, s, ctl);
}
void launch_round_end(Ctl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k_round_end, dim3(1), dim3(1), 0, s, ctl);
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
void launch_read_value(const int64_t *e, int t, Ctl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k_read_value, dim3(1), dim3(1), 0, s, e, t, ctl);
}

}  // namespace mf
