// Persistent solver kernel: one cooperative launch runs a whole phase of the
// synchronous push-relabel method (Sec. 3.1, Listing 1): global relabels
// (Listing 2, one breadth-first level per step) and rounds (discharge, then
// merge), with a grid-wide barrier between steps instead of kernel launches
// and host round trips.  Every block takes the same control decisions from
// the same counters read after a barrier, so the blocks stay in lock step.
//
// The grid barrier waits a bounded time: if a block does not arrive within
// the limit (which no correct step comes near), the barrier sets an abort
// flag, every block leaves at its next barrier, and the host reports a
// device error.
#include "mf_device.h"
#include "mf_phase.h"
#include "mf_steps.h"

namespace mf {



// Memory ordering: every wave waits for its own outstanding stores before the
// block barrier; thread 0 then releases the block's writes to device scope
// (one L2 write-back for the block) before it arrives, and after the other
// blocks have arrived it acquires (one cache invalidation for the block's
// compute unit) before the block goes on.
__device__ __forceinline__ bool grid_sync(GridBar *bar, uint64_t limit_ticks)
{
    __shared__ int s_ok;
    __builtin_amdgcn_s_waitcnt(0);   // this wave's loads and stores have completed
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned g = __hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived =
            __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        if (arrived == gridDim.x) {
            __hip_atomic_store(&bar->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar->gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // Waiting blocks back off (up to about 2000 cycles between
            // polls): hundreds of blocks polling one line at full rate keep
            // its L2 channel busy and slow the blocks still working.
            const uint64_t t0 = wall_clock64();
            unsigned nap = 1, polls = 0;
            while (__hip_atomic_load(&bar->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if ((++polls & 15) == 0) {
                    if (__hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                    if (wall_clock64() - t0 > limit_ticks) {
                        __hip_atomic_store(&bar->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                }
                for (unsigned k = 0; k < nap; k++) __builtin_amdgcn_s_sleep(1);
                if (nap < 32) nap <<= 1;
            }
        }
        s_ok = __hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return s_ok != 0;
}

__device__ __forceinline__ int ld32(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t ld64(const int64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct GridTeam {
    GridBar *bar;
    uint64_t limit_ticks;
    __device__ int brank() const { return blockIdx.x; }
    __device__ int nblocks() const { return gridDim.x; }
    __device__ bool sync() { return grid_sync(bar, limit_ticks); }
};

struct BlockTeam {
    __device__ int brank() const { return 0; }
    __device__ int nblocks() const { return 1; }
    __device__ bool sync()
    {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        return true;
    }
};

// One phase of the solve run by a team of threads: the whole grid (GridTeam,
// grid barriers) or one block (BlockTeam, block barriers).
// ring[0..2]: per-round counters, round r uses ring[r % 3]; gc: global-relabel
// counters and the phase results.  Returns 0 done, 1 round limit, 2 aborted.
template <int G, class Team>
__device__ int run_phase_team(Team &tm, Stage &stage, const GraphView &g, const StateView &st,
                              const PhaseParams &P, Ctl *ring, Ctl *gc)
{
    constexpr int GPW = 64 / G;
    const int n = g.n;
    const int64_t m = g.slots;
    const int lane = lane_id();
    const int gl = lane & (G - 1);
    const int grp = lane / G;
    const int groups = blockDim.x / G;
    const int brank = tm.brank(), nblocks = tm.nblocks();
    const int gtid = brank * blockDim.x + threadIdx.x;
    const int gthreads = nblocks * blockDim.x;
    const int wave = gtid >> 6;
    const int nwaves = gthreads >> 6;
    const int sink = P.sink, other = P.other;
    const RoundParams rp{P.beta, sink, 0x7fffffff, P.simple};

    int64_t W = 0;
    int64_t depth = 0;           // depth of the last global relabel
    bool force = true;
    int count = 0;
    bool dense = false;
    int32_t *A = st.A, *A2 = st.A2;
    int64_t rounds = 0, grs = 0, levels = 0, dense_rounds = 0, bu_levels = 0;
    int status = 0;

    while (true) {
        bool just = false;
        if (force || P.freq_num * W > P.freq_den * (P.alpha * n + m + P.level_charge * depth)) {
            // ---------------- global relabel ----------------
            for (int v = gtid; v < n; v += gthreads) {
                const int lab = v == sink ? 0 : n;
                st.d[v] = lab;
                st.dn[v] = lab;
            }
            if (gtid == 0) {
                st.Q[0] = sink;
                gc->nq[0] = 1;
                gc->nq[1] = 0;
                gc->nq[2] = 0;
                gc->nh[0] = 0;
                gc->nh[1] = 0;
                gc->nh[2] = 0;
                gc->na = 0;
                gc->na2 = 0;
            }
            if (!tm.sync()) goto aborted;
            int level = 0;
            int64_t nq = 1, unvisited = n - 2;
            int32_t *qin = st.Q, *qout = st.Q2;
            while (nq > 0) {
                const int next = level + 1;
                int32_t *qcount = &gc->nq[next % 3];
                if (gtid == 0) {
                    gc->nq[(level + 2) % 3] = 0;
                    gc->nh[next % 3] = 0;
                }
                int64_t gslots = 0;
                stage_init(stage);
                if (nq * P.bu_factor > unvisited) {
                    bu_levels++;
                    // bottom-up: each unlabelled vertex looks for a neighbour of
                    // label `level` through its own residual slots
                    for (int base = brank * blockDim.x; base < n; base += gthreads) {
                        const int w = base + threadIdx.x;
                        bool found = false;
                        if (w < n && w != sink && w != other && st.d[w] == n) {
                            const int beg = g.off[w], end = g.off[w + 1];
                            for (int a = beg; a < end; a++) {
                                gslots++;
                                if (st.res[a] > 0 && st.d[g.head[a]] == level) {
                                    found = true;
                                    break;
                                }
                            }
                            if (found) {
                                st.d[w] = next;
                                st.dn[w] = next;
                            }
                        }
                        stage_append(stage, found, w, qout, qcount);
                    }
                    stage_flush(stage, qout, qcount);
                } else {
                    // top-down over the frontier list; hubs are set aside
                    for (int i = brank * groups + threadIdx.x / G; i < nq; i += nblocks * groups) {
                        const int v = qin[i];
                        const int beg = g.off[v], end = g.off[v + 1];
                        if (end - beg > P.hubdeg) {
                            wave_append(gl == 0, v, st.H, &gc->nh[level % 3]);
                            continue;
                        }
                        if (gl == 0) gslots += end - beg;
                        for (int base = beg; base < end; base += G) {
                            const int a = base + gl;
                            bool claim = false;
                            int w = 0;
                            if (a < end) {
                                w = g.head[a];
                                if (w != sink && w != other && st.d[w] == n && st.res[g.rev[a]] > 0) {
                                    if (atomicCAS(&st.d[w], n, next) == n) {
                                        claim = true;
                                        st.dn[w] = next;
                                    }
                                }
                            }
                            stage_append(stage, claim, w, qout, qcount);
                        }
                    }
                    stage_flush(stage, qout, qcount);
                    if (!tm.sync()) goto aborted;
                    const int nh = ld32(&gc->nh[level % 3]);
                    if (nh > 0) {
                        stage_init(stage);
                        for (int h = 0; h < nh; h++) {
                            const int v = st.H[h];
                            const int beg = g.off[v], end = g.off[v + 1];
                            if (gtid == 0) gslots += end - beg;
                            for (int base = beg + brank * blockDim.x; base < end; base += gthreads) {
                                const int a = base + threadIdx.x;
                                bool claim = false;
                                int w = 0;
                                if (a < end) {
                                    w = g.head[a];
                                    if (w != sink && w != other && st.d[w] == n && st.res[g.rev[a]] > 0) {
                                        if (atomicCAS(&st.d[w], n, next) == n) {
                                            claim = true;
                                            st.dn[w] = next;
                                        }
                                    }
                                }
                                stage_append(stage, claim, w, qout, qcount);
                            }
                        }
                        stage_flush(stage, qout, qcount);
                    }
                }
                block_add64(gslots, &gc->gslots);
                if (!tm.sync()) goto aborted;
                nq = ld32(qcount);
                unvisited -= nq;
                int32_t *tq = qin;
                qin = qout;
                qout = tq;
                level = next;
            }
            levels += level - 1;
            depth = level - 1;
            grs++;
            // working set: every non-terminal vertex with excess and label < n
            {
                int cnt = 0;
                for (int v = gtid; v < n; v += gthreads) {
                    const bool p = v != sink && v != other && st.e[v] > 0 && st.d[v] < n;
                    st.act[v] = p;
                    cnt += p;
                }
                block_add32(cnt, &gc->na2);
            }
            if (!tm.sync()) goto aborted;
            count = ld32(&gc->na2);
            dense = count > P.dense_threshold;
            if (!dense && count > 0) {
                stage_init(stage);
                for (int base = brank * blockDim.x; base < n; base += gthreads) {
                    const int v = base + threadIdx.x;
                    stage_append(stage, v < n && st.act[v], v, A, &gc->na);
                }
                stage_flush(stage, A, &gc->na);
                if (!tm.sync()) goto aborted;
            }
            W = 0;
            force = false;
            just = true;
        }
        if (count == 0) {
            if (just) break;           // a fresh global relabel found no active vertex
            force = true;
            continue;
        }
        if (P.max_rounds > 0 && rounds >= P.max_rounds) {
            status = 1;
            break;
        }
        // ---------------- one round ----------------
        {
            Ctl *rc = &ring[rounds % 3];
            if (gtid == 0) {
                Ctl *nx = &ring[(rounds + 1) % 3];
                nx->nc = 0;
                nx->na2 = 0;
                nx->na = 0;
                nx->work = 0;
            }
            StateView sr = st;
            sr.ctl = rc;
            sr.A = A;
            sr.A2 = A2;
            DisAcc dacc;
            if (dense) dense_rounds++;
            if (dense) {
                for (int base = wave * 64; base < n; base += nwaves * 64) {
                    const int v0 = base + lane;
                    const uint64_t mask = __ballot(v0 < n && st.act[v0] != 0);
                    const int cnt = __popcll(mask);
                    for (int k0 = 0; k0 < cnt; k0 += GPW) {
                        const int k = k0 + grp;
                        if (k < cnt) discharge_vertex<G, true>(g, sr, rp, base + nth_set_bit(mask, k), gl, dacc);
                    }
                }
            } else {
                for (int i = brank * groups + threadIdx.x / G; i < count; i += nblocks * groups)
                    discharge_vertex<G, false>(g, sr, rp, A[i], gl, dacc);
            }
            discharge_flush(sr, rp, dacc);
            if (!tm.sync()) goto aborted;
            MerAcc macc;
            stage_init(stage);
            if (dense) {
                for (int base = wave * 64; base < n; base += nwaves * 64) {
                    const int v0 = base + lane;
                    const uint64_t mask = __ballot(v0 < n && st.touched[v0] != 0);
                    const int cnt = __popcll(mask);
                    for (int k0 = 0; k0 < cnt; k0 += GPW) {
                        const int k = k0 + grp;
                        if (k < cnt)
                            merge_vertex<G, true>(g, sr, base + nth_set_bit(mask, k), gl, sink, other, macc, &stage);
                    }
                }
            } else {
                const int nc = ld32(&rc->nc);
                for (int i = brank * groups + threadIdx.x / G; i < nc; i += nblocks * groups) {
                    const int w = st.C[i];
                    if (st.owner[w] != i) continue;
                    merge_vertex<G, false>(g, sr, w, gl, sink, other, macc, &stage);
                }
            }
            stage_flush(stage, sr.A2, &sr.ctl->na2);
            merge_flush(sr, dense, macc);
            if (!tm.sync()) goto aborted;
            const int nxt = ld32(&rc->na2);
            W += ld64(&rc->work) + P.round_charge;
            rounds++;
            const bool was_dense = dense;
            dense = nxt > P.dense_threshold;
            if (!was_dense && !dense) {
                int32_t *t = A;
                A = A2;
                A2 = t;
            } else if (was_dense && !dense && nxt > 0) {
                stage_init(stage);
                for (int base = brank * blockDim.x; base < n; base += gthreads) {
                    const int v = base + threadIdx.x;
                    stage_append(stage, v < n && st.act[v], v, A, &rc->na);
                }
                stage_flush(stage, A, &rc->na);
                if (!tm.sync()) goto aborted;
            }
            count = nxt;
        }
    }
    if (gtid == 0) {
        gc->p_rounds = rounds;
        gc->p_grs = grs;
        gc->p_levels = levels;
        gc->p_status = status;
        gc->p_lists = A == st.A ? 0 : 1;
        gc->p_dense_rounds = dense_rounds;
        gc->p_bu_levels = bu_levels;
    }
    return status;
aborted:
    if (gtid == 0) gc->p_status = 2;
    return 2;
}


template <int G>
__global__ __launch_bounds__(256) void k_phase(GraphView g, StateView st, PhaseParams P, Ctl *ring,
                                               Ctl *gc, GridBar *bar)
{
    MF_STAGE(stage);
    GridTeam tm{bar, P.limit_ticks};
    run_phase_team<G>(tm, stage, g, st, P, ring, gc);
}

// ---------------------------------------------------------------------------
// Batched solver: one persistent launch over a table of instances; each block
// takes the next instance from a queue and solves it completely (init,
// saturation, phase 1, value / sink side / cut, phase 2, flow) with block
// barriers only, so instances of any mix of sizes run side by side.




__device__ void zero_ctls(Ctl *c, int k)
{
    int32_t *w = (int32_t *)c;
    const int words = k * (int)(sizeof(Ctl) / sizeof(int32_t));
    for (int i = threadIdx.x; i < words; i += blockDim.x) w[i] = 0;
}

// Copies `bytes` between host and device memory by one block; both ends
// 16-byte aligned.  Four 16-byte accesses are in flight per lane, since a
// load from host memory waits for a PCIe round trip.
__device__ __forceinline__ void block_copy(void *__restrict__ dst, const void *__restrict__ src, int64_t bytes)
{
    const int64_t nv = bytes >> 4;
    const int4 *__restrict__ s4 = (const int4 *)src;
    int4 *__restrict__ d4 = (int4 *)dst;
    const int B = blockDim.x;
    int64_t i = threadIdx.x;
    for (; i + 3 * B < nv; i += 4 * B) {
        const int4 x0 = s4[i], x1 = s4[i + B], x2 = s4[i + 2 * B], x3 = s4[i + 3 * B];
        d4[i] = x0;
        d4[i + B] = x1;
        d4[i + 2 * B] = x2;
        d4[i + 3 * B] = x3;
    }
    for (; i < nv; i += B) d4[i] = s4[i];
    const uint8_t *s1 = (const uint8_t *)src;
    uint8_t *d1 = (uint8_t *)dst;
    for (int64_t j = 16 * nv + threadIdx.x; j < bytes; j += B) d1[j] = s1[j];
}

__device__ __forceinline__ int32_t narrow_one(int64_t x, int64_t j, int64_t hi, int32_t &err, int32_t bit,
                                              bool self_fill)
{
    const bool ok = x >= 0 && x <= hi;
    if (!ok) err |= bit;
    return ok ? (int32_t)x : (self_fill ? (int32_t)j : 0);
}

// Narrows `count` int64 values from host memory into int32 device memory,
// flagging values outside [0, hi] (replaced by 0, or by their own index when
// self_fill, so that later reads stay in bounds).  src 16-byte aligned.
__device__ __forceinline__ void block_narrow(int32_t *__restrict__ dst, const int64_t *__restrict__ src,
                                             int64_t count, int64_t hi, int32_t &err, int32_t bit, bool self_fill)
{
    const int64_t np = count >> 1;          // pairs
    const int4 *__restrict__ s4 = (const int4 *)src;
    const int B = blockDim.x;
    auto put = [&](int64_t p, int4 q) {
        const int64_t x0 = (int64_t)(uint32_t)q.x | ((int64_t)q.y << 32);
        const int64_t x1 = (int64_t)(uint32_t)q.z | ((int64_t)q.w << 32);
        dst[2 * p] = narrow_one(x0, 2 * p, hi, err, bit, self_fill);
        dst[2 * p + 1] = narrow_one(x1, 2 * p + 1, hi, err, bit, self_fill);
    };
    int64_t p = threadIdx.x;
    for (; p + 3 * B < np; p += 4 * B) {
        const int4 q0 = s4[p], q1 = s4[p + B], q2 = s4[p + 2 * B], q3 = s4[p + 3 * B];
        put(p, q0);
        put(p + B, q1);
        put(p + 2 * B, q2);
        put(p + 3 * B, q3);
    }
    for (; p < np; p += B) put(p, s4[p]);
    if ((count & 1) && threadIdx.x == 0) dst[count - 1] = narrow_one(src[count - 1], count - 1, hi, err, bit, self_fill);
}

// Residency step done by the block that takes a served request: pull the
// graph from host memory, narrow the int64 offsets and reverse slots to
// int32, and check it (the checks of k_narrow and k_validate; eight lanes
// walk the slots of one vertex).  Returns true if the graph is valid.
__device__ __forceinline__ bool block_prepare(const BatchItem &it)
{
    __shared__ int s_err;
    const GraphView g = it.g;
    const int n = g.n, S = g.slots;
    // the host wrote the request before publishing it; drop any cached copy
    // of an earlier request that used the same host or device memory
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
    if (threadIdx.x == 0) s_err = 0;
    int32_t err = 0;
    int32_t *off = (int32_t *)g.off, *rev = (int32_t *)g.rev;
    block_narrow(off, it.off64, (int64_t)n + 1, S, err, 1, false);
    block_narrow(rev, it.rev64, S, (int64_t)S - 1, err, 2, true);
    block_copy((void *)g.head, it.head_h, 4 * (int64_t)S);
    block_copy((void *)g.cap, it.cap_h, 4 * (int64_t)S);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0 && (off[0] != 0 || off[n] != S)) err |= 1;
    constexpr int L = 8;
    const int team = threadIdx.x / L, gl = threadIdx.x % L, teams = blockDim.x / L;
    for (int v = team; v < n; v += teams) {
        const int a0 = off[v], a1 = off[v + 1];
        if (a1 < a0) err |= 1;
        for (int a = a0 + gl; a < a1; a += L) {
            const int w = g.head[a];
            if (w < 0 || w >= n) { err |= 4; continue; }
            if (w == v) err |= 8;
            const int b = rev[a];
            if (rev[b] != a || g.head[b] != v) err |= 16;
            const int64_t c = g.cap[a];
            if (c < 0) err |= 32;
            if (c + (int64_t)g.cap[b] > 2147483647LL) err |= 64;
        }
    }
    if (err) atomicOr(&s_err, err);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    return s_err == 0;
}

// Sends the sink side and the flow of a finished served request to its host
// buffers and makes them visible to the host before the block reports done.
__device__ __forceinline__ void block_publish(const BatchItem &it)
{
    if (it.side_h && it.side) block_copy(it.side_h, it.side, it.g.n);
    if (it.flow_h && it.flow) block_copy(it.flow_h, it.flow, 4 * (int64_t)it.g.slots);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
}

template <int G>
__device__ __forceinline__ void solve_block(const BatchItem &it, BatchResult *out, int32_t *sbuf,
                                            int32_t *scnt, int32_t *sbase)
{
    constexpr int GPW = 64 / G;
    Stage stage{sbuf, scnt, sbase};
    BlockTeam tm;
    const GraphView g = it.g;
    StateView st = it.st;
    Ctl *ctl = it.ctl;
    const int n = g.n;
    const int lane = lane_id();
    const int gl = lane & (G - 1);
    const int grp = lane / G;
    zero_ctls(ctl, 5);
    st.ctl = ctl;
    // Listing 1 initialisation and saturation of the arcs out of s
    for (int a = threadIdx.x; a < g.slots; a += blockDim.x) {
        st.res[a] = g.cap[a];
        st.delta[a] = 0;
    }
    for (int v = threadIdx.x; v < n; v += blockDim.x) {
        const int lab = v == g.s ? n : 0;
        st.d[v] = lab;
        st.dn[v] = lab;
        st.e[v] = 0;
        st.act[v] = 0;
        st.touched[v] = 0;
    }
    tm.sync();
    {
        int64_t to_sink = 0;
        for (int a = g.off[g.s] + threadIdx.x; a < g.off[g.s + 1]; a += blockDim.x) {
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
    tm.sync();
    {
        MerAcc macc;
        for (int base = (threadIdx.x >> 6) * 64; base < n; base += blockDim.x) {
            const int v0 = base + lane;
            const uint64_t mask = __ballot(v0 < n && st.touched[v0] != 0);
            const int cnt = __popcll(mask);
            for (int k0 = 0; k0 < cnt; k0 += GPW) {
                const int k = k0 + grp;
                if (k < cnt) merge_vertex<G, true>(g, st, base + nth_set_bit(mask, k), gl, g.t, g.s, macc, nullptr);
            }
        }
        merge_flush(st, true, macc);
    }
    tm.sync();
    PhaseParams P = it.p;
    P.sink = g.t;
    P.other = g.s;
    int status = run_phase_team<G>(tm, stage, g, st, P, ctl + 1, ctl + 4);
    tm.sync();
    BatchResult r{};
    if (threadIdx.x == 0) r.t_phase1 = wall_clock64();
    r.rounds = ctl[4].p_rounds;
    r.grs = ctl[4].p_grs;
    r.levels = ctl[4].p_levels;
    // value, sink side (exact labels of the last global relabel) and cut capacity
    uint8_t *side = it.side ? it.side : st.touched;
    for (int v = threadIdx.x; v < n; v += blockDim.x) side[v] = st.d[v] < n ? 1 : 0;
    tm.sync();
    {
        int64_t cut = 0;
        for (int a = threadIdx.x; a < g.slots; a += blockDim.x)
            if (side[g.head[a]] && !side[g.head[g.rev[a]]]) cut += g.cap[a];
        block_add64(cut, &ctl[0].cut);
    }
    tm.sync();
    r.value = st.e[g.t];
    r.cut = ctl[0].cut;
    for (int i = 1; i <= 3; i++) {
        r.pushes += ctl[i].pushes;
        r.relabels += ctl[i].relabels;
    }
    if (!it.preflow_only && status == 0) {
        tm.sync();
        zero_ctls(ctl + 1, 4);
        tm.sync();
        P.sink = g.s;
        P.other = g.t;
        status = run_phase_team<G>(tm, stage, g, st, P, ctl + 1, ctl + 4);
        tm.sync();
        r.rounds2 = ctl[4].p_rounds;
        r.grs2 = ctl[4].p_grs;
        if (it.flow)
            for (int a = threadIdx.x; a < g.slots; a += blockDim.x) it.flow[a] = g.cap[a] - st.res[a];
    } else if (status == 1 && it.flow) {
        // round limit: the flow output holds the preflow reached
        for (int a = threadIdx.x; a < g.slots; a += blockDim.x) it.flow[a] = g.cap[a] - st.res[a];
    }
    r.status = status;
    tm.sync();
    if (threadIdx.x == 0) {
        r.t_end = wall_clock64();
        r.t_start = out->t_start;
        r.t_solve = out->t_solve;
        r.block = blockIdx.x;
        *out = r;
    }
}

// One launch per lane count G: items[order[0 .. count)] are the instances of
// this launch.
template <int G>
__global__ __launch_bounds__(BATCH_BLOCK) void k_batch(const BatchItem *__restrict__ items,
                                                       const int32_t *__restrict__ order,
                                                       BatchResult *results, BatchQueue *q)
{
    __shared__ int32_t sbuf[STAGE_CAP];
    __shared__ int32_t scnt, sbase;
    __shared__ int s_i;
    const int count = q->count;
    while (true) {
        if (threadIdx.x == 0) s_i = atomicAdd(&q->next, 1);
        __syncthreads();
        // instance indices are block-uniform: keep them (and the descriptor
        // loads through them) in scalar registers
        const int j = __builtin_amdgcn_readfirstlane(s_i);
        __syncthreads();
        if (j >= count) break;
        const int i = __builtin_amdgcn_readfirstlane(order[j]);
        if (threadIdx.x == 0) results[i].t_start = wall_clock64();
        solve_block<G>(items[i], &results[i], sbuf, &scnt, &sbase);
        __syncthreads();
    }
}

hipError_t launch_batch(int G, int grid, const BatchItem *items, const int32_t *order, BatchResult *results,
                        BatchQueue *q, hipStream_t s)
{
    switch (G) {
    case 4: hipLaunchKernelGGL(k_batch<4>, dim3(grid), dim3(BATCH_BLOCK), 0, s, items, order, results, q); break;
    case 8: hipLaunchKernelGGL(k_batch<8>, dim3(grid), dim3(BATCH_BLOCK), 0, s, items, order, results, q); break;
    case 16: hipLaunchKernelGGL(k_batch<16>, dim3(grid), dim3(BATCH_BLOCK), 0, s, items, order, results, q); break;
    default: hipLaunchKernelGGL(k_batch<32>, dim3(grid), dim3(BATCH_BLOCK), 0, s, items, order, results, q); break;
    }
    return hipGetLastError();
}

__global__ void k_queue_init(BatchQueue *q, int count)
{
    q->next = 0;
    q->count = count;
}

void launch_queue_init(BatchQueue *q, int count, hipStream_t s)
{
    hipLaunchKernelGGL(k_queue_init, dim3(1), dim3(1), 0, s, q, count);
}

template <int G>
__device__ __forceinline__ void solve_block_any(const BatchItem &it, BatchResult *out, int32_t *sbuf,
                                                int32_t *scnt, int32_t *sbase)
{
    if constexpr (G > 0) {
        solve_block<G>(it, out, sbuf, scnt, sbase);
    } else {
        switch (it.G) {
        case 4: solve_block<4>(it, out, sbuf, scnt, sbase); break;
        case 8: solve_block<8>(it, out, sbuf, scnt, sbase); break;
        case 16: solve_block<16>(it, out, sbuf, scnt, sbase); break;
        default: solve_block<32>(it, out, sbuf, scnt, sbase); break;
        }
    }
}

// Served requests.  Workgroup 0 watches the host-side queue: it copies the
// published count and the shutdown flag into device memory (mirror[0],
// mirror[1]) about once a microsecond, so the other workgroups, which take
// the requests, poll device memory only.  A workgroup claims the next
// published item by compare-and-swap on `next` (an item is claimed only once
// it is published), solves it (G = 0: with the item's own lane count) and
// writes the result and a done mark to host memory.  Every workgroup leaves
// when the host asks for shutdown or when no request has arrived for
// idle_ticks, so every wave exits.
template <int G>
__global__ __launch_bounds__(BATCH_BLOCK) void k_serve(ServeHostQueue *hq, int32_t *next, uint64_t idle_ticks, int epoch)
{
    __shared__ int32_t sbuf[STAGE_CAP];
    __shared__ int32_t scnt, sbase;
    __shared__ int s_i;
    __shared__ BatchItem s_item;
    __shared__ BatchResult s_res;
    int32_t *mirror = next + 4;       // [0] published count, [1] shutdown
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            int last = __hip_atomic_load(&hq->count, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&mirror[0], last, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            uint64_t t0 = wall_clock64();
            while (true) {
                const int c = __hip_atomic_load(&hq->count, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
                if (c != last) {
                    last = c;
                    __hip_atomic_store(&mirror[0], c, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    t0 = wall_clock64();
                }
                if (__hip_atomic_load(&hq->shutdown, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) {
                    __hip_atomic_store(&mirror[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                // keep watching while requests are still being solved
                const int nx = __hip_atomic_load(next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int dn = __hip_atomic_load(&mirror[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (nx >= c && dn >= nx && wall_clock64() - t0 > idle_ticks) break;
                __builtin_amdgcn_s_sleep(32);
            }
            __hip_atomic_store(&mirror[3], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    while (true) {
        if (threadIdx.x == 0) {
            int claimed = -1;
            uint64_t t0 = wall_clock64();
            int seen = -1;
            int backoff = 1;
            while (true) {
                const int c = __hip_atomic_load(&mirror[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                int nx = __hip_atomic_load(next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (nx < c) {
                    if (__hip_atomic_compare_exchange_strong(next, &nx, nx + 1, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)) {
                        claimed = nx;
                        break;
                    }
                    continue;
                }
                if (c != seen) {
                    seen = c;
                    t0 = wall_clock64();
                }
                // leave when the watcher has left, on shutdown, or (a backstop
                // in case the watcher is not running) after a long quiet spell
                if (__hip_atomic_load(&mirror[3], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == epoch) break;
                if (__hip_atomic_load(&mirror[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                if (wall_clock64() - t0 > 50 * idle_ticks) break;
                // Idle workgroups back off exponentially (to about 50 us
                // between polls): hundreds of them polling one cache line
                // would keep its L2 channel busy and slow the solving
                // workgroups' loads that map to it.
                for (int k = 0; k < backoff; k++) __builtin_amdgcn_s_sleep(127);
                backoff = backoff < 16 ? 2 * backoff : 16;
            }
            s_i = claimed;
            if (claimed >= 0) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");    // the item is host-written
                s_item = hq->items[claimed % SERVE_CAP];
                s_res = BatchResult{};
                s_res.t_start = wall_clock64();
            }
        }
        __syncthreads();
        const int i = __builtin_amdgcn_readfirstlane(s_i);
        if (i < 0) break;
        // the descriptor is the same for the whole block: read it into scalar
        // registers (its pointers then need no vector registers)
        BatchItem it;
        {
            static_assert(sizeof(BatchItem) % 4 == 0, "descriptor of 32-bit words");
            const int *src = (const int *)&s_item;
            int *dst = (int *)&it;
#pragma unroll
            for (int k = 0; k < (int)(sizeof(BatchItem) / 4); k++) dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
        }
        if (block_prepare(it)) {
            if (threadIdx.x == 0) s_res.t_solve = wall_clock64();
            solve_block_any<G>(it, &s_res, sbuf, &scnt, &sbase);
        } else if (threadIdx.x == 0) {
            s_res.status = 3;    // invalid graph
        }
        __syncthreads();
        if (s_res.status == 0) block_publish(it);
        __syncthreads();
        if (threadIdx.x == 0) {
            s_res.t_end = wall_clock64();
            hq->results[i % SERVE_CAP] = s_res;
            __hip_atomic_store(&hq->done[i % SERVE_CAP], i + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_fetch_add(&mirror[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

hipError_t launch_serve(int G, int grid, ServeHostQueue *hq, int32_t *next, uint64_t idle_ticks, int epoch,
                        hipStream_t s)
{
    switch (G) {
    case 0: hipLaunchKernelGGL(k_serve<0>, dim3(grid), dim3(BATCH_BLOCK), 0, s, hq, next, idle_ticks, epoch); break;
    case 4: hipLaunchKernelGGL(k_serve<4>, dim3(grid), dim3(BATCH_BLOCK), 0, s, hq, next, idle_ticks, epoch); break;
    case 8: hipLaunchKernelGGL(k_serve<8>, dim3(grid), dim3(BATCH_BLOCK), 0, s, hq, next, idle_ticks, epoch); break;
    case 16: hipLaunchKernelGGL(k_serve<16>, dim3(grid), dim3(BATCH_BLOCK), 0, s, hq, next, idle_ticks, epoch); break;
    default: hipLaunchKernelGGL(k_serve<32>, dim3(grid), dim3(BATCH_BLOCK), 0, s, hq, next, idle_ticks, epoch); break;
    }
    return hipGetLastError();
}

int serve_blocks_per_cu(int G)
{
    int nb = 0;
    const void *f = G == 0 ? (const void *)k_serve<0> : G == 4 ? (const void *)k_serve<4>
                  : G == 8 ? (const void *)k_serve<8> : G == 16 ? (const void *)k_serve<16>
                  : (const void *)k_serve<32>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, BATCH_BLOCK, 0) != hipSuccess) return 0;
    return nb;
}

int batch_blocks_per_cu(int G)
{
    int nb = 0;
    const void *f = G == 4 ? (const void *)k_batch<4> : G == 8 ? (const void *)k_batch<8>
                  : G == 16 ? (const void *)k_batch<16> : (const void *)k_batch<32>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, BATCH_BLOCK, 0) != hipSuccess) return 0;
    return nb;
}

// ---------------------------------------------------------------------------

template <int G>
static hipError_t launch_phase_t(int grid, GraphView g, StateView st, PhaseParams P, Ctl *ring, Ctl *gc,
                                 GridBar *bar, hipStream_t s)
{
    void *args[] = {&g, &st, &P, &ring, &gc, &bar};
    return hipLaunchCooperativeKernel((const void *)k_phase<G>, dim3(grid), dim3(256), args, 0, s);
}

template <int G>
static int phase_blocks_per_cu_t()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)k_phase<G>, 256, 0) != hipSuccess)
        return 0;
    return nb;
}

#define MF_DISPATCH_G2(G, CALL)                   \
    switch (G) {                                  \
    case 1: return CALL(1);                       \
    case 2: return CALL(2);                       \
    case 4: return CALL(4);                       \
    case 8: return CALL(8);                       \
    case 16: return CALL(16);                     \
    case 32: return CALL(32);                     \
    default: return CALL(64);                     \
    }

hipError_t launch_phase(int G, int grid, GraphView g, StateView st, PhaseParams P, Ctl *ring, Ctl *gc,
                        GridBar *bar, hipStream_t s)
{
#define C_(X) launch_phase_t<X>(grid, g, st, P, ring, gc, bar, s)
    MF_DISPATCH_G2(G, C_)
#undef C_
}

int phase_blocks_per_cu(int G)
{
#define C_(X) phase_blocks_per_cu_t<X>()
    MF_DISPATCH_G2(G, C_)
#undef C_
}

}  // namespace mf
