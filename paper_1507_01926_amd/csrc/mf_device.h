// Device-side data layout and wave helpers shared by the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf {

// Library-owned device copy of a validated graph; int32 offsets and reverse
// slots (the library requires slots < 2^31 - 1).
struct GraphView {
    int32_t n, s, t;
    int32_t slots;
    const int32_t *off;    // [n+1]
    const int32_t *head;   // [slots]
    const int32_t *rev;    // [slots]
    const int32_t *cap;    // [slots]
};

// Counters written by the kernels and read back by the host driver.  Every
// counter that many blocks of one launch add to (one atomic per block) sits on
// a 256-byte line of its own (MF_HOT): device atomics on one line serialize,
// about 12 ns each on MI355X, so counters sharing a line cost their sum and
// counters on separate lines proceed in parallel.
#define MF_HOT alignas(256)
struct Ctl {
    MF_HOT int32_t na;     // entries of the current working-set list
    MF_HOT int32_t na2;    // size of the next working set (list entries or dense count)
    MF_HOT int32_t nc;     // entries of the candidate list
    MF_HOT int32_t nq[3];  // BFS frontier sizes, ring indexed by level % 3
    int32_t nh[3];         // BFS hub-list sizes, ring indexed by level % 3
    int32_t err;           // validation error bits
    MF_HOT int64_t work;   // relabel work of the round (sum of outdeg + beta)
    MF_HOT int64_t pushes;
    MF_HOT int64_t relabels;
    MF_HOT int64_t scans;
    MF_HOT int64_t dverts;     // vertices discharged and their slots (first pass)
    MF_HOT int64_t dslots;
    MF_HOT int64_t mverts;     // vertices merged and their slots
    MF_HOT int64_t mslots;
    MF_HOT int64_t gslots;     // slots examined by global-relabel levels
    // results of a persistent phase launch
    MF_HOT int64_t p_rounds;
    int64_t p_grs, p_levels, p_dense_rounds, p_bu_levels;
    int32_t p_status, p_lists;
    MF_HOT int64_t cut;    // cut capacity accumulator
    int64_t value;         // scratch for the host
    MF_HOT int64_t hslots; // slots examined by hub expansions (host-driven levels)
    int32_t maxdeg_inner;  // largest out-degree over vertices other than s and t
    int32_t deg_s, deg_t;  // out-degrees of s and t
    int32_t bfs_empty_level;   // first top-down level of this relabel that found its frontier empty
    int64_t gr_found;      // sum of the frontier sizes of the top-down levels of this relabel
    // speculative list rounds: rounds run since the batch began, the stop
    // flag (set by the round that ends the batch) and the relabel work W
    int32_t batch_rounds, batch_stop;
    int64_t batch_W;
    // hub vertices of a round (discharged / merged by a block each) and
    // the counters of the hub kernels
    int32_t nhd, nhm;
    MF_HOT int64_t dh_verts;
    int64_t dh_slots, dh_pushes, mh_verts, mh_slots;
    // global relabel: out-degree sum of each BFS frontier (ring by level % 3)
    // and of every vertex labelled so far (edge-based direction choice)
    MF_HOT int64_t fdeg[3];
    MF_HOT int64_t gr_found_deg;
    MF_HOT int64_t td_slots;   // profiling: slots expanded by the top-down levels of a relabel
    int32_t inv_err;       // MF_CHECK_INVARIANTS: bits of the checks that failed (k_check_state)
    MF_HOT int32_t ngc;    // gap rule: candidate labels of the round
    int32_t gap;           // gap rule: the round's gap (n: none)
    MF_HOT int64_t gap_lifts;  // gap rule: labels set to n by it
};

// Parameters of a discharge step (host-built, passed to the kernels by value).
struct RoundParams {
    int64_t beta;      // work per relabel = outdeg + beta
    int sink;          // pushes into the sink go straight to its reverse slot and excess
    int hubd = 0x7fffffff;   // vertices of higher degree are left to a block each (hub kernels)
    // The simple synchronous variant of Sec. 3 (the paper's first design):
    // every admissible arc is used, with no win criterion, and an active
    // vertex makes one pass over its arcs and at most one relabel per round.
    int simple = 0;
};

// Per-solve state.  Every array lives in device memory.
//   res[a]    residual capacity of slot a as of the last round end
//   delta[a]  push received on slot a during the current round (a push on
//             slot b by head[a] is stored at a = rev[b]); 0 outside rounds
//   d[v]      label at the start of the round; dn[v] label after v's discharge
//   e[v]      excess; act[v] 1 iff v is in the working set
//   owner[w]  index of the candidate-list entry that merges w this round
//   touched[w] 1 iff w was pushed to or discharged in the current round (dense
//             rounds only; all zero between rounds)
struct StateView {
    int32_t *res, *delta, *d, *dn, *owner;
    int64_t *e;
    uint8_t *act, *touched;
    int32_t *H;            // BFS hub list (frontier vertices of high degree)
    int32_t *A, *A2;       // working-set lists (current, next)
    int32_t *C;            // candidate list (vertices touched in the round)
    int32_t *Q, *Q2;       // BFS frontiers
    // hr[a] = head[a] with bit 31 set iff the reverse slot holds residual
    // capacity (res[rev a] > 0), rebuilt at the start of each global relabel:
    // a top-down level then reads one coalesced word per slot (each edge
    // carries its reverse edge's residual, the representation of Sec. 4.2).
    // Null where not provided; the levels then gather res[rev a].
    int32_t *hr;
    // Gap rule (null when off): lcount[k] = number of vertices other than the
    // terminals with label k < n; gcand lists the labels whose count fell to 0
    // during the current round (ctl->ngc entries).
    int32_t *lcount, *gcand;
    Ctl *ctl;
};

// Loads of counters other waves or blocks update with atomics: relaxed
// agent-scope atomic loads, which never return a stale cached copy.
__device__ __forceinline__ int ldc32(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t ldc64(const int64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Wave helpers (wave64).  A "group" is G consecutive lanes of a wave that
// cooperate on one vertex; G divides 64.

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `mask` below the calling lane.
__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <int G>
__device__ __forceinline__ int64_t group_incl_scan(int64_t x, int gl)
{
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        int64_t y = __shfl_up(x, (unsigned)o, G);
        if (gl >= o) x += y;
    }
    return x;
}

template <int G>
__device__ __forceinline__ int64_t group_bcast(int64_t x, int src)
{
    return G == 1 ? x : __shfl(x, src, G);
}

template <int G>
__device__ __forceinline__ int group_min(int x)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        int y = __shfl_xor(x, o, G);
        x = y < x ? y : x;
    }
    return x;
}

template <int G>
__device__ __forceinline__ int64_t group_sum(int64_t x)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, G);
    return x;
}

template <int G>
__device__ __forceinline__ int group_or(int x)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) x |= __shfl_xor(x, o, G);
    return x;
}

// Appends `val` for every calling lane with `pred` set to list[*count ...]
// with one atomic per wave: ballot, then each lane's rank among the set
// lanes below it.  Returns the slot index of the lane's entry (or -1).
__device__ __forceinline__ int wave_append(bool pred, int32_t val, int32_t *list, int32_t *count)
{
    uint64_t mask = __ballot(pred);
    if (mask == 0) return -1;
    int leader = __ffsll((unsigned long long)mask) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(count, (int32_t)__popcll(mask));
    base = __shfl(base, leader);
    int idx = -1;
    if (pred) {
        idx = base + lanes_below(mask);
        list[idx] = val;
    }
    return idx;
}

// Adds `delta` to lcount[key] for every calling lane with pred set, one
// atomic per distinct key in the wave.  Returns, in the lane that made it,
// the count before the atomic, else INT_MIN; *mine gets the amount that
// atomic added.
__device__ __forceinline__ int wave_count_add(bool pred, int key, int delta, int32_t *lcount, int *mine)
{
    uint64_t left = __ballot(pred);
    int before = (int)0x80000000;
    *mine = 0;
    while (left) {
        const int leader = __ffsll((unsigned long long)left) - 1;
        const int k = __shfl(key, leader);
        const uint64_t same = __ballot(pred && key == k) & left;
        if (lane_id() == leader) {
            *mine = delta * __popcll(same);
            before = atomicAdd(&lcount[k], *mine);
        }
        left &= ~same;
    }
    return before;
}

// Gap rule, for a vertex whose label moves from dold to dnew at a round end:
// the histogram follows, and a label whose count reaches 0 becomes a
// candidate for the round's gap.  Every lane of the wave must call it.
__device__ __forceinline__ void gap_relabel_count(const StateView &st, bool moved, int dold, int dnew, int n)
{
    int amt;
    const int before = wave_count_add(moved, dold, -1, st.lcount, &amt);
    if (before != (int)0x80000000 && before + amt == 0 && dold > 0) {
        const int i = atomicAdd(&st.ctl->ngc, 1);
        st.gcand[i] = dold;
    }
    (void)wave_count_add(moved && dnew < n, dnew, 1, st.lcount, &amt);
}

// Position of the k-th (0-based) set bit of m; k < popcount(m).
__device__ __forceinline__ int nth_set_bit(uint64_t m, int k)
{
    int pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const uint64_t low = (m >> pos) & ((1ull << w) - 1ull);
        const int c = __popcll(low);
        if (k >= c) {
            k -= c;
            pos += w;
        }
    }
    return pos;
}

// Block-staged list append.  Entries collect in an LDS buffer of the block
// (LDS atomics only); the block writes them to the global list with one
// global atomic when the kernel ends (stage_flush).  If the buffer is full the
// entries go straight to the global list with one atomic per wave.
constexpr int STAGE_CAP = 2048;

struct Stage {
    int32_t *buf;      // LDS [STAGE_CAP]
    int32_t *cnt;      // LDS counter
    int32_t *base;     // LDS: global position of the block's entries
};

__device__ __forceinline__ void stage_init(Stage &sg)
{
    if (threadIdx.x == 0) *sg.cnt = 0;
    __syncthreads();
}

__device__ __forceinline__ void stage_append(Stage &sg, bool pred, int32_t val, int32_t *list,
                                             int32_t *count)
{
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const int c = __popcll(mask);
    const int leader = __ffsll((unsigned long long)mask) - 1;
    int pos = 0;
    if (lane_id() == leader) pos = atomicAdd(sg.cnt, c);   // the LDS counter only grows
    pos = __shfl(pos, leader);
    // positions below STAGE_CAP go to LDS, the rest straight to the global list
    const int first_over = pos > STAGE_CAP ? pos : STAGE_CAP;
    const int n_over = pos + c - first_over;
    int g0 = 0;
    if (n_over > 0) {
        if (lane_id() == leader) g0 = atomicAdd(count, n_over);
        g0 = __shfl(g0, leader);
    }
    if (pred) {
        const int idx = pos + lanes_below(mask);
        if (idx < STAGE_CAP)
            sg.buf[idx] = val;
        else
            list[g0 + idx - first_over] = val;
    }
}

// Must be reached by every thread of the block.
__device__ __forceinline__ void stage_flush(Stage &sg, int32_t *list, int32_t *count)
{
    __syncthreads();
    const int total = *sg.cnt < STAGE_CAP ? *sg.cnt : STAGE_CAP;
    if (threadIdx.x == 0) *sg.base = total ? atomicAdd(count, total) : 0;
    __syncthreads();
    const int g0 = *sg.base;
    for (int j = threadIdx.x; j < total; j += blockDim.x) list[g0 + j] = sg.buf[j];
}

// As stage_append for the candidate list of a list round, whose entries
// carry their own index in owner[] (owner[w] = the entry that merges w).
// Entries that overflow the LDS buffer get their index at once; the others
// when the block flushes (stage_flush_owner).
__device__ __forceinline__ void stage_append_owner(Stage &sg, bool pred, int32_t val, int32_t *list,
                                                   int32_t *count, int32_t *owner)
{
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const int c = __popcll(mask);
    const int leader = __ffsll((unsigned long long)mask) - 1;
    int pos = 0;
    if (lane_id() == leader) pos = atomicAdd(sg.cnt, c);
    pos = __shfl(pos, leader);
    const int first_over = pos > STAGE_CAP ? pos : STAGE_CAP;
    const int n_over = pos + c - first_over;
    int g0 = 0;
    if (n_over > 0) {
        if (lane_id() == leader) g0 = atomicAdd(count, n_over);
        g0 = __shfl(g0, leader);
    }
    if (pred) {
        const int idx = pos + lanes_below(mask);
        if (idx < STAGE_CAP) {
            sg.buf[idx] = val;
        } else {
            const int at = g0 + idx - first_over;
            list[at] = val;
            owner[val] = at;
        }
    }
}

// Must be reached by every thread of the block.
__device__ __forceinline__ void stage_flush_owner(Stage &sg, int32_t *list, int32_t *count, int32_t *owner)
{
    __syncthreads();
    const int total = *sg.cnt < STAGE_CAP ? *sg.cnt : STAGE_CAP;
    if (threadIdx.x == 0) *sg.base = total ? atomicAdd(count, total) : 0;
    __syncthreads();
    const int g0 = *sg.base;
    for (int j = threadIdx.x; j < total; j += blockDim.x) {
        const int w = sg.buf[j];
        list[g0 + j] = w;
        owner[w] = g0 + j;
    }
}

#define MF_STAGE(name)                           \
    __shared__ int32_t name##_buf[STAGE_CAP];    \
    __shared__ int32_t name##_cnt, name##_base;  \
    Stage name{name##_buf, &name##_cnt, &name##_base}

// Block-wide sum of a per-thread int32 into *dst with one atomic per block.
__device__ __forceinline__ void block_add32(int32_t x, int32_t *dst)
{
    __shared__ int32_t part32[16];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    int w = threadIdx.x >> 6;
    if (lane_id() == 0) part32[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t s = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); i++) s += part32[i];
        if (s) atomicAdd(dst, s);
    }
    __syncthreads();
}

// Block-wide sum of a per-thread int64 into *dst with one atomic per block.
__device__ __forceinline__ void block_add64(int64_t x, int64_t *dst)
{
    __shared__ int64_t part[16];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    int w = threadIdx.x >> 6;
    if (lane_id() == 0) part[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); i++) s += part[i];
        if (s) atomicAdd((unsigned long long *)dst, (unsigned long long)s);
    }
    __syncthreads();
}

}  // namespace mf
