/*
 * CPU oracle for the maximum-flow library: plain, slow, sequential C in
 * exact int64 arithmetic.
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  The HIP library neither links,
 * includes nor calls anything here, and nothing here includes the library's
 * headers.
 *
 * Problem (Sec. 2, Eq. 1-2): directed graph with capacities c >= 0, source s
 * and sink t; a flow obeys f <= c, conservation off {s, t} and antisymmetry
 * f(v,w) = -f(w,v).  Residual capacity c_f = c - f.  The value of a maximum
 * flow equals the capacity of a minimum cut.
 *
 * Graph: CSR with paired reverse slots (the adjacency arrays of Sec. 4.2 in
 * which each edge knows its reverse).  Slots of tail v are off[v]..off[v+1]-1;
 * head[a] is the head; rev[a] the paired reverse slot; cap[a] >= 0.
 */
#ifndef MF_ORACLE_H
#define MF_ORACLE_H
#include <stdint.h>

typedef struct {
    int64_t n, slots;
    const int64_t *off;
    const int32_t *head;
    const int64_t *rev;
    const int32_t *cap;
    int64_t s, t;
} og_graph;

/* Input checks.  0 = valid, otherwise one of the negative codes below. */
enum {
    OG_OK = 0, OG_ESIZE = -1, OG_ETERM = -2, OG_EOFF = -3, OG_EHEAD = -4,
    OG_ESELF = -5, OG_EREV = -6, OG_ECAP = -7, OG_EPAIR = -8, OG_ENOMEM = -9
};
int og_validate(const og_graph *g);

typedef struct {
    int64_t value;            /* max-flow value = net inflow of t            */
    int64_t cut_tstar;        /* capacity of the cut (V \ T*, T*)            */
    int64_t cut_smin;         /* capacity of the cut (S_min, V \ S_min)      */
    int64_t pushes, relabels, global_relabels, rounds;
    int64_t pushes2, relabels2, global_relabels2, rounds2;   /* phase 2 */
    int64_t work;             /* sum of (out-degree + 12) over relabels, phase 1 */
    int64_t bfs_levels;       /* sum over global relabels of BFS depth, phase 1 */
    int64_t gap_lifts, gap_lifts2;  /* oracle B with the gap rule: labels set to n by it */
} og_result;

/*
 * Oracle A: sequential FIFO push-relabel (Goldberg-Tarjan, Sec. 2.1) with
 * current arcs and global relabeling after about 12n + 2m units of relabel
 * work (the hi_pr rule quoted in Sec. 3).  Phase 2 returns the excess that
 * cannot reach t back to s by the same method with s as the sink.
 *   res_out  [slots] final residual capacities (flow = cap - res), may be NULL
 *   tstar    [n] 1 iff v reaches t in the final residual graph, may be NULL
 *   smin     [n] 1 iff s reaches v in the final residual graph, may be NULL
 *   preflow_only: skip phase 2 (smin and cut_smin are then not computed)
 */
int og_fifo_maxflow(const og_graph *g, int preflow_only, int64_t *res_out,
                    uint8_t *tstar, uint8_t *smin, og_result *r);

/*
 * Oracle B: the synchronous parallel push-relabel rounds of the paper
 * (Sec. 3.1) with parallel global relabeling (Sec. 2.1, Sec. 3),
 * simulated one vertex at a time.  Every vertex of the working set is
 * discharged against the labels and excesses of the start of the round; a
 * push into a neighbour becomes visible in the neighbour's residual capacity
 * only at the end of the round (the reading of the race the paper permits in
 * which the loser of an edge sees the capacity from before the winner's
 * push).  The result of a round is thus a function of its start state.
 *   max_rounds  > 0 stops phase 1 after that many rounds (then returns 1)
 *   sched       global-relabel rule, NULL = the paper's constants
 *   res_out     [slots] residual capacities at the end, may be NULL
 *   d_out       [n] labels at the end of phase 1 (the exact labels of the global
 *               relabel that ended it, or the labels after max_rounds), may be NULL
 *   e_out       [n] excesses at the end, may be NULL
 *   tstar       [n] as for oracle A, may be NULL
 *   preflow_only: stop after phase 1
 */
typedef struct {
    /* global relabel when freq_num * W > freq_den * (alpha * n + m); a
     * relabel of v adds outdeg(v) + beta to W (Sec. 3: freq = 1/2,
     * alpha = 6, beta = 12, i.e. about every 12n + 2m arc scans) */
    int64_t freq_num, freq_den, alpha, beta;
    /* added to W once per round (0 in the paper's rule) */
    int64_t round_charge;
    /* 1: end as the listing does, by filtering the old working set after a
     * global relabel and stopping when it is empty (can end early, with
     * excess stranded at vertices whose label passed a winner that pushed
     * into them); 0: rebuild the working set at every global relabel and
     * stop only after one that finds no active vertex */
    int64_t literal_termination;
    /* added to alpha * n + m per level of the last global relabel's
     * breadth-first search (0 in the paper's rule) */
    int64_t level_charge;
    /* 1: the simple synchronous rounds that Sec. 3 describes first (one
     * pass over the arcs, pushes on every admissible arc with no win
     * criterion, at most one relabel); 0: the full discharges of Sec. 3.1 */
    int64_t simple;
    /* 1: the gap rule at the end of every round (Sec. 3 names gap
     * relabeling, after Cherkassky and Goldberg): when no vertex other than
     * the terminals holds label k, 0 < k < n, every label in (k, n) becomes
     * n, for the smallest such k */
    int64_t gap;
} og_sched;

int og_sync_maxflow(const og_graph *g, int preflow_only, int64_t max_rounds,
                    const og_sched *sched,
                    int64_t *res_out, int64_t *d_out, int64_t *e_out,
                    uint8_t *tstar, og_result *r);

/*
 * Certificate check for a claimed maximum flow and minimum cut.
 *   flow[a]  flow on slot a (int64 so that any input can be checked)
 *   side[v]  1 = sink side T, 0 = source side S
 * Checks antisymmetry, f <= c, conservation off {s,t}, that the value out of
 * s equals the value into t, side[s] = 0, side[t] = 1, and that the cut's
 * capacity equals the value (which proves both optimal).  If reach_check is
 * set it also checks that side[] is exactly the set of vertices that reach t
 * in the residual graph of `flow`.
 * Returns 0 if all hold, else a positive code naming the first failure.
 * value_out / cut_out receive the measured value and cut capacity.
 */
enum {
    OGC_ANTISYM = 1, OGC_CAP = 2, OGC_CONSERVE = 3, OGC_VALUE = 4, OGC_SIDE = 5,
    OGC_CUT = 6, OGC_REACH = 7
};
int og_check_certificate(const og_graph *g, const int64_t *flow, const uint8_t *side,
                         int reach_check, int64_t *value_out, int64_t *cut_out);

/* Exact BFS distance to `target` over residual arcs (w -> v with res > 0),
 * never entering `blocked`; unreachable vertices get n. */
void og_residual_distance(const og_graph *g, const int64_t *res, int64_t target,
                          int64_t blocked, int64_t *dist);

#endif
