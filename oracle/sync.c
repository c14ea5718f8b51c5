/*
 * Oracle B: the synchronous push-relabel method of Sec. 3.1 with the
 * parallel global relabel (a breadth-first search from the sink over the
 * reverse residual graph, Sec. 2.1 and Sec. 3), computed one vertex at a
 * time in exact int64 arithmetic.  Test infrastructure only (see oracle.h).
 *
 * State between rounds: cf[a] (residual capacity of slot a), lab[v] (label)
 * and exc[v] (excess).  A round is a pure function of that state:
 *
 *   discharge   every vertex of the working set, on its own, runs the full
 *               discharge of Sec. 3.1: it walks its residual arcs in slot
 *               order, pushing along each eligible arc (its raised label d'
 *               is one more than the neighbour's label at the round start),
 *               and raises d' when a walk ends with excess left, until the
 *               excess is gone, d' reaches n, or it has to give way on an
 *               eligible arc to an active neighbour that owns the edge (the
 *               ownership rule of Sec. 3.1, decided on round-start labels).
 *               Everything it reads about other vertices is round-start
 *               state; its own residuals fall as it pushes.
 *   round end   the pushes become visible to the heads: each push of x units
 *               on slot a raises cf[rev a] by x and moves x units of excess
 *               from tail to head; the raised labels replace the old ones.
 *
 * Deferring the reverse residuals to the round end is the reading of the race
 * Sec. 3.1 allows (a vertex that gives way may see the residual capacity from
 * before or after its neighbour's push; here always before).
 *
 * The working set of a round is the set of active vertices: neither
 * terminal, positive excess, label below n.  After a global relabel it is
 * rebuilt from all vertices (exact labels revive a vertex that an invalid
 * label had parked at n), and the phase ends only when a global relabel run
 * at that point finds no active vertex.  With sched->literal_termination the
 * set is instead the previous one with its label-n vertices removed, and the
 * phase ends as soon as that is empty (which can end early).
 *
 * A global relabel runs first and then whenever the relabel work since the
 * last one crosses the rule of Sec. 3 (see og_sched).
 *
 * With sched->simple the rounds are those of the simple synchronous
 * algorithm Sec. 3 starts from: one walk over the arcs with no ownership
 * rule, then at most one raise of the label.
 *
 * With sched->gap the gap rule (Sec. 3 mentions gap relabeling and cites
 * Cherkassky and Goldberg for it) runs at the end of every round: if no
 * vertex other than the two terminals holds some label k with 0 < k < n,
 * while some hold labels above k, none of those can reach the sink, and
 * every label in (k, n) becomes n (k the smallest such gap).
 *
 * Phase 2 (flow reconstruction; the paper leaves the method open) runs the
 * same rounds with s as the sink and t excluded, which returns every excess
 * that cannot reach t to s.
 */
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef struct {
    const og_graph *g;
    int64_t n, m;
    int64_t *cf, *lab, *exc;      /* state between rounds                         */
    /* round scratch */
    int64_t *raised;              /* d' of each discharged vertex                 */
    int64_t *change;              /* net excess change of each touched vertex     */
    int64_t *back;                /* residual returned to each slot at round end  */
    uint8_t *touched;             /* vertex pushed to or discharged this round    */
    int64_t *tlist, nt;           /* the touched vertices                         */
    int64_t *blist, nb;           /* slots with a nonzero back[]                  */
    /* working set */
    int64_t *ws, nws;
    uint8_t *in_ws;
    /* breadth-first search */
    int64_t *fifo;
    /* gap rule: number of non-terminal vertices per label below n */
    int64_t *count;
    /* tallies */
    int64_t pushes, relabels, grs, rounds, work, levels, gap_lifts;
} machine;

/* Exact distances to `sink` over residual arcs w -> v (cf of the reverse
 * slot of v's slot toward w), never through `other`; n where there is no
 * path.  Returns the largest distance given. */
static int64_t bfs_labels(machine *M, int64_t sink, int64_t other)
{
    const og_graph *g = M->g;
    const int64_t n = M->n;
    for (int64_t v = 0; v < n; v++) M->lab[v] = n;
    M->lab[sink] = 0;
    int64_t head = 0, tail = 0, depth = 0;
    M->fifo[tail++] = sink;
    while (head < tail) {
        const int64_t v = M->fifo[head++];
        for (int64_t a = g->off[v]; a < g->off[v + 1]; a++) {
            const int64_t w = g->head[a];
            if (w == other || M->lab[w] != n) continue;
            if (M->cf[g->rev[a]] > 0) {          /* w can send to v */
                M->lab[w] = M->lab[v] + 1;
                if (M->lab[w] > depth) depth = M->lab[w];
                M->fifo[tail++] = w;
            }
        }
    }
    M->levels += depth;
    M->grs++;
    return depth;
}

/* Whether v, active, owns the edge to the active neighbour w (Sec. 3.1):
 * v one level above w, or more than one level below it, or level with it and
 * of smaller id.  Exactly one of v and w owns it. */
static int owns_edge(int64_t dv, int64_t dw, int64_t v, int64_t w)
{
    return dv == dw + 1 || dv < dw - 1 || (dv == dw && v < w);
}

static void touch(machine *M, int64_t v)
{
    if (!M->touched[v]) {
        M->touched[v] = 1;
        M->tlist[M->nt++] = v;
    }
}

static int active(const machine *M, int64_t v, int64_t sink, int64_t other)
{
    return v != sink && v != other && M->exc[v] > 0 && M->lab[v] < M->n;
}

/* Full discharge of v against the round-start state (see the file header).
 * Round work: every raise of d' costs outdeg(v) + beta. */
static void discharge(machine *M, int64_t v, int simple, int64_t beta)
{
    const og_graph *g = M->g;
    const int64_t n = M->n, first = g->off[v], last = g->off[v + 1];
    const int64_t d0 = M->lab[v];
    int64_t dcur = d0;                /* d'(v) */
    int64_t left = M->exc[v];
    while (left > 0) {
        int64_t lowest = n;           /* smallest d(w)+1 over residual arcs with d(w) >= d' */
        int gave_way = 0;
        for (int64_t a = first; a < last && left > 0; a++) {
            if (M->cf[a] <= 0) continue;
            const int64_t w = g->head[a];
            const int64_t dw = M->lab[w];
            if (dcur == dw + 1) {
                if (!simple && M->exc[w] != 0 && !owns_edge(d0, dw, v, w)) {
                    gave_way = 1;     /* w is active and owns the edge */
                } else {
                    const int64_t x = M->cf[a] < left ? M->cf[a] : left;
                    M->cf[a] -= x;
                    const int64_t b = g->rev[a];
                    if (M->back[b] == 0) M->blist[M->nb++] = b;
                    M->back[b] += x;
                    M->change[w] += x;
                    left -= x;
                    touch(M, w);
                    M->pushes++;
                }
            }
            if (M->cf[a] > 0 && dw >= dcur && dw + 1 < lowest) lowest = dw + 1;
        }
        if (left == 0 || gave_way) break;
        dcur = lowest;                /* <= n */
        M->relabels++;
        M->work += (last - first) + beta;
        if (dcur == n || simple) break;
    }
    M->raised[v] = dcur;
    M->change[v] += left - M->exc[v];
    touch(M, v);
}

/* Labels below n held by non-terminal vertices, for the gap rule. */
static void count_labels(machine *M, int64_t sink, int64_t other)
{
    memset(M->count, 0, sizeof(int64_t) * (size_t)M->n);
    for (int64_t v = 0; v < M->n; v++)
        if (v != sink && v != other && M->lab[v] < M->n) M->count[M->lab[v]]++;
}

/* Gap rule (file header).  The labels that lost a vertex this round are the
 * only places a gap can open, since the rule leaves none behind; `lost`
 * lists them (the old labels of the vertices that were raised). */
static void apply_gap(machine *M, int64_t sink, int64_t other, const int64_t *lost, int64_t nlost)
{
    const int64_t n = M->n;
    int64_t gap = n;
    for (int64_t i = 0; i < nlost; i++)
        if (lost[i] > 0 && lost[i] < gap && M->count[lost[i]] == 0) gap = lost[i];
    if (gap == n) return;
    for (int64_t v = 0; v < n; v++) {
        if (v == sink || v == other) continue;
        if (M->lab[v] > gap && M->lab[v] < n) {
            M->count[M->lab[v]]--;
            M->lab[v] = n;
            M->gap_lifts++;
        }
    }
}

/* One phase toward `sink`.  Returns 1 if max_rounds stopped it. */
static int run_phase(machine *M, int64_t sink, int64_t other, int64_t max_rounds, const og_sched *sc)
{
    const og_graph *g = M->g;
    const int64_t n = M->n;
    int must_relabel = 1;            /* the first step is a global relabel */
    int64_t since = 0;               /* relabel work (and round charges) since the last one */
    int64_t depth = 0;               /* depth of the last global relabel */
    int64_t done = 0;                /* rounds of this phase */
    int64_t *lost = M->fifo;         /* gap rule: old labels of raised vertices (the search is idle) */
    while (1) {
        int fresh = 0;
        if (must_relabel ||
            sc->freq_num * since > sc->freq_den * (sc->alpha * n + M->m + sc->level_charge * depth)) {
            depth = bfs_labels(M, sink, other);
            since = 0;
            must_relabel = 0;
            fresh = 1;
            int64_t k = 0;
            if (sc->literal_termination) {
                for (int64_t i = 0; i < M->nws; i++)
                    if (M->lab[M->ws[i]] < n) M->ws[k++] = M->ws[i];
                    else M->in_ws[M->ws[i]] = 0;
            } else {
                for (int64_t i = 0; i < M->nws; i++) M->in_ws[M->ws[i]] = 0;
                for (int64_t v = 0; v < n; v++)
                    if (active(M, v, sink, other)) {
                        M->ws[k++] = v;
                        M->in_ws[v] = 1;
                    }
            }
            M->nws = k;
            if (sc->gap) count_labels(M, sink, other);
        }
        if (M->nws == 0) {
            if (fresh || sc->literal_termination) return 0;
            must_relabel = 1;        /* end only after a fresh relabel finds nothing */
            continue;
        }
        if (max_rounds > 0 && done >= max_rounds) return 1;
        done++;
        M->rounds++;

        /* discharge: every vertex of the working set against the round start */
        const int64_t work_before = M->work;
        M->nt = 0;
        M->nb = 0;
        for (int64_t i = 0; i < M->nws; i++) discharge(M, M->ws[i], (int)sc->simple, sc->beta);
        since += M->work - work_before + sc->round_charge;

        /* round end: labels, residuals returned to the heads, excesses */
        int64_t nlost = 0;
        for (int64_t i = 0; i < M->nws; i++) {
            const int64_t v = M->ws[i];
            if (M->raised[v] != M->lab[v]) {
                if (sc->gap) {
                    M->count[M->lab[v]]--;
                    if (M->raised[v] < n) M->count[M->raised[v]]++;
                    lost[nlost++] = M->lab[v];
                }
                M->lab[v] = M->raised[v];
            }
        }
        for (int64_t i = 0; i < M->nb; i++) {
            M->cf[M->blist[i]] += M->back[M->blist[i]];
            M->back[M->blist[i]] = 0;
        }
        for (int64_t i = 0; i < M->nt; i++) {
            const int64_t v = M->tlist[i];
            M->exc[v] += M->change[v];
            M->change[v] = 0;
        }
        if (sc->gap && nlost) apply_gap(M, sink, other, lost, nlost);

        /* next working set: the touched vertices that are active */
        for (int64_t i = 0; i < M->nws; i++) M->in_ws[M->ws[i]] = 0;
        int64_t k = 0;
        for (int64_t i = 0; i < M->nt; i++) {
            const int64_t v = M->tlist[i];
            M->touched[v] = 0;
            if (active(M, v, sink, other)) {
                M->ws[k++] = v;
                M->in_ws[v] = 1;
            }
        }
        M->nws = k;
    }
    (void)g;
}

int og_sync_maxflow(const og_graph *g, int preflow_only, int64_t max_rounds,
                    const og_sched *sched,
                    int64_t *res_out, int64_t *d_out, int64_t *e_out,
                    uint8_t *tstar, og_result *r)
{
    int rc = og_validate(g);
    if (rc) return rc;
    og_sched sc = {1, 2, 6, 12, 0, 0, 0, 0, 0};
    if (sched) sc = *sched;
    if (sc.freq_den <= 0 || sc.freq_num < 0 || sc.alpha < 0 || sc.beta < 0 || sc.round_charge < 0 ||
        sc.level_charge < 0)
        return OG_ESIZE;
    const int64_t n = g->n, S = g->slots > 0 ? g->slots : 1;
    machine M;
    memset(&M, 0, sizeof M);
    M.g = g;
    M.n = n;
    M.m = g->slots;
    M.cf = (int64_t *)malloc(sizeof(int64_t) * (size_t)S);
    M.back = (int64_t *)calloc((size_t)S, sizeof(int64_t));
    M.blist = (int64_t *)malloc(sizeof(int64_t) * (size_t)S);
    M.lab = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    M.exc = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    M.raised = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    M.change = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    M.touched = (uint8_t *)calloc((size_t)n, 1);
    M.in_ws = (uint8_t *)calloc((size_t)n, 1);
    M.tlist = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    M.ws = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    M.fifo = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    M.count = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!M.cf || !M.back || !M.blist || !M.lab || !M.exc || !M.raised || !M.change || !M.touched ||
        !M.in_ws || !M.tlist || !M.ws || !M.fifo || !M.count)
        return OG_ENOMEM;

    /* start: zero flow, labels 0 with d(s) = n, every arc out of s saturated */
    for (int64_t a = 0; a < g->slots; a++) M.cf[a] = g->cap[a];
    M.lab[g->s] = n;
    for (int64_t a = g->off[g->s]; a < g->off[g->s + 1]; a++) {
        const int64_t c = M.cf[a];
        if (c <= 0) continue;
        M.cf[a] = 0;
        M.cf[g->rev[a]] += c;
        M.exc[g->head[a]] += c;
        M.exc[g->s] -= c;
    }
    /* the first working set: every vertex the saturation gave excess */
    for (int64_t v = 0; v < n; v++)
        if (v != g->s && v != g->t && M.exc[v] > 0) {
            M.ws[M.nws++] = v;
            M.in_ws[v] = 1;
        }

    const int stopped = run_phase(&M, g->t, g->s, max_rounds, &sc);
    memset(r, 0, sizeof *r);
    r->value = M.exc[g->t];
    r->pushes = M.pushes;
    r->relabels = M.relabels;
    r->global_relabels = M.grs;
    r->rounds = M.rounds;
    r->work = M.work;
    r->bfs_levels = M.levels;
    r->gap_lifts = M.gap_lifts;
    if (d_out) memcpy(d_out, M.lab, sizeof(int64_t) * (size_t)n);

    /* T* and the capacity of its cut, from the residuals of the preflow */
    int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!dist) return OG_ENOMEM;
    og_residual_distance(g, M.cf, g->t, g->s, dist);
    int64_t cut = 0;
    for (int64_t v = 0; v < n; v++) {
        if (dist[v] < n) continue;
        for (int64_t a = g->off[v]; a < g->off[v + 1]; a++)
            if (dist[g->head[a]] < n) cut += g->cap[a];
    }
    r->cut_tstar = cut;
    if (tstar)
        for (int64_t v = 0; v < n; v++) tstar[v] = dist[v] < n;
    free(dist);

    if (!preflow_only && !stopped) {
        /* phase 2 from every vertex that still holds excess */
        for (int64_t i = 0; i < M.nws; i++) M.in_ws[M.ws[i]] = 0;
        M.nws = 0;
        for (int64_t v = 0; v < n; v++)
            if (v != g->s && v != g->t && M.exc[v] > 0) {
                M.ws[M.nws++] = v;
                M.in_ws[v] = 1;
            }
        const int64_t p1 = M.pushes, r1 = M.relabels, g1 = M.grs, k1 = M.rounds, w1 = M.work,
                      l1 = M.levels, x1 = M.gap_lifts;
        run_phase(&M, g->s, g->t, 0, &sc);
        r->pushes2 = M.pushes - p1;
        r->relabels2 = M.relabels - r1;
        r->global_relabels2 = M.grs - g1;
        r->rounds2 = M.rounds - k1;
        r->gap_lifts2 = M.gap_lifts - x1;
        (void)w1;
        (void)l1;
    }
    if (res_out) memcpy(res_out, M.cf, sizeof(int64_t) * (size_t)g->slots);
    if (e_out) memcpy(e_out, M.exc, sizeof(int64_t) * (size_t)n);
    free(M.cf); free(M.back); free(M.blist); free(M.lab); free(M.exc); free(M.raised);
    free(M.change); free(M.touched); free(M.in_ws); free(M.tlist); free(M.ws); free(M.fifo);
    free(M.count);
    return stopped;
}
