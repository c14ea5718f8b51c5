/*
 * Oracle B: the paper's synchronous push-relabel (prsn, Sec. 3.1, Listing 1)
 * with its parallel global relabeling (Listing 2), executed one vertex at a
 * time in exact int64.  Test infrastructure only (see oracle.h).
 *
 * Readings of points the pseudocode leaves open:
 *  - initial working set: the distinct heads of saturated source arcs other
 *    than s and t; the first iteration always runs a global relabel, which
 *    filters it;
 *  - parallel arcs out of s add their capacities to e(v);
 *  - "residual edge (v,w)" in the discharge means c_f(v,w) > 0 as v sees it;
 *    a neighbour's push into v becomes visible in v's residual capacities at
 *    the end of the round (the loser of an edge reads the capacity from
 *    before the winner's push, which the paper allows);
 *  - "if e(w)" tests the excess of w at the start of the round;
 *  - v.addedExcess accumulates (the listing's assignment would drop the
 *    neighbours' fetch-and-add contributions);
 *  - the test "e'(v)" means that v still holds excess after its discharge;
 *  - the filter of the new working set keeps the discovered vertices w with
 *    updated label d(w) < n, and the added excess of every vertex that
 *    received a push (t and filtered vertices included) is applied;
 *  - a global relabel rebuilds the working set from every vertex with
 *    positive excess and exact label below n, and the loop ends only when a
 *    global relabel run at that point finds none (see prsn_phase);
 *  - the global relabel follows residual arcs w -> v, i.e. tests
 *    c_f(w,v) > 0, which is what a BFS in the reverse residual graph needs.
 *
 * With og_sched.simple the rounds are those of the simple synchronous
 * algorithm Sec. 3 describes before its improvements: each active vertex
 * checks its arcs once, pushing on every admissible arc (no win criterion),
 * and if it still holds excess takes one new label, computed from the
 * round-start labels of the heads of its residual arcs with d(w) >= d(v)
 * (the candidates Listing 1 uses, so that a label never decreases).  Labels
 * and excess changes apply at the round's end, as in the other rounds.
 */
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef struct {
    const og_graph *g;
    int64_t n, m;
    int64_t *res;          /* residual capacity per slot as of the last round end    */
    int64_t *pending;      /* pushes into the reverse slot, applied at round end     */
    int64_t *d, *dprime, *e, *addedExcess, *work;
    uint8_t *isDiscovered;
    int64_t *workingSet, *next, nws;
    int64_t *touchedSlots, ntouchedSlots;
    int64_t *touchedVerts, ntouchedVerts;
    uint8_t *vertTouched;
    int64_t *Q, *Q2;
    int64_t pushes, relabels, grs, rounds, work_total, levels;
} sync_state;

/* Listing 2: level-synchronous BFS from the sink over the reverse residual
 * graph.  Returns its depth (the largest label it gives). */
static int64_t GlobalRelabel(sync_state *S, int64_t sink, int64_t other)
{
    const og_graph *g = S->g;
    int64_t n = S->n;
    for (int64_t v = 0; v < n; v++) S->d[v] = n;
    S->d[sink] = 0;
    int64_t nq = 0;
    S->Q[nq++] = sink;
    int64_t level = 0;
    while (nq > 0) {
        int64_t nq2 = 0;
        for (int64_t i = 0; i < nq; i++) {
            int64_t v = S->Q[i];
            for (int64_t a = g->off[v]; a < g->off[v + 1]; a++) {
                int64_t w = g->head[a];
                if (w == other) continue;
                if (S->res[g->rev[a]] <= 0) continue;        /* c_f(w,v) > 0 */
                if (w != sink && S->d[w] == n) {
                    S->d[w] = S->d[v] + 1;
                    S->Q2[nq2++] = w;
                }
            }
        }
        int64_t *tmp = S->Q; S->Q = S->Q2; S->Q2 = tmp;
        nq = nq2;
        if (nq) level++;
    }
    S->levels += level;
    S->grs++;
    for (int64_t v = 0; v < n; v++) S->dprime[v] = S->d[v];
    return level;
}

static void touch_vertex(sync_state *S, int64_t v)
{
    if (!S->vertTouched[v]) {
        S->vertTouched[v] = 1;
        S->touchedVerts[S->ntouchedVerts++] = v;
    }
}

/* Listing 1's main loop for one phase.  Returns 1 if max_rounds stopped it. */
static int prsn_phase(sync_state *S, int64_t sink, int64_t other, int64_t max_rounds,
                      const og_sched *sc)
{
    const og_graph *g = S->g;
    int64_t n = S->n;
    const int64_t beta = sc->beta;
    int grPending = 1;                     /* workSinceLastGR := infinity */
    int64_t workSinceLastGR = 0;
    int64_t lastDepth = 0;                 /* depth of the last global relabel */
    int64_t rounds_here = 0;
    while (1) {
        int justRelabeled = 0;
        /* freq * workSinceLastGR > alpha * n + m (+ level_charge * depth of
         * the last global relabel, 0 in the paper's rule) */
        if (grPending || sc->freq_num * workSinceLastGR >
                             sc->freq_den * (sc->alpha * n + S->m + sc->level_charge * lastDepth)) {
            grPending = 0;
            workSinceLastGR = 0;
            lastDepth = GlobalRelabel(S, sink, other);
            if (sc->literal_termination) {
                int64_t k = 0;
                for (int64_t i = 0; i < S->nws; i++)
                    if (S->d[S->workingSet[i]] < n) S->workingSet[k++] = S->workingSet[i];
                S->nws = k;
            } else {
                /* Every vertex with excess and an exact label below n is
                 * active again.  A loser that relabels past a winner pushing
                 * into it can leave an invalid label behind (Sec. 3.1 allows
                 * that case); the exact labels of the global relabel undo it,
                 * and a vertex that the invalid label had pushed to n is taken
                 * back in here. */
                S->nws = 0;
                for (int64_t v = 0; v < n; v++)
                    if (v != sink && v != other && S->e[v] > 0 && S->d[v] < n)
                        S->workingSet[S->nws++] = v;
            }
            justRelabeled = 1;
        }
        if (S->nws == 0) {
            /* stop only when a fresh global relabel finds no active vertex */
            if (justRelabeled || sc->literal_termination) return 0;
            grPending = 1;
            continue;
        }
        if (max_rounds > 0 && rounds_here >= max_rounds) return 1;
        rounds_here++;
        S->rounds++;

        int64_t nnext = 0;
        S->ntouchedSlots = 0;
        S->ntouchedVerts = 0;
        for (int64_t i = 0; i < S->nws; i++) {
            int64_t v = S->workingSet[i];
            S->dprime[v] = S->d[v];
            int64_t e = S->e[v];                 /* local copy */
            S->work[v] = 0;
            int64_t outDegree = g->off[v + 1] - g->off[v];
            while (e > 0) {
                int64_t newLabel = n;
                int skipped = 0;
                for (int64_t a = g->off[v]; a < g->off[v + 1]; a++) {
                    if (S->res[a] <= 0) continue;    /* residual edges only */
                    if (e == 0) break;               /* discharged completely */
                    int64_t w = g->head[a];
                    int admissible = (S->dprime[v] == S->d[w] + 1);
                    if (S->e[w] != 0 && !sc->simple) {   /* edge shared by two active vertices */
                        int win = (S->d[v] == S->d[w] + 1) || (S->d[v] < S->d[w] - 1) ||
                                  (S->d[v] == S->d[w] && v < w);
                        if (admissible && !win) { skipped = 1; continue; }
                    }
                    if (admissible && S->res[a] > 0) {
                        int64_t delta = S->res[a] < e ? S->res[a] : e;
                        S->res[a] -= delta;                  /* f(v,w) += delta */
                        int64_t b = g->rev[a];
                        if (S->pending[b] == 0) S->touchedSlots[S->ntouchedSlots++] = b;
                        S->pending[b] += delta;              /* f(w,v) -= delta, seen at round end */
                        e -= delta;
                        S->addedExcess[w] += delta;
                        touch_vertex(S, w);
                        S->pushes++;
                        if (w != sink && !S->isDiscovered[w]) {
                            S->isDiscovered[w] = 1;
                            S->next[nnext++] = w;
                        }
                    }
                    if (S->res[a] > 0 && S->d[w] >= S->dprime[v]) {
                        if (S->d[w] + 1 < newLabel) newLabel = S->d[w] + 1;
                    }
                }
                if (e == 0 || skipped) break;
                S->dprime[v] = newLabel;             /* relabel */
                S->work[v] += outDegree + beta;
                S->relabels++;
                if (S->dprime[v] == n) break;
                if (sc->simple) break;               /* simple rounds: one pass, one relabel */
            }
            S->addedExcess[v] += e - S->e[v];
            touch_vertex(S, v);
            if (e > 0 && !S->isDiscovered[v]) {
                S->isDiscovered[v] = 1;
                S->next[nnext++] = v;
            }
        }

        workSinceLastGR += sc->round_charge;
        /* apply the new labels of the old working set and sum the work */
        for (int64_t i = 0; i < S->nws; i++) {
            int64_t v = S->workingSet[i];
            S->d[v] = S->dprime[v];
            workSinceLastGR += S->work[v];
            S->work_total += S->work[v];
        }
        /* apply the excess changes and the deferred reverse residuals */
        for (int64_t i = 0; i < S->ntouchedVerts; i++) {
            int64_t v = S->touchedVerts[i];
            S->e[v] += S->addedExcess[v];
            S->addedExcess[v] = 0;
            S->vertTouched[v] = 0;
        }
        for (int64_t i = 0; i < S->ntouchedSlots; i++) {
            int64_t b = S->touchedSlots[i];
            S->res[b] += S->pending[b];
            S->pending[b] = 0;
        }
        /* new working set: discovered vertices whose label is below n */
        int64_t k = 0;
        for (int64_t i = 0; i < nnext; i++) {
            int64_t w = S->next[i];
            S->isDiscovered[w] = 0;
            if (S->d[w] < n) S->workingSet[k++] = w;
        }
        S->nws = k;
    }
}

int og_sync_maxflow(const og_graph *g, int preflow_only, int64_t max_rounds,
                    const og_sched *sched,
                    int64_t *res_out, int64_t *d_out, int64_t *e_out,
                    uint8_t *tstar, og_result *r)
{
    int rc = og_validate(g);
    if (rc) return rc;
    og_sched sc = {1, 2, 6, 12, 0, 0, 0, 0};
    if (sched) sc = *sched;
    if (sc.freq_den <= 0 || sc.freq_num < 0 || sc.alpha < 0 || sc.beta < 0 || sc.round_charge < 0 ||
        sc.level_charge < 0)
        return OG_ESIZE;
    int64_t n = g->n, M = g->slots > 0 ? g->slots : 1;
    sync_state S;
    memset(&S, 0, sizeof S);
    S.g = g;
    S.n = n;
    S.m = g->slots;
    S.res = (int64_t *)malloc(sizeof(int64_t) * (size_t)M);
    S.pending = (int64_t *)calloc((size_t)M, sizeof(int64_t));
    S.touchedSlots = (int64_t *)malloc(sizeof(int64_t) * (size_t)M);
    S.d = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    S.dprime = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    S.e = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    S.addedExcess = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    S.work = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    S.isDiscovered = (uint8_t *)calloc((size_t)n, 1);
    S.vertTouched = (uint8_t *)calloc((size_t)n, 1);
    S.workingSet = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    S.next = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    S.touchedVerts = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    S.Q = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    S.Q2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!S.res || !S.pending || !S.touchedSlots || !S.d || !S.dprime || !S.e || !S.addedExcess ||
        !S.work || !S.isDiscovered || !S.vertTouched || !S.workingSet || !S.next ||
        !S.touchedVerts || !S.Q || !S.Q2)
        return OG_ENOMEM;

    /* Listing 1 initialisation: d = 0, e = 0, f = 0, d(s) = n */
    for (int64_t a = 0; a < g->slots; a++) S.res[a] = g->cap[a];
    S.d[g->s] = n;
    S.dprime[g->s] = n;
    /* saturate every arc out of s */
    for (int64_t a = g->off[g->s]; a < g->off[g->s + 1]; a++) {
        int64_t c = g->cap[a];
        if (c <= 0) continue;
        int64_t w = g->head[a];
        S.res[a] -= c;
        S.res[g->rev[a]] += c;
        S.e[w] += c;
        S.e[g->s] -= c;
        if (w != g->s && w != g->t && !S.isDiscovered[w]) {
            S.isDiscovered[w] = 1;
            S.workingSet[S.nws++] = w;
        }
    }
    for (int64_t i = 0; i < S.nws; i++) S.isDiscovered[S.workingSet[i]] = 0;

    int stopped = prsn_phase(&S, g->t, g->s, max_rounds, &sc);
    memset(r, 0, sizeof *r);
    r->value = S.e[g->t];
    r->pushes = S.pushes;
    r->relabels = S.relabels;
    r->global_relabels = S.grs;
    r->rounds = S.rounds;
    r->work = S.work_total;
    r->bfs_levels = S.levels;
    if (d_out) memcpy(d_out, S.d, sizeof(int64_t) * (size_t)n);

    int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    og_residual_distance(g, S.res, g->t, g->s, dist);
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
        /* phase 2: the same rounds with s as the sink and t excluded, starting
         * from every vertex that still holds excess */
        S.nws = 0;
        for (int64_t v = 0; v < n; v++)
            if (v != g->s && v != g->t && S.e[v] > 0) S.workingSet[S.nws++] = v;
        S.pushes = S.relabels = S.grs = S.rounds = 0;
        int64_t wt = S.work_total, lv = S.levels;
        prsn_phase(&S, g->s, g->t, 0, &sc);
        r->pushes2 = S.pushes;
        r->relabels2 = S.relabels;
        r->global_relabels2 = S.grs;
        r->rounds2 = S.rounds;
        S.work_total = wt;
        S.levels = lv;
    }
    if (res_out) memcpy(res_out, S.res, sizeof(int64_t) * (size_t)g->slots);
    if (e_out) memcpy(e_out, S.e, sizeof(int64_t) * (size_t)n);
    free(S.res); free(S.pending); free(S.touchedSlots); free(S.d); free(S.dprime); free(S.e);
    free(S.addedExcess); free(S.work); free(S.isDiscovered); free(S.vertTouched);
    free(S.workingSet); free(S.next); free(S.touchedVerts); free(S.Q); free(S.Q2);
    return stopped;
}
