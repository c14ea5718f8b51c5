/*
 * Oracle A: sequential FIFO push-relabel in exact int64.  Test
 * infrastructure only (see oracle.h).
 *
 * Generic push-relabel of Goldberg and Tarjan as summarised in Sec. 2.1:
 * a preflow with excess e, labels d estimating the distance to the sink,
 * pushes along admissible residual arcs (d(v) = d(w) + 1) and a relabel
 * when no admissible arc remains.  Active vertices are taken in FIFO order
 * (Sec. 2.1, Sec. 3).  Global relabeling (Sec. 2.1) sets d to the exact
 * reverse-residual BFS distance, at the start and again whenever the relabel
 * work since the last one exceeds 12n + 2m (the hi_pr rule, Sec. 3 footnote;
 * a relabel of v costs outdeg(v) + 12).
 *
 * Phase 1 stops at a maximum preflow (Sec. 2.1): value = e(t).  Phase 2
 * turns the preflow into a flow by running the same method with s as the
 * sink and t excluded, which returns every remaining excess to s (Sec. 2.1
 * and 3 leave the decomposition method open).
 */
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef struct {
    const og_graph *g;
    int64_t *res, *e, *d, *cur;
    int64_t *q;          /* circular FIFO of capacity n */
    int64_t qh, qn;
    uint8_t *inq;
    int64_t pushes, relabels, grs, work_total, levels;
} fifo_state;

static void enqueue(fifo_state *S, int64_t v)
{
    int64_t n = S->g->n;
    S->q[(S->qh + S->qn) % n] = v;
    S->qn++;
    S->inq[v] = 1;
}

static int64_t dequeue(fifo_state *S)
{
    int64_t v = S->q[S->qh];
    S->qh = (S->qh + 1) % S->g->n;
    S->qn--;
    S->inq[v] = 0;
    return v;
}

static void global_relabel(fifo_state *S, int64_t target, int64_t blocked)
{
    const og_graph *g = S->g;
    og_residual_distance(g, S->res, target, blocked, S->d);
    int64_t depth = 0;
    for (int64_t v = 0; v < g->n; v++)
        if (S->d[v] < g->n && S->d[v] > depth) depth = S->d[v];
    S->levels += depth;
    for (int64_t v = 0; v < g->n; v++) S->cur[v] = g->off[v];
    S->grs++;
}

/* One push-relabel phase toward `target`; `blocked` never becomes active. */
static void fifo_phase(fifo_state *S, int64_t target, int64_t blocked)
{
    const og_graph *g = S->g;
    int64_t n = g->n;
    int64_t threshold = 12 * n + 2 * g->slots;
    int64_t work = 0;
    global_relabel(S, target, blocked);
    S->qh = 0;
    S->qn = 0;
    for (int64_t v = 0; v < n; v++) {
        S->inq[v] = 0;
        if (v != target && v != blocked && S->e[v] > 0 && S->d[v] < n) enqueue(S, v);
    }
    while (S->qn > 0) {
        if (work > threshold) {
            global_relabel(S, target, blocked);
            work = 0;
        }
        int64_t v = dequeue(S);
        if (S->d[v] >= n || S->e[v] <= 0) continue;
        /* discharge v */
        while (S->e[v] > 0) {
            if (S->cur[v] == g->off[v + 1]) {
                /* relabel: one more than the lowest residual neighbour, at most n */
                int64_t nd = n;
                for (int64_t a = g->off[v]; a < g->off[v + 1]; a++)
                    if (S->res[a] > 0 && S->d[g->head[a]] + 1 < nd) nd = S->d[g->head[a]] + 1;
                S->d[v] = nd;
                S->relabels++;
                int64_t cost = (g->off[v + 1] - g->off[v]) + 12;
                work += cost;
                S->work_total += cost;
                S->cur[v] = g->off[v];
                if (nd >= n) break;
                continue;
            }
            int64_t a = S->cur[v];
            int64_t w = g->head[a];
            if (S->res[a] > 0 && S->d[v] == S->d[w] + 1) {
                int64_t delta = S->e[v] < S->res[a] ? S->e[v] : S->res[a];
                S->res[a] -= delta;
                S->res[g->rev[a]] += delta;
                S->e[v] -= delta;
                S->e[w] += delta;
                S->pushes++;
                if (w != target && w != blocked && !S->inq[w]) enqueue(S, w);
                if (S->res[a] == 0) S->cur[v]++;
            } else {
                S->cur[v]++;
            }
        }
    }
}

int og_fifo_maxflow(const og_graph *g, int preflow_only, int64_t *res_out,
                    uint8_t *tstar, uint8_t *smin, og_result *r)
{
    int rc = og_validate(g);
    if (rc) return rc;
    int64_t n = g->n, S_ = g->slots;
    fifo_state S;
    memset(&S, 0, sizeof S);
    S.g = g;
    S.res = (int64_t *)malloc(sizeof(int64_t) * (size_t)(S_ > 0 ? S_ : 1));
    S.e = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    S.d = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    S.cur = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    S.q = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    S.inq = (uint8_t *)calloc((size_t)n, 1);
    if (!S.res || !S.e || !S.d || !S.cur || !S.q || !S.inq) return OG_ENOMEM;
    for (int64_t a = 0; a < S_; a++) S.res[a] = g->cap[a];

    /* saturate every arc out of s */
    for (int64_t a = g->off[g->s]; a < g->off[g->s + 1]; a++) {
        int64_t c = S.res[a];
        if (c <= 0) continue;
        S.res[a] -= c;
        S.res[g->rev[a]] += c;
        S.e[g->head[a]] += c;
        S.e[g->s] -= c;
    }
    fifo_phase(&S, g->t, g->s);
    memset(r, 0, sizeof *r);
    r->value = S.e[g->t];
    r->pushes = S.pushes;
    r->relabels = S.relabels;
    r->global_relabels = S.grs;
    r->work = S.work_total;
    r->bfs_levels = S.levels;

    /* T*: vertices that reach t in the residual graph of the maximum preflow */
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

    if (!preflow_only) {
        S.pushes = S.relabels = S.grs = 0;
        fifo_phase(&S, g->s, g->t);
        r->pushes2 = S.pushes;
        r->relabels2 = S.relabels;
        r->global_relabels2 = S.grs;
        /* S_min: vertices reachable from s in the residual graph of the flow */
        for (int64_t v = 0; v < n; v++) dist[v] = -1;
        int64_t qh = 0, qt = 0;
        dist[g->s] = 0;
        S.q[qt++] = g->s;
        while (qh < qt) {
            int64_t v = S.q[qh++];
            for (int64_t a = g->off[v]; a < g->off[v + 1]; a++) {
                int64_t w = g->head[a];
                if (dist[w] < 0 && S.res[a] > 0) {
                    dist[w] = dist[v] + 1;
                    S.q[qt++] = w;
                }
            }
        }
        int64_t cs = 0;
        for (int64_t v = 0; v < n; v++) {
            if (dist[v] < 0) continue;
            for (int64_t a = g->off[v]; a < g->off[v + 1]; a++)
                if (dist[g->head[a]] < 0) cs += g->cap[a];
        }
        r->cut_smin = cs;
        if (smin)
            for (int64_t v = 0; v < n; v++) smin[v] = dist[v] >= 0;
    }
    if (res_out) memcpy(res_out, S.res, sizeof(int64_t) * (size_t)S_);
    free(dist);
    free(S.res); free(S.e); free(S.d); free(S.cur); free(S.q); free(S.inq);
    return 0;
}
