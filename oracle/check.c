/*
 * Oracle support: input validation, residual distances and the max-flow /
 * min-cut certificate.  Test infrastructure only (see oracle.h).
 */
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

/* The graph model of Sec. 2: s != t, c >= 0, no self-loops (Eq. 1 sums
 * exclude v = w), and every slot paired with a reverse slot (Sec. 4.2). */
int og_validate(const og_graph *g)
{
    if (g->n < 2 || g->slots < 0) return OG_ESIZE;
    if (g->s < 0 || g->s >= g->n || g->t < 0 || g->t >= g->n || g->s == g->t) return OG_ETERM;
    if (g->off[0] != 0 || g->off[g->n] != g->slots) return OG_EOFF;
    for (int64_t v = 0; v < g->n; v++)
        if (g->off[v + 1] < g->off[v]) return OG_EOFF;
    for (int64_t v = 0; v < g->n; v++) {
        for (int64_t a = g->off[v]; a < g->off[v + 1]; a++) {
            int64_t w = g->head[a];
            if (w < 0 || w >= g->n) return OG_EHEAD;
            if (w == v) return OG_ESELF;
            int64_t b = g->rev[a];
            if (b < 0 || b >= g->slots) return OG_EREV;
            if (g->rev[b] != a || g->head[b] != v) return OG_EREV;
            if (g->cap[a] < 0) return OG_ECAP;
            if ((int64_t)g->cap[a] + (int64_t)g->cap[b] > 2147483647LL) return OG_EPAIR;
        }
    }
    return OG_OK;
}

/* Breadth-first search from `target` in the reverse residual graph: w gets
 * distance d(v)+1 when the arc w -> v has positive residual capacity. */
void og_residual_distance(const og_graph *g, const int64_t *res, int64_t target,
                          int64_t blocked, int64_t *dist)
{
    int64_t n = g->n;
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t v = 0; v < n; v++) dist[v] = n;
    dist[target] = 0;
    int64_t qh = 0, qt = 0;
    q[qt++] = target;
    while (qh < qt) {
        int64_t v = q[qh++];
        for (int64_t a = g->off[v]; a < g->off[v + 1]; a++) {
            int64_t w = g->head[a];
            if (w == blocked || dist[w] != n) continue;
            if (res[g->rev[a]] > 0) {          /* residual arc w -> v */
                dist[w] = dist[v] + 1;
                q[qt++] = w;
            }
        }
    }
    free(q);
}

int og_check_certificate(const og_graph *g, const int64_t *flow, const uint8_t *side,
                         int reach_check, int64_t *value_out, int64_t *cut_out)
{
    int64_t n = g->n;
    int rc = 0;
    for (int64_t a = 0; a < g->slots; a++) {
        if (flow[a] != -flow[g->rev[a]]) return OGC_ANTISYM;     /* Eq. 2 */
        if (flow[a] > g->cap[a]) return OGC_CAP;                 /* f <= c */
    }
    int64_t out_s = 0, in_t = 0;
    for (int64_t v = 0; v < n; v++) {
        int64_t net_out = 0;
        for (int64_t a = g->off[v]; a < g->off[v + 1]; a++) net_out += flow[a];
        if (v == g->s) out_s = net_out;
        else if (v == g->t) in_t = -net_out;
        else if (net_out != 0) return OGC_CONSERVE;              /* Eq. 1 */
    }
    if (value_out) *value_out = out_s;
    if (out_s != in_t) return OGC_VALUE;
    if (side[g->s] != 0 || side[g->t] != 1) return OGC_SIDE;
    int64_t cut = 0;
    for (int64_t v = 0; v < n; v++) {
        if (side[v]) continue;
        for (int64_t a = g->off[v]; a < g->off[v + 1]; a++)
            if (side[g->head[a]]) cut += g->cap[a];
    }
    if (cut_out) *cut_out = cut;
    if (cut != out_s) rc = OGC_CUT;
    if (rc == 0 && reach_check) {
        int64_t *res = (int64_t *)malloc(sizeof(int64_t) * (size_t)g->slots);
        int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        for (int64_t a = 0; a < g->slots; a++) res[a] = (int64_t)g->cap[a] - flow[a];
        og_residual_distance(g, res, g->t, -1, dist);
        for (int64_t v = 0; v < n; v++)
            if ((dist[v] < n) != (side[v] != 0)) { rc = OGC_REACH; break; }
        free(res);
        free(dist);
    }
    return rc;
}
