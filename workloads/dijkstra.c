/*
 * Batched single-source shortest paths for route generation.
 *
 * Routes are an *input* of the per-timestep vehicle update: the paper computes
 * them once, before the simulation, with a priority-queue Dijkstra run only for
 * the origin/destination pairs that are needed (Sec. II-C).  This file is part
 * of the seeded input generators; it holds none of the simulation arithmetic.
 *
 * Deterministic tie-break, independent of thread count:
 *   - the heap is ordered by (cost, node id);
 *   - a label is relaxed only on strict improvement;
 *   - out-edges of a node are relaxed in ascending edge id.
 * Each origin is solved independently, so threads never share a label array.
 *
 * Interface (two calls, so the caller can size the output):
 *   dij_solve(...)  -> opaque result holding one malloc'd path per OD row
 *   dij_lengths()   -> number of edges per OD row (-1: unreachable or O == D)
 *   dij_copy()      -> concatenate the paths into a caller buffer
 *   dij_free()
 *
 * dij_solve_to() runs the same search from each *destination* over the
 * reversed graph (the caller passes edge_to/edge_from swapped and in-edge
 * lists): the label tree then points every node along its shortest path to
 * the destination, and the path of an origin is read off in travel order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef struct {
    double cost;
    int32_t node;
} hitem;

static int hless(const hitem *a, const hitem *b) {
    if (a->cost != b->cost) return a->cost < b->cost;
    return a->node < b->node;
}

typedef struct {
    hitem *h;
    int64_t n, cap;
} heap_t;

/* 4-ary min-heap on (cost, node).  Every (cost, node) pair is pushed at most
 * once (labels only improve strictly), so the pop order is fixed by the
 * ordering alone and does not depend on the heap's shape. */
static int heap_push(heap_t *hp, double c, int32_t node) {
    if (hp->n == hp->cap) {
        int64_t nc = hp->cap ? 2 * hp->cap : 1024;
        hitem *nh = (hitem *)realloc(hp->h, (size_t)nc * sizeof(hitem));
        if (!nh) return -1;
        hp->h = nh;
        hp->cap = nc;
    }
    hitem x = {c, node};
    int64_t i = hp->n++;
    while (i > 0) {
        int64_t p = (i - 1) / 4;
        if (!hless(&x, &hp->h[p])) break;
        hp->h[i] = hp->h[p];
        i = p;
    }
    hp->h[i] = x;
    return 0;
}

static hitem heap_pop(heap_t *hp) {
    hitem top = hp->h[0];
    hitem x = hp->h[--hp->n];
    int64_t i = 0, n = hp->n;
    for (;;) {
        int64_t c0 = 4 * i + 1;
        if (c0 >= n) break;
        int64_t m = c0, ce = c0 + 4 < n ? c0 + 4 : n;
        for (int64_t c = c0 + 1; c < ce; c++)
            if (hless(&hp->h[c], &hp->h[m])) m = c;
        if (!hless(&hp->h[m], &x)) break;
        hp->h[i] = hp->h[m];
        i = m;
    }
    if (n > 0) hp->h[i] = x;
    return top;
}

typedef struct {
    int32_t n_od;
    int32_t **paths;   /* per OD row: malloc'd edge list (NULL if none) */
    int32_t *plen;     /* per OD row: edges, -1 if unreachable or O == D */
} dij_result;

typedef struct {
    int32_t head;      /* node the edge leads to */
    int32_t edge;      /* edge id */
    double w;
} arc_t;

typedef struct {
    int32_t n_nodes;
    const int32_t *out_off, *out_edge, *edge_from, *edge_to;
    arc_t *arcs;       /* out_edge order, head and weight copied alongside */
    const double *w;
    int32_t n_groups;
    const int32_t *grp_origin, *grp_off, *od_idx, *od_dst;
    dij_result *R;
    int32_t keep_order;   /* 1: the walk from the OD row's node already lists edges in travel order */
    int32_t next_group;
    pthread_mutex_t mu;
    int failed;
} job_t;

static void *worker(void *arg) {
    job_t *J = (job_t *)arg;
    int32_t n = J->n_nodes;
    double *dist = (double *)malloc((size_t)n * sizeof(double));
    int32_t *pred = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *need = (int32_t *)malloc((size_t)n * sizeof(int32_t));   /* group stamp of a wanted node */
    int32_t *tmp = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    heap_t hp = {0, 0, 0};
    int bad = (!dist || !pred || !need || !tmp);
    if (!bad)
        for (int32_t i = 0; i < n; i++) need[i] = -1;
    while (!bad) {
        pthread_mutex_lock(&J->mu);
        int32_t g = J->next_group++;
        pthread_mutex_unlock(&J->mu);
        if (g >= J->n_groups) break;
        int32_t src = J->grp_origin[g];
        for (int32_t i = 0; i < n; i++) { dist[i] = 1e300; pred[i] = -1; }
        /* the search stops once every node an OD row of this group needs is
         * settled: a settled label and its tree edge are final */
        int32_t wanted = 0;
        for (int32_t q = J->grp_off[g]; q < J->grp_off[g + 1]; q++) {
            int32_t d = J->od_dst[J->od_idx[q]];
            if (need[d] != g) { need[d] = g; wanted++; }
        }
        dist[src] = 0.0;
        hp.n = 0;
        if (heap_push(&hp, 0.0, src)) { bad = 1; break; }
        while (hp.n > 0 && !bad && wanted > 0) {
            hitem it = heap_pop(&hp);
            int32_t u = it.node;
            if (it.cost > dist[u]) continue;           /* stale entry: u was settled earlier */
            if (need[u] == g) { need[u] = -1; wanted--; }
            for (int32_t k = J->out_off[u]; k < J->out_off[u + 1]; k++) {
                const arc_t *a = &J->arcs[k];
                int32_t v = a->head;
                double nd = dist[u] + a->w;
                if (nd < dist[v]) {
                    dist[v] = nd;
                    pred[v] = a->edge;
                    if (heap_push(&hp, nd, v)) { bad = 1; break; }
                }
            }
        }
        /* rows whose node was never reached stay unreachable */
        for (int32_t q = J->grp_off[g]; q < J->grp_off[g + 1]; q++) need[J->od_dst[J->od_idx[q]]] = -1;
        if (bad) break;
        for (int32_t q = J->grp_off[g]; q < J->grp_off[g + 1]; q++) {
            int32_t od = J->od_idx[q];
            int32_t d = J->od_dst[od];
            if (d == src || pred[d] < 0) { J->R->plen[od] = -1; J->R->paths[od] = NULL; continue; }
            int32_t m = 0, cur = d;
            while (cur != src) {
                int32_t e = pred[cur];
                tmp[m++] = e;
                cur = J->edge_from[e];
            }
            int32_t *p = (int32_t *)malloc((size_t)m * sizeof(int32_t));
            if (!p) { bad = 1; break; }
            for (int32_t j = 0; j < m; j++) p[j] = J->keep_order ? tmp[j] : tmp[m - 1 - j];
            J->R->paths[od] = p;
            J->R->plen[od] = m;
        }
    }
    if (bad) { pthread_mutex_lock(&J->mu); J->failed = 1; pthread_mutex_unlock(&J->mu); }
    free(dist); free(pred); free(need); free(tmp); free(hp.h);
    return NULL;
}

void dij_free(dij_result *R) {
    if (!R) return;
    if (R->paths)
        for (int32_t i = 0; i < R->n_od; i++) free(R->paths[i]);
    free(R->paths);
    free(R->plen);
    free(R);
}

static dij_result *solve(int32_t n_nodes, const int32_t *out_off, const int32_t *out_edge,
                         const int32_t *edge_from, const int32_t *edge_to, const double *w,
                         int32_t n_od, const int32_t *od_dst,
                         int32_t n_groups, const int32_t *grp_origin, const int32_t *grp_off,
                         const int32_t *od_idx, int32_t n_threads, int32_t keep_order) {
    dij_result *R = (dij_result *)calloc(1, sizeof(dij_result));
    if (!R) return NULL;
    R->n_od = n_od;
    R->paths = (int32_t **)calloc((size_t)(n_od > 0 ? n_od : 1), sizeof(int32_t *));
    R->plen = (int32_t *)calloc((size_t)(n_od > 0 ? n_od : 1), sizeof(int32_t));
    if (!R->paths || !R->plen) { dij_free(R); return NULL; }
    for (int32_t i = 0; i < n_od; i++) R->plen[i] = -1;
    job_t J;
    memset(&J, 0, sizeof(J));
    J.n_nodes = n_nodes; J.out_off = out_off; J.out_edge = out_edge;
    J.edge_from = edge_from; J.edge_to = edge_to; J.w = w;
    J.n_groups = n_groups; J.grp_origin = grp_origin; J.grp_off = grp_off;
    J.od_idx = od_idx; J.od_dst = od_dst; J.R = R; J.keep_order = keep_order;
    J.arcs = (arc_t *)malloc((size_t)(out_off[n_nodes] > 0 ? out_off[n_nodes] : 1) * sizeof(arc_t));
    if (!J.arcs) { dij_free(R); return NULL; }
    for (int32_t k = 0; k < out_off[n_nodes]; k++) {
        int32_t e = out_edge[k];
        J.arcs[k].head = edge_to[e];
        J.arcs[k].edge = e;
        J.arcs[k].w = w[e];
    }
    pthread_mutex_init(&J.mu, NULL);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 64) n_threads = 64;
    pthread_t th[64];
    int started = 0;
    for (int i = 0; i < n_threads; i++) {
        if (pthread_create(&th[i], NULL, worker, &J) == 0) started++;
        else break;
    }
    if (started == 0) worker(&J);
    for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
    pthread_mutex_destroy(&J.mu);
    free(J.arcs);
    if (J.failed) { dij_free(R); return NULL; }
    return R;
}

/* Solve every OD row.  Origins are pre-grouped by the caller:
 * group g has origin grp_origin[g] and OD rows od_idx[grp_off[g] .. grp_off[g+1]). */
dij_result *dij_solve(int32_t n_nodes, const int32_t *out_off, const int32_t *out_edge,
                      const int32_t *edge_from, const int32_t *edge_to, const double *w,
                      int32_t n_od, const int32_t *od_dst,
                      int32_t n_groups, const int32_t *grp_origin, const int32_t *grp_off,
                      const int32_t *od_idx, int32_t n_threads) {
    return solve(n_nodes, out_off, out_edge, edge_from, edge_to, w, n_od, od_dst, n_groups, grp_origin,
                 grp_off, od_idx, n_threads, 0);
}

/* Solve every OD row grouped by destination: group g has destination
 * grp_dest[g] and OD rows od_idx[grp_off[g] .. grp_off[g+1]) whose origins
 * are od_orig[].  in_off/in_edge list the edges *into* each node (ascending
 * edge id); the paths are in travel order from the origin. */
dij_result *dij_solve_to(int32_t n_nodes, const int32_t *in_off, const int32_t *in_edge,
                         const int32_t *edge_from, const int32_t *edge_to, const double *w,
                         int32_t n_od, const int32_t *od_orig,
                         int32_t n_groups, const int32_t *grp_dest, const int32_t *grp_off,
                         const int32_t *od_idx, int32_t n_threads) {
    return solve(n_nodes, in_off, in_edge, edge_to, edge_from, w, n_od, od_orig, n_groups, grp_dest,
                 grp_off, od_idx, n_threads, 1);
}

void dij_lengths(const dij_result *R, int32_t *out) {
    for (int32_t i = 0; i < R->n_od; i++) out[i] = R->plen[i];
}

/* route_off[n_od+1] is the caller's prefix sum of max(plen, 0). */
void dij_copy(const dij_result *R, const int64_t *route_off, int32_t *route_edges) {
    for (int32_t i = 0; i < R->n_od; i++)
        if (R->plen[i] > 0)
            memcpy(route_edges + route_off[i], R->paths[i], (size_t)R->plen[i] * sizeof(int32_t));
}
