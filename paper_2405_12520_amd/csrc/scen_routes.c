/* Shortest-path routes for the synthetic demand generator (input
 * preparation, shared by every consumer of a scenario; no part of the
 * simulated model).
 *
 * For each destination node, Dijkstra from that node over the reversed road
 * graph gives every node's next road toward it; each trip then follows those
 * roads from its origin.  Roads are the directed edges (from[r] -> to[r],
 * length len[r]).  Ties between equal path lengths keep the first road
 * relaxed in increasing road id order, so the result does not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double d;
    int32_t v;
} item_t;

/* binary heap on (d, v) */
static void heap_push(item_t *h, int64_t *n, item_t x)
{
    int64_t i = (*n)++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].d < x.d || (h[p].d == x.d && h[p].v <= x.v)) break;
        h[i] = h[p];
        i = p;
    }
    h[i] = x;
}

static item_t heap_pop(item_t *h, int64_t *n)
{
    item_t top = h[0], x = h[--(*n)];
    int64_t i = 0;
    for (;;) {
        int64_t c = 2 * i + 1;
        if (c >= *n) break;
        if (c + 1 < *n && (h[c + 1].d < h[c].d || (h[c + 1].d == h[c].d && h[c + 1].v < h[c].v)))
            ++c;
        if (x.d < h[c].d || (x.d == h[c].d && x.v <= h[c].v)) break;
        h[i] = h[c];
        i = c;
    }
    h[i] = x;
    return top;
}

/* next[k * n_nodes + x]: first road of a shortest path from x to dests[k]
 * (-1 at the destination itself or where it cannot be reached).  Returns 0. */
int scen_next_roads(int32_t n_nodes, int32_t n_roads, const int32_t *from, const int32_t *to,
                    const float *len, int32_t n_dest, const int32_t *dests, int32_t *next,
                    int32_t threads)
{
    /* incoming roads of each node (reverse adjacency), in road id order */
    int32_t *off = calloc((size_t)n_nodes + 1, 4), *in = malloc(4 * (size_t)(n_roads ? n_roads : 1));
    for (int32_t r = 0; r < n_roads; ++r) off[to[r] + 1]++;
    for (int32_t j = 0; j < n_nodes; ++j) off[j + 1] += off[j];
    int32_t *fill = malloc(4 * (size_t)(n_nodes ? n_nodes : 1));
    memcpy(fill, off, 4 * (size_t)n_nodes);
    for (int32_t r = 0; r < n_roads; ++r) in[fill[to[r]]++] = r;
    free(fill);
#pragma omp parallel num_threads(threads > 0 ? threads : 1)
    {
        double *dist = malloc(8 * (size_t)n_nodes);
        uint8_t *done = malloc((size_t)n_nodes);
        item_t *heap = malloc(sizeof(item_t) * ((size_t)n_roads + 1));
#pragma omp for schedule(dynamic, 4)
        for (int32_t k = 0; k < n_dest; ++k) {
            int32_t *nx = next + (size_t)k * n_nodes;
            for (int32_t x = 0; x < n_nodes; ++x) { dist[x] = INFINITY; nx[x] = -1; done[x] = 0; }
            int64_t hn = 0;
            dist[dests[k]] = 0.0;
            heap_push(heap, &hn, (item_t){0.0, dests[k]});
            while (hn > 0) {
                item_t it = heap_pop(heap, &hn);
                if (done[it.v]) continue;
                done[it.v] = 1;
                for (int32_t q = off[it.v]; q < off[it.v + 1]; ++q) {
                    const int32_t r = in[q], u = from[r];
                    const double nd = it.d + (double)len[r];
                    if (nd < dist[u]) {
                        dist[u] = nd;
                        nx[u] = r;
                        heap_push(heap, &hn, (item_t){nd, u});
                    }
                }
            }
        }
        free(dist);
        free(done);
        free(heap);
    }
    free(off);
    free(in);
    return 0;
}

/* Route lengths (pass 1, out_len[i]) or roads (pass 2, into flat at
 * off[i]) of trips orig[i] -> dests[dk[i]] along next.  Returns -1 if some
 * trip does not reach its destination (unreachable, or more than max_hops
 * roads). */
int scen_walk_routes(int32_t n_nodes, const int32_t *to, const int32_t *next, int64_t n_trips,
                     const int32_t *orig, const int32_t *dests, const int32_t *dk,
                     int32_t max_hops, int32_t *out_len,
                     const int64_t *off, int32_t *flat, int32_t threads)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad) num_threads(threads > 0 ? threads : 1)
    for (int64_t i = 0; i < n_trips; ++i) {
        const int32_t *nx = next + (size_t)dk[i] * n_nodes;
        int32_t x = orig[i], h = 0, r;
        while ((r = nx[x]) >= 0 && h < max_hops) {
            if (flat) flat[off[i] + h] = r;
            ++h;
            x = to[r];
        }
        if (x != dests[dk[i]]) bad = 1;
        if (out_len) out_len[i] = h;
    }
    return bad ? -1 : 0;
}
