/*
 * oracle/apps_oracle.c -- plain CPU references for the heap-driven workloads.
 *
 * TEST INFRASTRUCTURE ONLY (same rule as gheap_oracle.c): only the tests, the
 * smoke check and the benchmark's CPU baseline leg use it.
 *
 *  - gho_dijkstra: textbook Dijkstra single-source shortest paths with a
 *    binary heap and lazy deletion; exact uint32 distances.  The paper's
 *    SSSP application (Sec. 5.7.1) prioritises frontier vertices by their
 *    tentative distance; shortest-path distances themselves are unique, so
 *    any correct method must reproduce these values exactly.
 *  - gho_knapsack_dp: 0/1 knapsack optimum by dynamic programming over
 *    capacities (the problem statement of Sec. 5.7.2); exact.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- binary min-heap of uint64 (dist << 32 | vertex) ------------------ */
typedef struct { uint64_t *a; uint64_t n, cap; } bheap;

static int bh_push(bheap *h, uint64_t x) {
    if (h->n == h->cap) {
        uint64_t nc = h->cap ? 2 * h->cap : 1024;
        uint64_t *na = (uint64_t *)realloc(h->a, nc * sizeof(uint64_t));
        if (!na) return -1;
        h->a = na; h->cap = nc;
    }
    uint64_t i = h->n++;
    while (i > 0) {
        uint64_t p = (i - 1) / 2;
        if (h->a[p] <= x) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i] = x;
    return 0;
}

static uint64_t bh_pop(bheap *h) {
    uint64_t top = h->a[0];
    uint64_t x = h->a[--h->n];
    uint64_t i = 0;
    for (;;) {
        uint64_t l = 2 * i + 1, r = l + 1, c = i;
        uint64_t best = x;
        if (l < h->n && h->a[l] < best) { c = l; best = h->a[l]; }
        if (r < h->n && h->a[r] < best) { c = r; best = h->a[r]; }
        if (c == i) break;
        h->a[i] = h->a[c];
        i = c;
    }
    if (h->n > 0) h->a[i] = x;
    return top;
}

int gho_dijkstra(uint32_t V, const uint64_t *rowptr, const uint32_t *col,
                 const uint32_t *w, uint32_t src, uint32_t *dist) {
    bheap h = {0, 0, 0};
    for (uint32_t v = 0; v < V; v++) dist[v] = UINT32_MAX;
    if (src >= V) return -1;
    dist[src] = 0;
    if (bh_push(&h, ((uint64_t)0 << 32) | src)) return -1;
    while (h.n > 0) {
        uint64_t e = bh_pop(&h);
        uint32_t d = (uint32_t)(e >> 32), u = (uint32_t)e;
        if (d != dist[u]) continue; /* stale entry */
        for (uint64_t j = rowptr[u]; j < rowptr[u + 1]; j++) {
            uint64_t nd = (uint64_t)d + w[j];
            uint32_t v = col[j];
            if (nd < dist[v]) {
                dist[v] = (uint32_t)nd;
                if (bh_push(&h, (nd << 32) | v)) { free(h.a); return -1; }
            }
        }
    }
    free(h.a);
    return 0;
}

uint64_t gho_knapsack_dp(uint32_t n, const uint32_t *wt, const uint32_t *val,
                         uint64_t cap) {
    uint64_t *best = (uint64_t *)calloc(cap + 1, sizeof(uint64_t));
    if (!best) return UINT64_MAX;
    for (uint32_t i = 0; i < n; i++) {
        if (wt[i] > cap) continue;
        for (uint64_t c = cap; c >= wt[i]; c--) {
            uint64_t cand = best[c - wt[i]] + val[i];
            if (cand > best[c]) best[c] = cand;
            if (c == wt[i]) break;
        }
    }
    uint64_t r = best[cap];
    free(best);
    return r;
}
