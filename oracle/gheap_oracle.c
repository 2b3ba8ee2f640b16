/*
 * oracle/gheap_oracle.c -- plain sequential CPU oracle for the generalized heap.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or helper with the
 * HIP library.
 *
 * What it computes (Chen et al., "Accelerating Concurrent Heap on GPUs"):
 *   - a generalized min-heap whose nodes each hold a sorted batch of k entries
 *     (Sec. 3.1), kept in an implicit binary tree, node c at array slots
 *     [(c-1)k, ck), root first;
 *   - a partial buffer of at most k-1 sorted entries, all >= the root's
 *     largest entry (Sec. 3.1, Property 3);
 *   - MergeAndSort (Sec. 3.2, the display equation defining (hi, lo)): the
 *     merge of two sorted batches split into the smallest |a| and the rest;
 *   - DEL (Sec. 3.2.1): output the root, refill it from the last node,
 *     MAX-fill that node, then sift down with the "lo goes to the child whose
 *     maximum was larger" rule, stopping once the property holds;
 *   - top-down INS (Sec. 3.2.2, "Top-down INS" paragraph): merge the batch
 *     with every node on the root-to-target path, the node keeping the k
 *     smallest, and place the carry at the target;
 *   - bottom-up INS (Sec. 3.2.2, "Bottom-up INS" paragraph): place the batch
 *     at the target, then MergeAndSort each node on the insert path with its
 *     parent, the parent keeping the k smallest, until the root or until the
 *     parent's largest entry is no larger than the node's smallest;
 *   - partial batches (Sec. 3.3.2, last two paragraphs before the
 *     linearizability proof): insert keys merge with the partial buffer
 *     first; a DEL reads the partial buffer only when no node exists; and, as
 *     Sec. 3.3.4 states, the partial buffer is handled whenever an operation
 *     holds the root, so a DEL re-establishes Property 3 after refilling the
 *     root;
 *   - DEL of c < k entries (variable count; a reading, see gho_delete_min_n):
 *     the root's c smallest, then the root's rest and the partial buffer
 *     refill the top, taking the last node only when they are fewer than k;
 *   - bulk build from an ascending array (Sec. 3.1) and a filter that keeps
 *     the entries below a bound (garbage collection, Sec. 5.7.2);
 *   - target order by bit-reversal permutation (Sec. 4.3, "Bit-Reversal
 *     Permutation"), DEL taking the last node in the reverse order.
 *
 * Entries are unsigned 64-bit integers compared as integers; the all-ones
 * value is reserved as the MAX filler and never inserted.  Callers that need
 * (key, id) pairs pack them as key<<32 | id.  Compiled with -DGHO_WIDE the
 * same file gives the oracle for 16-byte entries (a signed 64-bit key and a
 * 32-bit id, ordered by key, then id): an entry is then an unsigned 128-bit
 * integer whose high half is the biased key (key XOR 2^63) and whose low half
 * is the id, so that integer order is that lexicographic order, and every
 * exported name starts with ghow_ instead of gho_.
 *
 * Everything here is deliberately plain: two-pointer merges, qsort, no
 * blocking and no reordering beyond what the paper's steps state.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef GHO_WIDE
typedef unsigned __int128 gho_ent;
#define GHO_MAX (~(gho_ent)0)
#define gho_idx ghow_idx
#define gho_new ghow_new
#define gho_free ghow_free
#define gho_size ghow_size
#define gho_nodes ghow_nodes
#define gho_pb_size ghow_pb_size
#define gho_insert ghow_insert
#define gho_insert_bu ghow_insert_bu
#define gho_delete_min ghow_delete_min
#define gho_delete_min_n ghow_delete_min_n
#define gho_build ghow_build
#define gho_filter ghow_filter
#define gho_filter_key ghow_filter_key
#define gho_check ghow_check
#define gho_node_slots ghow_node_slots
#define gho_export ghow_export
#define gho_merge_and_sort ghow_merge_and_sort
#define gho_counters ghow_counters
#define gho_replay ghow_replay
#else
typedef uint64_t gho_ent;
#define GHO_MAX UINT64_MAX
#endif

typedef struct gho_heap {
    uint32_t k;        /* node capacity */
    uint64_t m;        /* number of nodes in use */
    uint64_t cap;      /* node slots allocated */
    gho_ent *node;     /* node c (1-based) at node[(c-1)*k] */
    gho_ent *pb;       /* partial buffer (capacity k-1) */
    uint64_t s;        /* partial-buffer size */
    gho_ent *tmp;      /* scratch of 2k entries */
    gho_ent *tmp2;     /* scratch of 2k entries */
    /* work counters (levels actually traversed), for byte accounting */
    uint64_t ins_ops, ins_full, ins_path_nodes, del_ops, del_levels;
    /* deleteMins that refilled the root from the last node, and the
     * algorithmic traffic of every operation in entries (count_insert,
     * count_delete) */
    uint64_t del_refill, traffic;
} gho_heap;

/* ---- bit-reversal target order (Sec. 4.3) ------------------------------ */

static int floor_log2(uint64_t p) {
    int l = 0;
    while ((p >> 1) != 0) { p >>= 1; l++; }
    return l;
}

static uint64_t reverse_low_bits(uint64_t x, int l) {
    uint64_t r = 0;
    for (int i = 0; i < l; i++) {
        r = (r << 1) | (x & 1);
        x >>= 1;
    }
    return r;
}

/* Node index of the p-th node added (p >= 1): level l = floor(log2 p), and
 * within the level the offset p - 2^l is bit-reversed over l bits.  The map is
 * its own inverse, so it also gives the position of a node index. */
uint64_t gho_idx(uint64_t p) {
    int l = floor_log2(p);
    uint64_t base = (uint64_t)1 << l;
    return base + reverse_low_bits(p - base, l);
}

/* ---- MergeAndSort (Sec. 3.2.1 display equation) ------------------------ */

/* Merge sorted a[0..na) and b[0..nb); the na smallest go to hi[0..na), the
 * remaining nb to lo[0..nb).  hi/lo may alias a/b (merge goes through tmp). */
static void merge_and_sort(gho_heap *h, const gho_ent *a, uint64_t na,
                           const gho_ent *b, uint64_t nb,
                           gho_ent *hi, gho_ent *lo) {
    gho_ent *t = h->tmp;
    uint64_t i = 0, j = 0, o = 0;
    while (i < na && j < nb) {
        if (a[i] <= b[j]) t[o++] = a[i++];
        else t[o++] = b[j++];
    }
    while (i < na) t[o++] = a[i++];
    while (j < nb) t[o++] = b[j++];
    memcpy(hi, t, na * sizeof(gho_ent));
    memcpy(lo, t + na, nb * sizeof(gho_ent));
}

/* plain merge of a and b into out (out must not alias) */
static void merge_into(const gho_ent *a, uint64_t na, const gho_ent *b,
                       uint64_t nb, gho_ent *out) {
    uint64_t i = 0, j = 0, o = 0;
    while (i < na && j < nb) {
        if (a[i] <= b[j]) out[o++] = a[i++];
        else out[o++] = b[j++];
    }
    while (i < na) out[o++] = a[i++];
    while (j < nb) out[o++] = b[j++];
}

static int cmp_ent(const void *x, const void *y) {
    gho_ent a = *(const gho_ent *)x, b = *(const gho_ent *)y;
    return (a > b) - (a < b);
}

/* ---- heap state -------------------------------------------------------- */

static gho_ent *node_at(gho_heap *h, uint64_t c) {
    return h->node + (c - 1) * (uint64_t)h->k;
}

static int node_exists(const gho_heap *h, uint64_t c) {
    return c >= 1 && gho_idx(c) <= h->m;
}

static int ensure_cap(gho_heap *h, uint64_t c) {
    if (c <= h->cap) return 0;
    uint64_t ncap = h->cap ? h->cap : 16;
    while (ncap < c) ncap *= 2;
    gho_ent *nn = (gho_ent *)realloc(h->node, ncap * (uint64_t)h->k * sizeof(gho_ent));
    if (!nn) return -1;
    for (uint64_t i = h->cap * (uint64_t)h->k; i < ncap * (uint64_t)h->k; i++) nn[i] = GHO_MAX;
    h->node = nn;
    h->cap = ncap;
    return 0;
}

gho_heap *gho_new(uint32_t k) {
    if (k == 0) return NULL;
    gho_heap *h = (gho_heap *)calloc(1, sizeof(gho_heap));
    if (!h) return NULL;
    h->k = k;
    h->pb = (gho_ent *)malloc((size_t)k * sizeof(gho_ent));
    h->tmp = (gho_ent *)malloc((size_t)2 * k * sizeof(gho_ent) + 16);
    h->tmp2 = (gho_ent *)malloc((size_t)2 * k * sizeof(gho_ent) + 16);
    if (!h->pb || !h->tmp || !h->tmp2 || ensure_cap(h, 16)) {
        free(h->pb); free(h->tmp); free(h->tmp2); free(h->node); free(h);
        return NULL;
    }
    return h;
}

void gho_free(gho_heap *h) {
    if (!h) return;
    free(h->node); free(h->pb); free(h->tmp); free(h->tmp2);
    free(h);
}

uint64_t gho_size(const gho_heap *h) { return h->m * (uint64_t)h->k + h->s; }
uint64_t gho_nodes(const gho_heap *h) { return h->m; }
uint64_t gho_pb_size(const gho_heap *h) { return h->s; }

/* ---- INS: one operation of n <= k entries (Sec. 3.2.2 and 3.3.2) ------- */

/* The partial-buffer rule shared by both INS forms (Sec. 3.3.2): an input
 * of n entries fits when the partial buffer (capacity k - 1) can take it. */
static int pb_takes(const gho_heap *h, uint64_t n) { return n + h->s <= h->k - 1; }

/* The pb keeps merged (its old entries and the n new ones); then, if a root
 * exists, root and pb are merged so that the pb's entries are >= the root's
 * (Property 3). */
static void keep_in_pb(gho_heap *h, const gho_ent *merged, uint64_t n) {
    const uint64_t k = h->k;
    memcpy(h->pb, merged, (n + h->s) * sizeof(gho_ent));
    h->s += n;
    if (h->m >= 1)
        merge_and_sort(h, node_at(h, 1), k, h->pb, h->s, node_at(h, 1), h->pb);
}

static int insert_batch(gho_heap *h, const gho_ent *x, uint64_t n) {
    const uint64_t k = h->k;
    gho_ent *in = h->tmp2;          /* sorted copy of the input */
    gho_ent *merged;
    memcpy(in, x, n * sizeof(gho_ent));
    qsort(in, n, sizeof(gho_ent), cmp_ent);
    merged = (gho_ent *)malloc((n + h->s) * sizeof(gho_ent) + 8);
    if (!merged) return -1;
    merge_into(in, n, h->pb, h->s, merged);
    h->ins_ops++;
    if (pb_takes(h, n)) {
        /* the partial buffer has room: keep everything there */
        keep_in_pb(h, merged, n);
        free(merged);
        return 0;
    }
    /* a full batch F (the k smallest) goes down from the root; the rest
     * stays in the partial buffer */
    uint64_t rest = n + h->s - k;
    gho_ent *F = h->tmp2;           /* reuse: the sorted input is consumed */
    memcpy(F, merged, k * sizeof(gho_ent));
    memcpy(h->pb, merged + k, rest * sizeof(gho_ent));
    h->s = rest;
    free(merged);
    h->ins_full++;
    uint64_t t = gho_idx(h->m + 1);
    if (ensure_cap(h, t)) return -1;
    h->m += 1;
    int L = floor_log2(t);
    for (int j = 0; j < L; j++) {
        uint64_t c = t >> (L - j);  /* the path node at depth j */
        merge_and_sort(h, node_at(h, c), k, F, k, node_at(h, c), F);
        h->ins_path_nodes++;
    }
    memcpy(node_at(h, t), F, k * sizeof(gho_ent));
    return 0;
}

/* Algorithmic traffic of one operation, counted in entries: what the
 * method moves between memory and the working copy along the path the
 * operation took (the node loads and stores, the partial buffer, the input
 * and the output).  An insert of n entries that found m0 nodes and s0
 * partial-buffer entries: kept in the partial buffer, 2 (n + s0) plus 2k
 * for the root merge if a root exists; a full batch to a target on level L,
 * (n + s0 + (n + s0 - k)) + (2 k L + k). */
static void count_insert(gho_heap *h, uint64_t n, uint64_t m0, uint64_t s0) {
    const uint64_t k = h->k;
    if (h->m > m0) {
        uint64_t L = (uint64_t)floor_log2(gho_idx(m0 + 1));
        h->traffic += (n + s0 + (n + s0 - k)) + (2 * k * L + k);
    } else {
        h->traffic += 2 * (n + s0) + (m0 >= 1 ? 2 * k : 0);
    }
}

/* A deleteMin that found m0 nodes and s0 partial-buffer entries: with no
 * node 2 s0; from the root alone 2k; refilled from the last node with L
 * levels merged, k (3 + 4 L) + 2 s0. */
static void count_delete(gho_heap *h, uint64_t m0, uint64_t s0, uint64_t lv0, int refilled) {
    const uint64_t k = h->k;
    if (m0 == 0) {
        h->traffic += 2 * s0;
    } else if (refilled) {
        h->del_refill++;
        h->traffic += k * (3 + 4 * (h->del_levels - lv0)) + 2 * s0;
    } else {
        h->traffic += 2 * k;
    }
}

/* ---- bottom-up INS (Sec. 3.2.2, "Bottom-up INS" paragraph) ------------
 * The partial buffer is handled at the root as for the top-down INS (Sec.
 * 3.3.4 says so for the BU-INS/TD-DEL heap): merged = merge(sorted input,
 * pb); if it fits the pb (n + s <= k - 1) everything stays there and the pb
 * is merged with the root, exactly as the top-down INS does.  Otherwise F =
 * its k smallest goes to the target (the next node position), the rest is
 * the new pb, and F climbs: the node on the insert path and its parent are
 * merged, the parent keeping the k smallest, until the root is reached or
 * the parent's largest entry is <= the node's smallest (the property holds
 * from there up).  After the climb the root is the k smallest of root and F,
 * so Property 3 holds again (the pb's entries are >= the k of F). */
static int insert_batch_bu(gho_heap *h, const gho_ent *x, uint64_t n, uint64_t *levels) {
    const uint64_t k = h->k;
    gho_ent *in = h->tmp2;
    memcpy(in, x, n * sizeof(gho_ent));
    qsort(in, n, sizeof(gho_ent), cmp_ent);
    gho_ent *merged = (gho_ent *)malloc((n + h->s) * sizeof(gho_ent) + 8);
    if (!merged) return -1;
    merge_into(in, n, h->pb, h->s, merged);
    h->ins_ops++;
    *levels = 0;
    if (pb_takes(h, n)) {
        keep_in_pb(h, merged, n);
        free(merged);
        return 0;
    }
    uint64_t rest = n + h->s - k;
    uint64_t t = gho_idx(h->m + 1);
    if (ensure_cap(h, t)) { free(merged); return -1; }
    memcpy(node_at(h, t), merged, k * sizeof(gho_ent));
    memcpy(h->pb, merged + k, rest * sizeof(gho_ent));
    h->s = rest;
    h->m += 1;
    free(merged);
    h->ins_full++;
    uint64_t c = t;
    while (c > 1) {
        gho_ent *C = node_at(h, c), *P = node_at(h, c / 2);
        if (P[k - 1] <= C[0]) break;             /* the property holds from here up */
        merge_and_sort(h, P, k, C, k, P, C);     /* parent keeps the k smallest */
        h->ins_path_nodes++;
        (*levels)++;
        c /= 2;
    }
    return 0;
}

/* Insert n entries bottom-up: chunks of k as gho_insert takes them.  The
 * traffic counted for a full batch that merged L times: the input and pb as
 * for a top-down insert, the target written (k), and per merge the parent
 * read and both nodes written (3k), plus the parent read by the check that
 * stopped the climb below the root (k). */
int gho_insert_bu(gho_heap *h, const gho_ent *x, uint64_t n) {
    const uint64_t k = h->k;
    uint64_t done = 0;
    while (done < n) {
        uint64_t c = n - done < k ? n - done : k;
        uint64_t m0 = h->m, s0 = h->s, L = 0;
        if (insert_batch_bu(h, x + done, c, &L)) return -1;
        if (h->m > m0) {
            uint64_t t = gho_idx(m0 + 1);
            int stopped = (uint64_t)floor_log2(t) > L;   /* a check stopped below the root */
            h->traffic += (c + s0 + (c + s0 - k)) + k + 3 * k * L + (stopped ? k : 0);
        } else {
            h->traffic += 2 * (c + s0) + (m0 >= 1 ? 2 * k : 0);
        }
        done += c;
    }
    return 0;
}

/* Insert n entries: n <= k is one INS; larger inputs are split into
 * consecutive chunks of k (footnote to the INS paragraph, Sec. 3.2.2). */
int gho_insert(gho_heap *h, const gho_ent *x, uint64_t n) {
    uint64_t done = 0;
    while (done < n) {
        uint64_t c = n - done < h->k ? n - done : h->k;
        uint64_t m0 = h->m, s0 = h->s;
        if (insert_batch(h, x + done, c)) return -1;
        count_insert(h, c, m0, s0);
        done += c;
    }
    return 0;
}

/* ---- DEL (Sec. 3.2.1, partial buffer per Sec. 3.3.2/3.3.4) ------------- */

static void sift_down(gho_heap *h);

/* Removes and returns the min(k, size) smallest entries, ascending. */
static uint64_t delete_root(gho_heap *h, gho_ent *out) {
    const uint64_t k = h->k;
    h->del_ops++;
    if (h->m == 0) {
        /* no node: the partial buffer holds everything */
        uint64_t cnt = h->s;
        memcpy(out, h->pb, cnt * sizeof(gho_ent));
        h->s = 0;
        return cnt;
    }
    memcpy(out, node_at(h, 1), k * sizeof(gho_ent));
    if (h->m == 1) {
        h->m = 0;
        for (uint64_t i = 0; i < k; i++) node_at(h, 1)[i] = GHO_MAX;
        return k;
    }
    /* refill the root from the last node, then MAX-fill that node */
    uint64_t last = gho_idx(h->m);
    memcpy(node_at(h, 1), node_at(h, last), k * sizeof(gho_ent));
    for (uint64_t i = 0; i < k; i++) node_at(h, last)[i] = GHO_MAX;
    h->m -= 1;
    if (h->s > 0)
        merge_and_sort(h, node_at(h, 1), k, h->pb, h->s, node_at(h, 1), h->pb);
    sift_down(h);
    return k;
}

/* ---- DEL of c < k entries (variable-count deleteMin) -------------------
 * The plain definition fixes the result: the min(c, size) smallest live
 * entries, ascending.  The steps are a reading of Sec. 3.2.1 and Sec. 3.3.2
 * (the paper only defines deleteMin of a whole root): the root's c smallest
 * are the answer; its k - c others and the partial buffer, merged, are what
 * must stay above every node.  If they are at least k entries, the k smallest
 * form the new root and the rest the partial buffer (no node goes away);
 * otherwise the last node is taken as for a full DEL, and the new root is the
 * k smallest of it and the merged rest, the remainder (< k entries) the
 * partial buffer.  Either way the root sifts down as in DEL.  With no node
 * the partial buffer gives its c smallest; with one node and fewer than k
 * entries left at the top, they all become the partial buffer.  For c = k
 * this is exactly gho_delete_min. */
uint64_t gho_delete_min(gho_heap *h, gho_ent *out) {
    uint64_t m0 = h->m, s0 = h->s, lv0 = h->del_levels;
    uint64_t got = delete_root(h, out);
    count_delete(h, m0, s0, lv0, m0 >= 2);
    return got;
}

static uint64_t delete_n(gho_heap *h, gho_ent *out, uint64_t c) {
    const uint64_t k = h->k;
    if (c == 0 || c > k) return UINT64_MAX;
    if (c == k) return gho_delete_min(h, out);
    h->del_ops++;
    if (h->m == 0) {
        uint64_t cnt = h->s < c ? h->s : c;
        memcpy(out, h->pb, cnt * sizeof(gho_ent));
        memmove(h->pb, h->pb + cnt, (h->s - cnt) * sizeof(gho_ent));
        h->s -= cnt;
        return cnt;
    }
    gho_ent *root = node_at(h, 1);
    memcpy(out, root, c * sizeof(gho_ent));
    /* what stays at the top: the root's other k - c entries and the pb */
    uint64_t nrest = k - c + h->s;
    gho_ent *rest = h->tmp2;
    merge_into(root + c, k - c, h->pb, h->s, rest);
    if (nrest >= k) {
        memcpy(root, rest, k * sizeof(gho_ent));
        memcpy(h->pb, rest + k, (nrest - k) * sizeof(gho_ent));
        h->s = nrest - k;
    } else if (h->m == 1) {
        memcpy(h->pb, rest, nrest * sizeof(gho_ent));
        h->s = nrest;
        h->m = 0;
        for (uint64_t i = 0; i < k; i++) root[i] = GHO_MAX;
        return c;
    } else {
        uint64_t last = gho_idx(h->m);
        merge_and_sort(h, node_at(h, last), k, rest, nrest, root, h->pb);
        for (uint64_t i = 0; i < k; i++) node_at(h, last)[i] = GHO_MAX;
        h->m -= 1;
        h->s = nrest;
    }
    sift_down(h);
    return c;
}

uint64_t gho_delete_min_n(gho_heap *h, gho_ent *out, uint64_t c) {
    if (c == 0 || c >= h->k) return delete_n(h, out, c);   /* c = k: counted by gho_delete_min */
    uint64_t m0 = h->m, s0 = h->s, lv0 = h->del_levels;
    uint64_t got = delete_n(h, out, c);
    count_delete(h, m0, s0, lv0, m0 >= 2 && h->k - c + s0 < h->k);
    return got;
}

/* Sift the root down (Sec. 3.2.1): at each node, stop once its largest
 * entry is <= every existing child's smallest; with two children, their
 * MergeAndSort leaves lo in the child whose maximum was larger and hi merges
 * with the node, whose k smallest stay; with one child, the node merges with
 * it. */
static void sift_down(gho_heap *h) {
    const uint64_t k = h->k;
    uint64_t c = 1;
    for (;;) {
        uint64_t l = 2 * c, r = 2 * c + 1;
        int el = node_exists(h, l), er = node_exists(h, r);
        gho_ent *cur = node_at(h, c);
        if (!el && !er) break;
        if (el && er) {
            gho_ent *L = node_at(h, l), *R = node_at(h, r);
            gho_ent cmin = L[0] < R[0] ? L[0] : R[0];
            if (cur[k - 1] <= cmin) break;
            /* lo goes to the child whose maximum was larger (on a tie, r) */
            uint64_t big = (L[k - 1] > R[k - 1]) ? l : r;
            uint64_t small = (big == l) ? r : l;
            gho_ent *hi = h->tmp2;
            merge_and_sort(h, L, k, R, k, hi, h->tmp2 + k);
            memcpy(node_at(h, big), h->tmp2 + k, k * sizeof(gho_ent));
            merge_and_sort(h, cur, k, hi, k, cur, node_at(h, small));
            h->del_levels++;
            c = small;
        } else {
            uint64_t x = el ? l : r;
            gho_ent *X = node_at(h, x);
            if (cur[k - 1] <= X[0]) break;
            merge_and_sort(h, cur, k, X, k, cur, X);
            h->del_levels++;
            c = x;
        }
    }
}

/* ---- bulk build and filter (Sec. 3.1: a sorted array is a heap) -------- */

/* Build an empty heap from n ascending entries: the p-th chunk of k becomes
 * the node added p-th (node index idx(p)), the rest the partial buffer.
 * Returns 0, -1 when the heap is not empty or memory runs out, -2 when the
 * input is not ascending or holds the reserved entry. */
int gho_build(gho_heap *h, const gho_ent *sorted, uint64_t n) {
    const uint64_t k = h->k;
    if (h->m != 0 || h->s != 0) return -1;
    for (uint64_t i = 0; i < n; i++) {
        if (sorted[i] == GHO_MAX) return -2;
        if (i > 0 && sorted[i - 1] > sorted[i]) return -2;
    }
    uint64_t m = n / k;
    for (uint64_t p = 1; p <= m; p++) {
        uint64_t c = gho_idx(p);
        if (ensure_cap(h, c)) return -1;
        memcpy(node_at(h, c), sorted + (p - 1) * k, k * sizeof(gho_ent));
    }
    h->m = m;
    h->s = n - m * k;
    memcpy(h->pb, sorted + m * k, h->s * sizeof(gho_ent));
    return 0;
}

/* Filter: remove every entry >= bound (the garbage collection of a
 * branch-and-bound search, Sec. 5.7.2, with the bound as the cut).  The
 * entries kept are gathered, sorted and built again as above.  Returns the
 * number kept, or UINT64_MAX when memory runs out. */
uint64_t gho_filter(gho_heap *h, gho_ent bound) {
    const uint64_t k = h->k;
    uint64_t size = gho_size(h), kept = 0;
    gho_ent *buf = (gho_ent *)malloc(size * sizeof(gho_ent) + 8);
    if (!buf) return UINT64_MAX;
    for (uint64_t p = 1; p <= h->m; p++) {
        gho_ent *N = node_at(h, gho_idx(p));
        for (uint64_t i = 0; i < k; i++)
            if (N[i] < bound) buf[kept++] = N[i];
        for (uint64_t i = 0; i < k; i++) N[i] = GHO_MAX;
    }
    for (uint64_t i = 0; i < h->s; i++)
        if (h->pb[i] < bound) buf[kept++] = h->pb[i];
    h->m = 0;
    h->s = 0;
    qsort(buf, kept, sizeof(gho_ent), cmp_ent);
    int rc = gho_build(h, buf, kept);
    free(buf);
    return rc == 0 ? kept : UINT64_MAX;
}

#ifdef GHO_WIDE
/* Filter of a 16-byte heap by a key word: every entry whose biased key is
 * >= key_word goes (the entry bound is (key_word, id 0)). */
uint64_t gho_filter_key(gho_heap *h, uint64_t key_word) {
    return gho_filter(h, (gho_ent)key_word << 64);
}
#endif

/* ---- invariant checker (Sec. 3.1, Properties 1-3) ---------------------- */

/* Returns 0 if the heap satisfies Properties 1-3 and its bookkeeping, else a
 * positive code naming the first violation found. */
int gho_check(const gho_heap *h) {
    const uint64_t k = h->k;
    if (h->s > k - 1) return 10;                                   /* pb capacity */
    for (uint64_t i = 1; i < h->s; i++)
        if (h->pb[i - 1] > h->pb[i]) return 3;                     /* Property 3 order */
    if (h->m >= 1 && h->s >= 1 && h->pb[0] < h->node[k - 1]) return 4; /* Property 3 bound */
    for (uint64_t c = 1; c <= h->cap; c++) {
        const gho_ent *N = h->node + (c - 1) * k;
        if (node_exists(h, c)) {
            for (uint64_t i = 0; i < k; i++) {
                if (N[i] == GHO_MAX) return 5;                     /* reserved value live */
                if (i > 0 && N[i - 1] > N[i]) return 2;            /* Property 2 */
            }
            if (c > 1) {
                const gho_ent *P = h->node + (c / 2 - 1) * k;
                if (N[0] < P[k - 1]) return 1;                     /* Property 1 */
            }
        } else {
            for (uint64_t i = 0; i < k; i++)
                if (N[i] != GHO_MAX) return 6;                     /* stale node */
        }
    }
    return 0;
}

/* copy out the node array (m-independent: slots 1..cap) and the pb */
uint64_t gho_node_slots(const gho_heap *h) { return h->cap; }
void gho_export(const gho_heap *h, gho_ent *nodes_out, gho_ent *pb_out) {
    if (nodes_out) memcpy(nodes_out, h->node, h->cap * (uint64_t)h->k * sizeof(gho_ent));
    if (pb_out) memcpy(pb_out, h->pb, h->s * sizeof(gho_ent));
}

/* MergeAndSort exposed for the tests (na + nb <= 2k of this heap). */
void gho_merge_and_sort(gho_heap *h, const gho_ent *a, uint64_t na,
                        const gho_ent *b, uint64_t nb, gho_ent *hi, gho_ent *lo) {
    merge_and_sort(h, a, na, b, nb, hi, lo);
}

void gho_counters(const gho_heap *h, uint64_t out[7]) {
    out[0] = h->ins_ops; out[1] = h->ins_full; out[2] = h->ins_path_nodes;
    out[3] = h->del_ops; out[4] = h->del_levels; out[5] = h->del_refill;
    out[6] = h->traffic;
}

/* ---- log replay --------------------------------------------------------
 * Apply ops in the given order: type 0 = INS of n[i] entries read from
 * in_keys + off[i] (type 2: the same, bottom-up); type 1 = DEL of n[i] entries (0 = k; more than k fails)
 * whose output goes to out_keys + off[i] and whose count goes to
 * out_count[i].  With check != 0 the invariants are
 * verified after every op.  Returns 0, or -(1 + index) of the first op that
 * failed (allocation or invariant), or -(1<<40) on a bad type. */
int64_t gho_replay(gho_heap *h, uint64_t nops, const uint8_t *type,
                   const uint32_t *n, const uint64_t *off,
                   const gho_ent *in_keys, gho_ent *out_keys,
                   uint32_t *out_count, int check) {
    for (uint64_t i = 0; i < nops; i++) {
        if (type[i] == 0 || type[i] == 2) {
            /* type 2: the bottom-up INS */
            int rc = type[i] == 0 ? gho_insert(h, in_keys + off[i], n[i])
                                  : gho_insert_bu(h, in_keys + off[i], n[i]);
            if (rc) return -(int64_t)(i + 1);
            if (out_count) out_count[i] = 0;
        } else if (type[i] == 1) {
            /* n[i] = entries requested, 0 meaning k */
            uint64_t want = n[i] ? n[i] : h->k;
            uint64_t c = gho_delete_min_n(h, out_keys + off[i], want);
            if (c == UINT64_MAX) return -(int64_t)(i + 1);
            if (out_count) out_count[i] = (uint32_t)c;
        } else {
            return -((int64_t)1 << 40);
        }
        if (check && gho_check(h)) return -(int64_t)(i + 1);
    }
    return 0;
}
