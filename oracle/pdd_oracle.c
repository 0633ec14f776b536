/*
 * pdd_oracle.c -- plain sequential CPU reference for k-NN-cost Poisson-disk
 * decimation.  TEST INFRASTRUCTURE ONLY: it is built and called by the test
 * suite, the smoke check and the benchmark's CPU-baseline leg, never by the
 * product path.  It shares no code with the HIP library.
 *
 * What it computes (all integer, exact):
 *
 *   - d2(i, j)  = sum over axes of (P_i - P_j)^2 in int64, P in int32 mm.
 *   - term(D)   = floor(2^56 / D) for D >= 1, and 2^58 for D = 0.  This is
 *                 the fixed-point reading of the inverse squared distance of
 *                 Eq. 11/12 (Sec. 4.2); coincident points (D = 0, for which
 *                 the real-valued cost is infinite) get a term above every
 *                 finite one.
 *   - W(i; S)   = sum of term(D) over the min(k, |S| - 1) smallest values of
 *                 the multiset { d2(i, j) : j in S, j != i }  (Eq. 12: the
 *                 cost is a sum over the k-neighbourhood).
 *   - key(i)    = (W descending, original index ascending).
 *   - greedy    : repeatedly remove the alive point of highest key, emit
 *                 (index, W) and update the costs that the removal changes
 *                 (Sec. 4: sort by cost, remove the highest, update the
 *                 neighbours of the removed sample; Sec. 4.2 applies it with
 *                 the k-neighbourhood cost), until exactly keep points are
 *                 left (Sec. 3, |C'| = lambda |C| with lambda = m / |C|).
 *
 * How it computes it:
 *   - an index-based kd-tree (median splits, leaves of <= 8 points, tight
 *     boxes, alive counts per node) answers exact top-K queries ordered by
 *     (d2, index) over the alive points;
 *   - every point keeps a buffer of its K = k + b nearest alive points from
 *     its last search (the extended k+b neighbourhood of Sec. 5); while at
 *     least k buffer entries are alive, its first k alive entries are its k
 *     nearest alive points; otherwise it is searched again at once (the
 *     buffer is only a cache, so the result does not depend on b);
 *   - reverse lists (the set N(p) of Sec. 5: the points holding p in their
 *     neighbourhood) find the points to re-cost after a removal;
 *   - an indexed binary max-heap holds the keys; costs only decrease, so an
 *     update is a sift-down.
 *
 * With check != 0 it also asserts the invariants the method relies on
 * (Sec. 5, step 2: removing a point never raises a cost): every re-cost is
 * <= the old cost, the emitted keys strictly decrease, exactly keep points
 * remain, and at the end every kept point's maintained cost equals a fresh
 * computation from scratch.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PDDO_OK 0
#define PDDO_EINVAL -1
#define PDDO_ENOMEM -2
#define PDDO_ECHECK_RISE -10   /* a re-cost increased a cost */
#define PDDO_ECHECK_ORDER -11  /* emitted keys did not strictly decrease */
#define PDDO_ECHECK_KEEP -12   /* kept count differs from keep */
#define PDDO_ECHECK_FINAL -13  /* a maintained cost differs from a fresh one */
#define PDDO_ECHECK_NEXT -14   /* a kept key exceeds the last removed key */

#define LEAF_SIZE 8
#define MAX_K 64

uint64_t pddo_term(int64_t d2) {
    if (d2 == 0) return (uint64_t)1 << 58;
    return ((uint64_t)1 << 56) / (uint64_t)d2;
}

static inline int64_t dist2(const int32_t *P, int64_t a, int64_t b) {
    int64_t dx = (int64_t)P[3 * a] - P[3 * b];
    int64_t dy = (int64_t)P[3 * a + 1] - P[3 * b + 1];
    int64_t dz = (int64_t)P[3 * a + 2] - P[3 * b + 2];
    return dx * dx + dy * dy + dz * dz;
}

/* ------------------------------------------------------------------------ */
/* kd-tree                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t lo, hi;          /* range of perm[] */
    int64_t left, right;     /* children, -1 for a leaf */
    int64_t parent;
    int64_t alive;           /* alive points below this node */
    int32_t bmin[3], bmax[3];
} node_t;

typedef struct {
    const int32_t *P;
    int64_t n;
    int64_t *perm;
    int64_t *leaf_of;
    node_t *nodes;
    int64_t nnodes, cap;
} kdtree_t;

static inline int32_t coord(const int32_t *P, int64_t i, int axis) { return P[3 * i + axis]; }

/* Rearrange a[lo..hi] (inclusive) so that a[kth] holds the element of that
 * rank along `axis`, smaller-or-equal ones before it, larger-or-equal after. */
static void nth_element(int64_t *a, int64_t lo, int64_t hi, int64_t kth, const int32_t *P, int axis) {
    while (lo < hi) {
        int64_t m = lo + (hi - lo) / 2;
        int32_t x = coord(P, a[lo], axis), y = coord(P, a[m], axis), z = coord(P, a[hi], axis);
        int32_t pv;
        if (x < y) pv = (y < z) ? y : ((x < z) ? z : x);
        else pv = (x < z) ? x : ((y < z) ? z : y);
        int64_t i = lo, j = hi;
        while (i <= j) {
            while (coord(P, a[i], axis) < pv) i++;
            while (coord(P, a[j], axis) > pv) j--;
            if (i <= j) {
                int64_t t = a[i]; a[i] = a[j]; a[j] = t;
                i++; j--;
            }
        }
        if (kth <= j) hi = j;
        else if (kth >= i) lo = i;
        else return;
    }
}

static int64_t new_node(kdtree_t *t) {
    if (t->nnodes == t->cap) {
        int64_t nc = t->cap ? t->cap * 2 : 1024;
        node_t *nn = (node_t *)realloc(t->nodes, (size_t)nc * sizeof(node_t));
        if (!nn) return -1;
        t->nodes = nn;
        t->cap = nc;
    }
    return t->nnodes++;
}

static int64_t build_rec(kdtree_t *t, int64_t lo, int64_t hi, int64_t parent) {
    int64_t id = new_node(t);
    if (id < 0) return -1;
    node_t nd;
    nd.lo = lo; nd.hi = hi; nd.parent = parent; nd.alive = hi - lo;
    nd.left = nd.right = -1;
    for (int a = 0; a < 3; a++) { nd.bmin[a] = INT32_MAX; nd.bmax[a] = INT32_MIN; }
    for (int64_t p = lo; p < hi; p++) {
        for (int a = 0; a < 3; a++) {
            int32_t c = coord(t->P, t->perm[p], a);
            if (c < nd.bmin[a]) nd.bmin[a] = c;
            if (c > nd.bmax[a]) nd.bmax[a] = c;
        }
    }
    if (hi - lo <= LEAF_SIZE) {
        for (int64_t p = lo; p < hi; p++) t->leaf_of[t->perm[p]] = id;
        t->nodes[id] = nd;
        return id;
    }
    int axis = 0;
    int64_t ext = (int64_t)nd.bmax[0] - nd.bmin[0];
    for (int a = 1; a < 3; a++) {
        int64_t e = (int64_t)nd.bmax[a] - nd.bmin[a];
        if (e > ext) { ext = e; axis = a; }
    }
    int64_t mid = lo + (hi - lo) / 2;
    nth_element(t->perm, lo, hi - 1, mid, t->P, axis);
    t->nodes[id] = nd;
    int64_t l = build_rec(t, lo, mid, id);
    if (l < 0) return -1;
    int64_t r = build_rec(t, mid, hi, id);
    if (r < 0) return -1;
    t->nodes[id].left = l;
    t->nodes[id].right = r;
    return id;
}

static void kd_free(kdtree_t *t) {
    free(t->perm); free(t->leaf_of); free(t->nodes);
    memset(t, 0, sizeof(*t));
}

static int kd_build(kdtree_t *t, const int32_t *P, int64_t n) {
    memset(t, 0, sizeof(*t));
    t->P = P; t->n = n;
    t->perm = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    t->leaf_of = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!t->perm || !t->leaf_of) { kd_free(t); return PDDO_ENOMEM; }
    for (int64_t i = 0; i < n; i++) t->perm[i] = i;
    if (build_rec(t, 0, n, -1) < 0) { kd_free(t); return PDDO_ENOMEM; }
    return PDDO_OK;
}

static void kd_remove(kdtree_t *t, int64_t j) {
    for (int64_t id = t->leaf_of[j]; id >= 0; id = t->nodes[id].parent) t->nodes[id].alive--;
}

static inline int64_t box_dist2(const kdtree_t *t, const node_t *nd, int64_t q) {
    int64_t s = 0;
    for (int a = 0; a < 3; a++) {
        int64_t c = coord(t->P, q, a), d = 0;
        if (c < nd->bmin[a]) d = nd->bmin[a] - c;
        else if (c > nd->bmax[a]) d = c - nd->bmax[a];
        s += d * d;
    }
    return s;
}

typedef struct { int64_t d2; int64_t idx; } ent_t;

static inline int ent_less(ent_t a, ent_t b) { return a.d2 < b.d2 || (a.d2 == b.d2 && a.idx < b.idx); }

/* Exact K nearest alive points of q (q excluded), sorted by (d2, index).
 * alive == NULL means every point is alive.  Returns the number found,
 * min(K, alive others). */
static int kd_knn(const kdtree_t *t, int64_t q, int K, const uint8_t *alive, ent_t *out) {
    int cnt = 0;
    int64_t stack[256];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const node_t *nd = &t->nodes[stack[--sp]];
        if (nd->alive == 0) continue;
        if (cnt == K && box_dist2(t, nd, q) > out[K - 1].d2) continue;
        if (nd->left < 0) {
            for (int64_t p = nd->lo; p < nd->hi; p++) {
                int64_t j = t->perm[p];
                if (j == q || (alive && !alive[j])) continue;
                ent_t e = { dist2(t->P, q, j), j };
                if (cnt == K && !ent_less(e, out[K - 1])) continue;
                int pos = (cnt < K) ? cnt++ : K - 1;
                while (pos > 0 && ent_less(e, out[pos - 1])) { out[pos] = out[pos - 1]; pos--; }
                out[pos] = e;
            }
        } else {
            const node_t *l = &t->nodes[nd->left], *r = &t->nodes[nd->right];
            int64_t dl = box_dist2(t, l, q), dr = box_dist2(t, r, q);
            /* push the farther child first so the nearer one is visited first */
            if (dl <= dr) { stack[sp++] = nd->right; stack[sp++] = nd->left; }
            else { stack[sp++] = nd->left; stack[sp++] = nd->right; }
        }
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* k-NN lists and initial costs                                              */
/* ------------------------------------------------------------------------ */

/* nbr [n*K]: original indices of the K nearest, sorted by (d2, index), -1
 * padded; d2 [n*K]: their squared distances (-1 padded). */
int pddo_knn(const int32_t *P, int64_t n, int32_t K, int32_t *nbr, int64_t *d2) {
    if (!P || n < 1 || K < 1 || K > MAX_K || !nbr) return PDDO_EINVAL;
    kdtree_t t;
    int rc = kd_build(&t, P, n);
    if (rc) return rc;
    ent_t buf[MAX_K];
    for (int64_t i = 0; i < n; i++) {
        int c = kd_knn(&t, i, K, NULL, buf);
        for (int j = 0; j < K; j++) {
            nbr[i * K + j] = j < c ? (int32_t)buf[j].idx : -1;
            if (d2) d2[i * K + j] = j < c ? buf[j].d2 : -1;
        }
    }
    kd_free(&t);
    return PDDO_OK;
}

/* Initial state of the method: the k+b lists, the k-th squared distance
 * r2k (of the min(k, n-1)-th neighbour) and the cost W of every point. */
int pddo_knn_cost(const int32_t *P, int64_t n, int32_t k, int32_t b, int32_t *nbr, int64_t *r2k,
                  uint64_t *cost) {
    if (!P || n < 2 || k < 1 || b < 0 || k + b > MAX_K || !cost) return PDDO_EINVAL;
    int K = k + b;
    kdtree_t t;
    int rc = kd_build(&t, P, n);
    if (rc) return rc;
    ent_t buf[MAX_K];
    for (int64_t i = 0; i < n; i++) {
        int c = kd_knn(&t, i, K, NULL, buf);
        uint64_t w = 0;
        int kk = c < k ? c : k;
        for (int j = 0; j < kk; j++) w += pddo_term(buf[j].d2);
        cost[i] = w;
        if (r2k) r2k[i] = buf[kk - 1].d2;
        if (nbr)
            for (int j = 0; j < K; j++) nbr[i * K + j] = j < c ? (int32_t)buf[j].idx : -1;
    }
    kd_free(&t);
    return PDDO_OK;
}

/* ------------------------------------------------------------------------ */
/* greedy decimation                                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    const int32_t *P;
    int64_t n;
    int k, K;
    kdtree_t tree;
    int64_t *buf;      /* [n*K] buffered neighbours (original indices) */
    int32_t *bcnt;     /* entries filled at the last search */
    uint64_t *W;       /* maintained cost */
    uint8_t *alive;
    /* reverse lists: linked nodes in a pool, never pruned (stale entries
     * only cause a harmless re-check) */
    int64_t *head;
    int64_t *pool_z, *pool_next;
    int64_t pool_n, pool_cap;
    /* indexed max-heap */
    int64_t *heap, *pos;
    int64_t hsize;
    int64_t researches;
} gstate_t;

/* key order: a ranks above b if its cost is larger, or equal with a smaller index */
static inline int above(const gstate_t *g, int64_t a, int64_t b) {
    return g->W[a] > g->W[b] || (g->W[a] == g->W[b] && a < b);
}

static void heap_swap(gstate_t *g, int64_t i, int64_t j) {
    int64_t a = g->heap[i], b = g->heap[j];
    g->heap[i] = b; g->heap[j] = a;
    g->pos[b] = i; g->pos[a] = j;
}

static void sift_down(gstate_t *g, int64_t i) {
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < g->hsize && above(g, g->heap[l], g->heap[m])) m = l;
        if (r < g->hsize && above(g, g->heap[r], g->heap[m])) m = r;
        if (m == i) return;
        heap_swap(g, i, m);
        i = m;
    }
}

static int64_t heap_pop(gstate_t *g) {
    int64_t top = g->heap[0];
    g->hsize--;
    if (g->hsize > 0) {
        g->heap[0] = g->heap[g->hsize];
        g->pos[g->heap[0]] = 0;
        sift_down(g, 0);
    }
    g->pos[top] = -1;
    return top;
}

static int rev_push(gstate_t *g, int64_t target, int64_t z) {
    if (g->pool_n == g->pool_cap) {
        int64_t nc = g->pool_cap * 2 + 1024;
        int64_t *a = (int64_t *)realloc(g->pool_z, (size_t)nc * sizeof(int64_t));
        if (!a) return PDDO_ENOMEM;
        g->pool_z = a;
        int64_t *b = (int64_t *)realloc(g->pool_next, (size_t)nc * sizeof(int64_t));
        if (!b) return PDDO_ENOMEM;
        g->pool_next = b;
        g->pool_cap = nc;
    }
    g->pool_z[g->pool_n] = z;
    g->pool_next[g->pool_n] = g->head[target];
    g->head[target] = g->pool_n++;
    return PDDO_OK;
}

/* search the buffer of z again over the alive points and register the
 * reverse edges of its new members */
static int research(gstate_t *g, int64_t z) {
    ent_t e[MAX_K];
    int c = kd_knn(&g->tree, z, g->K, g->alive, e);
    g->bcnt[z] = c;
    for (int j = 0; j < c; j++) {
        g->buf[z * g->K + j] = e[j].idx;
        int rc = rev_push(g, e[j].idx, z);
        if (rc) return rc;
    }
    g->researches++;
    return PDDO_OK;
}

/* W of z over the alive points, from its buffer (re-searching it if fewer
 * than k alive entries remain and the buffer did not hold every alive
 * point at its last search). */
static int current_cost(gstate_t *g, int64_t z, uint64_t *out) {
    for (int pass = 0; pass < 2; pass++) {
        uint64_t w = 0;
        int valid = 0;
        for (int j = 0; j < g->bcnt[z] && valid < g->k; j++) {
            int64_t y = g->buf[z * g->K + j];
            if (!g->alive[y]) continue;
            w += pddo_term(dist2(g->P, z, y));
            valid++;
        }
        if (valid == g->k || g->bcnt[z] < g->K || pass == 1) {
            *out = w;
            return PDDO_OK;
        }
        int rc = research(g, z);
        if (rc) return rc;
    }
    return PDDO_OK;
}

static void gfree(gstate_t *g) {
    kd_free(&g->tree);
    free(g->buf); free(g->bcnt); free(g->W); free(g->alive);
    free(g->head); free(g->pool_z); free(g->pool_next);
    free(g->heap); free(g->pos);
}

/*
 * kept [keep]        : indices of the remaining points, ascending
 * order [n-keep]     : removed indices in removal order (may be NULL)
 * order_cost [n-keep]: the cost each had when removed (may be NULL)
 * stats [4] (or NULL): researches, reverse-list nodes, -, -
 */
int pddo_decimate(const int32_t *P, int64_t n, int32_t k, int32_t b, int64_t keep, int32_t *kept,
                  int32_t *order, uint64_t *order_cost, int32_t check, int64_t *stats) {
    if (!P || n < 2 || k < 1 || b < 0 || k + b > MAX_K || keep < 1 || keep > n || !kept)
        return PDDO_EINVAL;
    gstate_t g;
    memset(&g, 0, sizeof(g));
    g.P = P; g.n = n; g.k = k; g.K = k + b;
    int rc = kd_build(&g.tree, P, n);
    if (rc) return rc;
    g.buf = (int64_t *)malloc((size_t)n * g.K * sizeof(int64_t));
    g.bcnt = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    g.W = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    g.alive = (uint8_t *)malloc((size_t)n);
    g.head = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    g.heap = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    g.pos = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!g.buf || !g.bcnt || !g.W || !g.alive || !g.head || !g.heap || !g.pos) { gfree(&g); return PDDO_ENOMEM; }
    memset(g.alive, 1, (size_t)n);
    for (int64_t i = 0; i < n; i++) g.head[i] = -1;

    ent_t e[MAX_K];
    for (int64_t i = 0; i < n; i++) {
        int c = kd_knn(&g.tree, i, g.K, NULL, e);
        g.bcnt[i] = c;
        for (int j = 0; j < c; j++) {
            g.buf[i * g.K + j] = e[j].idx;
            if ((rc = rev_push(&g, e[j].idx, i))) { gfree(&g); return rc; }
        }
    }
    for (int64_t i = 0; i < n; i++)
        if ((rc = current_cost(&g, i, &g.W[i]))) { gfree(&g); return rc; }
    g.hsize = n;
    for (int64_t i = 0; i < n; i++) { g.heap[i] = i; g.pos[i] = i; }
    for (int64_t i = n / 2 - 1; i >= 0; i--) sift_down(&g, i);

    int64_t removed = 0, target = n - keep;
    int64_t prev = -1;
    uint64_t prev_w = 0;
    /* stamp dedups the reverse-list walk of one removal */
    int64_t *stamp = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!stamp) { gfree(&g); return PDDO_ENOMEM; }
    for (int64_t i = 0; i < n; i++) stamp[i] = -1;

    while (removed < target) {
        int64_t x = heap_pop(&g);
        uint64_t wx = g.W[x];
        if (check && prev >= 0 && !(wx < prev_w || (wx == prev_w && x > prev))) {
            rc = PDDO_ECHECK_ORDER; goto out;
        }
        if (order) order[removed] = (int32_t)x;
        if (order_cost) order_cost[removed] = wx;
        prev = x; prev_w = wx;
        removed++;
        g.alive[x] = 0;
        kd_remove(&g.tree, x);
        for (int64_t p = g.head[x]; p >= 0; p = g.pool_next[p]) {
            int64_t z = g.pool_z[p];
            if (!g.alive[z] || stamp[z] == removed) continue;
            stamp[z] = removed;
            uint64_t w;
            if ((rc = current_cost(&g, z, &w))) goto out;
            if (check && w > g.W[z]) { rc = PDDO_ECHECK_RISE; goto out; }
            if (w != g.W[z]) {
                g.W[z] = w;
                sift_down(&g, g.pos[z]);
            }
        }
    }
    {
        int64_t c = 0;
        for (int64_t i = 0; i < n; i++)
            if (g.alive[i]) {
                if (c < keep) kept[c] = (int32_t)i;
                c++;
            }
        if (check && c != keep) { rc = PDDO_ECHECK_KEEP; goto out; }
    }
    if (check) {
        /* every maintained cost equals a fresh k-NN evaluation, and no kept
         * key ranks above the last removed key */
        for (int64_t i = 0; i < n; i++) {
            if (!g.alive[i]) continue;
            int c = kd_knn(&g.tree, i, k, g.alive, e);
            uint64_t w = 0;
            for (int j = 0; j < c; j++) w += pddo_term(e[j].d2);
            if (w != g.W[i]) { rc = PDDO_ECHECK_FINAL; goto out; }
            if (prev >= 0 && (w > prev_w || (w == prev_w && i < prev))) { rc = PDDO_ECHECK_NEXT; goto out; }
        }
    }
    if (stats) {
        stats[0] = g.researches;
        stats[1] = g.pool_n;
        stats[2] = 0;
        stats[3] = 0;
    }
    rc = PDDO_OK;
out:
    free(stamp);
    gfree(&g);
    return rc;
}
