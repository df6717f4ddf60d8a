/*
 * Reference k-clique counter -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded C.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the product library
 * never calls it and shares no code, header or table with it.
 *
 * What it computes (Lonkar & Beamer, "Accelerating Clique Counting in Sparse
 * Real-World Graphs via Communication-Reducing Optimizations"):
 *
 *   count_k(G) = number of k-vertex subsets of V that are pairwise adjacent
 *   (Section II, definition of a clique).
 *
 * It reaches that number the way the paper's method does, written out
 * directly with no blocking or fusion:
 *
 *   1. Degree ordering (Section IV, Algorithm 3): u -> v is kept iff
 *      d(u) < d(v), or d(u) == d(v) and u < v, with d the undirected
 *      degree.  Out-lists keep the ascending id order of the input rows.
 *   2. Counting (Section III, Algorithm 2, with the subgraph build of
 *      Section V-B, Algorithm 5): the k-cliques are the sum over vertices u
 *      of the (k-1)-cliques of the subgraph induced on N->(u); a subgraph's
 *      vertex set is the sorted intersection of the parent's vertex set with
 *      an out-list; at the level with two vertices left only intersection
 *      sizes are summed (Section V-B, "Other Optimizations", second
 *      heuristic); a subgraph with fewer vertices than the clique it still
 *      has to hold is skipped when pruning is on (first heuristic, taken
 *      with the exact bound).
 *
 * Counts are uint64 and wrap; a flag records whether any addition carried,
 * which with non-negative addends happens iff the true total is >= 2^64.
 *
 * It also lists the k-cliques (oracle_list_dag) by the same recursion,
 * writing each clique out instead of counting it.
 *
 * Pinned, in the CPU test-suite, by: brute-force subset enumeration on small
 * graphs (counts, and the listed cliques as a set), closed forms (complete,
 * Turan, bipartite, wheel, disjoint-clique, Paley, Kneser and empty graphs),
 * the worked example of Fig. 1, trace(A^3)/6 computed by a sparse-matrix
 * library, and invariance under vertex relabelling.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_ENOMEM 2

/* ---------------------------------------------------------------- input */

/* Checks that (row_ptr, col) is a symmetric simple graph with sorted rows.
 * Symmetry is checked by binary search of u in the row of each neighbour. */
static int row_has(const int32_t* row_ptr, const int32_t* col, int32_t u, int32_t x)
{
    int64_t lo = row_ptr[u], hi = row_ptr[u + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo < row_ptr[u + 1] && col[lo] == x;
}

int oracle_check_csr(int32_t n, const int32_t* row_ptr, const int32_t* col)
{
    if (n < 0 || !row_ptr) return ORACLE_EINVAL;
    if (row_ptr[0] != 0) return ORACLE_EINVAL;
    for (int32_t u = 0; u < n; ++u) {
        if (row_ptr[u + 1] < row_ptr[u]) return ORACLE_EINVAL;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t v = col[e];
            if (v < 0 || v >= n || v == u) return ORACLE_EINVAL;
            if (e > row_ptr[u] && col[e - 1] >= v) return ORACLE_EINVAL;
            if (!row_has(row_ptr, col, v, u)) return ORACLE_EINVAL;
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------- ordering (Algorithm 3) */

/* omega(u) < omega(v): lower degree first, ties by lower id. */
static int before(const int32_t* row_ptr, int32_t u, int32_t v)
{
    int64_t du = row_ptr[u + 1] - row_ptr[u];
    int64_t dv = row_ptr[v + 1] - row_ptr[v];
    return du < dv || (du == dv && u < v);
}

/* dag_ptr: int32[n+1], dag_col: int32[m] with m = nnz / 2. */
int oracle_orient(int32_t n, const int32_t* row_ptr, const int32_t* col,
                  int32_t* dag_ptr, int32_t* dag_col)
{
    int32_t* cursor = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!cursor) return ORACLE_ENOMEM;
    /* first pass: out-degree of every vertex */
    dag_ptr[0] = 0;
    for (int32_t u = 0; u < n; ++u) {
        int32_t outdeg = 0;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
            if (before(row_ptr, u, col[e])) ++outdeg;
        dag_ptr[u + 1] = outdeg;
    }
    /* prefix sum */
    for (int32_t u = 0; u < n; ++u) dag_ptr[u + 1] += dag_ptr[u];
    /* second pass: place the kept neighbours, a private cursor per row */
    memcpy(cursor, dag_ptr, sizeof(int32_t) * (size_t)(n + 1));
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
            if (before(row_ptr, u, col[e])) dag_col[cursor[u]++] = col[e];
    free(cursor);
    return ORACLE_OK;
}

/* ----------------------------------------------- counting (Algorithm 2/5) */

typedef struct {
    const int32_t* dptr;     /* oriented graph */
    const int32_t* dcol;
    int prune;
    int overflow;
    uint64_t count;
    uint64_t* visits;        /* visits[j] = j-cliques met, j = 1..k (NULL ok) */
    int32_t** level_buf;     /* one candidate buffer per recursion level */
} count_ctx;

static void add_checked(count_ctx* c, uint64_t x)
{
    uint64_t r;
    if (__builtin_add_overflow(c->count, x, &r)) c->overflow = 1;
    c->count = r;
}

static void add_visits(count_ctx* c, int j, uint64_t x)
{
    if (c->visits) c->visits[j] += x;
}

/* Sorted-list intersection by a two-pointer merge; writes into out (may be
 * NULL to count only). */
static int64_t intersect(const int32_t* a, int64_t na, const int32_t* b, int64_t nb,
                         int32_t* out)
{
    int64_t i = 0, j = 0, s = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) ++i;
        else if (a[i] > b[j]) ++j;
        else {
            if (out) out[s] = a[i];
            ++s; ++i; ++j;
        }
    }
    return s;
}

/* Number of r-cliques of the oriented subgraph induced on the sorted vertex
 * set cand[0..s), where `have` vertices of the clique are already chosen
 * (used only for the per-size visit counts). */
static void cliques_in(count_ctx* c, const int32_t* cand, int64_t s, int r, int have)
{
    add_visits(c, have + 1, (uint64_t)s);
    if (r == 1) { add_checked(c, (uint64_t)s); return; }
    if (c->prune && s < r) return;
    if (r == 2) {
        /* penultimate level: degrees only, no adjacency is built */
        for (int64_t i = 0; i < s; ++i) {
            int32_t w = cand[i];
            int64_t d = intersect(c->dcol + c->dptr[w], c->dptr[w + 1] - c->dptr[w],
                                  cand, s, NULL);
            add_checked(c, (uint64_t)d);
            add_visits(c, have + 2, (uint64_t)d);
        }
        return;
    }
    int32_t* next = c->level_buf[r];
    for (int64_t i = 0; i < s; ++i) {
        int32_t w = cand[i];
        int64_t sn = intersect(c->dcol + c->dptr[w], c->dptr[w + 1] - c->dptr[w],
                               cand, s, next);
        cliques_in(c, next, sn, r - 1, have + 1);
    }
}

static int32_t max_outdeg_of(int32_t n, const int32_t* dptr)
{
    int32_t mx = 0;
    for (int32_t u = 0; u < n; ++u)
        if (dptr[u + 1] - dptr[u] > mx) mx = dptr[u + 1] - dptr[u];
    return mx;
}

static int ctx_init(count_ctx* c, int32_t n, const int32_t* dptr, const int32_t* dcol,
                    int k, int prune, uint64_t* visits)
{
    memset(c, 0, sizeof(*c));
    c->dptr = dptr;
    c->dcol = dcol;
    c->prune = prune;
    c->visits = visits;
    if (visits) memset(visits, 0, sizeof(uint64_t) * (size_t)(k + 1));
    c->level_buf = (int32_t**)calloc((size_t)k + 2, sizeof(int32_t*));
    if (!c->level_buf) return ORACLE_ENOMEM;
    int32_t mx = max_outdeg_of(n, dptr);
    for (int r = 0; r <= k + 1; ++r) {
        c->level_buf[r] = (int32_t*)malloc(sizeof(int32_t) * ((size_t)mx + 1));
        if (!c->level_buf[r]) return ORACLE_ENOMEM;
    }
    return ORACLE_OK;
}

static void ctx_free(count_ctx* c, int k)
{
    if (!c->level_buf) return;
    for (int r = 0; r <= k + 1; ++r) free(c->level_buf[r]);
    free(c->level_buf);
}

/* Count k-cliques of the oriented graph (dptr, dcol) rooted at the vertices
 * u = first, first+step, ... < last (all of V for 0, 1, n), added to a
 * starting value `base` (0 for a plain count; a base near 2^64 exercises the
 * overflow flag: the flag is set iff base + the count is >= 2^64, the
 * reading of the unstated counter width as uint64).  k >= 1.
 * visits: NULL or uint64[k+1]. */
int oracle_count_dag_from(int32_t n, const int32_t* dptr, const int32_t* dcol, int32_t k,
                          int32_t first, int32_t last, int32_t step, int32_t prune,
                          uint64_t base, uint64_t* count, int32_t* overflow, uint64_t* visits)
{
    if (k < 1 || step < 1 || first < 0 || last > n) return ORACLE_EINVAL;
    count_ctx c;
    if (ctx_init(&c, n, dptr, dcol, k, prune, visits) != ORACLE_OK) {
        ctx_free(&c, k);
        return ORACLE_ENOMEM;
    }
    c.count = base;
    for (int32_t u = first; u < last; u += step) {
        int64_t du = dptr[u + 1] - dptr[u];
        add_visits(&c, 1, 1);
        if (k == 1) { add_checked(&c, 1); continue; }
        cliques_in(&c, dcol + dptr[u], du, k - 1, 1);
    }
    *count = c.count;
    *overflow = c.overflow;
    ctx_free(&c, k);
    return ORACLE_OK;
}

/* The same, starting from 0. */
int oracle_count_dag(int32_t n, const int32_t* dptr, const int32_t* dcol, int32_t k,
                     int32_t first, int32_t last, int32_t step, int32_t prune,
                     uint64_t* count, int32_t* overflow, uint64_t* visits)
{
    return oracle_count_dag_from(n, dptr, dcol, k, first, last, step, prune, 0, count, overflow,
                                 visits);
}

/* Whole pipeline: orient, then count.  Visits as above. */
int oracle_count(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t k,
                 int32_t prune, uint64_t* count, int32_t* overflow, uint64_t* visits)
{
    if (k < 1) return ORACLE_EINVAL;
    int64_t m = (int64_t)row_ptr[n] / 2;
    int32_t* dptr = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t* dcol = (int32_t*)malloc(sizeof(int32_t) * ((size_t)m + 1));
    if (!dptr || !dcol) { free(dptr); free(dcol); return ORACLE_ENOMEM; }
    int st = oracle_orient(n, row_ptr, col, dptr, dcol);
    if (st == ORACLE_OK)
        st = oracle_count_dag(n, dptr, dcol, k, 0, n, 1, prune, count, overflow, visits);
    free(dptr);
    free(dcol);
    return st;
}

/* Edge-rooted counts: for each listed arc u -> v (which must be an arc of
 * the oriented graph), the number of k-cliques whose two omega-lowest
 * vertices are u and v, i.e. the (k-2)-cliques of the subgraph induced on
 * N->(u) cap N->(v).  k >= 2. */
int oracle_count_arcs(int32_t n, const int32_t* dptr, const int32_t* dcol, int32_t k,
                      const int32_t* arc_u, const int32_t* arc_v, int64_t narcs,
                      uint64_t* out, int32_t* overflow)
{
    if (k < 2) return ORACLE_EINVAL;
    count_ctx c;
    if (ctx_init(&c, n, dptr, dcol, k, 1, NULL) != ORACLE_OK) {
        ctx_free(&c, k);
        return ORACLE_ENOMEM;
    }
    int32_t* cand = c.level_buf[k + 1];
    int any_overflow = 0;
    for (int64_t i = 0; i < narcs; ++i) {
        int32_t u = arc_u[i], v = arc_v[i];
        c.count = 0;
        c.overflow = 0;
        if (k == 2) { out[i] = 1; continue; }
        int64_t s = intersect(dcol + dptr[u], dptr[u + 1] - dptr[u],
                              dcol + dptr[v], dptr[v + 1] - dptr[v], cand);
        cliques_in(&c, cand, s, k - 2, 2);
        out[i] = c.count;
        any_overflow |= c.overflow;
    }
    *overflow = any_overflow;
    ctx_free(&c, k);
    return ORACLE_OK;
}

/* Per-arc work statistics of the edge-rooted unit, over every arc:
 *   stats[0] = number of arcs (m)
 *   stats[1] = sum over arcs of d->(u) + d->(v)
 *   stats[2] = sum over arcs of s = |N->(u) cap N->(v)|   (= triangles)
 *   stats[3] = sum over arcs of sum_{w in C_uv} d->(w)
 *   stats[4] = max s
 *   stats[5] = number of arcs with s >= k - 2   (the arcs that survive pruning)
 *   stats[6] = sum over those arcs of d->(u) + d->(v)
 *   stats[7] = sum over those arcs of s
 *   stats[8] = sum over those arcs of sum_{w in C_uv} d->(w)
 *   stats[9] = max out-degree
 * hist (may be NULL): hist[b] = arcs with s in [2^(b-1), 2^b) for b >= 1,
 *   hist[0] = arcs with s = 0; 33 entries. */
int oracle_arc_stats(int32_t n, const int32_t* dptr, const int32_t* dcol, int32_t k,
                     uint64_t* stats, uint64_t* hist)
{
    memset(stats, 0, sizeof(uint64_t) * 10);
    if (hist) memset(hist, 0, sizeof(uint64_t) * 33);
    int32_t mx = max_outdeg_of(n, dptr);
    int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * ((size_t)mx + 1));
    if (!cand) return ORACLE_ENOMEM;
    stats[9] = (uint64_t)mx;
    for (int32_t u = 0; u < n; ++u) {
        for (int64_t e = dptr[u]; e < dptr[u + 1]; ++e) {
            int32_t v = dcol[e];
            uint64_t duv = (uint64_t)(dptr[u + 1] - dptr[u]) + (uint64_t)(dptr[v + 1] - dptr[v]);
            int64_t s = intersect(dcol + dptr[u], dptr[u + 1] - dptr[u],
                                  dcol + dptr[v], dptr[v + 1] - dptr[v], cand);
            uint64_t sumw = 0;
            for (int64_t i = 0; i < s; ++i)
                sumw += (uint64_t)(dptr[cand[i] + 1] - dptr[cand[i]]);
            stats[0] += 1;
            stats[1] += duv;
            stats[2] += (uint64_t)s;
            stats[3] += sumw;
            if ((uint64_t)s > stats[4]) stats[4] = (uint64_t)s;
            if (s >= k - 2) {
                stats[5] += 1;
                stats[6] += duv;
                stats[7] += (uint64_t)s;
                stats[8] += sumw;
            }
            if (hist) {
                int b = 0;
                while (b < 32 && ((int64_t)1 << b) <= s) ++b;
                hist[b] += 1;
            }
        }
    }
    free(cand);
    return ORACLE_OK;
}

/* ------------------------------------------- listing (Section VII note) */

/* k-clique listing: the same recursion as the count (Section III,
 * Algorithm 2, subgraphs by sorted intersection as in Algorithm 5), but
 * every clique is written out instead of counted, so no level is reduced
 * to intersection sizes.  The conclusion of the paper names listing as the
 * natural extension of the counting method.  A clique is written as its
 * vertices in increasing degree order (the order of the DAG's arcs), which
 * is a unique form per clique. */
typedef struct {
    const int32_t* dptr;
    const int32_t* dcol;
    int32_t k;
    int32_t* clique;         /* the vertices chosen so far */
    int32_t** level_buf;
    int32_t* out;            /* cap cliques of k vertices */
    uint64_t cap;
    uint64_t total;          /* cliques found, also beyond cap */
} list_ctx;

static void emit(list_ctx* c)
{
    if (c->total < c->cap)
        memcpy(c->out + c->total * (uint64_t)c->k, c->clique, sizeof(int32_t) * (size_t)c->k);
    c->total += 1;
}

/* cand[0..s): the out-neighbours shared by the `have` chosen vertices; r
 * more vertices to choose from them. */
static void list_in(list_ctx* c, const int32_t* cand, int64_t s, int r, int have)
{
    if (s < r) return;
    int32_t* next = c->level_buf[r];
    for (int64_t i = 0; i < s; ++i) {
        int32_t w = cand[i];
        c->clique[have] = w;
        if (r == 1) { emit(c); continue; }
        int64_t sn = intersect(c->dcol + c->dptr[w], c->dptr[w + 1] - c->dptr[w], cand, s, next);
        list_in(c, next, sn, r - 1, have + 1);
    }
}

static int list_init(list_ctx* c, int32_t n, const int32_t* dptr, const int32_t* dcol, int32_t k,
                     int32_t* out, uint64_t cap)
{
    memset(c, 0, sizeof(*c));
    c->dptr = dptr;
    c->dcol = dcol;
    c->k = k;
    c->out = out;
    c->cap = cap;
    c->clique = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
    /* one candidate buffer per level, plus one for an arc's C_uv */
    c->level_buf = (int32_t**)calloc((size_t)k + 2, sizeof(int32_t*));
    if (!c->clique || !c->level_buf) return ORACLE_ENOMEM;
    int32_t mx = max_outdeg_of(n, dptr);
    for (int r = 0; r <= k + 1; ++r) {
        c->level_buf[r] = (int32_t*)malloc(sizeof(int32_t) * ((size_t)mx + 1));
        if (!c->level_buf[r]) return ORACLE_ENOMEM;
    }
    return ORACLE_OK;
}

static void list_free(list_ctx* c)
{
    if (c->level_buf)
        for (int r = 0; r <= c->k + 1; ++r) free(c->level_buf[r]);
    free(c->level_buf);
    free(c->clique);
}

/* Lists the k-cliques rooted at u = first, first+step, ... < last of the
 * oriented graph (dptr, dcol): out receives min(total, cap) cliques of k
 * int32 each, in the order found; *total the number of cliques.  k >= 1. */
int oracle_list_dag(int32_t n, const int32_t* dptr, const int32_t* dcol, int32_t k,
                    int32_t first, int32_t last, int32_t step, int32_t* out, uint64_t cap,
                    uint64_t* total)
{
    if (k < 1 || step < 1 || first < 0 || last > n || (cap > 0 && !out)) return ORACLE_EINVAL;
    list_ctx c;
    int st = list_init(&c, n, dptr, dcol, k, out, cap);
    if (st == ORACLE_OK) {
        for (int32_t u = first; u < last; u += step) {
            c.clique[0] = u;
            if (k == 1) { emit(&c); continue; }
            list_in(&c, dcol + dptr[u], dptr[u + 1] - dptr[u], k - 1, 1);
        }
        *total = c.total;
    }
    list_free(&c);
    return st;
}

/* Edge-rooted listing: for each listed arc u -> v of the oriented graph, in
 * the order given, the k-cliques whose two lowest vertices are u and v
 * (u, v and a (k-2)-clique of the subgraph induced on N->(u) cap N->(v)).
 * per_arc[i] receives the number of cliques of arc i; out and *total as in
 * oracle_list_dag.  k >= 2. */
int oracle_list_arcs(int32_t n, const int32_t* dptr, const int32_t* dcol, int32_t k,
                     const int32_t* arc_u, const int32_t* arc_v, int64_t narcs,
                     uint64_t* per_arc, int32_t* out, uint64_t cap, uint64_t* total)
{
    if (k < 2 || narcs < 0 || (cap > 0 && !out)) return ORACLE_EINVAL;
    list_ctx c;
    int st = list_init(&c, n, dptr, dcol, k, out, cap);
    if (st == ORACLE_OK) {
        int32_t* cand = c.level_buf[k + 1];
        for (int64_t i = 0; i < narcs; ++i) {
            int32_t u = arc_u[i], v = arc_v[i];
            uint64_t before = c.total;
            c.clique[0] = u;
            c.clique[1] = v;
            if (k == 2) {
                emit(&c);
            } else {
                int64_t s = intersect(dcol + dptr[u], dptr[u + 1] - dptr[u],
                                      dcol + dptr[v], dptr[v + 1] - dptr[v], cand);
                list_in(&c, cand, s, k - 2, 2);
            }
            per_arc[i] = c.total - before;
        }
        *total = c.total;
    }
    list_free(&c);
    return st;
}

/* ----------------------------------- core ordering (Section III, Alg. 1) */

/* Core (degeneracy) ordering of Algorithm 1: repeatedly remove a vertex of
 * smallest current degree (ties: smallest id) and lower its neighbours'
 * degrees.  Reading of the algorithm's rank formula, which is garbled: the
 * vertex removed first gets the lowest rank (rank = removal position), and
 * arcs go from lower to higher rank, so each vertex points to the
 * neighbours still present when it is removed; the maximum out-degree is
 * then the degeneracy, the property the paper gives the ordering.  A binary
 * heap of (degree, id) entries with stale entries skipped on pop. */
typedef struct { int32_t deg, id; } heap_item;

static int item_less(heap_item a, heap_item b)
{
    return a.deg < b.deg || (a.deg == b.deg && a.id < b.id);
}

static void heap_push(heap_item* h, int64_t* size, heap_item x)
{
    int64_t i = (*size)++;
    h[i] = x;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!item_less(h[i], h[p])) break;
        heap_item t = h[i]; h[i] = h[p]; h[p] = t;
        i = p;
    }
}

static heap_item heap_pop(heap_item* h, int64_t* size)
{
    heap_item top = h[0];
    h[0] = h[--(*size)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < *size && item_less(h[l], h[s])) s = l;
        if (r < *size && item_less(h[r], h[s])) s = r;
        if (s == i) break;
        heap_item t = h[i]; h[i] = h[s]; h[s] = t;
        i = s;
    }
    return top;
}

/* rank[v] = position of v in the removal order (0 = removed first). */
int oracle_core_rank(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* rank)
{
    if (n < 0) return ORACLE_EINVAL;
    int64_t nnz = row_ptr[n];
    int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    heap_item* h = (heap_item*)malloc(sizeof(heap_item) * ((size_t)(n + nnz) + 1));
    if (!deg || !h) { free(deg); free(h); return ORACLE_ENOMEM; }
    int64_t size = 0;
    for (int32_t v = 0; v < n; ++v) {
        deg[v] = (int32_t)(row_ptr[v + 1] - row_ptr[v]);
        rank[v] = -1;
        heap_item x = {deg[v], v};
        heap_push(h, &size, x);
    }
    int32_t r = 0;
    while (size > 0) {
        heap_item x = heap_pop(h, &size);
        if (rank[x.id] >= 0 || x.deg != deg[x.id]) continue;   /* stale */
        rank[x.id] = r++;
        for (int64_t e = row_ptr[x.id]; e < row_ptr[x.id + 1]; ++e) {
            int32_t w = col[e];
            if (rank[w] >= 0) continue;
            deg[w] -= 1;
            heap_item y = {deg[w], w};
            heap_push(h, &size, y);
        }
    }
    free(deg);
    free(h);
    return ORACLE_OK;
}

/* The DAG of a rank: u -> v iff rank[u] < rank[v]; out-lists keep the
 * ascending id order of the input rows.  dag_ptr int32[n+1], dag_col
 * int32[m]. */
int oracle_orient_rank(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* rank,
                       int32_t* dag_ptr, int32_t* dag_col)
{
    if (n < 0) return ORACLE_EINVAL;
    dag_ptr[0] = 0;
    for (int32_t u = 0; u < n; ++u) {
        int32_t c = 0;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
            if (rank[u] < rank[col[e]]) dag_col[dag_ptr[u] + c++] = col[e];
        dag_ptr[u + 1] = dag_ptr[u] + c;
    }
    return ORACLE_OK;
}

/* --------------------------- level-synchronous core ordering (peeling) */

/* A parallel form of the core ordering: Algorithm 1 removes one vertex of
 * smallest current degree at a time, which the paper calls inherently
 * sequential; here every vertex whose current degree is at most a
 * threshold t leaves in the same round.  t starts at the smallest degree;
 * a round removes the set F = {present v : deg(v) <= t} at once and then
 * lowers the degrees of the neighbours still present; when F is empty, t
 * rises to the smallest degree still present.  round[v] receives the round
 * in which v left.  Ordering vertices by (round, id) and directing every
 * edge from the earlier to the later vertex bounds each out-degree by the
 * degree the vertex had when it left, which is at most t, and t never
 * exceeds the degeneracy: the largest out-degree is the degeneracy, as for
 * Algorithm 1.  Written as the plain sequence of rounds. */
int oracle_peel_rounds(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* round)
{
    if (n < 0) return ORACLE_EINVAL;
    int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t* frontier = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    if (!deg || !frontier) { free(deg); free(frontier); return ORACLE_ENOMEM; }
    int32_t remaining = n, t = 0, r = 0;
    for (int32_t v = 0; v < n; ++v) {
        deg[v] = (int32_t)(row_ptr[v + 1] - row_ptr[v]);
        round[v] = -1;
    }
    while (remaining > 0) {
        /* the vertices present with degree <= t */
        int32_t nf = 0;
        for (int32_t v = 0; v < n; ++v)
            if (round[v] < 0 && deg[v] <= t) frontier[nf++] = v;
        if (nf == 0) {
            /* raise t to the smallest degree present */
            int32_t mn = -1;
            for (int32_t v = 0; v < n; ++v)
                if (round[v] < 0 && (mn < 0 || deg[v] < mn)) mn = deg[v];
            t = mn;
            continue;
        }
        /* they leave together ... */
        for (int32_t i = 0; i < nf; ++i) round[frontier[i]] = r;
        /* ... and their neighbours still present lose one degree per edge */
        for (int32_t i = 0; i < nf; ++i) {
            int32_t v = frontier[i];
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
                if (round[col[e]] < 0) deg[col[e]] -= 1;
        }
        remaining -= nf;
        r += 1;
    }
    free(deg);
    free(frontier);
    return ORACLE_OK;
}
