/*
 * CPU oracle for exact betweenness with respect to a target set.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may link, load or call this
 * file: only the tests, the package's smoke check and the bench's CPU-baseline leg use
 * it. It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (Erdos, Ishakian, Bestavros, Terzi, "A Divide-and-Conquer
 * Algorithm for Betweenness Centrality"):
 *   - Sec. 3, eq. (parentsall): shortest-path distances d(s,.) and path counts
 *     sigma(s,v) = sum over tight parents u of sigma(s,u), found by one Dijkstra run
 *     (or BFS for unit weights) per source s.
 *   - Sec. 3, eq. (brandes): the target-set dependency
 *     delta(s|u) = sum over children v of sigma(s,u)/sigma(s,v) * (I[v in S] + delta(s|v)),
 *     summed in reverse order of distance from s.
 *   - Sec. 3, eq. (centrality): C(v) = sum over sources s in S of delta(s|v), v != s.
 *     This counts every unordered pair {s,t} twice; by default the result is halved to
 *     the unordered-pair score (flag ORACLE_ORDERED keeps the paper's ordered sum).
 *   - Sec. 4, eq. (frontierparents): Dijkstra_SK, the same search restricted to one
 *     part G_i = G[P_i] in which sigma only sums over tight parents that are not
 *     frontier nodes, the source itself excepted, with sigma(f,f) = 1.
 *
 * Integers: distances are int64; path counts are uint64 and every addition is checked:
 * a count that reaches 2^64 makes the call return ORACLE_OVERFLOW. Dependencies and
 * scores are IEEE double. Weights must be integers >= 1 (w == NULL means all 1).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_INVAL 1
#define ORACLE_OVERFLOW 2
#define ORACLE_NOMEM 3

#define ORACLE_ORDERED 1u

/* ---------------------------------------------------------------- binary heap -- */

typedef struct {
    int64_t key;
    int32_t node;
} heap_item;

typedef struct {
    heap_item* a;
    int64_t size;
    int64_t cap;
} heap;

static int heap_push(heap* h, int64_t key, int32_t node) {
    if (h->size == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        heap_item* na = (heap_item*)realloc(h->a, (size_t)nc * sizeof(heap_item));
        if (!na) return ORACLE_NOMEM;
        h->a = na;
        h->cap = nc;
    }
    int64_t i = h->size++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h->a[p].key <= key) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i].key = key;
    h->a[i].node = node;
    return ORACLE_OK;
}

static heap_item heap_pop(heap* h) {
    heap_item top = h->a[0];
    heap_item last = h->a[--h->size];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1;
        if (l >= h->size) break;
        int64_t c = l;
        if (l + 1 < h->size && h->a[l + 1].key < h->a[l].key) c = l + 1;
        if (h->a[c].key >= last.key) break;
        h->a[i] = h->a[c];
        i = c;
    }
    if (h->size > 0) h->a[i] = last;
    return top;
}

/* ------------------------------------------------------- single-source search -- */

/*
 * One search from s. Fills d (int64, -1 = unreachable), sigma (0 = unreachable) and
 * the settle order (nodes in nondecreasing distance; *nsettled entries).
 *
 * allowed(u): when `label` is non-NULL the search stays inside the part of s
 * (label[u] == label[s]) and a tight parent u adds sigma only if frontier[u] == 0 or
 * u == s (eq. frontierparents). With label == NULL it is the plain search of
 * eq. (parentsall).
 */
static int search(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w,
                  int32_t s, const int32_t* label, const uint8_t* frontier,
                  int64_t* d, uint64_t* sigma, int32_t* order, int32_t* nsettled,
                  heap* h, uint8_t* done) {
    for (int32_t v = 0; v < n; ++v) {
        d[v] = -1;
        sigma[v] = 0;
        done[v] = 0;
    }
    int32_t cnt = 0;
    d[s] = 0;
    sigma[s] = 1;
    if (w == NULL) {
        /* unit weights: breadth-first search; the queue is the settle order */
        int32_t head = 0;
        order[cnt++] = s;
        done[s] = 1;
        while (head < cnt) {
            int32_t u = order[head++];
            int parent_ok = (label == NULL) || frontier[u] == 0 || u == s;
            for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int32_t v = col[e];
                if (label != NULL && label[v] != label[s]) continue;
                if (d[v] < 0) {
                    d[v] = d[u] + 1;
                    order[cnt++] = v;
                }
                if (d[v] == d[u] + 1 && parent_ok) {
                    uint64_t t = sigma[v] + sigma[u];
                    if (t < sigma[v]) return ORACLE_OVERFLOW;
                    sigma[v] = t;
                }
            }
        }
    } else {
        /* Dijkstra with a binary heap and lazy deletion */
        h->size = 0;
        if (heap_push(h, 0, s)) return ORACLE_NOMEM;
        while (h->size > 0) {
            heap_item it = heap_pop(h);
            int32_t u = it.node;
            if (done[u] || it.key != d[u]) continue;
            done[u] = 1;
            order[cnt++] = u;
            /* sigma[u] is final here: its parents are strictly closer (w >= 1) */
            int parent_ok = (label == NULL) || frontier[u] == 0 || u == s;
            for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int32_t v = col[e];
                if (label != NULL && label[v] != label[s]) continue;
                int64_t nd = d[u] + (int64_t)w[e];
                if (d[v] < 0 || nd < d[v]) {
                    d[v] = nd;
                    sigma[v] = parent_ok ? sigma[u] : 0;
                    if (heap_push(h, nd, v)) return ORACLE_NOMEM;
                } else if (nd == d[v] && parent_ok) {
                    uint64_t t = sigma[v] + sigma[u];
                    if (t < sigma[v]) return ORACLE_OVERFLOW;
                    sigma[v] = t;
                }
            }
        }
    }
    *nsettled = cnt;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ public ---- */

int oracle_sssp(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w,
                int32_t s, int64_t* d, uint64_t* sigma) {
    if (n <= 0 || s < 0 || s >= n) return ORACLE_INVAL;
    int32_t* order = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    uint8_t* done = (uint8_t*)malloc((size_t)n);
    heap h = {0, 0, 0};
    int32_t cnt = 0;
    int rc = (order && done) ? search(n, row_ptr, col, w, s, NULL, NULL, d, sigma, order,
                                      &cnt, &h, done)
                             : ORACLE_NOMEM;
    free(order);
    free(done);
    free(h.a);
    return rc;
}

/* Dijkstra_SK from frontier node f inside its part (eq. frontierparents). */
int oracle_dijkstra_sk(int32_t n, const int64_t* row_ptr, const int32_t* col,
                       const int32_t* w, const int32_t* label, const uint8_t* frontier,
                       int32_t f, int64_t* d, uint64_t* sigma) {
    if (n <= 0 || f < 0 || f >= n || !label || !frontier) return ORACLE_INVAL;
    int32_t* order = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    uint8_t* done = (uint8_t*)malloc((size_t)n);
    heap h = {0, 0, 0};
    int32_t cnt = 0;
    int rc = (order && done) ? search(n, row_ptr, col, w, f, label, frontier, d, sigma,
                                      order, &cnt, &h, done)
                             : ORACLE_NOMEM;
    free(order);
    free(done);
    free(h.a);
    return rc;
}

/*
 * Target-set Brandes (Sec. 3, eqs. dep, brandes, centrality). Sources are taken in the
 * order given; S must hold distinct ids in [0, n). C_out gets n doubles.
 */
int oracle_bc(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w,
              int32_t nS, const int32_t* S, uint32_t flags, double* C_out) {
    if (n < 0 || nS < 0) return ORACLE_INVAL;
    for (int32_t v = 0; v < n; ++v) C_out[v] = 0.0;
    if (n == 0 || nS == 0) return ORACLE_OK;
    int64_t* d = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    uint64_t* sigma = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
    double* delta = (double*)malloc((size_t)n * sizeof(double));
    int32_t* order = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    uint8_t* done = (uint8_t*)malloc((size_t)n);
    uint8_t* in_s = (uint8_t*)calloc((size_t)n, 1);
    heap h = {0, 0, 0};
    int rc = ORACLE_OK;
    if (!d || !sigma || !delta || !order || !done || !in_s) {
        rc = ORACLE_NOMEM;
        goto out;
    }
    for (int32_t i = 0; i < nS; ++i) {
        if (S[i] < 0 || S[i] >= n || in_s[S[i]]) {
            rc = ORACLE_INVAL;
            goto out;
        }
        in_s[S[i]] = 1;
    }
    for (int32_t i = 0; i < nS; ++i) {
        int32_t s = S[i];
        int32_t cnt = 0;
        rc = search(n, row_ptr, col, w, s, NULL, NULL, d, sigma, order, &cnt, &h, done);
        if (rc) goto out;
        for (int32_t j = 0; j < cnt; ++j) delta[order[j]] = 0.0;
        /* reverse order of distance: every child is finished before its parent */
        for (int32_t j = cnt - 1; j >= 0; --j) {
            int32_t u = order[j];
            for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int32_t v = col[e];
                int64_t len = w ? (int64_t)w[e] : 1;
                if (d[v] >= 0 && d[v] == d[u] + len) {
                    delta[u] += (double)sigma[u] / (double)sigma[v] *
                                ((double)in_s[v] + delta[v]);
                }
            }
            if (u != s) C_out[u] += delta[u];
        }
    }
    if (!(flags & ORACLE_ORDERED)) {
        for (int32_t v = 0; v < n; ++v) C_out[v] *= 0.5;
    }
out:
    free(d);
    free(sigma);
    free(delta);
    free(order);
    free(done);
    free(in_s);
    free(h.a);
    return rc;
}
