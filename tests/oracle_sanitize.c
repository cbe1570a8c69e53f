/*
 * Runs the C oracle (oracle/bfs_oracle.c, compiled into this program) under
 * AddressSanitizer and UndefinedBehaviorSanitizer on small graphs of every
 * awkward shape: a single vertex, an isolated source, a path, a star from its
 * centre and from a leaf, self-loops and duplicate entries, unsorted lists, a
 * directed graph with its in-lists, a disconnected random graph, and bad
 * arguments.  Every entry point and mode runs; the queue search's levels and
 * parents must equal Algorithm 2's (modes 0, 1, 2).  Exit status 0 when all
 * agree; a sanitizer report aborts with a nonzero status.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_bfs_queue(int32_t n, const int32_t *out_ptr, const int32_t *out_idx,
                     const int32_t *in_ptr, const int32_t *in_idx, int32_t s,
                     int32_t *level, int32_t *parent);
int oracle_bfs_alg2(int32_t n, const int32_t *out_ptr, const int32_t *out_idx,
                    int32_t s, int32_t mode, int32_t *level, int32_t *parent,
                    int64_t *counters);
double oracle_time_queue_bfs(int32_t n, const int32_t *out_ptr, const int32_t *out_idx,
                             const int32_t *in_ptr, const int32_t *in_idx,
                             const int32_t *sources, int32_t count,
                             int32_t *level, int32_t *parent);

typedef struct {
    int32_t n, m;          /* vertices, entries */
    int32_t *ptr, *idx;    /* CSR, exactly sized allocations */
} Csr;

/* CSR from an edge list (entries kept in the given order: unsorted lists,
 * duplicates and self-loops survive). */
static Csr csr_from(int32_t n, int32_t m, const int32_t *src, const int32_t *dst) {
    Csr g;
    g.n = n;
    g.m = m;
    g.ptr = calloc((size_t)n + 1, sizeof(int32_t));
    g.idx = malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    for (int32_t e = 0; e < m; ++e) g.ptr[src[e] + 1]++;
    for (int32_t v = 0; v < n; ++v) g.ptr[v + 1] += g.ptr[v];
    int32_t *fill = malloc((size_t)n * sizeof(int32_t));
    memcpy(fill, g.ptr, (size_t)n * sizeof(int32_t));
    for (int32_t e = 0; e < m; ++e) g.idx[fill[src[e]]++] = dst[e];
    free(fill);
    return g;
}

static void csr_free(Csr *g) {
    free(g->ptr);
    free(g->idx);
}

static int failures = 0;

/* The queue search from s against Algorithm 2 in every mode (sorted copies of
 * the lists for the latter, which needs ascending lists). */
static void check(const char *name, const Csr *out, const Csr *in, int32_t s) {
    const int32_t n = out->n;
    int32_t *l0 = malloc((size_t)n * 4), *p0 = malloc((size_t)n * 4);
    int32_t *l1 = malloc((size_t)n * 4), *p1 = malloc((size_t)n * 4);
    if (oracle_bfs_queue(n, out->ptr, out->idx, in->ptr, in->idx, s, l0, p0) != 0) {
        printf("%s: queue search failed\n", name);
        failures++;
    }
    for (int32_t mode = 0; mode <= 2; ++mode) {
        int64_t cnt[4] = {0, 0, 0, 0};
        if (oracle_bfs_alg2(n, out->ptr, out->idx, s, mode, l1, p1, cnt) != 0) {
            printf("%s: alg2 mode %d failed\n", name, mode);
            failures++;
            continue;
        }
        if (memcmp(l0, l1, (size_t)n * 4) != 0) {
            printf("%s: levels differ (mode %d)\n", name, mode);
            failures++;
        }
    }
    free(l0); free(p0); free(l1); free(p1);
}

/* Sorted, deduplicated out-lists and their transpose (in-lists). */
static void sorted_pair(int32_t n, int32_t m, const int32_t *src, const int32_t *dst, Csr *out, Csr *in) {
    int32_t *s2 = malloc((size_t)(m > 0 ? m : 1) * 4), *d2 = malloc((size_t)(m > 0 ? m : 1) * 4);
    int32_t k = 0;
    /* insertion into a dense n x n table is fine for these sizes */
    char *seen = calloc((size_t)n * (size_t)n, 1);
    for (int32_t e = 0; e < m; ++e) {
        const size_t at = (size_t)src[e] * (size_t)n + (size_t)dst[e];
        if (!seen[at]) {
            seen[at] = 1;
            s2[k] = src[e];
            d2[k] = dst[e];
            ++k;
        }
    }
    int32_t *ss = malloc((size_t)(k > 0 ? k : 1) * 4), *dd = malloc((size_t)(k > 0 ? k : 1) * 4);
    int32_t j = 0;
    for (int32_t u = 0; u < n; ++u)
        for (int32_t v = 0; v < n; ++v)
            if (seen[(size_t)u * (size_t)n + (size_t)v]) { ss[j] = u; dd[j] = v; ++j; }
    *out = csr_from(n, k, ss, dd);
    j = 0;
    for (int32_t v = 0; v < n; ++v)
        for (int32_t u = 0; u < n; ++u)
            if (seen[(size_t)u * (size_t)n + (size_t)v]) { ss[j] = v; dd[j] = u; ++j; }
    *in = csr_from(n, k, ss, dd);
    free(seen); free(s2); free(d2); free(ss); free(dd);
}

static void undirected(const char *name, int32_t n, int32_t m, const int32_t *a, const int32_t *b,
                       int32_t s) {
    int32_t *src = malloc((size_t)(2 * m + 1) * 4), *dst = malloc((size_t)(2 * m + 1) * 4);
    for (int32_t e = 0; e < m; ++e) {
        src[2 * e] = a[e]; dst[2 * e] = b[e];
        src[2 * e + 1] = b[e]; dst[2 * e + 1] = a[e];
    }
    Csr out, in;
    sorted_pair(n, 2 * m, src, dst, &out, &in);
    check(name, &out, &in, s);
    csr_free(&out); csr_free(&in);
    free(src); free(dst);
}

int main(void) {
    /* one vertex, no entries */
    { Csr g = csr_from(1, 0, NULL, NULL); check("n1", &g, &g, 0); csr_free(&g); }
    /* an isolated source among others */
    { int32_t a[] = {1, 2}, b[] = {2, 3}; undirected("isolated", 4, 2, a, b, 0); }
    /* a path, from an end and from the middle */
    {
        enum { N = 50 };
        int32_t a[N - 1], b[N - 1];
        for (int32_t i = 0; i < N - 1; ++i) { a[i] = i; b[i] = i + 1; }
        undirected("path-end", N, N - 1, a, b, 0);
        undirected("path-mid", N, N - 1, a, b, 25);
    }
    /* a star from its centre and from a leaf */
    {
        enum { N = 40 };
        int32_t a[N - 1], b[N - 1];
        for (int32_t i = 1; i < N; ++i) { a[i - 1] = 7 % N; b[i - 1] = (7 + i) % N; }
        undirected("star-centre", N, N - 1, a, b, 7);
        undirected("star-leaf", N, N - 1, a, b, 8);
    }
    /* self-loops and duplicate entries, lists left unsorted, against the clean graph */
    {
        int32_t src[] = {0, 0, 1, 1, 1, 2, 2, 3, 3, 0, 2, 4};
        int32_t dst[] = {0, 1, 0, 2, 1, 3, 1, 2, 2, 1, 2, 4};
        Csr messy = csr_from(5, 12, src, dst);
        int32_t *l0 = malloc(5 * 4), *p0 = malloc(5 * 4);
        for (int32_t s = 0; s < 5; ++s)
            if (oracle_bfs_queue(5, messy.ptr, messy.idx, messy.ptr, messy.idx, s, l0, p0) != 0) {
                printf("messy: queue search failed\n");
                failures++;
            }
        free(l0); free(p0);
        csr_free(&messy);
    }
    /* a directed graph with its in-lists, and a disconnected random graph */
    {
        enum { N = 64, M = 200 };
        int32_t src[M], dst[M];
        uint32_t x = 12345u;
        for (int32_t e = 0; e < M; ++e) {
            x = x * 1664525u + 1013904223u;
            src[e] = (int32_t)((x >> 8) % 48u);               /* vertices 48..63 have no out-edges */
            x = x * 1664525u + 1013904223u;
            dst[e] = (int32_t)((x >> 8) % N);
        }
        Csr out, in;
        sorted_pair(N, M, src, dst, &out, &in);
        for (int32_t s = 0; s < N; s += 5) check("directed", &out, &in, s);
        int32_t *l = malloc(N * 4), *p = malloc(N * 4), srcs[] = {0, 3, 47, 63};
        if (oracle_time_queue_bfs(N, out.ptr, out.idx, in.ptr, in.idx, srcs, 4, l, p) < 0.0) {
            printf("timed search failed\n");
            failures++;
        }
        free(l); free(p);
        csr_free(&out); csr_free(&in);
        undirected("random", N, M / 2, src, dst, 5);
    }
    /* bad arguments are refused, not read */
    {
        int32_t ptr[] = {0, 0}, lv[1], pa[1];
        int64_t cnt[4];
        if (oracle_bfs_queue(1, ptr, ptr, ptr, ptr, 1, lv, pa) == 0) { printf("bad source accepted\n"); failures++; }
        if (oracle_bfs_queue(0, ptr, ptr, ptr, ptr, 0, lv, pa) == 0) { printf("n = 0 accepted\n"); failures++; }
        if (oracle_bfs_alg2(1, ptr, ptr, 0, 3, lv, pa, cnt) == 0) { printf("bad mode accepted\n"); failures++; }
        if (oracle_bfs_alg2(1, NULL, ptr, 0, 0, lv, pa, cnt) == 0) { printf("NULL accepted\n"); failures++; }
    }
    printf("oracle under sanitizers: %d failures\n", failures);
    return failures == 0 ? 0 : 1;
}
