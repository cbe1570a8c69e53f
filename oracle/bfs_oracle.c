/*
 * CPU oracle for the masked sparse-matrix x sparse-vector BFS.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
 * CPU-baseline leg load this file's shared library.  It shares no code, header
 * or table with the GPU library and is built with plain gcc.
 *
 * Conventions (0-based; the paper labels vertices 1..n, Notation section):
 *   A(i,j) = 1 for an edge i -> j (rows are egress, directed-graph paragraph of
 *   the "Bounds on algebraic operations" section), so the search follows A^T:
 *   x_{k+1} = A^T[V_{k+1}, V_k] x_k.  out_ptr/out_idx is the CSR of A (row i
 *   lists the out-neighbours of i); in_ptr/in_idx is the CSC of A (column j
 *   lists the in-neighbours of j).
 *   level[v] = number of edges on a shortest path s -> v, -1 if unreached.
 *   parent[s] = s; parent[v] = min{u in N-(v) : level[u] = level[v]-1};
 *   parent[v] = -1 if unreached.
 *
 * Return codes: 0 ok, -1 bad arguments, -2 out of memory.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/*
 * O-A.  Textbook FIFO-queue BFS (Moore's algorithm, Background section) for the
 * levels, followed by a separate pass that applies the parent definition above
 * by scanning every in-neighbour of every reached vertex.
 */
int oracle_bfs_queue(int32_t n, const int32_t *out_ptr, const int32_t *out_idx,
                     const int32_t *in_ptr, const int32_t *in_idx, int32_t s,
                     int32_t *level, int32_t *parent)
{
    if (n <= 0 || s < 0 || s >= n || !out_ptr || !out_idx || !in_ptr || !in_idx ||
        !level || !parent)
        return -1;
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!queue) return -2;
    for (int32_t v = 0; v < n; ++v) { level[v] = -1; parent[v] = -1; }
    int64_t head = 0, tail = 0;
    queue[tail++] = s;
    level[s] = 0;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int64_t e = out_ptr[u]; e < out_ptr[u + 1]; ++e) {
            int32_t v = out_idx[e];
            if (level[v] < 0) {
                level[v] = level[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    parent[s] = s;
    for (int32_t v = 0; v < n; ++v) {
        if (level[v] <= 0) continue;
        int32_t best = -1;
        for (int64_t e = in_ptr[v]; e < in_ptr[v + 1]; ++e) {
            int32_t u = in_idx[e];
            if (level[u] == level[v] - 1 && (best < 0 || u < best)) best = u;
        }
        parent[v] = best;
    }
    return 0;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * O-B.  The CSR form of the method (Algorithm 2 and the text after it), with the
 * semiring kept explicit: the vector value of a frontier vertex j is x(j) = j+1
 * (vertex 0 must be a nonzero), "multiply" returns the vector operand (A is a
 * 0/1 pattern) and "add" is min over nonzeros.  The output vector y then holds
 * parent+1 for every vertex it reaches; before the next step each new frontier
 * entry is given its own index (+1) as its value.
 *
 * mode 0 - the algorithm as printed: the visited array T is updated as soon as
 *          a row entry is accepted (short-circuit, one nonzero per row, the
 *          n-1 bound of Thm 2).  Each level's frontier L[start, end) is sorted
 *          ascending first, so the first frontier vertex that reaches i is the
 *          smallest one and the result is the min-parent.
 * mode 1 - every unmasked entry contributes (the Lemma 1 form): the mask used
 *          during a step is the visited set as it stood when the step began
 *          (V_{k+1}), so every pair (j, i) with j in the frontier and i not yet
 *          visited is multiplied and min-reduced.  The frontier is walked in
 *          DESCENDING order to show the result does not depend on order.
 * mode 2 - the modification described in the text after Algorithm 2, literally:
 *          test T[j] before the row loop, drop the T update inside it, let L
 *          hold duplicates.  Only the counters are meaningful in this mode; the
 *          paper reports that it multiplies m nonzeros on a connected
 *          undirected graph.  level is filled from the step in which a
 *          vertex's row is first processed; parent is left -1 (source: s).
 *
 * counters (may be NULL), int64[4]:
 *   [0] multiplications performed (semiring products x(j) (x) A(i,j))
 *   [1] membership tests against the visited array
 *   [2] number of steps (levels with a nonempty frontier)
 *   [3] entries appended to L
 */
int oracle_bfs_alg2(int32_t n, const int32_t *out_ptr, const int32_t *out_idx,
                    int32_t s, int32_t mode, int32_t *level, int32_t *parent,
                    int64_t *counters)
{
    if (n <= 0 || s < 0 || s >= n || !out_ptr || !out_idx || !level || !parent ||
        mode < 0 || mode > 2)
        return -1;
    int64_t nnz = out_ptr[n];
    int64_t lcap = (mode == 2) ? nnz + 1 : (int64_t)n;
    int32_t *L = (int32_t *)malloc((size_t)(lcap > 0 ? lcap : 1) * sizeof(int32_t));
    int64_t *x = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int64_t *y = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    unsigned char *T = (unsigned char *)calloc((size_t)n, 1);
    if (!L || !x || !y || !T) {
        free(L); free(x); free(y); free(T);
        return -2;
    }
    int64_t mults = 0, tests = 0, steps = 0, appended = 1;
    for (int32_t v = 0; v < n; ++v) { level[v] = -1; parent[v] = -1; }

    /* Initialise x and L with the source; the source is visited from the start
       (Algorithm 1 removes supp(x_1) from V before the first step). */
    L[0] = s;
    x[s] = (int64_t)s + 1;
    level[s] = 0;
    parent[s] = s;
    if (mode != 2) T[s] = 1;
    int64_t start = 0, end = 1, z = 1;

    for (int32_t k = 0; start < end; ++k) {
        steps++;
        if (mode == 0) qsort(L + start, (size_t)(end - start), sizeof(int32_t), cmp_i32);
        if (mode == 1) {
            /* descending frontier order */
            qsort(L + start, (size_t)(end - start), sizeof(int32_t), cmp_i32);
            for (int64_t a = start, b = end - 1; a < b; ++a, --b) {
                int32_t t = L[a]; L[a] = L[b]; L[b] = t;
            }
        }
        for (int64_t p = start; p < end; ++p) {
            int32_t j = L[p];
            if (mode == 2) {
                if (T[j]) continue;          /* test before the row loop */
                if (level[j] < 0) level[j] = k;   /* first processing fixes the level */
            }
            for (int64_t e = out_ptr[j]; e < out_ptr[j + 1]; ++e) {
                int32_t i = out_idx[e];
                tests++;
                if (mode == 0) {
                    if (T[i] == 0) {
                        mults++;
                        int64_t prod = x[j];                 /* x(j) (x) A(i,j) */
                        if (y[i] == 0 || prod < y[i]) y[i] = prod;   /* (+) = min */
                        L[z++] = i;
                        T[i] = 1;
                    }
                } else if (mode == 1) {
                    /* V_{k+1} as it stood when the step began: level[] of this
                       step's discoveries is only written after the step */
                    if (level[i] < 0) {
                        mults++;
                        int64_t prod = x[j];
                        if (y[i] == 0) { L[z++] = i; T[i] = 1; }
                        if (y[i] == 0 || prod < y[i]) y[i] = prod;
                    }
                } else {
                    if (T[i] == 0) {
                        mults++;
                        if (z < lcap) L[z++] = i;
                    }
                }
            }
            T[j] = 1;
            if (mode != 2) x[j] = 0;
        }
        if (mode != 2) {
            /* the new frontier's values: level and parent from y; then each new
               frontier entry takes its own index as its value (x(i) = i+1) so
               the next product reports which frontier vertex reached a row */
            for (int64_t p = end; p < z; ++p) {
                int32_t i = L[p];
                level[i] = k + 1;
                parent[i] = (int32_t)(y[i] - 1);
                y[i] = (int64_t)i + 1;
            }
            /* exchange x and y: y becomes the input, the old x (all zero) the output */
            int64_t *t = x; x = y; y = t;
        }
        appended += z - end;
        start = end;
        end = z;
    }
    if (counters) {
        counters[0] = mults;
        counters[1] = tests;
        counters[2] = steps;
        counters[3] = appended;
    }
    free(L); free(x); free(y); free(T);
    return 0;
}

/*
 * Timing helper for the CPU baseline: runs O-A from each of `count` sources and
 * returns the total wall time in seconds (CLOCK_MONOTONIC).  Results of the last
 * source are left in level/parent.
 */
#include <time.h>
double oracle_time_queue_bfs(int32_t n, const int32_t *out_ptr, const int32_t *out_idx,
                             const int32_t *in_ptr, const int32_t *in_idx,
                             const int32_t *sources, int32_t count,
                             int32_t *level, int32_t *parent)
{
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (int32_t q = 0; q < count; ++q) {
        if (oracle_bfs_queue(n, out_ptr, out_idx, in_ptr, in_idx, sources[q], level, parent))
            return -1.0;
    }
    clock_gettime(CLOCK_MONOTONIC, &t1);
    return (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
}
