/*
 * distance_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * The distance front end in plain C: the distance matrix PaLD takes as input,
 * built from points (Section 6 applies PaLD to Euclidean distances between
 * word-embedding vectors).  The definition the library follows, entry by
 * entry:
 *
 *   acc = 0
 *   for k = 0, 1, ..., dim-1:   delta = p_xk - p_yk      (double precision)
 *                               acc   = fma(delta, delta, acc)
 *   D[x][y] = float(acc)            squared Euclidean
 *   D[x][y] = float(sqrt(acc))      Euclidean
 *
 * with float32 coordinates promoted exactly to double, every operation
 * rounded to nearest even, and the dimensions summed in index order.  Every
 * entry is computed on its own here (no mirroring): symmetry and the zero
 * diagonal are properties the tests check.  Compiled without contraction of
 * other multiply-adds and without fast-math.  Shares no code with the GPU
 * library.
 *
 * The second function below gives the graph version of the front end
 * (shortest-path hop counts), one plain breadth-first search per row.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

enum { ORACLE_METRIC_EUCLIDEAN = 0, ORACLE_METRIC_SQEUCLIDEAN = 1 };
enum { ORACLE_F32 = 0, ORACLE_F64 = 1 };

static double coord(const void *P, int dtype, int64_t ldp, int64_t i, int64_t k)
{
    if (dtype == ORACLE_F64)
        return ((const double *)P)[i * ldp + k];
    return (double)((const float *)P)[i * ldp + k];
}

/*
 * Rows rows[0..nrows) of D (rows == NULL: all n rows in order) into
 * D_rows[r * ldd + y], y < n.  P is n x dim row-major with leading dimension
 * ldp, float32 (dtype 0) or float64 (dtype 1), host memory.
 * Returns 0, or -1 on bad arguments.
 */
int pald_oracle_distances(const void *P, int dtype, int64_t n, int64_t dim,
                          int64_t ldp, int metric, const int64_t *rows,
                          int64_t nrows, float *D_rows, int64_t ldd)
{
    if (!P || !D_rows || n < 1 || dim < 1 || ldp < dim || ldd < n)
        return -1;
    if ((dtype != ORACLE_F32 && dtype != ORACLE_F64) ||
        (metric != ORACLE_METRIC_EUCLIDEAN && metric != ORACLE_METRIC_SQEUCLIDEAN))
        return -1;
    if (!rows)
        nrows = n;
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t x = rows ? rows[r] : r;
        if (x < 0 || x >= n)
            return -1;
        for (int64_t y = 0; y < n; ++y) {
            double acc = 0.0;
            for (int64_t k = 0; k < dim; ++k) {
                const double delta = coord(P, dtype, ldp, x, k) - coord(P, dtype, ldp, y, k);
                acc = fma(delta, delta, acc);
            }
            D_rows[r * ldd + y] = (float)(metric == ORACLE_METRIC_EUCLIDEAN ? sqrt(acc) : acc);
        }
    }
    return 0;
}

/*
 * Graph front end: all-pairs shortest-path (hop) distances of an unweighted
 * graph (the paper builds the distance matrices of its collaboration-network
 * experiments this way, appendix on SNAP datasets).  The graph is CSR on the
 * host: the neighbours of v are col[row_ptr[v] .. row_ptr[v+1]); neighbours
 * outside [0, n) are ignored.  One breadth-first search per source row:
 * D[s][v] = number of edges on a shortest path from s to v, D[s][s] = 0, and
 * n for a vertex that s cannot reach (larger than every hop distance, so it
 * compares like +infinity).  rows == NULL: all n rows in order.
 * Returns 0, or -1 on bad arguments or allocation failure.
 */
int pald_oracle_graph_distances(const int64_t *row_ptr, const int32_t *col, int64_t n,
                                const int64_t *rows, int64_t nrows, float *D_rows, int64_t ldd)
{
    if (!row_ptr || n < 1 || ldd < n)
        return -1;
    if (!rows)
        nrows = n;
    int64_t *dist = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!dist || !queue) {
        free(dist);
        free(queue);
        return -1;
    }
    int rc = 0;
    for (int64_t r = 0; r < nrows && rc == 0; ++r) {
        const int64_t s = rows ? rows[r] : r;
        if (s < 0 || s >= n) {
            rc = -1;
            break;
        }
        for (int64_t v = 0; v < n; ++v)
            dist[v] = -1;
        int64_t head = 0, tail = 0;
        dist[s] = 0;
        queue[tail++] = s;
        while (head < tail) {
            const int64_t u = queue[head++];
            for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                const int64_t w = col[e];
                if (w < 0 || w >= n || dist[w] >= 0)
                    continue;
                dist[w] = dist[u] + 1;
                queue[tail++] = w;
            }
        }
        for (int64_t v = 0; v < n; ++v)
            D_rows[r * ldd + v] = (float)(dist[v] >= 0 ? dist[v] : n);
    }
    free(dist);
    free(queue);
    return rc;
}
