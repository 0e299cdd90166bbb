/*
 * pald_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU evaluation of partitioned local depths
 * (PaLD) in double precision, written straight from the definitions of
 * Devarakonda & Ballard, "Sequential and Shared-Memory Parallel Algorithms for
 * Partitioned Local Depths" (arXiv 2307.16652):
 *
 *   local focus (Section 2, Background):
 *     U_xy = { z : d_xz <= d_xy  or  d_yz <= d_xy },   u_xy = |U_xy|
 *   cohesion by total probability (Section 3, Eq. (fxz)/(gxyz)):
 *     c_xz = 1/(n-1) * sum_{y != x} s(d_xz, d_yz) * [d_xz <= d_xy] / u_xy
 *   where the support s(p, q) = [p < q] + 1/2 [p == q] splits a tie between
 *   the two candidates (Section 5, the paragraph on ties), and y ranges over
 *   S \ {x} because the second point Y of Eq. (LD) is drawn from S \ {x}.
 *
 * Nothing here is blocked, fused or reordered beyond the definition: for each
 * row x and each second point y, one sweep over z counts the focus, and a
 * second sweep over z adds that focus's contributions to row x of C.  The
 * only parallelism is one thread per group of rows (rows are independent).
 *
 * This file shares no code with the GPU library; only tests, the smoke check
 * and the CPU-baseline leg of the benchmark load it.  Build with a plain C
 * compiler and NO fast-math flags (they would flush denormal distances to
 * zero and change comparison outcomes).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* One row x of U and C.  Urow[y] = u_xy for every y (y = x included: the
 * focus definition at y = x counts the points at distance 0 from x).
 * Crow[z] = c_xz in double precision. */
static void oracle_row(const float *D, int64_t n, int64_t ldd, int64_t x,
                       int32_t *Urow, double *Crow)
{
    const float *Dx = D + x * ldd;
    for (int64_t z = 0; z < n; ++z)
        Crow[z] = 0.0;

    for (int64_t y = 0; y < n; ++y) {
        const float *Dy = D + y * ldd;
        const double dxy = (double)Dx[y];

        /* u_xy = #{ z : d_xz <= d_xy or d_yz <= d_xy } */
        int64_t u = 0;
        for (int64_t z = 0; z < n; ++z) {
            const double dxz = (double)Dx[z];
            const double dyz = (double)Dy[z];
            if (dxz <= dxy || dyz <= dxy)
                ++u;
        }
        Urow[y] = (int32_t)u;

        if (y == x)          /* Y is drawn from S \ {x} */
            continue;

        /* g_xyz = s(d_xz, d_yz) * [d_xz <= d_xy] / u_xy */
        for (int64_t z = 0; z < n; ++z) {
            const double dxz = (double)Dx[z];
            const double dyz = (double)Dy[z];
            if (!(dxz <= dxy))
                continue;
            double s;
            if (dxz < dyz)
                s = 1.0;
            else if (dxz == dyz)
                s = 0.5;
            else
                s = 0.0;
            Crow[z] += s / (double)u;
        }
    }

    for (int64_t z = 0; z < n; ++z)
        Crow[z] /= (double)(n - 1);
}

typedef struct {
    const float *D;
    int64_t n, ldd;
    const int64_t *rows;
    int64_t nrows;
    int32_t *U;
    double *C;
    int tid, nthreads;
} oracle_job;

static void *oracle_worker(void *arg)
{
    oracle_job *j = (oracle_job *)arg;
    for (int64_t r = j->tid; r < j->nrows; r += j->nthreads)
        oracle_row(j->D, j->n, j->ldd, j->rows[r], j->U + r * j->n,
                   j->C + r * j->n);
    return NULL;
}

/*
 * Evaluate rows `rows[0..nrows)` of U and C.  D is row-major n x n with
 * leading dimension ldd (host memory).  U_rows and C_rows are nrows x n,
 * row r holding row rows[r].  nthreads <= 0 uses one thread.
 * Returns 0 on success, -1 on bad arguments or thread failure.
 */
int pald_oracle_rows(const float *D, int64_t n, int64_t ldd,
                     const int64_t *rows, int64_t nrows,
                     int32_t *U_rows, double *C_rows, int nthreads)
{
    if (!D || !rows || !U_rows || !C_rows || n < 2 || ldd < n || nrows < 0)
        return -1;
    for (int64_t r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= n)
            return -1;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > nrows)
        nthreads = nrows > 0 ? (int)nrows : 1;

    oracle_job *jobs = (oracle_job *)calloc((size_t)nthreads, sizeof(oracle_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return -1;
    }
    int rc = 0, started = 0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (oracle_job){D, n, ldd, rows, nrows, U_rows, C_rows, t, nthreads};
        if (pthread_create(&th[t], NULL, oracle_worker, &jobs[t]) != 0) {
            rc = -1;
            break;
        }
        ++started;
    }
    for (int t = 0; t < started; ++t)
        pthread_join(th[t], NULL);
    free(jobs);
    free(th);
    return rc;
}

/* All rows: U is n x n int32, C is n x n double (both row-major, ld = n). */
int pald_oracle_full(const float *D, int64_t n, int64_t ldd, int32_t *U,
                     double *C, int nthreads)
{
    if (n < 2)
        return -1;
    int64_t *rows = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!rows)
        return -1;
    for (int64_t i = 0; i < n; ++i)
        rows[i] = i;
    int rc = pald_oracle_rows(D, n, ldd, rows, n, U, C, nthreads);
    free(rows);
    return rc;
}
