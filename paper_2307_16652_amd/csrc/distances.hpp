// distances.hpp -- the distance front end: an exactly symmetric float32
// distance matrix with a zero diagonal from n points in R^dim (Section 6
// feeds PaLD Euclidean distances between embedding vectors).
//
// Every entry follows one definition: in float64, delta_k = p_xk - p_yk and
// acc = fma(delta_k, delta_k, acc) for k = 0, 1, ..., dim-1 in order, then
// D = fl32(acc) (squared Euclidean) or fl32(sqrt(acc)) (Euclidean).  Since
// fl(p_yk - p_xk) = -fl(p_xk - p_yk), one evaluation serves D[x][y] and
// D[y][x], and D[x][x] = 0.
//
// Work is the upper triangle of 64 x 64 (x, y) tiles; 256 threads, 4 x 4
// float64 accumulators each; the coordinates of both point blocks are staged
// through LDS as float64, 16 dimensions at a time.  A tile writes its block
// and, off the diagonal, the mirrored block.  For small dim the kernel is
// bound by the HBM write of D (4 n^2 bytes); for large dim by float64 VALU
// work (2 operations per pair and dimension).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pald {

constexpr int DIST_T = 64;   // tile edge (points)
constexpr int DIST_K = 16;   // dimensions per LDS stage
constexpr int DIST_THREADS = 256;

// k -> (bx, by), bx <= by, enumerating the upper triangle of tile pairs row
// by row of by: k = by (by + 1) / 2 + bx.
__device__ __forceinline__ void upper_tile_of(int32_t k, int32_t &bx, int32_t &by) {
    int32_t r = (int32_t)((sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
    if ((int64_t)r * (r + 1) / 2 > k) --r;
    if ((int64_t)(r + 1) * (r + 2) / 2 <= k) ++r;
    by = r;
    bx = k - (int32_t)((int64_t)r * (r + 1) / 2);
}

template <bool SQRT>
__device__ __forceinline__ float distance_of(double acc) {
    return SQRT ? (float)sqrt(acc) : (float)acc;
}

template <typename T, bool SQRT>
__global__ __launch_bounds__(DIST_THREADS) void distances_kernel(const T *__restrict__ P, int64_t n, int64_t dim,
                                                                 int64_t ldp, float *__restrict__ D, int64_t ldd,
                                                                 int vec, int32_t tile0) {
    __shared__ double xs[DIST_K][DIST_T];
    __shared__ double ys[DIST_K][DIST_T];
    int32_t bx, by;
    upper_tile_of(tile0 + (int32_t)blockIdx.x, bx, by);
    const int64_t x0 = (int64_t)bx * DIST_T, y0 = (int64_t)by * DIST_T;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;

    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

    for (int64_t k0 = 0; k0 < dim; k0 += DIST_K) {
        // stage coordinates k0 .. k0+15 of both blocks (rows past n read as 0, never stored)
#pragma unroll
        for (int e = threadIdx.x; e < DIST_T * DIST_K; e += DIST_THREADS) {
            const int r = e / DIST_K, k = e % DIST_K;
            const int64_t gk = k0 + k;
            double vx = 0.0, vy = 0.0;
            if (gk < dim) {
                if (x0 + r < n) vx = (double)P[(x0 + r) * ldp + gk];
                if (y0 + r < n) vy = (double)P[(y0 + r) * ldp + gk];
            }
            xs[k][r] = vx;
            ys[k][r] = vy;
        }
        __syncthreads();
        const int kend = (int)min<int64_t>(DIST_K, dim - k0);
        for (int k = 0; k < kend; ++k) {  // dimensions strictly in order
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = xs[k][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = ys[k][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const double d = a[i] - b[j];
                    acc[i][j] = __builtin_fma(d, d, acc[i][j]);
                }
        }
        __syncthreads();
    }

    float out[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) out[i][j] = distance_of<SQRT>(acc[i][j]);

    // D[x][y], x in this thread's 4 rows, y in its 4 columns
    const int64_t yb = y0 + tx * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t x = x0 + ty * 4 + i;
        if (x >= n) continue;
        float *dst = D + x * ldd + yb;
        if (vec && yb + 3 < n) {
            *reinterpret_cast<float4 *>(dst) = make_float4(out[i][0], out[i][1], out[i][2], out[i][3]);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (yb + j < n) dst[j] = out[i][j];
        }
    }
    if (bx == by) return;
    // the mirrored block D[y][x]
    const int64_t xb = x0 + ty * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t y = y0 + tx * 4 + j;
        if (y >= n) continue;
        float *dst = D + y * ldd + xb;
        if (vec && xb + 3 < n) {
            *reinterpret_cast<float4 *>(dst) = make_float4(out[0][j], out[1][j], out[2][j], out[3][j]);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (xb + i < n) dst[i] = out[i][j];
        }
    }
}

}  // namespace pald

// ---------------------------------------------------------------------------
// Graph front end: all-pairs shortest-path hop counts of an unweighted graph
// (the distance matrices of the appendix's collaboration-network runs).
//
// Multi-source breadth-first search, 64 sources per workgroup: every vertex
// v keeps 64-bit words visit[v] (sources that have reached v) and front[v]
// (sources that reached v in the last level).  A level sets, for every v,
//   next[v] = (OR over neighbours u of front[u]) & ~visit[v]
// -- the bottom-up step for all 64 searches at once -- and writes the level
// to D[s][v] for every source s whose bit is new.  The searches end when a
// level reaches nothing.  Vertices no source of the batch reaches get n
// (larger than any hop count, so it compares like +infinity); D[s][s] = 0.
// The level loop needs only workgroup barriers: each workgroup owns its 64
// rows of D and its three words per vertex in the workspace.
//
// Work per level is one pass over the edges; the 64 output rows are written
// once each, in coalesced stores (lanes hold consecutive v).
constexpr int BFS_THREADS = 1024;
constexpr int BFS_SOURCES = 64;

__global__ __launch_bounds__(BFS_THREADS) void graph_bfs_kernel(const int64_t *__restrict__ row_ptr,
                                                                const int32_t *__restrict__ col, int64_t nnz,
                                                                int64_t n, float *__restrict__ D, int64_t ldd,
                                                                uint64_t *__restrict__ ws, int64_t batch0) {
    const int64_t s0 = (batch0 + (int64_t)blockIdx.x) * BFS_SOURCES;
    const int nsrc = (int)min<int64_t>(BFS_SOURCES, n - s0);
    const uint64_t all = nsrc == 64 ? ~0ull : ((1ull << nsrc) - 1ull);
    uint64_t *visit = ws + (int64_t)blockIdx.x * 3 * n;
    uint64_t *cur = visit + n;
    uint64_t *nxt = cur + n;
    const int t = threadIdx.x;

    for (int64_t v = t; v < n; v += BFS_THREADS) {
        const uint64_t m = (v >= s0 && v < s0 + nsrc) ? (1ull << (v - s0)) : 0ull;
        visit[v] = m;
        cur[v] = m;
    }
    __syncthreads();

    for (int level = 1;; ++level) {
        int any = 0;
        for (int64_t v = t; v < n; v += BFS_THREADS) {
            const uint64_t vis = visit[v];
            uint64_t acc = 0;
            if (vis != all) {
                // the sources that have not reached v yet; once all of them are
                // found among the neighbours, the rest of the list adds nothing
                const uint64_t missing = all & ~vis;
                const int64_t e0 = min(max(row_ptr[v], (int64_t)0), nnz);
                const int64_t e1 = min(max(row_ptr[v + 1], e0), nnz);
                int64_t e = e0;
                for (; e + 8 <= e1 && (acc & missing) != missing; e += 8) {  // eight loads in flight
                    uint32_t u[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) u[k] = (uint32_t)col[e + k];
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        if (u[k] < (uint64_t)n) acc |= cur[u[k]];
                }
                for (; e < e1 && (acc & missing) != missing; ++e) {
                    const uint32_t u = (uint32_t)col[e];
                    if (u < (uint64_t)n) acc |= cur[u];
                }
                acc &= missing;
            }
            nxt[v] = acc;
            if (acc) {
                visit[v] = vis | acc;
                any = 1;
                const float lv = (float)level;
                for (int b = 0; b < nsrc; ++b)
                    if ((acc >> b) & 1ull) D[(s0 + b) * ldd + v] = lv;
            }
        }
        __syncthreads();  // this level's words are visible to the whole workgroup
        if (!__syncthreads_or(any)) break;
        uint64_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }

    // the diagonal, and every vertex a source never reached
    const float far = (float)n;
    for (int64_t v = t; v < n; v += BFS_THREADS) {
        const uint64_t vis = visit[v];
        for (int b = 0; b < nsrc; ++b) {
            if (s0 + b == v)
                D[(s0 + b) * ldd + v] = 0.0f;
            else if (!((vis >> b) & 1ull))
                D[(s0 + b) * ldd + v] = far;
        }
    }
}
