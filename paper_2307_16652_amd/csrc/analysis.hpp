// analysis.hpp -- kernels that read a finished cohesion matrix C:
//
//  * local depths  l_x = sum_z c_xz   (Section 2: cohesion partitions the
//    local depth of Eq. (LD)); one float64 row sum per x, rounded once;
//  * the strong-tie graph: for every row x the columns z != x with
//    c_xz > threshold, in increasing z, as CSR (count, scan, fill).
//
// All three read C row by row in coalesced 16-byte segments; they are bound
// by HBM bandwidth.  Each row is handled by one workgroup of 256 threads in a
// fixed order, so results are deterministic.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pald {

constexpr int AN_THREADS = 256;
constexpr int AN_WAVES = AN_THREADS / 64;
constexpr int SCAN_THREADS = 1024;

// Sum of one double per thread over the workgroup, in a fixed order; the
// result is valid in thread 0.  `red` is AN_WAVES doubles of LDS.
__device__ __forceinline__ double block_sum_f64(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < AN_WAVES; ++w) s += red[w];
    }
    __syncthreads();
    return s;
}

__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t s = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < AN_WAVES; ++w) s += red[w];
    }
    __syncthreads();
    return s;
}

// Applies f(value, column) to every entry of row `row` (n columns) in a fixed
// per-thread order: 4 float4 segments in flight per thread when the row is
// 16-byte aligned (vec), else one float at a time.
template <typename F>
__device__ __forceinline__ void for_row(const float *__restrict__ row, int64_t n, bool vec, F &&f) {
    const int t = threadIdx.x;
    if (vec) {
        const float4 *r4 = reinterpret_cast<const float4 *>(row);
        const int64_t n4 = n >> 2;
        int64_t j = t;
        for (; j + 3 * AN_THREADS < n4; j += 4 * AN_THREADS) {
            float4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = r4[j + u * AN_THREADS];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t c = 4 * (j + u * AN_THREADS);
                f(v[u].x, c);
                f(v[u].y, c + 1);
                f(v[u].z, c + 2);
                f(v[u].w, c + 3);
            }
        }
        for (; j < n4; j += AN_THREADS) {
            const float4 v = r4[j];
            f(v.x, 4 * j);
            f(v.y, 4 * j + 1);
            f(v.z, 4 * j + 2);
            f(v.w, 4 * j + 3);
        }
        for (int64_t c = 4 * n4 + t; c < n; c += AN_THREADS) f(row[c], c);
    } else {
        for (int64_t c = t; c < n; c += AN_THREADS) f(row[c], c);
    }
}

// depth[x] = fl32( sum_z C[x][z] ), summed in float64.
__global__ __launch_bounds__(AN_THREADS) void local_depths_kernel(const float *__restrict__ C, int64_t n,
                                                                  int64_t ldc, float *__restrict__ depth,
                                                                  int vec) {
    __shared__ double red[AN_WAVES];
    for (int64_t x = blockIdx.x; x < n; x += gridDim.x) {
        double acc = 0.0;
        for_row(C + x * ldc, n, vec != 0, [&](float v, int64_t) { acc += (double)v; });
        const double s = block_sum_f64(acc, red);
        if (threadIdx.x == 0) depth[x] = (float)s;
    }
}

// row_ptr[x + 1] = #{ z != x : C[x][z] > t }.
__global__ __launch_bounds__(AN_THREADS) void ties_count_kernel(const float *__restrict__ C, int64_t n,
                                                                int64_t ldc, float t,
                                                                int64_t *__restrict__ row_ptr, int vec) {
    __shared__ int64_t red[AN_WAVES];
    for (int64_t x = blockIdx.x; x < n; x += gridDim.x) {
        int64_t cnt = 0;
        for_row(C + x * ldc, n, vec != 0, [&](float v, int64_t z) { cnt += (v > t && z != x) ? 1 : 0; });
        const int64_t s = block_sum_i64(cnt, red);
        if (threadIdx.x == 0) row_ptr[x + 1] = s;
    }
}

// One workgroup: turns the counts in row_ptr[1..n] into the CSR offsets
// (inclusive prefix sums) and sets row_ptr[0] = 0.
__global__ __launch_bounds__(SCAN_THREADS) void ties_scan_kernel(int64_t *__restrict__ row_ptr, int64_t n) {
    __shared__ int64_t part[SCAN_THREADS];
    const int t = threadIdx.x;
    const int64_t per = (n + SCAN_THREADS - 1) / SCAN_THREADS;
    const int64_t b = min(n, (int64_t)t * per), e = min(n, b + per);
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += row_ptr[1 + i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - s;
    for (int64_t i = b; i < e; ++i) {
        run += row_ptr[1 + i];
        row_ptr[1 + i] = run;
    }
    if (t == 0) row_ptr[0] = 0;
}

// col[row_ptr[x] + k] = the k-th column z != x (increasing) with C[x][z] > t,
// val[...] = C[x][z] (val may be null); entries at positions >= cap are not
// written.  256 columns per step: a wave ballot gives each selected lane its
// rank among the wave's, the per-wave totals (LDS) its wave's offset.
__global__ __launch_bounds__(AN_THREADS) void ties_fill_kernel(const float *__restrict__ C, int64_t n,
                                                               int64_t ldc, float t,
                                                               const int64_t *__restrict__ row_ptr,
                                                               int32_t *__restrict__ col, float *__restrict__ val,
                                                               int64_t cap) {
    __shared__ int wcount[2][AN_WAVES];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int parity = 0;
    for (int64_t x = blockIdx.x; x < n; x += gridDim.x) {
        int64_t base = row_ptr[x];
        const int64_t end = row_ptr[x + 1];
        const float *row = C + x * ldc;
        for (int64_t z0 = 0; z0 < n && base < end && base < cap; z0 += AN_THREADS) {
            const int64_t z = z0 + threadIdx.x;
            float v = 0.0f;
            bool p = false;
            if (z < n) {
                v = row[z];
                p = v > t && z != x;
            }
            const uint64_t m = __ballot(p);
            if (lane == 0) wcount[parity][w] = __popcll(m);
            __syncthreads();
            int off = 0, tot = 0;
#pragma unroll
            for (int k = 0; k < AN_WAVES; ++k) {
                const int c = wcount[parity][k];
                off += k < w ? c : 0;
                tot += c;
            }
            if (p) {
                const int64_t i = base + off + __popcll(m & below);
                if (i < cap) {
                    col[i] = (int32_t)z;
                    if (val) val[i] = v;
                }
            }
            base += tot;
            parity ^= 1;  // the next step writes the other slot: one barrier per step suffices
        }
    }
}

}  // namespace pald
