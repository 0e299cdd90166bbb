// pairwise.hpp -- gfx950 kernels of the pairwise PaLD algorithm.
//
// Pass 1 (local focus sizes, Section 2 definition; the first z-loop of the
// pairwise algorithm in Section 3):
//     U_xy = #{ z : min(d_zx, d_zy) <= d_xy }
// Pass 2 (cohesion, Section 3 Eq. (fxz) with the Section 5 tie split):
//     C_xz = 1/(n-1) sum_{y != x} W_xy/2 * ( [t <= min(a,b)] + [t <= a and t < b] )
// with t = d_zx, a = d_xy, b = d_zy and W_xy = fl32(1/U_xy), W_xx = 0.  The
// bracket sum is 2 [z in U_xy] s(t, b): given t <= b, membership of z in the
// focus reduces to t <= a, and it counts 2 for t < b, 1 for a tie.
//
// GPU mapping (what replaces the paper's cache blocking):
//  * every workgroup owns an output tile -- (x,y) in pass 1, (x,z) in pass 2 --
//    and each thread keeps an RX x RY register sub-tile of accumulators plus
//    the stationary distances d_xy (pass 1) or d_xz (pass 2);
//  * the reduction index (z, resp. y) is streamed: KZ rows of D (and of W) are
//    staged through LDS per step with coalesced row loads; since D and W are
//    symmetric, the column segments the loops need are read as row segments;
//  * comparisons are made on "keys": the float bits with the sign bit
//    cleared, which order non-negative floats exactly like the floats
//    themselves (denormals included, -0 mapped to +0), so min/compare are
//    single full-rate integer instructions and no select on NaN handling is
//    needed;
//  * pass 1 uses the symmetry of U: only tiles with bx <= by run and they
//    write their transpose too;
//  * pass 2 accumulates float32 runs of 8 terms, folds each run into a Kahan
//    (sum, compensation) pair, and reduces the pair in float64 at the end.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pald {

constexpr uint32_t KEY_INF = 0x7f800000u;  // key of +infinity: larger than every finite key

__device__ __forceinline__ uint32_t key_of(float d) { return __float_as_uint(d) & 0x7fffffffu; }

__device__ __forceinline__ uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Upper-triangular tile enumeration: k -> (bx, by) with bx <= by, by-major.
__device__ __forceinline__ void tri_tile(int32_t k, int32_t &bx, int32_t &by) {
    int32_t r = (int32_t)((sqrtf(8.0f * (float)k + 1.0f) - 1.0f) * 0.5f);
    while ((int64_t)r * (r + 1) / 2 > k) --r;
    while ((int64_t)(r + 1) * (r + 2) / 2 <= k) ++r;
    by = r;
    bx = k - (int32_t)((int64_t)r * (r + 1) / 2);
}

// Loads 4 consecutive floats of row `row` starting at column `col` of a
// row-major matrix as keys; out-of-range rows/columns give `fill`.
__device__ __forceinline__ uint4 load_keys4(const float *__restrict__ M, int64_t ld, int64_t row,
                                            int64_t col, int64_t nrows, int64_t ncols, bool vec_ok,
                                            uint32_t fill) {
    uint4 r = make_uint4(fill, fill, fill, fill);
    if (row >= nrows) return r;
    const float *p = M + row * ld + col;
    if (vec_ok && col + 3 < ncols) {
        float4 v = *reinterpret_cast<const float4 *>(p);
        r.x = key_of(v.x); r.y = key_of(v.y); r.z = key_of(v.z); r.w = key_of(v.w);
    } else {
        if (col + 0 < ncols) r.x = key_of(p[0]);
        if (col + 1 < ncols) r.y = key_of(p[1]);
        if (col + 2 < ncols) r.z = key_of(p[2]);
        if (col + 3 < ncols) r.w = key_of(p[3]);
    }
    return r;
}

// Same for plain float values (the weights W); out of range gives 0.
__device__ __forceinline__ uint4 load_vals4(const float *__restrict__ M, int64_t ld, int64_t row,
                                            int64_t col, int64_t nrows, int64_t ncols, bool vec_ok) {
    uint4 r = make_uint4(0u, 0u, 0u, 0u);
    if (row >= nrows) return r;
    const float *p = M + row * ld + col;
    if (vec_ok && col + 3 < ncols) {
        float4 v = *reinterpret_cast<const float4 *>(p);
        r.x = __float_as_uint(v.x); r.y = __float_as_uint(v.y);
        r.z = __float_as_uint(v.z); r.w = __float_as_uint(v.w);
    } else {
        if (col + 0 < ncols) r.x = __float_as_uint(p[0]);
        if (col + 1 < ncols) r.y = __float_as_uint(p[1]);
        if (col + 2 < ncols) r.z = __float_as_uint(p[2]);
        if (col + 3 < ncols) r.w = __float_as_uint(p[3]);
    }
    return r;
}

// fl32(1 / u): the division is done in float64 and rounded once to float32,
// which equals the correctly rounded float32 quotient for integer u.
__device__ __forceinline__ float weight_of(int32_t u) { return (float)(1.0 / (double)u); }

// ---------------------------------------------------------------------------
// Pass 1: focus sizes.
//
// Grid: blockIdx.x enumerates the upper-triangular tiles (bx <= by) of T x T
// tiles; blockIdx.y is the z-chunk.  With one z-chunk the tile writes U (and,
// if W != nullptr, the weights W) directly; with several it atomically adds
// its counts into U, which must be zero on entry.

template <int T, int RX, int RY, int KZ>
struct Pass1Cfg {
    static constexpr int TX = T / RX;  // threads along x
    static constexpr int TY = T / RY;  // threads along y
    static constexpr int NT = TX * TY;
    static constexpr int ROW = 2 * T;                 // keys per staged z row
    static constexpr int VEC_PER_CHUNK = KZ * ROW / 4; // uint4 per staged chunk
    static constexpr int VEC_PER_THREAD = VEC_PER_CHUNK / NT;
    static_assert(VEC_PER_CHUNK % NT == 0, "chunk must split evenly over threads");
    static_assert(T % 4 == 0, "tile must be a multiple of 4");
};

template <int T, int RX, int RY, int KZ>
__global__ __launch_bounds__((Pass1Cfg<T, RX, RY, KZ>::NT)) void pass1_focus_kernel(
    const float *__restrict__ D, int64_t n, int64_t ldd, int32_t *__restrict__ U, int64_t ldu,
    float *__restrict__ W, int64_t ldw, int32_t z_per_chunk, int32_t atomic_mode, int32_t vec_ok) {
    using Cfg = Pass1Cfg<T, RX, RY, KZ>;
    __shared__ uint4 sm[2][Cfg::VEC_PER_CHUNK];

    int32_t bx, by;
    tri_tile((int32_t)blockIdx.x, bx, by);
    const int64_t X0 = (int64_t)bx * T, Y0 = (int64_t)by * T;
    const int tid = threadIdx.x;
    const int tx = tid % Cfg::TX, ty = tid / Cfg::TX;
    const int64_t zbeg = (int64_t)blockIdx.y * z_per_chunk;
    const int64_t zend = min(n, zbeg + (int64_t)z_per_chunk);

    // stationary keys a_ij = d_xy
    uint32_t a[RX][RY];
    int32_t cnt[RX][RY];
#pragma unroll
    for (int i = 0; i < RX; ++i) {
        const int64_t x = X0 + tx * RX + i;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int64_t y = Y0 + ty * RY + j;
            a[i][j] = (x < n && y < n) ? key_of(D[x * ldd + y]) : 0u;
            cnt[i][j] = 0;
        }
    }

    // staging: chunk element v (uint4) = row v / (ROW/4), column group v % (ROW/4);
    // the first T/4 groups are D[z][X0..], the rest D[z][Y0..].
    uint4 pre[Cfg::VEC_PER_THREAD];
    auto fetch = [&](int64_t zc) {
#pragma unroll
        for (int k = 0; k < Cfg::VEC_PER_THREAD; ++k) {
            const int v = tid + k * Cfg::NT;
            const int r = v / (Cfg::ROW / 4);
            const int g = v % (Cfg::ROW / 4);
            const int64_t z = zc + r;
            const int64_t col = (g < T / 4) ? X0 + 4 * g : Y0 + 4 * (g - T / 4);
            pre[k] = load_keys4(D, ldd, z, col, zend, n, vec_ok != 0, KEY_INF);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int k = 0; k < Cfg::VEC_PER_THREAD; ++k) sm[buf][tid + k * Cfg::NT] = pre[k];
    };

    const int64_t nz = zend - zbeg;
    const int64_t nchunks = (nz + KZ - 1) / KZ;
    if (nchunks > 0) {
        fetch(zbeg);
        stash(0);
    }
    __syncthreads();

    for (int64_t c = 0; c < nchunks; ++c) {
        const int buf = (int)(c & 1);
        if (c + 1 < nchunks) fetch(zbeg + (c + 1) * KZ);
        const uint32_t *s = reinterpret_cast<const uint32_t *>(sm[buf]);
#pragma unroll 1
        for (int z = 0; z < KZ; ++z) {
            uint32_t xs[RX], ys[RY];
#pragma unroll
            for (int i = 0; i < RX; ++i) xs[i] = s[z * Cfg::ROW + tx * RX + i];
#pragma unroll
            for (int j = 0; j < RY; ++j) ys[j] = s[z * Cfg::ROW + T + ty * RY + j];
#pragma unroll
            for (int i = 0; i < RX; ++i)
#pragma unroll
                for (int j = 0; j < RY; ++j) cnt[i][j] += (umin(xs[i], ys[j]) <= a[i][j]) ? 1 : 0;
        }
        if (c + 1 < nchunks) stash(buf ^ 1);
        __syncthreads();
    }

    // epilogue
    const bool mirror = bx != by;
#pragma unroll
    for (int i = 0; i < RX; ++i) {
        const int64_t x = X0 + tx * RX + i;
        if (x >= n) continue;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int64_t y = Y0 + ty * RY + j;
            if (y >= n) continue;
            if (atomic_mode) {
                atomicAdd(&U[x * ldu + y], cnt[i][j]);
                if (mirror) atomicAdd(&U[y * ldu + x], cnt[i][j]);
            } else {
                if (U) {
                    U[x * ldu + y] = cnt[i][j];
                    if (mirror) U[y * ldu + x] = cnt[i][j];
                }
                if (W) {
                    const float w = (x == y) ? 0.0f : weight_of(cnt[i][j]);
                    W[x * ldw + y] = w;
                    if (mirror) W[y * ldw + x] = w;
                }
            }
        }
    }
}

// W_xy = fl32(1/U_xy) off the diagonal, 0 on it (used after a split pass 1).
__global__ void weights_kernel(const int32_t *__restrict__ U, int64_t ldu, float *__restrict__ W,
                               int64_t ldw, int64_t n) {
    for (int64_t x = blockIdx.y; x < n; x += gridDim.y)
        for (int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; y < n;
             y += (int64_t)gridDim.x * blockDim.x)
            W[x * ldw + y] = (x == y) ? 0.0f : weight_of(U[x * ldu + y]);
}

// Fills an int32 n x n block with zeros (a kernel, so that it can sit inside a
// captured graph).
__global__ void zero_i32_kernel(int32_t *__restrict__ P, int64_t ld, int64_t n) {
    for (int64_t x = blockIdx.y; x < n; x += gridDim.y)
        for (int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; y < n;
             y += (int64_t)gridDim.x * blockDim.x)
            P[x * ld + y] = 0;
}

// ---------------------------------------------------------------------------
// Pass 2: cohesion.
//
// Grid: blockIdx.x = bx + nbx * bz over (x,z) tiles of TXx x TZ; blockIdx.y is
// the y-chunk.  With one y-chunk the tile writes C = fl32(sum / (n-1))
// directly; otherwise it writes its float64 partial sum to
// partial[chunk][x][z] (ld n) for finalize_kernel.
//
// Per y the tile needs row y of D restricted to the x and z ranges (a = d_yx,
// b = d_yz; D symmetric) and row y of W restricted to x (W_yx = W_xy).
// Rows y >= n, and rows past the chunk, stage W = 0 and so add nothing; the
// term y = x adds nothing because W_xx = 0.

template <int TXx, int TZ, int RX, int RZ, int KY>
struct Pass2Cfg {
    static constexpr int TX = TXx / RX;
    static constexpr int TZt = TZ / RZ;
    static constexpr int NT = TX * TZt;
    static constexpr int ROW = 2 * TXx + TZ;            // a keys | W values | b keys
    static constexpr int VEC_PER_CHUNK = KY * ROW / 4;
    static constexpr int VEC_PER_THREAD = VEC_PER_CHUNK / NT;
    static constexpr int RUN = 8;                       // float32 run length before a Kahan fold
    static_assert(VEC_PER_CHUNK % NT == 0, "chunk must split evenly over threads");
    static_assert(KY % RUN == 0, "KY must be a multiple of the run length");
    static_assert(TXx % 4 == 0 && TZ % 4 == 0, "tile sides must be multiples of 4");
};

template <int TXx, int TZ, int RX, int RZ, int KY, bool F64>
__global__ __launch_bounds__((Pass2Cfg<TXx, TZ, RX, RZ, KY>::NT)) void pass2_cohesion_kernel(
    const float *__restrict__ D, int64_t n, int64_t ldd, const float *__restrict__ W, int64_t ldw,
    float *__restrict__ C, int64_t ldc, double *__restrict__ partial, int32_t nbx,
    int32_t y_per_chunk, int32_t vec_ok_d, int32_t vec_ok_w) {
    using Cfg = Pass2Cfg<TXx, TZ, RX, RZ, KY>;
    __shared__ uint4 sm[2][Cfg::VEC_PER_CHUNK];

    const int32_t bx = (int32_t)blockIdx.x % nbx, bz = (int32_t)blockIdx.x / nbx;
    const int64_t X0 = (int64_t)bx * TXx, Z0 = (int64_t)bz * TZ;
    const int tid = threadIdx.x;
    const int tx = tid % Cfg::TX, tz = tid / Cfg::TX;
    const int64_t ybeg = (int64_t)blockIdx.y * y_per_chunk;
    const int64_t yend = min(n, ybeg + (int64_t)y_per_chunk);

    // stationary keys t_ij = d_xz
    uint32_t t[RX][RZ];
#pragma unroll
    for (int i = 0; i < RX; ++i) {
        const int64_t x = X0 + tx * RX + i;
#pragma unroll
        for (int j = 0; j < RZ; ++j) {
            const int64_t z = Z0 + tz * RZ + j;
            t[i][j] = (x < n && z < n) ? key_of(D[x * ldd + z]) : 0u;
        }
    }

    float sum[RX][RZ], comp[RX][RZ], run[RX][RZ];
    double acc[RX][RZ];
#pragma unroll
    for (int i = 0; i < RX; ++i)
#pragma unroll
        for (int j = 0; j < RZ; ++j) {
            sum[i][j] = 0.0f;
            comp[i][j] = 0.0f;
            run[i][j] = 0.0f;
            acc[i][j] = 0.0;
        }

    uint4 pre[Cfg::VEC_PER_THREAD];
    auto fetch = [&](int64_t yc) {
#pragma unroll
        for (int k = 0; k < Cfg::VEC_PER_THREAD; ++k) {
            const int v = tid + k * Cfg::NT;
            const int r = v / (Cfg::ROW / 4);
            const int g = v % (Cfg::ROW / 4);
            const int64_t y = yc + r;
            if (g < TXx / 4) {
                pre[k] = load_keys4(D, ldd, y, X0 + 4 * g, yend, n, vec_ok_d != 0, 0u);
            } else if (g < TXx / 2) {
                pre[k] = load_vals4(W, ldw, y, X0 + 4 * (g - TXx / 4), yend, n, vec_ok_w != 0);
            } else {
                pre[k] = load_keys4(D, ldd, y, Z0 + 4 * (g - TXx / 2), yend, n, vec_ok_d != 0, 0u);
            }
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int k = 0; k < Cfg::VEC_PER_THREAD; ++k) sm[buf][tid + k * Cfg::NT] = pre[k];
    };

    const int64_t ny = yend - ybeg;
    const int64_t nchunks = ny > 0 ? (ny + KY - 1) / KY : 0;
    if (nchunks > 0) {
        fetch(ybeg);
        stash(0);
    }
    __syncthreads();

    for (int64_t c = 0; c < nchunks; ++c) {
        const int buf = (int)(c & 1);
        if (c + 1 < nchunks) fetch(ybeg + (c + 1) * KY);
        const uint32_t *s = reinterpret_cast<const uint32_t *>(sm[buf]);
#pragma unroll 1
        for (int y0 = 0; y0 < KY; y0 += Cfg::RUN) {
#pragma unroll
            for (int yy = 0; yy < Cfg::RUN; ++yy) {
                const uint32_t *row = s + (y0 + yy) * Cfg::ROW;
                uint32_t av[RX], bv[RZ];
                float w[RX], wh[RX];
#pragma unroll
                for (int i = 0; i < RX; ++i) {
                    av[i] = row[tx * RX + i];
                    w[i] = __uint_as_float(row[TXx + tx * RX + i]);
                    wh[i] = 0.5f * w[i];
                }
#pragma unroll
                for (int j = 0; j < RZ; ++j) bv[j] = row[2 * TXx + tz * RZ + j];
#pragma unroll
                for (int i = 0; i < RX; ++i)
#pragma unroll
                    for (int j = 0; j < RZ; ++j) {
                        const uint32_t tt = t[i][j];
                        const uint32_t m = umin(av[i], bv[j]);
                        const float v = (tt < bv[j]) ? w[i] : wh[i];
                        const float term = (tt <= m) ? v : 0.0f;
                        if (F64) {
                            acc[i][j] += (double)term;
                        } else if (yy == 0) {
                            run[i][j] = term;
                        } else {
                            run[i][j] += term;
                        }
                    }
            }
            if (!F64) {
                // Kahan fold of the finished run: sum - comp tracks the exact total.
#pragma unroll
                for (int i = 0; i < RX; ++i)
#pragma unroll
                    for (int j = 0; j < RZ; ++j) {
                        const float yk = run[i][j] - comp[i][j];
                        const float tk = sum[i][j] + yk;
                        comp[i][j] = (tk - sum[i][j]) - yk;
                        sum[i][j] = tk;
                    }
            }
        }
        if (c + 1 < nchunks) stash(buf ^ 1);
        __syncthreads();
    }

    const double nm1 = (double)(n - 1);
    const bool direct = (gridDim.y == 1);
#pragma unroll
    for (int i = 0; i < RX; ++i) {
        const int64_t x = X0 + tx * RX + i;
        if (x >= n) continue;
#pragma unroll
        for (int j = 0; j < RZ; ++j) {
            const int64_t z = Z0 + tz * RZ + j;
            if (z >= n) continue;
            const double tot = F64 ? acc[i][j] : ((double)sum[i][j] - (double)comp[i][j]);
            if (direct) {
                C[x * ldc + z] = (float)(tot / nm1);
            } else {
                partial[((int64_t)blockIdx.y * n + x) * n + z] = tot;
            }
        }
    }
}

// C_xz = fl32( sum_k partial[k][x][z] / (n-1) ), the only cross-tile reduction.
__global__ void finalize_kernel(const double *__restrict__ partial, int32_t nchunks, int64_t n,
                                float *__restrict__ C, int64_t ldc) {
    const double nm1 = (double)(n - 1);
    for (int64_t x = blockIdx.y; x < n; x += gridDim.y)
        for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < n;
             z += (int64_t)gridDim.x * blockDim.x) {
            double s = 0.0;
            for (int32_t k = 0; k < nchunks; ++k) s += partial[((int64_t)k * n + x) * n + z];
            C[x * ldc + z] = (float)(s / nm1);
        }
}

// ---------------------------------------------------------------------------
// Input validation: sets bits in *flags (1 NaN, 2 inf, 4 negative,
// 8 asymmetric, 16 nonzero diagonal).
__global__ void check_input_kernel(const float *__restrict__ D, int64_t n, int64_t ldd,
                                   uint32_t *__restrict__ flags) {
    uint32_t f = 0;
    for (int64_t x = blockIdx.y; x < n; x += gridDim.y)
        for (int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; y < n;
             y += (int64_t)gridDim.x * blockDim.x) {
            const float v = D[x * ldd + y];
            if (v != v) f |= 1u;
            else if (__builtin_isinf(v)) f |= 2u;
            if (v < 0.0f) f |= 4u;
            const float w = D[y * ldd + x];
            if (!(v == w) && !(v != v && w != w)) f |= 8u;
            if (x == y && v != 0.0f) f |= 16u;
        }
    if (f) atomicOr(flags, f);
}

}  // namespace pald
