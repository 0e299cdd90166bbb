// triplet.hpp -- the triplet PaLD algorithm (Section 3, triplet algorithm;
// costs in Section 4, Thm 2): every unordered triple {p < q < r} is visited
// once per pass and its comparisons are shared by all three pairs.
//
// For a triple with a = d_pq, b = d_pr, c = d_qr and m = min(a, b, c), let
// e_a = [a == m], e_b = [b == m], e_c = [c == m] (at least one holds).  With
// ties handled exactly (the printed triplet algorithm is not tie-exact):
//   pass 1:  u_pq += e_b | e_c,  u_pr += e_a | e_c,  u_qr += e_a | e_b
//            (z joins the focus of (x, y) iff min(d_zx, d_zy) <= d_xy, i.e. iff
//            one of the other two distances is the minimum), starting from
//            u = 2 for every pair (x and y are in their own focus);
//   pass 2 (W/2 = half weight; "e ? A : B" are selects):
//            c_pr += e_b ? (e_c ? W_pq/2 : W_pq) : 0     c_qr += e_c ? (e_b ? W_pq/2 : W_pq) : 0
//            c_pq += e_a ? (e_c ? W_pr/2 : W_pr) : 0     c_rq += e_c ? (e_a ? W_pr/2 : W_pr) : 0
//            c_qp += e_a ? (e_b ? W_qr/2 : W_qr) : 0     c_rp += e_b ? (e_a ? W_qr/2 : W_qr) : 0
//   (each is [third point in the focus] * support with ties split, Section 5);
//   plus the terms whose third point is one of the pair (the diagonal of C and
//   the coincident-point terms), added per pair by triplet_init_c_kernel.
//
// GPU mapping.  An owner workgroup takes a 64 x 64 block pair (X, Z), X <= Z,
// and every triple whose smallest index is in X and largest in Z; the middle
// index q streams through LDS in stages of 16 rows.  Each thread owns 4 x 4
// pairs (p, r): the (p, r) terms accumulate in registers; the (p, q) terms of a
// q are summed over the thread's r, then over the 16 lanes that share p (lane
// shuffles), and added to the float64 accumulator with one atomic per value;
// the (q, r) terms are summed over the wave's p with shuffles, then over the
// four waves through LDS.  Every pair's terms come from several owners, so the
// global sums use integer atomics, which commute: int32 on the upper triangle
// of U (mirrored to the lower one after the pass) and, for C, 64-bit
// fixed-point accumulators A with F = 61 - ceil(log2 n) fraction bits.  Each
// owner's float32 partial sum is a multiple of its last mantissa bit, at
// least 2^-(ceil(log2 n) + 24) (every term is W_xy or W_xy / 2 with
// W_xy >= 1/n), so for n <= 2^18 it converts to fixed point exactly, and
// every sum stays below n/2, so below 2^60 in fixed point.  The result is
// the exact sum of the owners' partials whatever order the atomics land in:
// C is bitwise reproducible, and accurate to the same bound as the pairwise
// path.
//
// On a GPU this variant does fewer comparisons than the pairwise one but
// moves O(n^3 / 64) partial sums through atomics, where the pairwise tiles
// keep every output in registers: it is kept as the paper's second algorithm
// and as a comparator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pairwise.hpp"
#include "pald.h"

namespace pald {

constexpr int TRI_T = 64;         // owner tile side
constexpr int TRI_R = 4;          // 4 x 4 (p, r) per thread
constexpr int TRI_KQ = 16;        // q rows per LDS stage
constexpr int TRI_THREADS = 256;  // tid = tx * 16 + tz; p = X0 + 4 tx + i, r = Z0 + 4 tz + j
constexpr int TRI_RUN = 8;        // float32 run length of the (p, r) sums before a Kahan fold

// U_xy = 2 off the diagonal, U_xx = #{z : d_xz <= 0}.
__global__ void triplet_init_u_kernel(const float *__restrict__ D, int64_t n, int64_t ldd, int32_t *__restrict__ U,
                                      int64_t ldu) {
    __shared__ int32_t red[256];
    for (int64_t x = blockIdx.x; x < n; x += gridDim.x) {
        int32_t cnt = 0;
        for (int64_t y = threadIdx.x; y < n; y += blockDim.x) {
            U[x * ldu + y] = 2;
            cnt += (key_of(D[x * ldd + y]) == 0u) ? 1 : 0;
        }
        red[threadIdx.x] = cnt;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) U[x * ldu + x] = red[0];
        __syncthreads();
    }
}

// Fixed point of the C accumulators: value v is stored as v 2^F in 64 bits.
__host__ __device__ inline int32_t triplet_fixed_bits(int64_t n) {
    int32_t lg = 0;
    while (((int64_t)1 << lg) < n) ++lg;
    return 61 - lg;
}
__device__ __forceinline__ unsigned long long to_fixed(double v, double scale) {
    return (unsigned long long)__double2ll_rn(v * scale);
}

// The terms whose third point is one of the pair, into the fixed-point accumulator A:
//   A_xx = sum_{y != x} s(0, d_xy) W_xy       (third point x in the focus of (x, y))
//   A_xy = s(d_xy, 0) W_xy, x != y            (third point y; nonzero only if d_xy = 0)
// with s(p, q) = [p < q] + 1/2 [p == q]; the diagonal sum runs in float64 in a
// fixed order (tree over the workgroup) and is converted once.
__global__ void triplet_init_c_kernel(const float *__restrict__ D, int64_t n, int64_t ldd, const float *__restrict__ W,
                                      int64_t ldw, unsigned long long *__restrict__ A, double scale) {
    __shared__ double red[256];
    for (int64_t x = blockIdx.x; x < n; x += gridDim.x) {
        double diag = 0.0;
        for (int64_t y = threadIdx.x; y < n; y += blockDim.x) {
            if (y == x) continue;
            const bool zero = key_of(D[x * ldd + y]) == 0u;
            const float w = W[x * ldw + y];
            diag += zero ? 0.5 * (double)w : (double)w;
            A[x * n + y] = zero ? to_fixed(0.5 * (double)w, scale) : 0ull;
        }
        red[threadIdx.x] = diag;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) A[x * n + x] = to_fixed(red[0], scale);
        __syncthreads();
    }
}

// Pass 1 accumulates only the upper triangle of U (every triple adds to
// U[lo][hi], lo < hi); this copies it to the lower triangle: U[y][x] = U[x][y]
// for x < y.  32 x 32 tiles transposed through LDS; tile (ty, tx) with ty > tx
// reads tile (tx, ty), diagonal tiles mirror within themselves.
__global__ __launch_bounds__(256) void triplet_mirror_u_kernel(int32_t *__restrict__ U, int64_t ldu, int64_t n,
                                                               int32_t tiles) {
    __shared__ int32_t t[32][33];
    const int64_t nb = (n + 31) / 32;
    for (int64_t k = blockIdx.x; k < (int64_t)tiles; k += gridDim.x) {
        // k enumerates the lower-triangle tiles (ty >= tx) row by row
        int64_t ty = (int64_t)((sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
        if (ty * (ty + 1) / 2 > k) --ty;
        if ((ty + 1) * (ty + 2) / 2 <= k) ++ty;
        const int64_t tx = k - ty * (ty + 1) / 2;
        if (ty >= nb) break;
        // load source tile (tx, ty): rows tx*32.., columns ty*32..
        for (int e = threadIdx.x; e < 32 * 32; e += 256) {
            const int i = e / 32, j = e % 32;
            const int64_t row = tx * 32 + i, col = ty * 32 + j;
            t[i][j] = (row < n && col < n) ? U[row * ldu + col] : 0;
        }
        __syncthreads();
        // write destination tile (ty, tx): U[ty*32 + j][tx*32 + i] = t[i][j] where row < col in the source
        for (int e = threadIdx.x; e < 32 * 32; e += 256) {
            const int j = e / 32, i = e % 32;
            const int64_t srow = tx * 32 + i, scol = ty * 32 + j;
            if (srow < n && scol < n && srow < scol) U[scol * ldu + srow] = t[i][j];
        }
        __syncthreads();
    }
}

// C = fl32(A 2^-F / (n - 1)).
__global__ void triplet_finalize_kernel(const unsigned long long *__restrict__ A, int64_t n, float *__restrict__ C,
                                        int64_t ldc, double inv_scale) {
    const double nm1 = (double)(n - 1);
    for (int64_t x = blockIdx.y; x < n; x += gridDim.y)
        for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < n; z += (int64_t)gridDim.x * blockDim.x)
            C[x * ldc + z] = (float)((double)(long long)A[x * n + z] * inv_scale / nm1);
}

// k -> (bx, bz), bx <= bz < nb, with the owner tiles listed by decreasing
// bz - bx: an owner streams bz - bx + 1 blocks of middle indices, so the
// longest tiles start first and the short diagonal ones fill in at the end
// (longest processing time first).  Diagonal bz - bx = nb - m holds m tiles.
__device__ __forceinline__ void tri_tile_heavy_first(int32_t k, int32_t nb, int32_t &bx, int32_t &bz) {
    int64_t m = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)k)) * 0.5);
    while (m * (m - 1) / 2 > k) --m;
    while ((m + 1) * m / 2 <= k) ++m;
    bx = (int32_t)(k - m * (m - 1) / 2);
    bz = bx + (nb - (int32_t)m);
}

// Sum of v over the 16 lanes of a row (lane bits 0-3).
template <typename V>
__device__ __forceinline__ V row_sum16(V v) {
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}
// Sum of v over the 4 rows of a wave (lane bits 4-5).
template <typename V>
__device__ __forceinline__ V wave_rows_sum(V v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// One owner tile of either pass.  PASS2 = false: focus sizes into U (int32,
// atomics); PASS2 = true: cohesion sums into A (64-bit fixed point with scale
// 2^F, atomics).
template <bool PASS2>
__global__ __launch_bounds__(TRI_THREADS, 2) void triplet_kernel(const float *__restrict__ D, int64_t n, int64_t ldd,
                                                              const float *__restrict__ W, int64_t ldw,
                                                              int32_t *__restrict__ U, int64_t ldu,
                                                              unsigned long long *__restrict__ A, int32_t vec_d,
                                                              int32_t vec_w, int32_t tile0, double scale) {
    constexpr int T = TRI_T, R = TRI_R, KQ = TRI_KQ, NT = TRI_THREADS;
    constexpr int ROW = PASS2 ? 4 * T : 2 * T;     // loaded per q: a | (W_qp) | c | (W_qr)
    constexpr int LDS_ROW = PASS2 ? 6 * T : 2 * T; // staged: ... | W_qp/2 | W_qr/2
    constexpr int VPC = KQ * ROW / 4;              // uint4 loaded per stage
    constexpr int VPT = VPC / NT;
    static_assert(VPC % NT == 0, "stage must split evenly");
    using Part = typename std::conditional<PASS2, float, int32_t>::type;
    __shared__ uint4 sm[2 * KQ * LDS_ROW / 4];
    __shared__ Part qbuf[4][KQ][T][PASS2 ? 2 : 1];  // per-wave (q, r) partials of one stage

    int32_t bx, bz;
    tri_tile_heavy_first(tile0 + (int32_t)blockIdx.x, (int32_t)((n + T - 1) / T), bx, bz);
    const int64_t X0 = (int64_t)bx * T, Z0 = (int64_t)bz * T;
    const int tid = threadIdx.x;
    const int tx = tid / 16, tz = tid % 16, wave = tid / 64, row = (tid % 64) / 16;
    const bool diag_owner = bx == bz;

    // p_i = X0 + 4 tx + i, r_j = Z0 + 4 tz + j (recomputed where used: no
    // registers held for them across the q loop)
    auto p = [&](int i) { return X0 + tx * R + i; };
    auto r = [&](int j) { return Z0 + tz * R + j; };
    // stationary (p, r) data
    uint32_t b[R][R];
    float wpr[R][R];
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const bool in = p(i) < n && r(j) < n;
            b[i][j] = in ? key_of(D[p(i) * ldd + r(j)]) : 0u;
            const float w = (PASS2 && in) ? W[p(i) * ldw + r(j)] : 0.0f;
            wpr[i][j] = w;
        }
    // (p, r) accumulators: float32 runs r and Kahan sums s (a run starts from
    // the negated compensation of the previous fold, as in the pairwise pass 2)
    int32_t upr[R][R];
    float rpr[R][R], rrp[R][R], spr[R][R], srp[R][R];
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            upr[i][j] = 0;
            rpr[i][j] = rrp[i][j] = 0.0f;
            spr[i][j] = srp[i][j] = 0.0f;
        }

    // the middle index runs over [X0, min(n, Z0 + T)); triples outside p < q < r
    // (or with r >= n) are masked out
    const int64_t qlo = X0, qhi = min(n, Z0 + T);
    const int64_t nst = (qhi - qlo + KQ - 1) / KQ;

    uint4 pre[VPT];
    auto fetch = [&](int64_t qc) {
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int v = tid + k * NT;
            const int rr = v / (ROW / 4), g = v % (ROW / 4);
            const int seg = g / (T / 4);
            const int64_t q = qc + rr;
            if (PASS2) {
                const int64_t col = ((seg < 2) ? X0 : Z0) + 4 * (g % (T / 4));
                if (seg == 0 || seg == 2)
                    pre[k] = load_keys4(D, ldd, q, col, qhi, n, vec_d != 0, 0u);
                else
                    pre[k] = load_vals4(W, ldw, q, col, qhi, n, vec_w != 0);
            } else {
                const int64_t col = ((seg < 1) ? X0 : Z0) + 4 * (g % (T / 4));
                pre[k] = load_keys4(D, ldd, q, col, qhi, n, vec_d != 0, 0u);
            }
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int v = tid + k * NT;
            const int rr = v / (ROW / 4), g = v % (ROW / 4);
            uint4 *dst = sm + buf * (KQ * LDS_ROW / 4) + rr * (LDS_ROW / 4);
            dst[g] = pre[k];
            if (PASS2) {
                const int seg = g / (T / 4);
                if (seg == 1 || seg == 3) {
                    const uint4 w = pre[k];
                    dst[T + (seg == 1 ? 0 : T / 4) + g % (T / 4)] = make_uint4(
                        __float_as_uint(0.5f * __uint_as_float(w.x)), __float_as_uint(0.5f * __uint_as_float(w.y)),
                        __float_as_uint(0.5f * __uint_as_float(w.z)), __float_as_uint(0.5f * __uint_as_float(w.w)));
                }
            }
        }
    };

    if (nst > 0) {
        fetch(qlo);
        stash(0);
    }
    __syncthreads();

    for (int64_t st = 0; st < nst; ++st) {
        const int buf = (int)(st & 1);
        const int64_t qc = qlo + st * KQ;
        if (st + 1 < nst) fetch(qc + KQ);
        const uint32_t *s = reinterpret_cast<const uint32_t *>(sm + buf * (KQ * LDS_ROW / 4));
#pragma unroll 1
        for (int qq = 0; qq < KQ; ++qq) {
            const int64_t q = qc + qq;
            const uint32_t *rowp = s + qq * LDS_ROW;
            uint32_t av[R], cv[R];
            float wpq[R], whpq[R], wqr[R], whqr[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                av[i] = rowp[tx * R + i];
                cv[i] = rowp[(PASS2 ? 2 : 1) * T + tz * R + i];
                if (PASS2) {
                    wpq[i] = __uint_as_float(rowp[T + tx * R + i]);
                    wqr[i] = __uint_as_float(rowp[3 * T + tz * R + i]);
                    whpq[i] = __uint_as_float(rowp[4 * T + tx * R + i]);
                    whqr[i] = __uint_as_float(rowp[5 * T + tz * R + i]);
                }
            }
            uint64_t vp[R], vr[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                vp[i] = lane_mask(p(i) < q);
                vr[i] = lane_mask(q < r(i) && r(i) < n);
            }
            Part tpq[R], tqp[R], tqr[R], trq[R];
#pragma unroll
            for (int i = 0; i < R; ++i) tpq[i] = tqp[i] = tqr[i] = trq[i] = (Part)0;
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const uint64_t valid = vp[i] & vr[j];
                    const uint32_t m = umin(av[i], umin(b[i][j], cv[j]));
                    const uint64_t ea = lane_mask(av[i] == m) & valid;
                    const uint64_t eb = lane_mask(b[i][j] == m) & valid;
                    const uint64_t ec = lane_mask(cv[j] == m) & valid;
                    if (!PASS2) {
                        tpq[i] += lane_bit(eb | ec) ? 1 : 0;
                        upr[i][j] += lane_bit(ea | ec) ? 1 : 0;
                        tqr[j] += lane_bit(ea | eb) ? 1 : 0;
                    } else {
                        const float t1 = lane_bit(eb) ? (lane_bit(ec) ? whpq[i] : wpq[i]) : 0.0f;  // c_pr
                        const float t2 = lane_bit(ec) ? (lane_bit(eb) ? whpq[i] : wpq[i]) : 0.0f;  // c_qr
                        const float whpr = 0.5f * wpr[i][j];  // exact; not kept across q
                        const float t3 = lane_bit(ea) ? (lane_bit(ec) ? whpr : wpr[i][j]) : 0.0f;  // c_pq
                        const float t4 = lane_bit(ec) ? (lane_bit(ea) ? whpr : wpr[i][j]) : 0.0f;  // c_rq
                        const float t5 = lane_bit(ea) ? (lane_bit(eb) ? whqr[j] : wqr[j]) : 0.0f;  // c_qp
                        const float t6 = lane_bit(eb) ? (lane_bit(ea) ? whqr[j] : wqr[j]) : 0.0f;  // c_rp
                        rpr[i][j] += t1;
                        rrp[i][j] += t6;
                        tpq[i] += t3;
                        tqp[i] += t5;
                        tqr[j] += t2;
                        trq[j] += t4;
                    }
                }
            if (PASS2 && (qq % TRI_RUN) == TRI_RUN - 1) {
#pragma unroll
                for (int i = 0; i < R; ++i)
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        float tk = spr[i][j] + rpr[i][j];
                        rpr[i][j] = rpr[i][j] - (tk - spr[i][j]);
                        spr[i][j] = tk;
                        tk = srp[i][j] + rrp[i][j];
                        rrp[i][j] = rrp[i][j] - (tk - srp[i][j]);
                        srp[i][j] = tk;
                    }
            }
            // (p, q) and (q, p): sum over the 16 lanes sharing p; lane tz = k emits value k
#pragma unroll
            for (int i = 0; i < R; ++i) {
                tpq[i] = row_sum16(tpq[i]);
                if (PASS2) tqp[i] = row_sum16(tqp[i]);
            }
            if (q < n) {
                if (tz < R) {
                    Part v = tpq[0];
#pragma unroll
                    for (int i = 1; i < R; ++i)
                        if (tz == i) v = tpq[i];
                    const int64_t pi = p(tz);
                    if (pi < n && v != (Part)0) {
                        if (PASS2) {
                            atomicAdd(&A[pi * n + q], to_fixed((double)v, scale));
                        } else {
                            atomicAdd(&U[pi * ldu + q], (int32_t)v);  // p < q: upper triangle only
                        }
                    }
                } else if (PASS2 && tz < 2 * R) {
                    Part v = tqp[0];
#pragma unroll
                    for (int i = 1; i < R; ++i)
                        if (tz - R == i) v = tqp[i];
                    const int64_t pi = p(tz - R);
                    if (pi < n && v != (Part)0) atomicAdd(&A[q * n + pi], to_fixed((double)v, scale));
                }
            }
            // (q, r) and (r, q): sum over the wave's p, then stage per wave in LDS
#pragma unroll
            for (int j = 0; j < R; ++j) {
                tqr[j] = wave_rows_sum(tqr[j]);
                if (PASS2) trq[j] = wave_rows_sum(trq[j]);
            }
            if (row == 0) {
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    qbuf[wave][qq][tz * R + j][0] = tqr[j];
                    if (PASS2) qbuf[wave][qq][tz * R + j][PASS2 ? 1 : 0] = trq[j];
                }
            }
        }
        if (st + 1 < nst) stash(buf ^ 1);
        __syncthreads();
        // sum the four waves' (q, r) partials of this stage and add them
        for (int e = tid; e < KQ * T * (PASS2 ? 2 : 1); e += NT) {
            const int d = PASS2 ? (e % 2) : 0;
            const int rl = (PASS2 ? e / 2 : e) % T;
            const int qq = (PASS2 ? e / 2 : e) / T;
            const int64_t q = qc + qq, rr = Z0 + rl;
            if (q >= n || rr >= n) continue;
            const Part v = qbuf[0][qq][rl][d] + qbuf[1][qq][rl][d] + qbuf[2][qq][rl][d] + qbuf[3][qq][rl][d];
            if (v == (Part)0) continue;
            if (PASS2) {
                atomicAdd(d == 0 ? &A[q * n + rr] : &A[rr * n + q], to_fixed((double)v, scale));
            } else {
                atomicAdd(&U[q * ldu + rr], (int32_t)v);  // q < r: upper triangle only
            }
        }
        __syncthreads();
    }

    // the (p, r) sums of this owner
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (p(i) >= n || r(j) >= n || (diag_owner && p(i) >= r(j))) continue;
            if (PASS2) {
                const double f = (double)spr[i][j] + (double)rpr[i][j];
                const double g = (double)srp[i][j] + (double)rrp[i][j];
                if (f != 0.0) atomicAdd(&A[p(i) * n + r(j)], to_fixed(f, scale));
                if (g != 0.0) atomicAdd(&A[r(j) * n + p(i)], to_fixed(g, scale));
            } else if (upr[i][j] != 0) {
                atomicAdd(&U[p(i) * ldu + r(j)], upr[i][j]);  // p < r: upper triangle only
            }
        }
}

}  // namespace pald
