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
// index q streams through LDS in stages of 8 rows.  Each thread owns 4 x 4
// pairs (p, r) and runs, per q, a branch-free block per triple: one min and
// three compares, then float32 adds of half weights under EXEC masks
// (triplet_cohesion4, triplet_count4).  The (p, r) terms accumulate in
// registers; the (p, q) terms of a q are summed over the 16 lanes that share
// p (DPP), the (q, r) terms over the wave's rows (lane swaps), both into LDS,
// and once per stage the workgroup adds them to the global sums with integer
// atomics, which commute: int32 for U and, for C, 64-bit fixed-point
// accumulators with F = 61 - ceil(log2 n) fraction bits.  Every sum lands in
// row q of its accumulator: u_pq in the lower triangle of U (u_qr, u_pr in
// the upper one; a last kernel adds the two triangles), c_qp and c_qr in A,
// c_pq and c_rq transposed in B (C = A + B^T at the end).  The atomics of a
// wave then touch one or two rows instead of 64 rows n elements apart, which
// land on few memory channels: with the sums in A alone both passes took
// 2-3x longer.  Each owner's float32 partial
// sum is a multiple of 2^-(ceil(log2 n) + 24) (every term is a half weight
// W_xy / 2 with W_xy >= 1/n, a float32 of 24 bits, and float32 sums of such
// multiples stay multiples of it), so for n <= 2^18 it converts to fixed
// point exactly, and every sum stays below n/2, so below 2^60 in fixed
// point.  The result is the exact sum of the owners' partials whatever order
// the atomics land in: C is bitwise reproducible, and accurate to the same
// bound as the pairwise path.
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
constexpr int TRI_R = 4;          // r per thread; p per thread: tri_rp<PASS2>() (4 x 4 or 2 x 4 pairs)
constexpr int TRI_KQ = 8;         // q rows per LDS stage
// p per thread of pass 1 / pass 2 (pass 2 holds twice the registers per pair)
#ifndef PALD_TRI_RP2
#define PALD_TRI_RP2 2
#endif
template <bool PASS2>
constexpr int tri_rp() { return PASS2 ? PALD_TRI_RP2 : 4; }
// threads: tid = tx * 16 + tz, p = X0 + RP tx + i, r = Z0 + 4 tz + j
template <bool PASS2>
constexpr int tri_threads() { return 16 * 64 / tri_rp<PASS2>(); }
constexpr int TRI_RUN = 8;        // q values per float32 run of the (p, r) sums (one term each)
// minimum waves per SIMD each pass is compiled for (its register budget)
#ifndef PALD_TRI_MIN_WAVES1
#define PALD_TRI_MIN_WAVES1 4
#endif
#ifndef PALD_TRI_MIN_WAVES2
#define PALD_TRI_MIN_WAVES2 (PALD_TRI_RP2 == 2 ? 4 : 3)
#endif
// U_xy = 2 above the diagonal, 0 below it (pass 1 adds into both triangles
// and triplet_mirror_u_kernel sums them), U_xx = #{z : d_xz <= 0}.
__global__ void triplet_init_u_kernel(const float *__restrict__ D, int64_t n, int64_t ldd, int32_t *__restrict__ U,
                                      int64_t ldu) {
    __shared__ int32_t red[256];
    for (int64_t x = blockIdx.x; x < n; x += gridDim.x) {
        int32_t cnt = 0;
        for (int64_t y = threadIdx.x; y < n; y += blockDim.x) {
            U[x * ldu + y] = y < x ? 0 : 2;
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
                                      int64_t ldw, unsigned long long *__restrict__ A,
                                      unsigned long long *__restrict__ B, double scale) {
    __shared__ double red[256];
    for (int64_t x = blockIdx.x; x < n; x += gridDim.x) {
        double diag = 0.0;
        for (int64_t y = threadIdx.x; y < n; y += blockDim.x) {
            B[x * n + y] = 0ull;
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

// Pass 1 accumulates into both triangles of U; this makes U symmetric:
// U[x][y] = U[y][x] = U[x][y] + U[y][x] for x < y.  32 x 32 tiles through
// LDS; the lower-triangle tile (ty, tx), ty >= tx, pairs with the upper tile
// (tx, ty), and diagonal tiles pair with themselves.
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
        // the upper tile (tx, ty): rows tx*32.., columns ty*32..
        for (int e = threadIdx.x; e < 32 * 32; e += 256) {
            const int i = e / 32, j = e % 32;
            const int64_t row = tx * 32 + i, col = ty * 32 + j;
            t[i][j] = (row < n && col < n) ? U[row * ldu + col] : 0;
        }
        __syncthreads();
        // the lower tile (ty, tx): U[ty*32 + j][tx*32 + i] pairs with t[i][j] where row < col
        for (int e = threadIdx.x; e < 32 * 32; e += 256) {
            const int j = e / 32, i = e % 32;
            const int64_t srow = tx * 32 + i, scol = ty * 32 + j;
            if (srow < n && scol < n && srow < scol) {
                const int32_t v = t[i][j] + U[scol * ldu + srow];
                t[i][j] = v;
                U[scol * ldu + srow] = v;
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 32 * 32; e += 256) {
            const int i = e / 32, j = e % 32;
            const int64_t row = tx * 32 + i, col = ty * 32 + j;
            if (row < n && col < n && row < col) U[row * ldu + col] = t[i][j];
        }
        __syncthreads();
    }
}

// C = fl32((A + B^T) 2^-F / (n - 1)), B read transposed through LDS in
// 32 x 32 tiles; tile k covers rows 32 (k / nb).. and columns 32 (k % nb).. of C.
__global__ __launch_bounds__(256) void triplet_finalize_kernel(const unsigned long long *__restrict__ A,
                                                               const unsigned long long *__restrict__ B, int64_t n,
                                                               float *__restrict__ C, int64_t ldc, double inv_scale,
                                                               int64_t tiles) {
    __shared__ unsigned long long t[32][33];
    const double nm1 = (double)(n - 1);
    const int64_t nb = (n + 31) / 32;
    for (int64_t k = blockIdx.x; k < tiles; k += gridDim.x) {
        const int64_t x0 = (k / nb) * 32, z0 = (k % nb) * 32;
        for (int e = threadIdx.x; e < 32 * 32; e += 256) {  // B[z0 + i][x0 + j]
            const int i = e / 32, j = e % 32;
            t[i][j] = (z0 + i < n && x0 + j < n) ? B[(z0 + i) * n + x0 + j] : 0ull;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 32 * 32; e += 256) {
            const int i = e / 32, j = e % 32;
            const int64_t x = x0 + i, z = z0 + j;
            if (x < n && z < n) C[x * ldc + z] = (float)((double)(long long)(A[x * n + z] + t[j][i]) * inv_scale / nm1);
        }
        __syncthreads();
    }
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

// Sum of v over the 16 lanes of a row (lane bits 0-3), by DPP butterflies:
// quad_perm [1,0,3,2] and [2,3,0,1], then the half-row and row mirrors.
__device__ __forceinline__ float row_sum16(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, true));
    return v;
}
// x over lane halves in lanes 0-31, y over lane halves in lanes 32-63:
// v_permlane32_swap exchanges the upper half of x with the lower half of y.
__device__ __forceinline__ float halves_sum(float x, float y) {
    const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}
// x over row pairs (0, 1) and (2, 3) in rows 0 and 2, y in rows 1 and 3:
// v_permlane16_swap exchanges the odd rows of x with the even rows of y.
__device__ __forceinline__ float row_pairs_sum(float x, float y) {
    const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}

// v * 2^fbits as an integer, for v > 0 normal and a multiple of 2^-fbits
// (exact): v = m 2^(e - 150) with the 24-bit significand m.
__device__ __forceinline__ unsigned long long fixed_of(float v, int32_t fbits) {
    const uint32_t bits = __float_as_uint(v);
    const unsigned long long m = (unsigned long long)((bits & 0x7fffffu) | 0x800000u);
    const int32_t sh = (int32_t)(bits >> 23) - 150 + fbits;
    return sh >= 0 ? (m << sh) : (m >> -sh);
}

// The block of one triple (p, q, r) and three more with the same p and q
// (the thread's r_0..r_3), registers only.  a = key d_pq, b = key d_pr,
// c = key d_qr; m = min(a, b, c), e_a = [a == m], e_b = [b == m], e_c =
// [c == m], computed with EXEC = the lanes whose triple is valid, so that the
// masks are 0 elsewhere.  Then EXEC takes each mask in turn:
//   pass 1: u_pq += e_b | e_c, u_pr += e_a | e_c, u_qr += e_a | e_b
//           (counts in float32, exact below 2^24);
//   pass 2, with f_x = 2 - [e_x]:
//           under e_a: c_pq += W_pr/2 f_c, c_qp += W_qr/2 f_b;
//           under e_b: c_pr += W_pq/2 f_c, c_rp += W_qr/2 f_a;
//           under e_c: c_qr += W_pq/2 f_b, c_rq += W_pr/2 f_a
//           (a full weight without a tie, half of it on a tie).
// The last instruction restores EXEC to `full`; the s_nop keeps the lane
// permutations that read the sums clear of the last writes.
#define PALD_T_CMP(k, e)                                                                                         \
    "s_and_b64 exec, %[vp], %[vr" #k "]\n\t"                                                                  \
    "v_min3_u32 %[m], %[a], %[b" #k "], %[c" #k "]\n\t"                                                       \
    "v_cmp_eq_u32_e64 %[ea" #e "], %[a], %[m]\n\t"                                                            \
    "v_cmp_eq_u32_e64 %[eb" #e "], %[b" #k "], %[m]\n\t"                                                      \
    "v_cmp_eq_u32_e64 %[ec" #e "], %[c" #k "], %[m]\n\t"
#define PALD_T_U(k, e)                                                                                              \
    "s_or_b64 exec, %[eb" #e "], %[ec" #e "]\n\t"                                                             \
    "v_add_f32 %[tpq], 1.0, %[tpq]\n\t"                                                                        \
    "s_or_b64 exec, %[ea" #e "], %[ec" #e "]\n\t"                                                             \
    "v_add_f32 %[rf" #k "], 1.0, %[rf" #k "]\n\t"                                                             \
    "s_or_b64 exec, %[ea" #e "], %[eb" #e "]\n\t"                                                             \
    "v_add_f32 %[tqr" #k "], 1.0, %[tqr" #k "]\n\t"
// Pass 2 adds each term with one multiply-add: under EXEC = e_a, c_pq +=
// W_pr/2 f_c and c_qp += W_qr/2 f_b, and so on, with f_x = 2 - [e_x] (1 on a
// tie with x, else 2) from a select; the products are exact, so each term is
// one rounding, as an add.
#define PALD_T_CMPF(k, e)                                                                                        \
    PALD_T_CMP(k, e)                                                                                             \
    "v_cndmask_b32_e64 %[fa" #e "], 2.0, 1.0, %[ea" #e "]\n\t"                                                \
    "v_cndmask_b32_e64 %[fb" #e "], 2.0, 1.0, %[eb" #e "]\n\t"                                                \
    "v_cndmask_b32_e64 %[fc" #e "], 2.0, 1.0, %[ec" #e "]\n\t"
#define PALD_T_F(k, e)                                                                                           \
    "s_mov_b64 exec, %[ea" #e "]\n\t"                                                                         \
    "v_fmac_f32 %[tpq], %[hpr" #k "], %[fc" #e "]\n\t"                                                        \
    "v_fmac_f32 %[tqp], %[hc" #k "], %[fb" #e "]\n\t"                                                         \
    "s_mov_b64 exec, %[eb" #e "]\n\t"                                                                         \
    "v_fmac_f32 %[rf" #k "], %[ha], %[fc" #e "]\n\t"                                                          \
    "v_fmac_f32 %[rr" #k "], %[hc" #k "], %[fa" #e "]\n\t"                                                    \
    "s_mov_b64 exec, %[ec" #e "]\n\t"                                                                         \
    "v_fmac_f32 %[tqr" #k "], %[ha], %[fb" #e "]\n\t"                                                         \
    "v_fmac_f32 %[trq" #k "], %[hpr" #k "], %[fa" #e "]\n\t"
#define PALD_T_MASKS(e) [ea##e] "=&s"(ea[e]), [eb##e] "=&s"(eb[e]), [ec##e] "=&s"(ec[e])
#define PALD_T_FS(e) [fa##e] "=&v"(fa[e]), [fb##e] "=&v"(fb[e]), [fc##e] "=&v"(fc[e])
#define PALD_T_IN(k) [b##k] "v"(b[k]), [c##k] "v"(c[k]), [vr##k] "s"(vr[k])
#define PALD_T_IN2(k) [hpr##k] "v"(hpr[k]), [hc##k] "v"(hc[k])

__device__ __forceinline__ void triplet_count4(float &tpq, float (&rf)[4], float (&tqr)[4], uint32_t a,
                                               const uint32_t (&b)[4], const uint32_t (&c)[4], uint64_t vp,
                                               const uint64_t (&vr)[4], uint64_t full) {
    uint64_t ea[2], eb[2], ec[2];
    uint32_t m;
    asm volatile(PALD_T_CMP(0, 0) PALD_T_CMP(1, 1) PALD_T_U(0, 0) PALD_T_CMP(2, 0) PALD_T_U(1, 1)
                 PALD_T_CMP(3, 1) PALD_T_U(2, 0) PALD_T_U(3, 1)
                 "s_mov_b64 exec, %[full]\n\t"
                 "s_nop 4"
                 : [tpq] "+v"(tpq), [rf0] "+v"(rf[0]), [rf1] "+v"(rf[1]), [rf2] "+v"(rf[2]), [rf3] "+v"(rf[3]),
                   [tqr0] "+v"(tqr[0]), [tqr1] "+v"(tqr[1]), [tqr2] "+v"(tqr[2]), [tqr3] "+v"(tqr[3]),
                   [m] "=&v"(m), PALD_T_MASKS(0), PALD_T_MASKS(1)
                 : [a] "v"(a), [vp] "s"(vp), [full] "s"(full), PALD_T_IN(0), PALD_T_IN(1), PALD_T_IN(2),
                   PALD_T_IN(3)
                 : "scc");
}

__device__ __forceinline__ void triplet_cohesion4(float &tpq, float &tqp, float (&rf)[4], float (&rr)[4],
                                                  float (&tqr)[4], float (&trq)[4], uint32_t a, float ha,
                                                  const uint32_t (&b)[4], const float (&hpr)[4],
                                                  const uint32_t (&c)[4], const float (&hc)[4], uint64_t vp,
                                                  const uint64_t (&vr)[4], uint64_t full) {
    uint64_t ea[2], eb[2], ec[2];
    uint32_t m;
    float fa[2], fb[2], fc[2];
    asm volatile(PALD_T_CMPF(0, 0) PALD_T_CMPF(1, 1) PALD_T_F(0, 0) PALD_T_CMPF(2, 0) PALD_T_F(1, 1)
                 PALD_T_CMPF(3, 1) PALD_T_F(2, 0) PALD_T_F(3, 1)
                 "s_mov_b64 exec, %[full]\n\t"
                 "s_nop 4"
                 : [tpq] "+v"(tpq), [tqp] "+v"(tqp), [rf0] "+v"(rf[0]), [rf1] "+v"(rf[1]), [rf2] "+v"(rf[2]),
                   [rf3] "+v"(rf[3]), [rr0] "+v"(rr[0]), [rr1] "+v"(rr[1]), [rr2] "+v"(rr[2]), [rr3] "+v"(rr[3]),
                   [tqr0] "+v"(tqr[0]), [tqr1] "+v"(tqr[1]), [tqr2] "+v"(tqr[2]), [tqr3] "+v"(tqr[3]),
                   [trq0] "+v"(trq[0]), [trq1] "+v"(trq[1]), [trq2] "+v"(trq[2]), [trq3] "+v"(trq[3]),
                   [m] "=&v"(m), PALD_T_MASKS(0), PALD_T_MASKS(1), PALD_T_FS(0), PALD_T_FS(1)
                 : [a] "v"(a), [ha] "v"(ha), [vp] "s"(vp), [full] "s"(full), PALD_T_IN(0), PALD_T_IN(1),
                   PALD_T_IN(2), PALD_T_IN(3), PALD_T_IN2(0), PALD_T_IN2(1), PALD_T_IN2(2), PALD_T_IN2(3)
                 : "scc");

}
#undef PALD_T_CMP
#undef PALD_T_U
#undef PALD_T_MASKS
#undef PALD_T_CMPF
#undef PALD_T_F
#undef PALD_T_FS
#undef PALD_T_IN
#undef PALD_T_IN2

// RP consecutive 32-bit values of a staged row, and the RP sums of a row of
// lanes into LDS.
template <int RP, typename V>
__device__ __forceinline__ void load_row_vals(V (&v)[RP], const V *src) {
    if constexpr (RP == 4) {
        const uint4 t = *reinterpret_cast<const uint4 *>(src);
        v[0] = __builtin_bit_cast(V, t.x); v[1] = __builtin_bit_cast(V, t.y);
        v[2] = __builtin_bit_cast(V, t.z); v[3] = __builtin_bit_cast(V, t.w);
    } else {
        const uint2 t = *reinterpret_cast<const uint2 *>(src);
        v[0] = __builtin_bit_cast(V, t.x); v[1] = __builtin_bit_cast(V, t.y);
    }
}
template <int RP>
__device__ __forceinline__ void store_row_vals(float *dst, const float (&v)[RP]) {
    if constexpr (RP == 4)
        *reinterpret_cast<float4 *>(dst) = make_float4(v[0], v[1], v[2], v[3]);
    else
        *reinterpret_cast<float2 *>(dst) = make_float2(v[0], v[1]);
}

// One owner tile of either pass.  PASS2 = false: focus sizes into U (int32,
// atomics, upper triangle); PASS2 = true: cohesion sums into A (64-bit fixed
// point with fbits fraction bits, atomics).
//
// Per middle index q a thread runs the blocks of its 4 x 4 triples (p_i, q,
// r_j); the (p, r) terms stay in its registers, the (p, q) terms are summed
// over the 16 lanes that share p (DPP) into a per-stage LDS buffer, and the
// (q, r) terms over the wave's 4 rows (lane swaps; each row ends up with a
// different pair of sums) into per-wave LDS buffers.  After each stage of KQ
// rows of q the workgroup adds the stage's (p, q) and (q, r) sums (the four
// waves' partials in wave order) to the global sums.  Stages whose q lie
// between the two blocks need no index masks.
template <bool PASS2>
__global__ __launch_bounds__(tri_threads<PASS2>(), PASS2 ? PALD_TRI_MIN_WAVES2 : PALD_TRI_MIN_WAVES1) void triplet_kernel(
    const float *__restrict__ D, int64_t n, int64_t ldd, const float *__restrict__ W, int64_t ldw,
    int32_t *__restrict__ U, int64_t ldu, unsigned long long *__restrict__ A, unsigned long long *__restrict__ B,
    int32_t vec_d, int32_t vec_w, int32_t tile0, int32_t fbits, double scale) {
    constexpr int T = TRI_T, R = TRI_R, RP = tri_rp<PASS2>(), KQ = TRI_KQ, NT = tri_threads<PASS2>();
    constexpr int NW = NT / 64;                  // waves
    constexpr int LROW = PASS2 ? 4 * T : 2 * T;  // per q: a | W_qp/2 | c | W_qr/2  (pass 1: a | c)
    constexpr int CSEG = PASS2 ? 2 * T : T;      // offset of c in a row
    constexpr int ND = PASS2 ? 2 : 1;            // (p, q) and (q, p); (q, r) and (r, q)
    constexpr int VPC = KQ * LROW / 4;           // uint4 per stage
    constexpr int VPT = VPC / NT;
    static_assert(VPC % NT == 0, "stage must split evenly");
    static_assert(KQ % TRI_RUN == 0, "stages hold whole runs");
    static_assert(R == 4 && T == 64 && (RP == 4 || RP == 2) && NT == 16 * T / RP,
                  "the lane reductions assume RP x 4 per thread, 16 lanes over r");
    __shared__ uint4 sm[2 * KQ * LROW / 4];
    __shared__ float pbuf[KQ][ND][T];      // (p, q) sums of the stage, by p
    __shared__ float qbuf[NW][KQ][ND][T];  // per-wave (q, r) sums of the stage, by r

    int32_t bx, bz;
    tri_tile_heavy_first(tile0 + (int32_t)blockIdx.x, (int32_t)((n + T - 1) / T), bx, bz);
    const int64_t X0 = (int64_t)bx * T, Z0 = (int64_t)bz * T;
    const int tid = threadIdx.x;
    const int tx = tid / 16, tz = tid % 16, wave = tid / 64, row = (tid % 64) / 16;
    const bool diag_owner = bx == bz;
    const uint64_t full = __builtin_amdgcn_read_exec();

    auto p = [&](int i) { return X0 + tx * RP + i; };
    auto r = [&](int j) { return Z0 + tz * R + j; };
    // stationary (p, r) data: keys and half weights
    uint32_t b[RP][R];
    float hpr[RP][R];
#pragma unroll
    for (int i = 0; i < RP; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const bool in = p(i) < n && r(j) < n;
            b[i][j] = in ? key_of(D[p(i) * ldd + r(j)]) : 0u;
            hpr[i][j] = (PASS2 && in) ? 0.5f * W[p(i) * ldw + r(j)] : 0.0f;
        }
    uint64_t rn[R];
#pragma unroll
    for (int j = 0; j < R; ++j) rn[j] = lane_mask(r(j) < n);
    // (p, r) accumulators: pass 1 counts in rf; pass 2 float32 runs rf (c_pr)
    // and rr (c_rp) with Kahan sums sf, sr (a run starts from the negated
    // compensation of the previous fold)
    float rf[RP][R], rr[RP][R], sf[RP][R], sr[RP][R];
#pragma unroll
    for (int i = 0; i < RP; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) rf[i][j] = rr[i][j] = sf[i][j] = sr[i][j] = 0.0f;

    // the middle index runs over [X0, min(n, Z0 + T)); triples outside
    // p < q < r < n are masked out
    const int64_t qlo = X0, qhi = min(n, Z0 + T);
    const int64_t nst = (qhi - qlo + KQ - 1) / KQ;

    uint4 pre[VPT];
    auto fetch = [&](int64_t qc) {
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int v = tid + k * NT;
            const int rw = v / (LROW / 4), g = v % (LROW / 4);
            const int seg = g / (T / 4);
            const int64_t q = qc + rw;
            const int64_t col = ((seg < ND) ? X0 : Z0) + 4 * (g % (T / 4));
            if (PASS2 && (seg & 1))
                pre[k] = load_vals4(W, ldw, q, col, qhi, n, vec_w != 0);
            else
                pre[k] = load_keys4(D, ldd, q, col, qhi, n, vec_d != 0, 0u);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int v = tid + k * NT;
            const int rw = v / (LROW / 4), g = v % (LROW / 4);
            const int seg = g / (T / 4);
            uint4 w = pre[k];
            if (PASS2 && (seg & 1))  // weights staged halved (exact)
                w = make_uint4(__float_as_uint(0.5f * __uint_as_float(w.x)),
                               __float_as_uint(0.5f * __uint_as_float(w.y)),
                               __float_as_uint(0.5f * __uint_as_float(w.z)),
                               __float_as_uint(0.5f * __uint_as_float(w.w)));
            sm[buf * (KQ * LROW / 4) + rw * (LROW / 4) + g] = w;
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
        const bool interior = qc >= X0 + T && qc + KQ <= Z0;
        const uint32_t *s = reinterpret_cast<const uint32_t *>(sm + buf * (KQ * LROW / 4));
#pragma unroll 1
        for (int h = 0; h < KQ; h += TRI_RUN) {
#pragma unroll 1
        for (int qq = h; qq < h + TRI_RUN; ++qq) {
            const int64_t q = qc + qq;
            const uint32_t *rowp = s + qq * LROW;
            uint32_t av[RP];
            float hav[RP];
            load_row_vals<RP>(av, rowp + tx * RP);
            if (PASS2) load_row_vals<RP>(hav, reinterpret_cast<const float *>(rowp + T + tx * RP));
            const uint4 c4 = *reinterpret_cast<const uint4 *>(rowp + CSEG + tz * R);
            const uint32_t cv[R] = {c4.x, c4.y, c4.z, c4.w};
            uint64_t vp[RP], vr[R];
            if (interior) {
#pragma unroll
                for (int i = 0; i < RP; ++i) vp[i] = full;
#pragma unroll
                for (int j = 0; j < R; ++j) vr[j] = rn[j];
            } else {
                const int32_t qx = (int32_t)(q - X0), qz = (int32_t)(q - Z0);
#pragma unroll
                for (int i = 0; i < RP; ++i) vp[i] = lane_mask(tx * RP + i < qx);
#pragma unroll
                for (int j = 0; j < R; ++j) vr[j] = lane_mask(qz < tz * R + j) & rn[j];
            }
            float tpq[RP], tqp[RP], tqr[R] = {0.0f, 0.0f, 0.0f, 0.0f}, trq[R] = {0.0f, 0.0f, 0.0f, 0.0f};
            if constexpr (PASS2) {
                const float4 hc4 = *reinterpret_cast<const float4 *>(rowp + 3 * T + tz * R);
                const float hcv[R] = {hc4.x, hc4.y, hc4.z, hc4.w};
#pragma unroll
                for (int i = 0; i < RP; ++i) {
                    tpq[i] = tqp[i] = 0.0f;
                    triplet_cohesion4(tpq[i], tqp[i], rf[i], rr[i], tqr, trq, av[i], hav[i], b[i], hpr[i], cv, hcv,
                                      vp[i], vr, full);
                }
            } else {
#pragma unroll
                for (int i = 0; i < RP; ++i) {
                    tpq[i] = 0.0f;
                    triplet_count4(tpq[i], rf[i], tqr, av[i], b[i], cv, vp[i], vr, full);
                }
            }
            // (p, q) [and (q, p)]: sums over the 16 lanes sharing p, stored by lane 0 [and 1] of the row
#pragma unroll
            for (int i = 0; i < RP; ++i) {
                tpq[i] = row_sum16(tpq[i]);
                if (PASS2) tqp[i] = row_sum16(tqp[i]);
            }
            if (tz == 0) store_row_vals<RP>(&pbuf[qq][0][tx * RP], tpq);
            if (PASS2 && tz == 1) store_row_vals<RP>(&pbuf[qq][ND - 1][tx * RP], tqp);
            // (q, r) [and (r, q)]: sums over the wave's 4 rows; row k keeps
            // pass 2: direction k / 2, r_j for j = 2 (k % 2) + {0, 1}; pass 1: r_k
            if constexpr (PASS2) {
                float u[R];
#pragma unroll
                for (int j = 0; j < R; ++j) u[j] = halves_sum(tqr[j], trq[j]);
                const float v0 = row_pairs_sum(u[0], u[2]), v1 = row_pairs_sum(u[1], u[3]);
                *reinterpret_cast<float2 *>(&qbuf[wave][qq][row >> 1][tz * R + 2 * (row & 1)]) = make_float2(v0, v1);
            } else {
                const float w0 = halves_sum(tqr[0], tqr[2]), w1 = halves_sum(tqr[1], tqr[3]);
                qbuf[wave][qq][0][tz * R + row] = row_pairs_sum(w0, w1);
            }
        }
        if constexpr (PASS2) {  // end of a run: fold it into the Kahan sums
#pragma unroll
            for (int i = 0; i < RP; ++i)
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    float tk = sf[i][j] + rf[i][j];
                    rf[i][j] = rf[i][j] - (tk - sf[i][j]);
                    sf[i][j] = tk;
                    tk = sr[i][j] + rr[i][j];
                    rr[i][j] = rr[i][j] - (tk - sr[i][j]);
                    sr[i][j] = tk;
                }
        }
        }
        if (st + 1 < nst) stash(buf ^ 1);
        __syncthreads();
        // add the stage's (p, q) and (q, r) sums
#pragma unroll 1
        for (int e = tid; e < KQ * ND * T; e += NT) {
            const int l = e % T, d = (e / T) % ND, qq = e / (ND * T);
            const int64_t q = qc + qq;
            if (q >= qhi) continue;
            const int64_t pp = X0 + l, rz = Z0 + l;
            const float v = pbuf[qq][d][l];
            float w = qbuf[0][qq][d][l];
#pragma unroll
            for (int k = 1; k < NW; ++k) w += qbuf[k][qq][d][l];
            if (PASS2) {
                // c_pq into B[q][p], c_qp into A[q][p], c_qr into A[q][r], c_rq into B[q][r]
                if (v != 0.0f) atomicAdd(d == 0 ? &B[q * n + pp] : &A[q * n + pp], fixed_of(v, fbits));
                if (w != 0.0f) atomicAdd(d == 0 ? &A[q * n + rz] : &B[q * n + rz], fixed_of(w, fbits));
            } else {
                // u_pq into U[q][p] (lower triangle), u_qr into U[q][r] (upper triangle)
                if (v != 0.0f) atomicAdd(&U[q * ldu + pp], (int32_t)v);
                if (w != 0.0f) atomicAdd(&U[q * ldu + rz], (int32_t)w);
            }
        }
        __syncthreads();
    }

    // the (p, r) sums of this owner
#pragma unroll
    for (int i = 0; i < RP; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (p(i) >= n || r(j) >= n || (diag_owner && p(i) >= r(j))) continue;
            if (PASS2) {
                const double f = (double)sf[i][j] + (double)rf[i][j];
                const double g = (double)sr[i][j] + (double)rr[i][j];
                if (f != 0.0) atomicAdd(&A[p(i) * n + r(j)], to_fixed(f, scale));
                if (g != 0.0) atomicAdd(&B[p(i) * n + r(j)], to_fixed(g, scale));  // c_rp
            } else if (rf[i][j] != 0.0f) {
                atomicAdd(&U[p(i) * ldu + r(j)], (int32_t)rf[i][j]);  // p < r: upper triangle
            }
        }
}

}  // namespace pald
