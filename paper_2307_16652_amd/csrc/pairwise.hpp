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
//    single integer instructions and no select on NaN handling is needed;
//  * pass 1 uses the symmetry of U: only tiles with bx <= by run and they
//    write their transpose too;
//  * pass 2 accumulates exact half weights in float32 runs, folds each run
//    into a Kahan (sum, compensation) pair, and reduces the pair in float64
//    at the end; the worst-case relative error is below 16 * 2^-24 < 1e-6
//    (rounding of W, the run, the fold and the final store; see P2_RUN).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace pald {

constexpr uint32_t KEY_INF = 0x7f800000u;  // key of +infinity: larger than every finite key

__device__ __forceinline__ uint32_t key_of(float d) { return __float_as_uint(d) & 0x7fffffffu; }

__device__ __forceinline__ uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Per-lane condition -> 64-lane mask in a scalar register pair, and back.
// Combining compare results as masks with scalar instructions keeps vector
// selects from waiting on a mask written by the preceding vector instruction.
// Only used where every lane of the wave is active.
__device__ __forceinline__ uint64_t lane_mask(bool c) { return __builtin_amdgcn_ballot_w64(c); }
__device__ __forceinline__ bool lane_bit(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// Focus counting for one x and eight y: c[j] += [min(x, y[j]) <= a[j]].
// Written as one block so that each compare mask is read by its v_addc (as the
// carry-in) seven instructions after it is written, which covers the wait
// states a vector read of a vector-written scalar register needs; the
// compiler's own schedule puts every compare into VCC and pads each one with
// s_nop.  Registers only, no memory access.
__device__ __forceinline__ void focus_count8(int32_t (&c)[8], uint32_t x, const uint32_t (&y)[8],
                                             const uint32_t (&a)[8]) {
    uint32_t m0, m1, m2, m3, m4, m5, m6, m7;
    uint64_t k0, k1, k2, k3, k4, k5, k6, k7, co;
    asm("v_min_u32 %[m0], %[x], %[y0]\n\t"
        "v_min_u32 %[m1], %[x], %[y1]\n\t"
        "v_min_u32 %[m2], %[x], %[y2]\n\t"
        "v_min_u32 %[m3], %[x], %[y3]\n\t"
        "v_min_u32 %[m4], %[x], %[y4]\n\t"
        "v_min_u32 %[m5], %[x], %[y5]\n\t"
        "v_min_u32 %[m6], %[x], %[y6]\n\t"
        "v_min_u32 %[m7], %[x], %[y7]\n\t"
        "v_cmp_le_u32_e64 %[k0], %[m0], %[a0]\n\t"
        "v_cmp_le_u32_e64 %[k1], %[m1], %[a1]\n\t"
        "v_cmp_le_u32_e64 %[k2], %[m2], %[a2]\n\t"
        "v_cmp_le_u32_e64 %[k3], %[m3], %[a3]\n\t"
        "v_cmp_le_u32_e64 %[k4], %[m4], %[a4]\n\t"
        "v_cmp_le_u32_e64 %[k5], %[m5], %[a5]\n\t"
        "v_cmp_le_u32_e64 %[k6], %[m6], %[a6]\n\t"
        "v_cmp_le_u32_e64 %[k7], %[m7], %[a7]\n\t"
        "v_addc_co_u32_e64 %[c0], %[co], 0, %[c0], %[k0]\n\t"
        "v_addc_co_u32_e64 %[c1], %[co], 0, %[c1], %[k1]\n\t"
        "v_addc_co_u32_e64 %[c2], %[co], 0, %[c2], %[k2]\n\t"
        "v_addc_co_u32_e64 %[c3], %[co], 0, %[c3], %[k3]\n\t"
        "v_addc_co_u32_e64 %[c4], %[co], 0, %[c4], %[k4]\n\t"
        "v_addc_co_u32_e64 %[c5], %[co], 0, %[c5], %[k5]\n\t"
        "v_addc_co_u32_e64 %[c6], %[co], 0, %[c6], %[k6]\n\t"
        "v_addc_co_u32_e64 %[c7], %[co], 0, %[c7], %[k7]"
        : [c0] "+v"(c[0]), [c1] "+v"(c[1]), [c2] "+v"(c[2]), [c3] "+v"(c[3]), [c4] "+v"(c[4]),
          [c5] "+v"(c[5]), [c6] "+v"(c[6]), [c7] "+v"(c[7]), [m0] "=&v"(m0), [m1] "=&v"(m1), [m2] "=&v"(m2),
          [m3] "=&v"(m3), [m4] "=&v"(m4), [m5] "=&v"(m5), [m6] "=&v"(m6), [m7] "=&v"(m7), [k0] "=&s"(k0),
          [k1] "=&s"(k1), [k2] "=&s"(k2), [k3] "=&s"(k3), [k4] "=&s"(k4), [k5] "=&s"(k5), [k6] "=&s"(k6),
          [k7] "=&s"(k7), [co] "=&s"(co)
        : [x] "v"(x), [y0] "v"(y[0]), [y1] "v"(y[1]), [y2] "v"(y[2]), [y3] "v"(y[3]), [y4] "v"(y[4]),
          [y5] "v"(y[5]), [y6] "v"(y[6]), [y7] "v"(y[7]), [a0] "v"(a[0]), [a1] "v"(a[1]), [a2] "v"(a[2]),
          [a3] "v"(a[3]), [a4] "v"(a[4]), [a5] "v"(a[5]), [a6] "v"(a[6]), [a7] "v"(a[7]));
}

// Focus counting over the lanes for 4 x 8 pairs (x_i, y_j), p = 8 i + j, the
// 64 lanes holding 64 different z:
//     c[p] += #{lanes : min(x[i], y[j]) <= a[p]}
// with a[p] and the counts c[p] the same in every lane (c[p] in scalar
// registers).  Operands are float bit patterns compared as floats: for finite
// values >= 0 (and +inf padding) that is the order of the values, -0 equal to
// +0 (denormals are compared exactly: the kernels are built without denormal
// flushing).
//
// The vector unit makes each pair's 64-lane mask (min, compare) and the
// scalar unit counts it (popcount, add).  Vector and scalar instructions
// strictly alternate, so that one wave's scalar work issues next to another
// wave's vector work on the same SIMD, and the mask of pair p is counted
// while the mask of pair p + 2 is made: the masks of the last two pairs stay
// in k[] and are counted by the next call (k[] must be 0 before the first
// call; focus_mask_flush() counts what is left after the last).  A scalar
// read of a vector-written scalar register needs no wait states (the
// hardware interlocks it).  Registers only, no memory access; every lane
// must be active.
#define PALD_FMC(M, X, Y, Q, KP, CP, T)                                                                         \
    "v_min_f32 %[m" #M "], %[x" #X "], %[y" #Y "]\n\t"                                                      \
    "s_bcnt1_i32_b64 %[q" #Q "], %[k" #KP "]\n\t"                                                           \
    "v_cmp_le_f32_e64 %[k" #KP "], %[m" #M "], %[a" #T "]\n\t"                                              \
    "s_add_u32 %[c" #CP "], %[c" #CP "], %[q" #Q "]\n\t"
__device__ __forceinline__ void focus_mask_count32(int32_t (&c)[32], const uint32_t (&x)[4], const uint32_t (&y)[8],
                                                   const uint32_t (&a)[32], uint64_t (&k)[2]) {
    uint32_t m0, m1, m2, m3, q0, q1;
    asm(
        PALD_FMC(0, 0, 0, 0, 0, 30, 0)
        PALD_FMC(1, 0, 1, 1, 1, 31, 1)
        PALD_FMC(2, 0, 2, 0, 0, 0, 2)
        PALD_FMC(3, 0, 3, 1, 1, 1, 3)
        PALD_FMC(0, 0, 4, 0, 0, 2, 4)
        PALD_FMC(1, 0, 5, 1, 1, 3, 5)
        PALD_FMC(2, 0, 6, 0, 0, 4, 6)
        PALD_FMC(3, 0, 7, 1, 1, 5, 7)
        PALD_FMC(0, 1, 0, 0, 0, 6, 8)
        PALD_FMC(1, 1, 1, 1, 1, 7, 9)
        PALD_FMC(2, 1, 2, 0, 0, 8, 10)
        PALD_FMC(3, 1, 3, 1, 1, 9, 11)
        PALD_FMC(0, 1, 4, 0, 0, 10, 12)
        PALD_FMC(1, 1, 5, 1, 1, 11, 13)
        PALD_FMC(2, 1, 6, 0, 0, 12, 14)
        PALD_FMC(3, 1, 7, 1, 1, 13, 15)
        PALD_FMC(0, 2, 0, 0, 0, 14, 16)
        PALD_FMC(1, 2, 1, 1, 1, 15, 17)
        PALD_FMC(2, 2, 2, 0, 0, 16, 18)
        PALD_FMC(3, 2, 3, 1, 1, 17, 19)
        PALD_FMC(0, 2, 4, 0, 0, 18, 20)
        PALD_FMC(1, 2, 5, 1, 1, 19, 21)
        PALD_FMC(2, 2, 6, 0, 0, 20, 22)
        PALD_FMC(3, 2, 7, 1, 1, 21, 23)
        PALD_FMC(0, 3, 0, 0, 0, 22, 24)
        PALD_FMC(1, 3, 1, 1, 1, 23, 25)
        PALD_FMC(2, 3, 2, 0, 0, 24, 26)
        PALD_FMC(3, 3, 3, 1, 1, 25, 27)
        PALD_FMC(0, 3, 4, 0, 0, 26, 28)
        PALD_FMC(1, 3, 5, 1, 1, 27, 29)
        PALD_FMC(2, 3, 6, 0, 0, 28, 30)
        PALD_FMC(3, 3, 7, 1, 1, 29, 31)
        : [c0] "+s"(c[0]), [c1] "+s"(c[1]), [c2] "+s"(c[2]), [c3] "+s"(c[3]), [c4] "+s"(c[4]), [c5] "+s"(c[5]),
          [c6] "+s"(c[6]), [c7] "+s"(c[7]), [c8] "+s"(c[8]), [c9] "+s"(c[9]), [c10] "+s"(c[10]),
          [c11] "+s"(c[11]), [c12] "+s"(c[12]), [c13] "+s"(c[13]), [c14] "+s"(c[14]), [c15] "+s"(c[15]),
          [c16] "+s"(c[16]), [c17] "+s"(c[17]), [c18] "+s"(c[18]), [c19] "+s"(c[19]), [c20] "+s"(c[20]),
          [c21] "+s"(c[21]), [c22] "+s"(c[22]), [c23] "+s"(c[23]), [c24] "+s"(c[24]), [c25] "+s"(c[25]),
          [c26] "+s"(c[26]), [c27] "+s"(c[27]), [c28] "+s"(c[28]), [c29] "+s"(c[29]), [c30] "+s"(c[30]),
          [c31] "+s"(c[31]), [k0] "+s"(k[0]), [k1] "+s"(k[1]), [m0] "=&v"(m0), [m1] "=&v"(m1), [m2] "=&v"(m2),
          [m3] "=&v"(m3), [q0] "=&s"(q0), [q1] "=&s"(q1)
        : [x0] "v"(x[0]), [x1] "v"(x[1]), [x2] "v"(x[2]), [x3] "v"(x[3]), [y0] "v"(y[0]), [y1] "v"(y[1]),
          [y2] "v"(y[2]), [y3] "v"(y[3]), [y4] "v"(y[4]), [y5] "v"(y[5]), [y6] "v"(y[6]), [y7] "v"(y[7]),
          [a0] "v"(a[0]), [a1] "v"(a[1]), [a2] "v"(a[2]), [a3] "v"(a[3]), [a4] "v"(a[4]), [a5] "v"(a[5]),
          [a6] "v"(a[6]), [a7] "v"(a[7]), [a8] "v"(a[8]), [a9] "v"(a[9]), [a10] "v"(a[10]), [a11] "v"(a[11]),
          [a12] "v"(a[12]), [a13] "v"(a[13]), [a14] "v"(a[14]), [a15] "v"(a[15]), [a16] "v"(a[16]),
          [a17] "v"(a[17]), [a18] "v"(a[18]), [a19] "v"(a[19]), [a20] "v"(a[20]), [a21] "v"(a[21]),
          [a22] "v"(a[22]), [a23] "v"(a[23]), [a24] "v"(a[24]), [a25] "v"(a[25]), [a26] "v"(a[26]),
          [a27] "v"(a[27]), [a28] "v"(a[28]), [a29] "v"(a[29]), [a30] "v"(a[30]), [a31] "v"(a[31])
        : "scc");
}
#undef PALD_FMC

// The first block of a tile: the same masks, but each count is written (the
// popcount into the count register) instead of added, so that the 32 counts
// need no zeroing; pairs 30 and 31, whose masks the block leaves in k[], start
// at 0.  No k[] on entry.
#define PALD_FMF0(M, X, Y, KP, CP, T)                                                                           \
    "v_min_f32 %[m" #M "], %[x" #X "], %[y" #Y "]\n\t"                                                      \
    "s_mov_b32 %[c" #CP "], 0\n\t"                                                                           \
    "v_cmp_le_f32_e64 %[k" #KP "], %[m" #M "], %[a" #T "]\n\t"
#define PALD_FMF(M, X, Y, KP, CP, T)                                                                            \
    "v_min_f32 %[m" #M "], %[x" #X "], %[y" #Y "]\n\t"                                                      \
    "s_bcnt1_i32_b64 %[c" #CP "], %[k" #KP "]\n\t"                                                          \
    "v_cmp_le_f32_e64 %[k" #KP "], %[m" #M "], %[a" #T "]\n\t"
__device__ __forceinline__ void focus_mask_count32_first(int32_t (&c)[32], const uint32_t (&x)[4],
                                                         const uint32_t (&y)[8], const uint32_t (&a)[32],
                                                         uint64_t (&k)[2]) {
    uint32_t m0, m1, m2, m3;
    asm(
        PALD_FMF0(0, 0, 0, 0, 30, 0)
        PALD_FMF0(1, 0, 1, 1, 31, 1)
        PALD_FMF(2, 0, 2, 0, 0, 2)
        PALD_FMF(3, 0, 3, 1, 1, 3)
        PALD_FMF(0, 0, 4, 0, 2, 4)
        PALD_FMF(1, 0, 5, 1, 3, 5)
        PALD_FMF(2, 0, 6, 0, 4, 6)
        PALD_FMF(3, 0, 7, 1, 5, 7)
        PALD_FMF(0, 1, 0, 0, 6, 8)
        PALD_FMF(1, 1, 1, 1, 7, 9)
        PALD_FMF(2, 1, 2, 0, 8, 10)
        PALD_FMF(3, 1, 3, 1, 9, 11)
        PALD_FMF(0, 1, 4, 0, 10, 12)
        PALD_FMF(1, 1, 5, 1, 11, 13)
        PALD_FMF(2, 1, 6, 0, 12, 14)
        PALD_FMF(3, 1, 7, 1, 13, 15)
        PALD_FMF(0, 2, 0, 0, 14, 16)
        PALD_FMF(1, 2, 1, 1, 15, 17)
        PALD_FMF(2, 2, 2, 0, 16, 18)
        PALD_FMF(3, 2, 3, 1, 17, 19)
        PALD_FMF(0, 2, 4, 0, 18, 20)
        PALD_FMF(1, 2, 5, 1, 19, 21)
        PALD_FMF(2, 2, 6, 0, 20, 22)
        PALD_FMF(3, 2, 7, 1, 21, 23)
        PALD_FMF(0, 3, 0, 0, 22, 24)
        PALD_FMF(1, 3, 1, 1, 23, 25)
        PALD_FMF(2, 3, 2, 0, 24, 26)
        PALD_FMF(3, 3, 3, 1, 25, 27)
        PALD_FMF(0, 3, 4, 0, 26, 28)
        PALD_FMF(1, 3, 5, 1, 27, 29)
        PALD_FMF(2, 3, 6, 0, 28, 30)
        PALD_FMF(3, 3, 7, 1, 29, 31)
        : [c0] "=&s"(c[0]), [c1] "=&s"(c[1]), [c2] "=&s"(c[2]), [c3] "=&s"(c[3]), [c4] "=&s"(c[4]),
          [c5] "=&s"(c[5]), [c6] "=&s"(c[6]), [c7] "=&s"(c[7]), [c8] "=&s"(c[8]), [c9] "=&s"(c[9]),
          [c10] "=&s"(c[10]), [c11] "=&s"(c[11]), [c12] "=&s"(c[12]), [c13] "=&s"(c[13]), [c14] "=&s"(c[14]),
          [c15] "=&s"(c[15]), [c16] "=&s"(c[16]), [c17] "=&s"(c[17]), [c18] "=&s"(c[18]), [c19] "=&s"(c[19]),
          [c20] "=&s"(c[20]), [c21] "=&s"(c[21]), [c22] "=&s"(c[22]), [c23] "=&s"(c[23]), [c24] "=&s"(c[24]),
          [c25] "=&s"(c[25]), [c26] "=&s"(c[26]), [c27] "=&s"(c[27]), [c28] "=&s"(c[28]), [c29] "=&s"(c[29]),
          [c30] "=&s"(c[30]), [c31] "=&s"(c[31]), [k0] "=&s"(k[0]), [k1] "=&s"(k[1]), [m0] "=&v"(m0),
          [m1] "=&v"(m1), [m2] "=&v"(m2), [m3] "=&v"(m3)
        : [x0] "v"(x[0]), [x1] "v"(x[1]), [x2] "v"(x[2]), [x3] "v"(x[3]), [y0] "v"(y[0]), [y1] "v"(y[1]),
          [y2] "v"(y[2]), [y3] "v"(y[3]), [y4] "v"(y[4]), [y5] "v"(y[5]), [y6] "v"(y[6]), [y7] "v"(y[7]),
          [a0] "v"(a[0]), [a1] "v"(a[1]), [a2] "v"(a[2]), [a3] "v"(a[3]), [a4] "v"(a[4]), [a5] "v"(a[5]),
          [a6] "v"(a[6]), [a7] "v"(a[7]), [a8] "v"(a[8]), [a9] "v"(a[9]), [a10] "v"(a[10]), [a11] "v"(a[11]),
          [a12] "v"(a[12]), [a13] "v"(a[13]), [a14] "v"(a[14]), [a15] "v"(a[15]), [a16] "v"(a[16]),
          [a17] "v"(a[17]), [a18] "v"(a[18]), [a19] "v"(a[19]), [a20] "v"(a[20]), [a21] "v"(a[21]),
          [a22] "v"(a[22]), [a23] "v"(a[23]), [a24] "v"(a[24]), [a25] "v"(a[25]), [a26] "v"(a[26]),
          [a27] "v"(a[27]), [a28] "v"(a[28]), [a29] "v"(a[29]), [a30] "v"(a[30]), [a31] "v"(a[31]));
}
#undef PALD_FMF0
#undef PALD_FMF

// The two masks focus_mask_count32 leaves in k[] (pairs 30 and 31).
__device__ __forceinline__ void focus_mask_flush(int32_t (&c)[32], const uint64_t (&k)[2]) {
    c[30] += __builtin_popcountll(k[0]);
    c[31] += __builtin_popcountll(k[1]);
}

// Cohesion terms of one x and four z for one second point y, both
// directions, as EXEC-masked additions of half weights.  With the keys
// t_j = d_x z_j, a = d_xy, b_j = d_z_j y and the half weights hx = W_xy / 2,
// hz_j = W_z_j y / 2, pair j takes four compares
//     i = [t_j <= a],  j = [t_j <= b_j],  p = [t_j < b_j],  q = [t_j < a]
// and adds
//     rf_j += hx    under i & j, and again under i & p   (c_xz: W_xy if t < b, W_xy/2 on a tie)
//     rr_j += hz_j  under i & j, and again under j & q   (c_zx: W_zy if t < a, W_zy/2 on a tie)
// i & j is focus membership, [t <= min(a, b)]; p implies j and q implies i,
// so i & p and j & q are membership together with the strict order.
//
// The compares run under the caller's EXEC and leave 0 in inactive lanes, so
// no mask enables a lane that was off; the scalar unit sets EXEC to each mask
// in turn and restores `full` (the caller's EXEC) at the end of a group of G
// pairs.  On gfx950 compares take the vector unit about 4 cycles per wave
// instruction while float32 additions issue beside them, so four compares and
// four masked additions cost little more than the compares alone -- less
// than a min, three compares, two selects of W or W/2 and two additions.
// G = 4 keeps 16 masks (32 scalar registers) live; G = 2 half of that, for
// kernels short of scalar registers.  Registers only, no memory access.
#define PALD_H_CMP(k)                                                                                            \
    "v_cmp_le_u32_e64 %[i" #k "], %[t" #k "], %[a]\n\t"                                                       \
    "v_cmp_le_u32_e64 %[j" #k "], %[t" #k "], %[b" #k "]\n\t"                                                 \
    "v_cmp_lt_u32_e64 %[p" #k "], %[t" #k "], %[b" #k "]\n\t"                                                 \
    "v_cmp_lt_u32_e64 %[q" #k "], %[t" #k "], %[a]\n\t"
#define PALD_H_ADD(k)                                                                                            \
    "s_and_b64 exec, %[i" #k "], %[j" #k "]\n\t"                                                              \
    "v_add_f32 %[rf" #k "], %[rf" #k "], %[hx]\n\t"                                                           \
    "v_add_f32 %[rr" #k "], %[rr" #k "], %[hz" #k "]\n\t"                                                     \
    "s_and_b64 exec, %[i" #k "], %[p" #k "]\n\t"                                                              \
    "v_add_f32 %[rf" #k "], %[rf" #k "], %[hx]\n\t"                                                           \
    "s_and_b64 exec, %[j" #k "], %[q" #k "]\n\t"                                                              \
    "v_add_f32 %[rr" #k "], %[rr" #k "], %[hz" #k "]\n\t"
#define PALD_H_ADD2(k)                                                                                           \
    "s_and_b64 exec, %[i" #k "], %[j" #k "]\n\t"                                                              \
    "v_add_f32 %[rf" #k "], %[rf" #k "], %[hx]\n\t"                                                           \
    "v_add_f32 %[rr" #k "], %[rr" #k "], %[hz" #k "]\n\t"                                                     \
    "s_and_b64 exec, %[i" #k "], %[p" #k "]\n\t"                                                              \
    "v_add_f32 %[gf" #k "], %[gf" #k "], %[hx]\n\t"                                                           \
    "s_and_b64 exec, %[j" #k "], %[q" #k "]\n\t"                                                              \
    "v_add_f32 %[gr" #k "], %[gr" #k "], %[hz" #k "]\n\t"
#define PALD_H_MASKS(k) [i##k] "=&s"(mi[k]), [j##k] "=&s"(mj[k]), [p##k] "=&s"(mp[k]), [q##k] "=&s"(mq[k])
#define PALD_H_ACC(k) [rf##k] "+v"(rf[k]), [rr##k] "+v"(rr[k])
#define PALD_H_ACC2(k) [gf##k] "+v"(gf[k]), [gr##k] "+v"(gr[k])
#define PALD_H_IN(k) [t##k] "v"(t[k]), [b##k] "v"(b[k]), [hz##k] "v"(hz[k])
template <int G>
__device__ __forceinline__ void cohesion_terms4(float (&rf)[4], float (&rr)[4], const uint32_t (&t)[4], uint32_t a,
                                                const uint32_t (&b)[4], float hx, const float (&hz)[4],
                                                uint64_t full) {
    static_assert(G == 2 || G == 4, "groups of 2 or 4 pairs");
    uint64_t mi[4], mj[4], mp[4], mq[4];
    if constexpr (G == 4) {
        asm(PALD_H_CMP(0) PALD_H_CMP(1) PALD_H_CMP(2) PALD_H_CMP(3)
            PALD_H_ADD(0) PALD_H_ADD(1) PALD_H_ADD(2) PALD_H_ADD(3)
            "s_mov_b64 exec, %[full]"
            : PALD_H_ACC(0), PALD_H_ACC(1), PALD_H_ACC(2), PALD_H_ACC(3),
              PALD_H_MASKS(0), PALD_H_MASKS(1), PALD_H_MASKS(2), PALD_H_MASKS(3)
            : [a] "v"(a), [hx] "v"(hx), [full] "s"(full), PALD_H_IN(0), PALD_H_IN(1), PALD_H_IN(2), PALD_H_IN(3)
            : "scc");
    } else {
        asm(PALD_H_CMP(0) PALD_H_CMP(1) PALD_H_ADD(0) PALD_H_ADD(1)
            "s_mov_b64 exec, %[full]"
            : PALD_H_ACC(0), PALD_H_ACC(1), PALD_H_MASKS(0), PALD_H_MASKS(1)
            : [a] "v"(a), [hx] "v"(hx), [full] "s"(full), PALD_H_IN(0), PALD_H_IN(1)
            : "scc");
        asm(PALD_H_CMP(2) PALD_H_CMP(3) PALD_H_ADD(2) PALD_H_ADD(3)
            "s_mov_b64 exec, %[full]"
            : PALD_H_ACC(2), PALD_H_ACC(3), PALD_H_MASKS(2), PALD_H_MASKS(3)
            : [a] "v"(a), [hx] "v"(hx), [full] "s"(full), PALD_H_IN(2), PALD_H_IN(3)
            : "scc");
    }
}
// The same block with the second half weight of each term added to its own
// accumulators gf (c_xz) and gr (c_zx), so that every accumulator receives at
// most one addition per y (G = 4).
__device__ __forceinline__ void cohesion_terms4_split(float (&rf)[4], float (&rr)[4], float (&gf)[4], float (&gr)[4],
                                                      const uint32_t (&t)[4], uint32_t a, const uint32_t (&b)[4],
                                                      float hx, const float (&hz)[4], uint64_t full) {
    uint64_t mi[4], mj[4], mp[4], mq[4];
    asm(PALD_H_CMP(0) PALD_H_CMP(1) PALD_H_CMP(2) PALD_H_CMP(3)
        PALD_H_ADD2(0) PALD_H_ADD2(1) PALD_H_ADD2(2) PALD_H_ADD2(3)
        "s_mov_b64 exec, %[full]"
        : PALD_H_ACC(0), PALD_H_ACC(1), PALD_H_ACC(2), PALD_H_ACC(3), PALD_H_ACC2(0), PALD_H_ACC2(1), PALD_H_ACC2(2),
          PALD_H_ACC2(3), PALD_H_MASKS(0), PALD_H_MASKS(1), PALD_H_MASKS(2), PALD_H_MASKS(3)
        : [a] "v"(a), [hx] "v"(hx), [full] "s"(full), PALD_H_IN(0), PALD_H_IN(1), PALD_H_IN(2), PALD_H_IN(3)
        : "scc");
}
#undef PALD_H_CMP
#undef PALD_H_ADD
#undef PALD_H_ADD2
#undef PALD_H_MASKS
#undef PALD_H_ACC
#undef PALD_H_ACC2
#undef PALD_H_IN

// threadIdx.x, passed through an empty volatile asm: values derived from it
// are then recomputed where a tile function is called instead of being
// hoisted out of an enclosing loop (the persistent batched kernel calls the
// tile functions once per work item; hoisted, those values would stay live
// across every tile and push the kernel past its register budget).
__device__ __forceinline__ int opaque_tid() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Upper-triangular tile enumeration: k -> (bx, by) with bx <= by, by-major.
__device__ __forceinline__ void tri_tile(int32_t k, int32_t &bx, int32_t &by) {
    int32_t r = (int32_t)((sqrtf(8.0f * (float)k + 1.0f) - 1.0f) * 0.5f);
    while ((int64_t)r * (r + 1) / 2 > k) --r;
    while ((int64_t)(r + 1) * (r + 2) / 2 <= k) ++r;
    by = r;
    bx = k - (int32_t)((int64_t)r * (r + 1) / 2);
}

// Launch order of the upper-triangular tiles, chosen for L2 reuse.
//
// Consecutive workgroups are dealt round robin over the 8 XCDs, each with its
// own L2.  xcd_order() makes every XCD take a contiguous run of the order
// instead (workgroup w of N runs on XCD w % 8 and gets position
// (w % 8) * (N / 8) + ... + w / 8, a bijection of [0, N)), and grouped_tile()
// lists the tiles by G x G groups (by rows of groups, tiles inside a group by
// rows), so the tiles an XCD runs at the same time share a few row panels of
// D and W in its L2 instead of each streaming its own.
constexpr int TILE_GROUP = 8;
constexpr int NUM_XCD = 8;

__device__ __forceinline__ int32_t xcd_order(int32_t w, int32_t N) {
    const int32_t q = N / NUM_XCD, r = N % NUM_XCD, c = w % NUM_XCD, i = w / NUM_XCD;
    return c * q + min(c, r) + i;
}

// k -> (bx, bz), bx <= bz < nb: the k-th tile in the grouped order.
__device__ __forceinline__ void grouped_tile(int32_t k, int32_t nb, int32_t &bx, int32_t &bz) {
    constexpr int64_t G = TILE_GROUP;
    const int64_t nsb = (nb + G - 1) / G;
    // tiles in the group rows before row S (all full): G^2 S(S-1)/2 + S G(G+1)/2
    auto P = [&](int64_t S) { return G * G * S * (S - 1) / 2 + S * G * (G + 1) / 2; };
    const double qa = 0.5 * G * G, qb = 0.5 * G * (G + 1) - 0.5 * G * G;
    int64_t S = k > 0 ? (int64_t)((-qb + sqrt(qb * qb + 4.0 * qa * (double)k)) / (2.0 * qa)) : 0;
    S = max((int64_t)0, min(S, nsb - 1));
    while (S > 0 && P(S) > k) --S;
    while (S + 1 < nsb && P(S + 1) <= k) ++S;
    const int64_t wz = min(G, (int64_t)nb - S * G);
    const int64_t rem = k - P(S), off = S * G * wz;
    if (rem < off) {  // a full G-wide group left of the diagonal
        const int64_t sx = rem / (G * wz), loc = rem % (G * wz);
        bx = (int32_t)(sx * G + loc % G);
        bz = (int32_t)(S * G + loc / G);
    } else {          // the diagonal group: its own upper triangle
        int32_t lx, lz;
        tri_tile((int32_t)(rem - off), lx, lz);
        bx = (int32_t)(S * G + lx);
        bz = (int32_t)(S * G + lz);
    }
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

// 4 consecutive floats of row `row` from column `col` as raw bit patterns;
// out-of-range rows/columns give `fill`.
__device__ __forceinline__ uint4 load_raw4(const float *__restrict__ M, int64_t ld, int64_t row, int64_t col,
                                           int64_t nrows, int64_t ncols, bool vec_ok, uint32_t fill) {
    uint4 r = make_uint4(fill, fill, fill, fill);
    if (row >= nrows) return r;
    const float *p = M + row * ld + col;
    if (vec_ok && col + 3 < ncols) return *reinterpret_cast<const uint4 *>(p);
    if (col + 0 < ncols) r.x = __float_as_uint(p[0]);
    if (col + 1 < ncols) r.y = __float_as_uint(p[1]);
    if (col + 2 < ncols) r.z = __float_as_uint(p[2]);
    if (col + 3 < ncols) r.w = __float_as_uint(p[3]);
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
// Grid: blockIdx.x picks an upper-triangular T x T tile (bx <= by) in the
// grouped, XCD-contiguous order of grouped_tile() / xcd_order(), offset by
// tile0 (large grids are launched in pieces); blockIdx.y is the z-chunk.
// With one z-chunk the tile writes U (and,
// if W != nullptr, the weights W) directly; with several it atomically adds
// its counts into U, which must be zero on entry.

// minimum waves per SIMD the pass-1 kernel is compiled for (its VGPR budget)
#ifndef PALD_P1_MIN_WAVES
#define PALD_P1_MIN_WAVES 4
#endif
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
    static_assert(RY == 8, "focus counting works on rows of 8 y");
    static constexpr int LDS_VEC = 2 * VEC_PER_CHUNK;  // uint4 of LDS, double-buffered
};

// One pass-1 tile (bx, by), bx <= by, over the z range [zbeg, zend).  Called
// by every thread of a workgroup of Pass1Cfg::NT threads; `sm` points to
// Pass1Cfg::LDS_VEC uint4 of LDS.  U may be null in direct mode.
template <int T, int RX, int RY, int KZ>
__device__ __forceinline__ void pass1_tile(int tid, uint4 *sm, const float *__restrict__ D, int64_t n, int64_t ldd,
                                           int32_t *__restrict__ U, int64_t ldu, float *__restrict__ W, int64_t ldw,
                                           int32_t bx, int32_t by, int64_t zbeg, int64_t zend, bool atomic_mode,
                                           bool vec_ok) {
    using Cfg = Pass1Cfg<T, RX, RY, KZ>;
    const int64_t X0 = (int64_t)bx * T, Y0 = (int64_t)by * T;
    const int tx = tid % Cfg::TX, ty = tid / Cfg::TX;

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
            pre[k] = load_keys4(D, ldd, z, col, zend, n, vec_ok, KEY_INF);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int k = 0; k < Cfg::VEC_PER_THREAD; ++k) sm[buf * Cfg::VEC_PER_CHUNK + tid + k * Cfg::NT] = pre[k];
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
        const uint32_t *s = reinterpret_cast<const uint32_t *>(sm + buf * Cfg::VEC_PER_CHUNK);
#pragma unroll 1
        for (int z = 0; z < KZ; ++z) {
            uint32_t xs[RX], ys[RY];
#pragma unroll
            for (int i = 0; i < RX; ++i) xs[i] = s[z * Cfg::ROW + tx * RX + i];
#pragma unroll
            for (int j = 0; j < RY; ++j) ys[j] = s[z * Cfg::ROW + T + ty * RY + j];
#pragma unroll
            for (int i = 0; i < RX; ++i) focus_count8(cnt[i], xs[i], ys, a[i]);
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

template <int T, int RX, int RY, int KZ>
__global__ __launch_bounds__((Pass1Cfg<T, RX, RY, KZ>::NT), PALD_P1_MIN_WAVES) void pass1_focus_kernel(
    const float *__restrict__ D, int64_t n, int64_t ldd, int32_t *__restrict__ U, int64_t ldu,
    float *__restrict__ W, int64_t ldw, int32_t z_per_chunk, int32_t atomic_mode, int32_t vec_ok, int32_t tile0) {
    using Cfg = Pass1Cfg<T, RX, RY, KZ>;
    __shared__ uint4 sm[Cfg::LDS_VEC];
    int32_t bx, by;
    grouped_tile(tile0 + xcd_order((int32_t)blockIdx.x, (int32_t)gridDim.x), (int32_t)((n + T - 1) / T), bx, by);
    const int64_t zbeg = (int64_t)blockIdx.y * z_per_chunk;
    const int64_t zend = min(n, zbeg + (int64_t)z_per_chunk);
    pass1_tile<T, RX, RY, KZ>((int)threadIdx.x, sm, D, n, ldd, U, ldu, W, ldw, bx, by, zbeg, zend, atomic_mode != 0, vec_ok != 0);
}

// ---------------------------------------------------------------------------
// Pass 1 with the lanes of a wave running over z.
//
// The kernel above gives every lane its own (x, y) pairs and streams z, which
// costs three vector instructions per (x, y, z): min, compare, add-with-carry.
// Here a wave owns 4 x 8 pairs whose keys d_xy are the same in every lane,
// and its 64 lanes hold 64 different z.  One min and one compare per pair
// give the 64-lane membership mask of a whole z block, and the scalar unit
// counts it (popcount + add into a per-pair scalar register).  That leaves two
// vector instructions per 64 (x, y, z) and moves the counting to the scalar
// unit, which issues alongside the vector unit from the other waves of the
// SIMD.
//
// A tile counts all of its pairs but writes only those with x <= y, and
// their mirror images.  Each stage stages ZS z of the TX + TY rows of D the
// tile reads (d_zx = D[x][z] by symmetry) through LDS; lane l works on
// z = NC l + c, c < NC, of each of its wave's 12 rows (one block of 32 pairs
// per c).
//
// Configuration of a lanes-over-z pass-1 tile: GX x GY waves of 4 x 8 pairs
// (TX = 4 GX x, TY = 8 GY y), NC z per lane and stage (ZS = 64 NC z staged
// per stage for the TX + TY rows of the tile).
template <int GX, int GY, int NC>
struct P1zCfg {
    static constexpr int WX = 4, WY = 8;
    static constexpr int TX = WX * GX, TY = WY * GY;
    static constexpr int NW = GX * GY;          // waves
    static constexpr int NT = 64 * NW;          // threads
    static constexpr int ZS = 64 * NC;          // z per stage
    static constexpr int ROWS = TX + TY;        // staged rows
    static constexpr int ROWS_PER_WAVE = ROWS / NW;  // rows each wave loads per stage
    static constexpr int LDS_WORDS = 2 * ROWS * ZS;  // double-buffered stage (uint32)
    static_assert(ROWS % NW == 0, "the staged rows must split evenly over the waves");
    static_assert(NC == 2 || NC == 4, "2 or 4 z per lane");
};

// NC consecutive floats per lane as raw bits (a uint2 or a uint4).
template <int NC>
struct P1zVec;
template <>
struct P1zVec<4> {
    uint32_t v[4];
};
template <>
struct P1zVec<2> {
    uint32_t v[2];
};

// The staged values one thread loads for one stage.
template <int RPW, int NC>
struct P1zStage {
    P1zVec<NC> r[RPW];
};

// Where a lanes-over-z pass-1 tile finds its rows of D: row x, x in
// [xlo, xhi), at Dx + (x - xlo) ldx and row y, y in [ylo, yhi), at
// Dy + (y - ylo) ldy, every row holding all n columns (d_zx = D[x][z] by
// symmetry).  For the whole matrix Dx = Dy = D, xlo = ylo = 0, xhi = yhi = n;
// a row panel or a streamed block of rows passes its own buffers.
struct P1Rows {
    const float *Dx;
    int64_t ldx, xlo, xhi;
    const float *Dy;
    int64_t ldy, ylo, yhi;
};

// Stage fetch for a stage that reaches past zend (or unaligned rows), whole
// matrix: bounds-checked loads, +inf outside.  Kept out of line so that the
// full-stage loads stay plain vector loads, and with few arguments: a call
// passes them in vector registers, which count against the kernel's budget.
// Row q of this wave is tile row wave + q NW (x rows first, then y rows);
// lane l loads z = zs + NC l + c.
template <int GX, int GY, int NC>
__device__ __noinline__ P1zStage<P1zCfg<GX, GY, NC>::ROWS_PER_WAVE, NC> p1z_fetch_edge(
    const float *__restrict__ D, int64_t ldd, int64_t n, int64_t X0, int64_t Y0, int wave, int lane, int64_t zs,
    int64_t zend, bool vec_ok) {
    using Cfg = P1zCfg<GX, GY, NC>;
    P1zStage<Cfg::ROWS_PER_WAVE, NC> out;
#pragma unroll
    for (int q = 0; q < Cfg::ROWS_PER_WAVE; ++q) {
        const int r = wave + q * Cfg::NW;
        const int64_t row = r < Cfg::TX ? X0 + r : Y0 + (r - Cfg::TX);
        const int64_t z0 = zs + (int64_t)NC * lane;
        if (NC == 4) {
            const uint4 v = load_raw4(D, ldd, row, z0, n, zend, vec_ok, KEY_INF);
            out.r[q].v[0] = v.x;
            out.r[q].v[NC > 1 ? 1 : 0] = v.y;
            out.r[q].v[NC > 2 ? 2 : 0] = v.z;
            out.r[q].v[NC > 3 ? 3 : 0] = v.w;
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c)
                out.r[q].v[c] = (row < n && z0 + c < zend) ? __float_as_uint(D[row * ldd + z0 + c]) : KEY_INF;
        }
    }
    return out;
}

// The same for a block of rows (RECT tiles): x row r of the tile (r < xrows
// exist) at xb + r ldx, y row r (r < yrows) at yb + r ldy.
template <int GX, int GY, int NC>
__device__ __noinline__ P1zStage<P1zCfg<GX, GY, NC>::ROWS_PER_WAVE, NC> p1z_fetch_edge_rows(
    const float *__restrict__ xb, int64_t ldx, int32_t xrows, const float *__restrict__ yb, int64_t ldy, int32_t yrows,
    int wave, int lane, int64_t zs, int64_t zend, bool vec_ok) {
    using Cfg = P1zCfg<GX, GY, NC>;
    P1zStage<Cfg::ROWS_PER_WAVE, NC> out;
#pragma unroll
    for (int q = 0; q < Cfg::ROWS_PER_WAVE; ++q) {
        const int r = wave + q * Cfg::NW;
        const bool is_x = r < Cfg::TX;
        const int rr = is_x ? r : r - Cfg::TX;
        const bool valid = rr < (is_x ? xrows : yrows);
        const float *base = is_x ? xb + rr * ldx : yb + rr * ldy;
        const int64_t z0 = zs + (int64_t)NC * lane;
        if (NC == 4) {
            const uint4 v = load_raw4(base, 0, 0, z0, valid ? 1 : 0, zend, vec_ok, KEY_INF);
            out.r[q].v[0] = v.x;
            out.r[q].v[NC > 1 ? 1 : 0] = v.y;
            out.r[q].v[NC > 2 ? 2 : 0] = v.z;
            out.r[q].v[NC > 3 ? 3 : 0] = v.w;
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c)
                out.r[q].v[c] = (valid && z0 + c < zend) ? __float_as_uint(base[z0 + c]) : KEY_INF;
        }
    }
    return out;
}

// One lanes-over-z pass-1 tile: pairs x in [X0, X0 + TX), y in [Y0, Y0 + TY),
// z over [zbeg, zend), rows of D as described by g.  Called by every thread
// of a workgroup of Cfg::NT threads (tid = thread index); `smw` points to
// Cfg::LDS_WORDS words of LDS.  Square mode (RECT false, whole matrix): writes
// U (if non-null) and W (if non-null) for the tile's pairs with x <= y and
// their mirror images, or, in atomic mode, adds the counts into U.  RECT
// (a block of rows x): writes every pair x < xhi, y < yhi of the tile, U at
// U[(x - xlo) ldu + y] and the weight transposed, W[y ldw + (x - xlo)]; no
// atomic mode.  Ends with a workgroup barrier, so the LDS can be reused at
// once.  AHEAD: the next z component's values are read from LDS while the
// block of the current one runs (12 more VGPRs); without it the waves of the
// SIMD cover that latency, which pays where the tile fits 8 waves per SIMD.
template <int GX, int GY, int NC, bool RECT = false, bool AHEAD = true>
__device__ __forceinline__ void pass1z_tile_g(int tid, uint32_t *smw, const P1Rows g, int64_t n,
                                              int32_t *__restrict__ U, int64_t ldu, float *__restrict__ W,
                                              int64_t ldw, int64_t X0, int64_t Y0, int64_t zbeg, int64_t zend,
                                              bool atomic_mode, bool vec_ok) {
    using Cfg = P1zCfg<GX, GY, NC>;
    constexpr int RPW = Cfg::ROWS_PER_WAVE;
    // (the lane index from the lane counter rather than from tid, so that no
    // register has to hold tid across the tile)
    const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wx = wave % GX, wy = wave / GX;
    const int64_t xw = X0 + wx * Cfg::WX, yw = Y0 + wy * Cfg::WY;

    // d_xy of every pair (the same in every lane), kept in vector registers so
    // that the scalar file holds only the counts; values stay float bit
    // patterns (focus_mask_count32 compares them as floats).  Pair p = 8 i + j
    // is (x, y) = (xw + i, yw + j).
    uint32_t t[Cfg::WX * Cfg::WY];
    int32_t cnt[Cfg::WX * Cfg::WY];  // written by the tile's first block (or zeroed if it has none)
    uint64_t carry[2];
    static_assert(Cfg::NW * Cfg::WX * Cfg::WY <= Cfg::ROWS * Cfg::ZS, "the keys fit in one stage buffer");
    // Lane p < 32 loads the key of pair p (row and column clamped into the
    // matrix: a pair outside it is counted but never written) and the wave
    // passes the 32 keys to every lane through LDS: one vector load and a few
    // LDS instructions instead of 32 scalar loads and their 64-bit address
    // arithmetic on the scalar unit, which also does the counting (per tile
    // and wave, 213 scalar instructions before the stage loop instead of
    // 508).  The keys sit in the second stage buffer, which the first stage
    // leaves alone and the stage loop first writes after a barrier.  The key
    // goes to LDS (take_keys) after the first stage's loads are issued, so
    // that the two loads are in flight together.
    uint32_t *kw = smw + Cfg::ROWS * Cfg::ZS + wave * (Cfg::WX * Cfg::WY);
    auto load_key = [&]() {
        uint32_t key = 0;
        if (lane < Cfg::WX * Cfg::WY) {
            const int64_t x = min(xw + lane / Cfg::WY, g.xhi - 1), y = min(yw + lane % Cfg::WY, n - 1);
            key = __float_as_uint(g.Dx[(x - g.xlo) * g.ldx + y]);
        }
        return key;
    };
    auto take_keys = [&](uint32_t key) {
        if (lane < Cfg::WX * Cfg::WY) kw[lane] = key;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int p = 0; p < Cfg::WX * Cfg::WY; ++p) t[p] = kw[p];
    };

    const int32_t nst = (int32_t)((zend - zbeg + Cfg::ZS - 1) / Cfg::ZS);
    // Stages that lie inside [zbeg, zend) of a tile whose rows all exist load
    // from fixed row pointers and one 32-bit offset, without checks (vector
    // loads when the rows are 16-byte aligned, else one load per value); the
    // others go through the bounds-checked p1z_fetch_edge().
    const bool rows_in = X0 + Cfg::TX <= g.xhi && Y0 + Cfg::TY <= g.yhi;
    const int32_t nst_fast = rows_in ? (int32_t)((zend - zbeg) / Cfg::ZS) : 0;  // leading stages needing no checks
    // Row pointers of the stages without checks.  Those run only when every
    // row of the tile exists, so the rows need no clamping here; the 64-bit
    // arithmetic is a product per tile and side plus a small one per row, all
    // of it wave-uniform (scalar unit).
    // (Row q of the wave is tile row wave + q NW: its first TX / NW rows are
    // x rows, the rest y rows.)
    static_assert(Cfg::TX % Cfg::NW == 0, "each wave's rows are x rows, then y rows");
    const char *rowp[RPW];
    {
        constexpr int QX = Cfg::TX / Cfg::NW;
        const uint64_t ldx4 = (uint64_t)g.ldx * sizeof(float), ldy4 = (uint64_t)g.ldy * sizeof(float);
        const uint64_t z4 = (uint64_t)zbeg * sizeof(float);
        const char *bx = reinterpret_cast<const char *>(g.Dx) + (uint64_t)(X0 - g.xlo + wave) * ldx4 + z4;
        const char *by = reinterpret_cast<const char *>(g.Dy) + (uint64_t)(Y0 - g.ylo + wave) * ldy4 + z4;
#pragma unroll
        for (int q = 0; q < RPW; ++q)
            rowp[q] = q < QX ? bx + (uint64_t)(q * Cfg::NW) * ldx4 : by + (uint64_t)((q - QX) * Cfg::NW) * ldy4;
    }
    // The stage loop, instantiated for aligned rows (VEC: vector loads) and for
    // unaligned ones (one load per value); one tile runs one of the two.
    auto run = [&](auto vec_tag) {
        constexpr bool VEC = decltype(vec_tag)::value;
        P1zStage<RPW, NC> pre;
        // stage st with no checks (st < nst_fast); `off` is its byte offset in
        // the rows, below 4 n (and n x n floats fit in memory)
        auto fetch_fast = [&](uint32_t off) {
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                if constexpr (!VEC) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        pre.r[q].v[c] = __float_as_uint(reinterpret_cast<const float *>(rowp[q] + off)[c]);
                } else if constexpr (NC == 4) {
                    const float4 v = *reinterpret_cast<const float4 *>(rowp[q] + off);
                    pre.r[q].v[0] = __float_as_uint(v.x);
                    pre.r[q].v[1] = __float_as_uint(v.y);
                    pre.r[q].v[2] = __float_as_uint(v.z);
                    pre.r[q].v[3] = __float_as_uint(v.w);
                } else {
                    const float2 v = *reinterpret_cast<const float2 *>(rowp[q] + off);
                    pre.r[q].v[0] = __float_as_uint(v.x);
                    pre.r[q].v[1] = __float_as_uint(v.y);
                }
            }
        };
        constexpr uint32_t STAGE_BYTES = Cfg::ZS * sizeof(float);
        const uint32_t lane_off = (uint32_t)NC * (uint32_t)lane * (uint32_t)sizeof(float);
        // the partial last stage of a tile whose rows all exist: the row
        // pointers of the stages without checks, each z clamped to the last
        // one (so that every load stays inside the row) and +inf put in place
        // of the values past it -- a few instructions per value instead of the
        // bounds-checked fetch with its 64-bit row arithmetic
        auto fetch_tail = [&](int32_t st) {
            const int32_t zlast = (int32_t)(zend - 1 - zbeg);  // z of the last value, relative to zbeg
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int32_t z = st * Cfg::ZS + NC * lane + c;
                const bool ok = z <= zlast;
                const uint32_t zo = (uint32_t)(ok ? z : zlast) * (uint32_t)sizeof(float);
#pragma unroll
                for (int q = 0; q < RPW; ++q) {
                    const uint32_t v = *reinterpret_cast<const uint32_t *>(rowp[q] + zo);
                    pre.r[q].v[c] = ok ? v : KEY_INF;
                }
            }
        };
        auto fetch = [&](int32_t st) {  // stage st: z = zbeg + ZS st + ...
            if (st < nst_fast)
                fetch_fast((uint32_t)st * STAGE_BYTES + lane_off);
            else if (rows_in)
                fetch_tail(st);
            else
                if constexpr (RECT)
                    pre = p1z_fetch_edge_rows<GX, GY, NC>(
                        g.Dx + (X0 - g.xlo) * g.ldx, g.ldx, (int32_t)min((int64_t)Cfg::TX, g.xhi - X0),
                        g.Dy + (Y0 - g.ylo) * g.ldy, g.ldy, (int32_t)min((int64_t)Cfg::TY, g.yhi - Y0), wave, lane,
                        zbeg + (int64_t)st * Cfg::ZS, zend, VEC);
                else  // whole matrix: g.Dx = g.Dy, rows [0, n)
                    pre = p1z_fetch_edge<GX, GY, NC>(g.Dx, g.ldx, n, X0, Y0, wave, lane,
                                                     zbeg + (int64_t)st * Cfg::ZS, zend, VEC);
        };
        // LDS layout of a stage: [row][c][lane], element = z zs + NC lane + c,
        // so that the reads of one component c are contiguous over the lanes
        auto stash = [&](int buf) {
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                uint32_t *dst = smw + buf * (Cfg::ROWS * Cfg::ZS) + (wave + q * Cfg::NW) * Cfg::ZS + lane;
#pragma unroll
                for (int c = 0; c < NC; ++c) dst[64 * c] = pre.r[q].v[c];
            }
        };
        // the counting of one staged buffer: component c + 1 is read before the
        // block of component c runs (the scheduling barriers keep the reads
        // there), so that the reads overlap it
        auto count = [&](int buf, auto first_tag) {  // first_tag: std::true_type for the tile's first stage
            const uint32_t *sb = smw + buf * (Cfg::ROWS * Cfg::ZS) + lane;
            if constexpr (AHEAD) {
                uint32_t av[2][Cfg::WX], bv[2][Cfg::WY];
                auto read_comp = [&](int c) {
#pragma unroll
                    for (int i = 0; i < Cfg::WX; ++i) av[c & 1][i] = sb[(wx * Cfg::WX + i) * Cfg::ZS + 64 * c];
#pragma unroll
                    for (int j = 0; j < Cfg::WY; ++j)
                        bv[c & 1][j] = sb[(Cfg::TX + wy * Cfg::WY + j) * Cfg::ZS + 64 * c];
                };
                read_comp(0);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    if (c + 1 < NC) read_comp(c + 1);
                    __builtin_amdgcn_sched_barrier(0);
                    if (decltype(first_tag)::value && c == 0)
                        focus_mask_count32_first(cnt, av[c & 1], bv[c & 1], t, carry);
                    else
                        focus_mask_count32(cnt, av[c & 1], bv[c & 1], t, carry);
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else {
                uint32_t av[Cfg::WX], bv[Cfg::WY];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
#pragma unroll
                    for (int i = 0; i < Cfg::WX; ++i) av[i] = sb[(wx * Cfg::WX + i) * Cfg::ZS + 64 * c];
#pragma unroll
                    for (int j = 0; j < Cfg::WY; ++j) bv[j] = sb[(Cfg::TX + wy * Cfg::WY + j) * Cfg::ZS + 64 * c];
                    __builtin_amdgcn_sched_barrier(0);
                    if (decltype(first_tag)::value && c == 0)
                        focus_mask_count32_first(cnt, av, bv, t, carry);
                    else
                        focus_mask_count32(cnt, av, bv, t, carry);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        };

        if (nst > 0 && !rows_in) {
            // a first stage through the out-of-line bounds-checked fetch:
            // the key goes to LDS first, so that it is not held across the call
            take_keys(load_key());
            fetch(0);
        } else {
            const uint32_t key = load_key();
            if (nst_fast > 0)
                fetch_fast(lane_off);
            else if (nst > 0)
                fetch_tail(0);
            take_keys(key);
        }
        if (nst > 0) stash(0);
        __syncthreads();
        int32_t st = 0;
        if (nst > 0) {  // stage 0 on its own: its first block starts the counts
            if (nst > 1) fetch(1);
            count(0, std::true_type{});
            if (nst > 1) stash(1);
            __syncthreads();
            st = 1;
        } else {
#pragma unroll
            for (int p = 0; p < Cfg::WX * Cfg::WY; ++p) cnt[p] = 0;
            carry[0] = carry[1] = 0;
        }
        // Stages whose successor loads without checks run two at a time with
        // fixed buffers (buffer 1 holds stage st on entry): little loop control
        // on the scalar unit, which also does the counting.
        uint32_t off = 2 * STAGE_BYTES + lane_off;  // of stage st + 1 (st = 1)
        for (; st + 2 < nst_fast; st += 2) {
            fetch_fast(off);
            count(1, std::false_type{});
            stash(0);
            __syncthreads();
            fetch_fast(off + STAGE_BYTES);
            count(0, std::false_type{});
            stash(1);
            __syncthreads();
            off += 2 * STAGE_BYTES;
        }
        for (; st < nst; ++st) {  // the rest, buffer st & 1
            const int buf = st & 1;
            if (st + 1 < nst) fetch(st + 1);
            count(buf, std::false_type{});
            if (st + 1 < nst) stash(buf ^ 1);
            __syncthreads();
        }
    };
    if (vec_ok)
        run(std::true_type{});
    else
        run(std::false_type{});

    focus_mask_flush(cnt, carry);
    // epilogue: lane p (p < 32) takes pair p (one lane write per count)
    int32_t mine = 0;
#pragma unroll
    for (int p = 0; p < Cfg::WX * Cfg::WY; ++p) asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(mine) : "s"(cnt[p]), "i"(p));
    // (the lane index passed through an empty asm, so that the pair indices
    // are formed here again rather than kept from the key loads across the
    // stage loop, where registers are short)
    int elane = lane;
    asm volatile("" : "+v"(elane));
    if (elane >= Cfg::WX * Cfg::WY) return;
    const int64_t x = xw + elane / Cfg::WY, y = yw + elane % Cfg::WY;
    if constexpr (RECT) {
        if (x >= g.xhi || y >= g.yhi) return;
        if (U) U[(x - g.xlo) * ldu + y] = mine;
        if (W) W[y * ldw + (x - g.xlo)] = x != y ? weight_of(mine) : 0.0f;
        return;
    }
    if (x >= n || y >= n || x > y) return;
    const bool mirror = x != y;
    if (atomic_mode) {
        atomicAdd(&U[x * ldu + y], mine);
        if (mirror) atomicAdd(&U[y * ldu + x], mine);
        return;
    }
    if (U) {
        U[x * ldu + y] = mine;
        if (mirror) U[y * ldu + x] = mine;
    }
    if (W) {
        const float w = mirror ? weight_of(mine) : 0.0f;
        W[x * ldw + y] = w;
        if (mirror) W[y * ldw + x] = w;
    }
}

// The whole-matrix form of pass1z_tile_g (square mode).
template <int GX, int GY, int NC, bool AHEAD = true>
__device__ __forceinline__ void pass1z_tile(int tid, uint32_t *smw, const float *__restrict__ D, int64_t n,
                                            int64_t ldd, int32_t *__restrict__ U, int64_t ldu,
                                            float *__restrict__ W, int64_t ldw, int64_t X0, int64_t Y0,
                                            int64_t zbeg, int64_t zend, bool atomic_mode, bool vec_ok) {
    pass1z_tile_g<GX, GY, NC, false, AHEAD>(tid, smw, P1Rows{D, ldd, 0, n, D, ldd, 0, n}, n, U, ldu, W, ldw, X0, Y0, zbeg,
                                     zend, atomic_mode, vec_ok);
}

// The single-matrix pass-1 kernel: 4 x 2 waves (16 x 16 pairs, 512 threads),
// 2 z per lane (128 per stage), 32 KB of LDS and 73 VGPRs: three workgroups
// per CU, 6 waves per SIMD, with independent barriers (4 z per lane: 64 KB
// and 91 VGPRs, 4 waves per SIMD, 5 % slower; PALD_P1Z_GY = 4: 16 x 32 tiles
// of 1024 threads, slower still).  The tiles cover every pair x <= y exactly
// once: tile (bi, bj) spans x in [TX bi, TX bi + TX), y in [TY bj, TY bj +
// TY), and the tiles with floor(bi / S) <= bj, S = TY / TX, are enumerated as
// the S parts of the square TY x TY tiles bx <= bj in the grouped order of
// grouped_tile().  blockIdx.y is the z-chunk; with one chunk the tile writes
// U and W directly, with several it atomically adds into U (zero on entry).
#ifndef PALD_P1Z_GX
#define PALD_P1Z_GX 4
#endif
#ifndef PALD_P1Z_GY
#define PALD_P1Z_GY 2
#endif
#ifndef PALD_P1Z_NC
#define PALD_P1Z_NC 2
#endif
// 8 waves per SIMD (4 workgroups per CU, 32 KB of LDS each) with the
// component reads not run ahead (64 VGPRs): 123 ms at n = 16384, against 130
// ms at 6 waves with them run ahead (76 VGPRs; at 6 waves without them, 132
// ms).  The bound keeps a code change from quietly taking the kernel past 64
// VGPRs and down to 3 workgroups per CU.
#ifndef PALD_P1Z_MIN_WAVES
#define PALD_P1Z_MIN_WAVES 8
#endif
#ifndef PALD_P1Z_AHEAD
#define PALD_P1Z_AHEAD 0
#endif
using P1zMain = P1zCfg<PALD_P1Z_GX, PALD_P1Z_GY, PALD_P1Z_NC>;
constexpr int P1Z_TX = P1zMain::TX, P1Z_TY = P1zMain::TY, P1Z_NT = P1zMain::NT, P1Z_ZS = P1zMain::ZS;
constexpr int P1Z_SPLIT = P1Z_TY / P1Z_TX;  // tiles per TY x TY square
static_assert(P1Z_SPLIT * P1Z_TX == P1Z_TY, "the y side must be a multiple of the x side");

__global__ __launch_bounds__(P1Z_NT, PALD_P1Z_MIN_WAVES) void pass1z_focus_kernel(const float *__restrict__ D, int64_t n,
                                                                 int64_t ldd, int32_t *__restrict__ U, int64_t ldu,
                                                                 float *__restrict__ W, int64_t ldw,
                                                                 int32_t z_per_chunk, int32_t atomic_mode,
                                                                 int32_t vec_ok, int32_t tile0) {
    __shared__ uint32_t smw[P1zMain::LDS_WORDS];
    const int32_t k = tile0 + xcd_order((int32_t)blockIdx.x, (int32_t)gridDim.x);
    int32_t bx, bj;
    grouped_tile(k / P1Z_SPLIT, (int32_t)((n + P1Z_TY - 1) / P1Z_TY), bx, bj);
    const int64_t X0 = (int64_t)(P1Z_SPLIT * bx + k % P1Z_SPLIT) * P1Z_TX, Y0 = (int64_t)bj * P1Z_TY;
    if (X0 >= n) return;  // a later part of a square tile at the edge: no pairs
    const int64_t zbeg = (int64_t)blockIdx.y * z_per_chunk;
    const int64_t zend = min(n, zbeg + (int64_t)z_per_chunk);
    pass1z_tile<PALD_P1Z_GX, PALD_P1Z_GY, PALD_P1Z_NC, (bool)PALD_P1Z_AHEAD>((int)threadIdx.x, smw, D, n, ldd, U, ldu, W, ldw, X0, Y0, zbeg, zend,
                                   atomic_mode != 0, vec_ok != 0);
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
// Pass 2: cohesion, both directions of every pair {x, z} at once.
//
// For a pair (x, z) and a second point y, the term of c_xz (focus of x and y,
// third point z) and the term of c_zx (focus of z and y, third point x) read
// the same three distances t = d_xz, a = d_xy, b = d_zy, and both vanish
// unless t <= min(a, b):
//     c_xz += [t <= min(a,b)] * (t < b ? W_xy : W_xy / 2)
//     c_zx += [t <= min(a,b)] * (t < a ? W_zy : W_zy / 2)
// One thread keeps both accumulators of its pairs and shares the membership
// test between them.
//
// Each thread owns RX x 4 pairs (x, z).
// Grid: blockIdx.x picks an upper-triangular T x T tile (bx <= bz) in the
// grouped, XCD-contiguous order of grouped_tile() / xcd_order(), offset by
// tile0 (large grids are launched in pieces); blockIdx.y is the y-chunk.  A
// tile with bx < bz writes C[X][Z] and C[Z][X];
// a diagonal tile covers every ordered pair of its block once as (x, z) and
// writes only C[x][z].  With one y-chunk the tile writes
// C = fl32(sum / (n-1)); otherwise it writes float64 partial sums
// partial[chunk][x][z] (ld n) for finalize_kernel.
//
// Per y the tile stages row y of D and the halves of row y of W, restricted
// to the x range and to the z range (a = d_yx, b = d_yz, W_yx / 2, W_yz / 2;
// D and W are symmetric; halving is exact).  Rows y >= n, and rows past the
// chunk, stage W = 0 and so add nothing; the terms y = x and y = z add
// nothing because W_xx = W_zz = 0.
//
// Each term is added as one or two exact half weights (cohesion_terms4).
// Float32 runs: in the single-accumulator form a run covers P2_RUN = 6 values
// of y, so it holds at most 12 additions and the relative error of a C entry
// stays below (12 + 3) 2^-24 = 8.9e-7 (the run, the Kahan fold, the rounding
// of W and the final store).  In the split form the second half weight of a
// term goes to accumulators of its own that join the run at each fold: runs
// of P2_RUN_SPLIT = 12 values of y, at most 12 additions per accumulator plus
// the join, below (11 + 1 + 2 + 1 + 1) 2^-24 = 9.5e-7.
constexpr int P2_RUN = 6, P2_RUN_SPLIT = 12;
// minimum waves per SIMD the pass-2 kernel is compiled for (its VGPR budget)
#ifndef PALD_P2_MIN_WAVES
#define PALD_P2_MIN_WAVES 3
#endif
template <int T, int RX, int KY>
struct Pass2Cfg {
    static constexpr int RZ = 4;                        // z per thread (the term block's width)
    static constexpr int TX = T / RX;                   // threads along x
    static constexpr int TZ = T / RZ;                   // threads along z
    static constexpr int NT = TX * TZ;
    static constexpr int ROW = 4 * T;                   // loaded per y: a | W_yx | b | W_yz
    static constexpr int LDS_ROW = 4 * T;               // staged per y: a | W_yx/2 | b | W_yz/2
    static constexpr int VEC_PER_CHUNK = KY * ROW / 4;
    static constexpr int VEC_PER_THREAD = (VEC_PER_CHUNK + NT - 1) / NT;  // the last round may be partial
    static constexpr bool VEC_EVEN = VEC_PER_CHUNK % NT == 0;
    static constexpr int LDS_VEC = 2 * KY * LDS_ROW / 4; // uint4 of LDS, double-buffered
    static_assert(KY % P2_RUN == 0 && KY % P2_RUN_SPLIT == 0, "KY must be a multiple of the run lengths");
    static_assert(T % 4 == 0, "tile side must be a multiple of 4");
};

// Where a pass-2 tile puts its sums: exactly one of
//   C     -- final cohesion, fl32(sum / (n-1)), leading dimension ldc;
//   slab  -- float64 partial sums of this y-chunk in an n x n array (ld n);
//   tile  -- float64 partial sums in tile-local order: [0][i][j] holds the
//            (X0+i, Z0+j) entry, [1][i][j] the mirrored (Z0+j, X0+i) entry.
struct Pass2Out {
    float *C;
    int64_t ldc;
    double *slab;
    double *tile;
};

// One pass-2 tile (bx, bz), bx <= bz, over the y range [ybeg, yend).  Called
// by every thread of a workgroup of Pass2Cfg::NT threads, all lanes active;
// `sm` points to Pass2Cfg::LDS_VEC uint4 of LDS.  FEW_SGPR: compare blocks of
// two pairs instead of four (fewer scalar registers).  SPLIT: the split-run
// form (16 more accumulator VGPRs for 2 x 4 pairs, runs twice as long).
template <int T, int RX, int KY, bool F64, bool FEW_SGPR = false, bool SPLIT = false>
__device__ __forceinline__ void pass2_tile(int tid, uint4 *sm, const float *__restrict__ D, int64_t n, int64_t ldd,
                                           const float *__restrict__ W, int64_t ldw, Pass2Out out, int32_t bx,
                                           int32_t bz, int64_t ybeg, int64_t yend, bool vec_ok_d, bool vec_ok_w) {
    using Cfg = Pass2Cfg<T, RX, KY>;
    const int64_t X0 = (int64_t)bx * T, Z0 = (int64_t)bz * T;
    constexpr int RZ = Cfg::RZ;
    const int tx = tid % Cfg::TX, tz = tid / Cfg::TX;

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

    // forward (c_xz) and reverse (c_zx) accumulators: Kahan sums s and run
    // accumulators r.  A run starts from the negated compensation left by the
    // previous fold, so r holds (run sum - c) when the run ends -- the
    // compensated summand of Kahan's algorithm -- and no separate compensation
    // register stays live during a run.
    // In the split form the second half weight of a term goes to gf / gr,
    // which join the run at the fold.
    float sf[RX][RZ], rf[RX][RZ], sr[RX][RZ], rr[RX][RZ];
    float gf[RX][RZ], gr[RX][RZ];
    double af[RX][RZ], ar[RX][RZ];
#pragma unroll
    for (int i = 0; i < RX; ++i)
#pragma unroll
        for (int j = 0; j < RZ; ++j) {
            sf[i][j] = rf[i][j] = 0.0f;
            sr[i][j] = rr[i][j] = 0.0f;
            gf[i][j] = gr[i][j] = 0.0f;
            af[i][j] = ar[i][j] = 0.0;
        }

    uint4 pre[Cfg::VEC_PER_THREAD];
    auto fetch = [&](int64_t yc) {
#pragma unroll
        for (int k = 0; k < Cfg::VEC_PER_THREAD; ++k) {
            const int v = tid + k * Cfg::NT;
            if (!Cfg::VEC_EVEN && v >= Cfg::VEC_PER_CHUNK) break;
            const int r = v / (Cfg::ROW / 4);
            const int g = v % (Cfg::ROW / 4);
            const int seg = g / (T / 4);           // 0: D x-range, 1: W x-range, 2: D z-range, 3: W z-range
            const int64_t col = ((seg < 2) ? X0 : Z0) + 4 * (g % (T / 4));
            const int64_t y = yc + r;
            if (seg == 0 || seg == 2)
                pre[k] = load_keys4(D, ldd, y, col, yend, n, vec_ok_d, 0u);
            else
                pre[k] = load_vals4(W, ldw, y, col, yend, n, vec_ok_w);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int k = 0; k < Cfg::VEC_PER_THREAD; ++k) {
            const int v = tid + k * Cfg::NT;
            if (!Cfg::VEC_EVEN && v >= Cfg::VEC_PER_CHUNK) break;
            const int r = v / (Cfg::ROW / 4);
            const int g = v % (Cfg::ROW / 4);
            const int seg = g / (T / 4);
            uint4 *row = sm + buf * (Cfg::LDS_VEC / 2) + r * (Cfg::LDS_ROW / 4);
            uint4 w = pre[k];
            if (seg == 1 || seg == 3)  // W segment: staged as its halves (exact)
                w = make_uint4(__float_as_uint(0.5f * __uint_as_float(w.x)), __float_as_uint(0.5f * __uint_as_float(w.y)),
                               __float_as_uint(0.5f * __uint_as_float(w.z)), __float_as_uint(0.5f * __uint_as_float(w.w)));
            row[g] = w;
        }
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
        const uint32_t *s = reinterpret_cast<const uint32_t *>(sm + buf * (Cfg::LDS_VEC / 2));
        // operands of staged row yr: a = d_yx, W_yx/2 over x; b = d_yz, W_yz/2 over z
        auto load_row = [&](int yr, uint32_t (&av)[RX], float (&whx)[RX], uint32_t (&bv)[RZ], float (&whz)[RZ]) {
            const uint32_t *row = s + yr * Cfg::LDS_ROW;
#pragma unroll
            for (int i = 0; i < RX; ++i) {
                av[i] = row[tx * RX + i];
                whx[i] = __uint_as_float(row[T + tx * RX + i]);
            }
#pragma unroll
            for (int j = 0; j < RZ; ++j) {
                bv[j] = row[2 * T + tz * RZ + j];
                whz[j] = __uint_as_float(row[3 * T + tz * RZ + j]);
            }
        };
        if (F64) {
            // reference form: plain float64 accumulation of W or W/2, no runs
#pragma unroll 2
            for (int yr = 0; yr < KY; ++yr) {
                uint32_t av[RX], bv[RZ];
                float whx[RX], whz[RZ];
                load_row(yr, av, whx, bv, whz);
#pragma unroll
                for (int i = 0; i < RX; ++i)
#pragma unroll
                    for (int j = 0; j < RZ; ++j) {
                        const uint32_t tt = t[i][j];
                        const uint64_t in = lane_mask(tt <= av[i]) & lane_mask(tt <= bv[j]);
                        float vf = lane_bit(in) ? whx[i] : 0.0f;
                        vf = lane_bit(in & lane_mask(tt < bv[j])) ? whx[i] + whx[i] : vf;
                        float vr = lane_bit(in) ? whz[j] : 0.0f;
                        vr = lane_bit(in & lane_mask(tt < av[i])) ? whz[j] + whz[j] : vr;
                        af[i][j] += (double)vf;
                        ar[i][j] += (double)vr;
                    }
            }
        } else {
            const uint64_t full = __builtin_amdgcn_read_exec();
            constexpr int RUN = SPLIT ? P2_RUN_SPLIT : P2_RUN;
            // (the runs of a stage fully unrolled: no register copies of the
            // Kahan state between runs)
#pragma unroll
            for (int y0 = 0; y0 < KY; y0 += RUN) {
#pragma unroll
                for (int yy = 0; yy < RUN; ++yy) {
                    uint32_t av[RX], bv[RZ];
                    float whx[RX], whz[RZ];
                    load_row(y0 + yy, av, whx, bv, whz);
#pragma unroll
                    for (int i = 0; i < RX; ++i) {
                        if constexpr (SPLIT)
                            cohesion_terms4_split(rf[i], rr[i], gf[i], gr[i], t[i], av[i], bv, whx[i], whz, full);
                        else
                            cohesion_terms4<FEW_SGPR ? 2 : 4>(rf[i], rr[i], t[i], av[i], bv, whx[i], whz, full);
                    }
                }
                // Kahan fold of the finished runs (r = run - c): s + r, with the
                // new negated compensation -c = r - ((s + r) - s) left in r.
#pragma unroll
                for (int i = 0; i < RX; ++i)
#pragma unroll
                    for (int j = 0; j < RZ; ++j) {
                        if constexpr (SPLIT) {  // the second halves join the run first
                            rf[i][j] += gf[i][j];
                            rr[i][j] += gr[i][j];
                            gf[i][j] = gr[i][j] = 0.0f;
                        }
                        float tk = sf[i][j] + rf[i][j];
                        rf[i][j] = rf[i][j] - (tk - sf[i][j]);
                        sf[i][j] = tk;
                        tk = sr[i][j] + rr[i][j];
                        rr[i][j] = rr[i][j] - (tk - sr[i][j]);
                        sr[i][j] = tk;
                    }
            }
        }
        if (c + 1 < nchunks) stash(buf ^ 1);
        __syncthreads();
    }

    const double nm1 = (double)(n - 1);
    const bool mirror = bx != bz;
#pragma unroll
    for (int i = 0; i < RX; ++i) {
        const int64_t x = X0 + tx * RX + i;
#pragma unroll
        for (int j = 0; j < RZ; ++j) {
            const int64_t z = Z0 + tz * RZ + j;
            const double tf = F64 ? af[i][j] : ((double)sf[i][j] + (double)rf[i][j]);
            const double tr = F64 ? ar[i][j] : ((double)sr[i][j] + (double)rr[i][j]);
            if (out.tile) {
                const int li = tx * RX + i, lj = tz * RZ + j;
                out.tile[li * T + lj] = tf;
                out.tile[T * T + li * T + lj] = tr;
                continue;
            }
            if (x >= n || z >= n) continue;
            if (out.C) {
                out.C[x * out.ldc + z] = (float)(tf / nm1);
                if (mirror) out.C[z * out.ldc + x] = (float)(tr / nm1);
            } else {
                out.slab[x * n + z] = tf;
                if (mirror) out.slab[z * n + x] = tr;
            }
        }
    }
}

template <int T, int RX, int KY, bool F64>
__global__ __launch_bounds__((Pass2Cfg<T, RX, KY>::NT), PALD_P2_MIN_WAVES) void pass2_cohesion_kernel(
    const float *__restrict__ D, int64_t n, int64_t ldd, const float *__restrict__ W, int64_t ldw,
    float *__restrict__ C, int64_t ldc, double *__restrict__ partial, int32_t y_per_chunk,
    int32_t vec_ok_d, int32_t vec_ok_w, int32_t tile0) {
    using Cfg = Pass2Cfg<T, RX, KY>;
    __shared__ uint4 sm[Cfg::LDS_VEC];
    int32_t bx, bz;
    grouped_tile(tile0 + xcd_order((int32_t)blockIdx.x, (int32_t)gridDim.x), (int32_t)((n + T - 1) / T), bx, bz);
    const int64_t ybeg = (int64_t)blockIdx.y * y_per_chunk;
    const int64_t yend = min(n, ybeg + (int64_t)y_per_chunk);
    Pass2Out out{nullptr, 0, nullptr, nullptr};
    if (gridDim.y == 1) {
        out.C = C;
        out.ldc = ldc;
    } else {
        out.slab = partial + (int64_t)blockIdx.y * n * n;
    }
    pass2_tile<T, RX, KY, F64, false, true>((int)threadIdx.x, sm, D, n, ldd, W, ldw, out, bx, bz, ybeg, yend,
                                           vec_ok_d != 0, vec_ok_w != 0);
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
