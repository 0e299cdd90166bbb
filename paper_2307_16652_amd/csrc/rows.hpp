// rows.hpp -- both passes for a block of rows x of U and C.
//
// Row x of U needs the focus sizes U_xy for all y, and row x of C needs
//     c_xz = 1/(n-1) sum_{y != x} [t <= min(a, b)] * (t < b ? W_xy : W_xy / 2)
// (t = d_xz, a = d_xy, b = d_zy) -- all of D but only row x of W.  So rows
// split over devices, or over panels of one device, with no exchange beyond
// D itself (the sharding the method allows: each row of C is a sum over y of
// terms that involve row x of the focus sizes only).
//
// The kernels take the rows of D through P1Rows: the x rows of the block
// (Dx, rows [xlo, xhi)) and the y rows the launch reads (Dy, rows [ylo, yhi));
// with D resident both are D itself, out of core they are a panel buffer and
// a streamed block of rows.  W of the block is stored transposed,
// Wt[y][x - xlo], so that a tile stages it per y as a contiguous row segment.
#pragma once

#include "pairwise.hpp"

namespace pald {

// Pass 1 of a block of rows: U[(x - xlo) ldu + y] for x in [xlo, xhi), y in
// [ylo, yhi), every z, and Wt[y ldwt + (x - xlo)] (0 at x = y).  The
// single-matrix lanes-over-z tile (16 x 16 pairs, 8 waves) without the
// symmetric mirror; tile k of the launch piece starting at tile0 covers x
// tile (tile0 + k) / ytiles and y tile (tile0 + k) % ytiles, so consecutive
// workgroups share their x rows.
// (the single-matrix tile's occupancy and component reads: 8 waves per SIMD,
// no reads run ahead)
#ifndef PALD_P1_ROWS_MIN_WAVES
#define PALD_P1_ROWS_MIN_WAVES PALD_P1Z_MIN_WAVES
#endif
#ifndef PALD_P1_ROWS_AHEAD
#define PALD_P1_ROWS_AHEAD PALD_P1Z_AHEAD
#endif
__global__ __launch_bounds__(P1Z_NT, PALD_P1_ROWS_MIN_WAVES) void pass1_rows_kernel(const P1Rows g, int64_t n,
                                                                                int32_t *__restrict__ U, int64_t ldu,
                                                                                float *__restrict__ Wt, int64_t ldwt,
                                                                                int32_t vec_ok, int64_t tile0) {
    __shared__ uint32_t smw[P1zMain::LDS_WORDS];
    const int64_t ytiles = (g.yhi - g.ylo + P1Z_TY - 1) / P1Z_TY;
    const int64_t k = tile0 + (int64_t)blockIdx.x;
    const int64_t X0 = g.xlo + (k / ytiles) * P1Z_TX, Y0 = g.ylo + (k % ytiles) * P1Z_TY;
    pass1z_tile_g<PALD_P1Z_GX, PALD_P1Z_GY, PALD_P1Z_NC, true, (bool)PALD_P1_ROWS_AHEAD>((int)threadIdx.x, smw, g, n, U, ldu, Wt, ldwt, X0, Y0,
                                                               0, n, false, vec_ok != 0);
}

// Forward cohesion terms of one x and four z for one second point y (c_xz
// only; the symmetric pass 2 also gets c_zx from the same compares, which a
// block of rows cannot use):
//     i = [t_j <= a],  j = [t_j <= b_j],  p = [t_j < b_j]
//     rf_j += hx under i & j, and again under i & p
// with hx = W_xy / 2; EXEC handled as in cohesion_terms4 (restored to `full`).
#define PALD_F_CMP(k)                                                                                            \
    "v_cmp_le_u32_e64 %[i" #k "], %[t" #k "], %[a]\n\t"                                                       \
    "v_cmp_le_u32_e64 %[j" #k "], %[t" #k "], %[b" #k "]\n\t"                                                 \
    "v_cmp_lt_u32_e64 %[p" #k "], %[t" #k "], %[b" #k "]\n\t"
#define PALD_F_ADD(k)                                                                                            \
    "s_and_b64 exec, %[i" #k "], %[j" #k "]\n\t"                                                              \
    "v_add_f32 %[rf" #k "], %[rf" #k "], %[hx]\n\t"                                                           \
    "s_and_b64 exec, %[i" #k "], %[p" #k "]\n\t"                                                              \
    "v_add_f32 %[rf" #k "], %[rf" #k "], %[hx]\n\t"
#define PALD_F_MASKS(k) [i##k] "=&s"(mi[k]), [j##k] "=&s"(mj[k]), [p##k] "=&s"(mp[k])
#define PALD_F_IN(k) [t##k] "v"(t[k]), [b##k] "v"(b[k])
__device__ __forceinline__ void cohesion_fwd4(float (&rf)[4], const uint32_t (&t)[4], uint32_t a, const uint32_t (&b)[4],
                                              float hx, uint64_t full) {
    uint64_t mi[4], mj[4], mp[4];
    asm(PALD_F_CMP(0) PALD_F_CMP(1) PALD_F_CMP(2) PALD_F_CMP(3)
        PALD_F_ADD(0) PALD_F_ADD(1) PALD_F_ADD(2) PALD_F_ADD(3)
        "s_mov_b64 exec, %[full]"
        : [rf0] "+v"(rf[0]), [rf1] "+v"(rf[1]), [rf2] "+v"(rf[2]), [rf3] "+v"(rf[3]), PALD_F_MASKS(0), PALD_F_MASKS(1),
          PALD_F_MASKS(2), PALD_F_MASKS(3)
        : [a] "v"(a), [hx] "v"(hx), [full] "s"(full), PALD_F_IN(0), PALD_F_IN(1), PALD_F_IN(2), PALD_F_IN(3)
        : "scc");
}
#undef PALD_F_CMP
#undef PALD_F_ADD
#undef PALD_F_MASKS
#undef PALD_F_IN

// Pass 2 of a block of rows: a 64 x 64 (x, z) tile, 4 x 4 pairs per thread
// (256 threads), y over [ybeg, yend) in stages of 12 rows of D and Wt through
// LDS (a = d_yx | W_xy / 2 over the tile's x, b = d_yz over its z), float32
// runs of 6 y (at most 12 additions) folded into Kahan sums.  Either writes
// C[(x - xlo) ldc + z] = fl32(sum / (n-1)) (acc null) or adds the sum to the
// float64 accumulator acc[(x - xlo) ldacc + z] (blocks of y streamed one after
// another).  Grid: blockIdx.x = z tile, blockIdx.y = x tile.
#ifndef PALD_P2R_RX
#define PALD_P2R_RX 2
#endif
constexpr int P2R_T = 64, P2R_RX = PALD_P2R_RX, P2R_RZ = 4, P2R_KY = 12, P2R_RUN = 6;
constexpr int P2R_TX = P2R_T / P2R_RX, P2R_TZ = P2R_T / P2R_RZ, P2R_NT = P2R_TX * P2R_TZ;
constexpr int P2R_ROW = 3 * P2R_T;                         // staged per y: a | W/2 | b
constexpr int P2R_VEC_PER_CHUNK = P2R_KY * P2R_ROW / 4;    // uint4 per stage
constexpr int P2R_VEC_PER_THREAD = (P2R_VEC_PER_CHUNK + P2R_NT - 1) / P2R_NT;
static_assert(P2R_KY % P2R_RUN == 0, "stages hold whole runs");

__global__ __launch_bounds__(P2R_NT, 2) void pass2_rows_kernel(const P1Rows g, int64_t n, const float *__restrict__ Wt,
                                                               int64_t ldwt, float *__restrict__ C, int64_t ldc,
                                                               double *__restrict__ acc, int64_t ldacc, int64_t ybeg,
                                                               int64_t yend, int32_t vec_d, int32_t vec_w) {
    __shared__ uint4 sm[2 * P2R_VEC_PER_CHUNK];
    const int tid = (int)threadIdx.x;
    const int tx = tid % P2R_TX, tz = tid / P2R_TX;
    const int64_t X0 = g.xlo + (int64_t)blockIdx.y * P2R_T, Z0 = (int64_t)blockIdx.x * P2R_T;

    // stationary keys t = d_xz (from the x rows)
    uint32_t t[P2R_RX][P2R_RZ];
#pragma unroll
    for (int i = 0; i < P2R_RX; ++i) {
        const int64_t x = X0 + tx * P2R_RX + i;
#pragma unroll
        for (int j = 0; j < P2R_RZ; ++j) {
            const int64_t z = Z0 + tz * P2R_RZ + j;
            t[i][j] = (x < g.xhi && z < n) ? key_of(g.Dx[(x - g.xlo) * g.ldx + z]) : 0u;
        }
    }
    float sf[P2R_RX][P2R_RZ], rf[P2R_RX][P2R_RZ];
#pragma unroll
    for (int i = 0; i < P2R_RX; ++i)
#pragma unroll
        for (int j = 0; j < P2R_RZ; ++j) sf[i][j] = rf[i][j] = 0.0f;

    // staging: element v of a stage (uint4) is row v / 48, column group v % 48:
    // groups 0-15 a = D[y][X0..], 16-31 W[x][y] / 2 over x = X0.., 32-47 b = D[y][Z0..]
    uint4 pre[P2R_VEC_PER_THREAD];
    auto fetch = [&](int64_t yc) {
#pragma unroll
        for (int k = 0; k < P2R_VEC_PER_THREAD; ++k) {
            const int v = tid + k * P2R_NT;
            if (v >= P2R_VEC_PER_CHUNK) break;
            const int r = v / (P2R_ROW / 4), gi = v % (P2R_ROW / 4), seg = gi / (P2R_T / 4), c4 = 4 * (gi % (P2R_T / 4));
            const int64_t y = yc + r;
            if (y >= yend) {
                pre[k] = make_uint4(0u, 0u, 0u, 0u);
                continue;
            }
            const float *drow = g.Dy + (y - g.ylo) * g.ldy;
            if (seg == 0)
                pre[k] = load_keys4(drow, 0, 0, X0 + c4, 1, g.xhi, vec_d != 0, 0u);
            else if (seg == 1)
                pre[k] = load_vals4(Wt + y * ldwt, 0, 0, X0 - g.xlo + c4, 1, g.xhi - g.xlo, vec_w != 0);
            else
                pre[k] = load_keys4(drow, 0, 0, Z0 + c4, 1, n, vec_d != 0, 0u);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int k = 0; k < P2R_VEC_PER_THREAD; ++k) {
            const int v = tid + k * P2R_NT;
            if (v >= P2R_VEC_PER_CHUNK) break;
            uint4 w = pre[k];
            if ((v % (P2R_ROW / 4)) / (P2R_T / 4) == 1)  // the weights, staged as their halves (exact)
                w = make_uint4(__float_as_uint(0.5f * __uint_as_float(w.x)), __float_as_uint(0.5f * __uint_as_float(w.y)),
                               __float_as_uint(0.5f * __uint_as_float(w.z)), __float_as_uint(0.5f * __uint_as_float(w.w)));
            sm[buf * P2R_VEC_PER_CHUNK + v] = w;
        }
    };

    const int64_t ny = yend - ybeg;
    const int64_t nchunks = ny > 0 ? (ny + P2R_KY - 1) / P2R_KY : 0;
    if (nchunks > 0) {
        fetch(ybeg);
        stash(0);
    }
    __syncthreads();
    const uint64_t full = __builtin_amdgcn_read_exec();
    for (int64_t c = 0; c < nchunks; ++c) {
        const int buf = (int)(c & 1);
        if (c + 1 < nchunks) fetch(ybeg + (c + 1) * P2R_KY);
        const uint32_t *s = reinterpret_cast<const uint32_t *>(sm + buf * P2R_VEC_PER_CHUNK);
#pragma unroll 1
        for (int y0 = 0; y0 < P2R_KY; y0 += P2R_RUN) {
#pragma unroll
            for (int yy = 0; yy < P2R_RUN; ++yy) {
                const uint32_t *row = s + (y0 + yy) * P2R_ROW;
                uint32_t bv[P2R_RZ];
#pragma unroll
                for (int j = 0; j < P2R_RZ; ++j) bv[j] = row[2 * P2R_T + tz * P2R_RZ + j];
#pragma unroll
                for (int i = 0; i < P2R_RX; ++i)
                    cohesion_fwd4(rf[i], t[i], row[tx * P2R_RX + i], bv, __uint_as_float(row[P2R_T + tx * P2R_RX + i]),
                                  full);
            }
            // Kahan fold of the runs (r holds run - c; see pass2_tile)
#pragma unroll
            for (int i = 0; i < P2R_RX; ++i)
#pragma unroll
                for (int j = 0; j < P2R_RZ; ++j) {
                    const float tk = sf[i][j] + rf[i][j];
                    rf[i][j] = rf[i][j] - (tk - sf[i][j]);
                    sf[i][j] = tk;
                }
        }
        if (c + 1 < nchunks) stash(buf ^ 1);
        __syncthreads();
    }

    const double nm1 = (double)(n - 1);
#pragma unroll
    for (int i = 0; i < P2R_RX; ++i) {
        const int64_t x = X0 + tx * P2R_RX + i;
        if (x >= g.xhi) continue;
#pragma unroll
        for (int j = 0; j < P2R_RZ; ++j) {
            const int64_t z = Z0 + tz * P2R_RZ + j;
            if (z >= n) continue;
            const double v = (double)sf[i][j] + (double)rf[i][j];
            if (acc)
                acc[(x - g.xlo) * ldacc + z] += v;
            else
                C[(x - g.xlo) * ldc + z] = (float)(v / nm1);
        }
    }
}

// C[r][z] = fl32(acc[r][z] / (n-1)) for rows r < rows, z < n.
__global__ void rows_finalize_kernel(const double *__restrict__ acc, int64_t ldacc, int64_t rows, int64_t n,
                                     float *__restrict__ C, int64_t ldc) {
    const double nm1 = (double)(n - 1);
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y)
        for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < n; z += (int64_t)gridDim.x * blockDim.x)
            C[r * ldc + z] = (float)(acc[r * ldacc + z] / nm1);
}

// acc[r][z] = 0 for rows r < rows, z < n (a kernel, so that it can sit in a
// captured graph).
__global__ void zero_f64_kernel(double *__restrict__ acc, int64_t ldacc, int64_t rows, int64_t n) {
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y)
        for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < n; z += (int64_t)gridDim.x * blockDim.x)
            acc[r * ldacc + z] = 0.0;
}

}  // namespace pald
