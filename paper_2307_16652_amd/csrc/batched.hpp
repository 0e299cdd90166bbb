// batched.hpp -- many independent PaLD problems of different sizes in one
// persistent launch (a GPU-side extension; the paper has no batching).
//
// Work items are pass-1 tiles and pass-2 tiles (optionally split over y) of
// every matrix, listed once in a queue built on the host.  Each workgroup of
// the persistent grid takes the next item with one atomic increment of a
// global head counter and runs it with the same tile functions as the
// single-matrix kernels.
//
// Ordering and progress:
//  * in the queue every pass-1 item of a matrix comes before any of its pass-2
//    items, and workgroups take items strictly in queue order;
//  * a pass-2 item first waits until the matrix's pass-1 counter reaches its
//    pass-1 tile count.  All those pass-1 items were taken earlier by running
//    workgroups, and pass-1 items never wait, so the wait always ends,
//    whatever the grid size and however many workgroups are resident;
//  * pass-1 writers fence their U/W stores at device (agent) scope before
//    bumping the counter, and the waiting side fences after seeing the count,
//    so the weights written on another XCD are visible (each XCD has its own
//    L2);
//  * a pass-2 tile split over y writes float64 partial tiles; the workgroup
//    that completes the last chunk of a tile (per-tile arrival counter) sums
//    the chunks in chunk order -- so the result does not depend on arrival
//    order -- and writes C.
#pragma once

#include "pairwise.hpp"

namespace pald {

// Per-matrix description, built on the host.
struct BatchMatrix {
    int64_t off;       // element offset of D / U / C in the packed arrays (ld = n)
    int64_t woff;      // float offset of this matrix's weights in the weight region
    int64_t poff;      // double offset of its first partial tile (y_chunks > 1)
    int32_t n;
    int32_t ldw;       // leading dimension of its weights (multiple of 4)
    int32_t tiles1;    // pass-1 tiles = number of pass-1 items
    int32_t y_chunks;  // pass-2 y split
    int32_t y_per_chunk;
    int32_t ctr2;      // index of its first per-tile arrival counter (y_chunks > 1)
    int32_t vec_d;     // rows of D start on 16-byte boundaries (given an aligned base)
    int32_t tile2;     // pass-2 tile side (BATCH_P2_T or BATCH_P2S_T)
};

// A value every lane of the wave holds, moved to a scalar register (the item
// and matrix records are read from LDS, which the compiler cannot prove
// uniform; as scalars they take no vector registers across the tile body).
__device__ __forceinline__ int32_t uniform_i32(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Item kinds.
constexpr int32_t ITEM_PASS1 = 0;
constexpr int32_t ITEM_PASS2 = 1;

#ifndef PALD_BATCH_THREADS
#define PALD_BATCH_THREADS 256
#endif
#ifndef PALD_BATCH_MIN_BLOCKS
#define PALD_BATCH_MIN_BLOCKS 3
#endif
constexpr int BATCH_THREADS = PALD_BATCH_THREADS;
// One pass-1 shape (64 x 64 tiles, 2 x 8 counters per thread) and one pass-2
// shape (64 x 64 tiles, 4 x 4 pairs), both inlined in one kernel compiled for
// 3 waves per SIMD (168 VGPRs).  The tile functions get the thread index
// through opaque_tid(), so the per-thread addressing they derive from it is
// recomputed per work item instead of being held across the item loop; the
// larger single-matrix pass-1 register tile would not fit that budget.
constexpr int BATCH_P1_T = 64, BATCH_P1_RX = BATCH_THREADS == 256 ? 2 : 1;
#ifndef PALD_P2_KY
#define PALD_P2_KY 12
#endif
constexpr int BATCH_P2_T = 64, BATCH_P2_RX = BATCH_THREADS == 256 ? 4 : 2, BATCH_P2_KY = PALD_P2_KY;
using BatchP1 = Pass1Cfg<BATCH_P1_T, BATCH_P1_RX, 8, 16>;
using BatchP2 = Pass2Cfg<BATCH_P2_T, BATCH_P2_RX, BATCH_P2_KY>;
// The small pass-2 shape: 32 x 32 tiles, one x and four z per thread (less
// padding and less duplicated work on diagonal tiles for mid-size matrices).
constexpr int BATCH_P2S_T = 32, BATCH_P2S_RX = BATCH_THREADS == 256 ? 1 : 0;
using BatchP2S = Pass2Cfg<BATCH_P2S_T, BATCH_P2S_RX, BATCH_P2_KY>;
static_assert(BatchP1::NT == BATCH_THREADS && BatchP2::NT == BATCH_THREADS && BatchP2S::NT == BATCH_THREADS,
              "all batched tile shapes use one workgroup size");
// Pass-1 items (64 x 64 pair regions) run as one lanes-over-pairs pass1_tile
// (default), or with PALD_BATCH_P1_LANES_Z = 1 as 8 x 16 lanes-over-z tiles
// (2 x 2 waves of 4 x 8 pairs, 2 z per lane and 128 z per stage), which are
// slower here at the kernel's 3 waves per SIMD.
#ifndef PALD_BATCH_P1_LANES_Z
#define PALD_BATCH_P1_LANES_Z 0
#endif
#ifndef PALD_BATCH_P1Z_NC
#define PALD_BATCH_P1Z_NC 2
#endif
using BatchP1z = P1zCfg<2, 2, PALD_BATCH_P1Z_NC>;
static_assert(BatchP1z::NT == BATCH_THREADS || !PALD_BATCH_P1_LANES_Z, "lanes-over-z pass-1 tiles use 4 waves");
static_assert(BATCH_P1_T % BatchP1z::TX == 0 && BATCH_P1_T % BatchP1z::TY == 0, "sub-tiles must tile a pass-1 item");
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int BATCH_LDS_VEC =
    cmax(PALD_BATCH_P1_LANES_Z ? BatchP1z::LDS_WORDS / 4 : BatchP1::LDS_VEC, cmax(BatchP2::LDS_VEC, BatchP2S::LDS_VEC));

// Counter layout (uint32): [0] queue head, [1 .. count] pass-1 done counts,
// [1 + count ..] per-tile arrival counters of split pass-2 tiles.
// Timestamps (uint64, optional): [2m] first item start, [2m+1] last item end.
__global__ void batch_reset_kernel(uint32_t *__restrict__ ctr, int64_t nctr, uint64_t *__restrict__ stamps,
                                   int64_t nmat) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nctr; i += (int64_t)gridDim.x * blockDim.x)
        ctr[i] = 0u;
    if (stamps)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nmat;
             i += (int64_t)gridDim.x * blockDim.x) {
            stamps[2 * i] = ~0ull;
            stamps[2 * i + 1] = 0ull;
        }
}

// Split mode, first launch: every pass-1 tile of every matrix as one
// workgroup of the single-matrix lanes-over-z tile (6 waves per SIMD), which
// the persistent kernel's register budget (set by its pass-2 tile) could not
// hold.  tiles[k] = {matrix, X0, Y0, 0}: the tiles of the upper-triangular
// TY x TY squares, listed largest matrix first and taken in list order, so
// the last tiles are the cheapest.  (Giving each XCD a contiguous eighth of
// the list, as the single-matrix kernels do for L2 reuse, would hand one XCD
// all the tiles of the largest matrices: 121.6 instead of 117.4 ms per
// 2000-matrix batch.)
// The tile is the single-matrix one, 16 x 16 pairs of 8 waves, compiled like
// it for 8 waves per SIMD (64 VGPRs, 4 workgroups of 32 KB of LDS per CU)
// with the component reads not run ahead: 95.0 ms per 2000-matrix batch,
// against 96.5 with an 8 x 16 tile of 4 waves at 6 waves per SIMD (its 24 KB
// of LDS allow no more than 6 workgroups per CU).
#ifndef PALD_BATCH_P1Z_GX
#define PALD_BATCH_P1Z_GX 4
#endif
#ifndef PALD_BATCH_P1Z_GY
#define PALD_BATCH_P1Z_GY 2
#endif
#ifndef PALD_BATCH_P1Z_MIN_WAVES
#define PALD_BATCH_P1Z_MIN_WAVES 8
#endif
#ifndef PALD_BATCH_P1Z_AHEAD
#define PALD_BATCH_P1Z_AHEAD 0
#endif
using BatchFocusCfg = P1zCfg<PALD_BATCH_P1Z_GX, PALD_BATCH_P1Z_GY, PALD_P1Z_NC>;
__device__ __forceinline__ void batched_focus_one(int tid, uint32_t *smw, const int4 t,
                                                  const BatchMatrix *__restrict__ mats, const float *__restrict__ D,
                                                  int32_t *__restrict__ U, float *__restrict__ Wr,
                                                  uint64_t *__restrict__ stamps, int32_t d_aligned) {
    const int32_t mi = t.x;
    const int64_t moff = mats[mi].off, mwoff = mats[mi].woff;
    const int64_t n = mats[mi].n, ldw = mats[mi].ldw;
    const bool vec_d = d_aligned && mats[mi].vec_d;
    if (stamps && tid == 0)
        atomicMin((unsigned long long *)&stamps[2 * mi], (unsigned long long)wall_clock64());
    pass1z_tile<PALD_BATCH_P1Z_GX, PALD_BATCH_P1Z_GY, PALD_P1Z_NC, (bool)PALD_BATCH_P1Z_AHEAD>(tid, smw, D + moff, n, n, U ? U + moff : nullptr, n,
                                                                 Wr + mwoff, ldw, t.y, t.z, 0, n, false, vec_d);
}

// One tile per workgroup; launched in pieces of gridDim.x tiles from tile0.
__global__ __launch_bounds__(BatchFocusCfg::NT, PALD_BATCH_P1Z_MIN_WAVES) void batched_focus_kernel(
    const int4 *__restrict__ tiles, const BatchMatrix *__restrict__ mats, const float *__restrict__ D,
    int32_t *__restrict__ U, float *__restrict__ Wr, uint64_t *__restrict__ stamps, int32_t d_aligned,
    int32_t tile0) {
    __shared__ uint32_t smw[BatchFocusCfg::LDS_WORDS];
    const int32_t k = tile0 + (int32_t)blockIdx.x;
    batched_focus_one((int)threadIdx.x, smw, tiles[k], mats, D, U, Wr, stamps, d_aligned);
}

// WITH_P1: the queue holds pass-1 items too (the one-launch form); without
// them (split mode) the kernel carries the pass-2 path only, with its own
// register allocation.  P2_FEW_SGPR picks the compare block's form.
#ifndef PALD_BATCH_SPLIT_FEW_SGPR
#define PALD_BATCH_SPLIT_FEW_SGPR 1
#endif
// Split mode, second launch when every matrix runs 64-wide pass-2 tiles with
// no y split (the tuned table's choice): a lean persistent kernel holding
// only what that needs across a tile.  Workgroups take the pass-2 items
// (largest matrix first) with one atomic increment of ctr[0] (zeroed by the
// reset kernel).  With less state live across the tile its loop reloads
// fewer spilled scalars than the general kernel's: 106.5 against 116.8 ms per
// 2000-matrix batch (107.5 with the scalar-register-saving compare block).
#ifndef PALD_BATCH_LEAN_PASS2
#define PALD_BATCH_LEAN_PASS2 1
#endif
// The one-launch form's lean kernel (batched_lean_kernel) under the same condition.
#ifndef PALD_BATCH_LEAN_ONE_LAUNCH
#define PALD_BATCH_LEAN_ONE_LAUNCH 1
#endif
#ifndef PALD_BATCH_LEAN_FEW_SGPR
#define PALD_BATCH_LEAN_FEW_SGPR 0
#endif
// The lean kernel's tile: 64 x 64 with 2 x 4 pairs per thread (512 threads,
// about 100 VGPRs), the single-matrix pass-2 shape -- more waves per SIMD than
// the general kernel's 4 x 4 pairs, so the compares of one wave issue beside
// the additions of another.
#ifndef PALD_BATCH_LEAN_RX
#define PALD_BATCH_LEAN_RX 2
#endif
#ifndef PALD_BATCH_LEAN_MIN_WAVES
#define PALD_BATCH_LEAN_MIN_WAVES 4
#endif
#ifndef PALD_BATCH_LEAN_KY
#define PALD_BATCH_LEAN_KY 24
#endif
using BatchLeanP2 = Pass2Cfg<BATCH_P2_T, PALD_BATCH_LEAN_RX, PALD_BATCH_LEAN_KY>;
constexpr int BATCH_LEAN_THREADS = BatchLeanP2::NT;
__global__ __launch_bounds__(BATCH_LEAN_THREADS, PALD_BATCH_LEAN_MIN_WAVES) void batched_pass2_lean_kernel(
    const int4 *__restrict__ items, int32_t total, const BatchMatrix *__restrict__ mats, const float *__restrict__ D,
    float *__restrict__ C, const float *__restrict__ Wr, uint32_t *__restrict__ ctr, uint64_t *__restrict__ stamps,
    int32_t d_aligned) {
    __shared__ uint4 sm[BatchLeanP2::LDS_VEC];
    __shared__ int32_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int32_t)atomicAdd(&ctr[0], 1u);
        __syncthreads();
        const int32_t it = uniform_i32(s_item);
        if (it >= total) break;
        const int4 item = items[it];
        const int32_t mi = item.x;
        const int64_t moff = mats[mi].off, mwoff = mats[mi].woff, n = mats[mi].n, ldw = mats[mi].ldw;
        const bool vec_d = d_aligned && mats[mi].vec_d;
        int32_t bx, bz;
        tri_tile(item.z, bx, bz);
        pass2_tile<BATCH_P2_T, PALD_BATCH_LEAN_RX, PALD_BATCH_LEAN_KY, false, (bool)PALD_BATCH_LEAN_FEW_SGPR, true>(
            opaque_tid(), sm, D + moff, n, n, Wr + mwoff, ldw, Pass2Out{C + moff, n, nullptr, nullptr}, bx, bz, 0, n,
            vec_d, true);
        if (stamps && threadIdx.x == 0) {
            __threadfence();
            atomicMax((unsigned long long *)&stamps[2 * mi + 1], (unsigned long long)wall_clock64());
        }
        __syncthreads();  // s_item and the tile buffers are reused by the next item
    }
}

// The one-launch form when every matrix runs 64-wide pass-2 tiles with no y
// split: the lean kernel's pass-2 tile and, for the pass-1 items (64 x 64
// regions of pairs x <= y), the single-matrix lanes-over-z tile walked over
// the region's 16 x 16 squares, in one persistent kernel of 512 threads with
// the one-launch protocol (a pass-2 item waits until its matrix's pass-1
// items are all counted; every pass-1 item of a matrix is earlier in the
// queue and pass-1 items never wait, so every wait ends).  On the
// 2000-matrix batch it takes 135 ms against 134 ms for the general kernel,
// with per-matrix latency p50 1.6 ms / p99 2.6 ms against 2.3 / 4.1 ms; the
// lanes-over-pairs 64 x 64 tile with 1 x 8 pairs per thread for the pass-1
// items took 139 ms.
constexpr int BATCH_LEAN1_LDS_VEC = cmax(BatchLeanP2::LDS_VEC, P1zMain::LDS_WORDS / 4);
static_assert(P1zMain::NT == BATCH_LEAN_THREADS && P1zMain::TX == 16 && P1zMain::TY == 16,
              "the one-launch lean kernel walks 16 x 16 pass-1 squares with the pass-2 tile's threads");
__global__ __launch_bounds__(BATCH_LEAN_THREADS, PALD_BATCH_LEAN_MIN_WAVES) void batched_lean_kernel(
    const int4 *__restrict__ items, int32_t total, const BatchMatrix *__restrict__ mats, const float *__restrict__ D,
    int32_t *__restrict__ U, float *__restrict__ C, float *__restrict__ Wr, uint32_t *__restrict__ ctr,
    uint64_t *__restrict__ stamps, int32_t d_aligned) {
    __shared__ uint4 sm[BATCH_LEAN1_LDS_VEC];
    __shared__ int32_t s_item;
    uint32_t *const done1 = ctr + 1;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int32_t)atomicAdd(&ctr[0], 1u);
        __syncthreads();
        const int32_t it = uniform_i32(s_item);
        if (it >= total) break;
        const int4 item = items[it];
        const int32_t mi = item.x;
        const int64_t moff = mats[mi].off, mwoff = mats[mi].woff, n = mats[mi].n, ldw = mats[mi].ldw;
        const int32_t tiles1 = mats[mi].tiles1;
        const bool vec_d = d_aligned && mats[mi].vec_d;
        if (stamps && threadIdx.x == 0)
            atomicMin((unsigned long long *)&stamps[2 * mi], (unsigned long long)wall_clock64());
        if (item.y == ITEM_PASS1) {
            int32_t bx, by;
            tri_tile(item.z, bx, by);
            for (int sy = 0; sy < BATCH_P1_T / 16; ++sy)
                for (int sx = 0; sx < BATCH_P1_T / 16; ++sx) {
                    const int64_t X0 = (int64_t)bx * BATCH_P1_T + 16 * sx, Y0 = (int64_t)by * BATCH_P1_T + 16 * sy;
                    if (X0 >= n || Y0 >= n || X0 > Y0) continue;  // squares holding a pair x <= y
                    pass1z_tile<PALD_P1Z_GX, PALD_P1Z_GY, PALD_P1Z_NC>(
                        opaque_tid(), reinterpret_cast<uint32_t *>(sm), D + moff, n, n, U ? U + moff : nullptr, n,
                        Wr + mwoff, ldw, X0, Y0, 0, n, false, vec_d);
                    __syncthreads();  // the next square reuses the stage buffers
                }
            __threadfence();  // release this thread's U / W stores at device scope
            __syncthreads();
            if (threadIdx.x == 0) atomicAdd(&done1[mi], 1u);
        } else {
            if (threadIdx.x == 0) {
                while (__hip_atomic_load(&done1[mi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (uint32_t)tiles1)
                    __builtin_amdgcn_s_sleep(2);
                __atomic_thread_fence(__ATOMIC_ACQUIRE);
            }
            __syncthreads();
            __threadfence();  // acquire for every wave before reading the weights
            int32_t bx, bz;
            tri_tile(item.z, bx, bz);
            pass2_tile<BATCH_P2_T, PALD_BATCH_LEAN_RX, PALD_BATCH_LEAN_KY, false, (bool)PALD_BATCH_LEAN_FEW_SGPR, true>(
                opaque_tid(), sm, D + moff, n, n, Wr + mwoff, ldw, Pass2Out{C + moff, n, nullptr, nullptr}, bx, bz, 0,
                n, vec_d, true);
        }
        if (stamps && threadIdx.x == 0) {
            __threadfence();
            atomicMax((unsigned long long *)&stamps[2 * mi + 1], (unsigned long long)wall_clock64());
        }
        __syncthreads();  // s_item and the tile buffers are reused by the next item
    }
}

template <bool WITH_P1, bool P2_FEW_SGPR>
__global__ __launch_bounds__(BATCH_THREADS, PALD_BATCH_MIN_BLOCKS) void batched_cohesion_kernel(
    const int4 *__restrict__ items, int32_t total, const BatchMatrix *__restrict__ mats, const float *__restrict__ D,
    int32_t *__restrict__ U, float *__restrict__ C, float *__restrict__ Wr, double *__restrict__ Pr,
    uint32_t *__restrict__ ctr, int32_t count, uint64_t *__restrict__ stamps, int32_t d_aligned) {
    __shared__ uint4 sm[BATCH_LDS_VEC];
    // The current item and its matrix record live in LDS and are re-read after
    // each tile: nothing has to stay in registers across the tile body.
    __shared__ int32_t s_item;
    __shared__ int4 s_it;
    __shared__ BatchMatrix s_m;
    __shared__ int32_t s_last;
    const int tid = threadIdx.x;
    uint32_t *const done1 = ctr + 1;

    for (;;) {
        if (tid == 0) {
            const int32_t it = (int32_t)atomicAdd(&ctr[0], 1u);
            s_item = it;
            if (it < total) {
                s_it = items[it];
                s_m = mats[s_it.x];
            }
        }
        __syncthreads();
        if (s_item >= total) break;  // uniform: every thread reads the same value

        {
            const int32_t mi = uniform_i32(s_it.x), kind = uniform_i32(s_it.y), tile = uniform_i32(s_it.z),
                          chunk = uniform_i32(s_it.w);
            const int64_t moff = uniform_i64(s_m.off), mwoff = uniform_i64(s_m.woff), mpoff = uniform_i64(s_m.poff);
            const int32_t mldw = uniform_i32(s_m.ldw), mtiles1 = uniform_i32(s_m.tiles1),
                          mychunks = uniform_i32(s_m.y_chunks), mypc = uniform_i32(s_m.y_per_chunk),
                          mctr2 = uniform_i32(s_m.ctr2);
            if (stamps && tid == 0)
                atomicMin((unsigned long long *)&stamps[2 * mi], (unsigned long long)wall_clock64());
            const int64_t n = uniform_i32(s_m.n);
            const bool vec_d = d_aligned && uniform_i32(s_m.vec_d);
            if (WITH_P1 && kind == ITEM_PASS1) {
                int32_t bx, by;
                tri_tile(tile, bx, by);
                int32_t *Um = U ? U + moff : nullptr;
                if (PALD_BATCH_P1_LANES_Z) {
                    // the region's sub-tiles holding a pair x <= y (each pair once:
                    // a sub-tile writes its pairs x <= y and their mirrors)
                    for (int sy = 0; sy < BATCH_P1_T / BatchP1z::TY; ++sy)
                        for (int sx = 0; sx < BATCH_P1_T / BatchP1z::TX; ++sx) {
                            const int64_t X0 = (int64_t)bx * BATCH_P1_T + sx * BatchP1z::TX;
                            const int64_t Y0 = (int64_t)by * BATCH_P1_T + sy * BatchP1z::TY;
                            if (X0 >= n || Y0 >= n || X0 > Y0 + (BatchP1z::TY - 1)) continue;
                            pass1z_tile<2, 2, PALD_BATCH_P1Z_NC>(opaque_tid(), reinterpret_cast<uint32_t *>(sm), D + moff, n, n, Um, n,
                                                 Wr + mwoff, mldw, X0, Y0, 0, n, false, vec_d);
                            __syncthreads();  // the next sub-tile reuses the stage buffers
                        }
                } else {
                    pass1_tile<BATCH_P1_T, BATCH_P1_RX, 8, 16>(opaque_tid(), sm, D + moff, n, n, Um, n, Wr + mwoff, mldw,
                                                               bx, by, 0, n, false, vec_d);
                }
                __threadfence();  // release this thread's U / W stores at device scope
                __syncthreads();
                if (tid == 0) atomicAdd(&done1[mi], 1u);
            } else {
                if (tid == 0) {
                    while (__hip_atomic_load(&done1[mi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                           (uint32_t)mtiles1)
                        __builtin_amdgcn_s_sleep(2);
                    __atomic_thread_fence(__ATOMIC_ACQUIRE);
                }
                __syncthreads();
                __threadfence();  // acquire for every wave before reading the weights
                int32_t bx, bz;
                tri_tile(tile, bx, bz);
                const int64_t ybeg = (int64_t)chunk * mypc;
                const int64_t yend = min(n, ybeg + (int64_t)mypc);
                const int32_t t2 = uniform_i32(s_m.tile2);
                const int64_t TT2 = 2 * (int64_t)t2 * t2;
                Pass2Out out{nullptr, 0, nullptr, nullptr};
                if (mychunks == 1) {
                    out.C = C + moff;
                    out.ldc = n;
                } else {
                    out.tile = Pr + mpoff + ((int64_t)tile * mychunks + chunk) * TT2;
                }
                if (t2 == BATCH_P2_T)
                    pass2_tile<BATCH_P2_T, BATCH_P2_RX, BATCH_P2_KY, false, P2_FEW_SGPR>(opaque_tid(), sm, D + moff, n, n, Wr + mwoff,
                                                                           mldw, out, bx, bz, ybeg, yend, vec_d, true);
                else
                    pass2_tile<BATCH_P2S_T, BATCH_P2S_RX, BATCH_P2_KY, false, P2_FEW_SGPR>(opaque_tid(), sm, D + moff, n, n,
                                                                             Wr + mwoff, mldw, out, bx, bz, ybeg, yend,
                                                                             vec_d, true);
                if (mychunks > 1) {
                    __threadfence();
                    __syncthreads();
                    if (tid == 0) {
                        const uint32_t prev = atomicAdd(&ctr[1 + count + mctr2 + tile], 1u);
                        s_last = (prev == (uint32_t)(mychunks - 1)) ? 1 : 0;
                        if (s_last) __atomic_thread_fence(__ATOMIC_ACQUIRE);
                    }
                    __syncthreads();
                    if (s_last) {
                        __threadfence();
                        const int32_t chunks = mychunks;
                        int32_t tbx, tbz;
                        tri_tile(tile, tbx, tbz);
                        const int32_t tt = uniform_i32(s_m.tile2);
                        const int64_t TTr = 2 * (int64_t)tt * tt;
                        const int64_t X0 = (int64_t)tbx * tt, Z0 = (int64_t)tbz * tt;
                        const double nm1 = (double)(n - 1);
                        const double *tiles = Pr + mpoff + (int64_t)tile * chunks * TTr;
                        float *Cm = C + moff;
                        for (int e = tid; e < tt * tt; e += BATCH_THREADS) {
                            const int i = e / tt, j = e % tt;
                            const int64_t x = X0 + i, z = Z0 + j;
                            if (x >= n || z >= n) continue;
                            double sf = 0.0, sr = 0.0;
                            for (int32_t k = 0; k < chunks; ++k) {
                                sf += tiles[k * TTr + e];
                                sr += tiles[k * TTr + (int64_t)tt * tt + e];
                            }
                            Cm[x * n + z] = (float)(sf / nm1);
                            if (tbx != tbz) Cm[z * n + x] = (float)(sr / nm1);
                        }
                    }
                }
            }
            if (stamps && tid == 0) {
                __threadfence();
                atomicMax((unsigned long long *)&stamps[2 * mi + 1], (unsigned long long)wall_clock64());
            }
        }
        __syncthreads();  // LDS (tile buffers, s_item, s_it, s_m, s_last) is reused by the next item
    }
}

}  // namespace pald
