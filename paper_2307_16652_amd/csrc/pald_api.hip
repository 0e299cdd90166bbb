// pald_api.hip -- host side of the libpald C ABI (declared in include/pald.h).
//
// Argument checking, launch planning (tile grids, z/y splits, workspace
// layout) and kernel launches on the caller's stream.  All arithmetic of the
// method happens in the kernels of pairwise.hpp / batched.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "pald.h"
#include "host_common.hpp"
#include "pairwise.hpp"
#include "batched.hpp"
#include "rows.hpp"
#include "triplet.hpp"
#include "tuned_gfx950.h"

namespace {

using namespace pald;
using namespace pald_host;

// ---- single-matrix tile configuration -------------------------------------
// pass 1: 128 x 128 (x,y) tiles, 4 x 8 counters per thread (512 threads, 4
// waves per SIMD: 128 VGPRs), 16 z rows per stage
#ifndef PALD_P1_RX
#define PALD_P1_RX 4
#endif
constexpr int P1_T = 128, P1_RX = PALD_P1_RX, P1_RY = 8, P1_KZ = 16;
using P1 = Pass1Cfg<P1_T, P1_RX, P1_RY, P1_KZ>;
// PALD_P1_LANES_Z = 1 (default): pass 1 runs pass1z_focus_kernel (lanes over z,
// counts on the scalar unit); 0: pass1_focus_kernel (lanes over pairs)
#ifndef PALD_P1_LANES_Z
#define PALD_P1_LANES_Z 1
#endif
constexpr bool P1_LANES_Z = PALD_P1_LANES_Z != 0;
// z granularity of a pass-1 chunk: one stage of whichever kernel runs
constexpr int P1_ZQ = P1_LANES_Z ? P1Z_ZS : P1_KZ;
// pass 2: symmetric 64 x 64 (x,z) tiles, P2_RX x 4 pairs (both directions) per thread,
// P2_KY y rows per stage.  2 x 4 pairs (512 threads, about 100 VGPRs: 5 waves per
// SIMD) against 4 x 4 (256 threads, 168 VGPRs: 3 waves): n = 16384 pass 2 in
// 442 against 498 ms -- the compares of one wave issue beside the float32
// additions of another, which needs more waves per SIMD than the larger
// register tile leaves.
#ifndef PALD_P2_RX
#define PALD_P2_RX 2
#endif
// 24 y rows per LDS stage (two split runs): 429 against 443 ms with 12
#ifndef PALD_P2_SINGLE_KY
#define PALD_P2_SINGLE_KY 24
#endif
constexpr int P2_T = 64, P2_RX = PALD_P2_RX, P2_KY = PALD_P2_SINGLE_KY;
using P2 = Pass2Cfg<P2_T, P2_RX, P2_KY>;

constexpr int TARGET_WORKGROUPS = 1024;  // >= 4 per CU on a 256-CU part
// Large tile grids are launched in pieces so that no single dispatch runs for
// more than a few seconds (n = 65536: about 2-3 s per piece).
constexpr int64_t P1_TILES_PER_LAUNCH = 32768;
constexpr int64_t P1Z_TILES_PER_LAUNCH = 1 << 20;  // n = 65536: 8 launches of about 1 s
constexpr int64_t P2_TILES_PER_LAUNCH = 65536;
// Triplet owner tiles differ in work by up to n / 64 times (a tile streams
// bz - bx + 1 blocks of middle indices), so their launches are cut by work:
// at most this many blocks summed over a launch's tiles (about 1 s), and at
// most TRI_TILES_PER_LAUNCH tiles.
constexpr int64_t TRI_BLOCKS_PER_LAUNCH = (int64_t)1 << 23;
constexpr int64_t TRI_TILES_PER_LAUNCH = (int64_t)1 << 20;
// A dispatch counts its work-items along x in 32 bits: every launched piece
// must stay below 2^32 of them.
constexpr int64_t MAX_X_ITEMS = (int64_t)1 << 32;
static_assert(P1_TILES_PER_LAUNCH * P1::NT < MAX_X_ITEMS && P1Z_TILES_PER_LAUNCH * P1Z_NT < MAX_X_ITEMS &&
                  P2_TILES_PER_LAUNCH * P2::NT < MAX_X_ITEMS &&
                  TRI_TILES_PER_LAUNCH * tri_threads<true>() < MAX_X_ITEMS &&
                  TRI_TILES_PER_LAUNCH * tri_threads<false>() < MAX_X_ITEMS,
              "launch pieces must hold fewer than 2^32 work-items");

// ---- options -----------------------------------------------------------------
struct Opts {
    int variant = PALD_VARIANT_AUTO;
    int accum = PALD_ACC_COMPENSATED;
    int y_chunks = 0;
    int z_chunks = 0;
    uint32_t flags = 0;
};

pald_status read_opts(const pald_options *o, Opts &out) {
    out = Opts{};
    if (!o) return PALD_OK;
    for (int r : o->reserved)
        if (r != 0) return PALD_ERR_UNSUPPORTED;
    if (o->variant < PALD_VARIANT_AUTO || o->variant > PALD_VARIANT_HYBRID2) return PALD_ERR_UNSUPPORTED;
    if (o->accum != PALD_ACC_COMPENSATED && o->accum != PALD_ACC_F64) return PALD_ERR_UNSUPPORTED;
    if (o->y_chunks < 0 || o->z_chunks < 0) return PALD_ERR_ARG;
    if (o->flags & ~PALD_FLAG_TIMING) return PALD_ERR_UNSUPPORTED;
    out.variant = o->variant;
    out.accum = o->accum;
    out.y_chunks = o->y_chunks;
    out.z_chunks = o->z_chunks;
    out.flags = o->flags;
    return PALD_OK;
}

// PALD_VARIANT_AUTO -> the tuned variant for n, unless it cannot take the
// other options (the triplet variant: compensated accumulation without
// splits; the hybrid: no z split), in which case pairwise.  With both splits
// automatic the tuned entry's splits are taken too.
void resolve_variant(int64_t n, Opts &o) {
    if (o.variant != PALD_VARIANT_AUTO) return;
    const pald_tuned::VariantPick *pick = &pald_tuned::kVariants[0];
    for (const auto &e : pald_tuned::kVariants)
        if (e.n <= n) pick = &e;
    int32_t v = pick->variant;
    if (o.y_chunks == 0 && o.z_chunks == 0) {
        const bool y_ok = v == PALD_VARIANT_PAIRWISE || v == PALD_VARIANT_HYBRID;
        const bool z_ok = v == PALD_VARIANT_PAIRWISE || v == PALD_VARIANT_HYBRID2;
        const bool f64_ok = v == PALD_VARIANT_PAIRWISE || v == PALD_VARIANT_HYBRID;
        if ((y_ok || pick->y_chunks == 0) && (z_ok || pick->z_chunks == 0) &&
            (f64_ok || o.accum == PALD_ACC_COMPENSATED)) {
            o.y_chunks = pick->y_chunks;
            o.z_chunks = pick->z_chunks;
        }
    }
    if (v == PALD_VARIANT_TRIPLET && (o.accum != PALD_ACC_COMPENSATED || o.y_chunks != 0 || o.z_chunks != 0))
        v = PALD_VARIANT_PAIRWISE;
    if (v == PALD_VARIANT_HYBRID && o.z_chunks != 0) v = PALD_VARIANT_PAIRWISE;
    if (v == PALD_VARIANT_HYBRID2 && (o.accum != PALD_ACC_COMPENSATED || o.y_chunks != 0)) v = PALD_VARIANT_PAIRWISE;
    // the triplet pass 2's fixed-point sums are exact up to 2^18 points
    if ((v == PALD_VARIANT_TRIPLET || v == PALD_VARIANT_HYBRID2) && n > ((int64_t)1 << 18)) v = PALD_VARIANT_PAIRWISE;
    o.variant = v;
}

// ---- launch planning ------------------------------------------------------
struct Plan {
    int64_t n = 0;
    int64_t nb1 = 0, tiles1 = 0;  // pass-1 tile grid (upper triangle)
    int32_t z_chunks = 1, z_per_chunk = 0;
    int64_t nb2 = 0, tiles2 = 0;  // pass-2 tile grid (upper triangle)
    int32_t y_chunks = 1, y_per_chunk = 0;
    int64_t ldw = 0;
    size_t off_w = 0, off_u = 0, off_part = 0, bytes = 0;
    bool need_u_scratch = false;
};

pald_status make_plan(int64_t n, const Opts &o, Plan &p) {
    p = Plan{};
    p.n = n;
    if (P1_LANES_Z) {  // P1Z_SPLIT tiles per upper-triangular P1Z_TY x P1Z_TY square
        p.nb1 = ceil_div(n, P1Z_TY);
        p.tiles1 = P1Z_SPLIT * (p.nb1 * (p.nb1 + 1) / 2);
    } else {
        p.nb1 = ceil_div(n, P1_T);
        p.tiles1 = p.nb1 * (p.nb1 + 1) / 2;
    }
    if (p.tiles1 > INT32_MAX) return PALD_ERR_UNSUPPORTED;
    int64_t zc = o.z_chunks;
    if (zc == 0) {
        zc = ceil_div(TARGET_WORKGROUPS, p.tiles1);
        zc = std::min<int64_t>(zc, std::max<int64_t>(1, n / (4 * P1_ZQ)));
        // very long tiles: z chunks of at most 16384, so that the tiles running
        // at the same time stay close in z and share their rows of D in L2
        // (n = 65536: pass 1 9.98 -> 8.78 s with 4 chunks; at n = 16384 a split
        // only adds its atomics: 132 -> 136 ms with 2 chunks)
        if (n > 32768) zc = std::max<int64_t>(zc, ceil_div(n, 16384));
    }
    zc = std::max<int64_t>(1, std::min<int64_t>(zc, ceil_div(n, P1_ZQ)));
    p.z_per_chunk = (int32_t)(ceil_div(ceil_div(n, zc), P1_ZQ) * P1_ZQ);
    p.z_chunks = (int32_t)ceil_div(n, p.z_per_chunk);

    p.nb2 = ceil_div(n, P2_T);
    p.tiles2 = p.nb2 * (p.nb2 + 1) / 2;
    if (p.tiles2 > INT32_MAX) return PALD_ERR_UNSUPPORTED;
    int64_t yc = o.y_chunks;
    if (yc == 0) {
        yc = ceil_div(TARGET_WORKGROUPS, p.tiles2);
        yc = std::min<int64_t>(yc, std::max<int64_t>(1, n / (2 * P2_KY)));
    }
    yc = std::max<int64_t>(1, std::min<int64_t>(yc, ceil_div(n, P2_KY)));
    p.y_per_chunk = (int32_t)(ceil_div(ceil_div(n, yc), P2_KY) * P2_KY);
    p.y_chunks = (int32_t)ceil_div(n, p.y_per_chunk);
    if (p.y_chunks > 65535 || p.z_chunks > 65535) return PALD_ERR_UNSUPPORTED;

    p.ldw = (int64_t)align_up((size_t)n, 64);
    size_t off = 0;
    p.off_w = off;
    off = align_up(off + (size_t)n * (size_t)p.ldw * sizeof(float), ALIGN);
    // a split pass 1 accumulates into U; the hybrid's triplet pass 1 always does
    p.need_u_scratch = p.z_chunks > 1 || o.variant == PALD_VARIANT_HYBRID;
    p.off_u = off;
    if (p.need_u_scratch) off = align_up(off + (size_t)n * (size_t)n * sizeof(int32_t), ALIGN);
    p.off_part = off;
    if (p.y_chunks > 1) off = align_up(off + (size_t)p.y_chunks * (size_t)n * (size_t)n * sizeof(double), ALIGN);
    p.bytes = std::max<size_t>(off, ALIGN);
    return PALD_OK;
}

// Pass 1 into (U, W); W may be null.  Returns after enqueueing.
pald_status run_pass1(const float *D, int64_t n, int64_t ldd, int32_t *U, int64_t ldu, float *W,
                      int64_t ldw, const Plan &p, hipStream_t s, bool timing) {
    const int vec = (aligned16(D) && ldd % 4 == 0) ? 1 : 0;
    if (p.z_chunks == 1) {
        const int64_t per_launch = P1_LANES_Z ? P1Z_TILES_PER_LAUNCH : P1_TILES_PER_LAUNCH;
        for (int64_t t0 = 0; t0 < p.tiles1; t0 += per_launch) {
            ScopedTiming tm(timing, 0, s);
            const unsigned g = (unsigned)std::min<int64_t>(per_launch, p.tiles1 - t0);
            if (P1_LANES_Z)
                pass1z_focus_kernel<<<dim3(g, 1), P1Z_NT, 0, s>>>(D, n, ldd, U, ldu, W, ldw, p.z_per_chunk, 0, vec,
                                                                  (int32_t)t0);
            else
                pass1_focus_kernel<P1_T, P1_RX, P1_RY, P1_KZ>
                    <<<dim3(g, 1), P1::NT, 0, s>>>(D, n, ldd, U, ldu, W, ldw, p.z_per_chunk, 0, vec, (int32_t)t0);
            if (pald_status st = launch_status(); st != PALD_OK) return st;
        }
        return PALD_OK;
    }
    {
        const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(n, 256), 64);
        zero_i32_kernel<<<dim3(gx, rows_grid(n)), 256, 0, s>>>(U, ldu, n);
        if (pald_status st = launch_status(); st != PALD_OK) return st;
    }
    // (in pieces of at most per_launch tiles, as above: a dispatch holds fewer
    // than 2^32 work-items along x)
    const int64_t per_launch = P1_LANES_Z ? P1Z_TILES_PER_LAUNCH : P1_TILES_PER_LAUNCH;
    for (int64_t t0 = 0; t0 < p.tiles1; t0 += per_launch) {
        ScopedTiming tm(timing, 0, s);
        const unsigned g = (unsigned)std::min<int64_t>(per_launch, p.tiles1 - t0);
        if (P1_LANES_Z)
            pass1z_focus_kernel<<<dim3(g, (unsigned)p.z_chunks), P1Z_NT, 0, s>>>(D, n, ldd, U, ldu, nullptr, ldw,
                                                                                p.z_per_chunk, 1, vec, (int32_t)t0);
        else
            pass1_focus_kernel<P1_T, P1_RX, P1_RY, P1_KZ><<<dim3(g, (unsigned)p.z_chunks), P1::NT, 0, s>>>(
                D, n, ldd, U, ldu, nullptr, ldw, p.z_per_chunk, 1, vec, (int32_t)t0);
        if (pald_status st = launch_status(); st != PALD_OK) return st;
    }
    if (W) {
        ScopedTiming tm(timing, 1, s);
        const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(n, 256), 64);
        weights_kernel<<<dim3(gx, rows_grid(n)), 256, 0, s>>>(U, ldu, W, ldw, n);
        return launch_status();
    }
    return PALD_OK;
}

pald_status run_pass2(const float *D, int64_t n, int64_t ldd, const float *W, int64_t ldw, float *C,
                      int64_t ldc, double *part, const Plan &p, bool f64, hipStream_t s, bool timing) {
    const int vecd = (aligned16(D) && ldd % 4 == 0) ? 1 : 0;
    const int vecw = (aligned16(W) && ldw % 4 == 0) ? 1 : 0;
    for (int64_t t0 = 0; t0 < p.tiles2; t0 += P2_TILES_PER_LAUNCH) {
        ScopedTiming tm(timing, 2, s);
        const dim3 grid((unsigned)std::min<int64_t>(P2_TILES_PER_LAUNCH, p.tiles2 - t0), (unsigned)p.y_chunks);
        if (f64)
            pass2_cohesion_kernel<P2_T, P2_RX, P2_KY, true>
                <<<grid, P2::NT, 0, s>>>(D, n, ldd, W, ldw, C, ldc, part, p.y_per_chunk, vecd, vecw, (int32_t)t0);
        else
            pass2_cohesion_kernel<P2_T, P2_RX, P2_KY, false>
                <<<grid, P2::NT, 0, s>>>(D, n, ldd, W, ldw, C, ldc, part, p.y_per_chunk, vecd, vecw, (int32_t)t0);
        if (pald_status st = launch_status(); st != PALD_OK) return st;
    }
    if (p.y_chunks > 1) {
        ScopedTiming tm(timing, 3, s);
        const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(n, 256), 64);
        finalize_kernel<<<dim3(gx, rows_grid(n)), 256, 0, s>>>(part, p.y_chunks, n, C, ldc);
        return launch_status();
    }
    return PALD_OK;
}

// ---- triplet variant ---------------------------------------------------------
struct TripletPlan {
    int64_t tiles = 0, ldw = 0;
    size_t off_w = 0, off_a = 0, off_b = 0, off_u = 0, bytes = 0;
};

TripletPlan triplet_plan(int64_t n) {
    TripletPlan t;
    const int64_t nb = ceil_div(n, TRI_T);
    t.tiles = nb * (nb + 1) / 2;
    t.ldw = (int64_t)align_up((size_t)n, 64);
    size_t off = 0;
    t.off_w = off;
    off = align_up(off + (size_t)n * (size_t)t.ldw * sizeof(float), ALIGN);
    t.off_a = off;
    off = align_up(off + (size_t)n * (size_t)n * sizeof(double), ALIGN);
    t.off_b = off;  // the transposed accumulator B
    off = align_up(off + (size_t)n * (size_t)n * sizeof(double), ALIGN);
    t.off_u = off;
    off = align_up(off + (size_t)n * (size_t)n * sizeof(int32_t), ALIGN);
    t.bytes = off;
    return t;
}

size_t triplet_workspace_bytes(int64_t n) { return triplet_plan(n).bytes; }

// The launch pieces of the nb (nb + 1) / 2 owner tiles, in the kernel's
// heavy-first order (diagonal d = bz - bx from nb - 1 down to 0: nb - d tiles
// of d + 1 blocks each): the first tile of every piece, then the tile count.
// One piece per dispatch; cutting by work rather than by tile count keeps a
// piece's last, long tiles from holding the GPU half idle at its end.
std::vector<int64_t> triplet_pieces(int64_t nb) {
    std::vector<int64_t> at{0};
    int64_t k = 0, blocks = 0;
    for (int64_t d = nb - 1; d >= 0; --d) {
        int64_t left = nb - d;
        while (left > 0) {
            int64_t fit = std::min((TRI_BLOCKS_PER_LAUNCH - blocks) / (d + 1), TRI_TILES_PER_LAUNCH - (k - at.back()));
            if (fit <= 0 && k == at.back()) fit = 1;  // a tile heavier than a piece runs alone
            if (fit <= 0) {
                at.push_back(k);
                blocks = 0;
                continue;
            }
            const int64_t take = std::min(fit, left);
            k += take;
            left -= take;
            blocks += take * (d + 1);
        }
    }
    at.push_back(k);
    return at;
}

// Triplet pass 1 into U (initialised here).
pald_status triplet_focus(const float *D, int64_t n, int64_t ldd, int32_t *U, int64_t ldu, hipStream_t s,
                          bool timing) {
    const TripletPlan t = triplet_plan(n);
    if (t.tiles > INT32_MAX) return PALD_ERR_UNSUPPORTED;
    triplet_init_u_kernel<<<rows_grid(n), 256, 0, s>>>(D, n, ldd, U, ldu);
    if (pald_status st = launch_status(); st != PALD_OK) return st;
    const int vec = (aligned16(D) && ldd % 4 == 0) ? 1 : 0;
    const std::vector<int64_t> pcs = triplet_pieces(ceil_div(n, TRI_T));
    for (size_t i = 0; i + 1 < pcs.size(); ++i) {
        ScopedTiming tm(timing, 5, s);
        const int64_t t0 = pcs[i];
        const unsigned g = (unsigned)(pcs[i + 1] - t0);
        triplet_kernel<false><<<g, tri_threads<false>(), 0, s>>>(D, n, ldd, nullptr, 0, U, ldu, nullptr, nullptr, vec, 0,
                                                         (int32_t)t0, 0, 1.0);
        if (pald_status st = launch_status(); st != PALD_OK) return st;
    }
    // the upper triangle holds U; mirror it
    const int64_t nb32 = ceil_div(n, 32);
    const int64_t mtiles = nb32 * (nb32 + 1) / 2;
    if (mtiles > INT32_MAX) return PALD_ERR_UNSUPPORTED;
    triplet_mirror_u_kernel<<<(unsigned)std::min<int64_t>(mtiles, 65536), 256, 0, s>>>(U, ldu, n, (int32_t)mtiles);
    return launch_status();
}

// The triplet pass 2 (PALD_VARIANT_TRIPLET: after the triplet pass 1;
// PALD_VARIANT_HYBRID2: after the pairwise pass 1 of options o).
pald_status triplet_cohesion(const float *D, int64_t n, int64_t ldd, int32_t *U, int64_t ldu, float *C, int64_t ldc,
                             void *ws, size_t ws_bytes, hipStream_t s, const Opts &o) {
    const bool timing = (o.flags & PALD_FLAG_TIMING) != 0;
    if (n > ((int64_t)1 << 18)) return PALD_ERR_UNSUPPORTED;  // the fixed-point sums are exact up to 2^18 points
    const TripletPlan t = triplet_plan(n);
    if (ws_bytes < t.bytes) return PALD_ERR_ARG;
    char *base = static_cast<char *>(ws);
    float *W = reinterpret_cast<float *>(base + t.off_w);
    unsigned long long *A = reinterpret_cast<unsigned long long *>(base + t.off_a);
    unsigned long long *B = reinterpret_cast<unsigned long long *>(base + t.off_b);
    const double scale = std::ldexp(1.0, triplet_fixed_bits(n));
    int32_t *Ub = U;
    int64_t ldub = ldu;
    if (!Ub) {
        Ub = reinterpret_cast<int32_t *>(base + t.off_u);
        ldub = n;
    }
    const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(n, 256), 64);
    if (o.variant == PALD_VARIANT_HYBRID2) {
        Opts o1 = o;
        o1.variant = PALD_VARIANT_PAIRWISE;
        Plan p1;
        if (pald_status st = make_plan(n, o1, p1); st != PALD_OK) return st;
        if (p1.ldw != t.ldw) return PALD_ERR_UNSUPPORTED;  // both lay W out with rows padded to 64
        if (pald_status st = run_pass1(D, n, ldd, Ub, ldub, W, t.ldw, p1, s, timing); st != PALD_OK) return st;
    } else {
        if (pald_status st = triplet_focus(D, n, ldd, Ub, ldub, s, timing); st != PALD_OK) return st;
        weights_kernel<<<dim3(gx, rows_grid(n)), 256, 0, s>>>(Ub, ldub, W, t.ldw, n);
        if (pald_status st = launch_status(); st != PALD_OK) return st;
    }
    triplet_init_c_kernel<<<rows_grid(n), 256, 0, s>>>(D, n, ldd, W, t.ldw, A, B, scale);
    if (pald_status st = launch_status(); st != PALD_OK) return st;
    const int vecd = (aligned16(D) && ldd % 4 == 0) ? 1 : 0;
    const std::vector<int64_t> pcs = triplet_pieces(ceil_div(n, TRI_T));
    for (size_t i = 0; i + 1 < pcs.size(); ++i) {
        ScopedTiming tm(timing, 6, s);
        const int64_t t0 = pcs[i];
        const unsigned g = (unsigned)(pcs[i + 1] - t0);
        triplet_kernel<true><<<g, tri_threads<true>(), 0, s>>>(D, n, ldd, W, t.ldw, nullptr, 0, A, B, vecd, 1, (int32_t)t0,
                                                        triplet_fixed_bits(n), scale);
        if (pald_status st = launch_status(); st != PALD_OK) return st;
    }
    ScopedTiming tm(timing, 7, s);
    const int64_t ftiles = ceil_div(n, 32) * ceil_div(n, 32);
    triplet_finalize_kernel<<<(unsigned)std::min<int64_t>(ftiles, 65536), 256, 0, s>>>(A, B, n, C, ldc, 1.0 / scale,
                                                                                      ftiles);
    return launch_status();
}

// Both passes of the pairwise or hybrid variant with plan p in the workspace
// at `base` (at least p.bytes, 256-byte aligned); arguments already checked.
pald_status run_cohesion(const float *D, int64_t n, int64_t ldd, int32_t *U, int64_t ldu, float *C, int64_t ldc,
                         char *base, const Plan &p, const Opts &o, hipStream_t s) {
    const bool timing = (o.flags & PALD_FLAG_TIMING) != 0;
    float *W = reinterpret_cast<float *>(base + p.off_w);
    int32_t *Ub = U;
    int64_t ldub = ldu;
    if (!Ub && p.need_u_scratch) {
        Ub = reinterpret_cast<int32_t *>(base + p.off_u);
        ldub = n;
    }
    if (o.variant == PALD_VARIANT_HYBRID) {
        // triplet pass 1 (one visit per unordered triple, integer atomics), then W
        if (pald_status st = triplet_focus(D, n, ldd, Ub, ldub, s, timing); st != PALD_OK) return st;
        ScopedTiming tm(timing, 1, s);
        const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(n, 256), 64);
        weights_kernel<<<dim3(gx, rows_grid(n)), 256, 0, s>>>(Ub, ldub, W, p.ldw, n);
        if (pald_status st = launch_status(); st != PALD_OK) return st;
    } else if (pald_status st = run_pass1(D, n, ldd, Ub, ldub, W, p.ldw, p, s, timing); st != PALD_OK) {
        return st;
    }
    double *part = p.y_chunks > 1 ? reinterpret_cast<double *>(base + p.off_part) : nullptr;
    return run_pass2(D, n, ldd, W, p.ldw, C, ldc, part, p, o.accum == PALD_ACC_F64, s, timing);
}

}  // namespace

// ---- blocks of rows ------------------------------------------------------------
constexpr int64_t ROWS_P1_TILES_PER_LAUNCH = 1 << 20;
static_assert(ROWS_P1_TILES_PER_LAUNCH * P1Z_NT < MAX_X_ITEMS, "launch pieces must hold fewer than 2^32 work-items");

// Row-block options: the pairwise variant, compensated accumulation, no forced splits.
pald_status rows_opts(const Opts &o) {
    if ((o.variant != PALD_VARIANT_AUTO && o.variant != PALD_VARIANT_PAIRWISE) || o.accum != PALD_ACC_COMPENSATED ||
        o.y_chunks != 0 || o.z_chunks != 0)
        return PALD_ERR_UNSUPPORTED;
    return PALD_OK;
}

inline int64_t rows_ldwt(int64_t rows) { return (int64_t)align_up((size_t)rows, 64); }

// Pass 1 of the pairs (x, y), x in [g.xlo, g.xhi), y in [g.ylo, g.yhi): U
// (may be null) and the transposed weights Wt.
pald_status rows_pass1(const P1Rows &g, int64_t n, int32_t *U, int64_t ldu, float *Wt, int64_t ldwt, bool vec,
                       hipStream_t s, bool timing) {
    const int64_t tiles = ceil_div(g.xhi - g.xlo, P1Z_TX) * ceil_div(g.yhi - g.ylo, P1Z_TY);
    for (int64_t t0 = 0; t0 < tiles; t0 += ROWS_P1_TILES_PER_LAUNCH) {
        ScopedTiming tm(timing, 13, s);
        const unsigned gx = (unsigned)std::min<int64_t>(ROWS_P1_TILES_PER_LAUNCH, tiles - t0);
        pass1_rows_kernel<<<gx, P1Z_NT, 0, s>>>(g, n, U, ldu, Wt, ldwt, vec ? 1 : 0, t0);
        if (pald_status st = launch_status(); st != PALD_OK) return st;
    }
    return PALD_OK;
}

// Pass 2 of the rows [g.xlo, g.xhi) over y in [g.ylo, g.yhi): C, or added into acc.
pald_status rows_pass2(const P1Rows &g, int64_t n, const float *Wt, int64_t ldwt, float *C, int64_t ldc, double *acc,
                       int64_t ldacc, bool vec_d, hipStream_t s, bool timing) {
    const int64_t xt = ceil_div(g.xhi - g.xlo, P2R_T), zt = ceil_div(n, P2R_T);
    if (xt > 65535 || zt > INT32_MAX) return PALD_ERR_UNSUPPORTED;
    ScopedTiming tm(timing, 14, s);
    pass2_rows_kernel<<<dim3((unsigned)zt, (unsigned)xt), P2R_NT, 0, s>>>(g, n, Wt, ldwt, C, ldc, acc, ldacc, g.ylo,
                                                                            g.yhi, vec_d ? 1 : 0, 1);
    return launch_status();
}

// Device workspace of the out-of-core mode for panels of P rows: the panel's
// rows of D, one block of P rows of D, the transposed weights (n x ldwt), the
// panel's U, its float64 accumulators and its C.
struct OocLayout {
    int64_t P = 0, ldp = 0, ldwt = 0;
    size_t off_dp = 0, off_db = 0, off_wt = 0, off_u = 0, off_acc = 0, off_c = 0, bytes = 0;
};

OocLayout ooc_layout(int64_t n, int64_t P) {
    OocLayout L;
    L.P = P;
    L.ldp = (int64_t)align_up((size_t)n, 64);
    L.ldwt = rows_ldwt(P);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, ALIGN);
        return at;
    };
    L.off_dp = take((size_t)P * L.ldp * sizeof(float));
    L.off_db = take((size_t)P * L.ldp * sizeof(float));
    L.off_wt = take((size_t)n * L.ldwt * sizeof(float));
    L.off_u = take((size_t)P * n * sizeof(int32_t));
    L.off_acc = take((size_t)P * n * sizeof(double));
    L.off_c = take((size_t)P * n * sizeof(float));
    L.bytes = off;
    return L;
}

// ---- fixed workspace of pald_cohesion_noalloc// ---- fixed workspace of pald_cohesion_noalloc -------------------------------
// One array per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the symbol):
// noalloc_scratch() looks up its device address once per device and every use
// goes through that address.
static __device__ __align__(256) unsigned char scratch[PALD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

// Device address of `scratch` on the current device (looked up on the first
// call made on that device).
pald_status noalloc_scratch(char **out) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PALD_ERR_DEVICE;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PALD_ERR_DEVICE;
        addr[dev] = ptr;
    }
    *out = static_cast<char *>(addr[dev]);
    return PALD_OK;
}

}  // namespace

// ============================================================================
extern "C" {

const char *pald_status_string(int32_t s) {
    switch (s) {
    case PALD_OK: return "ok";
    case PALD_ERR_ARG: return "invalid argument";
    case PALD_ERR_INPUT: return "invalid input data";
    case PALD_ERR_DEVICE: return "device or launch error";
    case PALD_ERR_NOMEM: return "out of memory";
    case PALD_ERR_UNSUPPORTED: return "unsupported option";
    default: return "unknown status";
    }
}

int32_t pald_version(void) { return 10000 * 0 + 100 * 1 + 0; }

size_t pald_workspace_bytes(int64_t n, const pald_options *opt) {
    Opts o;
    if (n < 2 || read_opts(opt, o) != PALD_OK) return 0;
    resolve_variant(n, o);
    if (o.variant == PALD_VARIANT_TRIPLET || o.variant == PALD_VARIANT_HYBRID2) return triplet_workspace_bytes(n);
    Plan p;
    if (make_plan(n, o, p) != PALD_OK) return 0;
    return p.bytes;
}

int32_t pald_resolved_variant(int64_t n, const pald_options *opt) {
    Opts o;
    if (read_opts(opt, o) != PALD_OK) return -1;
    resolve_variant(n, o);
    return o.variant;
}

pald_status pald_focus_sizes(const float *D, int64_t n, int64_t ldd, int32_t *U, int64_t ldu, void *stream,
                             const pald_options *opt) {
    Opts o;
    if (pald_status st = read_opts(opt, o); st != PALD_OK) return st;
    if (!D || !U || n < 2 || ldd < n || ldu < n) return PALD_ERR_ARG;
    resolve_variant(n, o);
    if (o.variant == PALD_VARIANT_TRIPLET || o.variant == PALD_VARIANT_HYBRID)
        return triplet_focus(D, n, ldd, U, ldu, (hipStream_t)stream, (o.flags & PALD_FLAG_TIMING) != 0);
    Plan p;
    if (pald_status st = make_plan(n, o, p); st != PALD_OK) return st;
    return run_pass1(D, n, ldd, U, ldu, nullptr, p.ldw, p, (hipStream_t)stream, (o.flags & PALD_FLAG_TIMING) != 0);
}

pald_status pald_cohesion(const float *D, int64_t n, int64_t ldd, int32_t *U, int64_t ldu, float *C, int64_t ldc,
                          void *ws, size_t ws_bytes, void *stream, const pald_options *opt) {
    Opts o;
    if (pald_status st = read_opts(opt, o); st != PALD_OK) return st;
    if (!D || !C || !ws || n < 2 || ldd < n || ldc < n || (U && ldu < n)) return PALD_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & (ALIGN - 1)) != 0) return PALD_ERR_ARG;
    resolve_variant(n, o);
    hipStream_t s = (hipStream_t)stream;
    if (o.variant == PALD_VARIANT_TRIPLET || o.variant == PALD_VARIANT_HYBRID2) {
        if (o.accum != PALD_ACC_COMPENSATED || o.y_chunks != 0) return PALD_ERR_UNSUPPORTED;
        if (o.variant == PALD_VARIANT_TRIPLET && o.z_chunks != 0) return PALD_ERR_UNSUPPORTED;
        return triplet_cohesion(D, n, ldd, U, U ? ldu : 0, C, ldc, ws, ws_bytes, s, o);
    }
    if (o.variant == PALD_VARIANT_HYBRID && o.z_chunks != 0) return PALD_ERR_UNSUPPORTED;
    Plan p;
    if (pald_status st = make_plan(n, o, p); st != PALD_OK) return st;
    if (ws_bytes < p.bytes) return PALD_ERR_ARG;
    return run_cohesion(D, n, ldd, U, ldu, C, ldc, static_cast<char *>(ws), p, o, s);
}

pald_status pald_cohesion_noalloc(const float *D, int64_t n, int64_t ldd, int32_t *U, int64_t ldu, float *C,
                                  int64_t ldc, void *stream, const pald_options *opt) {
    Opts o;
    if (pald_status st = read_opts(opt, o); st != PALD_OK) return st;
    if (!D || !C || n < 2 || ldd < n || ldc < n || (U && ldu < n)) return PALD_ERR_ARG;
    if (o.variant != PALD_VARIANT_AUTO && o.variant != PALD_VARIANT_PAIRWISE) return PALD_ERR_UNSUPPORTED;
    o.variant = PALD_VARIANT_PAIRWISE;  // AUTO runs pairwise here
    Plan p;
    if (pald_status st = make_plan(n, o, p); st != PALD_OK) return st;
    // an automatic y split is lowered until its partial sums fit
    for (int32_t yc = p.y_chunks - 1; p.bytes > PALD_NOALLOC_SCRATCH_BYTES && o.y_chunks == 0 && yc >= 1; --yc) {
        Opts oy = o;
        oy.y_chunks = yc;
        if (pald_status st = make_plan(n, oy, p); st != PALD_OK) return st;
    }
    if (p.bytes > PALD_NOALLOC_SCRATCH_BYTES) return PALD_ERR_ARG;
    char *base = nullptr;
    if (pald_status st = noalloc_scratch(&base); st != PALD_OK) return st;
    return run_cohesion(D, n, ldd, U, ldu, C, ldc, base, p, o, (hipStream_t)stream);
}

size_t pald_rows_workspace_bytes(int64_t n, int64_t rows, const pald_options *opt) {
    Opts o;
    if (n < 2 || rows < 1 || rows > n || read_opts(opt, o) != PALD_OK || rows_opts(o) != PALD_OK) return 0;
    return std::max<size_t>(align_up((size_t)n * rows_ldwt(rows) * sizeof(float), ALIGN), ALIGN);
}

pald_status pald_cohesion_rows(const float *D, int64_t n, int64_t ldd, int64_t x0, int64_t x1, int32_t *U, int64_t ldu,
                               float *C, int64_t ldc, void *ws, size_t ws_bytes, void *stream, const pald_options *opt) {
    Opts o;
    if (pald_status st = read_opts(opt, o); st != PALD_OK) return st;
    if (pald_status st = rows_opts(o); st != PALD_OK) return st;
    if (!D || !C || !ws || n < 2 || ldd < n || ldc < n || (U && ldu < n) || x0 < 0 || x1 <= x0 || x1 > n)
        return PALD_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & (ALIGN - 1)) != 0 || ws_bytes < pald_rows_workspace_bytes(n, x1 - x0, opt))
        return PALD_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    const bool timing = (o.flags & PALD_FLAG_TIMING) != 0;
    float *Wt = static_cast<float *>(ws);
    const int64_t ldwt = rows_ldwt(x1 - x0);
    const bool vec = aligned16(D) && ldd % 4 == 0;
    const P1Rows g{D + x0 * ldd, ldd, x0, x1, D, ldd, 0, n};
    if (pald_status st = rows_pass1(g, n, U, ldu, Wt, ldwt, vec, s, timing); st != PALD_OK) return st;
    return rows_pass2(g, n, Wt, ldwt, C, ldc, nullptr, 0, vec && x0 % 4 == 0, s, timing);
}

size_t pald_ooc_workspace_bytes(int64_t n, int64_t panel_rows) {
    if (n < 2 || panel_rows < 1) return 0;
    return ooc_layout(n, std::min(panel_rows, n)).bytes;
}

pald_status pald_cohesion_ooc(const float *D_host, int64_t n, int64_t ldd, int32_t *U_host, int64_t ldu, float *C_host,
                              int64_t ldc, void *ws, size_t ws_bytes, void *stream, const pald_options *opt) {
    Opts o;
    if (pald_status st = read_opts(opt, o); st != PALD_OK) return st;
    if (pald_status st = rows_opts(o); st != PALD_OK) return st;
    if (!D_host || !C_host || !ws || n < 2 || ldd < n || ldc < n || (U_host && ldu < n)) return PALD_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & (ALIGN - 1)) != 0) return PALD_ERR_ARG;
    // the tallest panel (a multiple of 16 rows, at most n) whose layout fits
    int64_t P = 0;
    for (int64_t lo = 1, hi = ceil_div(n, 16); lo <= hi;) {
        const int64_t mid = (lo + hi) / 2;
        if (ooc_layout(n, std::min(16 * mid, n)).bytes <= ws_bytes) {
            P = std::min(16 * mid, n);
            lo = mid + 1;
        } else {
            hi = mid - 1;
        }
    }
    if (P == 0) return PALD_ERR_ARG;
    const OocLayout L = ooc_layout(n, P);
    char *base = static_cast<char *>(ws);
    float *Dp = reinterpret_cast<float *>(base + L.off_dp), *Db = reinterpret_cast<float *>(base + L.off_db);
    float *Wt = reinterpret_cast<float *>(base + L.off_wt), *Cp = reinterpret_cast<float *>(base + L.off_c);
    int32_t *Up = reinterpret_cast<int32_t *>(base + L.off_u);
    double *acc = reinterpret_cast<double *>(base + L.off_acc);
    hipStream_t s = (hipStream_t)stream;
    const bool timing = (o.flags & PALD_FLAG_TIMING) != 0;
    const size_t row_bytes = (size_t)n * sizeof(float), ldp_bytes = (size_t)L.ldp * sizeof(float);
    auto rows_to_device = [&](float *dst, int64_t r0, int64_t r1) {
        ScopedTiming tm(timing, 15, s);
        return hipMemcpy2DAsync(dst, ldp_bytes, D_host + r0 * ldd, (size_t)ldd * sizeof(float), row_bytes,
                                (size_t)(r1 - r0), hipMemcpyHostToDevice, s) == hipSuccess;
    };
    for (int64_t x0 = 0; x0 < n; x0 += P) {
        const int64_t x1 = std::min(n, x0 + P), rows = x1 - x0;
        if (!rows_to_device(Dp, x0, x1)) return PALD_ERR_DEVICE;
        // pass 1, one block of y rows at a time
        for (int64_t y0 = 0; y0 < n; y0 += P) {
            const int64_t y1 = std::min(n, y0 + P);
            if (!rows_to_device(Db, y0, y1)) return PALD_ERR_DEVICE;
            const P1Rows g{Dp, L.ldp, x0, x1, Db, L.ldp, y0, y1};
            if (pald_status st = rows_pass1(g, n, Up, n, Wt, L.ldwt, true, s, timing); st != PALD_OK) return st;
        }
        // pass 2 into float64 accumulators, then C
        const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(n, 256), 64);
        zero_f64_kernel<<<dim3(gx, rows_grid(rows)), 256, 0, s>>>(acc, n, rows, n);
        if (pald_status st = launch_status(); st != PALD_OK) return st;
        for (int64_t y0 = 0; y0 < n; y0 += P) {
            const int64_t y1 = std::min(n, y0 + P);
            if (!rows_to_device(Db, y0, y1)) return PALD_ERR_DEVICE;
            const P1Rows g{Dp, L.ldp, x0, x1, Db, L.ldp, y0, y1};
            if (pald_status st = rows_pass2(g, n, Wt, L.ldwt, nullptr, 0, acc, n, true, s, timing); st != PALD_OK)
                return st;
        }
        {
            ScopedTiming tm(timing, 14, s);
            rows_finalize_kernel<<<dim3(gx, rows_grid(rows)), 256, 0, s>>>(acc, n, rows, n, Cp, n);
            if (pald_status st = launch_status(); st != PALD_OK) return st;
        }
        ScopedTiming tm(timing, 15, s);
        if (hipMemcpy2DAsync(C_host + x0 * ldc, (size_t)ldc * sizeof(float), Cp, row_bytes, row_bytes, (size_t)rows,
                             hipMemcpyDeviceToHost, s) != hipSuccess)
            return PALD_ERR_DEVICE;
        if (U_host && hipMemcpy2DAsync(U_host + x0 * ldu, (size_t)ldu * sizeof(int32_t), Up, (size_t)n * sizeof(int32_t),
                                       (size_t)n * sizeof(int32_t), (size_t)rows, hipMemcpyDeviceToHost,
                                       s) != hipSuccess)
            return PALD_ERR_DEVICE;
    }
    return hipStreamSynchronize(s) == hipSuccess ? PALD_OK : PALD_ERR_DEVICE;
}

pald_status pald_check_input(const float *D, int64_t n, int64_t ldd, void *ws, size_t ws_bytes, void *stream,
                             uint32_t *flags_out) {
    if (!D || !ws || n < 2 || ldd < n || ws_bytes < 256) return PALD_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    uint32_t *flag = static_cast<uint32_t *>(ws);
    zero_i32_kernel<<<dim3(1, 1), 64, 0, s>>>(reinterpret_cast<int32_t *>(flag), 1, 1);
    if (launch_status() != PALD_OK) return PALD_ERR_DEVICE;
    const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(n, 256), 64);
    check_input_kernel<<<dim3(gx, rows_grid(n)), 256, 0, s>>>(D, n, ldd, flag);
    if (launch_status() != PALD_OK) return PALD_ERR_DEVICE;
    uint32_t h = 0;
    if (hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return PALD_ERR_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return PALD_ERR_DEVICE;
    if (flags_out) *flags_out = h;
    return h ? PALD_ERR_INPUT : PALD_OK;
}

int32_t pald_timings_collect(double *total_ms, int64_t *count, int32_t kinds) {
    std::vector<TimingRec> recs;
    {
        std::lock_guard<std::mutex> g(timing_mutex());
        recs.swap(timing_records());
    }
    for (int32_t k = 0; k < kinds && k < NUM_KINDS; ++k) {
        if (total_ms) total_ms[k] = 0.0;
        if (count) count[k] = 0;
    }
    for (auto &r : recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess &&
            r.kind < kinds) {
            if (total_ms) total_ms[r.kind] += ms;
            if (count) count[r.kind] += 1;
        }
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    return NUM_KINDS;
}

}  // extern "C"

// ============================================================================
// batched mode

namespace {

// Built-in configuration: the autotuner's table for MI355X (tuned_gfx950.h).
constexpr const pald_batch_bucket *kDefaultBuckets = pald_tuned::kBatchBuckets;
constexpr int kDefaultNumBuckets = (int)(sizeof(pald_tuned::kBatchBuckets) / sizeof(pald_tuned::kBatchBuckets[0]));
static_assert(kDefaultNumBuckets >= 1 && kDefaultNumBuckets <= PALD_BATCH_MAX_BUCKETS, "tuned bucket table size");
constexpr int kDefaultLag = pald_tuned::kBatchQueueLag > 0 ? pald_tuned::kBatchQueueLag : 2;

// Launch form: the caller's flag if it sets one, else the tuned choice.
bool batch_split(const pald_batch_config *cfg) {
    if (cfg && (cfg->flags & PALD_BATCH_SPLIT_PASS1)) return true;
    if (cfg && (cfg->flags & PALD_BATCH_ONE_LAUNCH)) return false;
    return pald_tuned::kBatchSplitPass1;
}

struct BatchLayout {
    std::vector<BatchMatrix> mats;
    std::vector<int4> items;
    std::vector<int4> tiles1z;  // PALD_BATCH_SPLIT_PASS1: {matrix, X0, Y0, 0} of every pass-1 tile
    std::vector<int64_t> n, off;
    int64_t total_elems = 0;
    int64_t w_floats = 0;     // weight region size (floats)
    int64_t p_doubles = 0;    // partial-tile region size (doubles)
    int64_t nctr = 0;         // uint32 counters
};

pald_status check_config(const pald_batch_config *cfg) {
    if (!cfg) return PALD_OK;
    if (cfg->nbuckets < 0 || cfg->nbuckets > PALD_BATCH_MAX_BUCKETS || cfg->workgroups_per_cu < 0 ||
        cfg->queue_lag < 0 || (cfg->flags & ~(PALD_BATCH_TIMESTAMPS | PALD_BATCH_SPLIT_PASS1 | PALD_BATCH_ONE_LAUNCH)) ||
        ((cfg->flags & PALD_BATCH_SPLIT_PASS1) && (cfg->flags & PALD_BATCH_ONE_LAUNCH)))
        return PALD_ERR_ARG;
    for (int b = 0; b < cfg->nbuckets; ++b) {
        const pald_batch_bucket &k = cfg->bucket[b];
        if ((k.tile != 0 && k.tile != BATCH_P2_T && k.tile != BATCH_P2S_T) || k.y_chunks < 1 || k.n_max < 2 ||
            k.reserved != 0)
            return PALD_ERR_ARG;
        if (b > 0 && k.n_max <= cfg->bucket[b - 1].n_max) return PALD_ERR_ARG;
    }
    return PALD_OK;
}

const pald_batch_bucket &bucket_for(const pald_batch_config *cfg, int64_t n) {
    const pald_batch_bucket *tab = kDefaultBuckets;
    int nb = kDefaultNumBuckets;
    if (cfg && cfg->nbuckets > 0) {
        tab = cfg->bucket;
        nb = cfg->nbuckets;
    }
    for (int b = 0; b < nb; ++b)
        if (n <= tab[b].n_max) return tab[b];
    return tab[nb - 1];
}

// Per-matrix table, item queue and workspace sizes for a batch.
pald_status build_batch(int32_t count, const int64_t *n_host, const pald_batch_config *cfg, int32_t grid,
                        BatchLayout &L) {
    if (count < 1 || !n_host || grid < 1) return PALD_ERR_ARG;
    if (pald_status st = check_config(cfg); st != PALD_OK) return st;
    L = BatchLayout{};
    const bool split = batch_split(cfg);
    L.mats.resize(count);
    L.n.assign(n_host, n_host + count);
    L.off.resize(count);
    int64_t off = 0, woff = 0, poff = 0, ctr2 = 0;
    for (int32_t i = 0; i < count; ++i) {
        const int64_t n = n_host[i];
        if (n < 2 || n > (1 << 20)) return PALD_ERR_ARG;
        const pald_batch_bucket &bk = bucket_for(cfg, n);
        BatchMatrix &m = L.mats[i];
        m.off = off;
        L.off[i] = off;
        m.n = (int32_t)n;
        m.ldw = (int32_t)align_up((size_t)n, 4);
        m.woff = woff;
        const int64_t nb1 = ceil_div(n, BATCH_P1_T);
        m.tiles1 = split ? 0 : (int32_t)(nb1 * (nb1 + 1) / 2);
        const int64_t T2 = bk.tile ? bk.tile : BATCH_P2_T;
        m.tile2 = (int32_t)T2;
        const int64_t nb2 = ceil_div(n, T2);
        const int64_t tiles2 = nb2 * (nb2 + 1) / 2;
        int64_t yc = std::max<int64_t>(1, std::min<int64_t>(bk.y_chunks, ceil_div(n, BATCH_P2_KY)));
        m.y_per_chunk = (int32_t)(ceil_div(ceil_div(n, yc), BATCH_P2_KY) * BATCH_P2_KY);
        m.y_chunks = (int32_t)ceil_div(n, m.y_per_chunk);
        m.poff = poff;
        m.ctr2 = (int32_t)ctr2;
        if (m.y_chunks > 1) {
            poff += tiles2 * m.y_chunks * 2 * T2 * T2;
            ctr2 += tiles2;
        }
        m.vec_d = (off % 4 == 0 && n % 4 == 0) ? 1 : 0;
        off += n * n;
        woff += (int64_t)align_up((size_t)(n * m.ldw), 64);  // 256-byte aligned per matrix
    }
    L.total_elems = off;
    L.w_floats = woff;
    L.p_doubles = poff;
    L.nctr = 1 + (int64_t)count + ctr2;

    // matrices largest first
    std::vector<int32_t> order(count);
    for (int32_t i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return n_host[a] > n_host[b]; });
    const int64_t lag = (int64_t)((cfg && cfg->queue_lag > 0) ? cfg->queue_lag : kDefaultLag) * grid;

    auto emit_p2 = [&](int32_t i) {
        const BatchMatrix &m = L.mats[i];
        const int64_t nb2 = ceil_div(m.n, m.tile2);
        const int64_t tiles2 = nb2 * (nb2 + 1) / 2;
        for (int64_t t = 0; t < tiles2; ++t)
            for (int32_t c = 0; c < m.y_chunks; ++c) L.items.push_back(make_int4(i, ITEM_PASS2, (int)t, c));
    };
    if (split) {
        // pass-1 tiles of the first launch, largest matrix first; inside a
        // matrix the 16 x 16 tiles x <= y by groups of G x G (as grouped_tile)
        constexpr int64_t G = TILE_GROUP, TX = BatchFocusCfg::TX, TY = BatchFocusCfg::TY, S = TY / TX;
        static_assert(S * TX == TY, "a TY x TY square splits into whole tiles along x");
        for (int32_t i : order) {
            const int64_t n = L.n[i], nb = ceil_div(n, TY), nsb = ceil_div(nb, G);
            for (int64_t gy = 0; gy < nsb; ++gy)
                for (int64_t gx = 0; gx <= gy; ++gx)
                    for (int64_t by = gy * G; by < std::min(nb, gy * G + G); ++by)
                        for (int64_t bx = gx * G; bx < std::min(nb, gx * G + G) && bx <= by; ++bx)
                            for (int64_t sx = 0; sx < S && (S * bx + sx) * TX < n; ++sx)
                                L.tiles1z.push_back(make_int4(i, (int)((S * bx + sx) * TX), (int)(by * TY), 0));
            if (L.tiles1z.size() > (size_t)INT32_MAX) return PALD_ERR_UNSUPPORTED;
        }
        for (int32_t i : order) emit_p2(i);
        if (L.items.size() > (size_t)INT32_MAX) return PALD_ERR_UNSUPPORTED;
        return PALD_OK;
    }
    std::vector<std::pair<int32_t, int64_t>> pending;  // (matrix, queue position after its last pass-1 item)
    size_t head = 0;
    int64_t p1_emitted = 0;
    for (int32_t i : order) {
        for (int32_t t = 0; t < L.mats[i].tiles1; ++t) L.items.push_back(make_int4(i, ITEM_PASS1, t, 0));
        p1_emitted += L.mats[i].tiles1;
        pending.push_back({i, p1_emitted});
        while (head < pending.size() && p1_emitted - pending[head].second >= lag) emit_p2(pending[head++].first);
    }
    while (head < pending.size()) emit_p2(pending[head++].first);
    if (L.items.size() > (size_t)INT32_MAX) return PALD_ERR_UNSUPPORTED;
    return PALD_OK;
}

int32_t device_cus(int dev) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    return cus;
}

int32_t resident_per_cu() {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batched_cohesion_kernel<true, true>, BATCH_THREADS, 0) !=
            hipSuccess ||
        per < 1)
        per = 1;
    return per;
}

int32_t lean_resident_per_cu(bool one_launch) {
    int per = 0;
    const hipError_t e = one_launch
                             ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batched_lean_kernel, BATCH_LEAN_THREADS, 0)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batched_pass2_lean_kernel,
                                                                            BATCH_LEAN_THREADS, 0);
    if (e != hipSuccess || per < 1) per = 1;
    return per;
}

// Every matrix of the layout runs 64-wide pass-2 tiles without a y split.
bool lean_layout(const BatchLayout &L) {
    for (const BatchMatrix &m : L.mats)
        if (m.y_chunks != 1 || m.tile2 != BATCH_P2_T) return false;
    return true;
}

}  // namespace

struct pald_batch_plan {
    int32_t count = 0;
    int device = 0;
    uint32_t flags = 0;
    int32_t grid = 0;
    BatchLayout L;
    BatchMatrix *d_mats = nullptr;
    int4 *d_items = nullptr;
    int4 *d_tiles1z = nullptr;
    bool lean2 = false;  // split mode, every matrix 64-wide pass-2 tiles, no y split
    bool lean1 = false;  // the same in the one-launch form
    size_t off_w = 0, off_p = 0, off_ctr = 0, off_stamps = 0, ws_bytes = 0;
};

struct pald_batch_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int64_t kMaxGrid1 = (int64_t)1 << 22;  // pass-1 tiles per launch of the split mode
static_assert(kMaxGrid1 * BatchFocusCfg::NT < MAX_X_ITEMS, "launch pieces must hold fewer than 2^32 work-items");

pald_status enqueue_batch(const pald_batch_plan *plan, const float *D, int32_t *U, float *C, void *ws,
                          hipStream_t s) {
    char *base = static_cast<char *>(ws);
    float *Wr = reinterpret_cast<float *>(base + plan->off_w);
    double *Pr = reinterpret_cast<double *>(base + plan->off_p);
    uint32_t *ctr = reinterpret_cast<uint32_t *>(base + plan->off_ctr);
    uint64_t *stamps =
        (plan->flags & PALD_BATCH_TIMESTAMPS) ? reinterpret_cast<uint64_t *>(base + plan->off_stamps) : nullptr;
    const int64_t nreset = std::max<int64_t>(plan->L.nctr, plan->count);
    const unsigned rg = (unsigned)std::min<int64_t>(ceil_div(nreset, 256), 1024);
    batch_reset_kernel<<<rg, 256, 0, s>>>(ctr, plan->L.nctr, stamps, plan->count);
    if (pald_status st = launch_status(); st != PALD_OK) return st;
    const int64_t ntiles1 = (int64_t)plan->L.tiles1z.size();
        for (int64_t t0 = 0; t0 < ntiles1; t0 += kMaxGrid1) {
            const int64_t nt = std::min<int64_t>(kMaxGrid1, ntiles1 - t0);
            batched_focus_kernel<<<(unsigned)nt, BatchFocusCfg::NT, 0, s>>>(
                plan->d_tiles1z, plan->d_mats, D, U, Wr, stamps, aligned16(D) ? 1 : 0, (int32_t)t0);
            if (pald_status st = launch_status(); st != PALD_OK) return st;
        }
    if (plan->lean2) {
        batched_pass2_lean_kernel<<<(unsigned)plan->grid, BATCH_LEAN_THREADS, 0, s>>>(
            plan->d_items, (int32_t)plan->L.items.size(), plan->d_mats, D, C, Wr, ctr, stamps, aligned16(D) ? 1 : 0);
        return launch_status();
    }
    if (plan->lean1) {
        batched_lean_kernel<<<(unsigned)plan->grid, BATCH_LEAN_THREADS, 0, s>>>(
            plan->d_items, (int32_t)plan->L.items.size(), plan->d_mats, D, U, C, Wr, ctr, stamps,
            aligned16(D) ? 1 : 0);
        return launch_status();
    }
    auto kern = plan->L.tiles1z.empty() ? batched_cohesion_kernel<true, true>
                                        : batched_cohesion_kernel<false, (bool)PALD_BATCH_SPLIT_FEW_SGPR>;
    kern<<<(unsigned)plan->grid, BATCH_THREADS, 0, s>>>(
        plan->d_items, (int32_t)plan->L.items.size(), plan->d_mats, D, U, C, Wr, Pr, ctr, plan->count, stamps,
        aligned16(D) ? 1 : 0);
    return launch_status();
}

}  // namespace

extern "C" {

pald_status pald_batch_plan_create(int32_t count, const int64_t *n_host, const pald_batch_config *cfg,
                                   pald_batch_plan **plan_out) {
    if (!plan_out) return PALD_ERR_ARG;
    *plan_out = nullptr;
    if (count < 1 || !n_host) return PALD_ERR_ARG;
    if (pald_status st = check_config(cfg); st != PALD_OK) return st;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PALD_ERR_DEVICE;
    const int32_t cus = device_cus(dev);
    const int32_t per_cu = (cfg && cfg->workgroups_per_cu > 0)         ? cfg->workgroups_per_cu
                           : pald_tuned::kBatchWorkgroupsPerCu > 0 ? pald_tuned::kBatchWorkgroupsPerCu
                                                                   : resident_per_cu();
    const int32_t grid = cus * per_cu;
    pald_batch_plan *p = new (std::nothrow) pald_batch_plan();
    if (!p) return PALD_ERR_NOMEM;
    p->count = count;
    p->device = dev;
    p->flags = cfg ? cfg->flags : 0u;
    p->grid = grid;
    if (pald_status st = build_batch(count, n_host, cfg, grid, p->L); st != PALD_OK) {
        delete p;
        return st;
    }
    p->lean2 = PALD_BATCH_LEAN_PASS2 && !p->L.tiles1z.empty() && lean_layout(p->L);
    p->lean1 = PALD_BATCH_LEAN_ONE_LAUNCH && p->L.tiles1z.empty() && lean_layout(p->L);
    // the lean kernels' own resident capacity (a split-mode queue does not
    // depend on the grid; a one-launch queue does, through the lag)
    if ((p->lean2 || p->lean1) && !(cfg && cfg->workgroups_per_cu > 0) && pald_tuned::kBatchWorkgroupsPerCu <= 0) {
        p->grid = cus * lean_resident_per_cu(p->lean1);
        if (p->lean1 && p->grid != grid) {
            if (pald_status st = build_batch(count, n_host, cfg, p->grid, p->L); st != PALD_OK) {
                delete p;
                return st;
            }
        }
    }
    size_t off = 0;
    p->off_w = off;
    off = align_up(off + (size_t)p->L.w_floats * sizeof(float), ALIGN);
    p->off_p = off;
    off = align_up(off + (size_t)p->L.p_doubles * sizeof(double), ALIGN);
    p->off_ctr = off;
    off = align_up(off + (size_t)p->L.nctr * sizeof(uint32_t), ALIGN);
    p->off_stamps = off;
    if (p->flags & PALD_BATCH_TIMESTAMPS) off = align_up(off + (size_t)count * 2 * sizeof(uint64_t), ALIGN);
    p->ws_bytes = off;
    const size_t mbytes = p->L.mats.size() * sizeof(BatchMatrix), ibytes = p->L.items.size() * sizeof(int4);
    const size_t tbytes = p->L.tiles1z.size() * sizeof(int4);
    if (hipMalloc((void **)&p->d_mats, mbytes) != hipSuccess || hipMalloc((void **)&p->d_items, ibytes) != hipSuccess ||
        (tbytes && hipMalloc((void **)&p->d_tiles1z, tbytes) != hipSuccess)) {
        pald_batch_plan_destroy(p);
        return PALD_ERR_NOMEM;
    }
    if (hipMemcpy(p->d_mats, p->L.mats.data(), mbytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_items, p->L.items.data(), ibytes, hipMemcpyHostToDevice) != hipSuccess ||
        (tbytes && hipMemcpy(p->d_tiles1z, p->L.tiles1z.data(), tbytes, hipMemcpyHostToDevice) != hipSuccess)) {
        pald_batch_plan_destroy(p);
        return PALD_ERR_DEVICE;
    }
    *plan_out = p;
    return PALD_OK;
}

size_t pald_batch_workspace_bytes(const pald_batch_plan *plan) { return plan ? plan->ws_bytes : 0; }

int64_t pald_batch_total_elements(const pald_batch_plan *plan) { return plan ? plan->L.total_elems : -1; }

int64_t pald_batch_offset(const pald_batch_plan *plan, int32_t i) {
    if (!plan || i < 0 || i >= plan->count) return -1;
    return plan->L.off[i];
}

int32_t pald_batch_grid(const pald_batch_plan *plan) { return plan ? plan->grid : -1; }

pald_status pald_cohesion_batched(const pald_batch_plan *plan, const float *D_packed, int32_t *U_packed,
                                  float *C_packed, void *ws, size_t ws_bytes, void *stream) {
    if (!plan || !D_packed || !C_packed || !ws || ws_bytes < plan->ws_bytes) return PALD_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & (ALIGN - 1)) != 0) return PALD_ERR_ARG;
    return enqueue_batch(plan, D_packed, U_packed, C_packed, ws, (hipStream_t)stream);
}

pald_status pald_batch_timestamps(const pald_batch_plan *plan, const void *ws, void *stream, double *start_us,
                                  double *end_us) {
    if (!plan || !ws || !start_us || !end_us || !(plan->flags & PALD_BATCH_TIMESTAMPS)) return PALD_ERR_ARG;
    std::vector<uint64_t> h((size_t)plan->count * 2);
    hipStream_t s = (hipStream_t)stream;
    const char *base = static_cast<const char *>(ws);
    if (hipMemcpyAsync(h.data(), base + plan->off_stamps, h.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return PALD_ERR_DEVICE;
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, plan->device) != hipSuccess ||
        rate_khz <= 0)
        return PALD_ERR_DEVICE;
    uint64_t t0 = ~0ull;
    for (int32_t i = 0; i < plan->count; ++i) t0 = std::min(t0, h[2 * i]);
    const double us_per_tick = 1000.0 / (double)rate_khz;
    for (int32_t i = 0; i < plan->count; ++i) {
        start_us[i] = (double)(h[2 * i] - t0) * us_per_tick;
        end_us[i] = (double)(h[2 * i + 1] - t0) * us_per_tick;
    }
    return PALD_OK;
}

int64_t pald_batch_queue(int32_t count, const int64_t *n_host, const pald_batch_config *cfg, int32_t grid,
                         int32_t *items_out, int64_t cap, int32_t *tiles1_out) {
    BatchLayout L;
    if (build_batch(count, n_host, cfg, grid, L) != PALD_OK) return -1;
    const int64_t total = (int64_t)L.items.size();
    if (items_out)
        for (int64_t k = 0; k < total && k < cap; ++k) {
            items_out[4 * k + 0] = L.items[k].x;
            items_out[4 * k + 1] = L.items[k].y;
            items_out[4 * k + 2] = L.items[k].z;
            items_out[4 * k + 3] = L.items[k].w;
        }
    if (tiles1_out)
        for (int32_t i = 0; i < count; ++i) tiles1_out[i] = L.mats[i].tiles1;
    return total;
}

void pald_batch_plan_destroy(pald_batch_plan *plan) {
    if (!plan) return;
    if (plan->d_mats) (void)hipFree(plan->d_mats);
    if (plan->d_items) (void)hipFree(plan->d_items);
    if (plan->d_tiles1z) (void)hipFree(plan->d_tiles1z);
    delete plan;
}

pald_status pald_batch_graph_create(const pald_batch_plan *plan, const float *D_packed, int32_t *U_packed,
                                    float *C_packed, void *ws, size_t ws_bytes, pald_batch_graph **graph_out) {
    if (!graph_out) return PALD_ERR_ARG;
    *graph_out = nullptr;
    if (!plan || !D_packed || !C_packed || !ws || ws_bytes < plan->ws_bytes) return PALD_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & (ALIGN - 1)) != 0) return PALD_ERR_ARG;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return PALD_ERR_DEVICE;
    pald_batch_graph *g = new (std::nothrow) pald_batch_graph();
    if (!g) {
        (void)hipStreamDestroy(cs);
        return PALD_ERR_NOMEM;
    }
    pald_status st = PALD_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = PALD_ERR_DEVICE;
    if (st == PALD_OK) {
        const pald_status est = enqueue_batch(plan, D_packed, U_packed, C_packed, ws, cs);
        hipGraph_t graph = nullptr;
        const hipError_t ce = hipStreamEndCapture(cs, &graph);
        if (est != PALD_OK || ce != hipSuccess) {
            st = PALD_ERR_DEVICE;
            if (graph) (void)hipGraphDestroy(graph);
        } else {
            g->graph = graph;
            if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) st = PALD_ERR_DEVICE;
        }
    }
    (void)hipStreamDestroy(cs);
    if (st != PALD_OK) {
        pald_batch_graph_destroy(g);
        return st;
    }
    *graph_out = g;
    return PALD_OK;
}

pald_status pald_batch_graph_launch(pald_batch_graph *graph, void *stream) {
    if (!graph || !graph->exec) return PALD_ERR_ARG;
    return hipGraphLaunch(graph->exec, (hipStream_t)stream) == hipSuccess ? PALD_OK : PALD_ERR_DEVICE;
}

void pald_batch_graph_destroy(pald_batch_graph *graph) {
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

}  // extern "C"
