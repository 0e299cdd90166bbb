// frontend_api.hip -- host side of the C ABI entry points around the two
// passes (include/pald.h): the distance front end, local depths and the
// strong-tie export.  Argument checking and launches only; the arithmetic
// is in distances.hpp and analysis.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "pald.h"
#include "host_common.hpp"
#include "analysis.hpp"
#include "distances.hpp"

namespace {

using namespace pald;
using namespace pald_host;

constexpr int64_t DIST_TILES_PER_LAUNCH = 65536;
constexpr int64_t ROWS_GRID_MAX = 16384;  // workgroups of the row kernels (grid-strided)

inline unsigned row_blocks(int64_t n) { return (unsigned)std::min<int64_t>(n, ROWS_GRID_MAX); }

template <typename T>
pald_status launch_distances(const T *P, int64_t n, int64_t dim, int64_t ldp, float *D, int64_t ldd,
                             bool euclid, hipStream_t s, bool timing) {
    const int vec = (aligned16(D) && ldd % 4 == 0) ? 1 : 0;
    const int64_t nb = ceil_div(n, DIST_T);
    const int64_t tiles = nb * (nb + 1) / 2;
    if (tiles > INT32_MAX) return PALD_ERR_UNSUPPORTED;
    for (int64_t t0 = 0; t0 < tiles; t0 += DIST_TILES_PER_LAUNCH) {
        ScopedTiming tm(timing, 8, s);
        const unsigned g = (unsigned)std::min<int64_t>(DIST_TILES_PER_LAUNCH, tiles - t0);
        if (euclid)
            distances_kernel<T, true><<<g, DIST_THREADS, 0, s>>>(P, n, dim, ldp, D, ldd, vec, (int32_t)t0);
        else
            distances_kernel<T, false><<<g, DIST_THREADS, 0, s>>>(P, n, dim, ldp, D, ldd, vec, (int32_t)t0);
        if (pald_status st = launch_status(); st != PALD_OK) return st;
    }
    return PALD_OK;
}

inline bool row_vec(const float *C, int64_t ldc) { return aligned16(C) && ldc % 4 == 0; }

constexpr int64_t BFS_MAX_SLOTS = 1024;  // concurrent 64-source searches per launch

inline size_t bfs_slot_bytes(int64_t n) { return (size_t)3 * (size_t)n * sizeof(uint64_t); }

}  // namespace

extern "C" {

pald_status pald_distances(const void *P, int32_t dtype, int64_t n, int64_t dim, int64_t ldp, int32_t metric,
                           float *D, int64_t ldd, void *stream, uint32_t flags) {
    if (!P || !D || n < 1 || dim < 1 || ldp < dim || ldd < n) return PALD_ERR_ARG;
    if ((dtype != PALD_DTYPE_F32 && dtype != PALD_DTYPE_F64) ||
        (metric != PALD_METRIC_EUCLIDEAN && metric != PALD_METRIC_SQEUCLIDEAN) || (flags & ~PALD_FLAG_TIMING))
        return PALD_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const bool euclid = metric == PALD_METRIC_EUCLIDEAN, timing = (flags & PALD_FLAG_TIMING) != 0;
    if (dtype == PALD_DTYPE_F32)
        return launch_distances(static_cast<const float *>(P), n, dim, ldp, D, ldd, euclid, s, timing);
    return launch_distances(static_cast<const double *>(P), n, dim, ldp, D, ldd, euclid, s, timing);
}

pald_status pald_local_depths(const float *C, int64_t n, int64_t ldc, float *depth, void *stream, uint32_t flags) {
    if (!C || !depth || n < 1 || ldc < n) return PALD_ERR_ARG;
    if (flags & ~PALD_FLAG_TIMING) return PALD_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    ScopedTiming tm((flags & PALD_FLAG_TIMING) != 0, 9, s);
    local_depths_kernel<<<row_blocks(n), AN_THREADS, 0, s>>>(C, n, ldc, depth, row_vec(C, ldc) ? 1 : 0);
    return launch_status();
}

pald_status pald_strong_ties(const float *C, int64_t n, int64_t ldc, float threshold, int64_t *row_ptr,
                             int32_t *col, float *val, int64_t cap, void *stream, uint32_t flags) {
    if (!C || !row_ptr || n < 1 || ldc < n || cap < 0 || (cap > 0 && !col) || std::isnan(threshold))
        return PALD_ERR_ARG;
    if (n > INT32_MAX) return PALD_ERR_UNSUPPORTED;
    if (flags & ~PALD_FLAG_TIMING) return PALD_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const bool timing = (flags & PALD_FLAG_TIMING) != 0;
    const int vec = row_vec(C, ldc) ? 1 : 0;
    {
        ScopedTiming tm(timing, 10, s);
        ties_count_kernel<<<row_blocks(n), AN_THREADS, 0, s>>>(C, n, ldc, threshold, row_ptr, vec);
        if (pald_status st = launch_status(); st != PALD_OK) return st;
        ties_scan_kernel<<<1, SCAN_THREADS, 0, s>>>(row_ptr, n);
        if (pald_status st = launch_status(); st != PALD_OK) return st;
    }
    if (cap == 0) return PALD_OK;
    ScopedTiming tm(timing, 11, s);
    ties_fill_kernel<<<row_blocks(n), AN_THREADS, 0, s>>>(C, n, ldc, threshold, row_ptr, col, val, cap);
    return launch_status();
}

size_t pald_graph_distances_workspace_bytes(int64_t n) {
    if (n < 1) return 0;
    const int64_t slots = std::min<int64_t>(ceil_div(n, BFS_SOURCES), BFS_MAX_SLOTS);
    return align_up((size_t)slots * bfs_slot_bytes(n), ALIGN);
}

pald_status pald_graph_distances(const int64_t *row_ptr, const int32_t *col, int64_t nnz, int64_t n, float *D,
                                 int64_t ldd, void *ws, size_t ws_bytes, void *stream, uint32_t flags) {
    if (!row_ptr || !D || !ws || n < 1 || ldd < n || nnz < 0 || (nnz > 0 && !col)) return PALD_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & 7u) != 0 || ws_bytes < bfs_slot_bytes(n)) return PALD_ERR_ARG;
    if (n > INT32_MAX) return PALD_ERR_UNSUPPORTED;
    if (flags & ~PALD_FLAG_TIMING) return PALD_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const int64_t batches = ceil_div(n, BFS_SOURCES);
    const int64_t slots = std::min<int64_t>({batches, BFS_MAX_SLOTS, (int64_t)(ws_bytes / bfs_slot_bytes(n))});
    for (int64_t b0 = 0; b0 < batches; b0 += slots) {
        ScopedTiming tm((flags & PALD_FLAG_TIMING) != 0, 12, s);
        const unsigned g = (unsigned)std::min<int64_t>(slots, batches - b0);
        graph_bfs_kernel<<<g, BFS_THREADS, 0, s>>>(row_ptr, col, nnz, n, D, ldd, static_cast<uint64_t *>(ws), b0);
        if (pald_status st = launch_status(); st != PALD_OK) return st;
    }
    return PALD_OK;
}

}  // extern "C"
