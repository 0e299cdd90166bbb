/*
 * pald.h -- C ABI of libpald, partitioned local depths (PaLD) on AMD Instinct
 * MI355X (gfx950).
 *
 * PaLD (Devarakonda & Ballard, arXiv 2307.16652; the method itself is from
 * Berenhaut et al.) turns an n x n matrix of pairwise distances D into
 *
 *   U  -- local focus sizes (Section 2):
 *           U_xy = #{ z : d_zx <= d_xy  or  d_zy <= d_xy },  int32, symmetric.
 *         The diagonal follows the same formula at y = x, i.e.
 *         U_xx = #{ z : d_zx <= 0 } (1 unless distinct points coincide).
 *   C  -- cohesion (Section 2, Eq. (cohesion); Section 3, Eq. (fxz)):
 *           C_xz = 1/(n-1) * sum_{y != x} [z in U_xy] * s(d_zx, d_zy) / U_xy
 *         with the tie rule s(p, q) = [p < q] + 1/2 [p == q] (Section 5:
 *         support is split on ties), float32, not symmetric.  Row sums of C
 *         are the local depths; the sum of all entries is n/2.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are row-major with a leading dimension (elements between the
 *   starts of consecutive rows) >= n.  D, U, C and workspace pointers are
 *   DEVICE pointers owned by the caller; the library never frees them.
 * - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *   Work is enqueued asynchronously on it and PALD_OK means "enqueued";
 *   results are valid once the stream has been synchronised.
 * - Input contract: every d_ij finite and >= 0, D exactly symmetric, zero
 *   diagonal.  The hot calls do not check the data (use pald_check_input);
 *   on invalid data they produce unspecified values but never access memory
 *   outside the described buffers.  -0.0 is treated as +0.0.
 * - Argument errors (null pointers, n < 2, leading dimension < n, workspace
 *   too small, an unknown option) are reported synchronously with
 *   PALD_ERR_ARG / PALD_ERR_UNSUPPORTED and nothing is enqueued.  A failed
 *   launch reports PALD_ERR_DEVICE.
 * - The hot calls allocate no device memory.  Batch plans own a small device
 *   descriptor allocated at plan creation.  Workspace arguments are device
 *   memory (hipMalloc or a caller's pool); host or fine-grained memory is not
 *   supported there.
 * - Comparisons are made on the float32 input values exactly as given, so U
 *   is exact.  C accumulates float32 half weights 1/(2U) in float32 runs
 *   folded into per-tile Kahan-compensated partials; float64 is used only for
 *   the final cross-tile reduction and the 1/(n-1) scaling.  Relative error
 *   of every C entry <= 16 * 2^-24 (9.5e-7); entries whose exact value is 0
 *   are exactly 0.  Results are deterministic for a fixed configuration,
 *   the triplet variant included (its cross-workgroup sums are exact
 *   64-bit fixed-point integer additions).
 */
#ifndef PALD_H
#define PALD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pald_status {
    PALD_OK = 0,
    PALD_ERR_ARG = 1,         /* bad argument, nothing enqueued */
    PALD_ERR_INPUT = 2,       /* pald_check_input found invalid data */
    PALD_ERR_DEVICE = 3,      /* HIP runtime or launch error */
    PALD_ERR_NOMEM = 4,       /* host allocation or plan descriptor allocation failed */
    PALD_ERR_UNSUPPORTED = 5  /* option combination not implemented */
} pald_status;

/* Algorithm used for the two passes. */
enum {
    PALD_VARIANT_AUTO = 0,     /* the built-in tuned choice for n (autotuner
                                  table compiled into the library: pairwise at
                                  every tuned size on gfx950); pairwise where
                                  the choice does not take the other options */
    PALD_VARIANT_PAIRWISE = 1, /* Section 3 pairwise algorithm: output-stationary
                                  (x,y) tiles for U, (x,z) tiles for C */
    PALD_VARIANT_TRIPLET = 2,  /* Section 3 triplet algorithm: one visit per
                                  unordered triple, shared comparisons */
    PALD_VARIANT_HYBRID = 3,   /* triplet pass 1 + pairwise pass 2, the mix the
                                  appendix's per-pass breakdown suggests; U and
                                  C equal the pairwise variant's bit for bit;
                                  y_chunks applies, z_chunks must be 0 */
    PALD_VARIANT_HYBRID2 = 4   /* pairwise pass 1 + triplet pass 2, the faster
                                  pass of each on this GPU; U equals the pairwise
                                  variant's and C the triplet variant's bit for
                                  bit; z_chunks applies, y_chunks must be 0,
                                  compensated accumulation only */
};

/* Accumulation of the cohesion sums. */
enum {
    PALD_ACC_COMPENSATED = 0, /* float32 runs + Kahan partials, float64 final reduce */
    PALD_ACC_F64 = 1          /* plain float64 accumulator (reference form) */
};

/* Flags. */
#define PALD_FLAG_TIMING 1u /* record device time of every kernel launched by this
                               call; read with pald_timings_collect */

typedef struct pald_options {
    int32_t variant;     /* PALD_VARIANT_* */
    int32_t accum;       /* PALD_ACC_* */
    int32_t y_chunks;    /* pass-2 split of the y range over workgroups; 0 = automatic */
    int32_t z_chunks;    /* pass-1 split of the z range over workgroups; 0 = automatic */
    uint32_t flags;      /* PALD_FLAG_* */
    int32_t reserved[3]; /* must be zero */
} pald_options;

/* Human-readable name of a status code (static string, never NULL). */
const char *pald_status_string(int32_t status);

/* Library version as 10000*major + 100*minor + patch. */
int32_t pald_version(void);

/* Bytes of device workspace pald_cohesion needs for an n x n problem with
 * options `opt` (NULL = defaults).  Returns 0 if n < 2 or opt is invalid. */
size_t pald_workspace_bytes(int64_t n, const pald_options *opt);

/* The variant (PALD_VARIANT_PAIRWISE .. PALD_VARIANT_HYBRID2) that
 * pald_cohesion runs for an n x n problem with options `opt` (NULL =
 * defaults): the given one, or for PALD_VARIANT_AUTO the library's built-in
 * tuned choice for n (the autotuner's per-size table), falling back to the
 * pairwise variant where that choice does not take the other options.
 * Returns -1 if opt is invalid. */
int32_t pald_resolved_variant(int64_t n, const pald_options *opt);

/*
 * Pass 1 only: the local focus sizes U (Section 2 definition, the first loop
 * of the pairwise algorithm in Section 3).  Needs no workspace.
 *   D    [n x ldd]  float32 distances, device, read only
 *   U    [n x ldu]  int32 output, device; every entry of the n x n block written
 * Errors: PALD_ERR_ARG for null D/U, n < 2, ldd < n, ldu < n;
 * PALD_ERR_UNSUPPORTED for an unknown option or nonzero reserved field.
 */
pald_status pald_focus_sizes(const float *D, int64_t n, int64_t ldd,
                             int32_t *U, int64_t ldu,
                             void *stream, const pald_options *opt);

/*
 * Both passes: U (optional) and the cohesion matrix C (Section 3, Eq. (fxz)
 * with ties split as in Section 5 and y ranging over S \ {x}).
 *   D    [n x ldd]  float32 distances, device, read only
 *   U    [n x ldu]  int32 output, device, or NULL to skip writing U (ldu ignored)
 *   C    [n x ldc]  float32 output, device; every entry of the n x n block written
 *   ws   device workspace of at least pald_workspace_bytes(n, opt) bytes; its
 *        contents on entry are ignored and on exit unspecified
 * Errors: PALD_ERR_ARG for null D/C/ws, n < 2, a leading dimension < n, small
 * ws; PALD_ERR_UNSUPPORTED for an unknown variant/accum or nonzero reserved,
 * and for the triplet and second hybrid variants above n = 2^18 (the 64-bit
 * fixed-point sums of their pass 2 are exact up to there).
 */
pald_status pald_cohesion(const float *D, int64_t n, int64_t ldd,
                          int32_t *U, int64_t ldu,
                          float *C, int64_t ldc,
                          void *ws, size_t ws_bytes,
                          void *stream, const pald_options *opt);

/* Bytes of the fixed device workspace behind pald_cohesion_noalloc (64 MiB per
 * GPU, held by the library from the first call on that GPU until the process
 * ends). */
#define PALD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * pald_cohesion without a workspace argument, for callers that cannot allocate
 * device memory: code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc.  It calls no hipMalloc, hipFree or other allocating
 * routine; its workspace is a device array of PALD_NOALLOC_SCRATCH_BYTES
 * inside the library, one per GPU.  (Its pass-1 kernel keeps a few values
 * per lane in the private segment, 16 bytes, which the HIP runtime provides
 * at launch as for any kernel.)
 *   D, U, C, stream, opt  as for pald_cohesion (the caller still owns and
 *                         passes the inputs and outputs)
 * The plan is the one pald_cohesion uses with `opt`, except that an automatic
 * y split (y_chunks = 0) is lowered until its float64 partial sums fit; C
 * then differs from pald_cohesion's in rounding only (same error bound).
 * With default options every n <= 4096 fits.
 * Errors: as pald_cohesion; PALD_ERR_ARG also when the workspace the plan
 * needs exceeds PALD_NOALLOC_SCRATCH_BYTES; PALD_ERR_UNSUPPORTED for the
 * triplet and hybrid variants; PALD_ERR_DEVICE if the array's address cannot
 * be looked up (done once per GPU, on the first call made with it current).
 * Every call on one GPU uses the same array and leaves it holding that call's
 * intermediates: calls that can overlap in time on one GPU (different streams
 * or host threads without ordering between them) race and give wrong results,
 * so the caller must serialise them.
 */
pald_status pald_cohesion_noalloc(const float *D, int64_t n, int64_t ldd,
                                  int32_t *U, int64_t ldu,
                                  float *C, int64_t ldc,
                                  void *stream, const pald_options *opt);

/*
 * Validates D against the input contract.  Synchronous: enqueues a check on
 * `stream`, waits for it and returns PALD_OK or PALD_ERR_INPUT.  If
 * `flags_out` is not NULL it receives a bit set of the problems found:
 * 1 = NaN, 2 = infinity, 4 = negative value, 8 = asymmetric pair,
 * 16 = nonzero diagonal entry.  ws needs >= 256 bytes.
 */
pald_status pald_check_input(const float *D, int64_t n, int64_t ldd,
                             void *ws, size_t ws_bytes, void *stream,
                             uint32_t *flags_out);

/* ---------------------------------------------------------------------------
 * Blocks of rows.  Row x of U and of C depends on all of D but on row x of
 * the focus sizes only (Section 3, Eq. (fxz): c_xz sums over y the terms of
 * the foci of x and y), so the rows split over devices -- or over panels of
 * one device -- with D the only shared input.
 * ------------------------------------------------------------------------- */

/* Workspace bytes pald_cohesion_rows needs for `rows` rows of an n x n
 * problem (the weights of the block, transposed); 0 if n < 2, rows < 1,
 * rows > n or opt is invalid. */
size_t pald_rows_workspace_bytes(int64_t n, int64_t rows, const pald_options *opt);

/*
 * Rows x0 <= x < x1 of U and of C (the same values pald_cohesion gives for
 * these rows: U exactly, C within the same error bound).
 *   D     [n x ldd]  float32 distances, device, read only (every row is read)
 *   U     [(x1-x0) x ldu] int32 output, device, or NULL: row x at U + (x-x0) ldu
 *   C     [(x1-x0) x ldc] float32 output, device: row x at C + (x-x0) ldc
 *   ws    device workspace of at least pald_rows_workspace_bytes(n, x1-x0, opt)
 *         bytes, 256-byte aligned
 * Pass 1 counts the focus sizes of the block's pairs (x, y) for every y; pass 2
 * accumulates only c_xz for x in the block (the whole-matrix pass 2 shares
 * each compare between c_xz and c_zx, which a block of rows cannot), in
 * float32 runs of at most 12 additions folded into Kahan sums, reduced in
 * float64.  Options: variant AUTO or PAIRWISE, compensated accumulation, no
 * forced splits (else PALD_ERR_UNSUPPORTED).
 * Errors: PALD_ERR_ARG for null D/C/ws, n < 2, a leading dimension < n,
 * x0 < 0, x1 <= x0, x1 > n, a small or misaligned ws.
 */
pald_status pald_cohesion_rows(const float *D, int64_t n, int64_t ldd,
                               int64_t x0, int64_t x1,
                               int32_t *U, int64_t ldu,
                               float *C, int64_t ldc,
                               void *ws, size_t ws_bytes,
                               void *stream, const pald_options *opt);

/*
 * Out of core: U and C of a distance matrix that stays in host memory, for
 * n beyond what fits in device memory (D alone is 4 n^2 bytes; the whole-
 * matrix call keeps D, U, C and W resident, 16 n^2 bytes), in panels of rows
 * sized to a device workspace of ws_bytes.  Per panel of P rows the library
 * copies the panel's rows of D to the device, streams D in blocks of P rows
 * twice (pass 1, then pass 2, each block read once per pass), and copies the
 * panel's rows of U and C back.  U equals pald_cohesion's exactly; C is
 * accumulated per block of y (float32 runs and Kahan sums as in
 * pald_cohesion_rows) and summed over the blocks in float64, within the same
 * error bound.  Host traffic: 8 n^2 (n / P) bytes of D plus 8 n^2 of U and C.
 *   D_host  [n x ldd]  float32, host memory (pinned memory copies fastest)
 *   U_host  [n x ldu]  int32 output, host memory, or NULL
 *   C_host  [n x ldc]  float32 output, host memory
 *   ws      device workspace, 256-byte aligned, of at least
 *           pald_ooc_workspace_bytes(n, 16) bytes; the panel height P is the
 *           largest multiple of 16 (at most n) whose pald_ooc_workspace_bytes
 *           fits in ws_bytes
 * Synchronous: returns once the results are in host memory (work runs on
 * `stream`, which is synchronised).  Options as pald_cohesion_rows.
 * Errors: PALD_ERR_ARG for null D_host/C_host/ws, n < 2, a leading dimension
 * < n, a small or misaligned ws; PALD_ERR_DEVICE for a failed copy or launch.
 */
size_t pald_ooc_workspace_bytes(int64_t n, int64_t panel_rows);
pald_status pald_cohesion_ooc(const float *D_host, int64_t n, int64_t ldd,
                              int32_t *U_host, int64_t ldu,
                              float *C_host, int64_t ldc,
                              void *ws, size_t ws_bytes,
                              void *stream, const pald_options *opt);

/* ---------------------------------------------------------------------------
 * Before and after the two passes.
 * ------------------------------------------------------------------------- */

/* Coordinate types and metrics of the distance front end. */
enum { PALD_DTYPE_F32 = 0, PALD_DTYPE_F64 = 1 };
enum { PALD_METRIC_EUCLIDEAN = 0, PALD_METRIC_SQEUCLIDEAN = 1 };

/*
 * Distance front end: the n x n distance matrix of n points in R^dim, the
 * input PaLD takes (Section 6 applies it to Euclidean distances between
 * word-embedding vectors).  Every entry is, in float64 with round-to-nearest,
 *   acc = 0;  for k = 0 .. dim-1 in order: delta = p_xk - p_yk,
 *                                           acc = fma(delta, delta, acc)
 *   D[x][y] = (float)acc               PALD_METRIC_SQEUCLIDEAN
 *   D[x][y] = (float)sqrt(acc)         PALD_METRIC_EUCLIDEAN
 * so D is exactly symmetric with a zero diagonal and meets the input
 * contract whenever the coordinates are finite.
 *   P   [n x ldp]  coordinates, device, float32 or float64 (dtype), read only
 *   D   [n x ldd]  float32 output, device; every entry of the n x n block written
 *   flags          0 or PALD_FLAG_TIMING (kind 8)
 * Errors: PALD_ERR_ARG for null P/D, n < 1, dim < 1, ldp < dim, ldd < n;
 * PALD_ERR_UNSUPPORTED for an unknown dtype, metric or flag.
 */
pald_status pald_distances(const void *P, int32_t dtype, int64_t n, int64_t dim, int64_t ldp,
                           int32_t metric, float *D, int64_t ldd, void *stream, uint32_t flags);

/*
 * Graph front end: all-pairs shortest-path hop counts of an unweighted graph,
 * the distance matrices of the paper's collaboration-network runs (appendix,
 * SNAP datasets).  D[s][v] = number of edges on a shortest s-v path,
 * D[s][s] = 0, and n for pairs in different components (n exceeds every hop
 * count, so PaLD's comparisons treat it exactly like +infinity while D stays
 * finite).  The graph must be undirected for D to be symmetric: store both
 * directions of every edge.
 *   row_ptr [n + 1]  int64 CSR offsets, device: the neighbours of v are
 *                    col[row_ptr[v] .. row_ptr[v+1]); offsets are clamped to
 *                    [0, nnz], so a malformed array cannot cause reads past col
 *   col     [nnz]    int32 neighbour ids, device (NULL if nnz = 0); ids outside
 *                    [0, n) are ignored
 *   D       [n x ldd] float32 output, device; every entry of the n x n block written
 *   ws      device workspace, 8-byte aligned: at least 24 n bytes (one search
 *           batch of 64 sources at a time);
 *           pald_graph_distances_workspace_bytes(n) runs up to 1024 batches
 *           concurrently
 *   flags   0 or PALD_FLAG_TIMING (kind 12)
 * Errors: PALD_ERR_ARG for null row_ptr/D/ws, null col with nnz > 0, n < 1,
 * nnz < 0, ldd < n, a small or misaligned ws; PALD_ERR_UNSUPPORTED for
 * n > 2^31-1 or an unknown flag.
 */
size_t pald_graph_distances_workspace_bytes(int64_t n);
pald_status pald_graph_distances(const int64_t *row_ptr, const int32_t *col, int64_t nnz, int64_t n,
                                 float *D, int64_t ldd, void *ws, size_t ws_bytes, void *stream,
                                 uint32_t flags);

/*
 * Local depths (Section 2: cohesion partitions the local depth of Eq. (LD),
 * l_x = sum_z c_xz): depth[x] = (float)(sum_z C[x][z]), summed in float64 in
 * a fixed order.  With C from pald_cohesion the relative error of each depth
 * is below 1e-6 and the depths sum to n/2.
 *   C      [n x ldc]  float32, device, read only
 *   depth  [n]        float32 output, device
 *   flags             0 or PALD_FLAG_TIMING (kind 9)
 * Errors: PALD_ERR_ARG for null pointers, n < 1, ldc < n;
 * PALD_ERR_UNSUPPORTED for an unknown flag.
 */
pald_status pald_local_depths(const float *C, int64_t n, int64_t ldc, float *depth, void *stream,
                              uint32_t flags);

/*
 * Strong-tie graph (Sections 2 and 6 read community structure off C by a
 * threshold; the threshold itself is the caller's): the directed edges
 * x -> z, z != x, with C[x][z] > threshold (compared in float32), in CSR
 * form with the columns of each row increasing:
 *   row_ptr [n + 1]  int64 output, device: row_ptr[0] = 0, row x's edges are
 *                    positions row_ptr[x] .. row_ptr[x+1]-1; always written
 *   col     [cap]    int32 output, device: the z of each edge
 *   val     [cap]    float32 output, device, or NULL: C[x][z] of each edge
 * Only positions < cap are written; row_ptr[n] is the edge count, so a
 * caller that does not know it calls once with cap = 0 (col may then be
 * NULL), reads row_ptr[n] after synchronising, and calls again.
 * flags: 0 or PALD_FLAG_TIMING (kinds 10 and 11).
 * Errors: PALD_ERR_ARG for null C/row_ptr, null col with cap > 0, n < 1,
 * ldc < n, cap < 0, a NaN threshold; PALD_ERR_UNSUPPORTED for n > 2^31-1 or
 * an unknown flag.
 */
pald_status pald_strong_ties(const float *C, int64_t n, int64_t ldc, float threshold, int64_t *row_ptr,
                             int32_t *col, float *val, int64_t cap, void *stream, uint32_t flags);

/*
 * Batched mode: many independent matrices of different sizes in one
 * persistent launch, or with PALD_BATCH_SPLIT_PASS1 one launch over every
 * matrix's pass-1 tiles followed by the persistent launch (no batching in the
 * paper; a GPU-side extension).
 *
 * Packed layout: matrix i has n_i rows, leading dimension n_i, and starts at
 * element offset off_i = sum_{j<i} n_j^2 of D_packed, U_packed and C_packed.
 *
 * Work queue: every pass-1 tile and every pass-2 tile (times its y-chunks) of
 * every matrix is one item; matrices are taken largest first, and the pass-2
 * items of a matrix are placed `queue_lag` grid-sizes of items after its last
 * pass-1 item.  All pass-1 items of a matrix precede its pass-2 items, which
 * is what makes the in-kernel wait of a pass-2 item always terminate.  In
 * split mode the queue holds the pass-2 items only (largest matrix first) and
 * no item waits.
 */
typedef struct pald_batch_plan pald_batch_plan;

/* Choices for the matrices with n <= n_max (entries sorted by n_max; matrices
 * larger than the last n_max use the last entry). */
typedef struct pald_batch_bucket {
    int32_t n_max;
    int32_t tile;      /* pass-2 tile side: 64 or 32 (0 = 64); pass-1 tiles are 64 */
    int32_t y_chunks;  /* pass-2 split of the y range (1 = no split) */
    int32_t reserved;  /* must be zero */
} pald_batch_bucket;

#define PALD_BATCH_MAX_BUCKETS 8
#define PALD_BATCH_TIMESTAMPS 1u /* record per-matrix first-start / last-end device clocks */
/* Pass 1 of every matrix runs first, as its own launch over all 16 x 16
 * pass-1 tiles of the batch (the single-matrix lanes-over-z tile, 6 waves per
 * SIMD); the persistent queue then holds only pass-2 items, which never wait.
 * Without it, pass-1 items (64 x 64 lanes-over-pairs tiles) share the queue
 * and the persistent kernel's register budget with the pass-2 items. */
#define PALD_BATCH_SPLIT_PASS1 2u
/* The one-launch form: pass-1 and pass-2 items share the persistent queue. */
#define PALD_BATCH_ONE_LAUNCH 4u

/* Built-in configuration: the autotuner's table for MI355X, compiled into the
 * library from its records (buckets, grid, queue lag and launch form; on
 * gfx950 the split form with 64-wide pass-2 tiles and no y split).  A NULL
 * config means all of it; in a config, every field left 0 takes its built-in
 * value, and the launch form is the built-in one unless exactly one of
 * PALD_BATCH_SPLIT_PASS1 / PALD_BATCH_ONE_LAUNCH is set. */
typedef struct pald_batch_config {
    int32_t nbuckets;          /* entries used in bucket[]; 0 = the built-in tuned table */
    int32_t workgroups_per_cu; /* persistent grid = CUs x this; 0 = built-in (resident capacity) */
    int32_t queue_lag;         /* in units of the grid size; 0 = built-in (2) */
    uint32_t flags;            /* PALD_BATCH_* */
    pald_batch_bucket bucket[PALD_BATCH_MAX_BUCKETS];
} pald_batch_config;

/*
 * Builds the plan for `count` matrices of sizes n_host[0..count) (host array,
 * every n_i >= 2) on the current device: chooses tiles and y-splits per size
 * (cfg NULL = the built-in tuned configuration), builds the queue and uploads
 * it and the per-matrix table.  Synchronous; the only allocating call of the
 * batched mode.
 * Errors: PALD_ERR_ARG (count < 1, null pointers, n_i < 2, bad config, both
 * launch-form flags),
 * PALD_ERR_NOMEM, PALD_ERR_DEVICE.
 */
pald_status pald_batch_plan_create(int32_t count, const int64_t *n_host,
                                   const pald_batch_config *cfg,
                                   pald_batch_plan **plan_out);

/* Workspace bytes pald_cohesion_batched needs with this plan (0 for NULL). */
size_t pald_batch_workspace_bytes(const pald_batch_plan *plan);

/* Total packed elements sum n_i^2 (so callers can size D/U/C); -1 for NULL. */
int64_t pald_batch_total_elements(const pald_batch_plan *plan);

/* Element offset of matrix i in the packed arrays, or -1 if i is out of range. */
int64_t pald_batch_offset(const pald_batch_plan *plan, int32_t i);

/* Persistent grid size (workgroups) the plan launches; -1 for NULL. */
int32_t pald_batch_grid(const pald_batch_plan *plan);

/*
 * Runs the whole batch: U_packed (may be NULL) and C_packed from D_packed,
 * all device pointers of pald_batch_total_elements() elements.  Enqueues one
 * counter-reset kernel, with PALD_BATCH_SPLIT_PASS1 the pass-1 launch(es),
 * and one persistent kernel on `stream` (no allocation, no memset node, so
 * the sequence can be captured into a hipGraph).  Calls that
 * share a workspace must not overlap.  C accumulates as in pald_cohesion
 * (float32 runs, Kahan partials, float64 final reduction).
 * Errors: PALD_ERR_ARG for null plan/D/C/ws or a small/misaligned ws.
 */
pald_status pald_cohesion_batched(const pald_batch_plan *plan,
                                  const float *D_packed, int32_t *U_packed,
                                  float *C_packed, void *ws, size_t ws_bytes,
                                  void *stream);

/*
 * Per-matrix device timestamps of the last batched run made with
 * PALD_BATCH_TIMESTAMPS: start_us[i] = first item start and end_us[i] = last
 * item end of matrix i, in microseconds from the earliest start.
 * Synchronous (waits for `stream`).  PALD_ERR_ARG if the plan records none.
 */
pald_status pald_batch_timestamps(const pald_batch_plan *plan, const void *ws,
                                  void *stream, double *start_us, double *end_us);

/*
 * Host only, touches no GPU: writes the queue a plan for these sizes and
 * settings would run with a persistent grid of `grid` workgroups, as 4 int32
 * per item {matrix, kind (0 = pass-1 tile, 1 = pass-2 tile), tile index,
 * y-chunk}, and per matrix its pass-1 item count -- the count its pass-2
 * items wait for; 0 with PALD_BATCH_SPLIT_PASS1 -- to tiles1_out (may be
 * NULL).
 * Returns the number of items (writing at most `cap`), or -1 on bad arguments.
 */
int64_t pald_batch_queue(int32_t count, const int64_t *n_host,
                         const pald_batch_config *cfg, int32_t grid,
                         int32_t *items_out, int64_t cap, int32_t *tiles1_out);

void pald_batch_plan_destroy(pald_batch_plan *plan);

/*
 * hipGraph of one batched run with fixed buffers: captures the reset and the
 * persistent kernel once (on a private stream) and instantiates the graph.
 * Launching it on any stream is equivalent to pald_cohesion_batched with the
 * same arguments.  The plan and buffers must outlive the graph.
 */
typedef struct pald_batch_graph pald_batch_graph;

pald_status pald_batch_graph_create(const pald_batch_plan *plan,
                                    const float *D_packed, int32_t *U_packed,
                                    float *C_packed, void *ws, size_t ws_bytes,
                                    pald_batch_graph **graph_out);
pald_status pald_batch_graph_launch(pald_batch_graph *graph, void *stream);
void pald_batch_graph_destroy(pald_batch_graph *graph);

/*
 * Device timings recorded by calls made with PALD_FLAG_TIMING since the last
 * collect.  Waits for the recorded events, then for kernel kind k writes the
 * summed milliseconds to total_ms[k] and the number of launches to count[k]
 * for k < kinds, and forgets the records.  Kinds: 0 pass-1 focus sizes,
 * 1 weight preparation, 2 pass-2 cohesion, 3 cross-chunk finalize,
 * 4 batched persistent kernel, 5 triplet pass 1, 6 triplet pass 2,
 * 7 triplet finalize, 8 distances, 9 local depths, 10 strong-tie count and
 * scan, 11 strong-tie fill, 12 graph distances, 13 row-block pass 1,
 * 14 row-block pass 2 (with its finalize), 15 host <-> device copies of the
 * out-of-core mode.  Returns the number of kinds defined (16).
 */
int32_t pald_timings_collect(double *total_ms, int64_t *count, int32_t kinds);

#ifdef __cplusplus
}
#endif

#endif /* PALD_H */
