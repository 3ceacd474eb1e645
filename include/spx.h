/*
 * spx.h -- C ABI of the MI355X (gfx950) CSR sparse-matrix library.
 *
 * Problem statement (paper Sec. 1 and Sec. 3): for an m x n sparse matrix A
 * stored in compressed row storage -- rptrs (here `rowptr`, m+1 entries,
 * rowptr[0] = 0, rowptr[m] = tau), cids (here `colind`, tau column ids) and
 * val (here `values`, tau entries) -- compute y <- A x (SpMV) and, for a dense
 * n x k matrix X, Y <- A X (SpMM, Sec. 5).  Indices are 32-bit (Sec. 4).
 *
 * Conventions for every entry point below:
 *  - Pointers are DEVICE pointers unless the parameter name starts with
 *    `host_`.  The caller owns every buffer (including workspaces sized by the
 *    matching *_workspace_bytes call); the library never allocates or frees
 *    device memory on the compute path and never frees caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    are asynchronous and stream ordered, except where a comment says the call
 *    synchronises.
 *  - Errors are returned as spx_status; spx_last_error() returns a text for
 *    the last non-OK status of the calling thread.  Argument checks (sizes,
 *    null pointers, dtype pairs, workspace size) happen before any launch; a
 *    call that returns an error has launched nothing.
 *  - Structural validity of the CSR arrays (monotone rowptr, rowptr[m] = nnz,
 *    0 <= colind < n) is NOT re-checked by the compute calls; use
 *    csr_validate first for untrusted input.  Columns need not be sorted
 *    within a row for SpMV/SpMM; csr_from_coo produces sorted columns.
 *  - Outputs are overwritten (beta = 0).  An empty row gives +0.0.  m == 0 is a
 *    no-op returning SPX_OK.
 *  - Sizes: nonzero positions are int32, and the kernels look up to 2^24
 *    positions past a row's end before comparing, so every call that takes
 *    nnz (or nnz_in) rejects nnz > SPX_MAX_NNZ = 2^31 - 2^25 with
 *    SPX_ERR_UNSUPPORTED, and plans reject split_chunk > SPX_MAX_SPLIT_CHUNK.
 *  - Floating point: FP64 values use FP64 arithmetic throughout.  FP32/BF16
 *    values with FP32 x/y accumulate in FP32; rows longer than the plan's
 *    kahan_len use compensated accumulation and an FP64 cross-lane reduction.
 *    Results are deterministic: the same inputs and plan give the same bits.
 */
#ifndef SPX_H
#define SPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPX_OK = 0,
  SPX_ERR_INVALID = 1,     /* bad size, null pointer, bad option */
  SPX_ERR_UNSUPPORTED = 2, /* dtype pair or layout not implemented */
  SPX_ERR_WORKSPACE = 3,   /* workspace missing or too small */
  SPX_ERR_HIP = 4          /* a HIP runtime call or launch failed */
} spx_status;

#define SPX_MAX_NNZ 2113929216       /* 2^31 - 2^25 */
#define SPX_MAX_SPLIT_CHUNK 16777216 /* 2^24 */

typedef enum {
  SPX_F64 = 0,
  SPX_F32 = 1,
  SPX_BF16 = 2 /* raw IEEE bfloat16 bits in uint16 */
} spx_dtype;

#define SPX_MAX_BINS 12

/* Row-binning plan options (rows grouped by length; the GPU analogue of the
 * paper's dynamic row chunks, Sec. 4.1).  Bin b holds the rows whose length
 * L satisfies upper[b-1] < L <= upper[b]; the last bin takes all longer
 * rows (its upper[] entry is ignored).  lanes[b] is the number of threads that
 * cooperate on one row of bin b: 1, 2, 4, 8, 16, 32, 64 (one wavefront) or
 * 256 (one workgroup); SPX_LANES_STREAM makes a stream bin (SpMV: a
 * workgroup loads the nonzeros of 256 consecutive bin rows as one flat,
 * coalesced sequence and reduces each row from LDS; SpMM treats it as lanes
 * = 1); 0 marks a split bin (allowed only as the last bin): each row is cut
 * into segments of split_chunk nonzeros, one workgroup per segment, and the
 * segment partial sums are reduced in segment order. */
#define SPX_LANES_STREAM 512
#define SPX_FLAG_NO_NT_STORE 1u  /* plain (temporal) stores for y / Y */
#define SPX_FLAG_SCALAR_X 2u     /* SpMM: one element per lane, no vector loads of X */
#define SPX_FLAG_NO_XCD_MAP 4u   /* keep hardware workgroup order (no per-XCD contiguous tiles) */
#define SPX_FLAG_ONE_ROW 8u      /* one row per row group (no multi-row groups for short rows) */
#define SPX_FLAG_KEEP_STREAM 16u /* SpMV: keep a stream bin as 256-row tiles even when it has fewer
                                  * than 2 tiles per compute unit (by default such a bin is served
                                  * by row groups of 8 lanes, which keep more workgroups in flight) */
typedef struct spx_plan_opts {
  int32_t nbins;
  int32_t upper[SPX_MAX_BINS];
  int32_t lanes[SPX_MAX_BINS];
  int32_t split_chunk; /* 256 .. SPX_MAX_SPLIT_CHUNK; nonzeros per segment of a split row */
  int32_t kahan_len;   /* FP32 accumulation: rows with L > kahan_len are compensated */
  int32_t max_k;       /* widest SpMM right-hand side the plan serves (>= 1) */
  uint32_t flags;      /* SPX_FLAG_* */
  int32_t occupancy;   /* 0, or the most workgroups per CU the product launch may hold
                        * (1..8): enforced by padding each workgroup's LDS, for
                        * latency / occupancy sweeps (the GPU analogue of the paper's
                        * threads-per-core scaling, Sec. 4.2).  Rejected with
                        * SPX_ERR_UNSUPPORTED at launch if the device's LDS limits
                        * cannot express it. */
  int32_t row_period;  /* 0, or P > 0: inside each bin, rows are listed by band
                        * floor(8 (r mod P) / P), then ascending.  The product
                        * launch gives XCD j the j-th eighth of every bin's tiles,
                        * so with P the matrix's bandwidth (csr_bandwidth, Sec.
                        * 4.4) each XCD sweeps its own band of every period: on a
                        * grid matrix a slab of the grid, whose X rows then stay in
                        * that XCD's L2 from one period to the next instead of being
                        * fetched again per neighbouring plane (the vector
                        * re-transfers of Sec. 4.4 and Sec. 5).  P >= m gives the
                        * ascending order.  Results are bitwise those of P = 0. */
  int32_t reserved[2];
} spx_plan_opts;

typedef struct spx_plan spx_plan;   /* opaque host object */
typedef struct spx_batch spx_batch; /* opaque host object */

/* Text for the last non-OK status returned on this thread ("" if none). */
const char *spx_last_error(void);

/* Library version string and the device it was compiled for ("gfx950"). */
const char *spx_version(void);

/* Default plan options for SpMV (k = 1) or SpMM with k right-hand sides and
 * values of type vtype.  Never fails for k >= 1. */
spx_status spx_plan_default_opts(int32_t k, spx_dtype vtype, spx_plan_opts *opts);

/* ---------------------------------------------------------------- assembly
 * COO triplets -> canonical CSR (Sec. 3): rows ascending, columns strictly
 * ascending within a row.  Duplicate (i, j) triplets are merged by summing
 * their values in input order (FP64, one add at a time).  r, c: int32[nnz_in];
 * v: f64[nnz_in].  Outputs rowptr int32[m+1], colind int32[nnz_in] and values
 * f64[nnz_in] (capacity nnz_in); *nnz_out (device int32) receives the stored
 * count, or -1 if some triplet is out of range (then the other outputs are
 * unspecified).  Requires nnz_in <= SPX_MAX_NNZ.  Workspace: csr_from_coo_workspace_bytes. */
spx_status csr_from_coo_workspace_bytes(int32_t m, int32_t n, int64_t nnz_in, size_t *bytes);
spx_status csr_from_coo(int32_t m, int32_t n, int64_t nnz_in, const int32_t *r, const int32_t *c,
                        const double *v, int32_t *rowptr, int32_t *colind, double *values,
                        int32_t *nnz_out, void *workspace, size_t ws_bytes, void *stream);

/* Structural check of CSR arrays on the device.  *status_out (device int32)
 * receives 0 if rowptr[0] = 0, rowptr is non-decreasing, rowptr[m] = nnz and
 * 0 <= colind[p] < n for every p; otherwise the code of the most severe
 * problem found: 4 rowptr[0] != 0 or rowptr[m] != nnz, 3 a row whose range is
 * decreasing or outside [0, nnz], 2 a column out of range, 1 an unsorted or
 * repeated column inside a row (checked only when check_sorted != 0). */
spx_status csr_validate(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr,
                        const int32_t *colind, int32_t check_sorted, int32_t *status_out,
                        void *stream);

/* The same assembly on HOST arrays (Sec. 3's CRS arrays built from triplets
 * held in host memory); synchronous, makes no HIP call.  host_r, host_c:
 * int32[nnz_in]; host_v: f64[nnz_in].  Outputs host_rowptr int32[m+1],
 * host_colind int32[nnz_in] and host_values f64[nnz_in] (capacity nnz_in,
 * caller-owned); *host_nnz_out receives the stored count.  Canonical result:
 * rows ascending, columns strictly ascending in a row, duplicate (i, j)
 * summed in input order in FP64 -- bitwise the result of csr_from_coo on the
 * same triplets.  A triplet outside m x n returns SPX_ERR_INVALID with
 * *host_nnz_out = -1 and the outputs unspecified. */
spx_status csr_from_coo_host(int32_t m, int32_t n, int64_t nnz_in, const int32_t *host_r,
                             const int32_t *host_c, const double *host_v, int32_t *host_rowptr,
                             int32_t *host_colind, double *host_values, int32_t *host_nnz_out);

/* Structural check of CSR arrays in host memory (synchronous, no HIP call):
 * SPX_OK if rowptr[0] = 0, rowptr is non-decreasing, every entry lies in
 * [0, nnz], rowptr[m] = nnz and 0 <= colind[p] < n; otherwise
 * SPX_ERR_INVALID, with spx_last_error() naming the first violation found
 * (rows before columns).  Column order inside a row is not required. */
spx_status csr_validate_host(int32_t m, int32_t n, int32_t nnz, const int32_t *host_rowptr,
                             const int32_t *host_colind);

/* ---------------------------------------------------------------- plans
 * A plan bins the rows of one sparsity pattern by length (row_perm lists bin
 * 0's rows, then bin 1's, ..., ascending inside each bin) and, for a split
 * bin, cuts its rows into segments.  The plan's device arrays live in the
 * caller's workspace, which must stay allocated and unmodified while the plan
 * is used.  csr_plan_create reads the device rowptr and SYNCHRONISES `stream`
 * (it copies the bin sizes back to the host).  The plan may be used with any
 * values/x/X of the same pattern; SpMM with the plan needs k <= opts.max_k.
 * A plan with split rows keeps per-row arrival counters and partial sums in
 * its workspace: products through one such plan must not run concurrently
 * (order them on one stream, or give each stream its own plan); calls in
 * sequence are fine, since the last segment of each row resets its counter.
 * The same holds for a batch and its workspace. */
spx_status csr_plan_workspace_bytes(int32_t m, int32_t nnz, const spx_plan_opts *opts, size_t *bytes);
spx_status csr_plan_create(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr,
                           const spx_plan_opts *opts, void *workspace, size_t ws_bytes,
                           void *stream, spx_plan **out);
/* Copies row_perm (int32[m]) and bin_off (int32[nbins+1]) to host memory;
 * synchronous. */
spx_status csr_plan_export_bins(const spx_plan *plan, int32_t *host_row_perm, int32_t *host_bin_off);
/* Number of split segments and split rows of the plan. */
spx_status csr_plan_info(const spx_plan *plan, int32_t *nbins, int32_t *nsplit_rows, int32_t *nsegments);
void csr_plan_destroy(spx_plan *plan);

/* Staged plan for SpMM (Sec. 5's reuse of X rows by rows that share
 * columns): rows are cut into tiles of R consecutive rows, R = min(128 / L,
 * 64) with L the lanes that cover one X row at this k and X type; for each
 * tile the plan stores the sorted list of the columns its nonzeros touch
 * and, per nonzero, the 16-bit index of its column in that list.  A product
 * through the plan runs one workgroup per tile, copies the tile's X rows
 * (its window), values, indices and row offsets into LDS in one round of
 * vector loads, and computes from there.  A tile with more than 2,048
 * nonzeros or a window above 32 KB gathers X from memory instead, with the
 * same per-row arithmetic.  Built on the device from rowptr and colind
 * (columns need not be sorted), in the caller's workspace
 * (csr_plan_staged_workspace_bytes), which must stay allocated and
 * unmodified while the plan is used; SYNCHRONISES `stream`.  Serves csr_spmm
 * with exactly this k and X type, and X, Y that allow 16-byte loads
 * (16-byte aligned, ldx and ldy multiples of the vector); other calls return
 * SPX_ERR_UNSUPPORTED, as do csr_spmv_t, csr_sddmm and
 * csr_plan_export_bins.  k in [2, 128], a multiple of the 16-byte vector (2
 * FP64 or 4 FP32 elements); xtype F64 or F32 (the X / Y type). */
spx_status csr_plan_staged_workspace_bytes(int32_t m, int32_t n, int32_t nnz, int32_t k, spx_dtype xtype,
                                           size_t *bytes);
spx_status csr_plan_create_staged(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr,
                                  const int32_t *colind, int32_t k, spx_dtype xtype, void *workspace,
                                  size_t ws_bytes, void *stream, spx_plan **out);
/* Rows per tile, tiles, tiles staged in LDS, and the largest window (X rows). */
spx_status csr_plan_staged_info(const spx_plan *plan, int32_t *tile_rows, int32_t *ntiles, int32_t *nstaged,
                                int32_t *max_cols);
/* enable != 0: products through this staged plan run the pipelined kernel
 * (persistent workgroups, two LDS tile buffers: tile t + 1's window, values
 * and indices arrive through direct global-to-LDS loads while tile t is
 * computed; the X reuse of Sec. 5 with the wait for each tile's loads
 * overlapped) instead of one workgroup per tile; tiles that are not staged
 * still gather directly, in a second launch.  Same results, bitwise.
 * enable == 0 restores the default.  SPX_ERR_INVALID for a plan that is not
 * staged. */
spx_status csr_plan_staged_pipeline(spx_plan *plan, int32_t enable);

/* Hot x for SpMV (the x reuse of Sec. 4.1-4.2): ranks the pattern's columns
 * by use (as csr_degree_order) and keeps the `hot` most used, 1 <= hot <=
 * 2^20.  Every later csr_spmv through the plan (k = 1, x of type xtype: F64
 * or F32) first copies those hot x entries into a compact plan buffer (one
 * small kernel) and reads them from there, many to a cache line, instead of
 * one line of x each.
 * Results are bitwise those of the plan without hot x.  colind are the
 * pattern's column indices (the plan's n and nnz); the workspace
 * (csr_plan_hot_x_workspace_bytes) holds the plan's copy of them with hot
 * columns marked, the hot list and the x buffer, and must outlive the plan.
 * SpMM, the transpose and the sampled dot ignore the hot x.  Calls through
 * one plan with hot x share its x buffer: calls that may overlap (several
 * streams) race, as they do on a plan's split-row partials.  A staged plan
 * is rejected (SPX_ERR_UNSUPPORTED); an x of another type at call time is
 * SPX_ERR_INVALID. */
spx_status csr_plan_hot_x_workspace_bytes(int32_t n, int32_t nnz, int32_t hot, size_t *bytes);
spx_status csr_plan_attach_hot_x(spx_plan *plan, int32_t n, int32_t nnz, const int32_t *colind, int32_t hot,
                                 spx_dtype xtype, void *workspace, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- products
 * y <- A x.  vtype/xytype pairs: (F64, F64) plain FP64; (F32, F32) and
 * (BF16, F32) reduced-precision values with FP32 vectors.  x has n entries,
 * y has m.  plan == NULL uses a single unbinned kernel (lanes per row chosen
 * from nnz/m) and needs no workspace. */
spx_status csr_spmv(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr, const int32_t *colind,
                    const void *values, spx_dtype vtype, const void *x, void *y, spx_dtype xytype,
                    const spx_plan *plan, void *stream);

/* Y <- A X (Sec. 5).  X is n x k row-major with leading dimension ldx >= k,
 * Y is m x k row-major with ldy >= k (element strides).  Same dtype pairs as
 * csr_spmv.  For each row a zeroed accumulator of k entries collects
 * val[p] * X[colind[p], :]. */
spx_status csr_spmm(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr, const int32_t *colind,
                    const void *values, spx_dtype vtype, int32_t k, const void *X, int64_t ldx,
                    void *Y, int64_t ldy, spx_dtype xytype, const spx_plan *plan, void *stream);

/* ---------------------------------------------------------------- transpose / gradients
 * CSC index of a CSR pattern (the CCS dual, Sec. 3), built on the device:
 * colptr int32[n+1]; rowind int32[nnz] and perm int32[nnz] list, column by
 * column and in ascending row order inside a column, the row and the CSR
 * position of each nonzero.  Deterministic. */
spx_status csr_transpose_index_workspace_bytes(int32_t m, int32_t n, int32_t nnz, size_t *bytes);
spx_status csr_transpose_index(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr,
                               const int32_t *colind, int32_t *colptr, int32_t *rowind,
                               int32_t *perm, void *workspace, size_t ws_bytes, void *stream);

/* dX <- A^T dY.  dY is m x k (lddy), dX is n x k (lddx), row-major;
 * lddy and lddx are at least k, also for k = 1 (SPX_ERR_INVALID otherwise).
 * mode 0 (CSC index, deterministic): needs colptr/rowind from
 * csr_transpose_index; every column is a gather in ascending row order, run
 * by the product kernels over the CSC pattern.  With perm (from the same
 * call) the CSR-order values are read through it; with perm == NULL,
 * `values` must already be in CSC order (csr_values_to_csc), and the result
 * is bitwise the same.
 * `plan` (nullable) must then be a plan of the CSC pattern: created from
 * colptr with n rows.  mode 1 (atomic scatter): colptr/rowind/perm may be
 * NULL; dX is zeroed and then accumulated with atomic adds (summation order
 * not deterministic); `plan` (nullable) is then a plan of the CSR pattern and
 * only sets the traversal. */
spx_status csr_spmv_t(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr, const int32_t *colind,
                      const int32_t *colptr, const int32_t *rowind, const int32_t *perm,
                      const void *values, spx_dtype vtype, int32_t k, const void *dY, int64_t lddy,
                      void *dX, int64_t lddx, spx_dtype xytype, int32_t mode, const spx_plan *plan,
                      void *stream);

/* Values in CSC order, values_csc[q] = values[perm[q]] (perm from
 * csr_transpose_index), moved without per-element random reads: a one-time
 * map of the pattern (csr_csc_value_map: dest int32[nnz], local
 * uint16[nnz]) groups the nonzeros by block of SPX_CSC_BLOCK CSC positions;
 * csr_values_to_csc then streams values into `staging` (nnz elements of
 * vtype) block by block and reorders each block in LDS into values_csc.
 * Bitwise a permutation of the input.  Workspace of the map:
 * csr_csc_value_map_workspace_bytes.  Asynchronous on `stream`. */
#define SPX_CSC_BLOCK 8192
spx_status csr_csc_value_map_workspace_bytes(int32_t nnz, size_t *bytes);
spx_status csr_csc_value_map(int32_t nnz, const int32_t *perm, int32_t *dest, uint16_t *local, void *workspace,
                             size_t ws_bytes, void *stream);
spx_status csr_values_to_csc(int32_t nnz, const int32_t *dest, const uint16_t *local, const void *values,
                             spx_dtype vtype, void *staging, void *values_csc, void *stream);

/* csr_values_to_csc without the caller's staging buffer, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  It allocates nothing: the
 * staging lives in a fixed device array of SPX_NOALLOC_SCRATCH_BYTES that
 * the library holds on every GPU it runs on until the process ends; its
 * address on the current device is looked up once, on the first call on that
 * device.  Same arguments and result as csr_values_to_csc (bitwise).
 * nnz * sizeof(vtype) above SPX_NOALLOC_SCRATCH_BYTES (6,291,456 FP64,
 * 12,582,912 FP32 or 25,165,824 BF16 values) returns SPX_ERR_UNSUPPORTED
 * and launches nothing.  Every call on one GPU shares that GPU's array (no
 * part of it needs clearing: each call writes every staging slot it reads):
 * calls that may overlap on one GPU (different streams, or host threads
 * without ordering) race and must be serialised by the caller. */
#define SPX_NOALLOC_SCRATCH_BYTES 50331648 /* 48 MiB */
spx_status csr_values_to_csc_noalloc(int32_t nnz, const int32_t *dest, const uint16_t *local,
                                     const void *values, spx_dtype vtype, void *values_csc, void *stream);

/* Sampled dot: out[p] = sum_t dY[row(p), t] * X[colind[p], t] for every
 * stored nonzero p (the gradient of y = A(values) x with respect to values).
 * dtype F64 or F32 for dY, X and out alike.  dY is m x k (lddy) and X is
 * n x k (ldx), row-major, with lddy and ldx at least k, also for k = 1
 * (SPX_ERR_INVALID otherwise).  `plan` (nullable) is a plan of the CSR
 * pattern and only sets the traversal (rows by bins). */
spx_status csr_sddmm(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr, const int32_t *colind,
                     int32_t k, const void *dY, int64_t lddy, const void *X, int64_t ldx, void *out,
                     spx_dtype dtype, const spx_plan *plan, void *stream);

/* y <- A x as csr_spmv (same arguments, plans and bitwise the same y), and
 * also xsave[p] = x[colind[p]] for every stored nonzero p: nnz elements of
 * xytype, written in CSR order (device memory of the caller).  The sampled
 * dot of a later backward can then read that operand as a stream
 * (csr_sddmm_saved) instead of gathering x again: nnz x sizeof(xytype) more
 * bytes written here, a random gather fewer there.  A staged plan is
 * rejected (SPX_ERR_UNSUPPORTED); xsave == NULL with nnz > 0 is
 * SPX_ERR_INVALID.  Asynchronous on `stream`. */
spx_status csr_spmv_save(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr, const int32_t *colind,
                         const void *values, spx_dtype vtype, const void *x, void *y, spx_dtype xytype,
                         void *xsave, const spx_plan *plan, void *stream);

/* Sampled dot from a saved gather (k = 1): out[p] = dy[row(p)] * xsave[p]
 * for every stored nonzero p, with xsave from csr_spmv_save.  Bitwise equal
 * to csr_sddmm(k = 1) with the x that was saved.  dtype F64 or F32 for dy,
 * xsave and out alike; dy has m entries, xsave and out nnz.  `plan`
 * (nullable, not staged) is a plan of the CSR pattern and only sets the
 * traversal.  Asynchronous on `stream`. */
spx_status csr_sddmm_saved(int32_t m, int32_t nnz, const int32_t *rowptr, const void *dy, const void *xsave,
                           void *out, spx_dtype dtype, const spx_plan *plan, void *stream);

/* ---------------------------------------------------------------- batches
 * Many independent products Y_b <- A_b X_b in one kernel launch per lane
 * layout present (the layout follows from each matrix's k: at most a few
 * launches, whatever the number of matrices).  Each descriptor names one CSR
 * matrix, its right-hand side and its plan options (from an autotuner or
 * spx_plan_default_opts).  csr_batch_create bins every matrix on the device,
 * builds the work-tile list in the caller's workspace (grouped by layout,
 * heaviest estimated tiles first) and SYNCHRONISES `stream`.  csr_batch_run
 * launches, on `stream`, one workgroup per tile of each layout's group; it
 * uses no memset and no atomics outside the split-row reductions, so it can
 * be captured into a HIP graph.  Each matrix's result is bit-identical to
 * csr_spmm (k > 1) or csr_spmv (k = 1) with a plan created from the same
 * options plus SPX_FLAG_KEEP_STREAM: the batch fills the device as a whole,
 * so it keeps every stream bin as 256-row tiles. */
typedef struct spx_csr_desc {
  int32_t m, n, nnz, k;
  const int32_t *rowptr;
  const int32_t *colind;
  const void *values;
  const void *X; /* x when k = 1 */
  void *Y;       /* y when k = 1 */
  int64_t ldx, ldy;
  spx_dtype vtype, xytype;
  spx_plan_opts opts;
} spx_csr_desc;

spx_status csr_batch_workspace_bytes(int32_t count, const spx_csr_desc *host_descs, size_t *bytes);
spx_status csr_batch_create(int32_t count, const spx_csr_desc *host_descs, void *workspace,
                            size_t ws_bytes, void *stream, spx_batch **out);
spx_status csr_batch_run(const spx_batch *batch, void *stream);
/* Tiles, workgroups of the largest per-layout launch, and total split segments. */
spx_status csr_batch_info(const spx_batch *batch, int64_t *ntiles, int32_t *grid, int64_t *nsegments);
void csr_batch_destroy(spx_batch *batch);

/* ---------------------------------------------------------------- ordering and structure metrics
 * Reverse Cuthill-McKee ordering (Sec. 4.4: permuting rows and columns to
 * pull the nonzeros toward the diagonal, applied before the product).  Host
 * function on host arrays of a square CSR matrix; fills host_perm[new] = old
 * (a permutation of 0..m-1).  The graph is the pattern of A + A^T without
 * the diagonal.  Ties are fixed (the paper used MATLAB's routine and states
 * none): each component starts from the unnumbered vertex of least (degree,
 * index), moved to a pseudo-peripheral vertex by George and Liu's rule; the
 * unnumbered neighbours of each vertex follow in ascending (degree, index);
 * the breadth-first numbering is reversed at the end.  Checks the CSR
 * structure; SPX_ERR_INVALID for m != n or bad arrays. */
spx_status csr_rcm(int32_t m, int32_t n, int32_t nnz, const int32_t *host_rowptr,
                   const int32_t *host_colind, int32_t *host_perm);

/* P A P^T on the device for a device permutation perm[new] = old of
 * 0..m-1 (square m x m matrix, FP64 values): row i of the result is row
 * perm[i] of A with every column j renamed to the new index of j; the output
 * is canonical CSR (columns ascending).  Outputs rowptr_out int32[m+1],
 * colind_out int32[nnz], values_out f64[nnz]; *nnz_out (device int32)
 * receives nnz, or -1 if perm is not a permutation.  Workspace:
 * csr_permute_workspace_bytes.  Asynchronous on `stream`. */
spx_status csr_permute_workspace_bytes(int32_t m, int32_t nnz, size_t *bytes);
spx_status csr_permute(int32_t m, int32_t nnz, const int32_t *rowptr, const int32_t *colind,
                       const double *values, const int32_t *perm, int32_t *rowptr_out,
                       int32_t *colind_out, double *values_out, int32_t *nnz_out, void *workspace,
                       size_t ws_bytes, void *stream);

/* Degree ordering: columns by descending number of nonzeros, ties in
 * ascending index; perm int32[n] receives perm[new] = old.  For a square
 * matrix, csr_permute with this perm relabels rows and columns together, so
 * the most-referenced x entries share cache lines (an alternative to the
 * paper's RCM step, Sec. 4.4, for matrices whose column use is skewed rather
 * than banded).  colind int32[nnz] on the device; entries outside [0, n) are
 * not counted.  Workspace: csr_degree_order_workspace_bytes.  Asynchronous
 * on `stream`. */
spx_status csr_degree_order_workspace_bytes(int32_t n, int32_t nnz, size_t *bytes);
spx_status csr_degree_order(int32_t n, int32_t nnz, const int32_t *colind, int32_t *perm, void *workspace,
                            size_t ws_bytes, void *stream);

/* Bandwidth (Sec. 4.4): *bw_out (device int32) receives the largest distance
 * |colind[p] - r| between a nonzero and the diagonal over all rows r (0 for a
 * matrix without nonzeros), the row period to give a plan that orders a banded
 * matrix's rows band by band (spx_plan_opts.row_period).  rowptr int32[m+1],
 * colind int32[nnz] on the device, assumed valid (csr_validate).  One thread
 * per row.  Asynchronous on `stream`. */
spx_status csr_bandwidth(int32_t m, int32_t nnz, const int32_t *rowptr, const int32_t *colind,
                         int32_t *bw_out, void *stream);

/* Vector access (Sec. 4.2, Sec. 4.4): the expected number of times x is moved
 * from memory when rows are dealt round-robin, in chunks of `chunk`
 * consecutive rows, to `parts` caches that never evict: distinct (part,
 * x cacheline) pairs divided by ceil(n / line), `line` = x elements per
 * cacheline.  Host function on host arrays; *out is host. */
spx_status csr_vector_access(int32_t m, int32_t n, int32_t nnz, const int32_t *host_rowptr,
                             const int32_t *host_colind, int32_t line, int32_t parts, int32_t chunk,
                             double *out);

/* Distinct x cachelines per row tile (Sec. 4.1 and 4.2 count the cachelines
 * a row's or a core's gathers touch; this is the count for a workgroup that
 * serves `tile` consecutive rows): *out receives the number of distinct
 * (tile, x line) pairs over the tiles [t*tile, (t+1)*tile), x line =
 * column / line.  Divided by the tile count it is the mean distinct lines a
 * tile gathers; nnz divided by it is the mean number of gathers per line
 * inside a tile.  Host function on host arrays of a structurally valid
 * matrix (a column outside [0, n) returns SPX_ERR_INVALID); *out is host. */
spx_status csr_tile_lines(int32_t m, int32_t n, int32_t nnz, const int32_t *host_rowptr,
                          const int32_t *host_colind, int32_t line, int32_t tile, int64_t *out);

/* Useful cacheline density (Sec. 4.1): the mean over nonempty rows of
 * L / (line x distinct x cachelines the row touches); columns ascending in
 * each row.  Host function on host arrays; *out is host. */
spx_status csr_ucld(int32_t m, int32_t nnz, const int32_t *host_rowptr, const int32_t *host_colind,
                    int32_t line, double *out);

/* ---------------------------------------------------------------- register blocking
 * Register-blocked CRS (Sec. 4.5): A is cut into a x b blocks (a, b in
 * {1, 2, 4, 8}); every block that holds a nonzero is kept, block rows
 * ascending and block columns ascending inside a block row.  browptr
 * int32[ceil(m/a)+1] and bcol int32[nblocks] index the blocks.  Dense form
 * (bitmap = 0): bvals f64[nblocks*a*b], row-major inside each block, zeros
 * explicit (the paper's register blocking).  Bitmap form (bitmap = 1): bmask
 * uint64[nblocks] has bit r*b+c set for a nonzero at (r, c) of the block;
 * bvals f64[nnz] holds the nonzeros block after block in bit order and
 * boff int32[nblocks] the index of each block's first value (the sparse block
 * storage the paper proposes as its next step).  The input CSR must have
 * ascending columns inside rows (csr_from_coo's output does).
 * csr_bcsr_count writes the block count to *nblocks_out (device int32) so the
 * caller can size the outputs; csr_to_bcsr then fills them.  Both use the
 * workspace of bcsr_workspace_bytes and run asynchronously on `stream`. */
spx_status bcsr_workspace_bytes(int32_t m, int32_t n, int32_t nnz, size_t *bytes);
spx_status csr_bcsr_count(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr, const int32_t *colind,
                          int32_t a, int32_t b, int32_t *nblocks_out, void *workspace, size_t ws_bytes,
                          void *stream);
spx_status csr_to_bcsr(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr, const int32_t *colind,
                       const double *values, int32_t a, int32_t b, int32_t bitmap, int32_t *browptr,
                       int32_t *bcol, double *bvals, uint64_t *bmask, int32_t *boff, void *workspace,
                       size_t ws_bytes, void *stream);

/* y <- A x with A in register-blocked form (Sec. 4.5), FP64.  Each block row
 * is served by `lanes` threads (a power of two <= 64; 0 picks it from the
 * mean blocks per block row); every thread multiplies whole blocks and the
 * group reduces its a partial sums.  x f64[n], y f64[m] (overwritten). */
spx_status bcsr_spmv(int32_t m, int32_t n, int32_t a, int32_t b, int32_t bitmap, int32_t nblocks,
                     const int32_t *browptr, const int32_t *bcol, const double *bvals, const uint64_t *bmask,
                     const int32_t *boff, const double *x, double *y, int32_t lanes, void *stream);

/* Y <- A X with A in register-blocked form (Sec. 4.5) applied to the
 * multi-vector product (Sec. 5): dense a x 1 blocks (a in {2, 4, 8}, b = 1,
 * bitmap form not taken).  Each X row a block refers to is gathered once and
 * multiplied into a rows of Y, so a banded matrix whose consecutive rows
 * share columns gathers fewer X rows than through CSR, at the price of the
 * block's explicit zeros.  bvals holds the blocks' values as csr_to_bcsr
 * lays them out, in vtype; (vtype, xytype) is (F64, F64) -- FP64 throughout
 * -- or (F32 / BF16, F32): FP32 products and sums, without the compensated
 * sums of the CSR kernels' long rows (blocked storage serves banded matrices,
 * whose rows are short).  X n x k, row stride ldx >= k; Y m x k, row stride
 * ldy >= k, overwritten.  `slots` blocks of a block row are walked at a time
 * (a power of two; 0 picks it from the mean blocks per block row); k above
 * 32 x (elements per 16 bytes) runs in column slabs.  row_period: 0, or
 * P > 0 as in spx_plan_opts.row_period (rows; the bandwidth, csr_bandwidth):
 * XCD j serves band j of every period of ceil(P / a) block rows, in ascending
 * order, instead of the j-th eighth of the block rows; the same bits either
 * way.  Asynchronous on `stream`.  Other block shapes or type pairs return
 * SPX_ERR_UNSUPPORTED. */
spx_status bcsr_spmm(int32_t m, int32_t n, int32_t a, int32_t b, int32_t nblocks, const int32_t *browptr,
                     const int32_t *bcol, const void *bvals, spx_dtype vtype, int32_t k, const void *X,
                     int64_t ldx, void *Y, int64_t ldy, spx_dtype xytype, int32_t slots, int32_t row_period,
                     void *stream);

/* ---------------------------------------------------------------- probes
 * Memory-system probes (the GPU counterparts of the paper's read / write
 * bandwidth microbenchmarks, Sec. 2.1 and 2.2), used to calibrate measured
 * bandwidth.  kind 0: streaming read of buf (buf2: optional device double
 * that keeps the loads live); 1: write buf; 2: non-temporal write of buf;
 * 3: non-temporal copy buf -> buf2; 4: read-modify-write of buf (a cache
 * flush); 5: random gather of 128-byte rows of buf (8 lanes x 16 bytes per
 * row, the SpMM X access at k = 16 FP64); 6: random gather of 8-byte
 * elements of buf (the SpMV x access).  Kinds 5 and 6 make 256 rounds per
 * wavefront (4 wavefronts per workgroup); a round reads 8 rows (kind 5) or
 * 64 elements (kind 6); they give the random-access ceiling of a working set
 * of `bytes` (Sec. 4.2's latency argument).  bytes is rounded down to
 * 16-byte units; buffers must be 16-byte aligned; blocks <= 0 picks 4096
 * workgroups of 256 threads. */
spx_status spx_probe(int32_t kind, void *buf, void *buf2, size_t bytes, int32_t blocks, void *stream);

/* The x access of an SpMV in isolation (Sec. 4.2 attributes SpMV time to the
 * x gather): idx int32[nidx] is streamed (non-temporal loads, as the products
 * stream colind) and, with gather != 0, x[idx[p]] is read through L2 for every
 * p; with gather == 0 only the index stream is read.  blocks workgroups (a
 * positive multiple of 8) each take one contiguous range of idx, XCD-
 * contiguous like the product tiles, and write the sum of what they read to
 * sink[tile] (f64[blocks]; per-workgroup sums in a fixed order).  With
 * gather != 0, entries outside [0, n) are skipped (not read).  Counter runs of the two modes
 * separate the gather's L2 hits and misses from the index stream's. */
spx_status spx_probe_index_gather(const int32_t *idx, int64_t nidx, const double *x, int32_t n,
                                  int32_t gather, double *sink, int32_t blocks, void *stream);

/* Load-to-use latency (the paper's latency argument, Sec. 4.2): one wavefront
 * whose lane l follows i <- next[i] & (n - 1) from start[l] for `hops`
 * dependent loads and writes its final index to out[l] (int32[64]).  next is
 * int32[n] with n a power of two (a single random cycle gives one new line
 * per hop); start int32[64] (equal entries: one address per load; distinct
 * entries: 64 independent chains, one gather per hop).  Time / hops is the
 * latency per dependent load of a working set of 4n bytes. */
spx_status spx_probe_chase(const int32_t *next, int64_t n, const int32_t *start, int64_t hops, int32_t *out,
                           void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SPX_H */
