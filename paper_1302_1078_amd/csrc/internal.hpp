// internal.hpp -- host/device structures shared by the translation units of
// libspx (not part of the public ABI; see include/spx.h for that).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "spx.h"

namespace spx {

// ------------------------------------------------------------------ errors

spx_status fail(spx_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
spx_status hip_fail(hipError_t e, const char* what);

#define SPX_HIP(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return spx::hip_fail(e_, #call); \
  } while (0)

// Launch error check right after a <<<>>> launch.
#define SPX_LAUNCHED(name)                                   \
  do {                                                       \
    hipError_t e_ = hipGetLastError();                       \
    if (e_ != hipSuccess) return spx::hip_fail(e_, name);    \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// nnz within the int32 position range the kernels assume: a position plus
// one split chunk plus the widest look-ahead past a row's end (U x S <= 2,048
// slots) stays below 2^31.
static_assert(static_cast<int64_t>(SPX_MAX_NNZ) + SPX_MAX_SPLIT_CHUNK + 4096 <= 0x7fffffffLL,
              "position headroom");
inline spx_status check_nnz(int64_t nnz, const char* who) {
  if (nnz > SPX_MAX_NNZ)
    return fail(SPX_ERR_UNSUPPORTED, "%s: nnz=%lld above SPX_MAX_NNZ=%d", who, static_cast<long long>(nnz),
                SPX_MAX_NNZ);
  return SPX_OK;
}

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Bump allocator over a caller workspace (256-byte aligned pieces).
struct Carve {
  char* base;
  size_t cap;
  size_t used = 0;
  Carve(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <typename T>
  T* take(size_t count) {
    size_t off = align_up(used);
    used = off + align_up(count * sizeof(T));
    if (base == nullptr) return nullptr;  // sizing pass
    return reinterpret_cast<T*>(base + off);
  }
  bool ok() const { return used <= cap; }
};

// ------------------------------------------------------------------ device primitives
// (scan_sort.hip)

constexpr int kScanTile = 4096;  // 256 threads x 16 items

// Exclusive scan of n int32 values (in may equal out).  *total (device, may be
// null) receives the sum.  Workspace from scan_workspace_bytes(n).
size_t scan_workspace_bytes(int64_t n);
spx_status exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total,
                              void* ws, hipStream_t st);

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the
// key.  keys/vals are sorted in place (ping-pong buffers come from ws).
size_t radix_workspace_bytes(int64_t n, int key_bytes);
spx_status radix_sort_u32(uint32_t* keys, int32_t* vals, int64_t n, int bits, void* ws,
                          hipStream_t st);
spx_status radix_sort_u64(uint64_t* keys, int32_t* vals, int64_t n, int bits, void* ws,
                          hipStream_t st);

// ------------------------------------------------------------------ products

struct BinDesc {
  int32_t blk_begin;  // first workgroup (multiple of 8)
  int32_t nblk;       // workgroups of this bin
  int32_t row_begin;  // offset into row_perm (unused when row_perm is null)
  int32_t nrows;      // rows of the bin (segments for a split bin)
  int32_t lanes;      // threads per row (0 = split segments)
  int32_t bin;        // index of the plan bin this entry serves
  int32_t rpg;        // rows per row group (1, or 4 for short-row bins)
  int32_t pad;
};

struct ProdArgs {
  const int32_t* rowptr;
  const int32_t* colind;
  const void* values;
  const int32_t* vperm;  // value index indirection (CSC gather), or null
  const void* X;
  void* Y;
  int64_t ldx, ldy;
  const void* X2;  // sampled dot: the second dense operand (n x k), or the saved gather;
                   // hot-x SpMV: the compact hot x entries (ldx2 of them)
  int64_t ldx2;
  void* xsave;     // SpMV with save: x[colind[p]] is also stored at xsave[p] (XT)
  int32_t k;
  int32_t kahan_len;
  const int32_t* row_perm;   // null = identity order
  const int32_t* prange;     // per binned row: rowptr[row], rowptr[row + 1]
  const int32_t* seg_row;    // split: segment -> split-row index
  const int32_t* seg_first;  // split: split-row -> first segment (nsplit + 1 entries)
  const int32_t* split_rows; // split: split-row index -> row
  int32_t* counters;         // split: arrival counters, zero between calls
  double* partials;          // split: max_k doubles per segment
  int32_t chunk;
  int32_t max_k;
  uint32_t flags;
  int32_t occupancy;         // 0, or the workgroups-per-CU cap of the launch
  int32_t nbins;
  BinDesc bins[SPX_MAX_BINS];
};

}  // namespace spx

// The opaque plan object.
struct spx_plan {
  int32_t m, n, nnz;
  spx_plan_opts opts;
  int32_t bin_off[SPX_MAX_BINS + 1];  // host copy
  int32_t nsplit;                     // rows in the split bin (0 if none)
  int32_t nseg;                       // total split segments
  int32_t cus;                        // compute units of the plan's device
  int32_t* row_perm;                  // device, [m]
  int32_t* prange;                    // device, [2 m]: nonzero range of row_perm[i]
  int32_t* seg_row;                   // device, [nseg]
  int32_t* seg_first;                 // device, [nsplit + 1]
  int32_t* counters;                  // device, [nsplit]
  double* partials;                   // device, [nseg * max_k]
  // X staging (csr_plan_create_staged; zero for a binned plan): rows in tiles
  // of tile_rows consecutive rows, each tile's distinct X rows staged in LDS
  int32_t staged;                     // 1 for a staged plan, 2 for one run by the pipelined kernel
  int32_t k;                          // right-hand sides the windows were sized for
  int32_t xtype;                      // spx_dtype of X / Y
  int32_t kl, vec;                    // lane layout of the product (lanes per X row, elements per lane)
  int32_t tile_rows;                  // rows per tile (kWG / kl)
  int32_t ntiles;
  int32_t nstaged;                    // tiles whose window is staged (the rest gather directly)
  int32_t max_cols;                   // largest staged window, in X rows
  int32_t max_nnz;                    // most nonzeros in a staged tile
  int32_t* tile_cols;                 // device, [ntiles]: window size, or -1 (direct gathers)
  int32_t* tile_off;                  // device, [ntiles + 1]: offset of the tile's column list
  int32_t* tcols;                     // device: the tiles' sorted distinct columns, concatenated
  uint16_t* loc;                      // device, [nnz]: window index of each nonzero of a staged tile
  // hot x (csr_plan_attach_hot_x; hot == 0: none): SpMV keeps the x entries
  // of the hot most-used columns in LDS
  int32_t hot;                        // number of hot columns
  int32_t hot_xtype;                  // spx_dtype of the x it serves
  const int32_t* hot_cols;            // device, [hot]: the hot columns, most used first
  const int32_t* colind_hot;          // device, [nnz]: colind with hot columns as ~slot
  void* x_hot;                        // device, [hot] of hot_xtype: x of the hot columns, per call
};

namespace spx {
// Launch one fused product over a prepared bin table (product.hip).
spx_status launch_product(ProdArgs& a, int vt, int xt, int kl, int vec, hipStream_t st);
spx_status launch_product_save(ProdArgs& a, int vt, int xt, hipStream_t st);
// SpMV through a plan with hot x (a.colind = the plan's colind_hot, a.X2 = its
// x_hot, already filled, a.ldx2 = hot).
spx_status launch_product_hot(ProdArgs& a, int vt, int xt, hipStream_t st);
// Fill plan->x_hot from x (hot.hip).
spx_status gather_hot_x(const spx_plan* plan, const void* x, hipStream_t st);
// Fill a ProdArgs bin table from a plan, or from the unbinned heuristic.
// `own_launch`: the table drives a launch of its own (not a tile list shared
// with other matrices), so a stream bin too small to fill the device is
// served by row groups instead (unless SPX_FLAG_KEEP_STREAM).
void bins_from_plan(const spx_plan* plan, ProdArgs& a, int kl, bool own_launch);
void bins_unbinned(int32_t m, int32_t nnz, int kl, ProdArgs& a);
int lanes_valid(int lanes);
// Lanes per X row (KL) and elements per lane (VEC) for k right-hand sides.
void layout_for_k(int32_t k, spx_dtype xt, const void* X, int64_t ldx, const void* Y, int64_t ldy,
                  uint32_t flags, int* kl, int* vec);
// Product through a staged plan (staged.hip).
spx_status launch_staged(ProdArgs& a, const spx_plan* plan, int32_t m, int vt, int xt, int kl, int vec,
                         hipStream_t st);
// Backward traversals (grad.hip).
spx_status launch_scatter_t(ProdArgs& a, const spx_plan* plan, int32_t m, int32_t n, int32_t nnz,
                            int vt, int xt, hipStream_t st);
spx_status launch_sddmm(ProdArgs& a, const spx_plan* plan, int32_t m, int32_t nnz, int dt, bool saved,
                        hipStream_t st);
}  // namespace spx
