// grad.hip -- per-nonzero traversals for the backward of y = A(values) x:
//   mode kScatterT: dX[colind[p], :] += values[p] * dY[row(p), :] (atomic)
//   mode kSddmm:    out[p] = sum_t dY[row(p), t] * X[colind[p], t]
//   mode kSddmmSaved (k = 1): out[p] = dY[row(p)] * xg[p], with xg[p] the
//                   x[colind[p]] that the forward stored (the save variant of
//                   the SpMV): the same products, read as a stream
// Rows are visited through the same bin table as the products (row groups of
// G lanes, or one workgroup per segment of a split row); no cross-lane
// reduction is needed because every nonzero is independent.
#include <mutex>

#include "device.hpp"
#include "internal.hpp"

namespace spx {

namespace {

enum { kScatterT = 0, kSddmm = 1, kSddmmSaved = 2 };

// The nonzeros p, p + step, ... < p1 of one row, kVisit at a time: the index
// (and value) loads of a round are issued before any gather, and the gathers
// before any use, so a lane keeps kVisit load chains in flight.  Each
// nonzero's arithmetic is the same expression whatever the batching.
constexpr int kVisit = 4;

// Scatter-add merging (A^T dy with k = 1): a workgroup first adds its
// contributions into an LDS table keyed by column (linear probing, a slot
// claimed by compare-and-swap), then adds each occupied slot to dX with one
// atomic.  L2 forwards every global atomic to memory, so the scatter is
// bound by how many atomics it issues; the table removes the repeats of a
// column inside a workgroup (on a power-law matrix, the hottest columns).
// A contribution that finds no slot within kProbes goes straight to memory.
constexpr int kMergeSlots = 2048;
constexpr int kMergeBits = 11;
constexpr int kProbes = 8;
static_assert((1 << kMergeBits) == kMergeSlots, "slots a power of two");

template <typename XT>
struct MergeTab {
  int32_t* key;  // column, or -1
  XT* val;
};

template <typename XT>
__device__ __forceinline__ void merge_add(const MergeTab<XT>& tb, XT* y, int64_t ldy, int32_t c, XT v) {
  const uint32_t h = (static_cast<uint32_t>(c) * 2654435761u) >> (32 - kMergeBits);
#pragma unroll
  for (int q = 0; q < kProbes; ++q) {
    const uint32_t sl = (h + q) & (kMergeSlots - 1);
    int32_t k = tb.key[sl];
    if (k == -1) {
      k = atomicCAS(&tb.key[sl], -1, c);
      if (k == -1) k = c;  // claimed
    }
    if (k == c) {  // an LDS add, kept apart from the global fallback below
      auto* lv = reinterpret_cast<__attribute__((address_space(3))) XT*>(
          reinterpret_cast<uintptr_t>(tb.val + sl) & 0xffffffffu);
      __hip_atomic_fetch_add(lv, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return;
    }
  }
  atomicAdd(y + static_cast<int64_t>(c) * ldy, v);
}

template <typename VT, typename XT, int MODE, bool MERGE = false>
__device__ __forceinline__ void visit_run(const ProdArgs& a, int32_t row, int32_t p, int32_t p1, int step,
                                          const MergeTab<XT>& tb = MergeTab<XT>{nullptr, nullptr}) {
  const XT* dy = static_cast<const XT*>(a.X) + static_cast<int64_t>(row) * a.ldx;
  const XT dy0 = (p < p1) ? dy[0] : XT(0);  // k = 1: one dY entry per row
  for (; p < p1; p += kVisit * step) {
    bool h[kVisit];
    int32_t c[kVisit];
#pragma unroll
    for (int u = 0; u < kVisit; ++u) {
      h[u] = p + u * step < p1;
      c[u] = (h[u] && MODE != kSddmmSaved) ? ld_stream(a.colind + p + u * step) : 0;
    }
    if constexpr (MODE == kScatterT) {
      XT v[kVisit];
#pragma unroll
      for (int u = 0; u < kVisit; ++u)
        v[u] = h[u] ? static_cast<XT>(ValueLoad<VT>::get(static_cast<const VT*>(a.values) + p + u * step)) : XT(0);
#pragma unroll
      for (int u = 0; u < kVisit; ++u) {
        if (!h[u]) continue;
        XT* dst = static_cast<XT*>(a.Y) + static_cast<int64_t>(c[u]) * a.ldy;
        if constexpr (MERGE) merge_add(tb, static_cast<XT*>(a.Y), a.ldy, c[u], v[u] * dy0);
        else if (a.k == 1) atomicAdd(dst, v[u] * dy0);
        else
          for (int t = 0; t < a.k; ++t) atomicAdd(dst + t, v[u] * dy[t]);
      }
    } else {
      const XT* X2 = static_cast<const XT*>(a.X2);
      if (MODE == kSddmmSaved || a.k == 1) {
        XT xr[kVisit];
#pragma unroll
        for (int u = 0; u < kVisit; ++u) {
          if constexpr (MODE == kSddmmSaved) xr[u] = h[u] ? ld_stream(X2 + p + u * step) : XT(0);
          else xr[u] = h[u] ? X2[static_cast<int64_t>(c[u]) * a.ldx2] : XT(0);
        }
#pragma unroll
        for (int u = 0; u < kVisit; ++u) {
          XT s = XT(0);
          s = s + dy0 * xr[u];
          if (h[u]) __builtin_nontemporal_store(s, static_cast<XT*>(a.Y) + p + u * step);
        }
      } else {
#pragma unroll
        for (int u = 0; u < kVisit; ++u) {
          if (!h[u]) continue;
          const XT* xr = X2 + static_cast<int64_t>(c[u]) * a.ldx2;
          XT s = XT(0);
          for (int t = 0; t < a.k; ++t) s = s + dy[t] * xr[t];
          __builtin_nontemporal_store(s, static_cast<XT*>(a.Y) + p + u * step);
        }
      }
    }
  }
}

// Stream bin, k = 1: the tile's 256 rows (one per thread) are walked as one
// flat sequence of nonzeros, as the forward stream kernel does: lanes take
// consecutive nonzeros (coalesced index loads and output stores), the row of
// each comes from a lockstep search over the rows' offsets in LDS, and the
// rows' dY entries are staged in LDS once.
template <typename VT, typename XT, int MODE, bool MERGE = false>
__device__ __forceinline__ void visit_stream(const ProdArgs& a, const BinDesc& d, int tile,
                                             const MergeTab<XT>& tb = MergeTab<XT>{nullptr, nullptr}) {
  constexpr int kStreamRows = kWG;  // a stream tile: one bin row per thread (the bin table's layout)
  constexpr int kChunk = 1024, kPer = kChunk / kWG;
  __shared__ int32_t s_off[kStreamRows + 1];
  __shared__ int32_t s_p0[kStreamRows];
  __shared__ XT s_dy[kStreamRows];
  __shared__ int32_t s_wsum[kWG / kWave];
  if (tile * kStreamRows >= d.nrows) return;
  const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
  const int idx = tile * kStreamRows + t;
  int32_t row = 0, p0 = 0, p1 = 0;
  if (idx < d.nrows) {
    if (a.row_perm) {
      row = a.row_perm[d.row_begin + idx];
      const int2 pr = reinterpret_cast<const int2*>(a.prange)[d.row_begin + idx];
      p0 = pr.x;
      p1 = pr.y;
    } else {
      row = d.row_begin + idx;
      p0 = a.rowptr[row];
      p1 = a.rowptr[row + 1];
    }
  }
  const int32_t L = p1 - p0;
  const XT dyv = (L > 0) ? static_cast<const XT*>(a.X)[static_cast<int64_t>(row) * a.ldx] : XT(0);
  int32_t inc = L;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t u = __shfl_up(inc, off, kWave);
    if (lane >= off) inc += u;
  }
  if (lane == kWave - 1) s_wsum[w] = inc;
  __syncthreads();
  int32_t before = 0, total = 0;
#pragma unroll
  for (int i = 0; i < kWG / kWave; ++i) {
    if (i < w) before += s_wsum[i];
    total += s_wsum[i];
  }
  s_off[t] = before + inc - L;
  s_p0[t] = p0;
  s_dy[t] = dyv;
  if (t == kWG - 1) s_off[kStreamRows] = total;
  total = __builtin_amdgcn_readfirstlane(total);
  __syncthreads();
  for (int32_t base = 0; base < total; base += kChunk) {
    int32_t lo[kPer], p[kPer], c[kPer];
    bool ok[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int32_t j = base + u * kWG + t;
      ok[u] = j < total;
      lo[u] = 0;
      p[u] = ok[u] ? j : total - 1;  // the search key; past the end: the last element again
    }
#pragma unroll
    for (int step = kStreamRows / 2; step >= 1; step >>= 1) {
#pragma unroll
      for (int u = 0; u < kPer; ++u)
        if (s_off[lo[u] + step] <= p[u]) lo[u] += step;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      p[u] = s_p0[lo[u]] + (p[u] - s_off[lo[u]]);
      c[u] = (MODE != kSddmmSaved) ? ld_stream(a.colind + p[u]) : 0;
    }
    if constexpr (MODE == kScatterT) {
      XT v[kPer];
#pragma unroll
      for (int u = 0; u < kPer; ++u)
        v[u] = static_cast<XT>(ValueLoad<VT>::get(static_cast<const VT*>(a.values) + p[u]));
#pragma unroll
      for (int u = 0; u < kPer; ++u)
        if (ok[u]) {
          if constexpr (MERGE) merge_add(tb, static_cast<XT*>(a.Y), a.ldy, c[u], v[u] * s_dy[lo[u]]);
          else atomicAdd(static_cast<XT*>(a.Y) + static_cast<int64_t>(c[u]) * a.ldy, v[u] * s_dy[lo[u]]);
        }
    } else {
      XT xr[kPer];
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        if constexpr (MODE == kSddmmSaved) xr[u] = ld_stream(static_cast<const XT*>(a.X2) + p[u]);
        else xr[u] = static_cast<const XT*>(a.X2)[static_cast<int64_t>(c[u]) * a.ldx2];
      }
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        XT s = XT(0);
        s = s + s_dy[lo[u]] * xr[u];
        if (ok[u]) __builtin_nontemporal_store(s, static_cast<XT*>(a.Y) + p[u]);
      }
    }
  }
}

// One workgroup's share of a backward traversal: the bin and tile of this
// workgroup, then its split segment, stream tile or row groups.  With MERGE
// the scatter adds go through the workgroup's table `tb`.
template <typename VT, typename XT, int MODE, bool MERGE>
__device__ __forceinline__ void grad_tile(const ProdArgs& a, const MergeTab<XT>& tb) {
  const int b = blockIdx.x;
  int bi = 0;
  while (bi + 1 < a.nbins && b >= a.bins[bi + 1].blk_begin) ++bi;
  const BinDesc d = a.bins[bi];
  const int lb = b - d.blk_begin;
  const int tile = (a.flags & SPX_FLAG_NO_XCD_MAP) ? lb : xcd_tile(lb, d.nblk);
  const int t = threadIdx.x;
  if (d.lanes == 0) {  // one segment of a split row
    if (tile >= d.nrows) return;
    const int32_t s = a.seg_row[tile];
    const int32_t row = a.split_rows[s];
    const int32_t f = a.seg_first[s];
    const int32_t re = a.rowptr[row + 1];
    const int32_t p0 = a.rowptr[row] + (tile - f) * a.chunk;
    const int32_t p1 = min(p0 + a.chunk, re);
    visit_run<VT, XT, MODE, MERGE>(a, row, p0 + t, p1, kWG, tb);
    return;
  }
  if (d.lanes == SPX_LANES_STREAM && a.k == 1) {
    visit_stream<VT, XT, MODE, MERGE>(a, d, tile, tb);
    return;
  }
  // row groups of G lanes; a bin may give each group several rows (rpg),
  // taken in the same order as the product kernels.  A stream bin's 256 rows
  // per workgroup are served by 32 groups of 8 lanes, 8 rows each, so that
  // the per-nonzero loads and stores of a row are contiguous across lanes.
  const bool stream = (d.lanes == SPX_LANES_STREAM);
  const int G = stream ? 8 : d.lanes;
  const int rpg = stream ? 8 : d.rpg;  // 32 groups x 8 rows = the bin's 256 rows per workgroup
  const int ng = kWG / G;
  // every row id and range of the group first (independent loads), then the rows
  constexpr int kMaxRpg = 8;
  int32_t rows[kMaxRpg], q0[kMaxRpg], q1[kMaxRpg];
#pragma unroll
  for (int j = 0; j < kMaxRpg; ++j) {
    const int idx = (tile * rpg + j) * ng + t / G;
    rows[j] = -1;
    q0[j] = q1[j] = 0;
    if (j < rpg && idx < d.nrows) rows[j] = a.row_perm ? a.row_perm[d.row_begin + idx] : d.row_begin + idx;
  }
#pragma unroll
  for (int j = 0; j < kMaxRpg; ++j) {
    if (rows[j] < 0) continue;
    q0[j] = a.rowptr[rows[j]];
    q1[j] = a.rowptr[rows[j] + 1];
  }
#pragma unroll
  for (int j = 0; j < kMaxRpg; ++j)
    if (rows[j] >= 0) visit_run<VT, XT, MODE, MERGE>(a, rows[j], q0[j] + t % G, q1[j], G, tb);
}

template <typename VT, typename XT, int MODE>
__global__ __launch_bounds__(kWG) void k_grad(const ProdArgs a) {
  grad_tile<VT, XT, MODE, false>(a, MergeTab<XT>{nullptr, nullptr});
}

// A^T dy with k = 1 through the workgroup's merge table: the same traversal as
// k_grad<kScatterT>, then one atomic per distinct column of the workgroup.
template <typename VT, typename XT>
__global__ __launch_bounds__(kWG) void k_scatter_merged(const ProdArgs a) {
  __shared__ int32_t s_key[kMergeSlots];
  __shared__ XT s_val[kMergeSlots];
  const int t = threadIdx.x;
  for (int i = t; i < kMergeSlots; i += kWG) {
    s_key[i] = -1;
    s_val[i] = XT(0);
  }
  __syncthreads();
  // the traversal's only barriers (a stream tile's) are reached by the whole
  // workgroup, and every thread then returns here to the barrier below
  grad_tile<VT, XT, kScatterT, true>(a, MergeTab<XT>{s_key, s_val});
  __syncthreads();
  XT* y = static_cast<XT*>(a.Y);
  for (int i = t; i < kMergeSlots; i += kWG) {
    const int32_t c = s_key[i];
    if (c >= 0) atomicAdd(y + static_cast<int64_t>(c) * a.ldy, s_val[i]);
  }
}

template <typename XT>
__global__ void k_zero_2d(XT* __restrict__ p, int64_t rows, int32_t k, int64_t ld) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= rows * k) return;
  const int64_t r = i / k, c = i % k;
  p[r * ld + c] = XT(0);
}

}  // namespace

// Bin table for the per-nonzero traversals (bins_from_plan with KL = 1; the
// traversal serves stream bins with 8-lane row groups whatever their size).
static void grad_bins(const spx_plan* p, int32_t m, int32_t nnz, ProdArgs& a) {
  if (p) {
    bins_from_plan(p, a, 1, false);
  } else {
    const int32_t k = a.k;
    a.k = 1;
    bins_unbinned(m, nnz, 1, a);
    a.k = k;
  }
}

spx_status launch_scatter_t(ProdArgs& a, const spx_plan* plan, int32_t m, int32_t n, int32_t nnz,
                            int vt, int xt, hipStream_t st) {
  // zero dX (n x k, ld = a.ldy) with a kernel (graph safe, no memset)
  const int64_t total = static_cast<int64_t>(n) * a.k;
  if (total > 0) {
    const unsigned g = static_cast<unsigned>((total + 255) / 256);
    if (xt == SPX_F64) k_zero_2d<double><<<g, 256, 0, st>>>(static_cast<double*>(a.Y), n, a.k, a.ldy);
    else k_zero_2d<float><<<g, 256, 0, st>>>(static_cast<float*>(a.Y), n, a.k, a.ldy);
    SPX_LAUNCHED("k_zero_2d");
  }
  grad_bins(plan, m, nnz, a);
  int64_t grid = 0;
  for (int i = 0; i < a.nbins; ++i) grid = a.bins[i].blk_begin + a.bins[i].nblk;
  if (grid == 0) return SPX_OK;
  const unsigned g = static_cast<unsigned>(grid);
  if (a.k == 1) {  // contributions merged per workgroup first
    if (vt == SPX_F64 && xt == SPX_F64) k_scatter_merged<double, double><<<g, kWG, 0, st>>>(a);
    else if (vt == SPX_F32 && xt == SPX_F32) k_scatter_merged<float, float><<<g, kWG, 0, st>>>(a);
    else if (vt == SPX_BF16 && xt == SPX_F32) k_scatter_merged<uint16_t, float><<<g, kWG, 0, st>>>(a);
    else return fail(SPX_ERR_UNSUPPORTED, "csr_spmv_t: unsupported dtype pair");
    SPX_LAUNCHED("k_scatter_merged");
    return SPX_OK;
  }
  if (vt == SPX_F64 && xt == SPX_F64) k_grad<double, double, kScatterT><<<g, kWG, 0, st>>>(a);
  else if (vt == SPX_F32 && xt == SPX_F32) k_grad<float, float, kScatterT><<<g, kWG, 0, st>>>(a);
  else if (vt == SPX_BF16 && xt == SPX_F32) k_grad<uint16_t, float, kScatterT><<<g, kWG, 0, st>>>(a);
  else return fail(SPX_ERR_UNSUPPORTED, "csr_spmv_t: unsupported dtype pair");
  SPX_LAUNCHED("k_grad<scatter>");
  return SPX_OK;
}

spx_status launch_sddmm(ProdArgs& a, const spx_plan* plan, int32_t m, int32_t nnz, int dt, bool saved,
                        hipStream_t st) {
  grad_bins(plan, m, nnz, a);
  int64_t grid = 0;
  for (int i = 0; i < a.nbins; ++i) grid = a.bins[i].blk_begin + a.bins[i].nblk;
  if (grid == 0) return SPX_OK;
  const unsigned g = static_cast<unsigned>(grid);
  if (saved && a.k != 1) return fail(SPX_ERR_INVALID, "csr_sddmm_saved: k must be 1");
  if (dt == SPX_F64 && saved) k_grad<double, double, kSddmmSaved><<<g, kWG, 0, st>>>(a);
  else if (dt == SPX_F32 && saved) k_grad<float, float, kSddmmSaved><<<g, kWG, 0, st>>>(a);
  else if (dt == SPX_F64) k_grad<double, double, kSddmm><<<g, kWG, 0, st>>>(a);
  else if (dt == SPX_F32) k_grad<float, float, kSddmm><<<g, kWG, 0, st>>>(a);
  else return fail(SPX_ERR_UNSUPPORTED, "csr_sddmm: dtype must be F64 or F32");
  SPX_LAUNCHED(saved ? "k_grad<sddmm_saved>" : "k_grad<sddmm>");
  return SPX_OK;
}

}  // namespace spx

// ------------------------------------------------------------------ values in CSC order
// values_csc[q] = values[perm[q]] without the random reads of a gather (each
// would fetch a whole line for 2-8 useful bytes).  A one-time map groups the
// nonzeros by block of SPX_CSC_BLOCK consecutive CSC positions: dest[p] is
// p's slot in a staging array whose block b holds, in ascending p, the
// nonzeros whose CSC position lies in block b, and local[i] is the position
// inside block b of staging slot i.  Pass 1 streams values and writes each to
// dest[p]: a workgroup's writes to one block form a contiguous run that its
// neighbours (same XCD) continue, so lines fill in L2.  Pass 2 reads one block
// of staging coalesced, reorders it in LDS by local[], and writes it out
// coalesced.
namespace spx {
namespace {

__global__ void k_inv_perm(const int32_t* __restrict__ perm, int32_t nnz, int32_t* __restrict__ pos) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nnz) return;
  const int32_t p = perm[q];
  if (p >= 0 && p < nnz) pos[p] = static_cast<int32_t>(q);
}

__global__ void k_block_keys(const int32_t* __restrict__ pos, int32_t nnz, uint32_t* __restrict__ keys,
                             int32_t* __restrict__ vals) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  keys[p] = static_cast<uint32_t>(pos[p]) / SPX_CSC_BLOCK;
  vals[p] = static_cast<int32_t>(p);
}

// sorted[i] = the nonzero p at staging slot i (stable by p within a block)
__global__ void k_fill_map(const int32_t* __restrict__ sorted, const int32_t* __restrict__ pos, int32_t nnz,
                           int32_t* __restrict__ dest, uint16_t* __restrict__ local) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const int32_t p = sorted[i];
  dest[p] = static_cast<int32_t>(i);
  local[i] = static_cast<uint16_t>(static_cast<uint32_t>(pos[p]) % SPX_CSC_BLOCK);
}

// Pass 1 tiles are XCD-contiguous (grid a multiple of 8): XCD j streams one
// contiguous eighth of the nonzeros, so its part of every block's run is
// contiguous and the run's lines fill in that XCD's L2 instead of being
// written piecemeal from all eight.
constexpr int kStagePerThread = 8;

template <typename T>
__global__ __launch_bounds__(kWG) void k_to_staging(const T* __restrict__ values, const int32_t* __restrict__ dest,
                                                    int32_t nnz, T* __restrict__ staging) {
  const int64_t base = static_cast<int64_t>(xcd_tile(blockIdx.x, gridDim.x)) * (kWG * kStagePerThread);
  int32_t d[kStagePerThread];
  T v[kStagePerThread];
#pragma unroll
  for (int u = 0; u < kStagePerThread; ++u) {
    const int64_t p = base + u * kWG + threadIdx.x;
    d[u] = (p < nnz) ? ld_stream(dest + p) : -1;
    v[u] = (p < nnz) ? ld_stream(values + p) : T(0);
  }
#pragma unroll
  for (int u = 0; u < kStagePerThread; ++u)
    if (d[u] >= 0 && d[u] < nnz) staging[d[u]] = v[u];
}

// Pass 1 with the workgroup's nonzeros grouped by destination block first
// (tiles of 4,096 FP32 nonzeros, 32 KB of LDS plus the block-count table
// sized to the matrix; twice the tile halved the occupancy and ran 25 %
// slower):
// each loads kTile of them, counts them per block (LDS atomics; the rank an
// atomic returns only places an element inside its block's LDS segment), and
// stores them from LDS in block order, so that the lanes of one store write
// the consecutive slots of a few blocks' runs instead of 64 scattered slots.
// Every element still goes to dest[p]: the order inside LDS changes which
// lane stores it, never where.  Needs at most kMaxBlocks blocks.
constexpr int kMaxBlocks = 4096;

template <typename T>
constexpr int sort_tile() {
  return sizeof(T) >= 8 ? 2048 : 4096;
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_to_staging_sorted(const T* __restrict__ values,
                                                           const int32_t* __restrict__ dest, int32_t nnz,
                                                           int32_t nblocks, T* __restrict__ staging) {
  constexpr int kTile = sort_tile<T>();
  constexpr int kPer = kTile / kWG;
  extern __shared__ int32_t s_cnt[];  // nblocks entries (dynamic LDS, sized by the launch)
  __shared__ int32_t s_dest[kTile];
  __shared__ T s_val[kTile];
  __shared__ int32_t s_wsum[kWG / kWave];
  const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
  const int64_t base = static_cast<int64_t>(xcd_tile(blockIdx.x, gridDim.x)) * kTile;
  for (int i = t; i < nblocks; i += kWG) s_cnt[i] = 0;
  __syncthreads();
  int32_t d[kPer], rank[kPer];
  T v[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int64_t p = base + u * kWG + t;
    const bool ok = p < nnz;
    d[u] = ok ? ld_stream(dest + p) : -1;
    v[u] = ok ? ld_stream(values + p) : T(0);
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    rank[u] = -1;
    if (d[u] >= 0 && d[u] < nnz) rank[u] = atomicAdd(&s_cnt[d[u] / SPX_CSC_BLOCK], 1);
  }
  __syncthreads();
  // exclusive prefix of the block counts (thread t owns blocks [t * per, (t + 1) * per))
  const int per = (nblocks + kWG - 1) / kWG;
  int32_t mine = 0;
  for (int i = 0; i < per; ++i) {
    const int b = t * per + i;
    if (b < nblocks) mine += s_cnt[b];
  }
  int32_t inc = mine;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t u = __shfl_up(inc, off, kWave);
    if (lane >= off) inc += u;
  }
  if (lane == kWave - 1) s_wsum[w] = inc;
  __syncthreads();
  int32_t run = inc - mine;
  int32_t placed = 0;  // elements with a valid destination, all placed below
  for (int i = 0; i < kWG / kWave; ++i) {
    if (i < w) run += s_wsum[i];
    placed += s_wsum[i];
  }
  for (int i = 0; i < per; ++i) {
    const int b = t * per + i;
    if (b < nblocks) {
      const int32_t c = s_cnt[b];
      s_cnt[b] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    if (rank[u] < 0) continue;
    const int32_t q = s_cnt[d[u] / SPX_CSC_BLOCK] + rank[u];
    s_dest[q] = d[u];
    s_val[q] = v[u];
  }
  __syncthreads();
  for (int32_t i = t; i < placed; i += kWG) {
    const int32_t dd = s_dest[i];
    if (dd >= 0 && dd < nnz) staging[dd] = s_val[i];
  }
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_from_staging(const T* __restrict__ staging,
                                                      const uint16_t* __restrict__ local, int32_t nnz,
                                                      T* __restrict__ out) {
  constexpr int PER = SPX_CSC_BLOCK / kWG;
  static_assert(SPX_CSC_BLOCK % kWG == 0 && SPX_CSC_BLOCK <= 65536, "block of 16-bit positions");
  __shared__ T blk[SPX_CSC_BLOCK];
  const int64_t b0 = static_cast<int64_t>(blockIdx.x) * SPX_CSC_BLOCK;
  const int64_t left = static_cast<int64_t>(nnz) - b0;
  const int32_t cnt = static_cast<int32_t>(left < SPX_CSC_BLOCK ? left : SPX_CSC_BLOCK);
  // all of a thread's loads are issued before the first LDS store
  uint16_t l[PER];
  T v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int32_t i = u * kWG + threadIdx.x;
    l[u] = (i < cnt) ? ld_stream(local + b0 + i) : static_cast<uint16_t>(0xffff);
    v[u] = (i < cnt) ? ld_stream(staging + b0 + i) : T(0);
  }
#pragma unroll
  for (int u = 0; u < PER; ++u)
    if (l[u] < cnt) blk[l[u]] = v[u];
  __syncthreads();
  for (int32_t i = threadIdx.x; i < cnt; i += kWG) __builtin_nontemporal_store(blk[i], out + b0 + i);
}

unsigned grid256(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

int bits_for(int64_t v) {
  int b = 1;
  while ((int64_t(1) << b) <= v) ++b;
  return b;
}

}  // namespace
}  // namespace spx

using namespace spx;

extern "C" spx_status csr_csc_value_map_workspace_bytes(int32_t nnz, size_t* bytes) {
  if (!bytes || nnz < 0) return fail(SPX_ERR_INVALID, "csr_csc_value_map_workspace_bytes: bad argument");
  const size_t n = static_cast<size_t>(nnz > 0 ? nnz : 1);
  *bytes = 3 * align_up(n * 4) + radix_workspace_bytes(nnz, 4);
  return SPX_OK;
}

extern "C" spx_status csr_csc_value_map(int32_t nnz, const int32_t* perm, int32_t* dest, uint16_t* local,
                                        void* workspace, size_t ws_bytes, void* stream) {
  if (nnz < 0) return fail(SPX_ERR_INVALID, "csr_csc_value_map: negative size");
  {
    const spx_status s_nnz = check_nnz(nnz, "csr_csc_value_map");
    if (s_nnz != SPX_OK) return s_nnz;
  }
  if (nnz == 0) return SPX_OK;
  if (!perm || !dest || !local) return fail(SPX_ERR_INVALID, "csr_csc_value_map: null pointer");
  size_t need = 0;
  csr_csc_value_map_workspace_bytes(nnz, &need);
  if (!workspace || ws_bytes < need)
    return fail(SPX_ERR_WORKSPACE, "csr_csc_value_map: workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t st = as_stream(stream);
  char* w = static_cast<char*>(workspace);
  const size_t n4 = align_up(static_cast<size_t>(nnz) * 4);
  int32_t* pos = reinterpret_cast<int32_t*>(w);
  uint32_t* keys = reinterpret_cast<uint32_t*>(w + n4);
  int32_t* vals = reinterpret_cast<int32_t*>(w + 2 * n4);
  void* rws = w + 3 * n4;
  k_inv_perm<<<grid256(nnz), 256, 0, st>>>(perm, nnz, pos);
  SPX_LAUNCHED("k_inv_perm");
  k_block_keys<<<grid256(nnz), 256, 0, st>>>(pos, nnz, keys, vals);
  SPX_LAUNCHED("k_block_keys");
  const spx_status s = radix_sort_u32(keys, vals, nnz, bits_for((static_cast<int64_t>(nnz) - 1) / SPX_CSC_BLOCK), rws, st);
  if (s != SPX_OK) return s;
  k_fill_map<<<grid256(nnz), 256, 0, st>>>(vals, pos, nnz, dest, local);
  SPX_LAUNCHED("k_fill_map");
  return SPX_OK;
}

namespace spx {
namespace {

spx_status values_to_csc_impl(const char* who, int32_t nnz, const int32_t* dest, const uint16_t* local,
                              const void* values, spx_dtype vtype, void* staging, void* values_csc,
                              hipStream_t st) {
  const unsigned nb = static_cast<unsigned>((static_cast<int64_t>(nnz) + SPX_CSC_BLOCK - 1) / SPX_CSC_BLOCK);
  const int64_t tiles = (static_cast<int64_t>(nnz) + kWG * kStagePerThread - 1) / (kWG * kStagePerThread);
  const unsigned g1 = static_cast<unsigned>((tiles + 7) / 8 * 8);
  const int32_t nblocks = static_cast<int32_t>(nb);
#define SPX_TO_CSC(T)                                                                                    \
  if (nblocks <= kMaxBlocks) {                                                                           \
    const int64_t st_tiles = (static_cast<int64_t>(nnz) + sort_tile<T>() - 1) / sort_tile<T>();         \
    const unsigned gs = static_cast<unsigned>((st_tiles + 7) / 8 * 8);                                   \
    k_to_staging_sorted<T><<<gs, kWG, sizeof(int32_t) * nblocks, st>>>(static_cast<const T*>(values), dest, \
                                                                     nnz, nblocks,                        \
                                                static_cast<T*>(staging));                               \
  } else {                                                                                               \
    k_to_staging<T><<<g1, kWG, 0, st>>>(static_cast<const T*>(values), dest, nnz, static_cast<T*>(staging)); \
  }                                                                                                      \
  SPX_LAUNCHED("k_to_staging");                                                                          \
  k_from_staging<T><<<nb, kWG, 0, st>>>(static_cast<const T*>(staging), local, nnz, static_cast<T*>(values_csc)); \
  SPX_LAUNCHED("k_from_staging");                                                                        \
  return SPX_OK;
  if (vtype == SPX_F64) { SPX_TO_CSC(double) }
  if (vtype == SPX_F32) { SPX_TO_CSC(float) }
  if (vtype == SPX_BF16) { SPX_TO_CSC(uint16_t) }
#undef SPX_TO_CSC
  return fail(SPX_ERR_UNSUPPORTED, "%s: vtype %d", who, vtype);
}

spx_status values_to_csc_args(const char* who, int32_t nnz, const int32_t* dest, const uint16_t* local,
                              const void* values, void* values_csc) {
  if (nnz < 0) return fail(SPX_ERR_INVALID, "%s: negative size", who);
  const spx_status s_nnz = check_nnz(nnz, who);
  if (s_nnz != SPX_OK) return s_nnz;
  if (nnz > 0 && (!dest || !local || !values || !values_csc))
    return fail(SPX_ERR_INVALID, "%s: null pointer", who);
  return SPX_OK;
}

size_t value_bytes(spx_dtype vt) { return vt == SPX_F64 ? 8 : vt == SPX_F32 ? 4 : vt == SPX_BF16 ? 2 : 0; }

// Staging of csr_values_to_csc_noalloc: a fixed device array that every GPU
// the library runs on holds until the process ends.  Its name is a host-side
// stand-in in host code; kernels get the device address that
// hipGetSymbolAddress returns for the current device, resolved once per
// device (each device has its own copy at its own address).
__device__ __align__(256) unsigned char scratch[SPX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

spx_status scratch_for_current_device(void** out) {
  int dev = -1;
  SPX_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(SPX_ERR_UNSUPPORTED, "scratch: device %d beyond the %d the library tracks", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(SPX_ERR_HIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SPX_OK;
}

}  // namespace
}  // namespace spx

extern "C" spx_status csr_values_to_csc(int32_t nnz, const int32_t* dest, const uint16_t* local,
                                        const void* values, spx_dtype vtype, void* staging, void* values_csc,
                                        void* stream) {
  const spx_status s = values_to_csc_args("csr_values_to_csc", nnz, dest, local, values, values_csc);
  if (s != SPX_OK) return s;
  if (nnz == 0) return SPX_OK;
  if (!staging) return fail(SPX_ERR_INVALID, "csr_values_to_csc: null pointer");
  return values_to_csc_impl("csr_values_to_csc", nnz, dest, local, values, vtype, staging, values_csc,
                            as_stream(stream));
}

extern "C" spx_status csr_values_to_csc_noalloc(int32_t nnz, const int32_t* dest, const uint16_t* local,
                                                const void* values, spx_dtype vtype, void* values_csc,
                                                void* stream) {
  const char* who = "csr_values_to_csc_noalloc";
  spx_status s = values_to_csc_args(who, nnz, dest, local, values, values_csc);
  if (s != SPX_OK) return s;
  const size_t vb = value_bytes(vtype);
  if (vb == 0) return fail(SPX_ERR_UNSUPPORTED, "%s: vtype %d", who, vtype);
  const size_t need = static_cast<size_t>(nnz) * vb;
  if (need > static_cast<size_t>(SPX_NOALLOC_SCRATCH_BYTES))
    return fail(SPX_ERR_UNSUPPORTED,
                "%s: nnz=%d of %zu-byte values needs %zu bytes of staging, above SPX_NOALLOC_SCRATCH_BYTES=%d "
                "(use csr_values_to_csc with a caller staging buffer)",
                who, nnz, vb, need, SPX_NOALLOC_SCRATCH_BYTES);
  if (nnz == 0) return SPX_OK;
  void* staging = nullptr;
  s = scratch_for_current_device(&staging);
  if (s != SPX_OK) return s;
  return values_to_csc_impl(who, nnz, dest, local, values, vtype, staging, values_csc, as_stream(stream));
}
