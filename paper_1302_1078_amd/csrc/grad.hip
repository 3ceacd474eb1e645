// grad.hip -- per-nonzero traversals for the backward of y = A(values) x:
//   mode kScatterT: dX[colind[p], :] += values[p] * dY[row(p), :] (atomic)
//   mode kSddmm:    out[p] = sum_t dY[row(p), t] * X[colind[p], t]
// Rows are visited through the same bin table as the products (row groups of
// G lanes, or one workgroup per segment of a split row); no cross-lane
// reduction is needed because every nonzero is independent.
#include "device.hpp"
#include "internal.hpp"

namespace spx {

namespace {

enum { kScatterT = 0, kSddmm = 1 };

template <typename VT, typename XT, int MODE>
__device__ __forceinline__ void visit(const ProdArgs& a, int32_t row, int32_t p) {
  const int32_t c = ld_stream(a.colind + p);
  const XT* dy = static_cast<const XT*>(a.X) + static_cast<int64_t>(row) * a.ldx;
  if constexpr (MODE == kScatterT) {
    const XT v = static_cast<XT>(ValueLoad<VT>::get(static_cast<const VT*>(a.values) + p));
    XT* dst = static_cast<XT*>(a.Y) + static_cast<int64_t>(c) * a.ldy;
    for (int t = 0; t < a.k; ++t) atomicAdd(dst + t, v * dy[t]);
  } else {
    const XT* xr = static_cast<const XT*>(a.X2) + static_cast<int64_t>(c) * a.ldx2;
    XT s = XT(0);
    for (int t = 0; t < a.k; ++t) s = s + dy[t] * xr[t];
    __builtin_nontemporal_store(s, static_cast<XT*>(a.Y) + p);
  }
}

template <typename VT, typename XT, int MODE>
__global__ __launch_bounds__(kWG) void k_grad(const ProdArgs a) {
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
    for (int32_t p = p0 + t; p < p1; p += kWG) visit<VT, XT, MODE>(a, row, p);
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
  for (int j = 0; j < rpg; ++j) {
    const int idx = (tile * rpg + j) * ng + t / G;
    if (idx >= d.nrows) continue;
    const int32_t row = a.row_perm ? a.row_perm[d.row_begin + idx] : d.row_begin + idx;
    const int32_t p1 = a.rowptr[row + 1];
    for (int32_t p = a.rowptr[row] + t % G; p < p1; p += G) visit<VT, XT, MODE>(a, row, p);
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
  if (vt == SPX_F64 && xt == SPX_F64) k_grad<double, double, kScatterT><<<g, kWG, 0, st>>>(a);
  else if (vt == SPX_F32 && xt == SPX_F32) k_grad<float, float, kScatterT><<<g, kWG, 0, st>>>(a);
  else if (vt == SPX_BF16 && xt == SPX_F32) k_grad<uint16_t, float, kScatterT><<<g, kWG, 0, st>>>(a);
  else return fail(SPX_ERR_UNSUPPORTED, "csr_spmv_t: unsupported dtype pair");
  SPX_LAUNCHED("k_grad<scatter>");
  return SPX_OK;
}

spx_status launch_sddmm(ProdArgs& a, const spx_plan* plan, int32_t m, int32_t nnz, int dt,
                        int64_t ldx, hipStream_t st) {
  grad_bins(plan, m, nnz, a);
  (void)ldx;
  int64_t grid = 0;
  for (int i = 0; i < a.nbins; ++i) grid = a.bins[i].blk_begin + a.bins[i].nblk;
  if (grid == 0) return SPX_OK;
  const unsigned g = static_cast<unsigned>(grid);
  if (dt == SPX_F64) k_grad<double, double, kSddmm><<<g, kWG, 0, st>>>(a);
  else if (dt == SPX_F32) k_grad<float, float, kSddmm><<<g, kWG, 0, st>>>(a);
  else return fail(SPX_ERR_UNSUPPORTED, "csr_sddmm: dtype must be F64 or F32");
  SPX_LAUNCHED("k_grad<sddmm>");
  return SPX_OK;
}

}  // namespace spx
