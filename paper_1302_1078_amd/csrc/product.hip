// product.hip -- fused, row-binned CSR products on gfx950:
//   y <- A x  (SpMV, paper Sec. 3)        and        Y <- A X  (SpMM, Sec. 5)
// plus the same traversal for the transpose gather (CSC index), an SpMV
// variant that also stores each gathered x[colind[p]] at position p for the
// gradient with respect to the values, and an SpMV variant that reads the
// most-used columns' x entries from a compact copy (hot x, hot.hip).
//
// One launch covers every bin of a plan.  Workgroups [bins[i].blk_begin,
// bins[i+1].blk_begin) serve bin i; long-row bins come first so that their
// workgroups start early.  Inside a bin, a row is served by a group of
// S slots x KL lanes: the KL lanes cover the k columns of one X row (VEC
// elements each, one 16-byte load per lane when VEC > 1), the S slots walk
// the row's nonzeros with stride S.  SpMV is the case KL = VEC = 1.
//   - colind / values are streamed with non-temporal loads, x / X rows are
//     gathered through L2, y / Y rows are written with non-temporal stores
//     (the analogue of the paper's no-read, non-globally-ordered stores).
//   - Each lane keeps U = 4 independent nonzeros in flight per iteration: the
//     x gather is latency bound (paper Sec. 4.2), so memory-level parallelism
//     is what buys throughput.
//   - Partial sums of the S slots are combined with DPP / swizzle exchanges
//     (and LDS across the 4 waves of a workgroup-per-row bin).
//   - A split bin cuts each long row into segments of `chunk` nonzeros, one
//     workgroup per segment.  Segment partials go to workspace; the last
//     workgroup to arrive (agent-scope counter) sums them in segment order and
//     resets the counter, so results are deterministic and no second launch or
//     memset is needed.
// FP32/BF16 values with FP32 vectors accumulate in FP32; rows longer than
// kahan_len use error-free transforms (TwoProduct + TwoSum) per lane and an
// FP64 cross-lane / cross-segment reduction, rounded to FP32 once at the end.
#include "product_impl.hpp"

namespace spx {

namespace {

using namespace prod;

// MR: instantiate the multi-row path of short-row bins.  It costs VGPRs in
// the whole fused kernel, so launches whose bins do not use it run the MR =
// false variant (higher occupancy).
template <class C, bool MR>
__global__ __launch_bounds__(kWG) void k_product(const ProdArgs a) {
  const int b = blockIdx.x;
  int bi = 0;
  while (bi + 1 < a.nbins && b >= a.bins[bi + 1].blk_begin) ++bi;
  const BinDesc d = a.bins[bi];
  const int lb = b - d.blk_begin;
  const int tile = (a.flags & SPX_FLAG_NO_XCD_MAP) ? lb : xcd_tile(lb, d.nblk);
  switch (d.lanes + (d.rpg > 1 ? 1000 : 0)) {
    case 1: do_rows<C, 1, 1>(a, d, tile); break;
    case 2: do_rows<C, 2, 1>(a, d, tile); break;
    case 4: do_rows<C, 4, 1>(a, d, tile); break;
    case 8: do_rows<C, 8, 1>(a, d, tile); break;
    case 16: do_rows<C, 16, 1>(a, d, tile); break;
    case 32: do_rows<C, 32, 1>(a, d, tile); break;
    case 64: do_rows<C, 64, 1>(a, d, tile); break;
    case 256: do_rows<C, 256, 1>(a, d, tile); break;
    case 1001:
      if constexpr (MR && C::KL == 1 && C::VEC == 1) do_rows<C, 1, 4>(a, d, tile);
      else do_rows<C, 1, 1>(a, d, tile);
      break;
    case 1002:
      if constexpr (MR && C::KL == 1 && C::VEC == 1) do_rows<C, 2, 4>(a, d, tile);
      else do_rows<C, 2, 1>(a, d, tile);
      break;
    case 1004:
      if constexpr (MR && C::KL == 1 && C::VEC == 1) do_rows<C, 4, 4>(a, d, tile);
      else do_rows<C, 4, 1>(a, d, tile);
      break;
    case 1008:
      if constexpr (MR && C::KL == 1 && C::VEC == 1) do_rows<C, 8, 4>(a, d, tile);
      else do_rows<C, 8, 1>(a, d, tile);
      break;
    case 1016:
      if constexpr (MR && C::KL == 1 && C::VEC == 1) do_rows<C, 16, 4>(a, d, tile);
      else do_rows<C, 16, 1>(a, d, tile);
      break;
    case 1032:
      if constexpr (MR && C::KL == 1 && C::VEC == 1) do_rows<C, 32, 4>(a, d, tile);
      else do_rows<C, 32, 1>(a, d, tile);
      break;
    case SPX_LANES_STREAM:
      if constexpr (C::KL == 1 && C::VEC == 1) do_stream<C>(a, d, tile);
      else do_rows<C, 1, 1>(a, d, tile);
      break;
    default: do_split<C>(a, d, tile); break;
  }
}

// Dynamic LDS that lets at most `occ` workgroups of kernel `fn` share a CU
// (each workgroup then holds more than 1/(occ+1) of the CU's LDS).
spx_status occupancy_lds(const void* fn, int occ, size_t* dyn) {
  int dev = 0, per_cu = 0, per_block = 0;
  SPX_HIP(hipGetDevice(&dev));
  SPX_HIP(hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev));
  SPX_HIP(hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  hipFuncAttributes at;
  SPX_HIP(hipFuncGetAttributes(&at, fn));
  const size_t want = static_cast<size_t>(per_cu) / occ;
  if (want > static_cast<size_t>(per_block) || want < at.sharedSizeBytes)
    return fail(SPX_ERR_UNSUPPORTED,
                "occupancy=%d needs %zu B of LDS per workgroup (static %zu, device limit %d per "
                "workgroup, %d per CU)",
                occ, want, static_cast<size_t>(at.sharedSizeBytes), per_block, per_cu);
  *dyn = want - at.sharedSizeBytes;
  SPX_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(*dyn)));
  return SPX_OK;
}

template <class C, bool MR>
spx_status launch_k(const ProdArgs& a, unsigned grid, hipStream_t st) {
  size_t dyn = 0;
  if (a.occupancy > 0) {
    const spx_status s = occupancy_lds(reinterpret_cast<const void*>(&k_product<C, MR>), a.occupancy, &dyn);
    if (s != SPX_OK) return s;
  }
  k_product<C, MR><<<grid, kWG, dyn, st>>>(a);
  SPX_LAUNCHED("k_product");
  return SPX_OK;
}

template <typename VT, typename XT, int VECMAX>
spx_status launch_vt(ProdArgs& a, int kl, int vec, unsigned grid, hipStream_t st) {
  bool mr = false;
  for (int i = 0; i < a.nbins; ++i) mr = mr || (a.bins[i].rpg > 1);
#define SPX_CASE(KL_, VEC_)                                                   \
  if (kl == KL_ && vec == VEC_) {                                             \
    if (KL_ == 1 && VEC_ == 1 && mr)                                          \
      return launch_k<Cfg<VT, XT, KL_, VEC_>, true>(a, grid, st);             \
    return launch_k<Cfg<VT, XT, KL_, VEC_>, false>(a, grid, st);              \
  }
  SPX_CASE(1, 1) SPX_CASE(2, 1) SPX_CASE(4, 1) SPX_CASE(8, 1) SPX_CASE(16, 1) SPX_CASE(32, 1)
  SPX_CASE(1, VECMAX) SPX_CASE(2, VECMAX) SPX_CASE(4, VECMAX) SPX_CASE(8, VECMAX)
  SPX_CASE(16, VECMAX) SPX_CASE(32, VECMAX)
#undef SPX_CASE
  return fail(SPX_ERR_UNSUPPORTED, "no product kernel for KL=%d VEC=%d", kl, vec);
}

// SpMV that keeps its gathered operand (a.xsave): the KL = VEC = 1 kernel
// compiled with the stores, so that the plain product carries none of them.
template <typename VT, typename XT>
spx_status launch_save(ProdArgs& a, unsigned grid, hipStream_t st) {
  bool mr = false;
  for (int i = 0; i < a.nbins; ++i) mr = mr || (a.bins[i].rpg > 1);
  if (mr) return launch_k<Cfg<VT, XT, 1, 1, true>, true>(a, grid, st);
  return launch_k<Cfg<VT, XT, 1, 1, true>, false>(a, grid, st);
}

// SpMV with hot x (a.X2: the compact hot entries).
template <typename VT, typename XT>
spx_status launch_hot(ProdArgs& a, unsigned grid, hipStream_t st) {
  bool mr = false;
  for (int i = 0; i < a.nbins; ++i) mr = mr || (a.bins[i].rpg > 1);
  if (mr) return launch_k<Cfg<VT, XT, 1, 1, false, true>, true>(a, grid, st);
  return launch_k<Cfg<VT, XT, 1, 1, false, true>, false>(a, grid, st);
}

}  // namespace

spx_status launch_product_hot(ProdArgs& a, int vt, int xt, hipStream_t st) {
  if (a.k != 1 || !a.X2 || a.ldx2 <= 0) return fail(SPX_ERR_INVALID, "hot x: k must be 1 with hot entries set");
  int64_t grid = 0;
  for (int i = 0; i < a.nbins; ++i) grid = a.bins[i].blk_begin + a.bins[i].nblk;
  if (grid == 0) return SPX_OK;
  if (grid > 0x7fffffff) return fail(SPX_ERR_UNSUPPORTED, "grid too large");
  const unsigned g = static_cast<unsigned>(grid);
  if (vt == SPX_F64 && xt == SPX_F64) return launch_hot<double, double>(a, g, st);
  if (vt == SPX_F32 && xt == SPX_F32) return launch_hot<float, float>(a, g, st);
  if (vt == SPX_BF16 && xt == SPX_F32) return launch_hot<uint16_t, float>(a, g, st);
  return fail(SPX_ERR_UNSUPPORTED, "unsupported value/vector dtype pair (%d, %d)", vt, xt);
}

spx_status launch_product_save(ProdArgs& a, int vt, int xt, hipStream_t st) {
  if (a.k != 1 || !a.xsave) return fail(SPX_ERR_INVALID, "saved gather: k must be 1 and xsave set");
  int64_t grid = 0;
  for (int i = 0; i < a.nbins; ++i) grid = a.bins[i].blk_begin + a.bins[i].nblk;
  if (grid == 0) return SPX_OK;
  if (grid > 0x7fffffff) return fail(SPX_ERR_UNSUPPORTED, "grid too large");
  const unsigned g = static_cast<unsigned>(grid);
  if (vt == SPX_F64 && xt == SPX_F64) return launch_save<double, double>(a, g, st);
  if (vt == SPX_F32 && xt == SPX_F32) return launch_save<float, float>(a, g, st);
  if (vt == SPX_BF16 && xt == SPX_F32) return launch_save<uint16_t, float>(a, g, st);
  return fail(SPX_ERR_UNSUPPORTED, "unsupported value/vector dtype pair (%d, %d)", vt, xt);
}

spx_status launch_product(ProdArgs& a, int vt, int xt, int kl, int vec, hipStream_t st) {
  int64_t grid = 0;
  for (int i = 0; i < a.nbins; ++i) grid = a.bins[i].blk_begin + a.bins[i].nblk;
  if (grid == 0) return SPX_OK;
  if (grid > 0x7fffffff) return fail(SPX_ERR_UNSUPPORTED, "grid too large");
  const unsigned g = static_cast<unsigned>(grid);
  if (vt == SPX_F64 && xt == SPX_F64) return launch_vt<double, double, 2>(a, kl, vec, g, st);
  if (vt == SPX_F32 && xt == SPX_F32) return launch_vt<float, float, 4>(a, kl, vec, g, st);
  if (vt == SPX_BF16 && xt == SPX_F32) return launch_vt<uint16_t, float, 4>(a, kl, vec, g, st);
  return fail(SPX_ERR_UNSUPPORTED, "unsupported value/vector dtype pair (%d, %d)", vt, xt);
}

}  // namespace spx
