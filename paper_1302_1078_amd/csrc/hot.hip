// hot.hip -- hot x for SpMV: the x entries of the most-used columns packed
// together (the x reuse the paper attributes to the caches and to the
// nonzeros that share a cache line, Sec. 4.1-4.2).  On a matrix whose column
// use is skewed a few thousand columns carry a large share of the nonzeros
// (on the 1M-row power-law workload the top 4,096 carry 39 %), but in x each
// of them has a 128-byte line to itself, so the caches hold few of them.
// Packed 16 (FP64) or 32 (FP32) to a line they stay in L1 / L2, and their
// gathers stop being L1 misses, the resource the SpMV gather is bound by.
//
// csr_plan_attach_hot_x ranks the columns by use (csr_degree_order), keeps
// the first `hot` as hot_cols and writes the plan's own copy of the column
// indices, colind_hot, with every hot column replaced by ~slot.  A product
// through the plan first gathers x[hot_cols[s]] into the plan's x_hot (one
// small kernel), then reads hot entries from x_hot.  Each row's products and
// their order are unchanged, so results are bitwise those of the plan
// without hot x.  (Copying x_hot into LDS per workgroup was measured too: it
// only paid for 1,024 entries, since every workgroup repeats the copy.)
#include "internal.hpp"

extern "C" spx_status csr_degree_order_workspace_bytes(int32_t n, int32_t nnz, size_t* bytes);
extern "C" spx_status csr_degree_order(int32_t n, int32_t nnz, const int32_t* colind, int32_t* perm,
                                       void* workspace, size_t ws_bytes, void* stream);

namespace spx {
namespace {

constexpr int32_t kMaxHot = 1 << 20;

__global__ void k_hot_slots(const int32_t* __restrict__ perm, int32_t n, int32_t hot, int32_t* __restrict__ slot,
                            int32_t* __restrict__ hot_cols) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // perm[r] is the column of rank r (most used first)
  const int32_t c = perm[i];
  slot[c] = (i < hot) ? static_cast<int32_t>(i) : -1;
  if (i < hot) hot_cols[i] = c;
}

__global__ void k_hot_colind(const int32_t* __restrict__ colind, int32_t nnz, const int32_t* __restrict__ slot,
                             int32_t* __restrict__ out) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const int32_t c = colind[p];
  const int32_t s = slot[c];
  out[p] = (s >= 0) ? ~s : c;
}

template <typename XT>
__global__ void k_hot_gather(const XT* __restrict__ x, const int32_t* __restrict__ hot_cols, int32_t hot,
                             XT* __restrict__ x_hot) {
  const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < hot) x_hot[i] = x[hot_cols[i]];
}

struct HotWs {
  int32_t* colind_hot;
  int32_t* hot_cols;
  void* x_hot;
  int32_t* perm;
  int32_t* slot;
  void* deg;
  size_t deg_bytes;
};

HotWs carve_hot(void* ws, int32_t n, int32_t nnz, int32_t hot, size_t* bytes) {
  Carve cv(ws, ~size_t(0));
  HotWs w;
  w.colind_hot = cv.take<int32_t>(nnz > 0 ? nnz : 1);
  w.hot_cols = cv.take<int32_t>(hot > 0 ? hot : 1);
  w.x_hot = cv.take<double>(hot > 0 ? hot : 1);
  w.perm = cv.take<int32_t>(n > 0 ? n : 1);
  w.slot = cv.take<int32_t>(n > 0 ? n : 1);
  w.deg_bytes = 0;
  csr_degree_order_workspace_bytes(n, nnz, &w.deg_bytes);
  w.deg = cv.take<char>(w.deg_bytes);
  *bytes = cv.used;
  return w;
}

unsigned blocks256(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

}  // namespace

spx_status gather_hot_x(const spx_plan* p, const void* x, hipStream_t st) {
  const unsigned g = blocks256(p->hot);
  if (p->hot_xtype == SPX_F64)
    k_hot_gather<double><<<g, 256, 0, st>>>(static_cast<const double*>(x), p->hot_cols, p->hot,
                                            static_cast<double*>(p->x_hot));
  else
    k_hot_gather<float><<<g, 256, 0, st>>>(static_cast<const float*>(x), p->hot_cols, p->hot,
                                           static_cast<float*>(p->x_hot));
  SPX_LAUNCHED("k_hot_gather");
  return SPX_OK;
}

}  // namespace spx

using namespace spx;

extern "C" spx_status csr_plan_hot_x_workspace_bytes(int32_t n, int32_t nnz, int32_t hot, size_t* bytes) {
  if (!bytes) return fail(SPX_ERR_INVALID, "csr_plan_hot_x_workspace_bytes: bytes is null");
  if (n < 0 || nnz < 0) return fail(SPX_ERR_INVALID, "csr_plan_hot_x_workspace_bytes: negative size");
  if (hot < 1 || hot > kMaxHot)
    return fail(SPX_ERR_UNSUPPORTED, "csr_plan_hot_x_workspace_bytes: hot=%d outside [1, %d]", hot, kMaxHot);
  const spx_status s = check_nnz(nnz, "csr_plan_hot_x_workspace_bytes");
  if (s != SPX_OK) return s;
  carve_hot(nullptr, n, nnz, hot, bytes);
  return SPX_OK;
}

extern "C" spx_status csr_plan_attach_hot_x(spx_plan* p, int32_t n, int32_t nnz, const int32_t* colind, int32_t hot,
                                            spx_dtype xtype, void* workspace, size_t ws_bytes, void* stream) {
  const char* who = "csr_plan_attach_hot_x";
  if (!p) return fail(SPX_ERR_INVALID, "%s: plan is null", who);
  if (p->staged) return fail(SPX_ERR_UNSUPPORTED, "%s: a staged plan has no hot x", who);
  if (p->n != n || p->nnz != nnz)
    return fail(SPX_ERR_INVALID, "%s: plan built for %d columns / %d nonzeros, called with %d / %d", who, p->n,
                p->nnz, n, nnz);
  if (xtype != SPX_F64 && xtype != SPX_F32) return fail(SPX_ERR_UNSUPPORTED, "%s: x type %d", who, xtype);
  size_t need = 0;
  spx_status s = csr_plan_hot_x_workspace_bytes(n, nnz, hot, &need);
  if (s != SPX_OK) return s;
  if (nnz > 0 && !colind) return fail(SPX_ERR_INVALID, "%s: colind is null", who);
  if (!workspace || ws_bytes < need) return fail(SPX_ERR_WORKSPACE, "%s: workspace %zu < %zu bytes", who, ws_bytes, need);
  hipStream_t st = as_stream(stream);
  HotWs w = carve_hot(workspace, n, nnz, hot, &need);
  const int32_t h = hot < n ? hot : n;
  if (n > 0) {
    s = csr_degree_order(n, nnz, colind, w.perm, w.deg, w.deg_bytes, stream);
    if (s != SPX_OK) return s;
    k_hot_slots<<<blocks256(n), 256, 0, st>>>(w.perm, n, h, w.slot, w.hot_cols);
    SPX_LAUNCHED("k_hot_slots");
  }
  if (nnz > 0) {
    k_hot_colind<<<blocks256(nnz), 256, 0, st>>>(colind, nnz, w.slot, w.colind_hot);
    SPX_LAUNCHED("k_hot_colind");
  }
  p->hot = h;
  p->hot_xtype = xtype;
  p->hot_cols = w.hot_cols;
  p->colind_hot = w.colind_hot;
  p->x_hot = w.x_hot;
  return SPX_OK;
}
