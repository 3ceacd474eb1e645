// abi.hip -- C entry points of the products (y <- A x, Y <- A X), the
// transpose product and the sampled dot: argument checks, choice of the lane
// layout, and the launch on the caller's stream.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "internal.hpp"

namespace spx {

namespace {
thread_local char g_err[512] = {0};
}

spx_status fail(spx_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

spx_status hip_fail(hipError_t e, const char* what) {
  snprintf(g_err, sizeof(g_err), "%s: %s", what, hipGetErrorString(e));
  return SPX_ERR_HIP;
}

static bool aligned16_(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

void layout_for_k(int32_t k, spx_dtype xt, const void* X, int64_t ldx, const void* Y, int64_t ldy,
                  uint32_t flags, int* kl, int* vec) {
  if (k == 1) {
    *kl = 1;
    *vec = 1;
    return;
  }
  const int V = (xt == SPX_F64) ? 2 : 4;
  const bool vec_ok = !(flags & SPX_FLAG_SCALAR_X) && (k % V == 0) && (ldx % V == 0) &&
                      (ldy % V == 0) && aligned16_(X) && aligned16_(Y);
  *vec = vec_ok ? V : 1;

  const int per = (k + *vec - 1) / *vec;
  int l = 1;
  while (l < per && l < 32) l <<= 1;
  *kl = l;
}

namespace {

bool pair_ok(spx_dtype vt, spx_dtype xt) {
  return (vt == SPX_F64 && xt == SPX_F64) || (vt == SPX_F32 && xt == SPX_F32) ||
         (vt == SPX_BF16 && xt == SPX_F32);
}

spx_status check_plan(const spx_plan* plan, int32_t rows, int32_t nnz, int32_t k, const char* who,
                      bool staged_ok = true) {
  if (!plan) return SPX_OK;
  if (plan->staged && !staged_ok)
    return fail(SPX_ERR_UNSUPPORTED, "%s: a staged plan serves csr_spmv / csr_spmm only", who);
  if (plan->m != rows || plan->nnz != nnz)
    return fail(SPX_ERR_INVALID, "%s: plan built for %d rows / %d nonzeros, called with %d / %d", who,
                plan->m, plan->nnz, rows, nnz);
  if (plan->nseg > 0 && k > plan->opts.max_k)
    return fail(SPX_ERR_INVALID, "%s: k=%d exceeds the plan's max_k=%d", who, k, plan->opts.max_k);
  return SPX_OK;
}

spx_status product(const char* who, int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                   const int32_t* colind, const void* values, const int32_t* vperm, spx_dtype vt,
                   int32_t k, const void* X, int64_t ldx, void* Y, int64_t ldy, spx_dtype xt,
                   const spx_plan* plan, void* stream, void* xsave = nullptr) {
  if (m < 0 || n < 0 || nnz < 0) return fail(SPX_ERR_INVALID, "%s: negative size", who);
  {
    const spx_status s_nnz = check_nnz(nnz, who);
    if (s_nnz != SPX_OK) return s_nnz;
  }
  if (k < 1) return fail(SPX_ERR_INVALID, "%s: k=%d < 1", who, k);
  if (ldx < k || ldy < k)
    return fail(SPX_ERR_INVALID, "%s: ldx=%lld / ldy=%lld smaller than k=%d", who, (long long)ldx,
                (long long)ldy, k);
  if (!pair_ok(vt, xt)) return fail(SPX_ERR_UNSUPPORTED, "%s: dtype pair (%d, %d)", who, vt, xt);
  if (m == 0) return SPX_OK;
  if (!rowptr || !Y) return fail(SPX_ERR_INVALID, "%s: null rowptr or output", who);
  if (nnz > 0 && (!colind || !values || !X))
    return fail(SPX_ERR_INVALID, "%s: null colind, values or input", who);
  spx_status s = check_plan(plan, m, nnz, k, who);
  if (s != SPX_OK) return s;
  ProdArgs a;
  memset(&a, 0, sizeof(a));
  a.rowptr = rowptr;
  a.colind = colind;
  a.values = values;
  a.vperm = vperm;
  a.X = X;
  a.Y = Y;
  a.ldx = ldx;
  a.ldy = ldy;
  a.k = k;
  int kl, vec;
  layout_for_k(k, xt, X, a.ldx, Y, a.ldy, plan ? plan->opts.flags : 0u, &kl, &vec);
  if (plan && plan->staged) {
    if (vperm) return fail(SPX_ERR_UNSUPPORTED, "%s: a staged plan serves CSR-order values only", who);
    return launch_staged(a, plan, m, vt, xt, kl, vec, as_stream(stream));
  }
  if (plan) bins_from_plan(plan, a, kl, true);
  else bins_unbinned(m, nnz, kl, a);
  if (xsave) {
    a.xsave = xsave;
    return launch_product_save(a, vt, xt, as_stream(stream));
  }
  if (plan && plan->hot > 0 && k == 1 && !vperm && nnz > 0) {
    if (xt != plan->hot_xtype)
      return fail(SPX_ERR_INVALID, "%s: the plan's hot x was attached for x type %d, called with %d", who,
                  plan->hot_xtype, xt);
    a.colind = plan->colind_hot;
    a.X2 = plan->x_hot;
    a.ldx2 = plan->hot;
    const spx_status sh = gather_hot_x(plan, X, as_stream(stream));
    if (sh != SPX_OK) return sh;
    return launch_product_hot(a, vt, xt, as_stream(stream));
  }
  return launch_product(a, vt, xt, kl, vec, as_stream(stream));
}

}  // namespace
}  // namespace spx

using namespace spx;

extern "C" const char* spx_last_error(void) { return g_err; }

extern "C" const char* spx_version(void) { return "spx 0.1 gfx950"; }

extern "C" spx_status csr_spmv(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                               const int32_t* colind, const void* values, spx_dtype vtype,
                               const void* x, void* y, spx_dtype xytype, const spx_plan* plan,
                               void* stream) {
  return product("csr_spmv", m, n, nnz, rowptr, colind, values, nullptr, vtype, 1, x, 1, y, 1,
                 xytype, plan, stream);
}

extern "C" spx_status csr_spmv_save(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                                    const int32_t* colind, const void* values, spx_dtype vtype,
                                    const void* x, void* y, spx_dtype xytype, void* xsave,
                                    const spx_plan* plan, void* stream) {
  if (nnz > 0 && !xsave) return fail(SPX_ERR_INVALID, "csr_spmv_save: xsave is null");
  if (plan && plan->staged)
    return fail(SPX_ERR_UNSUPPORTED, "csr_spmv_save: a staged plan serves csr_spmv / csr_spmm only");
  return product("csr_spmv_save", m, n, nnz, rowptr, colind, values, nullptr, vtype, 1, x, 1, y, 1,
                 xytype, plan, stream, nnz > 0 ? xsave : nullptr);
}

extern "C" spx_status csr_spmm(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                               const int32_t* colind, const void* values, spx_dtype vtype, int32_t k,
                               const void* X, int64_t ldx, void* Y, int64_t ldy, spx_dtype xytype,
                               const spx_plan* plan, void* stream) {
  return product("csr_spmm", m, n, nnz, rowptr, colind, values, nullptr, vtype, k, X, ldx, Y, ldy,
                 xytype, plan, stream);
}

extern "C" spx_status csr_spmv_t(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                                 const int32_t* colind, const int32_t* colptr,
                                 const int32_t* rowind, const int32_t* perm, const void* values,
                                 spx_dtype vtype, int32_t k, const void* dY, int64_t lddy, void* dX,
                                 int64_t lddx, spx_dtype xytype, int32_t mode,
                                 const spx_plan* plan, void* stream) {
  if (mode == 0) {
    if (nnz > 0 && (!colptr || !rowind))
      return fail(SPX_ERR_INVALID, "csr_spmv_t: CSC index arrays are required for mode 0");
    if (n > 0 && !colptr) return fail(SPX_ERR_INVALID, "csr_spmv_t: colptr is null");
    // gather over the CSC pattern: n "rows", values read through perm (or,
    // with perm == NULL, values already in CSC order)
    return product("csr_spmv_t", n, m, nnz, colptr, rowind, values, perm, vtype, k, dY, lddy, dX,
                   lddx, xytype, plan, stream);
  }
  if (mode != 1) return fail(SPX_ERR_INVALID, "csr_spmv_t: mode=%d (0 or 1)", mode);
  if (m < 0 || n < 0 || nnz < 0) return fail(SPX_ERR_INVALID, "csr_spmv_t: negative size");
  {
    const spx_status s_nnz = check_nnz(nnz, "csr_spmv_t");
    if (s_nnz != SPX_OK) return s_nnz;
  }
  if (k < 1) return fail(SPX_ERR_INVALID, "csr_spmv_t: k=%d < 1", k);
  if (lddy < k || lddx < k) return fail(SPX_ERR_INVALID, "csr_spmv_t: leading dims < k");
  if (!pair_ok(vtype, xytype)) return fail(SPX_ERR_UNSUPPORTED, "csr_spmv_t: dtype pair");
  if (n > 0 && !dX) return fail(SPX_ERR_INVALID, "csr_spmv_t: dX is null");
  if (m > 0 && !rowptr) return fail(SPX_ERR_INVALID, "csr_spmv_t: rowptr is null");
  if (nnz > 0 && (!colind || !values || !dY))
    return fail(SPX_ERR_INVALID, "csr_spmv_t: null colind, values or dY");
  spx_status s = check_plan(plan, m, nnz, 1, "csr_spmv_t", false);
  if (s != SPX_OK) return s;
  ProdArgs a;
  memset(&a, 0, sizeof(a));
  a.rowptr = rowptr;
  a.colind = colind;
  a.values = values;
  a.X = dY;
  a.Y = dX;
  a.ldx = lddy;
  a.ldy = lddx;
  a.k = k;
  return launch_scatter_t(a, plan, m, n, nnz, vtype, xytype, as_stream(stream));
}

extern "C" spx_status csr_sddmm(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                                const int32_t* colind, int32_t k, const void* dY, int64_t lddy,
                                const void* X, int64_t ldx, void* out, spx_dtype dtype,
                                const spx_plan* plan, void* stream) {
  if (m < 0 || n < 0 || nnz < 0) return fail(SPX_ERR_INVALID, "csr_sddmm: negative size");
  {
    const spx_status s_nnz = check_nnz(nnz, "csr_sddmm");
    if (s_nnz != SPX_OK) return s_nnz;
  }
  if (k < 1) return fail(SPX_ERR_INVALID, "csr_sddmm: k=%d < 1", k);
  if (lddy < k || ldx < k) return fail(SPX_ERR_INVALID, "csr_sddmm: leading dims < k");
  if (dtype != SPX_F64 && dtype != SPX_F32)
    return fail(SPX_ERR_UNSUPPORTED, "csr_sddmm: dtype must be F64 or F32");
  if (m == 0 || nnz == 0) return SPX_OK;
  if (!rowptr || !colind || !dY || !X || !out)
    return fail(SPX_ERR_INVALID, "csr_sddmm: null pointer");
  spx_status s = check_plan(plan, m, nnz, 1, "csr_sddmm", false);
  if (s != SPX_OK) return s;
  ProdArgs a;
  memset(&a, 0, sizeof(a));
  a.rowptr = rowptr;
  a.colind = colind;
  a.X = dY;
  a.ldx = lddy;
  a.X2 = X;
  a.ldx2 = ldx;
  a.Y = out;
  a.k = k;
  return launch_sddmm(a, plan, m, nnz, dtype, false, as_stream(stream));
}

extern "C" spx_status csr_sddmm_saved(int32_t m, int32_t nnz, const int32_t* rowptr, const void* dy,
                                      const void* xsave, void* out, spx_dtype dtype, const spx_plan* plan,
                                      void* stream) {
  if (m < 0 || nnz < 0) return fail(SPX_ERR_INVALID, "csr_sddmm_saved: negative size");
  {
    const spx_status s_nnz = check_nnz(nnz, "csr_sddmm_saved");
    if (s_nnz != SPX_OK) return s_nnz;
  }
  if (dtype != SPX_F64 && dtype != SPX_F32)
    return fail(SPX_ERR_UNSUPPORTED, "csr_sddmm_saved: dtype must be F64 or F32");
  if (m == 0 || nnz == 0) return SPX_OK;
  if (!rowptr || !dy || !xsave || !out) return fail(SPX_ERR_INVALID, "csr_sddmm_saved: null pointer");
  spx_status s = check_plan(plan, m, nnz, 1, "csr_sddmm_saved", false);
  if (s != SPX_OK) return s;
  ProdArgs a;
  memset(&a, 0, sizeof(a));
  a.rowptr = rowptr;
  a.X = dy;
  a.ldx = 1;
  a.X2 = xsave;
  a.ldx2 = 1;
  a.Y = out;
  a.k = 1;
  return launch_sddmm(a, plan, m, nnz, dtype, true, as_stream(stream));
}
