// assemble.hip -- CSR assembly from triplets, structural validation and the
// CSC index of the transpose, all on the device.
//
// CRS (paper Sec. 3): rowptr[0] = 0, rowptr[m] = tau, the column ids of row i
// in colind[rowptr[i] .. rowptr[i+1]-1].  Canonical form here: columns
// strictly ascending inside a row; duplicate (i, j) triplets summed in input
// order.  A stable radix sort on the key (row, column) keeps duplicates in
// input order, so each run is summed front to back with plain FP64 adds.
#include "device.hpp"
#include "internal.hpp"

namespace spx {

namespace {

inline int bits_for(int64_t x) {  // bits needed to represent x >= 0
  int b = 0;
  while (x > 0) {
    ++b;
    x >>= 1;
  }
  return b;
}

__global__ void k_make_keys(const int32_t* __restrict__ r, const int32_t* __restrict__ c,
                            int64_t nnz, int32_t m, int32_t n, int cbits,
                            uint64_t* __restrict__ keys, int32_t* __restrict__ vals,
                            int32_t* __restrict__ bad) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const int32_t ri = r[i], ci = c[i];
  if (ri < 0 || ri >= m || ci < 0 || ci >= n) {
    atomicOr(bad, 1);
    keys[i] = 0;
  } else {
    keys[i] = (static_cast<uint64_t>(ri) << cbits) | static_cast<uint64_t>(ci);
  }
  vals[i] = static_cast<int32_t>(i);
}

__global__ void k_heads(const uint64_t* __restrict__ keys, int64_t nnz, int32_t* __restrict__ heads) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  heads[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// One thread per sorted position; heads emit their run.  `pos` holds the
// exclusive scan of the head flags (the output index of each head).
__global__ void k_emit(const uint64_t* __restrict__ keys, const int32_t* __restrict__ src,
                       const int32_t* __restrict__ pos, const double* __restrict__ v,
                       int64_t nnz, int32_t m, int cbits, int32_t* __restrict__ rowptr,
                       int32_t* __restrict__ colind, double* __restrict__ values) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const uint64_t key = keys[i];
  if (i > 0 && keys[i - 1] == key) return;  // not a head
  const int32_t out = pos[i];
  double s = v[src[i]];
  int64_t j = i + 1;
  while (j < nnz && keys[j] == key) {
    s = s + v[src[j]];
    ++j;
  }
  const uint64_t cmask = (cbits >= 64) ? ~0ull : ((1ull << cbits) - 1ull);
  colind[out] = static_cast<int32_t>(key & cmask);
  values[out] = s;
  const int32_t row = static_cast<int32_t>(key >> cbits);
  const int32_t prev = (i == 0) ? -1 : static_cast<int32_t>(keys[i - 1] >> cbits);
  for (int32_t rr = prev + 1; rr <= row; ++rr) rowptr[rr] = out;
  if (j == nnz)
    for (int32_t rr = row + 1; rr <= m; ++rr) rowptr[rr] = out + 1;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t value) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

__global__ void k_finish_count(const int32_t* __restrict__ bad, const int32_t* __restrict__ total,
                               int32_t* __restrict__ nnz_out) {
  *nnz_out = (*bad) ? -1 : *total;
}

__global__ void k_validate(int32_t m, int32_t n, int32_t nnz, const int32_t* __restrict__ rowptr,
                           const int32_t* __restrict__ colind, int32_t check_sorted,
                           int32_t* __restrict__ status) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i == 0 && (rowptr[0] != 0 || rowptr[m] != nnz)) atomicMax(status, 4);
  if (i >= m) return;
  const int32_t a = rowptr[i], b = rowptr[i + 1];
  if (a < 0 || b > nnz || a > b) {
    atomicMax(status, 3);
    return;
  }
  int32_t last = -1;
  for (int32_t p = a; p < b; ++p) {
    const int32_t c = colind[p];
    if (c < 0 || c >= n) {
      atomicMax(status, 2);
      return;
    }
    if (check_sorted && c <= last) {
      atomicMax(status, 1);
      return;
    }
    last = c;
  }
}

__global__ void k_col_keys(const int32_t* __restrict__ colind, int64_t nnz, uint32_t* __restrict__ keys,
                           int32_t* __restrict__ vals) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  keys[i] = static_cast<uint32_t>(colind[i]);
  vals[i] = static_cast<int32_t>(i);
}

// After the stable sort by column: rowind from the CSR position by binary
// search in rowptr, colptr from the column boundaries.
__global__ void k_csc_finish(const uint32_t* __restrict__ keys, const int32_t* __restrict__ perm,
                             const int32_t* __restrict__ rowptr, int32_t m, int32_t n, int64_t nnz,
                             int32_t* __restrict__ rowind, int32_t* __restrict__ colptr) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nnz) return;
  const int32_t p = perm[q];
  int32_t lo = 0, hi = m;  // largest row with rowptr[row] <= p
  while (hi - lo > 1) {
    int32_t mid = (lo + hi) >> 1;
    if (rowptr[mid] <= p) lo = mid; else hi = mid;
  }
  rowind[q] = lo;
  // column ids are assumed valid (0 <= col < n); clamp so a bad id cannot
  // write outside colptr
  const int32_t col = min(static_cast<int32_t>(keys[q]), n - 1);
  const int32_t prev = (q == 0) ? -1 : min(static_cast<int32_t>(keys[q - 1]), n - 1);
  if (q == 0 || prev != col)
    for (int32_t j = prev + 1; j <= col; ++j) colptr[j] = static_cast<int32_t>(q);
  if (q == nnz - 1)
    for (int32_t j = col + 1; j <= n; ++j) colptr[j] = static_cast<int32_t>(nnz);
}

inline unsigned grid_for(int64_t n, int bs = 256) {
  return static_cast<unsigned>((n + bs - 1) / bs);
}

struct CooWs {
  uint64_t* keys;
  int32_t* src;
  int32_t* heads;
  int32_t* bad;
  int32_t* total;
  void* radix;
  void* scan;
};

CooWs carve_coo(void* ws, int64_t nnz, size_t* bytes) {
  Carve cv(ws, ~size_t(0));
  CooWs w;
  w.keys = cv.take<uint64_t>(nnz > 0 ? nnz : 1);
  w.src = cv.take<int32_t>(nnz > 0 ? nnz : 1);
  w.heads = cv.take<int32_t>(nnz > 0 ? nnz : 1);
  w.bad = cv.take<int32_t>(1);
  w.total = cv.take<int32_t>(1);
  w.radix = cv.take<char>(radix_workspace_bytes(nnz, 8));
  w.scan = cv.take<char>(scan_workspace_bytes(nnz));
  *bytes = cv.used;
  return w;
}

}  // namespace
}  // namespace spx

using namespace spx;

extern "C" spx_status csr_from_coo_workspace_bytes(int32_t m, int32_t n, int64_t nnz_in,
                                                   size_t* bytes) {
  if (!bytes) return fail(SPX_ERR_INVALID, "csr_from_coo_workspace_bytes: bytes is null");
  if (m < 0 || n < 0 || nnz_in < 0)
    return fail(SPX_ERR_INVALID, "csr_from_coo_workspace_bytes: bad sizes m=%d n=%d nnz=%lld", m, n,
                (long long)nnz_in);
  {
    const spx_status s_nnz = check_nnz(nnz_in, "csr_from_coo_workspace_bytes");
    if (s_nnz != SPX_OK) return s_nnz;
  }
  carve_coo(nullptr, nnz_in, bytes);
  return SPX_OK;
}

extern "C" spx_status csr_from_coo(int32_t m, int32_t n, int64_t nnz_in, const int32_t* r,
                                   const int32_t* c, const double* v, int32_t* rowptr,
                                   int32_t* colind, double* values, int32_t* nnz_out,
                                   void* workspace, size_t ws_bytes, void* stream) {
  if (m < 0 || n < 0 || nnz_in < 0)
    return fail(SPX_ERR_INVALID, "csr_from_coo: bad sizes m=%d n=%d nnz=%lld", m, n, (long long)nnz_in);
  {
    const spx_status s_nnz = check_nnz(nnz_in, "csr_from_coo");
    if (s_nnz != SPX_OK) return s_nnz;
  }
  if (!rowptr || !nnz_out) return fail(SPX_ERR_INVALID, "csr_from_coo: null rowptr or nnz_out");
  if (nnz_in > 0 && (!r || !c || !v || !colind || !values))
    return fail(SPX_ERR_INVALID, "csr_from_coo: null triplet or output array");
  if (nnz_in > 0 && (m == 0 || n == 0))
    return fail(SPX_ERR_INVALID, "csr_from_coo: triplets given for an empty shape");
  size_t need;
  carve_coo(nullptr, nnz_in, &need);
  if (!workspace || ws_bytes < need)
    return fail(SPX_ERR_WORKSPACE, "csr_from_coo: workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t st = as_stream(stream);
  CooWs w = carve_coo(workspace, nnz_in, &need);
  const int cbits = bits_for(n > 0 ? n - 1 : 0);
  const int rbits = bits_for(m > 0 ? m - 1 : 0);
  k_fill_i32<<<1, 64, 0, st>>>(w.bad, 1, 0);
  SPX_LAUNCHED("k_fill_i32");
  if (nnz_in == 0) {
    k_fill_i32<<<grid_for(int64_t(m) + 1), 256, 0, st>>>(rowptr, int64_t(m) + 1, 0);
    SPX_LAUNCHED("k_fill_i32");
    k_fill_i32<<<1, 64, 0, st>>>(nnz_out, 1, 0);
    SPX_LAUNCHED("k_fill_i32");
    return SPX_OK;
  }
  k_make_keys<<<grid_for(nnz_in), 256, 0, st>>>(r, c, nnz_in, m, n, cbits, w.keys, w.src, w.bad);
  SPX_LAUNCHED("k_make_keys");
  spx_status s = radix_sort_u64(w.keys, w.src, nnz_in, cbits + rbits, w.radix, st);
  if (s != SPX_OK) return s;
  k_heads<<<grid_for(nnz_in), 256, 0, st>>>(w.keys, nnz_in, w.heads);
  SPX_LAUNCHED("k_heads");
  s = exclusive_scan_i32(w.heads, w.heads, nnz_in, w.total, w.scan, st);
  if (s != SPX_OK) return s;
  k_emit<<<grid_for(nnz_in), 256, 0, st>>>(w.keys, w.src, w.heads, v, nnz_in, m, cbits, rowptr,
                                           colind, values);
  SPX_LAUNCHED("k_emit");
  k_finish_count<<<1, 1, 0, st>>>(w.bad, w.total, nnz_out);
  SPX_LAUNCHED("k_finish_count");
  return SPX_OK;
}

extern "C" spx_status csr_validate(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                                   const int32_t* colind, int32_t check_sorted,
                                   int32_t* status_out, void* stream) {
  if (m < 0 || n < 0 || nnz < 0) return fail(SPX_ERR_INVALID, "csr_validate: negative size");
  {
    const spx_status s_nnz = check_nnz(nnz, "csr_validate");
    if (s_nnz != SPX_OK) return s_nnz;
  }
  if (!rowptr || !status_out || (nnz > 0 && !colind))
    return fail(SPX_ERR_INVALID, "csr_validate: null pointer");
  hipStream_t st = as_stream(stream);
  k_fill_i32<<<1, 64, 0, st>>>(status_out, 1, 0);
  SPX_LAUNCHED("k_fill_i32");
  k_validate<<<grid_for(int64_t(m) + 1), 256, 0, st>>>(m, n, nnz, rowptr, colind, check_sorted,
                                                       status_out);
  SPX_LAUNCHED("k_validate");
  return SPX_OK;
}

namespace {
size_t transpose_ws(int64_t nnz) {
  return align_up(static_cast<size_t>(nnz > 0 ? nnz : 1) * 4) + radix_workspace_bytes(nnz, 4);
}
}  // namespace

extern "C" spx_status csr_transpose_index_workspace_bytes(int32_t m, int32_t n, int32_t nnz,
                                                          size_t* bytes) {
  if (!bytes || m < 0 || n < 0 || nnz < 0)
    return fail(SPX_ERR_INVALID, "csr_transpose_index_workspace_bytes: bad arguments");
  *bytes = transpose_ws(nnz);
  return SPX_OK;
}

extern "C" spx_status csr_transpose_index(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                                          const int32_t* colind, int32_t* colptr, int32_t* rowind,
                                          int32_t* perm, void* workspace, size_t ws_bytes,
                                          void* stream) {
  if (m < 0 || n < 0 || nnz < 0) return fail(SPX_ERR_INVALID, "csr_transpose_index: negative size");
  {
    const spx_status s_nnz = check_nnz(nnz, "csr_transpose_index");
    if (s_nnz != SPX_OK) return s_nnz;
  }
  if (!colptr || (nnz > 0 && (!rowptr || !colind || !rowind || !perm)))
    return fail(SPX_ERR_INVALID, "csr_transpose_index: null pointer");
  if (!workspace || ws_bytes < transpose_ws(nnz))
    return fail(SPX_ERR_WORKSPACE, "csr_transpose_index: workspace %zu < %zu bytes", ws_bytes,
                transpose_ws(nnz));
  hipStream_t st = as_stream(stream);
  if (nnz == 0) {
    k_fill_i32<<<grid_for(int64_t(n) + 1), 256, 0, st>>>(colptr, int64_t(n) + 1, 0);
    SPX_LAUNCHED("k_fill_i32");
    return SPX_OK;
  }
  Carve cv(workspace, ws_bytes);
  uint32_t* keys = cv.take<uint32_t>(nnz);
  void* rws = cv.take<char>(radix_workspace_bytes(nnz, 4));
  k_col_keys<<<grid_for(nnz), 256, 0, st>>>(colind, nnz, keys, perm);
  SPX_LAUNCHED("k_col_keys");
  spx_status s = radix_sort_u32(keys, perm, nnz, bits_for(n > 0 ? n - 1 : 0), rws, st);
  if (s != SPX_OK) return s;
  k_csc_finish<<<grid_for(nnz), 256, 0, st>>>(keys, perm, rowptr, m, n, nnz, rowind, colptr);
  SPX_LAUNCHED("k_csc_finish");
  return SPX_OK;
}
