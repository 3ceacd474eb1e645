// host_csr.hip -- host-array versions of CSR assembly and validation (the
// CRS arrays of Sec. 3) for callers whose triplets or matrices live in host
// memory.  No HIP call is made here.
//
// Assembly is a two-pass least-significant-digit counting sort: the triplet
// indices are first ordered stably by column, then stably by row, which
// leaves them in (row, column, input position) order; equal (row, column)
// runs are then summed in that order.  The device assembly (csr_from_coo)
// and this one produce the same bits.
#include <stdint.h>
#include <string.h>

#include <new>
#include <vector>

#include "internal.hpp"

using namespace spx;

namespace {

// Stable counting sort of the index list `in` by key(t) in [0, nkeys);
// result in `out`.
template <typename Key>
void counting_pass(const std::vector<int64_t>& in, std::vector<int64_t>& out, int64_t nkeys, Key key) {
  std::vector<int64_t> start(static_cast<size_t>(nkeys) + 1, 0);
  for (int64_t t : in) ++start[static_cast<size_t>(key(t)) + 1];
  for (int64_t j = 0; j < nkeys; ++j) start[j + 1] += start[j];
  for (int64_t t : in) out[static_cast<size_t>(start[static_cast<size_t>(key(t))]++)] = t;
}

}  // namespace

extern "C" spx_status csr_from_coo_host(int32_t m, int32_t n, int64_t nnz_in, const int32_t* host_r,
                                        const int32_t* host_c, const double* host_v, int32_t* host_rowptr,
                                        int32_t* host_colind, double* host_values, int32_t* host_nnz_out) {
  if (host_nnz_out) *host_nnz_out = -1;
  if (m < 0 || n < 0 || nnz_in < 0) return fail(SPX_ERR_INVALID, "csr_from_coo_host: negative size");
  {
    const spx_status s = check_nnz(nnz_in, "csr_from_coo_host");
    if (s != SPX_OK) return s;
  }
  if (!host_rowptr || !host_nnz_out) return fail(SPX_ERR_INVALID, "csr_from_coo_host: null output");
  if (nnz_in > 0 && (!host_r || !host_c || !host_v || !host_colind || !host_values))
    return fail(SPX_ERR_INVALID, "csr_from_coo_host: null triplet or output array");
  for (int64_t t = 0; t < nnz_in; ++t) {
    if (host_r[t] < 0 || host_r[t] >= m || host_c[t] < 0 || host_c[t] >= n)
      return fail(SPX_ERR_INVALID, "csr_from_coo_host: triplet %lld = (%d, %d) outside %d x %d",
                  static_cast<long long>(t), host_r[t], host_c[t], m, n);
  }
  try {
    std::vector<int64_t> a(static_cast<size_t>(nnz_in)), b(static_cast<size_t>(nnz_in));
    for (int64_t t = 0; t < nnz_in; ++t) a[static_cast<size_t>(t)] = t;
    counting_pass(a, b, n, [&](int64_t t) { return host_c[t]; });  // by column, stable
    counting_pass(b, a, m, [&](int64_t t) { return host_r[t]; });  // by row, stable
    int64_t out = 0;
    host_rowptr[0] = 0;
    int64_t q = 0;
    for (int32_t i = 0; i < m; ++i) {
      while (q < nnz_in && host_r[a[static_cast<size_t>(q)]] == i) {
        const int64_t t0 = a[static_cast<size_t>(q)];
        const int32_t col = host_c[t0];
        double s = host_v[t0];
        ++q;
        while (q < nnz_in && host_r[a[static_cast<size_t>(q)]] == i && host_c[a[static_cast<size_t>(q)]] == col) {
          s = s + host_v[a[static_cast<size_t>(q)]];  // input order: the sort is stable
          ++q;
        }
        host_colind[out] = col;
        host_values[out] = s;
        ++out;
      }
      host_rowptr[i + 1] = static_cast<int32_t>(out);
    }
    *host_nnz_out = static_cast<int32_t>(out);
  } catch (const std::bad_alloc&) {
    return fail(SPX_ERR_INVALID, "csr_from_coo_host: out of host memory");
  }
  return SPX_OK;
}

extern "C" spx_status csr_validate_host(int32_t m, int32_t n, int32_t nnz, const int32_t* host_rowptr,
                                        const int32_t* host_colind) {
  if (m < 0 || n < 0 || nnz < 0) return fail(SPX_ERR_INVALID, "csr_validate_host: negative size");
  if (!host_rowptr) return fail(SPX_ERR_INVALID, "csr_validate_host: rowptr is null");
  if (nnz > 0 && !host_colind) return fail(SPX_ERR_INVALID, "csr_validate_host: colind is null");
  if (host_rowptr[0] != 0) return fail(SPX_ERR_INVALID, "csr_validate_host: rowptr[0] = %d, not 0", host_rowptr[0]);
  if (host_rowptr[m] != nnz)
    return fail(SPX_ERR_INVALID, "csr_validate_host: rowptr[m] = %d, not nnz = %d", host_rowptr[m], nnz);
  for (int32_t i = 0; i < m; ++i) {
    if (host_rowptr[i + 1] < host_rowptr[i] || host_rowptr[i + 1] > nnz)
      return fail(SPX_ERR_INVALID, "csr_validate_host: row %d has range [%d, %d) outside [0, %d] or decreasing",
                  i, host_rowptr[i], host_rowptr[i + 1], nnz);
  }
  for (int32_t p = 0; p < nnz; ++p) {
    if (host_colind[p] < 0 || host_colind[p] >= n)
      return fail(SPX_ERR_INVALID, "csr_validate_host: colind[%d] = %d outside [0, %d)", p, host_colind[p], n);
  }
  return SPX_OK;
}
