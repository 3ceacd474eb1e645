// bcsr.hip -- register-blocked CRS (paper Sec. 4.5): the matrix is cut into
// a x b blocks (a, b in {1, 2, 4, 8}); every block holding a nonzero is kept,
// listed in CRS order (block rows, then block columns ascending).  Two block
// encodings:
//   dense   a*b values per block, row-major inside the block, zeros explicit
//           (the paper's register blocking);
//   bitmap  a 64-bit mask of the block's nonzeros plus the nonzeros packed in
//           bit order (the sparse block storage the paper proposes as the
//           next step, after Buluc et al.).
// Conversion runs on the device (radix sort of block keys, one pass per
// block); it is one-time and untimed, as in the paper.  The product gives
// each block row to a group of G lanes; every lane multiplies whole blocks
// (A accumulators, the B-element slice of x loaded once per block) and the
// group reduces its A partial sums.
#include "device.hpp"
#include "internal.hpp"

namespace spx {
namespace {

inline int bits_for(int64_t x) {
  int b = 0;
  while (x > 0) {
    ++b;
    x >>= 1;
  }
  return b;
}

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

bool shape_ok(int a, int b) {
  auto p2 = [](int v) { return v == 1 || v == 2 || v == 4 || v == 8; };
  return p2(a) && p2(b);
}

struct BlockWs {
  uint64_t* keys;
  int32_t* src;
  int32_t* rowid;
  int32_t* index;  // exclusive scan of the block heads: block of each sorted entry
  int32_t* brow;   // block row of each block
  int32_t* total;
  void* radix;
  void* scan;
};

BlockWs carve_blocks(void* ws, int64_t nnz, size_t* bytes) {
  Carve cv(ws, ~size_t(0));
  const int64_t e = nnz > 0 ? nnz : 1;
  BlockWs w;
  w.keys = cv.take<uint64_t>(e);
  w.src = cv.take<int32_t>(e);
  w.rowid = cv.take<int32_t>(e);
  w.index = cv.take<int32_t>(e);
  w.brow = cv.take<int32_t>(e);
  w.total = cv.take<int32_t>(1);
  w.radix = cv.take<char>(radix_workspace_bytes(nnz, 8));
  w.scan = cv.take<char>(scan_workspace_bytes(nnz));
  *bytes = cv.used;
  return w;
}

// One thread per row: block key (block row, block column) of each nonzero.
__global__ void k_block_keys(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                             int32_t m, int a, int b, int cbits, uint64_t* __restrict__ keys,
                             int32_t* __restrict__ src, int32_t* __restrict__ rowid) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint64_t br = static_cast<uint64_t>(i / a) << cbits;
  for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
    keys[p] = br | static_cast<uint64_t>(colind[p] / b);
    src[p] = p;
    rowid[p] = static_cast<int32_t>(i);
  }
}

__global__ void k_block_heads(const uint64_t* __restrict__ keys, int64_t nnz, int32_t* __restrict__ heads) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  heads[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// One thread per sorted entry that starts a block: writes the block's column,
// its row and its values.  Entries of one block arrive in CSR order, which
// (columns ascending inside rows) is ascending position inside the block.
__global__ void k_block_fill(const uint64_t* __restrict__ keys, const int32_t* __restrict__ src,
                             const int32_t* __restrict__ rowid, const int32_t* __restrict__ index,
                             const int32_t* __restrict__ colind, const double* __restrict__ values,
                             int64_t nnz, int a, int b, int cbits, int bitmap, int32_t* __restrict__ bcol,
                             int32_t* __restrict__ brow, double* __restrict__ bvals,
                             uint64_t* __restrict__ bmask, int32_t* __restrict__ boff) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const uint64_t key = keys[i];
  if (i > 0 && keys[i - 1] == key) return;
  const int32_t q = index[i];
  bcol[q] = static_cast<int32_t>(key & ((uint64_t(1) << cbits) - 1));
  brow[q] = static_cast<int32_t>(key >> cbits);
  const int ab = a * b;
  if (!bitmap)
    for (int t = 0; t < ab; ++t) bvals[static_cast<int64_t>(q) * ab + t] = 0.0;
  uint64_t mask = 0;
  for (int64_t j = i; j < nnz && keys[j] == key; ++j) {
    const int32_t p = src[j];
    const int pos = (rowid[p] % a) * b + colind[p] % b;
    if (bitmap) {
      mask |= uint64_t(1) << pos;
      bvals[j] = values[p];
    } else {
      bvals[static_cast<int64_t>(q) * ab + pos] = values[p];
    }
  }
  if (bitmap) {
    bmask[q] = mask;
    boff[q] = static_cast<int32_t>(i);
  }
}

__global__ void k_zero_i32(int32_t* __restrict__ p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_copy_i32(const int32_t* __restrict__ src, int32_t* __restrict__ dst) { *dst = *src; }

// browptr[R] = first block whose block row is >= R (blocks are sorted).
__global__ void k_block_rowptr(const int32_t* __restrict__ brow, const int32_t* __restrict__ nblocks, int32_t mb,
                               int32_t* __restrict__ browptr) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r > mb) return;
  int32_t lo = 0, hi = *nblocks;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (brow[mid] < r) lo = mid + 1;
    else hi = mid;
  }
  browptr[r] = lo;
}

spx_status sort_blocks(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr, const int32_t* colind, int a,
                       int b, const BlockWs& w, int* cbits_out, hipStream_t st) {
  const int64_t mb = (static_cast<int64_t>(m) + a - 1) / a, nbc = (static_cast<int64_t>(n) + b - 1) / b;
  const int cbits = bits_for(nbc > 0 ? nbc - 1 : 0), rbits = bits_for(mb > 0 ? mb - 1 : 0);
  *cbits_out = cbits;
  k_block_keys<<<blocks_for(m), 256, 0, st>>>(rowptr, colind, m, a, b, cbits, w.keys, w.src, w.rowid);
  SPX_LAUNCHED("k_block_keys");
  spx_status s = radix_sort_u64(w.keys, w.src, nnz, cbits + rbits, w.radix, st);
  if (s != SPX_OK) return s;
  k_block_heads<<<blocks_for(nnz), 256, 0, st>>>(w.keys, nnz, w.index);
  SPX_LAUNCHED("k_block_heads");
  return exclusive_scan_i32(w.index, w.index, nnz, w.total, w.scan, st);
}

// ---------------------------------------------------------------- product

struct BcsrArgs {
  const int32_t* browptr;
  const int32_t* bcol;
  const double* bvals;
  const uint64_t* bmask;
  const int32_t* boff;
  const double* x;
  double* y;
  int32_t m, n, mb;
  int32_t lanes;  // lanes per block row (power of two, <= 64)
  int32_t lane_shift;
};

template <int B>
__device__ __forceinline__ void load_xs(const BcsrArgs& p, int32_t c, double (&xb)[B]) {
  const int64_t j0 = static_cast<int64_t>(c) * B;
  if (j0 + B <= p.n) {
#pragma unroll
    for (int j = 0; j < B; ++j) xb[j] = p.x[j0 + j];
  } else {
#pragma unroll
    for (int j = 0; j < B; ++j) xb[j] = (j0 + j < p.n) ? p.x[j0 + j] : 0.0;
  }
}

template <int A, int B, bool BITMAP>
__device__ __forceinline__ void block_fma(const BcsrArgs& p, int32_t q, const double (&xb)[B], double (&acc)[A]) {
  if constexpr (!BITMAP) {
    const double* v = p.bvals + static_cast<int64_t>(q) * (A * B);
    double vv[A * B];
#pragma unroll
    for (int t = 0; t < A * B; ++t) vv[t] = __builtin_nontemporal_load(v + t);
#pragma unroll
    for (int r = 0; r < A; ++r)
#pragma unroll
      for (int j = 0; j < B; ++j) acc[r] = __builtin_fma(vv[r * B + j], xb[j], acc[r]);
  } else {
    const uint64_t mask = p.bmask[q];
    const double* v = p.bvals + p.boff[q];
    // each set bit's value sits at the count of set bits below it
#pragma unroll
    for (int r = 0; r < A; ++r)
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int bit = r * B + j;
        if ((mask >> bit) & 1) {
          const int k = __builtin_popcountll(mask & ((uint64_t(1) << bit) - 1));
          acc[r] = __builtin_fma(__builtin_nontemporal_load(v + k), xb[j], acc[r]);
        }
      }
  }
}

template <int A, int B, bool BITMAP>
__global__ __launch_bounds__(kWG) void k_bcsr_spmv(const BcsrArgs p) {
  const int t = threadIdx.x;
  const int G = p.lanes;
  const int slot = t & (G - 1);
  const int64_t R = (static_cast<int64_t>(blockIdx.x) * kWG + t) >> p.lane_shift;
  const bool active = R < p.mb;
  double acc[A];
#pragma unroll
  for (int r = 0; r < A; ++r) acc[r] = 0.0;
  if (active) {
    const int32_t q0 = p.browptr[R], q1 = p.browptr[R + 1];
    // two blocks per iteration, the second masked, so two x slices and two
    // value blocks are in flight per lane
    for (int32_t q = q0 + slot; q < q1; q += 2 * G) {
      const bool two = q + G < q1;
      const int32_t c0 = p.bcol[q];
      const int32_t c1 = two ? p.bcol[q + G] : 0;
      double x0[B], x1[B];
      load_xs<B>(p, c0, x0);
      if (two) {
        load_xs<B>(p, c1, x1);
      } else {
#pragma unroll
        for (int j = 0; j < B; ++j) x1[j] = 0.0;
      }
      block_fma<A, B, BITMAP>(p, q, x0, acc);
      if (two) block_fma<A, B, BITMAP>(p, q + G, x1, acc);
    }
  }
  // reduce across the G lanes of the block row (xor butterfly inside the wave)
#pragma unroll
  for (int r = 0; r < A; ++r)
    for (int off = G >> 1; off > 0; off >>= 1) acc[r] += __shfl_xor(acc[r], off, kWave);
  if (active && slot == 0) {
#pragma unroll
    for (int r = 0; r < A; ++r) {
      const int64_t row = R * A + r;
      if (row < p.m) __builtin_nontemporal_store(acc[r], p.y + row);
    }
  }
}

template <bool BITMAP>
spx_status launch_bcsr(int a, int b, const BcsrArgs& p, unsigned grid, hipStream_t st) {
#define SPX_BCASE(A_, B_)                                          \
  if (a == A_ && b == B_) {                                        \
    k_bcsr_spmv<A_, B_, BITMAP><<<grid, kWG, 0, st>>>(p);          \
    SPX_LAUNCHED("k_bcsr_spmv");                                   \
    return SPX_OK;                                                 \
  }
  SPX_BCASE(1, 1) SPX_BCASE(1, 2) SPX_BCASE(1, 4) SPX_BCASE(1, 8)
  SPX_BCASE(2, 1) SPX_BCASE(2, 2) SPX_BCASE(2, 4) SPX_BCASE(2, 8)
  SPX_BCASE(4, 1) SPX_BCASE(4, 2) SPX_BCASE(4, 4) SPX_BCASE(4, 8)
  SPX_BCASE(8, 1) SPX_BCASE(8, 2) SPX_BCASE(8, 4) SPX_BCASE(8, 8)
#undef SPX_BCASE
  return fail(SPX_ERR_UNSUPPORTED, "bcsr_spmv: block %dx%d", a, b);
}

}  // namespace
}  // namespace spx

using namespace spx;

extern "C" spx_status bcsr_workspace_bytes(int32_t m, int32_t n, int32_t nnz, size_t* bytes) {
  if (!bytes || m < 0 || n < 0 || nnz < 0) return fail(SPX_ERR_INVALID, "bcsr_workspace_bytes: bad argument");
  carve_blocks(nullptr, nnz, bytes);
  return SPX_OK;
}

extern "C" spx_status csr_bcsr_count(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                                     const int32_t* colind, int32_t a, int32_t b, int32_t* nblocks_out,
                                     void* workspace, size_t ws_bytes, void* stream) {
  if (m < 0 || n < 0 || nnz < 0) return fail(SPX_ERR_INVALID, "csr_bcsr_count: negative size");
  {
    const spx_status s_nnz = check_nnz(nnz, "csr_bcsr_count");
    if (s_nnz != SPX_OK) return s_nnz;
  }
  if (!shape_ok(a, b)) return fail(SPX_ERR_UNSUPPORTED, "csr_bcsr_count: block %dx%d (a, b in {1,2,4,8})", a, b);
  if (!nblocks_out || !rowptr || (nnz > 0 && !colind)) return fail(SPX_ERR_INVALID, "csr_bcsr_count: null pointer");
  size_t need = 0;
  BlockWs w = carve_blocks(workspace, nnz, &need);
  if (!workspace || ws_bytes < need)
    return fail(SPX_ERR_WORKSPACE, "csr_bcsr_count: workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t st = as_stream(stream);
  if (nnz == 0 || m == 0) {
    k_zero_i32<<<1, 64, 0, st>>>(nblocks_out, 1);
    SPX_LAUNCHED("k_zero_i32");
    return SPX_OK;
  }
  int cbits = 0;
  spx_status s = sort_blocks(m, n, nnz, rowptr, colind, a, b, w, &cbits, st);
  if (s != SPX_OK) return s;
  k_copy_i32<<<1, 1, 0, st>>>(w.total, nblocks_out);
  SPX_LAUNCHED("k_copy_i32");
  return SPX_OK;
}

extern "C" spx_status csr_to_bcsr(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr, const int32_t* colind,
                                  const double* values, int32_t a, int32_t b, int32_t bitmap, int32_t* browptr,
                                  int32_t* bcol, double* bvals, uint64_t* bmask, int32_t* boff, void* workspace,
                                  size_t ws_bytes, void* stream) {
  if (m < 0 || n < 0 || nnz < 0) return fail(SPX_ERR_INVALID, "csr_to_bcsr: negative size");
  {
    const spx_status s_nnz = check_nnz(nnz, "csr_to_bcsr");
    if (s_nnz != SPX_OK) return s_nnz;
  }
  if (!shape_ok(a, b)) return fail(SPX_ERR_UNSUPPORTED, "csr_to_bcsr: block %dx%d (a, b in {1,2,4,8})", a, b);
  if (!rowptr || !browptr || (nnz > 0 && (!colind || !values || !bcol || !bvals)) ||
      (bitmap && nnz > 0 && (!bmask || !boff)))
    return fail(SPX_ERR_INVALID, "csr_to_bcsr: null pointer");
  size_t need = 0;
  BlockWs w = carve_blocks(workspace, nnz, &need);
  if (!workspace || ws_bytes < need)
    return fail(SPX_ERR_WORKSPACE, "csr_to_bcsr: workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t st = as_stream(stream);
  const int32_t mb = (m + a - 1) / a;
  if (nnz == 0 || m == 0) {
    k_zero_i32<<<blocks_for(static_cast<int64_t>(mb) + 1), 256, 0, st>>>(browptr, static_cast<int64_t>(mb) + 1);
    SPX_LAUNCHED("k_zero_i32");
    return SPX_OK;
  }
  int cbits = 0;
  spx_status s = sort_blocks(m, n, nnz, rowptr, colind, a, b, w, &cbits, st);
  if (s != SPX_OK) return s;
  k_block_fill<<<blocks_for(nnz), 256, 0, st>>>(w.keys, w.src, w.rowid, w.index, colind, values, nnz, a, b, cbits,
                                                bitmap ? 1 : 0, bcol, w.brow, bvals, bmask, boff);
  SPX_LAUNCHED("k_block_fill");
  k_block_rowptr<<<blocks_for(static_cast<int64_t>(mb) + 1), 256, 0, st>>>(w.brow, w.total, mb, browptr);
  SPX_LAUNCHED("k_block_rowptr");
  return SPX_OK;
}

extern "C" spx_status bcsr_spmv(int32_t m, int32_t n, int32_t a, int32_t b, int32_t bitmap, int32_t nblocks,
                                const int32_t* browptr, const int32_t* bcol, const double* bvals,
                                const uint64_t* bmask, const int32_t* boff, const double* x, double* y,
                                int32_t lanes, void* stream) {
  if (m < 0 || n < 0 || nblocks < 0) return fail(SPX_ERR_INVALID, "bcsr_spmv: negative size");
  if (!shape_ok(a, b)) return fail(SPX_ERR_UNSUPPORTED, "bcsr_spmv: block %dx%d", a, b);
  if (m == 0) return SPX_OK;
  if (!browptr || !y || (nblocks > 0 && (!bcol || !bvals || !x)) || (bitmap && nblocks > 0 && (!bmask || !boff)))
    return fail(SPX_ERR_INVALID, "bcsr_spmv: null pointer");
  const int32_t mb = (m + a - 1) / a;
  if (lanes <= 0) {  // lanes per block row from the mean blocks per block row
    const double mean = static_cast<double>(nblocks) / mb;
    lanes = 1;
    while (lanes < 64 && lanes < mean) lanes <<= 1;
  }
  if (lanes > 64 || (lanes & (lanes - 1))) return fail(SPX_ERR_INVALID, "bcsr_spmv: lanes=%d", lanes);
  BcsrArgs p{browptr, bcol, bvals, bmask, boff, x, y, m, n, mb, lanes, 0};
  while ((1 << p.lane_shift) < lanes) ++p.lane_shift;
  const int64_t threads = static_cast<int64_t>(mb) * lanes;
  const int64_t grid = (threads + kWG - 1) / kWG;
  if (grid > 0x7fffffff) return fail(SPX_ERR_UNSUPPORTED, "bcsr_spmv: grid too large");
  hipStream_t st = as_stream(stream);
  return bitmap ? launch_bcsr<true>(a, b, p, static_cast<unsigned>(grid), st)
                : launch_bcsr<false>(a, b, p, static_cast<unsigned>(grid), st);
}
