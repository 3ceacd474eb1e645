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
// group reduces its A partial sums.  The multi-vector product (a x 1 dense
// blocks) lays lanes out as the CSR SpMM does, KL lanes x VEC columns per X
// row and S slots walking a block row's blocks, and keeps a x VEC
// accumulators per lane, so each X row gathered serves a rows of Y.
#include <algorithm>
#include <type_traits>

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

// ---------------------------------------------------------------- multi-vector product

template <typename T, int N>
struct VecOf {
  typedef T type __attribute__((ext_vector_type(N)));
};

// VEC consecutive elements of an X row (16-byte aligned when VEC > 1)
template <typename T, int VEC>
__device__ __forceinline__ void ld_xrow(const T* q, T (&out)[VEC]) {
  if constexpr (VEC == 1) {
    out[0] = *q;
  } else {
    const typename VecOf<T, VEC>::type w = *reinterpret_cast<const typename VecOf<T, VEC>::type*>(q);
#pragma unroll
    for (int e = 0; e < VEC; ++e) out[e] = w[e];
  }
}

// a block value as 32 bits for the cross-lane moves (BF16: its bits)
__device__ __forceinline__ int32_t to_lane(float v) { return __float_as_int(v); }
__device__ __forceinline__ int32_t to_lane(uint16_t v) { return static_cast<int32_t>(v); }
template <typename VT>
__device__ __forceinline__ float from_lane(int32_t v) {
  if constexpr (std::is_same<VT, float>::value) return __int_as_float(v);
  else return bf16_to_f32(static_cast<uint16_t>(v));
}

struct BcsrMmArgs {
  const int32_t* browptr;
  const int32_t* bcol;
  const void* bvals;  // VT
  const void* X;      // XT, offset to this launch's first column
  void* Y;            // XT, likewise
  int64_t ldx, ldy;
  int32_t m, mb, k;  // k: columns of this launch (a slab of at most KL x VEC)
  int32_t slots;     // S: slots per block row, S x KL <= 64
  int32_t pb;        // 0, or a period of pb block rows: XCD j serves band j of every period
};

// Block row served by group g (in launch order) of workgroup b.  Without a
// period: the j-th eighth of the block rows on XCD j (workgroup b runs on
// XCD b mod 8).  With a period of pb block rows: XCD j serves band j,
// R mod pb in [ceil(j pb / 8), ceil((j + 1) pb / 8)), in ascending order, so
// the block rows that share X rows across neighbouring periods meet in one
// L2 (the row period of the CSR plans, computed instead of listed).
// Returns -1 past the end.
__device__ __forceinline__ int64_t bcsr_block_row(const BcsrMmArgs& p, int64_t b, int64_t nb, int64_t g,
                                                  int64_t groups_per_wg) {
  if (p.pb <= 0) {
    const int64_t R = static_cast<int64_t>(xcd_tile(static_cast<int>(b), static_cast<int>(nb))) * groups_per_wg + g;
    return R < p.mb ? R : -1;
  }
  const int64_t j = b & 7, i = (b >> 3) * groups_per_wg + g;  // i-th block row of band j
  const int64_t lo = (j * p.pb + 7) / 8, hi = ((j + 1) * p.pb + 7) / 8;
  const int64_t w = hi - lo;
  if (w <= 0) return -1;
  const int64_t R = (i / w) * p.pb + lo + i % w;
  return R < p.mb ? R : -1;
}

// Y[A R + r, :] = sum over the blocks q of block row R of bvals[A q + r] X[bcol[q], :].
// Every round a slot takes U blocks (q, q + S, ...); the KL lanes of the
// slot share that round's block columns and values: lane kl loads items kl,
// kl + KL, ... and the slot reads them back with cross-lane moves, so the
// address unit sees one lane per item instead of KL.  The next round's
// columns and values are loaded after this round's X gathers are issued:
// loads complete in issue order, so waiting for the gathers does not wait
// for them, and a round costs one memory round trip instead of two.
template <typename VT, typename XT, int A, int KL, int VEC>
__global__ __launch_bounds__(kWG) void k_bcsr_spmm(const BcsrMmArgs p) {
  // FP64 values: FP64 throughout.  FP32 / BF16 values with FP32 X: FP32
  // products and sums (no compensated sums: blocked storage serves banded
  // matrices, whose rows are short)
  constexpr int U = (A >= 8) ? 2 : 4;
  constexpr bool kF64 = std::is_same<VT, double>::value;
  using Lane = typename std::conditional<kF64, double, int32_t>::type;  // a value as moved across lanes
  const VT* bvals = static_cast<const VT*>(p.bvals);
  const XT* X = static_cast<const XT*>(p.X);
  constexpr int PC = (U + KL - 1) / KL;      // block columns per lane
  constexpr int PV = (U * A + KL - 1) / KL;  // values per lane
  const int S = p.slots;
  const int G = S * KL;
  const int t = threadIdx.x, lane = t % kWave;
  const int64_t R = bcsr_block_row(p, blockIdx.x, gridDim.x, t / G, kWG / G);
  const int kl = lane % KL, slot = (lane % G) / KL;
  const int sbase = lane - kl;
  const int col = kl * VEC;
  const bool active = R >= 0;
  const bool colok = col < p.k;
  XT acc[A][VEC];
#pragma unroll
  for (int r = 0; r < A; ++r)
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[r][e] = XT(0);
  int32_t q0 = 0, q1 = 0;
  if (active) {
    q0 = p.browptr[R];
    q1 = p.browptr[R + 1];
  }
  // block columns and values of the round starting at q (zero past q1)
  auto fetch = [&](int32_t q, int32_t (&cl)[PC], Lane (&vl)[PV]) {
#pragma unroll
    for (int j = 0; j < PC; ++j) {
      const int u = kl + j * KL;
      const int32_t qq = q + u * S;
      cl[j] = (u < U && qq < q1) ? __builtin_nontemporal_load(p.bcol + qq) : 0;
    }
#pragma unroll
    for (int j = 0; j < PV; ++j) {
      const int i = kl + j * KL, u = i / A, r = i % A;
      const int32_t qq = q + u * S;
      if constexpr (kF64)
        vl[j] = (i < U * A && qq < q1) ? __builtin_nontemporal_load(bvals + static_cast<int64_t>(qq) * A + r) : 0.0;
      else
        vl[j] = (i < U * A && qq < q1) ? to_lane(__builtin_nontemporal_load(bvals + static_cast<int64_t>(qq) * A + r))
                                       : 0;
    }
  };
  int32_t clA[PC];
  Lane vlA[PV];
  const int32_t qs = q0 + slot;
  if (qs < q1) fetch(qs, clA, vlA);
  for (int32_t q = qs; q < q1; q += U * S) {
    int32_t c[U];
    bool h[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      h[u] = q + u * S < q1;
      c[u] = __shfl(clA[u / KL], sbase + u % KL, kWave);
    }
    XT xv[U][VEC];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (h[u] && colok) {
        ld_xrow<XT, VEC>(X + static_cast<int64_t>(c[u]) * p.ldx + col, xv[u]);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) xv[u][e] = XT(0);
      }
    }
    const bool more = q + U * S < q1;  // the same for the KL lanes of a slot
    int32_t clB[PC];
    Lane vlB[PV];
    if (more) fetch(q + U * S, clB, vlB);
    XT v[U * A];
#pragma unroll
    for (int i = 0; i < U * A; ++i) {
      const Lane w = __shfl(vlA[i / KL], sbase + i % KL, kWave);
      if constexpr (kF64) v[i] = w;
      else v[i] = from_lane<VT>(w);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int r = 0; r < A; ++r)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          if (h[u]) acc[r][e] = fma_t(v[u * A + r], xv[u][e], acc[r][e]);
    if (more) {
#pragma unroll
      for (int j = 0; j < PC; ++j) clA[j] = clB[j];
#pragma unroll
      for (int j = 0; j < PV; ++j) vlA[j] = vlB[j];
    }
  }
  // slots of a block row are lanes KL apart inside one wavefront
#pragma unroll
  for (int r = 0; r < A; ++r)
#pragma unroll
    for (int e = 0; e < VEC; ++e)
      for (int off = KL; off < G; off <<= 1) acc[r][e] += __shfl_xor(acc[r][e], off, kWave);
  if (active && slot == 0 && colok) {
#pragma unroll
    for (int r = 0; r < A; ++r) {
      const int64_t row = R * A + r;
      if (row < p.m) {
        XT* y = static_cast<XT*>(p.Y) + row * p.ldy + col;
        if constexpr (VEC == 1) {
          y[0] = acc[r][0];
        } else {
          typename VecOf<XT, VEC>::type w;
#pragma unroll
          for (int e = 0; e < VEC; ++e) w[e] = acc[r][e];
          *reinterpret_cast<typename VecOf<XT, VEC>::type*>(y) = w;
        }
      }
    }
  }
}

template <typename VT, typename XT, int A, int V>
spx_status launch_bcsr_mm_a(int kl, int vec, const BcsrMmArgs& p, unsigned grid, hipStream_t st) {
#define SPX_MMCASE(KL_, VEC_)                                        \
  if (kl == KL_ && vec == VEC_) {                                    \
    k_bcsr_spmm<VT, XT, A, KL_, VEC_><<<grid, kWG, 0, st>>>(p);      \
    SPX_LAUNCHED("k_bcsr_spmm");                                     \
    return SPX_OK;                                                   \
  }
  SPX_MMCASE(1, 1) SPX_MMCASE(2, 1) SPX_MMCASE(4, 1) SPX_MMCASE(8, 1) SPX_MMCASE(16, 1) SPX_MMCASE(32, 1)
  SPX_MMCASE(1, V) SPX_MMCASE(2, V) SPX_MMCASE(4, V) SPX_MMCASE(8, V) SPX_MMCASE(16, V) SPX_MMCASE(32, V)
#undef SPX_MMCASE
  return fail(SPX_ERR_UNSUPPORTED, "bcsr_spmm: lanes %d x %d", kl, vec);
}

template <typename VT, typename XT, int V>
spx_status launch_bcsr_mm_t(int a, int kl, int vec, const BcsrMmArgs& p, unsigned grid, hipStream_t st) {
  if (a == 2) return launch_bcsr_mm_a<VT, XT, 2, V>(kl, vec, p, grid, st);
  if (a == 4) return launch_bcsr_mm_a<VT, XT, 4, V>(kl, vec, p, grid, st);
  return launch_bcsr_mm_a<VT, XT, 8, V>(kl, vec, p, grid, st);
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

extern "C" spx_status bcsr_spmm(int32_t m, int32_t n, int32_t a, int32_t b, int32_t nblocks,
                                const int32_t* browptr, const int32_t* bcol, const void* bvals, spx_dtype vtype,
                                int32_t k, const void* X, int64_t ldx, void* Y, int64_t ldy, spx_dtype xytype,
                                int32_t slots, int32_t row_period, void* stream) {
  if (m < 0 || n < 0 || nblocks < 0 || k < 0 || row_period < 0)
    return fail(SPX_ERR_INVALID, "bcsr_spmm: negative size or period");
  if (b != 1 || (a != 2 && a != 4 && a != 8))
    return fail(SPX_ERR_UNSUPPORTED, "bcsr_spmm: block %dx%d (a in {2, 4, 8}, b = 1, dense form)", a, b);
  const bool f64 = vtype == SPX_F64 && xytype == SPX_F64;
  if (!f64 && !((vtype == SPX_F32 || vtype == SPX_BF16) && xytype == SPX_F32))
    return fail(SPX_ERR_UNSUPPORTED, "bcsr_spmm: value / vector types (%d, %d)", vtype, xytype);
  if (m == 0 || k == 0) return SPX_OK;
  if (ldx < k || ldy < k) return fail(SPX_ERR_INVALID, "bcsr_spmm: ldx=%lld ldy=%lld < k=%d",
                                      static_cast<long long>(ldx), static_cast<long long>(ldy), k);
  if (!browptr || !Y || (nblocks > 0 && (!bcol || !bvals || !X))) return fail(SPX_ERR_INVALID, "bcsr_spmm: null pointer");
  const int32_t mb = (m + a - 1) / a;
  const int V = f64 ? 2 : 4;  // elements per 16-byte X load
  const size_t es = f64 ? 8 : 4;
  auto al16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
  const int vec = (k % V == 0 && ldx % V == 0 && ldy % V == 0 && al16(X) && al16(Y)) ? V : 1;
  const int width = 32 * vec;  // columns per launch
  hipStream_t st = as_stream(stream);
  for (int32_t c0 = 0; c0 < k; c0 += width) {
    const int32_t kc = (k - c0 < width) ? (k - c0) : width;
    const int per = (kc + vec - 1) / vec;
    int kl = 1;
    while (kl < per) kl <<= 1;
    int S = slots;
    if (S <= 0) {
      // About 16 lanes per block row (S x KL) measured best on the 27-point
      // stencil with FP64, FP32 and BF16 values at k = 8 to 32: 8 slots at 2
      // lanes per X row, 4 at 4, 2 at 8 and at 16 (one slot ran 1.2-2x
      // slower, so two at least); fewer when a block row holds less than a
      // round of blocks per slot
      const int U = (a >= 8) ? 2 : 4;
      const double mean = static_cast<double>(nblocks) / mb;
      S = (16 / kl > 2) ? 16 / kl : 2;
      if (S * kl > kWave) S = kWave / kl;
      while (S > 1 && S * U > mean) S >>= 1;
    }
    if ((S & (S - 1)) || S * kl > kWave)
      return fail(SPX_ERR_INVALID, "bcsr_spmm: slots=%d with %d lanes per X row (power of two, <= 64 lanes)", S, kl);
    // a period in block rows; one at least a block row beyond mb leaves the order ascending
    const int64_t pb = row_period > 0 ? (row_period + a - 1) / a : 0;
    // X may be null when there are no blocks (it is never read then)
    const void* Xc = X ? static_cast<const void*>(static_cast<const char*>(X) + c0 * es) : nullptr;
    BcsrMmArgs p{browptr, bcol, bvals, Xc, static_cast<char*>(Y) + c0 * es,
                 ldx, ldy, m, mb, kc, S, (pb > 0 && pb < mb) ? static_cast<int32_t>(pb) : 0};
    const int64_t per_wg = kWG / (S * kl);
    int64_t grid;
    if (p.pb > 0) {  // 8 x the workgroups of the largest band
      int64_t most = 0;
      for (int64_t j = 0; j < 8; ++j) {
        const int64_t lo = (j * p.pb + 7) / 8, hi = ((j + 1) * p.pb + 7) / 8;
        const int64_t rem = mb % p.pb;
        const int64_t nj = (mb / p.pb) * (hi - lo) + std::max<int64_t>(0, std::min(hi, rem) - lo);
        most = std::max(most, nj);
      }
      grid = 8 * ((most + per_wg - 1) / per_wg);
    } else {
      grid = (static_cast<int64_t>(mb) + per_wg - 1) / per_wg;
      grid = (grid + 7) / 8 * 8;  // whole eighths: XCD j serves the j-th eighth of the block rows
    }
    if (grid > 0x7fffffff) return fail(SPX_ERR_UNSUPPORTED, "bcsr_spmm: grid too large");
    const unsigned g = static_cast<unsigned>(grid);
    spx_status s = SPX_OK;
    if (f64) s = launch_bcsr_mm_t<double, double, 2>(a, kl, vec, p, g, st);
    else if (vtype == SPX_F32) s = launch_bcsr_mm_t<float, float, 4>(a, kl, vec, p, g, st);
    else s = launch_bcsr_mm_t<uint16_t, float, 4>(a, kl, vec, p, g, st);
    if (s != SPX_OK) return s;
  }
  return SPX_OK;
}
