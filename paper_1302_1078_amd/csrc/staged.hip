// staged.hip -- SpMM with each row tile's X window staged in LDS (the X
// reuse of Sec. 5: rows that share columns read the same rows of X).
//
// A staged plan cuts the rows into tiles of R consecutive rows, R = min(128 /
// KL, 64) (KL the lanes that cover one X row at the plan's k; each row gets
// 256 / R lanes, i.e. 256 / (R KL) slots).  At plan time every tile's
// distinct columns are sorted (a bitonic sort of (column, position) pairs in
// LDS, one workgroup per tile) into a column list, and each nonzero gets the
// 16-bit index of its column in that list.  A product then runs one
// workgroup per tile:
//   1. every load the tile needs -- its window (X rows tcols[0..U), 16-byte
//      vectors), its values, window indices and row pointers -- is issued
//      at once, then written to LDS (one global round trip per tile);
//   2. each row's lanes walk its nonzeros reading index, value and X only
//      from LDS, U nonzeros per slot and round, and reduce across slots.
// X rows are then fetched once per tile instead of once per nonzero: for the
// 27-point stencil 2.4-2.9 times fewer.  Tiles with more than 2,048 nonzeros
// or a window above 32 KB gather X from memory instead, with the same lane
// layout.  Results are deterministic; each slot sums its nonzeros in
// ascending position order and slots are reduced in a fixed order.  Staged
// plans need k to be a multiple of the 16-byte vector (2 FP64 or 4 FP32
// elements).  The tile size trades reuse against workgroups per CU: a
// workgroup waits for its tile's loads before computing, so the kernel
// needs several resident workgroups per CU to keep memory busy (32 KB
// windows and R = 128 / KL measured faster than 64 KB and 256 / KL).
#include <algorithm>
#include <new>
#include <vector>

#include "product_impl.hpp"

namespace spx {

namespace {

using namespace prod;

constexpr int kSortN = 2048;                   // nonzeros per staged tile (the plan sorts them in LDS)
constexpr int kSortPer = kSortN / kWG;         // keys per thread
constexpr int kWindowBytes = 32 * 1024;        // LDS budget of one window
constexpr int kMaxTileRows = 64;
constexpr int kWinVec = kWindowBytes / (16 * kWG);  // window vectors per thread (16 B each)
constexpr int kNzPer = kSortN / kWG;                // staged nonzeros per thread
constexpr uint64_t kPadKey = ~uint64_t(0);

// ---------------------------------------------------------------- plan

// Sorts the keys (column << 32 | local position) of one tile in LDS, padded
// to the power of two np >= n; then flags the first key of each column and
// scans the flags.  On return rank[i] (i < n) is the window index of key i's
// column and the function returns the number of distinct columns.
__device__ int32_t tile_sort_rank(uint64_t* s_key, int32_t* s_rank, int32_t* s_wsum, int n) {
  int np = 1;
  while (np < n) np <<= 1;
  for (int kk = 2; kk <= np; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int q = threadIdx.x; q < (np >> 1); q += kWG) {
        const int i = 2 * j * (q / j) + (q % j);
        const int l = i + j;
        const bool up = (i & kk) == 0;
        const uint64_t x = s_key[i], y = s_key[l];
        if ((x > y) == up) {
          s_key[i] = y;
          s_key[l] = x;
        }
      }
      __syncthreads();
    }
  }
  // flags of column starts, scanned: thread t owns keys [t * kSortPer, (t + 1) * kSortPer)
  const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
  int32_t mine = 0;
  for (int e = 0; e < kSortPer; ++e) {
    const int i = t * kSortPer + e;
    if (i < n) mine += (i == 0 || (s_key[i] >> 32) != (s_key[i - 1] >> 32)) ? 1 : 0;
  }
  int32_t inc = mine;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t u = __shfl_up(inc, off, kWave);
    if (lane >= off) inc += u;
  }
  if (lane == kWave - 1) s_wsum[w] = inc;
  __syncthreads();
  int32_t run = inc - mine, total = 0;
  for (int v = 0; v < kWG / kWave; ++v) {
    if (v < w) run += s_wsum[v];
    total += s_wsum[v];
  }
  for (int e = 0; e < kSortPer; ++e) {
    const int i = t * kSortPer + e;
    if (i < n) {
      run += (i == 0 || (s_key[i] >> 32) != (s_key[i - 1] >> 32)) ? 1 : 0;
      s_rank[i] = run - 1;
    }
  }
  __syncthreads();
  return total;
}

struct TileRange {
  int32_t p0, n;
};

__device__ __forceinline__ TileRange tile_range(const int32_t* rowptr, int32_t m, int32_t R, int32_t t) {
  const int64_t r0 = static_cast<int64_t>(t) * R;
  const int64_t r1 = r0 + R < m ? r0 + R : m;
  TileRange tr;
  tr.p0 = rowptr[r0];
  tr.n = rowptr[r1] - tr.p0;
  return tr;
}

// Window size of every tile (-1: not staged).
__global__ __launch_bounds__(kWG) void k_stage_count(const int32_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ colind, int32_t m, int32_t R,
                                                     int32_t umax, int32_t* __restrict__ tile_cols,
                                                     int32_t* __restrict__ counts, int32_t* __restrict__ tile_nnz) {
  __shared__ uint64_t s_key[kSortN];
  __shared__ int32_t s_rank[kSortN];
  __shared__ int32_t s_wsum[kWG / kWave];
  const int32_t t = blockIdx.x;
  const TileRange tr = tile_range(rowptr, m, R, t);
  if (threadIdx.x == 0) tile_nnz[t] = tr.n;
  if (tr.n > kSortN) {
    if (threadIdx.x == 0) {
      tile_cols[t] = -1;
      counts[t] = 0;
    }
    return;
  }
  for (int i = threadIdx.x; i < kSortN; i += kWG)
    s_key[i] = (i < tr.n) ? (static_cast<uint64_t>(static_cast<uint32_t>(colind[tr.p0 + i])) << 32) | i : kPadKey;
  __syncthreads();
  const int32_t u = tile_sort_rank(s_key, s_rank, s_wsum, tr.n);
  if (threadIdx.x == 0) {
    const bool ok = u <= umax;
    tile_cols[t] = ok ? u : -1;
    counts[t] = ok ? u : 0;
  }
}

// Column lists and window indices of the staged tiles.
__global__ __launch_bounds__(kWG) void k_stage_fill(const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ colind, int32_t m, int32_t R,
                                                    const int32_t* __restrict__ tile_cols,
                                                    const int32_t* __restrict__ tile_off, int32_t* __restrict__ tcols,
                                                    uint16_t* __restrict__ loc) {
  __shared__ uint64_t s_key[kSortN];
  __shared__ int32_t s_rank[kSortN];
  __shared__ int32_t s_wsum[kWG / kWave];
  const int32_t t = blockIdx.x;
  if (tile_cols[t] <= 0) return;  // uniform: not staged, or no nonzeros
  const TileRange tr = tile_range(rowptr, m, R, t);
  for (int i = threadIdx.x; i < kSortN; i += kWG)
    s_key[i] = (i < tr.n) ? (static_cast<uint64_t>(static_cast<uint32_t>(colind[tr.p0 + i])) << 32) | i : kPadKey;
  __syncthreads();
  tile_sort_rank(s_key, s_rank, s_wsum, tr.n);
  const int32_t off = tile_off[t];
  for (int i = threadIdx.x; i < tr.n; i += kWG) {
    const uint64_t key = s_key[i];
    const int32_t r = s_rank[i];
    const int32_t pos = static_cast<int32_t>(key & 0xffffffffu);
    if (i == 0 || (key >> 32) != (s_key[i - 1] >> 32)) tcols[off + r] = static_cast<int32_t>(key >> 32);
    loc[tr.p0 + pos] = static_cast<uint16_t>(r);
  }
}

struct StageWs {
  int32_t* tile_cols;
  int32_t* tile_off;
  int32_t* tile_nnz;
  int32_t* tcols;
  uint16_t* loc;
  void* scan;
};

StageWs carve_stage(void* ws, int32_t m, int32_t nnz, int32_t R, size_t* bytes) {
  const int64_t ntiles = (static_cast<int64_t>(m) + R - 1) / R;
  Carve cv(ws, ~size_t(0));
  StageWs w;
  w.tile_cols = cv.take<int32_t>(ntiles + 1);
  w.tile_off = cv.take<int32_t>(ntiles + 1);
  w.tile_nnz = cv.take<int32_t>(ntiles + 1);
  w.tcols = cv.take<int32_t>(nnz > 0 ? nnz : 1);
  w.loc = cv.take<uint16_t>(nnz > 0 ? nnz : 1);
  w.scan = cv.take<char>(scan_workspace_bytes(ntiles + 1));
  *bytes = cv.used;
  return w;
}

size_t elem_bytes(spx_dtype t) { return t == SPX_F64 ? 8 : 4; }

// Lane layout of a staged plan: that of an SpMM with contiguous, 16-byte
// aligned X and Y (what the plan assumes; products check it).
void staged_layout(int32_t k, spx_dtype xt, int* kl, int* vec) {
  static const double dummy[2] = {0.0, 0.0};
  const void* aligned = reinterpret_cast<const void*>((reinterpret_cast<uintptr_t>(dummy) + 15) & ~uintptr_t(15));
  layout_for_k(k, xt, aligned, k, aligned, k, 0u, kl, vec);
}

constexpr int tile_rows_for(int kl) { return 128 / kl < kMaxTileRows ? 128 / kl : kMaxTileRows; }

spx_status staged_args(int32_t m, int32_t n, int32_t nnz, int32_t k, spx_dtype xt, int* R, const char* who) {
  if (m < 0 || n < 0 || nnz < 0) return fail(SPX_ERR_INVALID, "%s: negative size", who);
  const spx_status s = check_nnz(nnz, who);
  if (s != SPX_OK) return s;
  if (k < 1 || k > 128) return fail(SPX_ERR_UNSUPPORTED, "%s: k=%d outside [1, 128]", who, k);
  if (xt != SPX_F64 && xt != SPX_F32) return fail(SPX_ERR_UNSUPPORTED, "%s: X type %d", who, xt);
  int kl, vec;
  staged_layout(k, xt, &kl, &vec);
  if (vec == 1)
    return fail(SPX_ERR_UNSUPPORTED, "%s: k=%d is not a multiple of the 16-byte vector (%d elements)", who, k,
                xt == SPX_F64 ? 2 : 4);
  *R = tile_rows_for(kl);
  return SPX_OK;
}

// ---------------------------------------------------------------- product

struct StageTiles {
  int32_t m;
  int32_t ntiles;
  int32_t max_cols;  // LDS window capacity, X rows
  int32_t max_nnz;   // LDS capacity for a staged tile's values and indices
  const int32_t* tile_cols;
  const int32_t* tile_off;
  const int32_t* tcols;
  const uint16_t* loc;
};

// One row's nonzeros p0..p1 read straight from memory (a tile that is not
// staged): the group's S slots stride the row, U nonzeros per slot and round,
// lane kl of a slot loading index and value of element kl of the round and
// the slot's KL lanes sharing them.
template <class C, int S>
__device__ __forceinline__ void accumulate_direct(const ProdArgs& a, int32_t p0, int32_t p1, int slot, int col,
                                                  bool comp, typename C::AT (&acc)[C::VEC],
                                                  Comp (&cacc)[C::VEC]) {
  accumulate<C, S>(a, p0, p1, slot, col, comp, acc, cacc);
}

// The same from the tile's LDS copy: values sv[], window indices sl[] (both
// indexed from the tile's first nonzero), X rows in the window xs (stride k).
template <class C, int S>
__device__ __forceinline__ void accumulate_lds(const ProdArgs& a, const typename C::XT* sv, const uint16_t* sl,
                                               const typename C::XT* xs, int32_t q0, int32_t q1, int slot, int col,
                                               bool comp, typename C::AT (&acc)[C::VEC], Comp (&cacc)[C::VEC]) {
  using XT = typename C::XT;
  constexpr int VEC = C::VEC, U = C::U;
  const bool colok = col < a.k;
  const XT* Xb = xs + col;
  for (int32_t q = q0 + slot; q < q1; q += U * S) {
    bool h[U];
    int32_t c[U];
    XT v[U];
#pragma unroll
    for (int uu = 0; uu < U; ++uu) {
      h[uu] = q + uu * S < q1;
      c[uu] = h[uu] ? static_cast<int32_t>(sl[q + uu * S]) : 0;
      v[uu] = h[uu] ? sv[q + uu * S] : XT(0);
    }
    XT xv[U][VEC];
#pragma unroll
    for (int uu = 0; uu < U; ++uu) {
      if (h[uu] && colok) {
        load_x<XT, VEC>(Xb + c[uu] * a.k, xv[uu]);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) xv[uu][e] = XT(0);
      }
    }
    if (!C::kComp || !comp) {
#pragma unroll
      for (int uu = 0; uu < U; ++uu)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          if (h[uu]) acc[e] = fma_t(v[uu], xv[uu][e], acc[e]);
    } else if constexpr (C::kComp) {
#pragma unroll
      for (int uu = 0; uu < U; ++uu)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          if (h[uu]) cacc[e].add_prod(v[uu], xv[uu][e]);
    }
  }
}

// One workgroup per tile of R = min(256 / KL, 64) rows, S = 256 / (R KL)
// slots per row.  Dynamic LDS: the window (max_cols rows of k elements),
// then the tile's values (as XT), window indices and row offsets.
// DIRECT_ONLY: serve only the tiles that are not staged (beside the
// pipelined kernel, which serves the staged ones).
template <class C, bool DIRECT_ONLY>
__global__ __launch_bounds__(kWG) void k_staged(const ProdArgs a, const StageTiles st) {
  extern __shared__ __align__(16) unsigned char s_lds[];
  using XT = typename C::XT;
  using AT = typename C::AT;
  using VL = ValueLoad<typename C::VT>;
  constexpr int KL = C::KL, VEC = C::VEC;
  constexpr int R = tile_rows_for(KL);
  constexpr int GG = kWG / R;   // lanes per row
  constexpr int S = GG / KL;    // slots per row
  static_assert(VEC > 1 && S >= 1 && GG * R == kWG, "staged layout");
  const int t = (a.flags & SPX_FLAG_NO_XCD_MAP) ? static_cast<int>(blockIdx.x)
                                                : xcd_tile(blockIdx.x, gridDim.x);
  if (t >= st.ntiles) return;  // grid padding (uniform)
  XT* xs = reinterpret_cast<XT*>(s_lds);
  XT* sv = xs + static_cast<int64_t>(st.max_cols) * a.k;
  uint16_t* sl = reinterpret_cast<uint16_t*>(sv + st.max_nnz);
  int32_t* srp = reinterpret_cast<int32_t*>(sl + ((st.max_nnz + 1) & ~1));
  const int32_t r0 = t * R;
  const int32_t ucols = __builtin_amdgcn_readfirstlane(st.tile_cols[t]);
  const int tid = threadIdx.x;
  const int grp = tid / GG, ln = tid % GG, slot = ln / KL, kl = ln % KL;
  const int32_t row = r0 + grp;
  const bool active = row < st.m;
  const bool nt = !(a.flags & SPX_FLAG_NO_NT_STORE);
  if (DIRECT_ONLY && ucols >= 0) return;  // uniform
  if (ucols >= 0) {
    // ---- one round trip: window vectors, values, indices, row offsets
    const int32_t pb = __builtin_amdgcn_readfirstlane(a.rowptr[r0]);
    const int32_t rend = min(r0 + R, st.m);
    const int32_t nz = __builtin_amdgcn_readfirstlane(a.rowptr[rend]) - pb;
    const int lpr = a.k / VEC;  // 16-byte vectors per X row
    const int32_t nvec = ucols * lpr;
    const int32_t* cols = st.tcols + __builtin_amdgcn_readfirstlane(st.tile_off[t]);
    const XT* X = static_cast<const XT*>(a.X);
    typedef typename VecT<XT, VEC>::type V;
    V wv[kWinVec];
#pragma unroll
    for (int q = 0; q < kWinVec; ++q) {
      const int32_t i = q * kWG + tid;
      if (i < nvec) {
        const int32_t j = i / lpr, c = (i - j * lpr) * VEC;
        wv[q] = *reinterpret_cast<const V*>(X + static_cast<int64_t>(cols[j]) * a.ldx + c);
      }
    }
    typename VL::Raw vr[kNzPer];
    uint16_t lr[kNzPer];
#pragma unroll
    for (int q = 0; q < kNzPer; ++q) {
      const int32_t i = q * kWG + tid;
      if (i < nz) {
        vr[q] = VL::template raw<false>(static_cast<const typename C::VT*>(a.values) + pb + i);
        lr[q] = st.loc[pb + i];
      }
    }
    int32_t rp = 0;
    if (tid <= R) rp = a.rowptr[min(r0 + tid, st.m)] - pb;
#pragma unroll
    for (int q = 0; q < kWinVec; ++q) {
      const int32_t i = q * kWG + tid;
      if (i < nvec) *reinterpret_cast<V*>(xs + i * VEC) = wv[q];
    }
#pragma unroll
    for (int q = 0; q < kNzPer; ++q) {
      const int32_t i = q * kWG + tid;
      if (i < nz) {
        sv[i] = static_cast<XT>(VL::widen(vr[q]));
        sl[i] = lr[q];
      }
    }
    if (tid <= R) srp[tid] = rp;
    __syncthreads();
    // ---- rows from LDS
    const int32_t q0 = active ? srp[grp] : 0, q1 = active ? srp[grp + 1] : 0;
    const bool comp = C::kComp && (q1 - q0 > a.kahan_len);
    for (int c0 = 0; c0 < a.k; c0 += KL * VEC) {
      const int col = c0 + kl * VEC;
      AT acc[VEC];
      Comp cacc[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        acc[e] = AT(0);
        cacc[e].init();
      }
      accumulate_lds<C, S>(a, sv, sl, xs, q0, q1, slot, col, comp, acc, cacc);
      finish_small<C, GG>(a, active, comp, slot, col, row, acc, cacc, nt);
    }
  } else {
    int32_t p0 = 0, p1 = 0;
    if (active) {
      p0 = a.rowptr[row];
      p1 = a.rowptr[row + 1];
    }
    const bool comp = C::kComp && (p1 - p0 > a.kahan_len);
    for (int c0 = 0; c0 < a.k; c0 += KL * VEC) {
      const int col = c0 + kl * VEC;
      AT acc[VEC];
      Comp cacc[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        acc[e] = AT(0);
        cacc[e].init();
      }
      accumulate_direct<C, S>(a, p0, p1, slot, col, comp, acc, cacc);
      finish_small<C, GG>(a, active, comp, slot, col, row, acc, cacc, nt);
    }
  }
}

// ---------------------------------------------------------------- pipelined product
// Persistent, double-buffered variant.  Each workgroup walks a sequence of
// tiles (the tiles of one XCD taken in turn by its workgroups) with two LDS
// tile buffers and five wavefronts.  In step t
// the four compute wavefronts
//   1. issue the loads of tile t + 1 into the other buffer -- window, values,
//      window indices, row offsets -- as direct global-to-LDS loads
//      (global_load_lds: no registers in between), and the column list of
//      tile t + 2, which addresses the next step's window loads;
//   2. compute tile t from LDS and leave its rows' results in an LDS output
//      buffer;
//   3. wait for their own loads and meet at the step's barrier.
// The fifth wavefront writes the previous step's results from LDS to Y.
// Why the split: a wavefront's vector-memory counter counts loads and stores
// together and completes in order, so a wavefront that waits for a prefetch
// would also wait for its own earlier stores.  The compute wavefronts issue
// no global store and no global load besides the prefetch, so waiting for
// their counter is waiting for the prefetch; the storing wavefront never
// waits.  The barrier is a bare s_barrier behind lgkmcnt(0) (a release
// fence would wait for every outstanding access).
// LDS bytes per element: window 16-byte vectors as stored; values 8 (FP64)
// or 4 (FP32; BF16 lands zero-extended in 4: 2-byte loads to LDS write one
// dword per lane); window indices 4; row offsets 4; column list 4; results
// as XT, R rows of k.
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glb_void;

constexpr int kPipeThreads = kWG + kWave;  // four compute wavefronts and the storing one

struct PipeLayout {
  int32_t win, val, loc, rp, buf;  // byte offsets inside one tile buffer, and its size (whole rounds of loads)
  int32_t cols, colbuf;            // the two column-list buffers: offset of the first, size of each
  int32_t out, outbuf;             // the two result buffers: offset of the first, size of each
  int32_t grid;                    // persistent workgroups
};

__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
// This wavefront's global-to-LDS loads have landed, then the barrier.  Inline
// asm, since the compiler's wait insertion may drop a builtin wait it does
// not see a register reason for.
__device__ __forceinline__ void loads_barrier() {
  asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// 4-byte words [0, words) of src into LDS dst, one word per thread and round
// of the 256 compute threads; threads past `words` read src[0] into the
// round's padding.
__device__ __forceinline__ void dma_words(const uint32_t* src, int32_t words, unsigned char* dst, int tid) {
  const int w = tid / kWave;
  for (int32_t r = 0; r * kWG < words; ++r) {
    const int32_t e = r * kWG + tid;
    __builtin_amdgcn_global_load_lds((glb_void*)(src + (e < words ? e : 0)),
                                     (lds_void*)(dst + (r * kWG + w * kWave) * 4), 4, 0, 0);
  }
}
// The same for 2-byte elements (each lands zero-extended in a dword).
__device__ __forceinline__ void dma_halves(const uint16_t* src, int32_t n, unsigned char* dst, int tid) {
  const int w = tid / kWave;
  for (int32_t r = 0; r * kWG < n; ++r) {
    const int32_t e = r * kWG + tid;
    __builtin_amdgcn_global_load_lds((glb_void*)(src + (e < n ? e : 0)),
                                     (lds_void*)(dst + (r * kWG + w * kWave) * 4), 2, 0, 0);
  }
}

template <class C>
__device__ __forceinline__ typename C::XT lds_value(const unsigned char* val, int32_t e) {
  using VT = typename C::VT;
  if constexpr (sizeof(VT) == 8) return reinterpret_cast<const double*>(val)[e];
  else if constexpr (sizeof(VT) == 4) return reinterpret_cast<const float*>(val)[e];
  else return bf16_to_f32(static_cast<uint16_t>(reinterpret_cast<const uint32_t*>(val)[e]));
}

// A row's nonzeros q0..q1 (tile-relative) from the LDS buffer: as
// accumulate_lds, with the values and window indices in their DMA layout.
template <class C, int S>
__device__ __forceinline__ void accumulate_pipe(const ProdArgs& a, const unsigned char* val, const uint32_t* loc,
                                                const typename C::XT* xs, int32_t q0, int32_t q1, int slot, int col,
                                                bool comp, typename C::AT (&acc)[C::VEC], Comp (&cacc)[C::VEC]) {
  using XT = typename C::XT;
  constexpr int VEC = C::VEC, U = C::U;
  const bool colok = col < a.k;
  const XT* Xb = xs + col;
  for (int32_t q = q0 + slot; q < q1; q += U * S) {
    bool h[U];
    int32_t c[U];
    XT v[U];
#pragma unroll
    for (int uu = 0; uu < U; ++uu) {
      h[uu] = q + uu * S < q1;
      c[uu] = h[uu] ? static_cast<int32_t>(loc[q + uu * S]) : 0;
      v[uu] = h[uu] ? lds_value<C>(val, q + uu * S) : XT(0);
    }
    XT xv[U][VEC];
#pragma unroll
    for (int uu = 0; uu < U; ++uu) {
      if (h[uu] && colok) {
        load_x<XT, VEC>(Xb + c[uu] * a.k, xv[uu]);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) xv[uu][e] = XT(0);
      }
    }
    if (!C::kComp || !comp) {
#pragma unroll
      for (int uu = 0; uu < U; ++uu)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          if (h[uu]) acc[e] = fma_t(v[uu], xv[uu][e], acc[e]);
    } else if constexpr (C::kComp) {
#pragma unroll
      for (int uu = 0; uu < U; ++uu)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          if (h[uu]) cacc[e].add_prod(v[uu], xv[uu][e]);
    }
  }
}

// Tile record: window size (-1: not staged), column-list offset, first
// nonzero and nonzero count.  All wave-uniform, read through the constant
// address space (scalar loads, outside the vector-memory counter; the plan
// arrays and rowptr are not written while a product runs).
template <typename T>
__device__ __forceinline__ T ld_uniform(const T* p) {
  return *(const __attribute__((address_space(4))) T*)(p);
}

struct PipeTile {
  int32_t ucols, off, pb, nz;
};

__device__ __forceinline__ PipeTile pipe_tile(const ProdArgs& a, const StageTiles& st, int32_t R, int32_t t,
                                              bool valid) {
  PipeTile pt{-1, 0, 0, 0};
  if (!valid) return pt;
  const int32_t r0 = t * R;
  const int32_t r1 = min(r0 + R, st.m);
  pt.ucols = ld_uniform(st.tile_cols + t);
  pt.off = ld_uniform(st.tile_off + t);
  pt.pb = ld_uniform(a.rowptr + r0);
  pt.nz = ld_uniform(a.rowptr + r1) - pt.pb;
  return pt;
}

// The group's final sums of one row (as finish_small, into LDS instead of Y).
template <class C, int GG>
__device__ __forceinline__ void finish_to_lds(bool comp, int slot, int col, int32_t k, typename C::AT (&acc)[C::VEC],
                                              Comp (&cacc)[C::VEC], typename C::XT* orow) {
  constexpr int KL = C::KL, VEC = C::VEC;
  using XT = typename C::XT;
#pragma unroll
  for (int e = 0; e < VEC; ++e) acc[e] = group_sum<GG, KL>(acc[e]);
  double dsum[VEC] = {};
  if constexpr (C::kComp) {
    if (__any(comp)) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) dsum[e] = group_sum<GG, KL>(comp ? cacc[e].value() : 0.0);
    }
  }
  if (slot == 0 && col < k) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      if constexpr (C::kComp) orow[col + e] = comp ? static_cast<XT>(dsum[e]) : acc[e];
      else orow[col + e] = acc[e];
    }
  }
}

template <class C>
__global__ __launch_bounds__(kPipeThreads) void k_staged_pipe(const ProdArgs a, const StageTiles st,
                                                              const PipeLayout L) {
  extern __shared__ __align__(16) unsigned char s_lds[];
  using XT = typename C::XT;
  using AT = typename C::AT;
  using VT = typename C::VT;
  constexpr int KL = C::KL, VEC = C::VEC;
  constexpr int R = tile_rows_for(KL);
  constexpr int GG = kWG / R;   // lanes per row
  constexpr int S = GG / KL;    // slots per row
  static_assert(VEC > 1 && S >= 1 && GG * R == kWG, "staged layout");
  const int tid = threadIdx.x;
  // Tile order: XCD j (workgroups g = j mod 8, all resident at once) walks
  // the contiguous eighth j of the tiles, its workgroups taking consecutive
  // tiles in turn, so the tiles in flight on one XCD are neighbours and the
  // X rows they share stay in that XCD's L2.  Step i of this workgroup is
  // tile base + i * stride, for i < nsteps.
  const int g = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x));
  const int32_t H = L.grid / 8, j = g % 8, h = g / 8;
  const int32_t lo = static_cast<int32_t>((static_cast<int64_t>(st.ntiles) * j) / 8);
  const int32_t hi = static_cast<int32_t>((static_cast<int64_t>(st.ntiles) * (j + 1)) / 8);
  const int32_t base = __builtin_amdgcn_readfirstlane(lo + h), stride = H;
  const int32_t nsteps = __builtin_amdgcn_readfirstlane(base < hi ? (hi - base + H - 1) / H : 0);
  if (nsteps <= 0) return;
  auto tile_at = [&](int32_t i) { return base + i * stride; };
  // (LDS pointers are formed from s_lds by arithmetic only, so that the
  // compiler keeps them in the LDS address space)
  auto colbuf = [&](int cb) { return s_lds + L.cols + cb * L.colbuf; };
  auto tilebuf = [&](int b) { return s_lds + b * L.buf; };
  auto outbuf = [&](int b) { return reinterpret_cast<XT*>(s_lds + L.out + b * L.outbuf); };

  if (tid >= kWG) {
    // ---- the storing wavefront: during step t it writes the results of
    // tile t - 1, and after the last step those of the last tile.  It meets
    // the compute wavefronts at every barrier (two in the prologue, one per
    // step).
    const int lane = tid - kWG;
    const bool nt = !(a.flags & SPX_FLAG_NO_NT_STORE);
    auto store_tile = [&](int32_t ip) {
      const int32_t tp = tile_at(ip);
      if (ld_uniform(st.tile_cols + tp) < 0) return;  // served by k_staged
      const XT* o = outbuf(ip & 1);
      const int32_t rows = min(R, st.m - tp * R);
      XT* Y = static_cast<XT*>(a.Y) + static_cast<int64_t>(tp) * R * a.ldy;
      for (int32_t i = lane; i < rows * a.k; i += kWave) {
        const int32_t r = i / a.k, c = i - r * a.k;
        const XT v = o[i];
        if (nt) __builtin_nontemporal_store(v, Y + static_cast<int64_t>(r) * a.ldy + c);
        else Y[static_cast<int64_t>(r) * a.ldy + c] = v;
      }
    };
    lds_barrier();
    lds_barrier();
    for (int32_t i = 0; i < nsteps; ++i) {
      if (i > 0) store_tile(i - 1);
      lds_barrier();
    }
    store_tile(nsteps - 1);
    return;
  }

  // ---- the compute wavefronts
  const int lpr = a.k / VEC;  // 16-byte vectors per X row
  const XT* X = static_cast<const XT*>(a.X);
  const VT* values = static_cast<const VT*>(a.values);
  const int w = tid / kWave;
  auto issue_cols = [&](const PipeTile& pt, int cb) {
    if (pt.ucols > 0) dma_words(reinterpret_cast<const uint32_t*>(st.tcols + pt.off), pt.ucols, colbuf(cb), tid);
  };
  // window (addressed by the column list in column buffer cb), values,
  // window indices and row offsets of a staged tile into tile buffer b
  auto issue_tile = [&](const PipeTile& pt, int32_t t, int cb, int b) {
    unsigned char* buf = tilebuf(b);
    const int32_t* cl = reinterpret_cast<const int32_t*>(colbuf(cb));
    const int32_t nvec = pt.ucols * lpr;
    for (int32_t q = 0; q * kWG < nvec; ++q) {
      const int32_t i = q * kWG + tid;
      const int32_t j = i < nvec ? i / lpr : 0;
      const int32_t c = i < nvec ? (i - j * lpr) * VEC : 0;
      __builtin_amdgcn_global_load_lds((glb_void*)(X + static_cast<int64_t>(cl[j]) * a.ldx + c),
                                       (lds_void*)(buf + L.win + (q * kWG + w * kWave) * 16), 16, 0, 0);
    }
    if constexpr (sizeof(VT) == 2)
      dma_halves(reinterpret_cast<const uint16_t*>(values + pt.pb), pt.nz, buf + L.val, tid);
    else
      dma_words(reinterpret_cast<const uint32_t*>(values + pt.pb), pt.nz * static_cast<int32_t>(sizeof(VT) / 4),
                buf + L.val, tid);
    dma_halves(st.loc + pt.pb, pt.nz, buf + L.loc, tid);
    dma_words(reinterpret_cast<const uint32_t*>(a.rowptr + t * R), min(R + 1, st.m - t * R + 1), buf + L.rp, tid);
  };
  const int grp = tid / GG, ln = tid % GG, slot = ln / KL, kl = ln % KL;
  PipeTile cur = pipe_tile(a, st, R, tile_at(0), true);
  PipeTile nxt = pipe_tile(a, st, R, tile_at(1), nsteps > 1);
  // prologue: step 0's column list, then its data and step 1's column list
  issue_cols(cur, 0);
  loads_barrier();
  if (cur.ucols >= 0) issue_tile(cur, tile_at(0), 0, 0);
  issue_cols(nxt, 1);
  loads_barrier();
  for (int32_t i = 0; i < nsteps; ++i) {
    const int b = i & 1;
    const int32_t t = tile_at(i);
    const PipeTile nn = pipe_tile(a, st, R, tile_at(i + 2), i + 2 < nsteps);
    // 1. prefetch: step i + 1's tile (column list in column buffer b ^ 1),
    //    and the column list of step i + 2 into column buffer b
    if (nxt.ucols >= 0) issue_tile(nxt, tile_at(i + 1), b ^ 1, b ^ 1);
    issue_cols(nn, b);
    // 2. tile t from buffer b into result buffer b
    if (cur.ucols >= 0) {
      const unsigned char* buf = tilebuf(b);
      const XT* xs = reinterpret_cast<const XT*>(buf + L.win);
      const unsigned char* val = buf + L.val;
      const uint32_t* loc = reinterpret_cast<const uint32_t*>(buf + L.loc);
      const int32_t* srp = reinterpret_cast<const int32_t*>(buf + L.rp);
      const bool active = t * R + grp < st.m;
      const int32_t q0 = active ? srp[grp] - cur.pb : 0, q1 = active ? srp[grp + 1] - cur.pb : 0;
      const bool comp = C::kComp && (q1 - q0 > a.kahan_len);
      XT* orow = outbuf(b) + grp * a.k;
      for (int c0 = 0; c0 < a.k; c0 += KL * VEC) {
        const int col = c0 + kl * VEC;
        AT acc[VEC];
        Comp cacc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          acc[e] = AT(0);
          cacc[e].init();
        }
        accumulate_pipe<C, S>(a, val, loc, xs, q0, q1, slot, col, comp, acc, cacc);
        finish_to_lds<C, GG>(comp, slot, col, a.k, acc, cacc, orow);
      }
    }
    // 3. the prefetch has landed (this wavefront's counter holds nothing else)
    loads_barrier();
    cur = nxt;
    nxt = nn;
  }
}

template <class C, bool DIRECT_ONLY>
spx_status launch_kc(const ProdArgs& a, const StageTiles& s, size_t lds, hipStream_t st) {
  const int64_t grid = (static_cast<int64_t>(s.ntiles) + 7) / 8 * 8;
  if (grid > 0x7fffffff) return fail(SPX_ERR_UNSUPPORTED, "staged product: grid too large");
  if (DIRECT_ONLY) lds = 0;
  if (lds > 0)
    SPX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_staged<C, DIRECT_ONLY>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  k_staged<C, DIRECT_ONLY><<<static_cast<unsigned>(grid), kWG, lds, st>>>(a, s);
  SPX_LAUNCHED("k_staged");
  return SPX_OK;
}

// LDS buffers of the pipelined kernel, sized to the plan's largest staged
// tile, and a persistent grid of as many workgroups as fit on the device.
template <class C>
spx_status launch_pipe(const ProdArgs& a, const StageTiles& s, int32_t tile_rows, hipStream_t st) {
  const int64_t xb = sizeof(typename C::XT);
  const int64_t vb = sizeof(typename C::VT) == 8 ? 8 : 4;
  // every region holds whole rounds of loads (lanes past the end write padding)
  auto rounds = [](int64_t elems, int64_t bytes_per_lane) {
    return ((elems + kWG - 1) / kWG) * kWG * bytes_per_lane;
  };
  PipeLayout L;
  L.win = 0;
  L.val = static_cast<int32_t>(rounds(static_cast<int64_t>(s.max_cols) * (a.k * xb / 16), 16));
  L.loc = L.val + static_cast<int32_t>(rounds(static_cast<int64_t>(s.max_nnz) * (vb / 4), 4));
  L.rp = L.loc + static_cast<int32_t>(rounds(s.max_nnz, 4));
  L.buf = L.rp + static_cast<int32_t>(rounds(tile_rows + 1, 4));
  L.cols = 2 * L.buf;
  L.colbuf = static_cast<int32_t>(rounds(s.max_cols, 4));
  L.out = L.cols + 2 * L.colbuf;
  L.outbuf = static_cast<int32_t>((static_cast<int64_t>(tile_rows) * a.k * xb + 15) & ~int64_t(15));
  const size_t lds = static_cast<size_t>(L.out) + 2 * static_cast<size_t>(L.outbuf);
  const void* fn = reinterpret_cast<const void*>(&k_staged_pipe<C>);
  SPX_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  int dev = 0, cus = 0, per_cu = 0;
  SPX_HIP(hipGetDevice(&dev));
  SPX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  SPX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kPipeThreads, lds));
  if (per_cu < 1) return fail(SPX_ERR_UNSUPPORTED, "staged product: %zu B of LDS per workgroup do not fit", lds);
  // all workgroups resident at once, a multiple of the 8 XCDs (8 at least)
  L.grid = static_cast<int32_t>(std::max<int64_t>(8, (static_cast<int64_t>(cus) * per_cu) / 8 * 8));
  k_staged_pipe<C><<<static_cast<unsigned>(L.grid), kPipeThreads, lds, st>>>(a, s, L);
  SPX_LAUNCHED("k_staged_pipe");
  return SPX_OK;
}

template <class C>
spx_status launch_staged_kernel(const ProdArgs& a, const StageTiles& s, size_t lds, int32_t tile_rows,
                                int32_t nstaged, bool pipelined, hipStream_t st) {
  if (!pipelined) return launch_kc<C, false>(a, s, lds, st);
  if (nstaged > 0) {
    const spx_status r = launch_pipe<C>(a, s, tile_rows, st);
    if (r != SPX_OK) return r;
  }
  if (nstaged < s.ntiles) return launch_kc<C, true>(a, s, lds, st);
  return SPX_OK;
}

template <typename VT, typename XT, int VECMAX>
spx_status launch_vt_staged(const ProdArgs& a, const StageTiles& s, size_t lds, int32_t tile_rows, int32_t nstaged,
                            bool pipelined, int kl, int vec, hipStream_t st) {
#define SPX_CASE(KL_, VEC_)                                                                      \
  if (kl == KL_ && vec == VEC_)                                                                  \
    return launch_staged_kernel<Cfg<VT, XT, KL_, VEC_>>(a, s, lds, tile_rows, nstaged, pipelined, st);
  SPX_CASE(1, VECMAX) SPX_CASE(2, VECMAX) SPX_CASE(4, VECMAX) SPX_CASE(8, VECMAX)
  SPX_CASE(16, VECMAX) SPX_CASE(32, VECMAX)
#undef SPX_CASE
  return fail(SPX_ERR_UNSUPPORTED, "no staged kernel for KL=%d VEC=%d", kl, vec);
}

}  // namespace

spx_status launch_staged(ProdArgs& a, const spx_plan* p, int32_t m, int vt, int xt, int kl, int vec,
                         hipStream_t st) {
  if (kl != p->kl || vec != p->vec || a.k != p->k || xt != p->xtype)
    return fail(SPX_ERR_UNSUPPORTED,
                "staged plan built for k=%d (X type %d, %d lanes x %d elements per X row); the call has "
                "k=%lld, X type %d, %d x %d (X and Y need 16-byte loads: aligned, ld a multiple of the vector)",
                p->k, p->xtype, p->kl, p->vec, static_cast<long long>(a.k), xt, kl, vec);
  a.kahan_len = p->opts.kahan_len;
  a.flags = p->opts.flags;
  StageTiles s{m, p->ntiles, p->max_cols, p->max_nnz, p->tile_cols, p->tile_off, p->tcols, p->loc};
  const size_t xb = elem_bytes(static_cast<spx_dtype>(xt));
  const size_t lds = (static_cast<size_t>(p->max_cols) * p->k + p->max_nnz) * xb +
                     static_cast<size_t>((p->max_nnz + 1) & ~1) * 2 + static_cast<size_t>(p->tile_rows + 1) * 4;
  if (p->ntiles == 0) return SPX_OK;
  const int32_t R = p->tile_rows, ns = p->nstaged;
  const bool pl = p->staged == 2;
  if (vt == SPX_F64 && xt == SPX_F64) return launch_vt_staged<double, double, 2>(a, s, lds, R, ns, pl, kl, vec, st);
  if (vt == SPX_F32 && xt == SPX_F32) return launch_vt_staged<float, float, 4>(a, s, lds, R, ns, pl, kl, vec, st);
  if (vt == SPX_BF16 && xt == SPX_F32)
    return launch_vt_staged<uint16_t, float, 4>(a, s, lds, R, ns, pl, kl, vec, st);
  return fail(SPX_ERR_UNSUPPORTED, "staged product: dtype pair (%d, %d)", vt, xt);
}

}  // namespace spx

using namespace spx;

extern "C" spx_status csr_plan_staged_workspace_bytes(int32_t m, int32_t n, int32_t nnz, int32_t k,
                                                      spx_dtype xtype, size_t* bytes) {
  if (!bytes) return fail(SPX_ERR_INVALID, "csr_plan_staged_workspace_bytes: bytes is null");
  int R = 0;
  const spx_status s = staged_args(m, n, nnz, k, xtype, &R, "csr_plan_staged_workspace_bytes");
  if (s != SPX_OK) return s;
  carve_stage(nullptr, m, nnz, R, bytes);
  return SPX_OK;
}

extern "C" spx_status csr_plan_create_staged(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                                             const int32_t* colind, int32_t k, spx_dtype xtype,
                                             void* workspace, size_t ws_bytes, void* stream, spx_plan** out) {
  const char* who = "csr_plan_create_staged";
  if (!out) return fail(SPX_ERR_INVALID, "%s: out is null", who);
  *out = nullptr;
  int R = 0;
  spx_status s = staged_args(m, n, nnz, k, xtype, &R, who);
  if (s != SPX_OK) return s;
  if (m > 0 && !rowptr) return fail(SPX_ERR_INVALID, "%s: rowptr is null", who);
  if (nnz > 0 && !colind) return fail(SPX_ERR_INVALID, "%s: colind is null", who);
  size_t need = 0;
  carve_stage(nullptr, m, nnz, R, &need);
  if (!workspace || ws_bytes < need)
    return fail(SPX_ERR_WORKSPACE, "%s: workspace %zu < %zu bytes", who, ws_bytes, need);
  hipStream_t st = as_stream(stream);
  StageWs w = carve_stage(workspace, m, nnz, R, &need);
  const int32_t ntiles = static_cast<int32_t>((static_cast<int64_t>(m) + R - 1) / R);
  const int64_t row_bytes = static_cast<int64_t>(k) * elem_bytes(xtype);
  const int32_t umax = static_cast<int32_t>(std::min<int64_t>(kWindowBytes / row_bytes, 65536));
  if (ntiles > 0) {
    int32_t* counts = w.tile_off;  // clamped window sizes, scanned in place below
    k_stage_count<<<static_cast<unsigned>(ntiles), kWG, 0, st>>>(rowptr, colind, m, R, umax, w.tile_cols, counts,
                                                                 w.tile_nnz);
    SPX_LAUNCHED("k_stage_count");
    s = exclusive_scan_i32(counts, w.tile_off, ntiles, w.tile_off + ntiles, w.scan, st);
    if (s != SPX_OK) return s;
    k_stage_fill<<<static_cast<unsigned>(ntiles), kWG, 0, st>>>(rowptr, colind, m, R, w.tile_cols, w.tile_off,
                                                                w.tcols, w.loc);
    SPX_LAUNCHED("k_stage_fill");
  }
  std::vector<int32_t> cols(static_cast<size_t>(ntiles)), tnnz(static_cast<size_t>(ntiles));
  if (ntiles > 0) {
    SPX_HIP(hipMemcpyAsync(cols.data(), w.tile_cols, sizeof(int32_t) * ntiles, hipMemcpyDeviceToHost, st));
    SPX_HIP(hipMemcpyAsync(tnnz.data(), w.tile_nnz, sizeof(int32_t) * ntiles, hipMemcpyDeviceToHost, st));
    SPX_HIP(hipStreamSynchronize(st));
  }
  spx_plan* p = new (std::nothrow) spx_plan();
  if (!p) return fail(SPX_ERR_INVALID, "%s: out of host memory", who);
  p->m = m;
  p->n = n;
  p->nnz = nnz;
  spx_plan_default_opts(k, xtype == SPX_F64 ? SPX_F64 : SPX_F32, &p->opts);
  p->opts.nbins = 1;
  p->opts.max_k = k;
  p->staged = 1;
  p->k = k;
  p->xtype = xtype;
  staged_layout(k, xtype, &p->kl, &p->vec);
  p->tile_rows = R;
  p->ntiles = ntiles;
  p->nstaged = 0;
  p->max_cols = 0;
  p->max_nnz = 0;
  for (int32_t i = 0; i < ntiles; ++i) {
    if (cols[i] < 0) continue;
    ++p->nstaged;
    p->max_cols = std::max(p->max_cols, cols[i]);
    p->max_nnz = std::max(p->max_nnz, tnnz[i]);
  }
  p->tile_cols = w.tile_cols;
  p->tile_off = w.tile_off;
  p->tcols = w.tcols;
  p->loc = w.loc;
  *out = p;
  return SPX_OK;
}

extern "C" spx_status csr_plan_staged_pipeline(spx_plan* p, int32_t enable) {
  if (!p) return fail(SPX_ERR_INVALID, "csr_plan_staged_pipeline: plan is null");
  if (!p->staged) return fail(SPX_ERR_INVALID, "csr_plan_staged_pipeline: not a staged plan");
  p->staged = enable ? 2 : 1;
  return SPX_OK;
}

extern "C" spx_status csr_plan_staged_info(const spx_plan* p, int32_t* tile_rows, int32_t* ntiles,
                                           int32_t* nstaged, int32_t* max_cols) {
  if (!p) return fail(SPX_ERR_INVALID, "csr_plan_staged_info: plan is null");
  if (!p->staged) return fail(SPX_ERR_INVALID, "csr_plan_staged_info: not a staged plan");
  if (tile_rows) *tile_rows = p->tile_rows;
  if (ntiles) *ntiles = p->ntiles;
  if (nstaged) *nstaged = p->nstaged;
  if (max_cols) *max_cols = p->max_cols;
  return SPX_OK;
}
