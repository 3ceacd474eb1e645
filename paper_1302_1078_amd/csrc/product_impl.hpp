// product_impl.hpp -- device side of the row-group products, shared by the
// single-matrix launch (product.hip) and the persistent batched launch
// (batch.hip).  See product.hip for the design.
#pragma once

#include <type_traits>

#include "device.hpp"
#include "internal.hpp"

namespace spx {
namespace prod {

// Independent nonzeros per lane and round (SpMV; SPX_UNROLL_MM for SpMM).
// Both can be overridden at build time for unroll-depth sweeps.
#ifndef SPX_UNROLL
#define SPX_UNROLL 4
#endif
constexpr int kUnroll = SPX_UNROLL;
#ifndef SPX_UNROLL_MM
#define SPX_UNROLL_MM 4
#endif

// SAVE_: SpMV that also stores every gathered x[colind[p]] at xsave[p], so
// that the gradient with respect to the values (out[p] = dy[row(p)] x[colind[p]])
// can stream the operand instead of gathering it again.
// HOT_: SpMV through a plan with hot x attached: the column indices are the
// plan's copy, in which the H most-used columns appear as ~slot (negative);
// their x entries are read from the compact copy x_hot (ProdArgs::X2, filled
// per call), where 16 (FP64) or 32 (FP32) of them share a 128-byte line
// instead of one per line of x.
template <typename VT_, typename XT_, int KL_, int VEC_, bool SAVE_ = false, bool HOT_ = false>
struct Cfg {
  using VT = VT_;  // stored value type: double, float or uint16_t (bf16 bits)
  using XT = XT_;  // vector / dense type: double or float
  using AT = XT_;  // accumulation type of the plain path
  static constexpr int KL = KL_;
  static constexpr int VEC = VEC_;
  static constexpr bool kComp = std::is_same<XT_, float>::value;
  // SpMV streams colind / values non-temporally; SpMM row groups revisit
  // their lines (see ld_mat)
  static constexpr bool kNT = (KL_ * VEC_ == 1);
  static constexpr int U = (KL_ * VEC_ == 1) ? kUnroll : SPX_UNROLL_MM;
  static constexpr bool kSave = SAVE_;
  static constexpr bool kHot = HOT_;
  static_assert(!SAVE_ || KL_ * VEC_ == 1, "the saved gather is an SpMV (k = 1) feature");
  static_assert(!HOT_ || (KL_ * VEC_ == 1 && !SAVE_), "hot x is a plain SpMV (k = 1) feature");
  // look-ahead past a row's end is at most U x 256 slots (SPX_MAX_NNZ headroom)
  static_assert(U >= 1 && U * kWG <= 4096, "unroll depth");
};

template <typename T, int N>
struct VecT {
  typedef T type __attribute__((ext_vector_type(N)));
};

template <typename T, int N>
__device__ __forceinline__ void load_x(const T* p, T (&out)[N]) {
  if constexpr (N == 1) {
    out[0] = *p;
  } else {
    typedef typename VecT<T, N>::type V;
    V v = *reinterpret_cast<const V*>(p);
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = v[i];
  }
}

// G consecutive elements starting at p, G x sizeof(T) <= 16 bytes and p
// aligned to that size: one load.
template <bool NT, int G, typename T>
__device__ __forceinline__ void load_group(const T* p, T (&out)[G]) {
  static_assert(G * sizeof(T) <= 16, "one load per group");
  if constexpr (G == 1) {
    out[0] = ld_mat<NT>(p);
  } else {
    typedef typename VecT<T, G>::type V;
    const V v = ld_mat<NT>(reinterpret_cast<const V*>(p));
#pragma unroll
    for (int i = 0; i < G; ++i) out[i] = v[i];
  }
}

template <typename T, int N>
__device__ __forceinline__ void store_y(T* p, const T (&in)[N], bool nt) {
  if constexpr (N == 1) {
    if (nt) __builtin_nontemporal_store(in[0], p); else *p = in[0];
  } else {
    typedef typename VecT<T, N>::type V;
    V v;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = in[i];
    if (nt) __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
    else *reinterpret_cast<V*>(p) = v;
  }
}

template <class C>
__device__ __forceinline__ typename C::XT value_at(const ProdArgs& a, int32_t p) {
  const int32_t q = a.vperm ? ld_mat<C::kNT>(a.vperm + p) : p;
  return static_cast<typename C::XT>(
      ValueLoad<typename C::VT>::template get<C::kNT>(static_cast<const typename C::VT*>(a.values) + q));
}

// x entry of column index c (SpMV): from the compact hot copy when c is a
// hot slot (~slot < 0, HOT variant), else from x.
template <class C>
__device__ __forceinline__ typename C::XT x_at(const ProdArgs& a, const typename C::XT* X, int32_t c, int64_t ldx) {
  if constexpr (C::kHot) {
    const typename C::XT* xh = static_cast<const typename C::XT*>(a.X2);
    return c < 0 ? xh[~c] : X[static_cast<int64_t>(c) * ldx];
  }
  return X[static_cast<int64_t>(c) * ldx];
}

// The gathered x[colind[p]] of nonzero p, kept for the backward (save variant).
template <class C>
__device__ __forceinline__ void save_x(const ProdArgs& a, int32_t p, typename C::XT x) {
  typename C::XT* dst = static_cast<typename C::XT*>(a.xsave) + p;
  if (a.flags & SPX_FLAG_NO_NT_STORE) *dst = x;
  else __builtin_nontemporal_store(x, dst);
}

// Accumulate the nonzeros p = p0 + slot, p0 + slot + S, ... < p1 of one row
// into acc (plain) or cacc (compensated) for the VEC columns at `col`
// (lanes with col >= k take part in the shared loads and gather nothing).
// Every round issues the loads of U nonzeros before using any; the last
// round is masked rather than finished one nonzero at a time, so a slot with
// n nonzeros waits for ceil(n / U) gather round trips.  Products are added in
// ascending p either way.
// In SpMM (KL > 1) the KL lanes of a group need the same colind / values:
// lane kl loads element kl (kl + KL, ...) of the round and the group shares
// them through ds_bpermute, so a round costs the texture addresser U lanes
// of index loads instead of U x KL (the address unit, not HBM, bounds the
// short-row SpMM).
template <class C, int S>
__device__ __forceinline__ void accumulate(const ProdArgs& a, int32_t p0, int32_t p1, int slot,
                                           int col, bool comp, typename C::AT (&acc)[C::VEC],
                                           Comp (&cacc)[C::VEC]) {
  using XT = typename C::XT;
  constexpr int VEC = C::VEC;
  constexpr int U = C::U;
  const XT* X = static_cast<const XT*>(a.X) + col;
  const int64_t ldx = a.ldx;
  const bool colok = col < a.k;
  for (int32_t p = p0 + slot; p < p1; p += U * S) {
    bool h[U];
    int32_t c[U];
    XT v[U];
    XT xv[U][VEC];
    if constexpr (C::KL > 1) {
      constexpr int KL = C::KL;
      constexpr int PER = (U + KL - 1) / KL;
      const int lane = threadIdx.x % kWave;
      const int kl = lane % KL, base = lane - kl;
      int32_t cl[PER];
      XT vl[PER];
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int u = kl + j * KL;
        const bool hl = u < U && p + u * S < p1;
        cl[j] = hl ? ld_mat<C::kNT>(a.colind + p + u * S) : 0;
        vl[j] = hl ? value_at<C>(a, p + u * S) : XT(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        h[u] = p + u * S < p1;
        c[u] = __shfl(cl[u / KL], base + u % KL, kWave);
        v[u] = __shfl(vl[u / KL], base + u % KL, kWave);
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        h[u] = p + u * S < p1;
        c[u] = h[u] ? ld_mat<C::kNT>(a.colind + p + u * S) : 0;
        v[u] = h[u] ? value_at<C>(a, p + u * S) : XT(0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (h[u] && colok) {
        if constexpr (C::kHot) xv[u][0] = x_at<C>(a, X, c[u], ldx);
        else load_x<XT, VEC>(X + static_cast<int64_t>(c[u]) * ldx, xv[u]);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) xv[u][e] = XT(0);
      }
    }
    if constexpr (C::kSave) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (h[u]) save_x<C>(a, p + u * S, xv[u][0]);
    }
    if (!C::kComp || !comp) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          if (h[u]) acc[e] = fma_t(v[u], xv[u][e], acc[e]);
    } else if constexpr (C::kComp) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          if (h[u]) cacc[e].add_prod(v[u], xv[u][e]);
    }
  }
}

// Begin/end of the rows served by a row group: binned rows read their id from
// row_perm and their nonzero range from prange (both precomputed by the plan,
// one independent load each); unbinned rows read rowptr.  Each header is read
// once per product, so its loads are non-temporal like the matrix stream and
// leave L2 to the gathered x lines.
__device__ __forceinline__ void row_range(const ProdArgs& a, const BinDesc& d, int idx, int32_t& row,
                                          int32_t& p0, int32_t& p1) {
  if (a.row_perm) {
    row = ld_stream(a.row_perm + d.row_begin + idx);
    using I2 = VecT<int32_t, 2>::type;
    const I2 pr = ld_stream(reinterpret_cast<const I2*>(a.prange) + d.row_begin + idx);
    p0 = pr.x;
    p1 = pr.y;
  } else {
    row = d.row_begin + idx;
    p0 = a.rowptr[row];
    p1 = a.rowptr[row + 1];
  }
}

// Sum over the S slots of a row group and store the row's VEC outputs.
template <class C, int GG>
__device__ __forceinline__ void finish_small(const ProdArgs& a, bool active, bool comp, int slot,
                                             int col, int32_t row, typename C::AT (&acc)[C::VEC],
                                             Comp (&cacc)[C::VEC], bool nt) {
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
  if (active && slot == 0 && col < a.k) {
    XT out[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      if constexpr (C::kComp) out[e] = comp ? static_cast<XT>(dsum[e]) : acc[e];
      else out[e] = acc[e];
    }
    store_y<XT, VEC>(static_cast<XT*>(a.Y) + static_cast<int64_t>(row) * a.ldy + col, out, nt);
  }
}

// Row groups of G threads (G in 1..64 or 256), R rows per group.
//  R == 1: the group walks its row with U independent nonzeros per lane.
//  R > 1 (short-row bins, at most one nonzero per slot and row): the group
//  serves R rows at once and issues all their loads before using any, so a
//  lane has R independent load chains in flight.  Rows of round j are the
//  consecutive bin entries tile*RPB + j*NG + group, which keeps the row_perm,
//  prange and y accesses of a round contiguous.
template <class C, int G, int R>
__device__ __forceinline__ void do_rows(const ProdArgs& a, const BinDesc& d, int tile) {
  constexpr int KL = C::KL, VEC = C::VEC;
  constexpr int S = (G >= KL) ? G / KL : 1;
  constexpr int GG = S * KL;
  constexpr int NG = kWG / GG;  // groups per workgroup
  constexpr int RPB = NG * R;   // rows per workgroup
  using XT = typename C::XT;
  using AT = typename C::AT;
  if (tile * RPB >= d.nrows) return;  // whole workgroup idle (uniform)
  const int t = threadIdx.x;
  const int ln = t % GG, slot = ln / KL, kl = ln % KL, grp = t / GG;
  const bool nt = !(a.flags & SPX_FLAG_NO_NT_STORE);

  if constexpr (R > 1) {
    static_assert(GG <= kWave, "multi-row groups live inside one wavefront");
    int32_t row[R], p0[R], p1[R];
    bool active[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int idx = tile * RPB + j * NG + grp;
      active[j] = idx < d.nrows;
      row[j] = 0;
      p0[j] = 0;
      p1[j] = 0;
      if (active[j]) row_range(a, d, idx, row[j], p0[j], p1[j]);
    }
    for (int c0 = 0; c0 < a.k; c0 += KL * VEC) {
      const int col = c0 + kl * VEC;
      const XT* X = static_cast<const XT*>(a.X) + col;
      int32_t c[R];
      XT v[R];
      bool has[R];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int32_t p = p0[j] + slot;
        has[j] = (p < p1[j]) && (col < a.k);
        c[j] = has[j] ? ld_mat<C::kNT>(a.colind + p) : 0;
        v[j] = has[j] ? value_at<C>(a, p) : XT(0);
      }
      XT xv[R][VEC];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (has[j]) {
          if constexpr (C::kHot) xv[j][0] = x_at<C>(a, X, c[j], a.ldx);
          else load_x<XT, VEC>(X + static_cast<int64_t>(c[j]) * a.ldx, xv[j]);
        } else {
#pragma unroll
          for (int e = 0; e < VEC; ++e) xv[j][e] = XT(0);
        }
      }
      if constexpr (C::kSave) {
#pragma unroll
        for (int j = 0; j < R; ++j)
          if (has[j]) save_x<C>(a, p0[j] + slot, xv[j][0]);
      }
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const bool comp = C::kComp && (p1[j] - p0[j] > a.kahan_len);
        AT acc[VEC];
        Comp cacc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          cacc[e].init();
          if (C::kComp && comp) {
            cacc[e].add_prod(v[j], xv[j][e]);
            acc[e] = AT(0);
          } else {
            acc[e] = fma_t(v[j], xv[j][e], AT(0));
          }
        }
        // the planner only gives R > 1 to bins whose rows fit one nonzero
        // per slot; any longer row is still summed, one nonzero at a time
        if (col < a.k) {
          for (int32_t p = p0[j] + S + slot; p < p1[j]; p += S) {
            const XT vv = value_at<C>(a, p);
            XT xx[VEC];
            if constexpr (C::kHot) xx[0] = x_at<C>(a, X, ld_mat<C::kNT>(a.colind + p), a.ldx);
            else load_x<XT, VEC>(X + static_cast<int64_t>(ld_mat<C::kNT>(a.colind + p)) * a.ldx, xx);
            if constexpr (C::kSave) save_x<C>(a, p, xx[0]);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
              if (C::kComp && comp) cacc[e].add_prod(vv, xx[e]);
              else acc[e] = fma_t(vv, xx[e], acc[e]);
            }
          }
        }
        finish_small<C, GG>(a, active[j], comp, slot, col, row[j], acc, cacc, nt);
      }
    }
    return;
  } else {
    const int idx = tile * NG + grp;
    const bool active = idx < d.nrows;
    int32_t row = 0, p0 = 0, p1 = 0;
    if constexpr (KL > 1) {
      // one lane per group reads the row's id and range; the group shares them
      if (active && kl == 0) row_range(a, d, idx, row, p0, p1);
      const int src = (t % kWave) - kl;
      row = __shfl(row, src, kWave);
      p0 = __shfl(p0, src, kWave);
      p1 = __shfl(p1, src, kWave);
    } else if (active) {
      row_range(a, d, idx, row, p0, p1);
    }
    const bool comp = C::kComp && (p1 - p0 > a.kahan_len);
    XT* Y = static_cast<XT*>(a.Y);

    for (int c0 = 0; c0 < a.k; c0 += KL * VEC) {
      const int col = c0 + kl * VEC;
      AT acc[VEC];
      Comp cacc[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        acc[e] = AT(0);
        cacc[e].init();
      }
      accumulate<C, S>(a, p0, p1, slot, col, comp, acc, cacc);  // every lane: shared loads

      if constexpr (GG <= kWave) {
        finish_small<C, GG>(a, active, comp, slot, col, row, acc, cacc, nt);
      } else {
        // one row per workgroup: waves reduce, then LDS across the 4 waves
        __shared__ double red[kWG / kWave][KL][VEC];
        const int w = t / kWave;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          double v;
          if constexpr (C::kComp) {
            v = comp ? group_sum<kWave, KL>(cacc[e].value())
                     : static_cast<double>(group_sum<kWave, KL>(acc[e]));
          } else {
            v = group_sum<kWave, KL>(acc[e]);
          }
          if ((t % kWave) < KL) red[w][t % kWave][e] = v;
        }
        __syncthreads();
        if (t < KL && col < a.k) {
          XT out[VEC];
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            if (C::kComp && comp) {
              double s = 0.0;
              for (int i = 0; i < kWG / kWave; ++i) s += red[i][t][e];
              out[e] = static_cast<XT>(s);
            } else {
              AT s = AT(0);
              for (int i = 0; i < kWG / kWave; ++i) s += static_cast<AT>(red[i][t][e]);
              out[e] = s;
            }
          }
          store_y<XT, VEC>(Y + static_cast<int64_t>(row) * a.ldy + col, out, nt);
        }
        __syncthreads();
      }
    }
  }
}

// Stream bin (SpMV only): one workgroup takes kStreamRows consecutive rows of
// the bin and treats their nonzeros as one flat sequence.  Lanes load that
// sequence in chunks (stream_chunk) with consecutive lanes on consecutive
// nonzeros (coalesced, 4 or 8 independent loads per lane), gather
// x, and park the products in LDS; then every thread sums its own row's
// products in ascending order.  A chunk costs two dependent global trips for
// up to 2,048 nonzeros, where a row group pays a trip chain per row.
constexpr int kStreamRows = 256;
// Nonzeros per chunk: 8 KB of products in LDS either way (1,024 FP64 or
// 2,048 FP32 accumulators); measured best for each type.
template <typename AT>
constexpr int stream_chunk() {
  return std::is_same<AT, double>::value ? 1024 : 2048;
}

template <class C>
__device__ __forceinline__ void do_stream(const ProdArgs& a, const BinDesc& d, int tile) {
  static_assert(C::KL == 1 && C::VEC == 1, "stream bins serve SpMV only");
  using XT = typename C::XT;
  using AT = typename C::AT;
  constexpr int kStreamChunk = stream_chunk<AT>();
  constexpr int kStreamPer = kStreamChunk / kWG;
  __shared__ int32_t s_off[kStreamRows + 1];
  __shared__ int32_t s_p0[kStreamRows];
  __shared__ AT s_prod[kStreamChunk];
  __shared__ int32_t s_wsum[kWG / kWave];
  __shared__ int32_t s_end;
  if (tile * kStreamRows >= d.nrows) return;
  const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
  const int idx = tile * kStreamRows + t;
  const bool active = idx < d.nrows;
  int32_t row = 0, p0 = 0, p1 = 0;
  if (active) row_range(a, d, idx, row, p0, p1);
  const int32_t L = p1 - p0;
  // exclusive prefix of the row lengths over the workgroup
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
  const int32_t off = before + inc - L;
  s_off[t] = off;
  s_p0[t] = p0;
  if (t == kWG - 1) s_off[kStreamRows] = total;
  if (idx == min(d.nrows, (tile + 1) * kStreamRows) - 1) s_end = p1;
  total = __builtin_amdgcn_readfirstlane(total);
  __syncthreads();
  // Rows of a bin are ascending, so the tile's nonzeros are one contiguous
  // run exactly when its last row ends total elements after its first row
  // begins (rows between them that are not in the bin are then empty).  In
  // that case element j sits at the first row's p0 + j and the search below
  // is skipped.
  const int32_t P0 = __builtin_amdgcn_readfirstlane(s_p0[0]);
  const bool contig = __builtin_amdgcn_readfirstlane(s_end) - P0 == total;

  const XT* X = static_cast<const XT*>(a.X);
  const bool comp = C::kComp && (L > a.kahan_len);
  AT acc = AT(0);
  // Loads of one chunk: the row of each element is the last r with
  // s_off[r] <= j, found by a fixed 8-step branchless search run for all
  // kStreamPer elements in lockstep (the LDS reads of a step are independent,
  // so a lane waits for 8 LDS round trips per chunk, not 8 per element).
  // Slots past the tile's last element load that element again instead of
  // branching around the loads (a masked load followed by a use makes the
  // compiler wait for it at once); their products are never summed.
  using VL = ValueLoad<typename C::VT>;
  using Raw = typename VL::Raw;
  // The save variant needs each element's position again when it stores the
  // gathered x; it keeps the row found by the search (an index below 256)
  // packed four to a register rather than the positions themselves.
  static_assert(kStreamPer % 4 == 0 && kStreamRows <= 256, "row indices packed as bytes");
  constexpr int kPack = kStreamPer / 4;
  // A contiguous tile whose colind and values start 16-byte aligned (no value
  // permutation, not the save variant) loads each lane's elements in groups
  // of G consecutive nonzeros: one index load and one 16-byte value load per
  // group (G = 2 for FP64 values, 4 for FP32 and BF16) instead of G of each.
  // The address unit, the bound of these streams, is charged per lane
  // address; each load still covers whole lines across the wavefront.
  // Chunks then start at the aligned position P0 - (P0 mod G), so the first
  // chunk also loads (and never sums) up to G - 1 elements of the rows before
  // the tile; only chunks that end inside the tile take groups, the last one
  // loads element by element, clamped.
  constexpr int G = sizeof(typename C::VT) == 8 ? 2 : 4;
  static_assert(kStreamPer % G == 0, "whole groups per chunk");
  const bool grouped = !C::kSave && contig && !a.vperm &&
                       ((reinterpret_cast<uintptr_t>(a.colind) | reinterpret_cast<uintptr_t>(a.values)) & 15) == 0;
  const int32_t cs0 = (grouped && total > 0) ? -(P0 & (G - 1)) : 0;
  auto grouped_chunk = [&](int32_t cs) { return grouped && cs + kStreamChunk <= total; };
  auto fetch = [&](int32_t base, int32_t (&cc)[kStreamPer], Raw (&vv)[kStreamPer],
                   uint32_t (&rows)[kPack]) {
    if (grouped_chunk(base)) {
#pragma unroll
      for (int g = 0; g < kStreamPer / G; ++g) {
        const int32_t q = P0 + base + g * G * kWG + G * t;
        int32_t cg[G];
        Raw vg[G];
        load_group<C::kNT, G>(a.colind + q, cg);
        load_group<C::kNT, G>(static_cast<const typename C::VT*>(a.values) + q, vg);
#pragma unroll
        for (int e = 0; e < G; ++e) {
          cc[G * g + e] = cg[e];
          vv[G * g + e] = vg[e];
        }
      }
      return;
    }
    int32_t jj[kStreamPer], pp[kStreamPer];
#pragma unroll
    for (int u = 0; u < kStreamPer; ++u) jj[u] = min(base + u * kWG + t, total - 1);
    if (contig) {
#pragma unroll
      for (int u = 0; u < kStreamPer; ++u) pp[u] = P0 + jj[u];
    } else {
      int32_t lo[kStreamPer];
#pragma unroll
      for (int u = 0; u < kStreamPer; ++u) lo[u] = 0;
#pragma unroll
      for (int step = kStreamRows / 2; step >= 1; step >>= 1) {
#pragma unroll
        for (int u = 0; u < kStreamPer; ++u)
          if (s_off[lo[u] + step] <= jj[u]) lo[u] += step;
      }
#pragma unroll
      for (int u = 0; u < kStreamPer; ++u) pp[u] = s_p0[lo[u]] + (jj[u] - s_off[lo[u]]);
      if constexpr (C::kSave) {
#pragma unroll
        for (int i = 0; i < kPack; ++i)
          rows[i] = static_cast<uint32_t>(lo[4 * i]) | (static_cast<uint32_t>(lo[4 * i + 1]) << 8) |
                    (static_cast<uint32_t>(lo[4 * i + 2]) << 16) | (static_cast<uint32_t>(lo[4 * i + 3]) << 24);
      }
    }
#pragma unroll
    for (int u = 0; u < kStreamPer; ++u) {
      const int32_t p = pp[u];
      cc[u] = ld_mat<C::kNT>(a.colind + p);
      const int32_t q = a.vperm ? ld_mat<C::kNT>(a.vperm + p) : p;
      vv[u] = VL::template raw<C::kNT>(static_cast<const typename C::VT*>(a.values) + q);
    }
  };
  // software pipeline: the next chunk's colind / values are in flight while
  // the current chunk gathers x and reduces through LDS
  // (row indices rA / rB: save variant only)
  int32_t cA[kStreamPer];
  Raw vA[kStreamPer];
  uint32_t rA[kPack];
  if (total > 0) fetch(cs0, cA, vA, rA);
  for (int32_t base = cs0; base < total; base += kStreamChunk) {
    const bool more = base + kStreamChunk < total;
    int32_t cB[kStreamPer];
    Raw vB[kStreamPer];
    uint32_t rB[kPack];
    if (more) fetch(base + kStreamChunk, cB, vB, rB);
    XT xv[kStreamPer];
    const bool gd = grouped_chunk(base);
    // element index of slot u of this chunk (only the elements of the tile,
    // 0 <= j < total, gather x)
    auto elem = [&](int u) {
      return gd ? base + (u / G) * G * kWG + G * t + (u % G) : base + u * kWG + t;
    };
#pragma unroll
    for (int u = 0; u < kStreamPer; ++u)
      xv[u] = (static_cast<uint32_t>(elem(u)) < static_cast<uint32_t>(total)) ? x_at<C>(a, X, cA[u], a.ldx)
                                                                              : XT(0);
    if constexpr (C::kSave) {
#pragma unroll
      for (int u = 0; u < kStreamPer; ++u) {
        const int32_t j = base + u * kWG + t;
        if (j >= total) continue;
        const int r = (rA[u / 4] >> (8 * (u % 4))) & 255;
        save_x<C>(a, contig ? P0 + j : s_p0[r] + (j - s_off[r]), xv[u]);
      }
    }
    if (gd) {
#pragma unroll
      for (int u = 0; u < kStreamPer; ++u)
        s_prod[(u / G) * G * kWG + G * t + (u % G)] = static_cast<XT>(VL::widen(vA[u])) * xv[u];
    } else {
#pragma unroll
      for (int u = 0; u < kStreamPer; ++u) s_prod[u * kWG + t] = static_cast<XT>(VL::widen(vA[u])) * xv[u];
    }
    __syncthreads();
    const int32_t b0 = max(off, base) - base;
    const int32_t b1 = min(off + L, base + kStreamChunk) - base;
#pragma unroll 8
    for (int32_t i = b0; i < b1; ++i) acc += s_prod[i];
    __syncthreads();
    if (more) {
#pragma unroll
      for (int u = 0; u < kStreamPer; ++u) {
        cA[u] = cB[u];
        vA[u] = vB[u];
      }
#pragma unroll
      for (int i = 0; i < kPack; ++i) rA[i] = rB[i];
    }
  }
  if (!active) return;
  XT out[1];
  if constexpr (C::kComp) {
    if (comp) {
      // rows above kahan_len (not placed in stream bins by the planner):
      // compensated sum of the row straight from memory
      Comp cc;
      cc.init();
      for (int32_t p = p0; p < p1; ++p)
        cc.add_prod(value_at<C>(a, p), x_at<C>(a, X, ld_mat<C::kNT>(a.colind + p), a.ldx));
      out[0] = static_cast<XT>(cc.value());
    } else {
      out[0] = acc;
    }
  } else {
    out[0] = acc;
  }
  store_y<XT, 1>(static_cast<XT*>(a.Y) + static_cast<int64_t>(row) * a.ldy, out,
                 !(a.flags & SPX_FLAG_NO_NT_STORE));
}

// One workgroup per segment of a split row; the last arrival reduces.
template <class C>
__device__ __forceinline__ void do_split(const ProdArgs& a, const BinDesc& d, int tile) {
  constexpr int KL = C::KL, VEC = C::VEC;
  constexpr int S = kWG / KL;
  using XT = typename C::XT;
  using AT = typename C::AT;
  if (tile >= d.nrows) return;
  __shared__ double red[kWG / kWave][KL][VEC];
  __shared__ int last;
  const int t = threadIdx.x, w = t / kWave, slot = t / KL, kl = t % KL;
  const int32_t s = a.seg_row[tile];
  const int32_t row = a.split_rows[s];
  const int32_t f = a.seg_first[s], nseg = a.seg_first[s + 1] - f;
  const int32_t rb = a.rowptr[row], re = a.rowptr[row + 1];
  const int32_t p0 = rb + (tile - f) * a.chunk;
  const int32_t p1 = min(p0 + a.chunk, re);
  const bool comp = C::kComp && (re - rb > a.kahan_len);
  double* part = a.partials + static_cast<int64_t>(tile) * a.max_k;

  for (int c0 = 0; c0 < a.k; c0 += KL * VEC) {
    const int col = c0 + kl * VEC;
    AT acc[VEC];
    Comp cacc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      acc[e] = AT(0);
      cacc[e].init();
    }
    accumulate<C, S>(a, p0, p1, slot, col, comp, acc, cacc);  // every lane: shared loads
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      double v;
      if constexpr (C::kComp) {
        v = comp ? group_sum<kWave, KL>(cacc[e].value())
                 : static_cast<double>(group_sum<kWave, KL>(acc[e]));
      } else {
        v = group_sum<kWave, KL>(acc[e]);
      }
      if ((t % kWave) < KL) red[w][t % kWave][e] = v;
    }
    __syncthreads();
    if (t < KL && col < a.k) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        double r;
        if (C::kComp && comp) {
          r = 0.0;
          for (int i = 0; i < kWG / kWave; ++i) r += red[i][t][e];
        } else {
          AT q = AT(0);
          for (int i = 0; i < kWG / kWave; ++i) q += static_cast<AT>(red[i][t][e]);
          r = static_cast<double>(q);
        }
        __hip_atomic_store(part + col + e, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
  }

  // ---- arrival.  The partials were written by the lanes t < KL of wave 0
  // with device-scope stores (written through to the device coherence
  // point); vmcnt(0) waits until they have completed, so they are visible to
  // device-scope loads of any XCD before the counter moves.  The last arrival
  // reads them with device-scope loads.  This avoids a release/acquire fence
  // pair, which on gfx950 writes back / invalidates the whole L2 of the XCD.
  if (t == 0) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    const int old = __hip_atomic_fetch_add(a.counters + s, 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
    last = (old == nseg - 1);
  }
  __syncthreads();
  if (!__builtin_amdgcn_readfirstlane(last)) return;
  const bool nt = !(a.flags & SPX_FLAG_NO_NT_STORE);
  XT* Y = static_cast<XT*>(a.Y);
  for (int c = t; c < a.k; c += kWG) {
    const double* pp = a.partials + static_cast<int64_t>(f) * a.max_k + c;
    XT out[1];
    if (C::kComp && comp) {
      double r = 0.0;
      for (int j = 0; j < nseg; ++j)
        r += __hip_atomic_load(pp + static_cast<int64_t>(j) * a.max_k, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      out[0] = static_cast<XT>(r);
    } else {
      AT r = AT(0);
      for (int j = 0; j < nseg; ++j)
        r += static_cast<AT>(__hip_atomic_load(pp + static_cast<int64_t>(j) * a.max_k,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      out[0] = r;
    }
    store_y<XT, 1>(Y + static_cast<int64_t>(row) * a.ldy + c, out, nt);
  }
  if (t == 0)
    __hip_atomic_store(a.counters + s, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace prod
}  // namespace spx
