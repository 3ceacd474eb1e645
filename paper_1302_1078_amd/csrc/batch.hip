// batch.hip -- many independent products Y_b <- A_b X_b in a few launches
// (the paper's motivation: many SpMV/SpMM-based requests served at once,
// Sec. 1 and Sec. 5).
//
// At creation every matrix is binned with its own plan options (from an
// autotuner or the defaults) and its row-group tiles are appended to a tile
// list grouped by lane layout (the (KL, VEC) that its k selects) and, inside
// a group, ordered by estimated cost (heaviest first).  At run time one
// kernel per layout present runs one workgroup per tile of its group: tile
// i of the group goes to workgroup i, so the hardware dispatcher starts the
// heaviest tiles first and fills each freed slot with the next one (a
// longest-first schedule with no queue, atomics or reset kernel).  A kernel
// per layout keeps each launch's register use, and so its occupancy, near
// that of the single-matrix kernel of the same layout.  A persistent
// version (a queue of tiles popped by a grid of CUs x 8 workgroups) needed
// 79-115 VGPRs for the loop around the same tile code, against 60-71 here,
// and ran at 4-6 instead of 7-8 waves per SIMD.  Each tile runs exactly the
// row-group code of the single-matrix launch with the matrix's own
// arguments, so every result is bit-identical to csr_spmv / csr_spmm with
// the same plan options.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "product_impl.hpp"

namespace spx {

namespace {

using namespace prod;

struct TileDesc {
  int32_t mat;
  int16_t slot;    // index into the matrix's bin table
  int16_t layout;  // lane layout (KL, VEC)
  int32_t tile;    // tile index inside the bin
};

struct BatchArgs {
  const ProdArgs* mats;
  const TileDesc* tiles;  // the layout's group of the tile list
};

// layouts: 0 -> (KL 1, VEC 1); i >= 1 -> (KL 2^(i-1), VEC V)
constexpr int kLayouts = 7;

template <class C, bool MR>
__device__ __forceinline__ void run_tile(const ProdArgs& a, const BinDesc& d, int tile) {
  constexpr bool kMulti = MR && C::KL == 1 && C::VEC == 1;
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
      if constexpr (kMulti) do_rows<C, 1, 4>(a, d, tile);
      else do_rows<C, 1, 1>(a, d, tile);
      break;
    case 1002:
      if constexpr (kMulti) do_rows<C, 2, 4>(a, d, tile);
      else do_rows<C, 2, 1>(a, d, tile);
      break;
    case 1004:
      if constexpr (kMulti) do_rows<C, 4, 4>(a, d, tile);
      else do_rows<C, 4, 1>(a, d, tile);
      break;
    case 1008:
      if constexpr (kMulti) do_rows<C, 8, 4>(a, d, tile);
      else do_rows<C, 8, 1>(a, d, tile);
      break;
    case 1016:
      if constexpr (kMulti) do_rows<C, 16, 4>(a, d, tile);
      else do_rows<C, 16, 1>(a, d, tile);
      break;
    case 1032:
      if constexpr (kMulti) do_rows<C, 32, 4>(a, d, tile);
      else do_rows<C, 32, 1>(a, d, tile);
      break;
    case SPX_LANES_STREAM:
      if constexpr (C::KL == 1 && C::VEC == 1) do_stream<C>(a, d, tile);
      else do_rows<C, 1, 1>(a, d, tile);
      break;
    default: do_split<C>(a, d, tile); break;
  }
}

// One workgroup per tile of a layout's group (blockIdx.x indexes the group,
// heaviest tiles first).  The tile's fields are wave-uniform (read through a
// uniform pointer), so every branch of the tile code is scalar, as in the
// single-matrix launch.
template <class C, bool MR>
__global__ __launch_bounds__(kWG) void k_batch(const BatchArgs b) {
  const TileDesc* tp = b.tiles + blockIdx.x;
  const int32_t mat = __builtin_amdgcn_readfirstlane(tp->mat);
  const int32_t slot = __builtin_amdgcn_readfirstlane(tp->slot);
  const int32_t tile = __builtin_amdgcn_readfirstlane(tp->tile);
  const ProdArgs& a = b.mats[mat];
  BinDesc d;
  d.blk_begin = 0;
  d.nblk = a.bins[slot].nblk;
  d.row_begin = a.bins[slot].row_begin;
  d.nrows = a.bins[slot].nrows;
  d.lanes = a.bins[slot].lanes;
  d.bin = 0;
  d.rpg = a.bins[slot].rpg;
  run_tile<C, MR>(a, d, tile);
}

bool pair_ok(spx_dtype vt, spx_dtype xt) {
  return (vt == SPX_F64 && xt == SPX_F64) || (vt == SPX_F32 && xt == SPX_F32) ||
         (vt == SPX_BF16 && xt == SPX_F32);
}

int layout_id(int kl, int vec) {
  if (vec == 1) return kl == 1 ? 0 : -1;
  int id = 1;
  for (int l = 1; l < kl; l <<= 1) ++id;
  return id < kLayouts ? id : -1;
}

// Options as the batch uses them: unpadded bins (the tile list, not the XCD
// map, orders the work) and partials wide enough for the matrix's k.
spx_plan_opts batch_opts(const spx_csr_desc& d) {
  spx_plan_opts o = d.opts;
  o.flags |= SPX_FLAG_NO_XCD_MAP;
  if (o.max_k < d.k) o.max_k = d.k;
  return o;
}

int64_t tile_bound(const spx_csr_desc& d, const spx_plan_opts& o) {
  // bins hold at most m rows in total; split segments at most nnz/chunk + m
  int64_t t = static_cast<int64_t>(d.m) + o.nbins + 1;
  if (o.lanes[o.nbins - 1] == 0) t += d.nnz / o.split_chunk + d.m + 1;
  return t;
}

struct BatchLayout {
  std::vector<size_t> plan_off;
  std::vector<size_t> plan_bytes;
  size_t mats_off, tiles_off, total;
  int64_t max_tiles;
};

spx_status layout_ws(int32_t count, const spx_csr_desc* descs, BatchLayout* L) {
  size_t off = 0;
  L->plan_off.resize(count);
  L->plan_bytes.resize(count);
  L->max_tiles = 0;
  for (int32_t i = 0; i < count; ++i) {
    const spx_plan_opts o = batch_opts(descs[i]);
    size_t b = 0;
    spx_status s = csr_plan_workspace_bytes(descs[i].m, descs[i].nnz, &o, &b);
    if (s != SPX_OK) return s;
    L->plan_off[i] = off;
    L->plan_bytes[i] = b;
    off = align_up(off + b);
    L->max_tiles += tile_bound(descs[i], o);
  }
  L->mats_off = off;
  off = align_up(off + sizeof(ProdArgs) * static_cast<size_t>(count > 0 ? count : 1));
  L->tiles_off = off;
  off = align_up(off + sizeof(TileDesc) * static_cast<size_t>(L->max_tiles + 1));
  L->total = off;
  return SPX_OK;
}

spx_status check_desc(const spx_csr_desc& d, int i, spx_dtype vt, spx_dtype xt) {
  if (d.m < 0 || d.n < 0 || d.nnz < 0 || d.k < 1)
    return fail(SPX_ERR_INVALID, "batch matrix %d: bad sizes", i);
  if (d.nnz > SPX_MAX_NNZ)
    return fail(SPX_ERR_UNSUPPORTED, "batch matrix %d: nnz=%d above SPX_MAX_NNZ", i, d.nnz);
  if (d.vtype != vt || d.xytype != xt)
    return fail(SPX_ERR_UNSUPPORTED, "batch matrix %d: all matrices must share one dtype pair", i);
  if (d.ldx < d.k || d.ldy < d.k) return fail(SPX_ERR_INVALID, "batch matrix %d: ld < k", i);
  if (d.m > 0 && (!d.rowptr || !d.Y)) return fail(SPX_ERR_INVALID, "batch matrix %d: null pointer", i);
  if (d.nnz > 0 && (!d.colind || !d.values || !d.X))
    return fail(SPX_ERR_INVALID, "batch matrix %d: null pointer", i);
  return SPX_OK;
}

}  // namespace
}  // namespace spx

struct spx_batch {
  spx_dtype vt, xt;
  int32_t count;
  int32_t ntiles;
  int32_t grid;  // workgroups of the largest per-layout launch
  int64_t nseg;
  spx::ProdArgs* mats;
  spx::TileDesc* tiles;
  int32_t first[spx::kLayouts];  // tiles of layout l: [first[l], first[l] + ntile[l])
  int32_t ntile[spx::kLayouts];
  bool multi_row;  // layout 0 has short-row bins served several rows per group
  std::vector<spx_plan*> plans;
};

using namespace spx;

extern "C" spx_status csr_batch_workspace_bytes(int32_t count, const spx_csr_desc* descs, size_t* bytes) {
  if (!bytes || count < 0 || (count > 0 && !descs))
    return fail(SPX_ERR_INVALID, "csr_batch_workspace_bytes: bad arguments");
  BatchLayout L;
  spx_status s = layout_ws(count, descs, &L);
  if (s != SPX_OK) return s;
  *bytes = L.total;
  return SPX_OK;
}

extern "C" spx_status csr_batch_create(int32_t count, const spx_csr_desc* descs, void* workspace,
                                       size_t ws_bytes, void* stream, spx_batch** out) {
  if (!out) return fail(SPX_ERR_INVALID, "csr_batch_create: out is null");
  *out = nullptr;
  if (count < 1 || !descs) return fail(SPX_ERR_INVALID, "csr_batch_create: need count >= 1 descriptors");
  const spx_dtype vt = descs[0].vtype, xt = descs[0].xytype;
  if (!pair_ok(vt, xt)) return fail(SPX_ERR_UNSUPPORTED, "csr_batch_create: dtype pair");
  for (int32_t i = 0; i < count; ++i) {
    spx_status s = check_desc(descs[i], i, vt, xt);
    if (s != SPX_OK) return s;
  }
  BatchLayout L;
  spx_status s = layout_ws(count, descs, &L);
  if (s != SPX_OK) return s;
  if (!workspace || ws_bytes < L.total)
    return fail(SPX_ERR_WORKSPACE, "csr_batch_create: workspace %zu < %zu bytes", ws_bytes, L.total);
  hipStream_t st = as_stream(stream);
  char* base = static_cast<char*>(workspace);

  spx_batch* B = new (std::nothrow) spx_batch();
  if (!B) return fail(SPX_ERR_INVALID, "csr_batch_create: out of host memory");
  B->multi_row = false;
  B->vt = vt;
  B->xt = xt;
  B->count = count;
  B->nseg = 0;
  std::vector<ProdArgs> mats(count);
  struct Entry {
    double cost;
    TileDesc td;
  };
  std::vector<Entry> entries;
  auto cleanup = [&](spx_status st_) {
    for (spx_plan* p : B->plans) csr_plan_destroy(p);
    delete B;
    return st_;
  };
  for (int32_t i = 0; i < count; ++i) {
    const spx_csr_desc& d = descs[i];
    const spx_plan_opts o = batch_opts(d);
    spx_plan* p = nullptr;
    s = csr_plan_create(d.m, d.n, d.nnz, d.rowptr, &o, base + L.plan_off[i], L.plan_bytes[i], stream, &p);
    if (s != SPX_OK) return cleanup(s);
    B->plans.push_back(p);
    B->nseg += p->nseg;
    int kl, vec;
    layout_for_k(d.k, d.xytype, d.X, d.ldx, d.Y, d.ldy, o.flags, &kl, &vec);
    const int lid = layout_id(kl, vec);
    if (lid < 0)
      return cleanup(fail(SPX_ERR_UNSUPPORTED,
                          "batch matrix %d: k=%d needs scalar X loads (ld or alignment); not batched", i,
                          d.k));
    ProdArgs& a = mats[i];
    memset(&a, 0, sizeof(a));
    a.rowptr = d.rowptr;
    a.colind = d.colind;
    a.values = d.values;
    a.X = d.X;
    a.Y = d.Y;
    a.ldx = d.ldx;
    a.ldy = d.ldy;
    a.k = d.k;
    bins_from_plan(p, a, kl, false);
    for (int j = 0; j < a.nbins; ++j) {
      const BinDesc& bd = a.bins[j];
      if (lid == 0 && bd.rpg > 1) B->multi_row = true;
      double per_tile;
      if (bd.lanes == 0) {
        per_tile = o.split_chunk;
      } else {
        const int gg = bd.lanes > kl ? bd.lanes : kl;
        const int rpb = (bd.lanes == SPX_LANES_STREAM) ? kWG : (kWG / gg) * bd.rpg;
        double len;
        if (bd.bin < o.nbins - 1) len = o.upper[bd.bin];
        else len = (o.nbins >= 2) ? 2.0 * o.upper[o.nbins - 2] : static_cast<double>(d.nnz) / (d.m > 0 ? d.m : 1);
        if (len < 1.0) len = 1.0;
        per_tile = rpb * len;
      }
      const double cost = per_tile * (1.0 + 0.25 * d.k);
      for (int32_t t = 0; t < bd.nblk; ++t) {
        Entry e;
        e.cost = cost;
        e.td.mat = i;
        e.td.slot = static_cast<int16_t>(j);
        e.td.layout = static_cast<int16_t>(lid);
        e.td.tile = t;
        entries.push_back(e);
      }
    }
  }
  // tiles grouped by layout (one launch each), heaviest first inside a group
  std::stable_sort(entries.begin(), entries.end(), [](const Entry& x, const Entry& y) {
    return x.td.layout != y.td.layout ? x.td.layout < y.td.layout : x.cost > y.cost;
  });
  if (static_cast<int64_t>(entries.size()) > L.max_tiles || entries.size() > 0x7fffffffu)
    return cleanup(fail(SPX_ERR_INVALID, "csr_batch_create: tile list overflow"));
  std::vector<TileDesc> tiles(entries.size());
  for (size_t t = 0; t < entries.size(); ++t) tiles[t] = entries[t].td;
  B->mats = reinterpret_cast<ProdArgs*>(base + L.mats_off);
  B->tiles = reinterpret_cast<TileDesc*>(base + L.tiles_off);
  B->ntiles = static_cast<int32_t>(tiles.size());
  B->grid = 0;
  for (int l = 0; l < kLayouts; ++l) {
    B->first[l] = 0;
    B->ntile[l] = 0;
  }
  for (size_t t = 0; t < tiles.size(); ++t) {
    const int l = tiles[t].layout;
    if (B->ntile[l]++ == 0) B->first[l] = static_cast<int32_t>(t);
  }
  for (int l = 0; l < kLayouts; ++l) B->grid = std::max(B->grid, B->ntile[l]);
  hipError_t e = hipMemcpyAsync(B->mats, mats.data(), sizeof(ProdArgs) * count, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !tiles.empty())
    e = hipMemcpyAsync(B->tiles, tiles.data(), sizeof(TileDesc) * tiles.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return cleanup(hip_fail(e, "csr_batch_create: upload"));
  *out = B;
  return SPX_OK;
}

namespace spx {
namespace {

template <typename VT, typename XT, int V>
spx_status launch_layout(const spx_batch* B, int l, hipStream_t st) {
  const BatchArgs a{B->mats, B->tiles + B->first[l]};
  const unsigned g = static_cast<unsigned>(B->ntile[l]);
  switch (l) {
    case 0:
      if (B->multi_row) k_batch<Cfg<VT, XT, 1, 1>, true><<<g, kWG, 0, st>>>(a);
      else k_batch<Cfg<VT, XT, 1, 1>, false><<<g, kWG, 0, st>>>(a);
      break;
    case 1: k_batch<Cfg<VT, XT, 1, V>, false><<<g, kWG, 0, st>>>(a); break;
    case 2: k_batch<Cfg<VT, XT, 2, V>, false><<<g, kWG, 0, st>>>(a); break;
    case 3: k_batch<Cfg<VT, XT, 4, V>, false><<<g, kWG, 0, st>>>(a); break;
    case 4: k_batch<Cfg<VT, XT, 8, V>, false><<<g, kWG, 0, st>>>(a); break;
    case 5: k_batch<Cfg<VT, XT, 16, V>, false><<<g, kWG, 0, st>>>(a); break;
    default: k_batch<Cfg<VT, XT, 32, V>, false><<<g, kWG, 0, st>>>(a); break;
  }
  SPX_LAUNCHED("k_batch");
  return SPX_OK;
}

}  // namespace
}  // namespace spx

extern "C" spx_status csr_batch_run(const spx_batch* B, void* stream) {
  if (!B) return fail(SPX_ERR_INVALID, "csr_batch_run: batch is null");
  if (B->ntiles == 0) return SPX_OK;
  hipStream_t st = as_stream(stream);
  for (int l = 0; l < kLayouts; ++l) {
    if (B->ntile[l] == 0) continue;
    spx_status s;
    if (B->vt == SPX_F64) s = launch_layout<double, double, 2>(B, l, st);
    else if (B->vt == SPX_F32) s = launch_layout<float, float, 4>(B, l, st);
    else s = launch_layout<uint16_t, float, 4>(B, l, st);
    if (s != SPX_OK) return s;
  }
  return SPX_OK;
}

extern "C" spx_status csr_batch_info(const spx_batch* B, int64_t* ntiles, int32_t* grid, int64_t* nseg) {
  if (!B) return fail(SPX_ERR_INVALID, "csr_batch_info: batch is null");
  if (ntiles) *ntiles = B->ntiles;
  if (grid) *grid = B->grid;
  if (nseg) *nseg = B->nseg;
  return SPX_OK;
}

extern "C" void csr_batch_destroy(spx_batch* B) {
  if (!B) return;
  for (spx_plan* p : B->plans) csr_plan_destroy(p);
  delete B;
}
