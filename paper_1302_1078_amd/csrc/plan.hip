// plan.hip -- row binning by length on the device (the GPU analogue of the
// paper's dynamic row chunks, Sec. 4.1) and split-row segmentation.
//
// Bin b holds rows with upper[b-1] < L <= upper[b] (the last bin is
// unbounded).  row_perm lists the rows of bin 0, then bin 1, ..., ascending
// inside each bin: a stable partition computed with per-tile counts, one
// device scan, and a ballot-ranked scatter.  With a row period P > 0 the
// partition key is (bin, band) with band = floor(8 (r mod P) / P), so a bin
// lists band 0's rows, then band 1's, ..., each ascending.
#include <new>

#include "device.hpp"
#include "internal.hpp"

namespace spx {

namespace {

constexpr int kRowsPerThread = 16;
constexpr int kBinTile = kWG * kRowsPerThread;  // 4096 rows per workgroup

constexpr int kBands = 8;  // one band of each row period per XCD
constexpr int kMaxKeys = SPX_MAX_BINS * kBands;

struct BinParams {
  int32_t nbins;
  int32_t upper[SPX_MAX_BINS];
  int32_t period;  // 0: rows ascending inside a bin; P > 0: by band of r mod P, then ascending
  int32_t nkeys;   // nbins, or nbins x kBands with a period
};

__device__ __forceinline__ int bin_of(int32_t L, const BinParams& bp) {
  int b = 0;
  while (b + 1 < bp.nbins && L > bp.upper[b]) ++b;
  return b;
}

// Partition key of row i (length L): its bin, and with a period its band.
__device__ __forceinline__ int key_of(int64_t i, int32_t L, const BinParams& bp) {
  const int b = bin_of(L, bp);
  if (bp.period <= 0) return b;
  return b * kBands + static_cast<int>((i % bp.period) * kBands / bp.period);
}

__global__ __launch_bounds__(kWG) void k_bin_count(const int32_t* __restrict__ rowptr, int32_t m,
                                                   const BinParams bp,
                                                   int32_t* __restrict__ counts, int nblk) {
  __shared__ int32_t cnt[kMaxKeys];
  const int t = threadIdx.x;
  if (t < kMaxKeys) cnt[t] = 0;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kBinTile;
  for (int j = 0; j < kRowsPerThread; ++j) {
    const int64_t i = base + j * kWG + t;
    if (i < m) atomicAdd(&cnt[key_of(i, rowptr[i + 1] - rowptr[i], bp)], 1);
  }
  __syncthreads();
  if (t < bp.nkeys) counts[static_cast<int64_t>(t) * nblk + blockIdx.x] = cnt[t];
}

// Stable scatter: rows ranked in (round, wave, lane) order = ascending row.
__global__ __launch_bounds__(kWG) void k_bin_scatter(const int32_t* __restrict__ rowptr, int32_t m,
                                                     const BinParams bp,
                                                     const int32_t* __restrict__ offs, int nblk,
                                                     int32_t* __restrict__ row_perm) {
  __shared__ int32_t run[kMaxKeys];
  __shared__ int32_t wcnt[kWG / kWave][kMaxKeys];
  const int t = threadIdx.x, w = t / kWave, lane = t % kWave;
  const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  if (t < bp.nkeys) run[t] = offs[static_cast<int64_t>(t) * nblk + blockIdx.x];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kBinTile;
  __syncthreads();
  for (int j = 0; j < kRowsPerThread; ++j) {
    const int64_t i = base + j * kWG + t;
    const bool valid = i < m;
    const int b = valid ? key_of(i, rowptr[i + 1] - rowptr[i], bp) : -1;
    int rank = 0;
    for (int q = 0; q < bp.nkeys; ++q) {
      const uint64_t mask = __ballot(b == q);
      if (b == q) rank = __popcll(mask & lt_mask);
      if (lane == 0) wcnt[w][q] = __popcll(mask);
    }
    __syncthreads();
    if (valid) {
      int32_t pos = run[b] + rank;
      for (int v = 0; v < w; ++v) pos += wcnt[v][b];
      row_perm[pos] = static_cast<int32_t>(i);
    }
    __syncthreads();
    if (t < bp.nkeys) {
      int32_t add = 0;
      for (int v = 0; v < kWG / kWave; ++v) add += wcnt[v][t];
      run[t] += add;
    }
    __syncthreads();
  }
}

// Bin b begins at its first key, b x keys_per_bin.
__global__ void k_bin_off(const int32_t* __restrict__ offs, int nblk, int32_t nbins, int32_t keys_per_bin,
                          int32_t m, int32_t* __restrict__ bin_off) {
  const int b = threadIdx.x;
  if (b < nbins) bin_off[b] = (nblk > 0) ? offs[static_cast<int64_t>(b) * keys_per_bin * nblk] : 0;
  if (b == nbins) bin_off[b] = m;
}

__global__ void k_seg_count(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ split_rows,
                            int32_t nsplit, int32_t chunk, int32_t* __restrict__ segs) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= nsplit) return;
  const int32_t r = split_rows[s];
  const int32_t L = rowptr[r + 1] - rowptr[r];
  segs[s] = max(1, (L + chunk - 1) / chunk);
}

__global__ void k_seg_fill(const int32_t* __restrict__ seg_first, int32_t nsplit,
                           int32_t* __restrict__ seg_row) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= nsplit) return;
  for (int32_t q = seg_first[s]; q < seg_first[s + 1]; ++q) seg_row[q] = static_cast<int32_t>(s);
}

// Nonzero range of every binned row, in row_perm order (one int2 per row).
__global__ void k_prange(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ row_perm,
                         int32_t m, int2* __restrict__ prange) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t r = row_perm[i];
  prange[i] = make_int2(rowptr[r], rowptr[r + 1]);
}

__global__ void k_zero_i32(int32_t* __restrict__ p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

inline unsigned grid_for(int64_t n, int bs = 256) {
  return static_cast<unsigned>((n + bs - 1) / bs);
}

struct PlanWs {
  int32_t* row_perm;
  int32_t* prange;
  int32_t* counts;
  int32_t* bin_off;
  int32_t* seg_first;
  int32_t* seg_row;
  int32_t* counters;
  double* partials;
  void* scan;
};

bool has_split(const spx_plan_opts& o) { return o.lanes[o.nbins - 1] == 0; }

int32_t keys_per_bin(const spx_plan_opts& o) { return o.row_period > 0 ? kBands : 1; }

// Upper bounds on split rows and segments, from sizes and options only.
void split_bounds(int32_t m, int32_t nnz, const spx_plan_opts& o, int64_t* nsplit, int64_t* nseg) {
  if (!has_split(o)) {
    *nsplit = 0;
    *nseg = 0;
    return;
  }
  const int64_t lo = (o.nbins >= 2) ? o.upper[o.nbins - 2] : 0;  // split rows have L > lo
  int64_t ns = (lo > 0) ? static_cast<int64_t>(nnz) / (lo + 1) : m;
  if (ns > m) ns = m;
  *nsplit = ns;
  *nseg = static_cast<int64_t>(nnz) / o.split_chunk + ns + 1;
}

PlanWs carve_plan(void* ws, int32_t m, int32_t nnz, const spx_plan_opts& o, size_t* bytes) {
  const int64_t nblk = (static_cast<int64_t>(m) + kBinTile - 1) / kBinTile;
  int64_t nsplit, nseg;
  split_bounds(m, nnz, o, &nsplit, &nseg);
  Carve cv(ws, ~size_t(0));
  PlanWs w;
  w.row_perm = cv.take<int32_t>(m > 0 ? m : 1);
  w.prange = cv.take<int32_t>(2 * static_cast<int64_t>(m > 0 ? m : 1));
  w.counts = cv.take<int32_t>(nblk * o.nbins * keys_per_bin(o) + 1);
  w.bin_off = cv.take<int32_t>(SPX_MAX_BINS + 1);
  w.seg_first = cv.take<int32_t>(nsplit + 1);
  w.seg_row = cv.take<int32_t>(nseg + 1);
  w.counters = cv.take<int32_t>(nsplit + 1);
  w.partials = cv.take<double>((nseg + 1) * o.max_k);
  const int64_t nk = nblk * o.nbins * keys_per_bin(o);
  const int64_t sc = nk > nsplit ? nk : nsplit;
  w.scan = cv.take<char>(scan_workspace_bytes(sc + 1));
  *bytes = cv.used;
  return w;
}

spx_status check_opts(const spx_plan_opts* o) {
  if (!o) return fail(SPX_ERR_INVALID, "plan options are null");
  if (o->nbins < 1 || o->nbins > SPX_MAX_BINS)
    return fail(SPX_ERR_INVALID, "nbins=%d outside [1, %d]", o->nbins, SPX_MAX_BINS);
  for (int b = 0; b + 1 < o->nbins; ++b) {
    if (o->upper[b] < 0) return fail(SPX_ERR_INVALID, "upper[%d] < 0", b);
    if (b > 0 && o->upper[b] <= o->upper[b - 1])
      return fail(SPX_ERR_INVALID, "upper[] must increase (upper[%d]=%d <= upper[%d]=%d)", b,
                  o->upper[b], b - 1, o->upper[b - 1]);
  }
  for (int b = 0; b < o->nbins; ++b) {
    const int l = o->lanes[b];
    if (l == 0 && b != o->nbins - 1)
      return fail(SPX_ERR_INVALID, "lanes[%d]=0 (split) allowed only for the last bin", b);
    if (l != 0 && !lanes_valid(l)) return fail(SPX_ERR_INVALID, "lanes[%d]=%d not supported", b, l);
  }
  if (has_split(*o) && (o->split_chunk < 256 || o->split_chunk > SPX_MAX_SPLIT_CHUNK))
    return fail(SPX_ERR_INVALID, "split_chunk=%d outside [256, %d]", o->split_chunk, SPX_MAX_SPLIT_CHUNK);
  if (o->kahan_len < 0) return fail(SPX_ERR_INVALID, "kahan_len < 0");
  if (o->max_k < 1) return fail(SPX_ERR_INVALID, "max_k < 1");
  if (o->occupancy < 0 || o->occupancy > 8)
    return fail(SPX_ERR_INVALID, "occupancy=%d outside [0, 8]", o->occupancy);
  if (o->row_period < 0) return fail(SPX_ERR_INVALID, "row_period=%d < 0", o->row_period);
  return SPX_OK;
}

}  // namespace

int lanes_valid(int l) {
  return l == 1 || l == 2 || l == 4 || l == 8 || l == 16 || l == 32 || l == 64 || l == 256 ||
         l == SPX_LANES_STREAM;
}

}  // namespace spx

using namespace spx;

extern "C" spx_status spx_plan_default_opts(int32_t k, spx_dtype vtype, spx_plan_opts* o) {
  if (!o) return fail(SPX_ERR_INVALID, "spx_plan_default_opts: opts is null");
  if (k < 1) return fail(SPX_ERR_INVALID, "spx_plan_default_opts: k=%d < 1", k);
  *o = spx_plan_opts{};
  o->kahan_len = 256;
  o->max_k = k;
  o->flags = 0;
  if (k == 1) {
    // SpMV: short rows streamed per workgroup, then a wavefront, a workgroup
    // per row, and split segments for the longest rows.
    const int32_t upper[] = {64, 512, 2048, 0};
    const int32_t lanes[] = {SPX_LANES_STREAM, 64, 256, 0};
    o->nbins = 4;
    for (int b = 0; b < 4; ++b) {
      o->upper[b] = upper[b];
      o->lanes[b] = lanes[b];
    }
    o->split_chunk = (vtype == SPX_F64) ? 4096 : 8192;
  } else {
    // SpMM: one X row per KL lanes; more nonzero slots for longer rows.
    // Y rows are written with ordinary stores; timed call by call against
    // non-temporal stores they measure the same (within 0.4 %, k = 1 to 64).
    const int32_t upper[] = {8, 32, 128, 1024, 0};
    const int32_t lanes[] = {1, 8, 32, 64, 0};
    o->flags = SPX_FLAG_NO_NT_STORE;
    o->nbins = 5;
    for (int b = 0; b < 5; ++b) {
      o->upper[b] = upper[b];
      o->lanes[b] = lanes[b];
    }
    o->split_chunk = 4096;
  }
  return SPX_OK;
}

extern "C" spx_status csr_plan_workspace_bytes(int32_t m, int32_t nnz, const spx_plan_opts* opts,
                                               size_t* bytes) {
  if (!bytes) return fail(SPX_ERR_INVALID, "csr_plan_workspace_bytes: bytes is null");
  if (m < 0 || nnz < 0) return fail(SPX_ERR_INVALID, "csr_plan_workspace_bytes: negative size");
  {
    const spx_status s_nnz = check_nnz(nnz, "csr_plan_workspace_bytes");
    if (s_nnz != SPX_OK) return s_nnz;
  }
  spx_status s = check_opts(opts);
  if (s != SPX_OK) return s;
  carve_plan(nullptr, m, nnz, *opts, bytes);
  return SPX_OK;
}

extern "C" spx_status csr_plan_create(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                                      const spx_plan_opts* opts, void* workspace, size_t ws_bytes,
                                      void* stream, spx_plan** out) {
  if (!out) return fail(SPX_ERR_INVALID, "csr_plan_create: out is null");
  *out = nullptr;
  if (m < 0 || n < 0 || nnz < 0) return fail(SPX_ERR_INVALID, "csr_plan_create: negative size");
  {
    const spx_status s_nnz = check_nnz(nnz, "csr_plan_create");
    if (s_nnz != SPX_OK) return s_nnz;
  }
  if (!rowptr) return fail(SPX_ERR_INVALID, "csr_plan_create: rowptr is null");
  spx_status s = check_opts(opts);
  if (s != SPX_OK) return s;
  size_t need;
  carve_plan(nullptr, m, nnz, *opts, &need);
  if (!workspace || ws_bytes < need)
    return fail(SPX_ERR_WORKSPACE, "csr_plan_create: workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t st = as_stream(stream);
  PlanWs w = carve_plan(workspace, m, nnz, *opts, &need);
  const int64_t nblk = (static_cast<int64_t>(m) + kBinTile - 1) / kBinTile;
  BinParams bp{};
  bp.nbins = opts->nbins;
  for (int b = 0; b < SPX_MAX_BINS; ++b) bp.upper[b] = opts->upper[b];
  bp.period = opts->row_period;
  bp.nkeys = opts->nbins * keys_per_bin(*opts);

  if (nblk > 0) {
    k_bin_count<<<static_cast<unsigned>(nblk), kWG, 0, st>>>(rowptr, m, bp, w.counts,
                                                             static_cast<int>(nblk));
    SPX_LAUNCHED("k_bin_count");
    s = exclusive_scan_i32(w.counts, w.counts, nblk * bp.nkeys, nullptr, w.scan, st);
    if (s != SPX_OK) return s;
    k_bin_scatter<<<static_cast<unsigned>(nblk), kWG, 0, st>>>(rowptr, m, bp, w.counts,
                                                               static_cast<int>(nblk), w.row_perm);
    SPX_LAUNCHED("k_bin_scatter");
    k_prange<<<grid_for(m), 256, 0, st>>>(rowptr, w.row_perm, m, reinterpret_cast<int2*>(w.prange));
    SPX_LAUNCHED("k_prange");
  }
  k_bin_off<<<1, 64, 0, st>>>(w.counts, static_cast<int>(nblk), opts->nbins, keys_per_bin(*opts), m,
                              w.bin_off);
  SPX_LAUNCHED("k_bin_off");

  spx_plan* p = new (std::nothrow) spx_plan();
  if (!p) return fail(SPX_ERR_INVALID, "csr_plan_create: out of host memory");
  p->m = m;
  p->n = n;
  p->nnz = nnz;
  p->opts = *opts;
  p->row_perm = w.row_perm;
  p->prange = w.prange;
  p->seg_row = w.seg_row;
  p->seg_first = w.seg_first;
  p->counters = w.counters;
  p->partials = w.partials;
  hipError_t e = hipMemcpyAsync(p->bin_off, w.bin_off, sizeof(int32_t) * (opts->nbins + 1),
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "csr_plan_create: bin offsets");
  }
  p->nsplit = 0;
  p->nseg = 0;
  p->cus = 0;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      p->cus = cus;
  }
  if (has_split(*opts)) {
    const int nb = opts->nbins;
    const int32_t nsplit = p->bin_off[nb] - p->bin_off[nb - 1];
    p->nsplit = nsplit;
    if (nsplit > 0) {
      const int32_t* split_rows = w.row_perm + p->bin_off[nb - 1];
      k_seg_count<<<grid_for(nsplit), 256, 0, st>>>(rowptr, split_rows, nsplit, opts->split_chunk,
                                                    w.seg_first);
      e = hipGetLastError();
      if (e == hipSuccess) {
        s = exclusive_scan_i32(w.seg_first, w.seg_first, nsplit, w.seg_first + nsplit, w.scan, st);
        if (s != SPX_OK) {
          delete p;
          return s;
        }
        k_seg_fill<<<grid_for(nsplit), 256, 0, st>>>(w.seg_first, nsplit, w.seg_row);
        e = hipGetLastError();
      }
      if (e == hipSuccess) {
        k_zero_i32<<<grid_for(nsplit), 256, 0, st>>>(w.counters, nsplit);
        e = hipGetLastError();
      }
      int32_t nseg = 0;
      if (e == hipSuccess)
        e = hipMemcpyAsync(&nseg, w.seg_first + nsplit, sizeof(int32_t), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "csr_plan_create: split segments");
      }
      p->nseg = nseg;
    }
  }
  *out = p;
  return SPX_OK;
}

extern "C" spx_status csr_plan_export_bins(const spx_plan* p, int32_t* host_row_perm,
                                           int32_t* host_bin_off) {
  if (!p) return fail(SPX_ERR_INVALID, "csr_plan_export_bins: plan is null");
  if (p->staged) return fail(SPX_ERR_INVALID, "csr_plan_export_bins: a staged plan has no bins");
  if (host_bin_off)
    for (int b = 0; b <= p->opts.nbins; ++b) host_bin_off[b] = p->bin_off[b];
  if (host_row_perm && p->m > 0)
    SPX_HIP(hipMemcpy(host_row_perm, p->row_perm, sizeof(int32_t) * p->m, hipMemcpyDeviceToHost));
  return SPX_OK;
}

extern "C" spx_status csr_plan_info(const spx_plan* p, int32_t* nbins, int32_t* nsplit_rows,
                                    int32_t* nsegments) {
  if (!p) return fail(SPX_ERR_INVALID, "csr_plan_info: plan is null");
  if (nbins) *nbins = p->opts.nbins;
  if (nsplit_rows) *nsplit_rows = p->nsplit;
  if (nsegments) *nsegments = p->nseg;
  return SPX_OK;
}

extern "C" void csr_plan_destroy(spx_plan* p) { delete p; }

namespace spx {

// A stream bin with fewer tiles than this many per compute unit leaves most
// of the device idle (one 256-row workgroup per CU cannot hide the gather
// latency); row groups of kSmallStreamLanes lanes give 8x the workgroups.
constexpr int kStreamTilesPerCU = 2;
constexpr int kSmallStreamLanes = 8;

void bins_from_plan(const spx_plan* p, ProdArgs& a, int kl, bool own_launch) {
  const spx_plan_opts& o = p->opts;
  int32_t blk = 0;
  int out = 0;
  const bool pad = !(o.flags & SPX_FLAG_NO_XCD_MAP);
  for (int b = o.nbins - 1; b >= 0; --b) {  // long-row bins first
    const int32_t rows = p->bin_off[b + 1] - p->bin_off[b];
    int32_t lanes = o.lanes[b];
    const bool stream = (lanes == SPX_LANES_STREAM);
    if (stream && !(kl == 1 && a.k == 1)) lanes = 1;  // SpMM: row groups of KL lanes
    if (stream && lanes == SPX_LANES_STREAM && own_launch && !(o.flags & SPX_FLAG_KEEP_STREAM) &&
        (static_cast<int64_t>(rows) + kWG - 1) / kWG < static_cast<int64_t>(kStreamTilesPerCU) * p->cus)
      lanes = kSmallStreamLanes;
    const int32_t units = (lanes == 0) ? p->nseg : rows;
    if (units == 0) continue;
    // short-row bins (every row fits one nonzero per slot) serve 4 rows per
    // group to raise the number of independent loads in flight
    int32_t rpg = 1;
    if (kl == 1 && a.k == 1 && !(o.flags & SPX_FLAG_ONE_ROW) && lanes != 0 && lanes <= 32 &&
        b < o.nbins - 1) {
      const int32_t slots = lanes >= kl ? lanes / kl : 1;
      if (o.upper[b] <= slots) rpg = 4;
    }
    int32_t rpb = 1;
    if (lanes == SPX_LANES_STREAM) rpb = kWG;  // one row per thread
    else if (lanes != 0) rpb = (kWG / (lanes > kl ? lanes : kl)) * rpg;
    if (rpb < 1) rpb = 1;
    int32_t nblk = (units + rpb - 1) / rpb;
    if (pad) nblk = (nblk + 7) / 8 * 8;
    BinDesc& d = a.bins[out++];
    d.blk_begin = blk;
    d.nblk = nblk;
    d.row_begin = p->bin_off[b];
    d.nrows = units;
    d.lanes = lanes;
    d.bin = b;
    d.rpg = rpg;
    blk += nblk;
  }
  a.nbins = out;
  a.row_perm = p->row_perm;
  a.prange = p->prange;
  a.seg_row = p->seg_row;
  a.seg_first = p->seg_first;
  a.split_rows = p->row_perm + p->bin_off[o.nbins - 1];
  a.counters = p->counters;
  a.partials = p->partials;
  a.chunk = o.split_chunk;
  a.max_k = o.max_k;
  a.kahan_len = o.kahan_len;
  a.flags = o.flags;
  a.occupancy = o.occupancy;
}

void bins_unbinned(int32_t m, int32_t nnz, int kl, ProdArgs& a) {
  // lanes per row from the mean row length (no plan: natural row order)
  const double mean = (m > 0) ? static_cast<double>(nnz) / m : 0.0;
  int lanes = 1;
  if (kl == 1) {
    while (lanes < 64 && lanes < mean) lanes <<= 1;
  } else {
    lanes = kl;
    while (lanes < 64 && lanes < kl * mean / 8.0) lanes <<= 1;
  }
  const int gg = lanes > kl ? lanes : kl;
  const int rpb = kWG / gg;
  int32_t nblk = (m + rpb - 1) / rpb;
  nblk = (nblk + 7) / 8 * 8;
  a.nbins = (m > 0) ? 1 : 0;
  BinDesc& d = a.bins[0];
  d.blk_begin = 0;
  d.nblk = nblk;
  d.row_begin = 0;
  d.nrows = m;
  d.lanes = lanes;
  d.bin = 0;
  d.rpg = 1;
  a.row_perm = nullptr;
  a.prange = nullptr;
  a.seg_row = nullptr;
  a.seg_first = nullptr;
  a.split_rows = nullptr;
  a.counters = nullptr;
  a.partials = nullptr;
  a.chunk = 0;
  a.max_k = a.k;
  a.kahan_len = 256;
  a.flags = 0;
}

}  // namespace spx
