// scan_sort.hip -- device-wide exclusive scan and stable LSD radix sort.
//
// Used once per sparsity pattern: to assemble CSR from triplets, to bin rows
// and to build the CSC index of the transpose.  Tiles are 4096 items (256
// threads x 16).  Integer arithmetic only; results are deterministic.
#include "device.hpp"
#include "internal.hpp"

namespace spx {

namespace {

constexpr int kItems = 16;

__device__ __forceinline__ int32_t wave_incl_scan(int32_t v, int lane) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int32_t u = __shfl_up(v, off, kWave);
    if (lane >= off) v += u;
  }
  return v;
}

// Exclusive scan of one value per thread over the 256-thread block; returns
// the thread's exclusive prefix and writes the block total to *total.
__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t* total) {
  __shared__ int32_t wsum[kWG / kWave];
  const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
  int32_t inc = wave_incl_scan(v, lane);
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  int32_t before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kWG / kWave; ++i) {
    if (i < w) before += wsum[i];
    all += wsum[i];
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

__global__ __launch_bounds__(kWG) void k_scan_reduce(const int32_t* __restrict__ in, int64_t n,
                                                     int32_t* __restrict__ sums) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
  int32_t s = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    int64_t i = base + j * kWG + threadIdx.x;
    if (i < n) s += in[i];
  }
  int32_t total;
  (void)block_excl_scan(s, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Scan one tile per block with the tile's offset (offs == null: offset 0).
__global__ __launch_bounds__(kWG) void k_scan_apply(const int32_t* in, int32_t* out, int64_t n,
                                                    const int32_t* __restrict__ offs,
                                                    int32_t* total_out) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kItems;
  int32_t item[kItems];
  int32_t s = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    int64_t i = base + j;
    item[j] = (i < n) ? in[i] : 0;
    s += item[j];
  }
  int32_t total;
  int32_t run = block_excl_scan(s, &total) + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    int64_t i = base + j;
    if (i < n) out[i] = run;
    run += item[j];
  }
  if (total_out && threadIdx.x == 0) *total_out = total;
}

template <typename K>
__global__ __launch_bounds__(kWG) void k_radix_hist(const K* __restrict__ keys, int64_t n,
                                                    int shift, int32_t* __restrict__ hist,
                                                    int nblk) {
  __shared__ int32_t cnt[256];
  const int t = threadIdx.x;
  cnt[t] = 0;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    int64_t i = base + j * kWG + t;
    if (i < n) atomicAdd(&cnt[static_cast<uint32_t>(keys[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[static_cast<int64_t>(t) * nblk + blockIdx.x] = cnt[t];
}

// Stable scatter: items are ranked in (round, wave, lane) order, which is
// their input order inside the tile.  Lanes with the same digit are found by
// matching the 8 digit bits with ballots.
template <typename K>
__global__ __launch_bounds__(kWG) void k_radix_scatter(const K* __restrict__ kin,
                                                       const int32_t* __restrict__ vin,
                                                       K* __restrict__ kout,
                                                       int32_t* __restrict__ vout, int64_t n,
                                                       int shift,
                                                       const int32_t* __restrict__ offs,
                                                       int nblk) {
  __shared__ int32_t run[256];
  __shared__ int32_t wcnt[kWG / kWave][256];
  const int t = threadIdx.x, w = t / kWave, lane = t % kWave;
  const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  run[t] = offs[static_cast<int64_t>(t) * nblk + blockIdx.x];
#pragma unroll
  for (int i = 0; i < kWG / kWave; ++i) wcnt[i][t] = 0;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = base + j * kWG + t;
    const bool valid = i < n;
    K key = valid ? kin[i] : K(0);
    int32_t val = valid ? vin[i] : 0;
    const uint32_t d = static_cast<uint32_t>(key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const int rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int32_t pos = run[d] + rank;
      for (int v = 0; v < w; ++v) pos += wcnt[v][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    int32_t add = 0;
#pragma unroll
    for (int v = 0; v < kWG / kWave; ++v) {
      add += wcnt[v][t];
      wcnt[v][t] = 0;
    }
    run[t] += add;
    __syncthreads();
  }
}

inline int64_t ntiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

}  // namespace

size_t scan_workspace_bytes(int64_t n) {
  size_t b = 0;
  while (n > kScanTile) {
    n = ntiles(n);
    b += align_up(static_cast<size_t>(n) * sizeof(int32_t));
  }
  return b + 256;
}

spx_status exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total,
                              void* ws, hipStream_t st) {
  if (n <= 0) {
    if (total) SPX_HIP(hipMemsetAsync(total, 0, sizeof(int32_t), st));
    return SPX_OK;
  }
  if (n <= kScanTile) {
    k_scan_apply<<<1, kWG, 0, st>>>(in, out, n, nullptr, total);
    SPX_LAUNCHED("k_scan_apply");
    return SPX_OK;
  }
  const int64_t nb = ntiles(n);
  int32_t* sums = static_cast<int32_t*>(ws);
  void* rest = static_cast<char*>(ws) + align_up(static_cast<size_t>(nb) * sizeof(int32_t));
  k_scan_reduce<<<static_cast<unsigned>(nb), kWG, 0, st>>>(in, n, sums);
  SPX_LAUNCHED("k_scan_reduce");
  spx_status s = exclusive_scan_i32(sums, sums, nb, total, rest, st);
  if (s != SPX_OK) return s;
  k_scan_apply<<<static_cast<unsigned>(nb), kWG, 0, st>>>(in, out, n, sums, nullptr);
  SPX_LAUNCHED("k_scan_apply");
  return SPX_OK;
}

size_t radix_workspace_bytes(int64_t n, int key_bytes) {
  const int64_t nb = ntiles(n > 0 ? n : 1);
  return align_up(static_cast<size_t>(n) * key_bytes) + align_up(static_cast<size_t>(n) * 4) +
         align_up(static_cast<size_t>(nb) * 256 * 4) + scan_workspace_bytes(nb * 256);
}

template <typename K>
static spx_status radix_sort(K* keys, int32_t* vals, int64_t n, int bits, void* ws, hipStream_t st) {
  if (n <= 1 || bits <= 0) return SPX_OK;
  const int64_t nb = ntiles(n);
  Carve cv(ws, ~size_t(0));
  K* k2 = cv.take<K>(n);
  int32_t* v2 = cv.take<int32_t>(n);
  int32_t* hist = cv.take<int32_t>(nb * 256);
  void* sws = cv.take<char>(scan_workspace_bytes(nb * 256));
  K* ka = keys;
  int32_t* va = vals;
  K* kb = k2;
  int32_t* vb = v2;
  int passes = 0;
  for (int shift = 0; shift < bits; shift += 8, ++passes) {
    k_radix_hist<K><<<static_cast<unsigned>(nb), kWG, 0, st>>>(ka, n, shift, hist, static_cast<int>(nb));
    SPX_LAUNCHED("k_radix_hist");
    spx_status s = exclusive_scan_i32(hist, hist, nb * 256, nullptr, sws, st);
    if (s != SPX_OK) return s;
    k_radix_scatter<K><<<static_cast<unsigned>(nb), kWG, 0, st>>>(ka, va, kb, vb, n, shift, hist,
                                                                 static_cast<int>(nb));
    SPX_LAUNCHED("k_radix_scatter");
    K* tk = ka; ka = kb; kb = tk;
    int32_t* tv = va; va = vb; vb = tv;
  }
  if (passes & 1) {
    SPX_HIP(hipMemcpyAsync(keys, ka, static_cast<size_t>(n) * sizeof(K), hipMemcpyDeviceToDevice, st));
    SPX_HIP(hipMemcpyAsync(vals, va, static_cast<size_t>(n) * 4, hipMemcpyDeviceToDevice, st));
  }
  return SPX_OK;
}

spx_status radix_sort_u32(uint32_t* keys, int32_t* vals, int64_t n, int bits, void* ws,
                          hipStream_t st) {
  return radix_sort<uint32_t>(keys, vals, n, bits, ws, st);
}
spx_status radix_sort_u64(uint64_t* keys, int32_t* vals, int64_t n, int bits, void* ws,
                          hipStream_t st) {
  return radix_sort<uint64_t>(keys, vals, n, bits, ws, st);
}

}  // namespace spx
