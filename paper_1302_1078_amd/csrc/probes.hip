// probes.hip -- memory-system probes, the GPU counterparts of the paper's
// read / write bandwidth microbenchmarks (Sec. 2.1, Sec. 2.2): a streaming
// read, a streaming write (plain or non-temporal), a copy, and a cache
// flush (read-modify-write of a large buffer).  They give the measured
// bandwidth the products are compared with.
#include "device.hpp"
#include "internal.hpp"

namespace spx {
namespace {

typedef double d2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(kWG) void k_probe_read(const d2* __restrict__ p, int64_t n, double* out) {
  d2 acc = {0.0, 0.0};
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kWG;
  int64_t i = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const d2 a = __builtin_nontemporal_load(p + i);
    const d2 b = __builtin_nontemporal_load(p + i + stride);
    const d2 c = __builtin_nontemporal_load(p + i + 2 * stride);
    const d2 e = __builtin_nontemporal_load(p + i + 3 * stride);
    acc += a + b + c + e;
  }
  for (; i < n; i += stride) acc += __builtin_nontemporal_load(p + i);
  const double s = acc[0] + acc[1];
  if (out && s == 12345.678) out[0] = s;  // keeps the loads live
}

__global__ __launch_bounds__(kWG) void k_probe_write(d2* __restrict__ p, int64_t n, int nt, double v) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kWG;
  const d2 val = {v, v};
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; i < n; i += stride) {
    if (nt) __builtin_nontemporal_store(val, p + i);
    else p[i] = val;
  }
}

__global__ __launch_bounds__(kWG) void k_probe_copy(const d2* __restrict__ s, d2* __restrict__ d, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kWG;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(s + i), d + i);
}

__global__ __launch_bounds__(kWG) void k_probe_flush(d2* __restrict__ p, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kWG;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; i < n; i += stride)
    p[i] = p[i] + 1.0;
}

// Random gathers: the access pattern of the products' x / X reads, without
// the matrix stream.  Every wave makes kGatherIters rounds; a round of
// kind 5 reads 8 random 128-byte rows (8 lanes x 16 bytes each, the SpMM
// layout for k = 16 FP64), a round of kind 6 reads 64 random 8-byte
// elements (the SpMV x gather).  Four rounds are in flight per lane.
constexpr int kGatherIters = 256;

__device__ __forceinline__ uint32_t scramble(uint32_t v) {  // an integer hash (xorshift-multiply)
  v ^= v >> 16;
  v *= 0x7feb352dU;
  v ^= v >> 15;
  v *= 0x846ca68bU;
  v ^= v >> 16;
  return v;
}

// A hash mapped onto [0, n) by its high product word (multiply-shift range
// reduction): one instruction, so the probe's own arithmetic stays far below
// its memory time (a 64-bit remainder here cost about 90 instructions per
// element).
__device__ __forceinline__ uint32_t below(uint32_t h, uint32_t n) { return __umulhi(h, n); }

template <bool ROWS>
__global__ __launch_bounds__(kWG) void k_probe_gather(const double* __restrict__ p, uint32_t n, double* out) {
  const int lane = threadIdx.x % kWave;
  const uint32_t wave = blockIdx.x * (kWG / kWave) + threadIdx.x / kWave;
  const uint32_t rows = n / 16;  // 128-byte rows
  double acc = 0.0;
  for (int it = 0; it < kGatherIters; it += 4) {
    d2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t h = scramble(wave * 977u + static_cast<uint32_t>(it + u) * 131u);
      if (ROWS) {
        const uint32_t r = below(scramble(h + lane / 8), rows);
        v[u] = *reinterpret_cast<const d2*>(p + static_cast<size_t>(r) * 16 + (lane % 8) * 2);
      } else {
        v[u] = d2{p[below(scramble(h + lane), n)], 0.0};
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += v[u][0] + v[u][1];
  }
  if (out && acc == 12345.678) out[0] = acc;
}

// Index-driven gather: the x access of an SpMV without its values.  Workgroup
// b serves one contiguous range of idx (XCD-contiguous like the product
// tiles); its lanes stream idx with non-temporal loads, 4 per lane in flight,
// and add x[idx[p]] (GATHER) or idx[p] itself (the index stream alone).  Each
// workgroup writes its partial sum to sink[tile], so the result is
// deterministic and every load stays live.
template <bool GATHER>
__global__ __launch_bounds__(kWG) void k_probe_idx(const int32_t* __restrict__ idx, int64_t nidx,
                                                   const double* __restrict__ x, int32_t n, int64_t per,
                                                   double* __restrict__ sink) {
  __shared__ double part[kWG / kWave];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t b = static_cast<int64_t>(tile) * per;
  const int64_t e = (b + per < nidx) ? b + per : nidx;
  double acc = 0.0;
  for (int64_t p = b + threadIdx.x; p < e; p += 4 * kWG) {
    int32_t c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) c[u] = (p + u * kWG < e) ? ld_stream(idx + p + u * kWG) : -1;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (c[u] < 0) continue;  // past the range
      if (GATHER) {
        if (c[u] < n) acc += x[c[u]];  // an index outside x is skipped, never read
      } else {
        acc += static_cast<double>(c[u]);
      }
    }
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
  if (threadIdx.x % kWave == 0) part[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kWG / kWave; ++w) s += part[w];
    sink[tile] = s;
  }
}

// Pointer chase: one wavefront; lane l starts at start[l] and follows
// i <- next[i] & mask for `hops` dependent loads, then writes its final index
// to out[l].  The mask keeps every load inside the buffer whatever it holds.
__global__ __launch_bounds__(kWave) void k_probe_chase(const int32_t* __restrict__ next, uint32_t mask,
                                                       const int32_t* __restrict__ start, int64_t hops,
                                                       int32_t* __restrict__ out) {
  uint32_t i = static_cast<uint32_t>(start[threadIdx.x]) & mask;
  for (int64_t h = 0; h < hops; ++h) i = static_cast<uint32_t>(next[i]) & mask;
  out[threadIdx.x] = static_cast<int32_t>(i);
}

}  // namespace
}  // namespace spx

using namespace spx;

extern "C" spx_status spx_probe_index_gather(const int32_t* idx, int64_t nidx, const double* x, int32_t n,
                                             int32_t gather, double* sink, int32_t blocks, void* stream) {
  if (nidx < 0 || n < 0) return fail(SPX_ERR_INVALID, "spx_probe_index_gather: negative size");
  if (blocks <= 0 || (blocks & 7)) return fail(SPX_ERR_INVALID, "spx_probe_index_gather: blocks=%d (a positive multiple of 8)", blocks);
  if (!sink) return fail(SPX_ERR_INVALID, "spx_probe_index_gather: sink is null");
  if (nidx > 0 && (!idx || (gather && !x))) return fail(SPX_ERR_INVALID, "spx_probe_index_gather: null input");
  if (gather && nidx > 0 && n == 0) return fail(SPX_ERR_INVALID, "spx_probe_index_gather: gather from an empty x");
  const int64_t per = (nidx + blocks - 1) / blocks;
  hipStream_t st = as_stream(stream);
  if (gather) k_probe_idx<true><<<static_cast<unsigned>(blocks), kWG, 0, st>>>(idx, nidx, x, n, per, sink);
  else k_probe_idx<false><<<static_cast<unsigned>(blocks), kWG, 0, st>>>(idx, nidx, x, n, per, sink);
  SPX_LAUNCHED("spx_probe_index_gather");
  return SPX_OK;
}

extern "C" spx_status spx_probe_chase(const int32_t* next, int64_t n, const int32_t* start, int64_t hops,
                                      int32_t* out, void* stream) {
  if (n < 1 || n > (int64_t(1) << 31) || (n & (n - 1)))
    return fail(SPX_ERR_INVALID, "spx_probe_chase: n=%lld is not a power of two in [1, 2^31]", (long long)n);
  if (hops < 0) return fail(SPX_ERR_INVALID, "spx_probe_chase: hops < 0");
  if (!next || !start || !out) return fail(SPX_ERR_INVALID, "spx_probe_chase: null pointer");
  k_probe_chase<<<1, kWave, 0, as_stream(stream)>>>(next, static_cast<uint32_t>(n - 1), start, hops, out);
  SPX_LAUNCHED("spx_probe_chase");
  return SPX_OK;
}

// kind: 0 read, 1 write, 2 write non-temporal, 3 copy (src = buf, dst = buf2),
// 4 flush (read-modify-write), 5 random 128-byte row gather, 6 random 8-byte
// gather.  bytes is rounded down to 16-byte units.
extern "C" spx_status spx_probe(int32_t kind, void* buf, void* buf2, size_t bytes, int32_t blocks,
                                void* stream) {
  if (!buf || bytes < 16) return fail(SPX_ERR_INVALID, "spx_probe: empty buffer");
  if (kind == 3 && !buf2) return fail(SPX_ERR_INVALID, "spx_probe: copy needs a destination");
  if ((reinterpret_cast<uintptr_t>(buf) & 15u) || (buf2 && (reinterpret_cast<uintptr_t>(buf2) & 15u)))
    return fail(SPX_ERR_INVALID, "spx_probe: buffers must be 16-byte aligned");
  const int64_t n = static_cast<int64_t>(bytes / 16);
  const unsigned g = static_cast<unsigned>(blocks > 0 ? blocks : 4096);
  hipStream_t st = as_stream(stream);
  d2* p = static_cast<d2*>(buf);
  switch (kind) {
    case 0: k_probe_read<<<g, kWG, 0, st>>>(p, n, static_cast<double*>(buf2)); break;
    case 1: k_probe_write<<<g, kWG, 0, st>>>(p, n, 0, 1.0); break;
    case 2: k_probe_write<<<g, kWG, 0, st>>>(p, n, 1, 1.0); break;
    case 3: k_probe_copy<<<g, kWG, 0, st>>>(p, static_cast<d2*>(buf2), n); break;
    case 4: k_probe_flush<<<g, kWG, 0, st>>>(p, n); break;
    case 5:
    case 6: {
      const int64_t elems = static_cast<int64_t>(bytes / 8);
      if ((kind == 5 && elems < 16) || elems < 1) return fail(SPX_ERR_INVALID, "spx_probe: gather buffer too small");
      if (elems > 0xffffffffLL) return fail(SPX_ERR_INVALID, "spx_probe: gather buffer above 2^32 elements");
      const uint32_t ne = static_cast<uint32_t>(elems);
      if (kind == 5) k_probe_gather<true><<<g, kWG, 0, st>>>(static_cast<const double*>(buf), ne, static_cast<double*>(buf2));
      else k_probe_gather<false><<<g, kWG, 0, st>>>(static_cast<const double*>(buf), ne, static_cast<double*>(buf2));
      break;
    }
    default: return fail(SPX_ERR_INVALID, "spx_probe: kind=%d", kind);
  }
  SPX_LAUNCHED("spx_probe");
  return SPX_OK;
}
