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

}  // namespace
}  // namespace spx

using namespace spx;

// kind: 0 read, 1 write, 2 write non-temporal, 3 copy (src = buf, dst = buf2),
// 4 flush (read-modify-write).  bytes is rounded down to 16-byte units.
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
    default: return fail(SPX_ERR_INVALID, "spx_probe: kind=%d", kind);
  }
  SPX_LAUNCHED("spx_probe");
  return SPX_OK;
}
