// device.hpp -- device helpers shared by the gfx950 kernels of libspx.
//
// Wavefronts are 64 lanes.  Cross-lane sums use DPP (quad_perm,
// row_half_mirror, row_mirror) inside 16-lane rows, ds_swizzle for the
// 16-lane exchange and ds_bpermute (__shfl_xor) across the two wave halves.
// Every reduction runs with all 64 lanes active and in a fixed order, so
// results are deterministic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spx {

constexpr int kWG = 256;   // threads per workgroup of every product kernel
constexpr int kWave = 64;  // CDNA wavefront width

// ------------------------------------------------------------------ loads / stores

// Loads of the matrix stream (colind, values).  With NT they are
// non-temporal, so a stream read once does not evict gathered x lines from
// L2; a kernel that comes back to a line (the lanes of an SpMM row group
// walk a row over several rounds) loads it normally.
template <bool NT, typename T>
__device__ __forceinline__ T ld_mat(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return ld_mat<true>(p);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

// Value element types: double, float, or bf16 stored as uint16.
template <typename VT>
struct ValueLoad;
template <>
struct ValueLoad<double> {
  using Raw = double;
  template <bool NT = true>
  static __device__ __forceinline__ double get(const double* p) { return ld_mat<NT>(p); }
  template <bool NT = true>
  static __device__ __forceinline__ Raw raw(const double* p) { return ld_mat<NT>(p); }
  static __device__ __forceinline__ double widen(Raw r) { return r; }
};
template <>
struct ValueLoad<float> {
  using Raw = float;
  template <bool NT = true>
  static __device__ __forceinline__ float get(const float* p) { return ld_mat<NT>(p); }
  template <bool NT = true>
  static __device__ __forceinline__ Raw raw(const float* p) { return ld_mat<NT>(p); }
  static __device__ __forceinline__ float widen(Raw r) { return r; }
};
// BF16: raw() keeps the stored bits so that a caller can defer the widening
// until the value is used (widening right after a masked load makes the
// compiler wait for that load on the spot).
template <>
struct ValueLoad<uint16_t> {
  using Raw = uint16_t;
  template <bool NT = true>
  static __device__ __forceinline__ float get(const uint16_t* p) {
    return bf16_to_f32(ld_mat<NT>(p));
  }
  template <bool NT = true>
  static __device__ __forceinline__ Raw raw(const uint16_t* p) { return ld_mat<NT>(p); }
  static __device__ __forceinline__ float widen(Raw r) { return bf16_to_f32(r); }
};

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// ------------------------------------------------------------------ cross-lane moves

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int XOR>
__device__ __forceinline__ int swz_i(int v) {
  static_assert(XOR > 0 && XOR < 32, "ds_swizzle bit mode covers lanes within 32");
  return __builtin_amdgcn_ds_swizzle(v, 0x1F | (XOR << 10));
}

// lane i receives the value of lane i ^ OFF (OFF a power of two < 64)
template <int OFF>
__device__ __forceinline__ int xchg_i(int v) {
  if constexpr (OFF == 32) {
    return __shfl_xor(v, 32, 64);
  } else {
    return swz_i<OFF>(v);
  }
}

template <typename T>
struct Lanes;
template <>
struct Lanes<float> {
  template <int CTRL>
  static __device__ __forceinline__ float dpp(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
  }
  template <int OFF>
  static __device__ __forceinline__ float xchg(float v) {
    return __int_as_float(xchg_i<OFF>(__float_as_int(v)));
  }
};
template <>
struct Lanes<double> {
  template <int CTRL>
  static __device__ __forceinline__ double dpp(double v) {
    int lo = dpp_i<CTRL>(__double2loint(v));
    int hi = dpp_i<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
  }
  template <int OFF>
  static __device__ __forceinline__ double xchg(double v) {
    int lo = xchg_i<OFF>(__double2loint(v));
    int hi = xchg_i<OFF>(__double2hiint(v));
    return __hiloint2double(hi, lo);
  }
};

// DPP controls (GFX9 encoding)
constexpr int kDppQuadXor1 = 0xB1;    // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;    // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <- lane 7-i within 8
constexpr int kDppMirror = 0x140;     // lane i <- lane 15-i within 16

// Sum over the lanes of an aligned group of G lanes that share (lane % KL).
// On return every such lane holds the group sum.  Must be called by all 64
// lanes of the wave (uniform control flow).  G, KL powers of two, KL <= G <= 64.
template <int G, int KL, typename T>
__device__ __forceinline__ T group_sum(T v) {
  using L = Lanes<T>;
  if constexpr (KL == 1) {
    if constexpr (G >= 2) v += L::template dpp<kDppQuadXor1>(v);
    if constexpr (G >= 4) v += L::template dpp<kDppQuadXor2>(v);
    if constexpr (G >= 8) v += L::template dpp<kDppHalfMirror>(v);
    if constexpr (G >= 16) v += L::template dpp<kDppMirror>(v);
    if constexpr (G >= 32) v += L::template xchg<16>(v);
    if constexpr (G >= 64) v += L::template xchg<32>(v);
  } else {
    if constexpr (KL <= 1 && G >= 2) v += L::template xchg<1>(v);
    if constexpr (KL <= 2 && G >= 4) v += L::template xchg<2>(v);
    if constexpr (KL <= 4 && G >= 8) v += L::template xchg<4>(v);
    if constexpr (KL <= 8 && G >= 16) v += L::template xchg<8>(v);
    if constexpr (KL <= 16 && G >= 32) v += L::template xchg<16>(v);
    if constexpr (KL <= 32 && G >= 64) v += L::template xchg<32>(v);
  }
  return v;
}

// ------------------------------------------------------------------ compensated FP32

// Error-free transforms (Knuth TwoSum; TwoProduct via FMA).  Contraction is
// switched off so the compiler cannot fuse the products into the sums.
struct Comp {
  float s;  // running sum
  float c;  // accumulated rounding errors (sum and products)
  __device__ __forceinline__ void init() { s = 0.0f; c = 0.0f; }
  __device__ __forceinline__ void add_prod(float a, float b) {
#pragma clang fp contract(off)
    float p = a * b;
    float pe = __builtin_fmaf(a, b, -p);
    float t = s + p;
    float bb = t - s;
    float e = (s - (t - bb)) + (p - bb);
    s = t;
    c = c + (e + pe);
  }
  __device__ __forceinline__ double value() const {
    return static_cast<double>(s) + static_cast<double>(c);
  }
};

// ------------------------------------------------------------------ XCD-aware tiles

// Workgroups of one launch are dispatched round-robin over the 8 XCDs
// (workgroup b runs on XCD b % 8).  For a range of `nblk` workgroups that
// starts at a multiple of 8, map local workgroup lb to a tile such that each
// XCD processes one contiguous eighth of the tiles: neighbouring rows then
// share an XCD's L2 (x lines of banded matrices stay in one L2).
__device__ __forceinline__ int xcd_tile(int lb, int nblk) {
  if (nblk & 7) return lb;
  int per = nblk >> 3;
  return (lb & 7) * per + (lb >> 3);
}

}  // namespace spx
