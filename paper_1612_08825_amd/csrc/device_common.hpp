// Device helpers shared by the gfx950 kernels: element conversion, vector
// loads of 8 pixels, error-free transformations, and wave64 cross-lane
// reductions built on DPP.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace ttc {

// Pointers into device memory given to the kernels are generic; reading through
// a generic pointer compiles to FLAT instructions, whose completion is counted
// together with LDS operations, so every wait on an LDS read would also wait
// for all outstanding frame loads.  Loads and stores of frame data and partial
// sums therefore go through explicitly global (address space 1) pointers.
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)(p);
}
template <typename T> __device__ __forceinline__ gptr<const T> as_global(const T* p) {
  return (gptr<const T>)(p);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// ---- scalar element conversion ---------------------------------------------
template <typename T> __device__ __forceinline__ float to_f32(T v);
template <> __device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_f32<uint8_t>(uint8_t v) { return (float)v; }
template <> __device__ __forceinline__ float to_f32<_Float16>(_Float16 v) { return (float)v; }

// ---- eight consecutive pixels held in raw form -------------------------------
// u8: 8 bytes in two dwords; f16: 8 halves in four dwords.  The raw form is what
// the fused TTC kernel keeps of the previous frame, so it is kept packed.
template <typename T> struct Raw8;

template <> struct Raw8<uint8_t> {
  uint32_t d[2];
  __device__ __forceinline__ void zero() { d[0] = d[1] = 0u; }
  __device__ __forceinline__ void load(const uint8_t* p) {
    const u32x2 v = *as_global(reinterpret_cast<const u32x2*>(p));
    d[0] = v.x;
    d[1] = v.y;
  }
  __device__ __forceinline__ void load_partial(const uint8_t* p, int n) {
    const gptr<const uint8_t> g = as_global(p);
    uint32_t w[2] = {0u, 0u};
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (c < n) w[c >> 2] |= (uint32_t)g[c] << (8 * (c & 3));
    d[0] = w[0];
    d[1] = w[1];
  }
  __device__ __forceinline__ void unpack(float* f) const {
#pragma unroll
    for (int c = 0; c < 8; ++c) f[c] = (float)((d[c >> 2] >> (8 * (c & 3))) & 0xffu);
  }
  // Temporal sum and difference with the same pixels of the previous frame:
  // S = old + this, D = this - old, in FP32 (exact: integers below 2^9).
  __device__ __forceinline__ void sum_diff(const Raw8& old, float (&S)[8], float (&D)[8]) const {
    float a[8], b[8];
    old.unpack(a);
    unpack(b);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      S[c] = a[c] + b[c];
      D[c] = b[c] - a[c];
    }
  }
};

template <> struct Raw8<_Float16> {
  uint32_t d[4];
  __device__ __forceinline__ void zero() { d[0] = d[1] = d[2] = d[3] = 0u; }
  __device__ __forceinline__ void load(const _Float16* p) {
    const u32x4 v = *as_global(reinterpret_cast<const u32x4*>(p));
    d[0] = v.x;
    d[1] = v.y;
    d[2] = v.z;
    d[3] = v.w;
  }
  __device__ __forceinline__ void load_partial(const _Float16* p, int n) {
    const gptr<const uint16_t> q = as_global(reinterpret_cast<const uint16_t*>(p));
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (c < n) w[c >> 1] |= (uint32_t)q[c] << (16 * (c & 1));
#pragma unroll
    for (int i = 0; i < 4; ++i) d[i] = w[i];
  }
  __device__ __forceinline__ void unpack(float* f) const {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const uint16_t h = (uint16_t)((d[c >> 1] >> (16 * (c & 1))) & 0xffffu);
      f[c] = (float)__builtin_bit_cast(_Float16, h);
    }
  }
};

// ---- error-free transformations ---------------------------------------------
// TwoSum (Knuth): s + e == a + b exactly, s = fl(a + b).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// (hi, lo) += v with the rounding error of the high part carried in lo.
__device__ __forceinline__ void comp_add(float& hi, float& lo, float v) {
  float s, e;
  two_sum(hi, v, s, e);
  hi = s;
  lo += e;
}

// (hi, lo) += (h2, l2).
__device__ __forceinline__ void comp_merge(float& hi, float& lo, float h2, float l2) {
  float s, e;
  two_sum(hi, h2, s, e);
  hi = s;
  lo = lo + l2 + e;
}

// ---- cross-lane moves ---------------------------------------------------------
// DPP controls (gfx9 encoding): quad_perm [1,0,3,2] swaps neighbours (lane ^ 1),
// quad_perm [2,3,0,1] swaps pairs (lane ^ 2), row_half_mirror reverses each
// group of 8 lanes, row_mirror reverses each row of 16 lanes.  Each of the four
// pairs every lane with a partner in the other half of the group it is
// summing, so applying them in this order leaves every lane of a 16-lane row
// holding the row total.
constexpr int kDppQuadXor1 = 0xB1;
constexpr int kDppQuadXor2 = 0x4E;
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

// Sum over the 16 lanes of the lane's row; every lane receives the total.
__device__ __forceinline__ float row16_allreduce(float v) {
  v += dpp_f32<kDppQuadXor1>(v);
  v += dpp_f32<kDppQuadXor2>(v);
  v += dpp_f32<kDppRowHalfMirror>(v);
  v += dpp_f32<kDppRowMirror>(v);
  return v;
}

// Sum over all 64 lanes; every lane receives the total.
__device__ __forceinline__ float wave64_allreduce(float v) {
  v = row16_allreduce(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

}  // namespace ttc
