// Materialised pyramid level and derivative cube (the decomposed path).
//
// pyramid_level: P_{l+1}[i][j] = ((P_l[2i][2j] + P_l[2i][2j+1]) + (P_l[2i+1][2j] + P_l[2i+1][2j+1])) * 0.25
// horn_cube:     E_x, E_y, E_t of the 2x2x2 first-difference cube between two
//                frames, one thread per cube; F32 outputs hold E, I32 outputs
//                (u8 frames) hold the exact numerators 4E.
#include "device_common.hpp"
#include "internal.hpp"

namespace ttc {
namespace {

// Grid rows for a kernel that loops over `rows` rows with a stride of
// gridDim.y (the grid's y extent is limited to 65535).
unsigned grid_rows(int64_t rows) { return (unsigned)(rows < 65535 ? (rows > 0 ? rows : 1) : 65535); }

template <typename T>
__global__ __launch_bounds__(256) void pyramid_level(const T* __restrict__ src, int64_t s0, int64_t s1,
                                                      float* __restrict__ dst, int64_t d0, int64_t d1, int Ho,
                                                      int Wo) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Wo) return;
  for (int i = blockIdx.y; i < Ho; i += gridDim.y) {
    const T* r0 = src + (int64_t)(2 * i) * s0 + (int64_t)(2 * j) * s1;
    const T* r1 = r0 + s0;
    const float a = to_f32<T>(r0[0]), b = to_f32<T>(r0[s1]);
    const float c = to_f32<T>(r1[0]), d = to_f32<T>(r1[s1]);
    dst[(int64_t)i * d0 + (int64_t)j * d1] = ((a + b) + (c + d)) * 0.25f;
  }
}

template <typename T, typename TO>
__global__ __launch_bounds__(256) void horn_cube(const T* __restrict__ p0, int64_t a0, int64_t a1,
                                                  const T* __restrict__ p1, int64_t b0, int64_t b1, int H, int W,
                                                  TO* __restrict__ ex, int64_t x0, int64_t x1, TO* __restrict__ ey,
                                                  int64_t y0, int64_t y1, TO* __restrict__ et, int64_t t0,
                                                  int64_t t1) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= W - 1) return;
  for (int i = blockIdx.y; i < H - 1; i += gridDim.y) {
    using TA = typename std::conditional<std::is_same<TO, int>::value, int, float>::type;
    auto ld = [](const T* p, int64_t s0, int64_t s1, int r, int c) -> TA {
      return (TA)to_f32<T>(p[(int64_t)r * s0 + (int64_t)c * s1]);
    };
    const TA a00 = ld(p0, a0, a1, i, j), a01 = ld(p0, a0, a1, i, j + 1);
    const TA a10 = ld(p0, a0, a1, i + 1, j), a11 = ld(p0, a0, a1, i + 1, j + 1);
    const TA b00 = ld(p1, b0, b1, i, j), b01 = ld(p1, b0, b1, i, j + 1);
    const TA b10 = ld(p1, b0, b1, i + 1, j), b11 = ld(p1, b0, b1, i + 1, j + 1);
    // the same grouping as the fused kernel: temporal sums S and differences D first
    const TA s00 = a00 + b00, s01 = a01 + b01, s10 = a10 + b10, s11 = a11 + b11;
    const TA d00 = b00 - a00, d01 = b01 - a01, d10 = b10 - a10, d11 = b11 - a11;
    const TA nx = (s01 - s00) + (s11 - s10);
    const TA ny = (s10 + s11) - (s00 + s01);
    const TA nt = (d00 + d01) + (d10 + d11);
    if constexpr (std::is_same<TO, int>::value) {
      ex[(int64_t)i * x0 + (int64_t)j * x1] = nx;
      ey[(int64_t)i * y0 + (int64_t)j * y1] = ny;
      et[(int64_t)i * t0 + (int64_t)j * t1] = nt;
    } else {
      ex[(int64_t)i * x0 + (int64_t)j * x1] = nx * 0.25f;
      ey[(int64_t)i * y0 + (int64_t)j * y1] = ny * 0.25f;
      et[(int64_t)i * t0 + (int64_t)j * t1] = nt * 0.25f;
    }
  }
}

// Gradient of one image with a 2x2 or 3x3 mask (the mask's integer weights
// summed first, then one scale), its magnitude sqrt(ex^2 + ey^2) and its
// four-quadrant direction atan2(ey, ex).  p(r, c) is the pixel at row r,
// column c of the mask's window.
//   ST 0 fd2      (1/2)[[-1, 1], [-1, 1]] and its transpose
//   ST 1 roberts  diagonal differences (x: (i+1,j+1) - (i,j); y: (i+1,j) - (i,j+1)) / sqrt(2)
//   ST 2 prewitt3 rows [-1, 0, 1] / 6 and the transpose
//   ST 3 sobel3   rows [-1, 0, 1] weighted 1, 2, 1, / 8, and the transpose
template <int ST, typename P>
__device__ __forceinline__ void grad_px(P p, float& gx, float& gy) {
  if constexpr (ST == 0) {
    gx = ((p(0, 1) - p(0, 0)) + (p(1, 1) - p(1, 0))) * 0.5f;
    gy = ((p(1, 0) - p(0, 0)) + (p(1, 1) - p(0, 1))) * 0.5f;
  } else if constexpr (ST == 1) {
    constexpr float r = 0.70710678118654752f;
    gx = (p(1, 1) - p(0, 0)) * r;
    gy = (p(1, 0) - p(0, 1)) * r;
  } else {
    constexpr float w1 = ST == 2 ? 1.f : 2.f;
    constexpr float sc = ST == 2 ? 1.f / 6.f : 0.125f;
    gx = ((p(0, 2) - p(0, 0)) + w1 * (p(1, 2) - p(1, 0)) + (p(2, 2) - p(2, 0))) * sc;
    gy = ((p(2, 0) - p(0, 0)) + w1 * (p(2, 1) - p(0, 1)) + (p(2, 2) - p(0, 2))) * sc;
  }
}

// Any strides: one thread per output pixel; an output whose pointer is null is
// not written.
template <typename T, int ST>
__global__ __launch_bounds__(256) void gradient_kernel(const T* __restrict__ src, int64_t s0, int64_t s1, int Ho,
                                                        int Wo, float* __restrict__ ex, int64_t e0, int64_t e1,
                                                        float* __restrict__ ey, int64_t f0, int64_t f1,
                                                        float* __restrict__ mag, int64_t m0, int64_t m1,
                                                        float* __restrict__ dir, int64_t g0, int64_t g1) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Wo) return;
  for (int i = blockIdx.y; i < Ho; i += gridDim.y) {
    float gx, gy;
    grad_px<ST>(
        [&](int r, int c) -> float { return to_f32<T>(src[(int64_t)(i + r) * s0 + (int64_t)(j + c) * s1]); }, gx,
        gy);
    if (ex) ex[(int64_t)i * e0 + (int64_t)j * e1] = gx;
    if (ey) ey[(int64_t)i * f0 + (int64_t)j * f1] = gy;
    if (mag) mag[(int64_t)i * m0 + (int64_t)j * m1] = sqrtf(gx * gx + gy * gy);
    if (dir) dir[(int64_t)i * g0 + (int64_t)j * g1] = atan2f(gy, gx);
  }
}

// Input rows of unit stride whose starts are aligned to four elements, outputs
// of unit stride (any row stride): each thread produces 4 adjacent outputs on
// each of GR consecutive output rows.  It reads every input row of its window
// once, as one aligned load of 4 elements and one of 2 (the K + 3 <= 6
// columns it needs), keeps the last K rows in registers, and writes each
// output row in float4 chunks aligned to that row's own 16-byte boundaries.
// Columns near the right edge fall back to guarded element loads and stores.
template <typename T> struct Vec4;
template <> struct Vec4<uint8_t> { typedef uint32_t lo; typedef uint16_t hi; };
template <> struct Vec4<_Float16> {
  typedef _Float16 lo __attribute__((ext_vector_type(4)));
  typedef _Float16 hi __attribute__((ext_vector_type(2)));
};
template <> struct Vec4<float> {
  typedef float lo __attribute__((ext_vector_type(4)));
  typedef float hi __attribute__((ext_vector_type(2)));
};

template <typename T>
__device__ __forceinline__ void load6(const T* p, float* v) {
  const typename Vec4<T>::lo a = *as_global(reinterpret_cast<const typename Vec4<T>::lo*>(p));
  const typename Vec4<T>::hi b = *as_global(reinterpret_cast<const typename Vec4<T>::hi*>(p + 4));
  if constexpr (std::is_same<T, uint8_t>::value) {
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = (float)((a >> (8 * c)) & 0xffu);
    v[4] = (float)(b & 0xffu);
    v[5] = (float)(b >> 8);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = (float)a[c];
    v[4] = (float)b[0];
    v[5] = (float)b[1];
  }
}

// Value of lane i + 1 (DPP wave_shl:1); lane 63 receives 0.
__device__ __forceinline__ float lane_next(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}

// Value of lane l (uniform).
__device__ __forceinline__ float lane_read(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Columns j .. j+3 of a row whose column j is 16-byte aligned: one float4
// store when all four lie before the row end n, else element stores.
__device__ __forceinline__ void store4(float* row, int j, int n, float a, float b, float c, float d) {
  if (j + 4 <= n) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    *as_global(reinterpret_cast<f4*>(row + j)) = f4{a, b, c, d};
  } else {
    const float v[4] = {a, b, c, d};
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (j + e < n) row[j + e] = v[e];
  }
}

template <typename T, int ST, int GR>
__global__ __launch_bounds__(256) void gradient_vec(const T* __restrict__ src, int64_t s0, int H, int W, int Ho,
                                                     int Wo, GradOut o) {
  constexpr int K = ST >= 2 ? 3 : 2;
  const int j0 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (j0 >= Wo) return;
  const bool vec_in = j0 + 6 <= W;   // both aligned loads inside the row
  const int lane = threadIdx.x & 63;
  const int wave_col = j0 - 4 * lane;  // first column of this wave's span
  const bool full_wave = wave_col + 256 <= Wo;
  for (int i0 = (int)blockIdx.y * GR; i0 < Ho; i0 += (int)gridDim.y * GR) {
    // every input row first: the output pointers may alias the input as far as
    // the compiler knows, so loads placed after a store would wait for it
    float win[GR + K - 1][6];
#pragma unroll
    for (int r = 0; r < GR + K - 1; ++r) {
      const int ir = i0 + r;
      float* v = win[r];
      if (ir < H) {
        const T* p = src + (int64_t)ir * s0 + j0;
        if (vec_in) {
          load6<T>(p, v);
        } else {
#pragma unroll
          for (int c = 0; c < 6; ++c) v[c] = j0 + c < W ? to_f32<T>(p[c]) : 0.f;
        }
      }
    }
#pragma unroll
    for (int r = K - 1; r < GR + K - 1; ++r) {
      const int oi = i0 + r - (K - 1);
      if (oi >= Ho) break;
      float gx[4], gy[4], gm[4], gd[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        grad_px<ST>([&](int a, int b) -> float { return win[r - (K - 1) + a][c + b]; }, gx[c], gy[c]);
        if (o.mag) gm[c] = sqrtf(gx[c] * gx[c] + gy[c] * gy[c]);
        if (o.dir) gd[c] = atan2f(gy[c], gx[c]);
      }
      auto put = [&](float* base, int64_t rs, const float* val) {
        if (!base) return;
        float* row = base + (int64_t)oi * rs;
        // first column of the row (and of every 256-column wave span) whose
        // address is 16-byte aligned
        const int sh = (4 - (int)((reinterpret_cast<uintptr_t>(row) >> 2) & 3)) & 3;
        if (sh == 0) {
          store4(row, j0, Wo, val[0], val[1], val[2], val[3]);
          return;
        }
        if (!full_wave) {  // the last wave of a row: element stores
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (j0 + c < Wo) row[j0 + c] = val[c];
          return;
        }
        // lanes 0..62 write the aligned chunk at j0 + sh: their values sh..3 and
        // the first sh values of the next lane.  The sh columns before lane 0's
        // chunk and lane 63's values sh..3 go out in one store by lanes 0..sh-1
        // and 60+sh..63, which take them from lane 0 and lane 63.
        const float n0 = lane_next(val[0]), n1 = lane_next(val[1]), n2 = lane_next(val[2]);
        const float h0 = lane_read(val[0], 0), h1 = lane_read(val[1], 0), h2 = lane_read(val[2], 0);
        const float t1 = lane_read(val[1], 63), t2 = lane_read(val[2], 63), t3 = lane_read(val[3], 63);
        if (lane != 63) {
          if (sh == 1) store4(row, j0 + 1, Wo, val[1], val[2], val[3], n0);
          else if (sh == 2) store4(row, j0 + 2, Wo, val[2], val[3], n0, n1);
          else store4(row, j0 + 3, Wo, val[3], n0, n1, n2);
        }
        if (lane < sh || lane >= 60 + sh) {
          const float v = lane == 0 ? h0 : lane == 1 ? h1 : lane == 2 ? h2 : lane == 61 ? t1 : lane == 62 ? t2 : t3;
          row[lane < sh ? wave_col + lane : wave_col + 192 + lane] = v;
        }
      };
      put(o.ex, o.ex0, gx);
      put(o.ey, o.ey0, gy);
      put(o.mag, o.mag0, gm);
      put(o.dir, o.dir0, gd);
    }
  }
}

}  // namespace

// True when tc_gradient's arguments allow the vector kernel.
static bool gradient_vec_ok(const Image2D& src, const GradOut& o) {
  const int es = src.dt == TC_U8 ? 1 : src.dt == TC_F16 ? 2 : 4;
  if (src.s1 != 1 || src.s0 % 4 != 0 || reinterpret_cast<uintptr_t>(src.p) % (4 * es) != 0) return false;
  const float* outs[4] = {o.ex, o.ey, o.mag, o.dir};
  const int64_t r1[4] = {o.ex1, o.ey1, o.mag1, o.dir1};
  for (int q = 0; q < 4; ++q)
    if (outs[q] && (r1[q] != 1 || reinterpret_cast<uintptr_t>(outs[q]) % 4 != 0)) return false;
  return true;
}

namespace {

constexpr int kGradRows = 4;

template <typename T, int ST>
hipError_t gradient_ts(const Image2D& src, int Ho, int Wo, const GradOut& o, hipStream_t st) {
  constexpr int K = ST >= 2 ? 3 : 2;
  if (gradient_vec_ok(src, o)) {
    const int64_t tx = (Wo + 3) / 4;
    const dim3 block(256), grid((unsigned)((tx + 255) / 256), grid_rows((Ho + kGradRows - 1) / kGradRows));
    hipLaunchKernelGGL((gradient_vec<T, ST, kGradRows>), grid, block, 0, st, static_cast<const T*>(src.p), src.s0,
                       Ho + K - 1, Wo + K - 1, Ho, Wo, o);
    return hipGetLastError();
  }
  const dim3 block(256), grid((unsigned)((Wo + 255) / 256), grid_rows(Ho));
  hipLaunchKernelGGL((gradient_kernel<T, ST>), grid, block, 0, st, static_cast<const T*>(src.p), src.s0, src.s1, Ho,
                     Wo, o.ex, o.ex0, o.ex1, o.ey, o.ey0, o.ey1, o.mag, o.mag0, o.mag1, o.dir, o.dir0, o.dir1);
  return hipGetLastError();
}

template <typename T>
hipError_t gradient_t(const Image2D& src, int stencil, int Ho, int Wo, const GradOut& o, hipStream_t st) {
  switch (stencil) {
    case TC_STENCIL_FD2: return gradient_ts<T, 0>(src, Ho, Wo, o, st);
    case TC_STENCIL_ROBERTS: return gradient_ts<T, 1>(src, Ho, Wo, o, st);
    case TC_STENCIL_PREWITT3: return gradient_ts<T, 2>(src, Ho, Wo, o, st);
    case TC_STENCIL_SOBEL3: return gradient_ts<T, 3>(src, Ho, Wo, o, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t pyr_t(const Image2D& s, float* dst, int64_t d0, int64_t d1, int Ho, int Wo, hipStream_t st) {
  const dim3 grid((unsigned)((Wo + 255) / 256), grid_rows(Ho));
  hipLaunchKernelGGL(pyramid_level<T>, grid, dim3(256), 0, st, reinterpret_cast<const T*>(s.p), s.s0, s.s1, dst, d0,
                     d1, Ho, Wo);
  return hipGetLastError();
}

template <typename T, typename TO>
hipError_t horn_t(const Image2D& a, const Image2D& b, int H, int W, void* ex, void* ey, void* et, const int64_t* os0,
                  const int64_t* os1, hipStream_t st) {
  const dim3 grid((unsigned)((W - 1 + 255) / 256), grid_rows(H - 1));
  hipLaunchKernelGGL((horn_cube<T, TO>), grid, dim3(256), 0, st, reinterpret_cast<const T*>(a.p), a.s0, a.s1,
                     reinterpret_cast<const T*>(b.p), b.s0, b.s1, H, W, reinterpret_cast<TO*>(ex), os0[0], os1[0],
                     reinterpret_cast<TO*>(ey), os0[1], os1[1], reinterpret_cast<TO*>(et), os0[2], os1[2]);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pyramid_level(const Image2D& src, float* dst, int64_t d0, int64_t d1, int Ho, int Wo,
                                hipStream_t s) {
  if (Ho <= 0 || Wo <= 0) return hipSuccess;
  switch (src.dt) {
    case TC_U8: return pyr_t<uint8_t>(src, dst, d0, d1, Ho, Wo, s);
    case TC_F16: return pyr_t<_Float16>(src, dst, d0, d1, Ho, Wo, s);
    case TC_F32: return pyr_t<float>(src, dst, d0, d1, Ho, Wo, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_horn(const Image2D& prev, const Image2D& next, int H, int W, void* ex, void* ey, void* et, int odt,
                       const int64_t* os0, const int64_t* os1, hipStream_t s) {
  if (H < 2 || W < 2) return hipSuccess;
  if (odt == TC_I32) {
    if (prev.dt != TC_U8) return hipErrorInvalidValue;
    return horn_t<uint8_t, int>(prev, next, H, W, ex, ey, et, os0, os1, s);
  }
  switch (prev.dt) {
    case TC_U8: return horn_t<uint8_t, float>(prev, next, H, W, ex, ey, et, os0, os1, s);
    case TC_F16: return horn_t<_Float16, float>(prev, next, H, W, ex, ey, et, os0, os1, s);
    case TC_F32: return horn_t<float, float>(prev, next, H, W, ex, ey, et, os0, os1, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gradient(const Image2D& src, int stencil, int Ho, int Wo, const GradOut& o, hipStream_t s) {
  if (Ho <= 0 || Wo <= 0) return hipSuccess;
  switch (src.dt) {
    case TC_U8: return gradient_t<uint8_t>(src, stencil, Ho, Wo, o, s);
    case TC_F16: return gradient_t<_Float16>(src, stencil, Ho, Wo, o, s);
    case TC_F32: return gradient_t<float>(src, stencil, Ho, Wo, o, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ttc
