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

template <typename T>
__global__ __launch_bounds__(256) void pyramid_level(const T* __restrict__ src, int64_t s0, int64_t s1,
                                                      float* __restrict__ dst, int64_t d0, int64_t d1, int Ho,
                                                      int Wo) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= Wo) return;
  const T* r0 = src + (int64_t)(2 * i) * s0 + (int64_t)(2 * j) * s1;
  const T* r1 = r0 + s0;
  const float a = to_f32<T>(r0[0]), b = to_f32<T>(r0[s1]);
  const float c = to_f32<T>(r1[0]), d = to_f32<T>(r1[s1]);
  dst[(int64_t)i * d0 + (int64_t)j * d1] = ((a + b) + (c + d)) * 0.25f;
}

template <typename T, typename TO>
__global__ __launch_bounds__(256) void horn_cube(const T* __restrict__ p0, int64_t a0, int64_t a1,
                                                  const T* __restrict__ p1, int64_t b0, int64_t b1, int H, int W,
                                                  TO* __restrict__ ex, int64_t x0, int64_t x1, TO* __restrict__ ey,
                                                  int64_t y0, int64_t y1, TO* __restrict__ et, int64_t t0,
                                                  int64_t t1) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= W - 1) return;
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

// Gradient of one image with a 2x2 or 3x3 mask (the mask's integer weights
// summed first, then one scale), its magnitude sqrt(ex^2 + ey^2) and its
// four-quadrant direction atan2(ey, ex).  One thread per output pixel; an
// output whose pointer is null is not written.
//   ST 0 fd2      (1/2)[[-1, 1], [-1, 1]] and its transpose
//   ST 1 roberts  diagonal differences (x: (i+1,j+1) - (i,j); y: (i+1,j) - (i,j+1)) / sqrt(2)
//   ST 2 prewitt3 rows [-1, 0, 1] / 6 and the transpose
//   ST 3 sobel3   rows [-1, 0, 1] weighted 1, 2, 1, / 8, and the transpose
template <typename T, int ST>
__global__ __launch_bounds__(256) void gradient_kernel(const T* __restrict__ src, int64_t s0, int64_t s1, int Ho,
                                                        int Wo, float* __restrict__ ex, int64_t e0, int64_t e1,
                                                        float* __restrict__ ey, int64_t f0, int64_t f1,
                                                        float* __restrict__ mag, int64_t m0, int64_t m1,
                                                        float* __restrict__ dir, int64_t g0, int64_t g1) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= Wo) return;
  auto p = [&](int r, int c) -> float { return to_f32<T>(src[(int64_t)(i + r) * s0 + (int64_t)(j + c) * s1]); };
  float gx, gy;
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
  if (ex) ex[(int64_t)i * e0 + (int64_t)j * e1] = gx;
  if (ey) ey[(int64_t)i * f0 + (int64_t)j * f1] = gy;
  if (mag) mag[(int64_t)i * m0 + (int64_t)j * m1] = sqrtf(gx * gx + gy * gy);
  if (dir) dir[(int64_t)i * g0 + (int64_t)j * g1] = atan2f(gy, gx);
}

template <typename T, int ST>
hipError_t gradient_ts(const Image2D& src, int Ho, int Wo, const GradOut& o, hipStream_t st) {
  const dim3 block(256), grid((unsigned)((Wo + 255) / 256), (unsigned)Ho);
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
  const dim3 grid((unsigned)((Wo + 255) / 256), (unsigned)Ho);
  hipLaunchKernelGGL(pyramid_level<T>, grid, dim3(256), 0, st, reinterpret_cast<const T*>(s.p), s.s0, s.s1, dst, d0,
                     d1, Ho, Wo);
  return hipGetLastError();
}

template <typename T, typename TO>
hipError_t horn_t(const Image2D& a, const Image2D& b, int H, int W, void* ex, void* ey, void* et, const int64_t* os0,
                  const int64_t* os1, hipStream_t st) {
  const dim3 grid((unsigned)((W - 1 + 255) / 256), (unsigned)(H - 1));
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
