// Time to contact of one frame pair through materialised levels, with a choice
// of derivative stencil and of the pyramid low-pass filter (the decomposed
// path used to compare the paper's variants; the fused pass serves the
// 2x2x2 cube without a low-pass filter).
//
// pyramid_pair:  the 2x2 block mean of both frames of the pair, one launch.
// lowpass3:      P <- [1, 2, 1]/4 along rows and columns, borders clamped
//                (Time to Contact, Results: a low-pass filter after the block
//                mean; the filter itself is a reading, binomial); both frames
//                in one launch.
// stencil_sums:  one level's ten sums of the normal equations (all levels in
//                one launch, stencil_sums_levels).  Per position
//                the derivatives are formed in FP32 from the two frames, then
//                G, the products and every sum are FP64; each block writes its
//                partial sums (fixed order, deterministic).
//   ST 0 cube      the 2x2x2 first-difference cube between pixels (i, j) and
//                  (i+1, j+1), centred at x = 2^l (j + 1) - W0/2
//   ST 2 prewitt3  E_x = (M_x * P0 + M_x * P1)/2, M_x = [1,1,1]^T/3 (x) [-1,0,1]/2,
//   ST 3 sobel3    M_x = [1,2,1]^T/4 (x) [-1,0,1]/2; E_y with the transposes;
//                  E_t = (s s^T) * (P1 - P0); centred at pixel (i, j),
//                  x = 2^l (j + 1/2) - W0/2, 1 <= i <= H_l - 2, 1 <= j <= W_l - 2
//                (Convolutions section: the centred 3x3 masks)
//   Spatial derivatives are per base pixel (divided by 2^l).
// variant_finish: per level (one wave each) the block partials in a fixed
//                order (FP64), the 3x3 solve, and the multi-scale choice by the
//                decreasing-TTC rule.
#include <math.h>

#include "device_common.hpp"
#include "internal.hpp"
#include "solve.hpp"

namespace ttc {
namespace {

constexpr int kSumThreads = 256;

// blockIdx.z: the frame (src[z] -> dst[z]).
__global__ __launch_bounds__(256) void lowpass3(VariantPair2 io, int H, int W) {
  const float* __restrict__ src = io.src[blockIdx.z];
  float* __restrict__ dst = io.dst[blockIdx.z];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= W) return;
  const int jm = j > 0 ? j - 1 : 0, jp = j + 1 < W ? j + 1 : W - 1;
  const float wr[3] = {0.25f, 0.5f, 0.25f};
  for (int i = blockIdx.y; i < H; i += gridDim.y) {
    float acc = 0.f;
#pragma unroll
    for (int a = -1; a <= 1; ++a) {
      const int r = min(max(i + a, 0), H - 1);
      const float* row = src + (int64_t)r * W;
      const float h = 0.25f * row[jm] + 0.5f * row[j] + 0.25f * row[jp];
      acc += wr[a + 1] * h;
    }
    dst[(int64_t)i * W + j] = acc;
  }
}

// The 2x2 block mean of both frames of the pair in one launch (blockIdx.z:
// the frame): P_{l+1}[i][j] = ((P[2i][2j] + P[2i][2j+1]) + (P[2i+1][2j] +
// P[2i+1][2j+1])) / 4, the same order as the pyramid kernel.
template <typename T>
__global__ __launch_bounds__(256) void pyramid_pair(VariantPlanes2 src, VariantPair2 io, int Ho, int Wo) {
  const T* __restrict__ sp = static_cast<const T*>(src.p[blockIdx.z]);
  const int64_t s0 = src.s0[blockIdx.z], s1 = src.s1[blockIdx.z];
  float* __restrict__ dst = io.dst[blockIdx.z];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Wo) return;
  for (int i = blockIdx.y; i < Ho; i += gridDim.y) {
    const T* r0 = sp + (int64_t)(2 * i) * s0 + (int64_t)(2 * j) * s1;
    const T* r1 = r0 + s0;
    const float a = to_f32<T>(r0[0]), b = to_f32<T>(r0[s1]);
    const float c = to_f32<T>(r1[0]), d = to_f32<T>(r1[s1]);
    dst[(int64_t)i * Wo + j] = ((a + b) + (c + d)) * 0.25f;
  }
}

struct Plane {
  const void* p;
  int64_t s0, s1;
};

template <typename T>
__device__ __forceinline__ float px(const Plane& q, int r, int c) {
  return to_f32<T>(static_cast<const T*>(q.p)[(int64_t)r * q.s0 + (int64_t)c * q.s1]);
}

// Sum of doubles over the 64 lanes of a wave (butterfly, every lane gets it).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// The sums of work-group blockIdx.x of `nblocks` (positions strided by nblocks
// work-groups).
template <typename T, int ST>
__device__ __forceinline__ void stencil_sums(Plane a, Plane b, int Hl, int Wl, int level, int H0, int W0,
                                             int nblocks, double* __restrict__ part) {
  constexpr int K = ST == 0 ? 2 : 3;
  constexpr int B0 = ST == 0 ? 0 : 1;  // first position row / column
  const int nr = Hl - K + 1, nc = Wl - K + 1;
  const int64_t n = (int64_t)nr * nc;
  const double sl = ldexp(1.0, level);
  const double cx = ST == 0 ? 1.0 : 0.5;  // position of pixel j's estimate: 2^l (j + cx) - W0/2
  double acc[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) acc[q] = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * kSumThreads + threadIdx.x; p < n; p += (int64_t)nblocks * kSumThreads) {
    const int i = B0 + (int)(p / nc), j = B0 + (int)(p % nc);
    float fx, fy, ft;
    if constexpr (ST == 0) {
      const float a00 = px<T>(a, i, j), a01 = px<T>(a, i, j + 1), a10 = px<T>(a, i + 1, j), a11 = px<T>(a, i + 1, j + 1);
      const float b00 = px<T>(b, i, j), b01 = px<T>(b, i, j + 1), b10 = px<T>(b, i + 1, j), b11 = px<T>(b, i + 1, j + 1);
      const float s00 = a00 + b00, s01 = a01 + b01, s10 = a10 + b10, s11 = a11 + b11;
      fx = ((s01 - s00) + (s11 - s10)) * 0.25f;
      fy = ((s10 + s11) - (s00 + s01)) * 0.25f;
      ft = ((b00 - a00) + (b01 - a01) + ((b10 - a10) + (b11 - a11))) * 0.25f;
    } else {
      constexpr float w1 = ST == 2 ? 1.f : 2.f;        // centre weight of the smoothing
      constexpr float sd = ST == 2 ? 1.f / 12.f : 1.f / 16.f;  // (1/2 frames)(1/2 difference)(1/sum w)
      constexpr float st = ST == 2 ? 1.f / 9.f : 1.f / 16.f;   // 1/(sum w)^2
      float S[3][3], D[3][3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float u = px<T>(a, i - 1 + r, j - 1 + c), v = px<T>(b, i - 1 + r, j - 1 + c);
          S[r][c] = u + v;
          D[r][c] = v - u;
        }
      fx = ((S[0][2] - S[0][0]) + w1 * (S[1][2] - S[1][0]) + (S[2][2] - S[2][0])) * sd;
      fy = ((S[2][0] - S[0][0]) + w1 * (S[2][1] - S[0][1]) + (S[2][2] - S[0][2])) * sd;
      const float r0 = D[0][0] + w1 * D[0][1] + D[0][2];
      const float r1 = D[1][0] + w1 * D[1][1] + D[1][2];
      const float r2 = D[2][0] + w1 * D[2][1] + D[2][2];
      ft = (r0 + w1 * r1 + r2) * st;
    }
    const double ex = (double)fx / sl, ey = (double)fy / sl, et = (double)ft;
    const double x = sl * (j + cx) - 0.5 * W0, y = sl * (i + cx) - 0.5 * H0;
    const double g = x * ex + y * ey;
    acc[0] += ex * ex;
    acc[1] += ex * ey;
    acc[2] += ey * ey;
    acc[3] += g * ex;
    acc[4] += g * ey;
    acc[5] += g * g;
    acc[6] += ex * et;
    acc[7] += ey * et;
    acc[8] += g * et;
    acc[9] += et * et;
  }
  __shared__ double red[kSumThreads / 64][10];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 10; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) red[wave][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < 10) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kSumThreads / 64; ++w) s += red[w][threadIdx.x];
    part[(int64_t)blockIdx.x * 10 + threadIdx.x] = s;
  }
}

// Every level's sums in one launch: blockIdx.y is the level (its planes are
// the frames themselves at level 0, FP32 level images above), and a level
// runs on its own first `blocks` work-groups, as separate launches would.
template <typename T, int ST>
__global__ __launch_bounds__(kSumThreads) void stencil_sums_levels(VariantSumLevels ls, int H0, int W0,
                                                                    double* __restrict__ part) {
  const int l = blockIdx.y;
  if ((int)blockIdx.x >= ls.blocks[l]) return;  // uniform
  const Plane a{ls.a[l], ls.s0[0][l], ls.s1[0][l]}, b{ls.b[l], ls.s0[1][l], ls.s1[1][l]};
  double* pl = part + ls.part_off[l] * 10;
  if (l == 0)
    stencil_sums<T, ST>(a, b, ls.Hl[l], ls.Wl[l], l, H0, W0, ls.blocks[l], pl);
  else
    stencil_sums<float, ST>(a, b, ls.Hl[l], ls.Wl[l], l, H0, W0, ls.blocks[l], pl);
}

__global__ __launch_bounds__(64 * TC_MAX_LEVELS) void variant_finish(const double* __restrict__ part, VariantLevels lv,
                                                                     tc_ttc_level* __restrict__ out,
                                                                     tc_ttc_pick* __restrict__ pick) {
  __shared__ tc_ttc_level res[TC_MAX_LEVELS];
  const int l = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (l < lv.levels) {
    // wave l: each lane adds every 64th block's partials, then a fixed butterfly
    double s[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) s[q] = 0.0;
    const double* p = part + lv.part_off[l] * 10;
    for (int bk = lane; bk < lv.blocks[l]; bk += 64)
#pragma unroll
      for (int q = 0; q < 10; ++q) s[q] += p[(int64_t)bk * 10 + q];
#pragma unroll
    for (int q = 0; q < 10; ++q) s[q] = wave_sum(s[q]);
    if (lane == 0) {
      tc_ttc_level r;
      solve_level(s, r);
      r.n = lv.n[l];
      r.level = l;
      res[l] = r;
      out[l] = r;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int k = 0;
    while (k + 1 < lv.levels && level_key(res[k + 1]) < level_key(res[k])) ++k;
    tc_ttc_pick pk;
    pk.ttc = res[k].ttc;
    pk.x0 = res[k].x0;
    pk.y0 = res[k].y0;
    pk.A = res[k].A;
    pk.B = res[k].B;
    pk.C = res[k].C;
    pk.level = k;
    pk.status = res[k].status;
    *pick = pk;
  }
}

template <typename T>
hipError_t sums_t(int stencil, const VariantSumLevels& ls, int levels, int H0, int W0, double* part, hipStream_t s) {
  int bmax = 1;
  for (int l = 0; l < levels; ++l) bmax = ls.blocks[l] > bmax ? ls.blocks[l] : bmax;
  const dim3 grid((unsigned)bmax, (unsigned)levels), block(kSumThreads);
  switch (stencil) {
    case TC_STENCIL_FD2:
      hipLaunchKernelGGL((stencil_sums_levels<T, 0>), grid, block, 0, s, ls, H0, W0, part);
      break;
    case TC_STENCIL_PREWITT3:
      hipLaunchKernelGGL((stencil_sums_levels<T, 2>), grid, block, 0, s, ls, H0, W0, part);
      break;
    case TC_STENCIL_SOBEL3:
      hipLaunchKernelGGL((stencil_sums_levels<T, 3>), grid, block, 0, s, ls, H0, W0, part);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t pyr_pair_t(const VariantPlanes2& src, const VariantPair2& io, int Ho, int Wo, hipStream_t s) {
  const unsigned gy = (unsigned)(Ho < 65535 ? Ho : 65535);
  hipLaunchKernelGGL(pyramid_pair<T>, dim3((unsigned)((Wo + 255) / 256), gy, 2), dim3(256), 0, s, src, io, Ho, Wo);
  return hipGetLastError();
}

}  // namespace

int variant_sum_blocks(int64_t positions) {
  const int64_t b = (positions + 2 * kSumThreads - 1) / (2 * kSumThreads);
  return (int)(b < 1 ? 1 : b > 2048 ? 2048 : b);
}

hipError_t launch_pyramid_pair(const VariantPlanes2& src, int dt, const VariantPair2& io, int Ho, int Wo,
                               hipStream_t s) {
  if (Ho <= 0 || Wo <= 0) return hipSuccess;
  switch (dt) {
    case TC_U8: return pyr_pair_t<uint8_t>(src, io, Ho, Wo, s);
    case TC_F16: return pyr_pair_t<_Float16>(src, io, Ho, Wo, s);
    case TC_F32: return pyr_pair_t<float>(src, io, Ho, Wo, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_lowpass3_pair(const VariantPair2& io, int H, int W, hipStream_t s) {
  if (H <= 0 || W <= 0) return hipSuccess;
  const unsigned gy = (unsigned)(H < 65535 ? H : 65535);
  hipLaunchKernelGGL(lowpass3, dim3((unsigned)((W + 255) / 256), gy, 2), dim3(256), 0, s, io, H, W);
  return hipGetLastError();
}

hipError_t launch_stencil_sums_levels(int stencil, int dt, const VariantSumLevels& ls, int levels, int H0, int W0,
                                      double* part, hipStream_t s) {
  switch (dt) {
    case TC_U8: return sums_t<uint8_t>(stencil, ls, levels, H0, W0, part, s);
    case TC_F16: return sums_t<_Float16>(stencil, ls, levels, H0, W0, part, s);
    case TC_F32: return sums_t<float>(stencil, ls, levels, H0, W0, part, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_variant_finish(const double* part, const VariantLevels& lv, tc_ttc_level* out, tc_ttc_pick* pick,
                                 hipStream_t s) {
  hipLaunchKernelGGL(variant_finish, dim3(1), dim3(64 * TC_MAX_LEVELS), 0, s, part, lv, out, pick);
  return hipGetLastError();
}

}  // namespace ttc
