// FFT branch of 2-D convolution (Convolutions section: the convolution theorem,
// y = F^-1(F(x) F(k)); Accelerating Convolutions: the hybrid that switches to
// it for large kernels).
//
// fft_twiddles: w[k] = exp(-2 pi i k / N), k < N/2, with sincospi (exact
//               argument k/N for N a power of two).
// fft_rows:     radix-2 Stockham transform of length N = 2^m <= 4096 along each
//               row, one work-group per row, the row held in LDS; stage s
//               (sub-transform length L = 2^(s+1)) maps a = v[j], b = v[j + N/2]
//               to v'[(j >> s) L + k] = a + w b and v'[(j >> s) L + k + L/2] =
//               a - w b, k = j mod L/2, w = exp(-+2 pi i k / L).  The inverse
//               uses conjugate twiddles and no scale.
// transpose_c:  complex R x C -> C x R through 32 x 33 LDS tiles.
// pad_real, mul_c, extract_real: the zero-padded complex images, the
//               pointwise product, and the real part scaled by 1/(P Q) and cut
//               to the requested mode.
#include <math.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace ttc {
namespace {

constexpr int kFftThreads = 256;
constexpr int kFftPerThread = kFftMaxN / 2 / kFftThreads;  // butterflies per thread per stage (max)

__global__ __launch_bounds__(256) void fft_twiddles(float2* __restrict__ tw, int N) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N / 2) return;
  float s, c;
  sincospif(-2.0f * (float)k / (float)N, &s, &c);
  tw[k] = make_float2(c, s);
}

template <bool INV>
__global__ __launch_bounds__(kFftThreads) void fft_rows(float2* __restrict__ data, int64_t row_stride, int N, int m,
                                                        const float2* __restrict__ tw) {
  __shared__ float2 buf[kFftMaxN];
  float2* row = data + (int64_t)blockIdx.x * row_stride;
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += kFftThreads) buf[i] = row[i];
  __syncthreads();
  const int half = N >> 1;
  for (int s = 0; s < m; ++s) {
    const int Ls = 1 << s;
    float2 o0[kFftPerThread], o1[kFftPerThread];
#pragma unroll
    for (int c = 0; c < kFftPerThread; ++c) {
      const int j = tid + c * kFftThreads;
      if (j < half) {
        const int k = j & (Ls - 1);
        const float2 a = buf[j], b = buf[j + half];
        float2 w = tw[k << (m - 1 - s)];
        if (INV) w.y = -w.y;
        const float2 wb = make_float2(w.x * b.x - w.y * b.y, w.x * b.y + w.y * b.x);
        o0[c] = make_float2(a.x + wb.x, a.y + wb.y);
        o1[c] = make_float2(a.x - wb.x, a.y - wb.y);
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kFftPerThread; ++c) {
      const int j = tid + c * kFftThreads;
      if (j < half) {
        const int k = j & (Ls - 1);
        const int base = ((j >> s) << (s + 1)) + k;
        buf[base] = o0[c];
        buf[base + Ls] = o1[c];
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < N; i += kFftThreads) row[i] = buf[i];
}

// dst[c][r] = src[r][c] for an R x C source.
__global__ __launch_bounds__(256) void transpose_c(const float2* __restrict__ src, int R, int C,
                                                   float2* __restrict__ dst) {
  __shared__ float2 tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
#pragma unroll
  for (int i = 0; i < 32; i += 8) {
    const int r = r0 + ty + i, c = c0 + tx;
    if (r < R && c < C) tile[ty + i][tx] = src[(int64_t)r * C + c];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 32; i += 8) {
    const int c = c0 + ty + i, r = r0 + tx;
    if (c < C && r < R) dst[(int64_t)c * R + r] = tile[tx][ty + i];
  }
}

__global__ __launch_bounds__(256) void pad_real(const float* __restrict__ x, int64_t s0, int64_t s1, int H, int W,
                                                float2* __restrict__ dst, int Q) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= Q) return;
  const float v = (i < H && j < W) ? x[(int64_t)i * s0 + (int64_t)j * s1] : 0.f;
  dst[(int64_t)i * Q + j] = make_float2(v, 0.f);
}

__global__ __launch_bounds__(256) void mul_c(float2* __restrict__ a, const float2* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float2 u = a[i], v = b[i];
  a[i] = make_float2(u.x * v.x - u.y * v.y, u.x * v.y + u.y * v.x);
}

__global__ __launch_bounds__(256) void extract_real(const float2* __restrict__ src, int Q, int o0, int o1, int OH,
                                                    int OW, float scale, float* __restrict__ y, int64_t y0,
                                                    int64_t y1) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= OW) return;
  y[(int64_t)i * y0 + (int64_t)j * y1] = src[(int64_t)(i + o0) * Q + (j + o1)].x * scale;
}

int ilog2(int n) {
  int m = 0;
  while ((1 << m) < n) ++m;
  return m;
}

hipError_t rows(float2* d, int n_rows, int N, const float2* tw, bool inv, hipStream_t s) {
  if (inv)
    hipLaunchKernelGGL(fft_rows<true>, dim3((unsigned)n_rows), dim3(kFftThreads), 0, s, d, (int64_t)N, N, ilog2(N),
                       tw);
  else
    hipLaunchKernelGGL(fft_rows<false>, dim3((unsigned)n_rows), dim3(kFftThreads), 0, s, d, (int64_t)N, N, ilog2(N),
                       tw);
  return hipGetLastError();
}

hipError_t transpose(const float2* src, int R, int C, float2* dst, hipStream_t s) {
  hipLaunchKernelGGL(transpose_c, dim3((unsigned)((C + 31) / 32), (unsigned)((R + 31) / 32)), dim3(256), 0, s, src,
                     R, C, dst);
  return hipGetLastError();
}

// forward 2-D transform of a real H x W image zero-padded to P x Q; the
// result is left transposed (Q x P) in `out`, `tmp` is P x Q scratch
hipError_t forward2d(const float* x, int64_t s0, int64_t s1, int H, int W, int P, int Q, const float2* twP,
                     const float2* twQ, float2* tmp, float2* out, hipStream_t s) {
  hipLaunchKernelGGL(pad_real, dim3((unsigned)((Q + 255) / 256), (unsigned)P), dim3(256), 0, s, x, s0, s1, H, W, tmp,
                     Q);
  hipError_t e;
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = rows(tmp, P, Q, twQ, false, s)) != hipSuccess) return e;
  if ((e = transpose(tmp, P, Q, out, s)) != hipSuccess) return e;
  return rows(out, Q, P, twP, false, s);
}

}  // namespace

hipError_t launch_conv2d_fft(const FftConv& f, hipStream_t s) {
  const int P = f.P, Q = f.Q;
  hipError_t e;
  hipLaunchKernelGGL(fft_twiddles, dim3((unsigned)((P / 2 + 255) / 256)), dim3(256), 0, s, f.twP, P);
  hipLaunchKernelGGL(fft_twiddles, dim3((unsigned)((Q / 2 + 255) / 256)), dim3(256), 0, s, f.twQ, Q);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = forward2d(f.x, f.xs0, f.xs1, f.H, f.W, P, Q, f.twP, f.twQ, f.A, f.B, s)) != hipSuccess) return e;
  if ((e = forward2d(f.k, f.KW, 1, f.KH, f.KW, P, Q, f.twP, f.twQ, f.A, f.C, s)) != hipSuccess) return e;
  const int64_t n = (int64_t)P * Q;
  hipLaunchKernelGGL(mul_c, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f.B, f.C, n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = rows(f.B, Q, P, f.twP, true, s)) != hipSuccess) return e;
  if ((e = transpose(f.B, Q, P, f.A, s)) != hipSuccess) return e;
  if ((e = rows(f.A, P, Q, f.twQ, true, s)) != hipSuccess) return e;
  if (f.OH > 0 && f.OW > 0)
    hipLaunchKernelGGL(extract_real, dim3((unsigned)((f.OW + 255) / 256), (unsigned)f.OH), dim3(256), 0, s, f.A, Q,
                       f.o0, f.o1, f.OH, f.OW, 1.0f / ((float)P * (float)Q), f.y, f.ys0, f.ys1);
  return hipGetLastError();
}

}  // namespace ttc
