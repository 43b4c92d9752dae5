// FFT branch of 2-D convolution (Convolutions section: the convolution theorem,
// y = F^-1(F(x) F(k)); Accelerating Convolutions: the hybrid that switches to
// it for large kernels).
//
// fft_twiddles: w[k] = exp(-2 pi i k / N), k < N, with sincospi (exact
//               argument k/N for N a power of two).
// fft_rows:     Stockham transform of length N = 2^m <= 4096 along each row,
//               one work-group per row, the row held in LDS: one radix-2
//               stage when m is odd, then radix-4 stages (described in the
//               kernel).  The inverse uses conjugate twiddles and no scale.
// transpose_c:  complex R x C -> C x R through 32 x 33 LDS tiles.
// mul_c:        the pointwise product.  The first forward pass reads the real
//               image and pads it in LDS; the last inverse pass writes the real
//               part, scaled by 1/(P Q), of the mode's window straight into y.
#include <math.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace ttc {
namespace {

constexpr int kFftThreads = 256;
constexpr int kFftPerThread = kFftMaxN / 2 / kFftThreads;   // radix-2 butterflies per thread (max)
constexpr int kFftPerThread4 = kFftMaxN / 4 / kFftThreads;  // radix-4 butterflies per thread (max)

__global__ __launch_bounds__(256) void fft_twiddles(float2* __restrict__ tw, int N) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  float s, c;
  sincospif(-2.0f * (float)k / (float)N, &s, &c);
  tw[k] = make_float2(c, s);
}

template <bool INV>
__device__ __forceinline__ float2 cmul_tw(float2 w, float2 b) {
  if (INV) w.y = -w.y;
  return make_float2(w.x * b.x - w.y * b.y, w.x * b.y + w.y * b.x);
}

// Where a row pass reads and writes besides the complex plane: IN_REAL rows
// come from a real H x W image (zero beyond it: the padding), OUT_REAL rows
// o0 .. o0 + OH - 1 leave as the real part times `scale`, columns o1 .. o1 +
// OW - 1, into y (the cut of the requested mode).
struct RowIO {
  const float* x;
  int64_t xs0, xs1;
  int H, W;
  float* y;
  int64_t ys0, ys1;
  int OH, OW, o0, o1;
  float scale;
};

template <bool INV, bool IN_REAL, bool OUT_REAL>
__global__ __launch_bounds__(kFftThreads) void fft_rows(float2* __restrict__ data, int64_t row_stride, int N, int m,
                                                        const float2* __restrict__ tw, RowIO io) {
  __shared__ float2 buf[kFftMaxN];
  // every radix-4 stage reads w^k = tw[k N / (4 Ls)] with k < Ls: the first
  // quarter of the table, staged in LDS once
  __shared__ float2 twl[kFftMaxN / 4];
  const int r = OUT_REAL ? io.o0 + (int)blockIdx.x : (int)blockIdx.x;
  float2* row = data + (int64_t)r * row_stride;
  const int tid = threadIdx.x;
  if (IN_REAL) {
    for (int i = tid; i < N; i += kFftThreads)
      buf[i] = make_float2((r < io.H && i < io.W) ? io.x[(int64_t)r * io.xs0 + (int64_t)i * io.xs1] : 0.f, 0.f);
  } else {
    for (int i = tid; i < N; i += kFftThreads) buf[i] = row[i];
  }
  for (int i = tid; i < (N >> 2); i += kFftThreads) twl[i] = tw[i];
  __syncthreads();
  int lg = 0;  // log2 of the sub-transform length done so far
  if (m & 1) {
    // one radix-2 stage (sub-length 1: no twiddles)
    const int half = N >> 1;
    float2 o0[kFftPerThread], o1[kFftPerThread];
#pragma unroll
    for (int c = 0; c < kFftPerThread; ++c) {
      const int j = tid + c * kFftThreads;
      if (j < half) {
        const float2 a = buf[j], b = buf[j + half];
        o0[c] = make_float2(a.x + b.x, a.y + b.y);
        o1[c] = make_float2(a.x - b.x, a.y - b.y);
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kFftPerThread; ++c) {
      const int j = tid + c * kFftThreads;
      if (j < half) {
        buf[2 * j] = o0[c];
        buf[2 * j + 1] = o1[c];
      }
    }
    __syncthreads();
    lg = 1;
  }
  // radix-4 stages: sub-length Ls = 2^lg; a_t = v[j + t N/4] w^(t k),
  // w = exp(-+2 pi i / (4 Ls)) = tw[k t N / (4 Ls)], k = j mod Ls; the 4-point
  // transform of (a_0..a_3) goes to v'[(j / Ls) 4 Ls + k + q Ls], q = 0..3
  const int q4 = N >> 2;
  for (; lg < m; lg += 2) {
    const int Ls = 1 << lg;
    const int tws = m - lg - 2;  // log2(N / (4 Ls))
    float2 o[kFftPerThread4][4];
#pragma unroll
    for (int c = 0; c < kFftPerThread4; ++c) {
      const int j = tid + c * kFftThreads;
      if (j < q4) {
        const int k = j & (Ls - 1);
        // one table read per butterfly: w^2k and w^3k as products of w^k
        const float2 w1 = twl[k << tws];
        const float2 w2 = make_float2(w1.x * w1.x - w1.y * w1.y, 2.f * w1.x * w1.y);
        const float2 w3 = make_float2(w2.x * w1.x - w2.y * w1.y, w2.x * w1.y + w2.y * w1.x);
        const float2 a0 = buf[j];
        const float2 a1 = cmul_tw<INV>(w1, buf[j + q4]);
        const float2 a2 = cmul_tw<INV>(w2, buf[j + 2 * q4]);
        const float2 a3 = cmul_tw<INV>(w3, buf[j + 3 * q4]);
        const float2 b0 = make_float2(a0.x + a2.x, a0.y + a2.y), b1 = make_float2(a0.x - a2.x, a0.y - a2.y);
        const float2 b2 = make_float2(a1.x + a3.x, a1.y + a3.y), b3 = make_float2(a1.x - a3.x, a1.y - a3.y);
        // forward: -i b3; inverse: +i b3
        const float2 r = INV ? make_float2(-b3.y, b3.x) : make_float2(b3.y, -b3.x);
        o[c][0] = make_float2(b0.x + b2.x, b0.y + b2.y);
        o[c][1] = make_float2(b1.x + r.x, b1.y + r.y);
        o[c][2] = make_float2(b0.x - b2.x, b0.y - b2.y);
        o[c][3] = make_float2(b1.x - r.x, b1.y - r.y);
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kFftPerThread4; ++c) {
      const int j = tid + c * kFftThreads;
      if (j < q4) {
        const int k = j & (Ls - 1);
        const int base = ((j >> lg) << (lg + 2)) + k;
#pragma unroll
        for (int q = 0; q < 4; ++q) buf[base + q * Ls] = o[c][q];
      }
    }
    __syncthreads();
  }
  if (OUT_REAL) {
    float* yr = io.y + (int64_t)(r - io.o0) * io.ys0;
    for (int i = tid; i < io.OW; i += kFftThreads) yr[(int64_t)i * io.ys1] = buf[io.o1 + i].x * io.scale;
  } else {
    for (int i = tid; i < N; i += kFftThreads) row[i] = buf[i];
  }
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

__global__ __launch_bounds__(256) void mul_c(float2* __restrict__ a, const float2* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float2 u = a[i], v = b[i];
  a[i] = make_float2(u.x * v.x - u.y * v.y, u.x * v.y + u.y * v.x);
}

int ilog2(int n) {
  int m = 0;
  while ((1 << m) < n) ++m;
  return m;
}

template <bool INV, bool IN_REAL, bool OUT_REAL>
hipError_t rows_t(float2* d, int n_rows, int N, const float2* tw, const RowIO& io, hipStream_t s) {
  hipLaunchKernelGGL((fft_rows<INV, IN_REAL, OUT_REAL>), dim3((unsigned)n_rows), dim3(kFftThreads), 0, s, d,
                     (int64_t)N, N, ilog2(N), tw, io);
  return hipGetLastError();
}

hipError_t rows(float2* d, int n_rows, int N, const float2* tw, bool inv, hipStream_t s) {
  const RowIO io{};
  return inv ? rows_t<true, false, false>(d, n_rows, N, tw, io, s)
             : rows_t<false, false, false>(d, n_rows, N, tw, io, s);
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
  RowIO io{};
  io.x = x;
  io.xs0 = s0;
  io.xs1 = s1;
  io.H = H;
  io.W = W;
  hipError_t e;
  // the first pass reads the real image itself (zero-padded in LDS)
  if ((e = rows_t<false, true, false>(tmp, P, Q, twQ, io, s)) != hipSuccess) return e;
  if ((e = transpose(tmp, P, Q, out, s)) != hipSuccess) return e;
  return rows(out, Q, P, twP, false, s);
}

}  // namespace

hipError_t launch_conv2d_fft(const FftConv& f, hipStream_t s) {
  const int P = f.P, Q = f.Q;
  hipError_t e;
  hipLaunchKernelGGL(fft_twiddles, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, f.twP, P);
  hipLaunchKernelGGL(fft_twiddles, dim3((unsigned)((Q + 255) / 256)), dim3(256), 0, s, f.twQ, Q);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = forward2d(f.x, f.xs0, f.xs1, f.H, f.W, P, Q, f.twP, f.twQ, f.A, f.B, s)) != hipSuccess) return e;
  if ((e = forward2d(f.k, f.KW, 1, f.KH, f.KW, P, Q, f.twP, f.twQ, f.A, f.C, s)) != hipSuccess) return e;
  const int64_t n = (int64_t)P * Q;
  hipLaunchKernelGGL(mul_c, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f.B, f.C, n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = rows(f.B, Q, P, f.twP, true, s)) != hipSuccess) return e;
  if ((e = transpose(f.B, Q, P, f.A, s)) != hipSuccess) return e;
  // the last pass transforms only the rows of the mode's window and writes
  // their real part, scaled, straight into y
  if (f.OH <= 0 || f.OW <= 0) return hipSuccess;
  RowIO io{};
  io.y = f.y;
  io.ys0 = f.ys0;
  io.ys1 = f.ys1;
  io.OH = f.OH;
  io.OW = f.OW;
  io.o0 = f.o0;
  io.o1 = f.o1;
  io.scale = 1.0f / ((float)P * (float)Q);
  return rows_t<true, false, true>(f.A, f.OH, Q, f.twQ, io, s);
}

}  // namespace ttc
