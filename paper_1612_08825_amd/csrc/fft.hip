// FFT branch of 2-D and 3-D convolution (Convolutions section: the convolution
// theorem, y = F^-1(F(x) F(k)); Accelerating Convolutions: the hybrid that
// switches to it for large kernels; Future Work: the n-dimensional extension).
//
// x and k are zero-padded to a volume n0 x .. x n_{d-1} (d = 2 or 3) whose
// extents are 2^a 3^b 5^c, at least the full output's, at most kFftMaxN each.
// A d-dimensional transform is d passes of 1-D transforms along the last axis,
// with a 2-D transpose between passes that moves the transformed axis out of
// the way:
//   forward: rows along n_{d-1}; [rest][n_{d-1}] -> [n_{d-1}][rest]; rows along
//            n_{d-2}; ...; rows along n_0.  The spectrum is left in the order
//            (n_1, .., n_{d-1}, n_0): the inverse undoes it without a final
//            transpose.
//   inverse: rows along n_0; [first][rest] -> [rest][first]; rows along n_1;
//            ...; the last pass (along n_{d-1}, back in the original order)
//            transforms only the rows of the mode's window and writes their
//            real part, scaled by 1 / (n_0 .. n_{d-1}), straight into y.
// The first forward pass reads the real image (or kernel) and pads it with
// zeros in LDS.
//
// fft_twiddles: w[m] = exp(-2 pi i m / N), m < N, evaluated in FP64 and rounded.
// fft_rows:     a Stockham transform of kFftMaxN / N rows per work-group (at
//               least one), the rows in LDS, in stages of radix 4, 2, 3 and 5
//               (the stage list comes from the host; described at
//               fft_stage).  The inverse uses conjugate twiddles and no scale.
// transpose_c:  complex R x C -> C x R through 32 x 33 LDS tiles.
// mul_c:        the pointwise product of the two spectra.
#include <math.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace ttc {
namespace {

constexpr int kFftThreads = 256;

__global__ __launch_bounds__(256) void fft_twiddles(float2* __restrict__ tw, int N) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  double s, c;
  sincospi(-2.0 * (double)m / (double)N, &s, &c);
  tw[m] = make_float2((float)c, (float)s);
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float s, float2 a) { return make_float2(s * a.x, s * a.y); }
// -i z for the forward transform, +i z for the inverse
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 z) {
  return INV ? make_float2(-z.y, z.x) : make_float2(z.y, -z.x);
}

// The R-point DFT of a[0..R-1] in place: a_q <- sum_t a_t e^(-+2 pi i t q / R).
template <int R, bool INV>
__device__ __forceinline__ void dft_small(float2 (&a)[R]) {
  if constexpr (R == 2) {
    const float2 b0 = cadd(a[0], a[1]), b1 = csub(a[0], a[1]);
    a[0] = b0;
    a[1] = b1;
  } else if constexpr (R == 3) {
    constexpr float kS3 = 0.86602540378443864676f;  // sin(2 pi / 3)
    const float2 t1 = cadd(a[1], a[2]);
    const float2 t2 = make_float2(a[0].x - 0.5f * t1.x, a[0].y - 0.5f * t1.y);
    const float2 t3 = mul_mi<INV>(cscale(kS3, csub(a[1], a[2])));
    a[0] = cadd(a[0], t1);
    a[1] = cadd(t2, t3);
    a[2] = csub(t2, t3);
  } else if constexpr (R == 4) {
    const float2 b0 = cadd(a[0], a[2]), b1 = csub(a[0], a[2]);
    const float2 b2 = cadd(a[1], a[3]), b3 = mul_mi<INV>(csub(a[1], a[3]));
    a[0] = cadd(b0, b2);
    a[1] = cadd(b1, b3);
    a[2] = csub(b0, b2);
    a[3] = csub(b1, b3);
  } else {
    static_assert(R == 5, "radix 2, 3, 4 or 5");
    constexpr float kC1 = 0.30901699437494742410f;   // cos(2 pi / 5)
    constexpr float kC2 = -0.80901699437494742410f;  // cos(4 pi / 5)
    constexpr float kS1 = 0.95105651629515357212f;   // sin(2 pi / 5)
    constexpr float kS2 = 0.58778525229247312917f;   // sin(4 pi / 5)
    const float2 t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
    const float2 t3 = csub(a[1], a[4]), t4 = csub(a[2], a[3]);
    const float2 r1 = make_float2(a[0].x + kC1 * t1.x + kC2 * t2.x, a[0].y + kC1 * t1.y + kC2 * t2.y);
    const float2 r2 = make_float2(a[0].x + kC2 * t1.x + kC1 * t2.x, a[0].y + kC2 * t1.y + kC1 * t2.y);
    const float2 i1 = mul_mi<INV>(make_float2(kS1 * t3.x + kS2 * t4.x, kS1 * t3.y + kS2 * t4.y));
    const float2 i2 = mul_mi<INV>(make_float2(kS2 * t3.x - kS1 * t4.x, kS2 * t3.y - kS1 * t4.y));
    a[0] = make_float2(a[0].x + t1.x + t2.x, a[0].y + t1.y + t2.y);
    a[1] = cadd(r1, i1);
    a[4] = csub(r1, i1);
    a[2] = cadd(r2, i2);
    a[3] = csub(r2, i2);
  }
}

// One Stockham stage of radix R on nr rows in LDS (row i at buf + i N; N
// points each, sub-transforms of length Ls done so far, N divisible by R Ls):
// for j < N / R with k = j mod Ls, a_t = v[j + t N / R] w^(t k), w = exp(-+2 pi
// i / (R Ls)) = tw[N / (R Ls)]; the R-point DFT of (a_t) goes to
// v'[(j / Ls) R Ls + k + q Ls], q < R.  One table read per butterfly: w^k
// from the table staged in LDS (k N / (R Ls) < N / 2), its higher powers by
// multiplication.  All reads before a barrier, all writes after it.
template <int R, bool INV>
__device__ __forceinline__ void fft_stage(float2* buf, const float2* twl, int N, int nr, int Ls) {
  constexpr int kPer = (kFftMaxN / R + kFftThreads - 1) / kFftThreads;
  const int nb = N / R;
  const int step = N / (R * Ls);
  const int tid = threadIdx.x;
  float2 o[kPer][R];
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int b = tid + c * kFftThreads;
    if (b < nr * nb) {
      const int i = b / nb, j = b - i * nb;
      const float2* v = buf + i * N;
      const int k = j % Ls;
      float2 w = twl[k * step];
      if (INV) w.y = -w.y;
      o[c][0] = v[j];
      float2 wt = w;
#pragma unroll
      for (int t = 1; t < R; ++t) {
        o[c][t] = cmul(wt, v[j + t * nb]);
        if (t + 1 < R) wt = cmul(wt, w);
      }
      dft_small<R, INV>(o[c]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int b = tid + c * kFftThreads;
    if (b < nr * nb) {
      const int i = b / nb, j = b - i * nb;
      const int k = j % Ls;
      float2* v = buf + i * N;
      const int base = (j / Ls) * R * Ls + k;
#pragma unroll
      for (int q = 0; q < R; ++q) v[base + q * Ls] = o[c][q];
    }
  }
  __syncthreads();
}

// Where a row pass reads and writes besides the complex volume.
//   IN_REAL: row r = a * nb + b of the padded volume is the source row at
//   src + a sa + b sb (element step s_in) when a < ea and b < eb, its first
//   w_in elements, zero elsewhere (the padding).
//   OUT_REAL: work-group g of an OA x OB grid is row (oa + g / OB) * nb +
//   (ob + g % OB); its elements oc .. oc + ow - 1 go, real part times scale,
//   to y + (g / OB) ya + (g % OB) yb + i yc.
struct RowIO {
  const float* src;
  int64_t sa, sb, s_in;
  int ea, eb, w_in;
  int nb;
  float* y;
  int64_t ya, yb, yc;
  int OA, OB, oa, ob, oc, ow;
  float scale;
};

// A work-group transforms nr = max(1, kFftMaxN / N) consecutive rows (rows
// 0 .. n_rows - 1 in all); dynamic LDS: nr N points, then N / 2 twiddles.
//
// HALF (the last axis, real data): the row is real and 2N long; it is
// transformed as N complex points z[m] = x[2m] + i x[2m+1] and kept as its
// N + 1 non-negative frequencies (a stored row is N + 1 long).  Forward (with
// IN_REAL), after the N-point transform Z: X[k] = E + W^k O for k <= N, with
// E = (Z[k] + conj Z[N-k]) / 2, O = -i (Z[k] - conj Z[N-k]) / 2 (the
// transforms of the even and the odd samples), W = exp(-2 pi i / 2N).
// Inverse (with OUT_REAL), before the transform: Z[k] = E + i O with
// E = (X[k] + conj X[N-k]) / 2, O = W^-k (X[k] - conj X[N-k]) / 2, and the
// inverse of Z holds N (x[2m] + i x[2m+1]).  tw is then the 2N-point table:
// the N-point transform reads every second entry.
template <bool INV, bool IN_REAL, bool OUT_REAL, bool HALF>
__global__ __launch_bounds__(kFftThreads) void fft_rows(float2* __restrict__ data, FftAxis ax,
                                                        const float2* __restrict__ tw, int64_t n_rows, RowIO io) {
  extern __shared__ float2 lds[];
  const int N = ax.n;
  const int ld = HALF ? N + 1 : N;  // stored row length
  const int nr = N >= kFftMaxN ? 1 : kFftMaxN / N;
  float2* buf = lds;
  float2* twl = lds + nr * N;
  const int64_t g0 = (int64_t)blockIdx.x * nr;
  const int nrow = (int)(n_rows - g0 < nr ? n_rows - g0 : nr);  // rows of this work-group
  const int tid = threadIdx.x;
  // the global row of local row i (OUT_REAL: the i-th row of the window)
  auto row_of = [&](int i) -> int64_t {
    const int64_t g = g0 + i;
    if (OUT_REAL) return (int64_t)(io.oa + g / io.OB) * io.nb + (io.ob + g % io.OB);
    return g;
  };
  if (IN_REAL) {
    // rows wholly in the padding transform to zero: write them and stop
    bool any = false;
    for (int i = 0; i < nrow; ++i) {
      const int64_t r = row_of(i);
      const int64_t a = r / io.nb, b = r - a * io.nb;
      any |= a < io.ea && b < io.eb;
    }
    if (!any) {
      for (int64_t e = tid; e < (int64_t)nrow * ld; e += kFftThreads) data[g0 * ld + e] = make_float2(0.f, 0.f);
      return;
    }
    for (int e = tid; e < nr * N; e += kFftThreads) {
      const int i = e / N, c = e - i * N;
      float2 v = make_float2(0.f, 0.f);
      if (i < nrow) {
        const int64_t r = row_of(i);
        const int64_t a = r / io.nb, b = r - a * io.nb;
        if (a < io.ea && b < io.eb) {
          const float* sr = io.src + a * io.sa + b * io.sb;
          if (HALF) {
            if (2 * c < io.w_in) v.x = sr[(int64_t)(2 * c) * io.s_in];
            if (2 * c + 1 < io.w_in) v.y = sr[(int64_t)(2 * c + 1) * io.s_in];
          } else if (c < io.w_in) {
            v.x = sr[(int64_t)c * io.s_in];
          }
        }
      }
      buf[e] = v;
    }
  } else if (HALF) {
    // the N + 1 stored frequencies of each row -> Z (the inverse's input)
    for (int e = tid; e < nr * N; e += kFftThreads) {
      const int i = e / N, k = e - i * N;
      float2 z = make_float2(0.f, 0.f);
      if (i < nrow) {
        const float2* row = data + row_of(i) * ld;
        const float2 xk = row[k], xc = row[N - k];
        const float2 ev = make_float2(0.5f * (xk.x + xc.x), 0.5f * (xk.y - xc.y));
        const float2 d = make_float2(0.5f * (xk.x - xc.x), 0.5f * (xk.y + xc.y));  // (X[k] - conj X[N-k]) / 2
        float2 w = tw[k];
        w.y = -w.y;  // W^-k
        const float2 od = cmul(w, d);
        z = make_float2(ev.x - od.y, ev.y + od.x);  // E + i O
      }
      buf[e] = z;
    }
  } else {
    for (int e = tid; e < nr * N; e += kFftThreads) {
      const int i = e / N, c = e - i * N;
      buf[e] = i < nrow ? data[row_of(i) * N + c] : make_float2(0.f, 0.f);
    }
  }
  for (int i = tid; i < (N >> 1); i += kFftThreads) twl[i] = tw[HALF ? 2 * i : i];
  __syncthreads();
  // the stage list runs radix 4, then 2, then 3, then 5: one loop per radix
  // (a switch over the radix inside one loop costs twice the registers)
  int Ls = 1, st = 0;
  for (; st < ax.n_stages && ax.radix[st] == 4; ++st, Ls *= 4) fft_stage<4, INV>(buf, twl, N, nr, Ls);
  for (; st < ax.n_stages && ax.radix[st] == 2; ++st, Ls *= 2) fft_stage<2, INV>(buf, twl, N, nr, Ls);
  for (; st < ax.n_stages && ax.radix[st] == 3; ++st, Ls *= 3) fft_stage<3, INV>(buf, twl, N, nr, Ls);
  for (; st < ax.n_stages && ax.radix[st] == 5; ++st, Ls *= 5) fft_stage<5, INV>(buf, twl, N, nr, Ls);
  if (OUT_REAL) {
    for (int i = 0; i < nrow; ++i) {
      const int64_t g = g0 + i;
      float* yr = io.y + (g / io.OB) * io.ya + (g % io.OB) * io.yb;
      for (int c = tid; c < io.ow; c += kFftThreads) {
        const int n = io.oc + c;
        float v;
        if (HALF) {
          const float2 z = buf[i * N + (n >> 1)];
          v = (n & 1) ? z.y : z.x;
        } else {
          v = buf[i * N + n].x;
        }
        yr[(int64_t)c * io.yc] = v * io.scale;
      }
    }
  } else if (HALF) {
    // the N + 1 non-negative frequencies of each real row
    for (int e = tid; e < nrow * ld; e += kFftThreads) {
      const int i = e / ld, k = e - i * ld;
      const float2 zk = buf[i * N + (k == N ? 0 : k)], zc = buf[i * N + (k == 0 ? 0 : N - k)];
      const float2 ev = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y - zc.y));
      const float2 d = make_float2(0.5f * (zk.x - zc.x), 0.5f * (zk.y + zc.y));  // (Z[k] - conj Z[N-k]) / 2
      const float2 od = make_float2(d.y, -d.x);                                    // -i d
      const float2 wo = cmul(tw[k], od);
      data[row_of(i) * ld + k] = make_float2(ev.x + wo.x, ev.y + wo.y);
    }
  } else {
    for (int e = tid; e < nrow * N; e += kFftThreads) {
      const int i = e / N, c = e - i * N;
      data[row_of(i) * N + c] = buf[e];
    }
  }
}

// dst[c][r] = src[r][c] for an R x C source (grid.y steps over row tiles).
__global__ __launch_bounds__(256) void transpose_c(const float2* __restrict__ src, int64_t R, int64_t C,
                                                   float2* __restrict__ dst) {
  __shared__ float2 tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t c0 = (int64_t)blockIdx.x * 32;
  for (int64_t r0 = (int64_t)blockIdx.y * 32; r0 < R; r0 += (int64_t)gridDim.y * 32) {
#pragma unroll
    for (int i = 0; i < 32; i += 8) {
      const int64_t r = r0 + ty + i, c = c0 + tx;
      if (r < R && c < C) tile[ty + i][tx] = src[r * C + c];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 32; i += 8) {
      const int64_t c = c0 + ty + i, r = r0 + tx;
      if (c < C && r < R) dst[c * R + r] = tile[tx][ty + i];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void mul_c(float2* __restrict__ a, const float2* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = cmul(a[i], b[i]);
}

template <bool INV, bool IN_REAL, bool OUT_REAL, bool HALF = false>
hipError_t rows_t(float2* d, int64_t n_rows, const FftAxis& ax, const float2* tw, const RowIO& io, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  const int N = ax.n;
  const int nr = N >= kFftMaxN ? 1 : kFftMaxN / N;
  const size_t lds = ((size_t)nr * N + (size_t)(N >> 1)) * sizeof(float2);
  hipLaunchKernelGGL((fft_rows<INV, IN_REAL, OUT_REAL, HALF>), dim3((unsigned)((n_rows + nr - 1) / nr)),
                     dim3(kFftThreads), lds, s, d, ax, tw, n_rows, io);
  return hipGetLastError();
}

hipError_t transpose(const float2* src, int64_t R, int64_t C, float2* dst, hipStream_t s) {
  const int64_t gy = (R + 31) / 32;
  hipLaunchKernelGGL(transpose_c, dim3((unsigned)((C + 31) / 32), (unsigned)(gy < 65535 ? gy : 65535)), dim3(256),
                     0, s, src, R, C, dst);
  return hipGetLastError();
}

// Stored extents of the spectrum: n_a for every axis but the last, whose
// real transform keeps its n / 2 + 1 non-negative frequencies (the axis plan
// of the last axis is for the half length).
void stored_extents(const FftConv& f, int64_t (&ext)[3], int64_t& T) {
  T = 1;
  for (int a = 0; a < f.rank; ++a) {
    ext[a] = a == f.rank - 1 ? (int64_t)f.ax[a].n + 1 : f.ax[a].n;
    T *= ext[a];
  }
}

// The forward transform of a real array (extents e[], strides st[], leading
// axis first) zero-padded to the volume; the spectrum ends in `out`, in the
// order (n_1, .., n_{d-1}, n_0) with the last axis halved; `tmp` is scratch of
// the same size.
hipError_t forward(const FftConv& f, const float* src, const int64_t* st, const int* e, float2* tmp, float2* out,
                   hipStream_t s) {
  const int d = f.rank;
  int64_t ext[3], T;
  stored_extents(f, ext, T);
  RowIO io{};
  io.src = src;
  io.s_in = st[d - 1];
  io.w_in = e[d - 1];
  if (d == 2) {
    io.nb = 1;
    io.sa = st[0];
    io.ea = e[0];
    io.sb = 0;
    io.eb = 1;
  } else {
    io.nb = f.ax[1].n;
    io.sa = st[0];
    io.ea = e[0];
    io.sb = st[1];
    io.eb = e[1];
  }
  // d - 1 transposes follow the first pass: start where the last pass must end
  float2* cur = ((d - 1) % 2 == 0) ? out : tmp;
  float2* other = (cur == out) ? tmp : out;
  hipError_t err;
  const RowIO none{};
  if ((err = rows_t<false, true, false, true>(cur, T / ext[d - 1], f.ax[d - 1], f.tw[d - 1], io, s)) != hipSuccess)
    return err;
  for (int a = d - 1; a >= 1; --a) {
    if ((err = transpose(cur, T / ext[a], ext[a], other, s)) != hipSuccess) return err;
    float2* t = cur;
    cur = other;
    other = t;
    if ((err = rows_t<false, false, false>(cur, T / ext[a - 1], f.ax[a - 1], f.tw[a - 1], none, s)) != hipSuccess)
      return err;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_conv_fft(const FftConv& f, hipStream_t s) {
  const int d = f.rank;
  hipError_t err;
  for (int a = 0; a < d; ++a) {
    const int n = a == d - 1 ? 2 * f.ax[a].n : f.ax[a].n;  // the last axis: the full real length
    hipLaunchKernelGGL(fft_twiddles, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f.tw[a], n);
  }
  if ((err = hipGetLastError()) != hipSuccess) return err;
  int64_t ext[3], T;
  stored_extents(f, ext, T);
  const int64_t kst[3] = {d == 3 ? (int64_t)f.kn[1] * f.kn[2] : (int64_t)f.kn[1], d == 3 ? (int64_t)f.kn[2] : 1, 1};
  if ((err = forward(f, f.x, f.xs, f.xn, f.A, f.B, s)) != hipSuccess) return err;
  if ((err = forward(f, f.k, kst, f.kn, f.A, f.C, s)) != hipSuccess) return err;
  const int64_t blocks = (T + 255) / 256;
  hipLaunchKernelGGL(mul_c, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, f.B, f.C, T);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  // inverse, from the order (n_1, .., n_{d-1}, n_0): rows along n_0, then for
  // each further axis a transpose [first][rest] -> [rest][first] and rows along
  // the axis now last; d - 1 transposes, the last rows pass (the real inverse
  // of the halved axis) writes y
  float2* cur = f.B;
  float2* other = f.A;
  const RowIO none{};
  if ((err = rows_t<true, false, false>(cur, T / ext[0], f.ax[0], f.tw[0], none, s)) != hipSuccess) return err;
  for (int a = 1; a < d; ++a) {
    // the current first axis is axis a
    if ((err = transpose(cur, ext[a], T / ext[a], other, s)) != hipSuccess) return err;
    float2* t = cur;
    cur = other;
    other = t;
    if (a < d - 1) {
      if ((err = rows_t<true, false, false>(cur, T / ext[a], f.ax[a], f.tw[a], none, s)) != hipSuccess) return err;
    }
  }
  int64_t n_out = 1;
  for (int a = 0; a < d; ++a) n_out *= f.yn[a];
  if (n_out == 0) return hipSuccess;
  // unnormalised inverses: n_a along every full axis, n / 2 along the halved one
  double norm = f.ax[d - 1].n;
  for (int a = 0; a < d - 1; ++a) norm *= f.ax[a].n;
  RowIO io{};
  io.y = f.y;
  io.yc = f.ys[d - 1];
  io.oc = f.o[d - 1];
  io.ow = f.yn[d - 1];
  io.scale = (float)(1.0 / norm);
  if (d == 2) {
    io.nb = 1;
    io.OA = f.yn[0];
    io.OB = 1;
    io.oa = f.o[0];
    io.ob = 0;
    io.ya = f.ys[0];
    io.yb = 0;
  } else {
    io.nb = f.ax[1].n;
    io.OA = f.yn[0];
    io.OB = f.yn[1];
    io.oa = f.o[0];
    io.ob = f.o[1];
    io.ya = f.ys[0];
    io.yb = f.ys[1];
  }
  return rows_t<true, false, true, true>(cur, (int64_t)io.OA * io.OB, f.ax[d - 1], f.tw[d - 1], io, s);
}

}  // namespace ttc
