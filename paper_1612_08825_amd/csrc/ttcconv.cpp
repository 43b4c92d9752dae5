// Host side of the C ABI declared in include/ttcconv.h: argument validation,
// work planning for the fused TTC pass, and kernel dispatch.  No device memory
// is allocated here; the only host allocations are plan objects (pinned work
// tables) and the small tap copy of integer convolutions.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "internal.hpp"

using namespace ttc;

namespace {

constexpr int kVersion = 100;  // 0.1.0

int elem_size(int dt) {
  switch (dt) {
    case TC_U8: return 1;
    case TC_F16: return 2;
    case TC_F32: return 4;
    case TC_I32: return 4;
    case TC_F64: return 8;
    default: return 0;
  }
}

int64_t numel(const tc_tensor* t) {
  int64_t n = 1;
  for (int d = 0; d < t->ndim; ++d) n *= t->shape[d];
  return n;
}

// Basic structural checks of a descriptor.
int check_tensor(const tc_tensor* t, bool need_data) {
  if (!t) return TC_EINVAL;
  if (t->ndim < 1 || t->ndim > TC_MAX_DIMS) return TC_ESHAPE;
  if (elem_size(t->dtype) == 0) return TC_EDTYPE;
  for (int d = 0; d < t->ndim; ++d) {
    if (t->shape[d] < 0 || t->shape[d] > (1LL << 40)) return TC_ESHAPE;
    if (t->shape[d] > 1 && t->stride[d] == 0) return TC_ESHAPE;
  }
  if (need_data && numel(t) > 0 && t->data == nullptr) return TC_EINVAL;
  return TC_OK;
}

bool is_contiguous(const tc_tensor* t) {
  int64_t s = 1;
  for (int d = t->ndim - 1; d >= 0; --d) {
    if (t->shape[d] > 1 && t->stride[d] != s) return false;
    s *= t->shape[d];
  }
  return true;
}

int hip_status(hipError_t e) { return e == hipSuccess ? TC_OK : TC_EDEVICE; }

int conv_dtypes_ok(int xdt, int kdt) {
  if (xdt == TC_F32 && kdt == TC_F32) return TC_F32;
  if (xdt == TC_F16 && kdt == TC_F32) return TC_F32;
  if (xdt == TC_U8 && kdt == TC_I32) return TC_I32;
  return -1;
}

int conv_geometry(const tc_tensor* x, const tc_tensor* k, int32_t mode, int64_t* out_shape, int64_t* off) {
  if (x->ndim != k->ndim) return TC_ESHAPE;
  const int r = x->ndim;
  if (mode == TC_FULL) {
    for (int d = 0; d < r; ++d) {
      out_shape[d] = x->shape[d] + k->shape[d] - 1;
      if (x->shape[d] == 0 || k->shape[d] == 0) out_shape[d] = 0;
      off[d] = 0;
    }
  } else if (mode == TC_SAME) {
    for (int d = 0; d < r; ++d) {
      out_shape[d] = x->shape[d];
      off[d] = (k->shape[d] - 1) / 2;
      if (k->shape[d] == 0) out_shape[d] = 0;
    }
  } else if (mode == TC_VALID) {
    bool ge = true, le = true;
    for (int d = 0; d < r; ++d) {
      ge = ge && x->shape[d] >= k->shape[d];
      le = le && x->shape[d] <= k->shape[d];
    }
    if (!ge && !le) return TC_ESHAPE;
    for (int d = 0; d < r; ++d) {
      const int64_t n = x->shape[d], m = k->shape[d];
      out_shape[d] = (n == 0 || m == 0) ? 0 : (n > m ? n - m : m - n) + 1;
      off[d] = std::min(n, m) - 1;
      if (off[d] < 0) off[d] = 0;
    }
  } else {
    return TC_EINVAL;
  }
  return TC_OK;
}

int current_cu_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}

}  // namespace

// ============================================================================ misc
extern "C" const char* tc_status_str(int status) {
  switch (status) {
    case TC_OK: return "ok";
    case TC_SINGULAR: return "singular normal matrix";
    case TC_NEED_PREV: return "no previous frame";
    case TC_NONFINITE: return "non-finite sums";
    case TC_EINVAL: return "invalid argument";
    case TC_ESHAPE: return "inconsistent shape or stride";
    case TC_EDTYPE: return "unsupported dtype";
    case TC_EOVERFLOW: return "integer result could overflow int32";
    case TC_ENOMEM: return "workspace too small";
    case TC_EDEVICE: return "HIP error or unsupported device";
    default: return "unknown status";
  }
}

extern "C" int tc_version(void) { return kVersion; }

extern "C" int tc_device_check(int device, int* n_cu) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return TC_EDEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TC_EDEVICE;
  if (n_cu) *n_cu = prop.multiProcessorCount;
  return TC_OK;
}

// ============================================================================ convolution
extern "C" int tc_conv_out_shape(const tc_tensor* x, const tc_tensor* k, int32_t mode, int64_t* out_shape) {
  int st;
  if ((st = check_tensor(x, false)) != TC_OK) return st;
  if ((st = check_tensor(k, false)) != TC_OK) return st;
  if (!out_shape) return TC_EINVAL;
  if (conv_dtypes_ok(x->dtype, k->dtype) < 0) return TC_EDTYPE;
  int64_t off[TC_MAX_DIMS];
  return conv_geometry(x, k, mode, out_shape, off);
}

namespace {

// Validation shared by the direct entry points; fills the output geometry.
int conv_validate(const tc_tensor* x, const tc_tensor* k, int32_t mode, const tc_tensor* y, int64_t* off) {
  int st;
  if ((st = check_tensor(x, true)) != TC_OK) return st;
  if ((st = check_tensor(k, true)) != TC_OK) return st;
  if ((st = check_tensor(y, true)) != TC_OK) return st;
  const int ydt = conv_dtypes_ok(x->dtype, k->dtype);
  if (ydt < 0 || y->dtype != ydt) return TC_EDTYPE;
  if (!is_contiguous(k)) return TC_ESHAPE;
  if (numel(k) > (1LL << 20)) return TC_EINVAL;
  int64_t oshape[TC_MAX_DIMS];
  if ((st = conv_geometry(x, k, mode, oshape, off)) != TC_OK) return st;
  if (y->ndim != x->ndim) return TC_ESHAPE;
  for (int d = 0; d < y->ndim; ++d)
    if (y->shape[d] != oshape[d]) return TC_ESHAPE;
  return TC_OK;
}

// The direct kernels.  For an integer kernel, k_abs_sum = sum |k| as stated by
// the caller: the int32 result is exact when 255 * sum|k| <= 2^31 - 1 (every
// partial sum then fits), and 24-bit multiplies are exact when sum|k| < 2^23.
int conv_direct(const tc_tensor* x, const tc_tensor* k, const tc_tensor* y, const int64_t* off, int64_t k_abs_sum,
                int band_rows, hipStream_t s) {
  bool small_taps = true;
  if (k->dtype == TC_I32) {
    if (k_abs_sum < 0) return TC_EINVAL;
    if (k_abs_sum > 2147483647LL / 255) return TC_EOVERFLOW;
    small_taps = k_abs_sum < (1LL << 23);
  }
  if (numel(y) == 0) return TC_OK;
  // zero-size x: the result is all zeros in full/same mode (a fill kernel, so
  // that the call stays safe to record into a HIP graph)
  if (numel(x) == 0 || numel(k) == 0) {
    if (is_contiguous(y)) return hip_status(launch_fill_zero(y->data, (size_t)numel(y) * 4, s));
    return TC_ESHAPE;
  }
  ConvND c{};
  c.ndim = x->ndim;
  c.xdt = x->dtype;
  c.x = x->data;
  c.k = k->data;
  c.y = y->data;
  for (int d = 0; d < c.ndim; ++d) {
    c.xshape[d] = x->shape[d];
    c.xstride[d] = x->stride[d];
    c.kshape[d] = k->shape[d];
    c.yshape[d] = y->shape[d];
    c.ystride[d] = y->stride[d];
    c.off[d] = off[d];
  }
  c.band_rows = band_rows;
  return hip_status(launch_conv(c, small_taps, s));
}

}  // namespace

extern "C" int tc_conv_nd(const tc_tensor* x, const tc_tensor* k, int32_t mode, const tc_tensor* y, void* stream) {
  int64_t off[TC_MAX_DIMS];
  int st;
  if ((st = conv_validate(x, k, mode, y, off)) != TC_OK) return st;
  // the exactness bound of an integer kernel is a host-side fact the caller
  // states through tc_conv_nd_ex; this entry point never reads the taps back
  if (k->dtype == TC_I32) return TC_EINVAL;
  return conv_direct(x, k, y, off, -1, 0, reinterpret_cast<hipStream_t>(stream));
}

// ============================================================================ separable kernels
extern "C" int tc_conv_kernel_rank1(const float* k, int32_t KH, int32_t KW, double tol, float* u, float* v) {
  if (!k || !u || !v || KH < 1 || KW < 1 || KH > 4096 || KW > 4096 || !(tol >= 0.0)) return TC_EINVAL;
  // pivot: the entry of largest magnitude; u = its column, v = its row over it
  int p = 0, q = 0;
  double kmax = 0.0;
  for (int a = 0; a < KH; ++a)
    for (int b = 0; b < KW; ++b) {
      const double m = std::fabs((double)k[(size_t)a * KW + b]);
      if (!(m <= kmax)) {
        if (!std::isfinite(m)) return 0;
        kmax = m;
        p = a;
        q = b;
      }
    }
  if (kmax == 0.0) {
    for (int a = 0; a < KH; ++a) u[a] = 0.f;
    for (int b = 0; b < KW; ++b) v[b] = 0.f;
    return 1;
  }
  const double piv = (double)k[(size_t)p * KW + q];
  const double sc = std::sqrt(std::fabs(piv));  // balance the two factors' magnitudes
  for (int a = 0; a < KH; ++a) u[a] = (float)((double)k[(size_t)a * KW + q] / sc);
  for (int b = 0; b < KW; ++b) v[b] = (float)((double)k[(size_t)p * KW + b] * sc / piv);
  for (int a = 0; a < KH; ++a)
    for (int b = 0; b < KW; ++b)
      if (std::fabs((double)k[(size_t)a * KW + b] - (double)u[a] * (double)v[b]) > tol * kmax) return 0;
  return 1;
}

namespace {

// x (*) (u v^T) for a K x K separable kernel whose factors `tp` carries.
int conv_separable(const tc_tensor* x, int K, const SepTaps& tp, int32_t mode, const tc_tensor* y, hipStream_t s) {
  if (!separable_variant(K)) return TC_EINVAL;
  if (x->dtype != TC_F32 || y->dtype != TC_F32) return TC_EDTYPE;
  if (x->ndim != 2 || y->ndim != 2) return TC_ESHAPE;
  if (x->stride[1] != 1 || y->stride[1] != 1) return TC_ESHAPE;
  // the geometry of the equivalent K x K kernel
  tc_tensor kv{};
  kv.dtype = TC_F32;
  kv.ndim = 2;
  kv.shape[0] = K;
  kv.shape[1] = K;
  kv.stride[0] = K;
  kv.stride[1] = 1;
  int64_t oshape[TC_MAX_DIMS], off[TC_MAX_DIMS];
  int st;
  if ((st = conv_geometry(x, &kv, mode, oshape, off)) != TC_OK) return st;
  if (y->shape[0] != oshape[0] || y->shape[1] != oshape[1]) return TC_ESHAPE;
  if (numel(y) == 0) return TC_OK;
  for (int d = 0; d < 2; ++d)
    if (x->shape[d] >= (1LL << 28) || y->shape[d] >= (1LL << 28) || off[d] >= (1LL << 28)) return TC_EINVAL;
  if (numel(x) == 0) {
    if (y->stride[0] == y->shape[1]) return hip_status(launch_fill_zero(y->data, (size_t)numel(y) * 4, s));
    return TC_ESHAPE;
  }
  SepConv c{};
  c.x = static_cast<const float*>(x->data);
  c.xs0 = x->stride[0];
  c.H = (int)x->shape[0];
  c.W = (int)x->shape[1];
  c.taps = tp;
  c.K = K;
  c.y = static_cast<float*>(y->data);
  c.ys0 = y->stride[0];
  c.OH = (int)y->shape[0];
  c.OW = (int)y->shape[1];
  c.off0 = (int)off[0];
  c.off1 = (int)off[1];
  return hip_status(launch_conv_separable(c, s));
}

}  // namespace

extern "C" int tc_conv_nd_separable(const tc_tensor* x, const tc_tensor* u, const tc_tensor* v, int32_t mode,
                                    const tc_tensor* y, void* stream) {
  int st;
  if ((st = check_tensor(x, true)) != TC_OK) return st;
  if ((st = check_tensor(u, true)) != TC_OK) return st;
  if ((st = check_tensor(v, true)) != TC_OK) return st;
  if ((st = check_tensor(y, true)) != TC_OK) return st;
  if (x->dtype != TC_F32 || u->dtype != TC_F32 || v->dtype != TC_F32 || y->dtype != TC_F32) return TC_EDTYPE;
  if (x->ndim != 2 || y->ndim != 2 || u->ndim != 1 || v->ndim != 1) return TC_ESHAPE;
  if (!is_contiguous(u) || !is_contiguous(v) || u->shape[0] != v->shape[0]) return TC_ESHAPE;
  SepTaps tp{};
  tp.u = static_cast<const float*>(u->data);
  tp.v = static_cast<const float*>(v->data);
  tp.byval = 0;
  return conv_separable(x, (int)u->shape[0], tp, mode, y, reinterpret_cast<hipStream_t>(stream));
}

namespace {

struct FftLayout {
  int rank = 0;
  FftAxis ax[3] = {};
  int64_t volume = 0;  // stored spectrum points: n_0 .. n_{d-2} (n_{d-1} / 2 + 1)
  size_t tw[3] = {0, 0, 0}, A = 0, B = 0, C = 0, total = 0;
  int64_t oshape[TC_MAX_DIMS], off[TC_MAX_DIMS];
};

size_t fft_align(size_t v) { return (v + 255) / 256 * 256; }

// The smallest 2^a 3^b 5^c >= n (n <= kFftMaxN), with its stages: radix 4 while
// two factors of 2 remain, a radix-2 stage for an odd one, then the 3s and 5s.
FftAxis fft_axis(int64_t n) {
  FftAxis ax{};
  for (int64_t m = n < 1 ? 1 : n;; ++m) {
    int64_t r = m;
    int a = 0, b = 0, c = 0;
    while (r % 2 == 0) r /= 2, ++a;
    while (r % 3 == 0) r /= 3, ++b;
    while (r % 5 == 0) r /= 5, ++c;
    if (r != 1) continue;
    ax.n = (int)m;
    int st = 0;
    for (int i = 0; i < a / 2; ++i) ax.radix[st++] = 4;
    if (a % 2) ax.radix[st++] = 2;
    for (int i = 0; i < b; ++i) ax.radix[st++] = 3;
    for (int i = 0; i < c; ++i) ax.radix[st++] = 5;
    ax.n_stages = st;
    return ax;
  }
}

// Every axis but the last is padded to the smallest 2^a 3^b 5^c holding the
// full output; the last (real) axis to twice the smallest such number holding
// half of it, transformed as half as many complex points and stored as its
// n / 2 + 1 non-negative frequencies.
int fft_layout(const tc_tensor* x, const tc_tensor* k, int32_t mode, FftLayout& L) {
  if (x->dtype != TC_F32 || k->dtype != TC_F32) return TC_EDTYPE;
  if (x->ndim != k->ndim || (x->ndim != 2 && x->ndim != 3)) return TC_ESHAPE;
  int st;
  if ((st = conv_geometry(x, k, mode, L.oshape, L.off)) != TC_OK) return st;
  L.rank = (int)x->ndim;
  L.volume = 1;
  int64_t ext_min = INT64_MAX;
  size_t tw_n[3];
  for (int a = 0; a < L.rank; ++a) {
    const int64_t full = x->shape[a] + k->shape[a] - 1;
    const bool last = a == L.rank - 1;
    L.ax[a] = fft_axis(last ? (full + 1) / 2 : full);
    const int64_t padded = last ? 2 * (int64_t)L.ax[a].n : L.ax[a].n;
    if (padded > kFftMaxN) return TC_ESHAPE;
    const int64_t ext = last ? L.ax[a].n + 1 : L.ax[a].n;
    L.volume *= ext;
    ext_min = std::min(ext_min, ext);
    tw_n[a] = (size_t)padded;
  }
  // one work-group per row at most: at most 2^31 - 1 rows along any axis
  if (L.volume / ext_min > INT32_MAX) return TC_ESHAPE;
  size_t o = 0;
  for (int a = 0; a < L.rank; ++a) {
    L.tw[a] = o;
    o += fft_align(tw_n[a] * sizeof(float2));
  }
  const size_t vol = fft_align((size_t)L.volume * sizeof(float2));
  L.A = o;
  L.B = o + vol;
  L.C = o + 2 * vol;
  L.total = o + 3 * vol;
  return TC_OK;
}

int conv_fft(const tc_tensor* x, const tc_tensor* k, int32_t mode, const tc_tensor* y, void* ws, size_t ws_bytes,
             void* stream) {
  int st;
  if ((st = check_tensor(x, true)) != TC_OK) return st;
  if ((st = check_tensor(k, true)) != TC_OK) return st;
  if ((st = check_tensor(y, true)) != TC_OK) return st;
  if (y->dtype != TC_F32) return TC_EDTYPE;
  FftLayout L;
  if ((st = fft_layout(x, k, mode, L)) != TC_OK) return st;
  if (!is_contiguous(k) || y->ndim != x->ndim) return TC_ESHAPE;
  for (int a = 0; a < L.rank; ++a)
    if (y->shape[a] != L.oshape[a]) return TC_ESHAPE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (numel(y) == 0) return TC_OK;
  if (numel(x) == 0 || numel(k) == 0) {
    if (is_contiguous(y)) return hip_status(launch_fill_zero(y->data, (size_t)numel(y) * 4, s));
    return TC_ESHAPE;
  }
  if (!ws) return TC_EINVAL;
  if (ws_bytes < L.total) return TC_ENOMEM;
  char* w = static_cast<char*>(ws);
  FftConv f{};
  f.rank = L.rank;
  f.x = static_cast<const float*>(x->data);
  f.k = static_cast<const float*>(k->data);
  f.y = static_cast<float*>(y->data);
  for (int a = 0; a < L.rank; ++a) {
    f.xs[a] = x->stride[a];
    f.xn[a] = (int)x->shape[a];
    f.kn[a] = (int)k->shape[a];
    f.ax[a] = L.ax[a];
    f.tw[a] = reinterpret_cast<float2*>(w + L.tw[a]);
    f.ys[a] = y->stride[a];
    f.yn[a] = (int)y->shape[a];
    f.o[a] = (int)L.off[a];
  }
  f.A = reinterpret_cast<float2*>(w + L.A);
  f.B = reinterpret_cast<float2*>(w + L.B);
  f.C = reinterpret_cast<float2*>(w + L.C);
  return hip_status(launch_conv_fft(f, s));
}

}  // namespace

extern "C" int tc_conv_fft_workspace_size(const tc_tensor* x, const tc_tensor* k, int32_t mode, size_t* ws_bytes) {
  if (!x || !k || !ws_bytes) return TC_EINVAL;
  int st;
  if ((st = check_tensor(x, false)) != TC_OK) return st;
  if ((st = check_tensor(k, false)) != TC_OK) return st;
  FftLayout L;
  if ((st = fft_layout(x, k, mode, L)) != TC_OK) return st;
  *ws_bytes = L.total;
  return TC_OK;
}

extern "C" int tc_conv_fft(const tc_tensor* x, const tc_tensor* k, int32_t mode, const tc_tensor* y, void* ws,
                           size_t ws_bytes, void* stream) {
  if (!x || !k || !y) return TC_EINVAL;
  return conv_fft(x, k, mode, y, ws, ws_bytes, stream);
}

extern "C" int tc_conv2d_fft_workspace_size(const tc_tensor* x, const tc_tensor* k, int32_t mode, size_t* ws_bytes) {
  if (!x || !k || !ws_bytes) return TC_EINVAL;
  if (x->ndim != 2 || k->ndim != 2) return TC_ESHAPE;
  return tc_conv_fft_workspace_size(x, k, mode, ws_bytes);
}

extern "C" int tc_conv2d_fft(const tc_tensor* x, const tc_tensor* k, int32_t mode, const tc_tensor* y, void* ws,
                             size_t ws_bytes, void* stream) {
  if (!x || !k || !y) return TC_EINVAL;
  if (x->ndim != 2 || k->ndim != 2) return TC_ESHAPE;
  return conv_fft(x, k, mode, y, ws, ws_bytes, stream);
}

// ============================================================================ dispatcher
namespace {

// The kernel side from which the FFT branch beats the direct kernels on
// MI355X (FP32, full mode, cubic kernels): 2048 x 2048 images, and 3-D
// volumes of 64 x 256 x 256.
constexpr int kFftThreshold2D = 19;
constexpr int kFftThreshold3D = 9;
// Relative tolerance of the rank-one test the dispatcher applies to a host copy
// of a square FP32 kernel (max |k - u v^T| <= tol * max |k|).
constexpr double kSeparableTol = 0x1p-20;

bool fft_eligible(const tc_tensor* x, const tc_tensor* k, int32_t mode, FftLayout& L) {
  return fft_layout(x, k, mode, L) == TC_OK;
}

}  // namespace

extern "C" int tc_conv_workspace_size(const tc_tensor* x, const tc_tensor* k, int32_t mode, int32_t method,
                                      size_t* ws_bytes) {
  if (!x || !k || !ws_bytes) return TC_EINVAL;
  int st;
  if ((st = check_tensor(x, false)) != TC_OK) return st;
  if ((st = check_tensor(k, false)) != TC_OK) return st;
  if (method != TC_CONV_AUTO && method != TC_CONV_DIRECT && method != TC_CONV_FFT) return TC_EINVAL;
  *ws_bytes = 0;
  if (method == TC_CONV_DIRECT) return TC_OK;
  FftLayout L;
  if (fft_eligible(x, k, mode, L)) *ws_bytes = L.total;
  else if (method == TC_CONV_FFT) return fft_layout(x, k, mode, L);
  return TC_OK;
}

extern "C" int tc_conv_nd_ex(const tc_tensor* x, const tc_tensor* k, int32_t mode, const tc_tensor* y,
                             const tc_conv_opts* opts, void* stream) {
  tc_conv_opts o{};
  o.method = TC_CONV_AUTO;
  o.k_abs_sum = -1;
  if (opts) o = *opts;
  if (o.method != TC_CONV_AUTO && o.method != TC_CONV_DIRECT && o.method != TC_CONV_FFT) return TC_EINVAL;
  if (o.fft_threshold < 0) return TC_EINVAL;
  if ((o.band_rows != 0 && o.band_rows != 2 && o.band_rows != 4 && o.band_rows != 8) || o.reserved != 0)
    return TC_EINVAL;
  int64_t off[TC_MAX_DIMS];
  int st;
  if ((st = conv_validate(x, k, mode, y, off)) != TC_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t ktaps = numel(k);

  // what the host copy of the kernel tells (read here, on the host)
  int64_t k_abs_sum = o.k_abs_sum;
  if (k->dtype == TC_I32 && o.k_host && ktaps > 0) {
    const int32_t* kh = static_cast<const int32_t*>(o.k_host);
    int64_t sa = 0;
    for (int64_t i = 0; i < ktaps; ++i) {
      sa += kh[i] < 0 ? -(int64_t)kh[i] : (int64_t)kh[i];
      if (sa > (int64_t)1 << 40) break;  // far past the bound already
    }
    k_abs_sum = sa;
  }
  if (k->dtype == TC_I32 && ktaps == 0) k_abs_sum = 0;
  if (o.method == TC_CONV_FFT || o.method == TC_CONV_AUTO) {
    FftLayout L;
    const bool ok = fft_eligible(x, k, mode, L);
    if (o.method == TC_CONV_FFT && !ok) {
      const int e = fft_layout(x, k, mode, L);
      return e != TC_OK ? e : TC_EINVAL;
    }
    int64_t kmax = 0;
    for (int d = 0; d < k->ndim; ++d) kmax = std::max(kmax, k->shape[d]);
    const int thr = o.fft_threshold > 0 ? o.fft_threshold : (x->ndim == 3 ? kFftThreshold3D : kFftThreshold2D);
    const bool want = o.method == TC_CONV_FFT || (ok && kmax >= thr && o.workspace && o.workspace_bytes >= L.total);
    if (want) return conv_fft(x, k, mode, y, o.workspace, o.workspace_bytes, stream);
  }
  // separable square F32 kernels, when the caller lent a host copy to test:
  // the factors travel by value in the kernel arguments
  if (o.method == TC_CONV_AUTO && o.k_host && x->dtype == TC_F32 && k->dtype == TC_F32 && x->ndim == 2 &&
      k->shape[0] == k->shape[1] && separable_variant((int)k->shape[0]) && x->stride[1] == 1 && y->stride[1] == 1) {
    const int K = (int)k->shape[0];
    SepTaps tp{};
    tp.byval = 1;
    if (tc_conv_kernel_rank1(static_cast<const float*>(o.k_host), K, K, kSeparableTol, tp.uh, tp.vh) == 1)
      return conv_separable(x, K, tp, mode, y, s);
  }
  return conv_direct(x, k, y, off, k_abs_sum, o.band_rows, s);
}

// ============================================================================ pyramid / derivatives
extern "C" int tc_pyramid_shape(int64_t H, int64_t W, int32_t level, int64_t* Hl, int64_t* Wl) {
  if (H < 0 || W < 0 || level < 0 || level > 62 || !Hl || !Wl) return TC_EINVAL;
  *Hl = H >> level;
  *Wl = W >> level;
  return TC_OK;
}

extern "C" int tc_image_pyramid(const tc_tensor* frame, int32_t levels, const tc_tensor* out, void* stream) {
  int st;
  if ((st = check_tensor(frame, true)) != TC_OK) return st;
  if (frame->ndim != 2) return TC_ESHAPE;
  if (frame->dtype != TC_U8 && frame->dtype != TC_F16 && frame->dtype != TC_F32) return TC_EDTYPE;
  if (levels < 1 || levels > 16) return TC_EINVAL;
  const int64_t H = frame->shape[0], W = frame->shape[1];
  if ((H >> (levels - 1)) < 1 || (W >> (levels - 1)) < 1) return TC_ESHAPE;
  if (H > (1LL << 24) || W > (1LL << 24)) return TC_ESHAPE;
  if (levels > 1 && !out) return TC_EINVAL;
  for (int l = 1; l < levels; ++l) {
    const tc_tensor* o = &out[l - 1];
    if ((st = check_tensor(o, true)) != TC_OK) return st;
    if (o->ndim != 2 || o->dtype != TC_F32) return o->dtype != TC_F32 ? TC_EDTYPE : TC_ESHAPE;
    if (o->shape[0] != (H >> l) || o->shape[1] != (W >> l)) return TC_ESHAPE;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Image2D src{frame->data, frame->dtype, frame->stride[0], frame->stride[1]};
  for (int l = 1; l < levels; ++l) {
    const tc_tensor* o = &out[l - 1];
    hipError_t e = launch_pyramid_level(src, reinterpret_cast<float*>(o->data), o->stride[0], o->stride[1],
                                        (int)o->shape[0], (int)o->shape[1], s);
    if (e != hipSuccess) return TC_EDEVICE;
    src = Image2D{o->data, TC_F32, o->stride[0], o->stride[1]};
  }
  return TC_OK;
}

extern "C" int tc_horn_derivs(const tc_tensor* prev, const tc_tensor* next, const tc_tensor* ex, const tc_tensor* ey,
                              const tc_tensor* et, void* stream) {
  int st;
  const tc_tensor* ins[2] = {prev, next};
  const tc_tensor* outs[3] = {ex, ey, et};
  for (auto t : ins) {
    if ((st = check_tensor(t, true)) != TC_OK) return st;
    if (t->ndim != 2) return TC_ESHAPE;
  }
  if (prev->dtype != next->dtype) return TC_EDTYPE;
  if (prev->dtype != TC_U8 && prev->dtype != TC_F16 && prev->dtype != TC_F32) return TC_EDTYPE;
  if (prev->shape[0] != next->shape[0] || prev->shape[1] != next->shape[1]) return TC_ESHAPE;
  const int64_t H = prev->shape[0], W = prev->shape[1];
  if (H < 2 || W < 2 || H > (1LL << 24) || W > (1LL << 24)) return TC_ESHAPE;
  const int odt = ex ? ex->dtype : -1;
  for (auto t : outs) {
    if ((st = check_tensor(t, true)) != TC_OK) return st;
    if (t->ndim != 2) return TC_ESHAPE;
    if (t->dtype != odt) return TC_EDTYPE;
    if (t->shape[0] != H - 1 || t->shape[1] != W - 1) return TC_ESHAPE;
  }
  if (odt != TC_F32 && odt != TC_I32) return TC_EDTYPE;
  if (odt == TC_I32 && prev->dtype != TC_U8) return TC_EDTYPE;
  const int64_t os0[3] = {ex->stride[0], ey->stride[0], et->stride[0]};
  const int64_t os1[3] = {ex->stride[1], ey->stride[1], et->stride[1]};
  Image2D a{prev->data, prev->dtype, prev->stride[0], prev->stride[1]};
  Image2D b{next->data, next->dtype, next->stride[0], next->stride[1]};
  return hip_status(launch_horn(a, b, (int)H, (int)W, ex->data, ey->data, et->data, odt, os0, os1,
                                reinterpret_cast<hipStream_t>(stream)));
}

extern "C" int tc_gradient(const tc_tensor* image, int32_t stencil, const tc_tensor* ex, const tc_tensor* ey,
                           const tc_tensor* mag, const tc_tensor* dir, void* stream) {
  int st;
  if ((st = check_tensor(image, true)) != TC_OK) return st;
  if (image->ndim != 2) return TC_ESHAPE;
  if (image->dtype != TC_U8 && image->dtype != TC_F16 && image->dtype != TC_F32) return TC_EDTYPE;
  if (stencil < TC_STENCIL_FD2 || stencil > TC_STENCIL_SOBEL3) return TC_EINVAL;
  const int k = stencil >= TC_STENCIL_PREWITT3 ? 3 : 2;
  const int64_t H = image->shape[0], W = image->shape[1];
  if (H > (1LL << 24) || W > (1LL << 24)) return TC_ESHAPE;
  const int64_t Ho = H >= k ? H - k + 1 : 0, Wo = W >= k ? W - k + 1 : 0;
  const tc_tensor* outs[4] = {ex, ey, mag, dir};
  float* ptr[4];
  int64_t s0[4], s1[4];
  for (int q = 0; q < 4; ++q) {
    const tc_tensor* t = outs[q];
    ptr[q] = nullptr;
    s0[q] = s1[q] = 0;
    if (!t || !t->data) continue;
    if ((st = check_tensor(t, true)) != TC_OK) return st;
    if (t->ndim != 2) return TC_ESHAPE;
    if (t->dtype != TC_F32) return TC_EDTYPE;
    if (t->shape[0] != Ho || t->shape[1] != Wo) return TC_ESHAPE;
    ptr[q] = reinterpret_cast<float*>(t->data);
    s0[q] = t->stride[0];
    s1[q] = t->stride[1];
  }
  const GradOut o{ptr[0], s0[0], s1[0], ptr[1], s0[1], s1[1], ptr[2], s0[2], s1[2], ptr[3], s0[3], s1[3]};
  if (!o.ex && !o.ey && !o.mag && !o.dir) return TC_OK;
  const Image2D src{image->data, image->dtype, image->stride[0], image->stride[1]};
  return hip_status(launch_gradient(src, stencil, (int)Ho, (int)Wo, o, reinterpret_cast<hipStream_t>(stream)));
}

extern "C" int tc_ttc_reselect(const tc_ttc_level* levels, int64_t n_pairs, int32_t levels_per_pair, int32_t rule,
                               tc_ttc_pick* picks_out, void* stream) {
  if (n_pairs < 0 || levels_per_pair < 1 || levels_per_pair > 16) return TC_EINVAL;
  if (rule != TC_SELECT_DECREASING_TTC && rule != TC_SELECT_MIN_RESIDUAL) return TC_EINVAL;
  if (n_pairs > (1LL << 40)) return TC_EINVAL;
  if (n_pairs == 0) return TC_OK;
  if (!levels || !picks_out) return TC_EINVAL;
  return hip_status(launch_ttc_reselect(levels, n_pairs, levels_per_pair, rule, picks_out,
                                        reinterpret_cast<hipStream_t>(stream)));
}

// ============================================================================ time to contact
struct tc_ttc_plan {
  int dtype = 0;
  int levels = 0;
  int band_rows = 0;
  int groups_per_cu = 0;
  size_t capacity = 0;  // bytes the pinned table buffer holds
  int n_seqs = 0;
  int64_t n_items = 0;
  int64_t n_pairs = 0;
  int64_t n_partial_floats = 0;
  size_t table_bytes = 0;
  size_t ws_bytes = 0;
  int grid = 0;
  size_t item_index_off = 0;  // byte offsets of the item -> stream and pair -> stream
  size_t pair_index_off = 0;  // index arrays inside the table region
  SeqDesc* table = nullptr;   // pinned host copy of the table region
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Built-in launch shape (band rows, work-groups per CU) per frame type and level
// count: the best of the fused pass's tuning sweep (autotune.py) on MI355X,
// f16 on the 64-stream batched workload, u8 on a 64-stream serving mix.  More
// work-groups than items means one item per work-group, dispatched by the
// hardware.  With column strips packed per wave every case is best at 128 rows
// x 128 work-groups per CU (the runner-up within 0.1-4%); 160-row bands, outside
// the sweep, measured within 1% of 128 on f16 at 4 levels.
tc_ttc_tuning default_tuning(int dtype, int levels) {
  static const tc_ttc_tuning f16[TC_MAX_LEVELS] = {{128, 128}, {128, 128}, {128, 128}, {128, 128}};
  static const tc_ttc_tuning u8[TC_MAX_LEVELS] = {{128, 128}, {128, 128}, {128, 128}, {128, 128}};
  const int l = levels < 1 ? 0 : (levels > TC_MAX_LEVELS ? TC_MAX_LEVELS - 1 : levels - 1);
  return dtype == TC_U8 ? u8[l] : f16[l];
}

// One frame pair per call (tc_ttc_solve): the shortest band, so that a single
// pair still spreads over many waves.
constexpr tc_ttc_tuning kPairTuning = {16, 32};

bool tuning_ok(const tc_ttc_tuning& t, int dtype, int levels) {
  return t.groups_per_cu >= 1 && t.groups_per_cu <= 256 && fused_variant_exists(dtype, levels, t.band_rows);
}

int validate_seq(const tc_seq& q, int dtype, int levels) {
  const int es = elem_size(dtype);
  if (!q.frame0) return TC_EINVAL;
  if (q.levels != levels) return TC_EINVAL;
  if (q.n_frames < 2) return TC_EINVAL;
  if (q.H < 2 || q.W < 2 || q.H > (1 << 20) || q.W > (1 << 20)) return TC_ESHAPE;
  if ((q.H >> (levels - 1)) < 2 || (q.W >> (levels - 1)) < 2) return TC_ESHAPE;
  if (q.row_stride < q.W) return TC_ESHAPE;
  if (reinterpret_cast<uintptr_t>(q.frame0) % (uintptr_t)es) return TC_EINVAL;
  return TC_OK;
}

// 8-pixel lane chunks start at multiples of 8 pixels; they can be fetched with
// one 8-byte (u8) or 16-byte (f16) load when frames and rows keep that alignment.
int vector_ok(const tc_seq& q, int dtype) {
  const int es = elem_size(dtype);
  const int64_t align = 8 * es;
  return (reinterpret_cast<uintptr_t>(q.frame0) % (uintptr_t)align) == 0 && (q.row_stride * es) % align == 0 &&
         (q.frame_stride * es) % align == 0;
}

// Column strips of the fused pass: owned base columns per segment (a multiple
// of 8, so that a lane's 8 columns are one level-3 column) with one lending lane
// each, as many segments as fit in a wave.  Narrow strips let frames narrower
// than a wave, and the last strip of a wider one, share a wave's lanes between
// bands instead of leaving them idle.
struct SegShape {
  int cols, lanes, per_wave;
};
constexpr SegShape kSegShapes[] = {{504, 64, 1}, {248, 32, 2}, {160, 21, 3}, {120, 16, 4}};

// The segment shape with the fewest waves per pair (every wave walks the same
// rows); among equals the widest, which has the fewest lending lanes and partials.
void choose_segments(SeqDesc& d) {
  int64_t best = INT64_MAX;
  for (const SegShape& g : kSegShapes) {
    const int64_t strips = (d.W - 1 + g.cols - 1) / g.cols;  // W - 1 cube columns at level 0
    const int64_t segs = strips * d.n_bands;
    const int64_t waves = (segs + g.per_wave - 1) / g.per_wave;
    if (waves < best) {
      best = waves;
      d.seg_cols = g.cols;
      d.seg_lanes = g.lanes;
      d.seg_per_wave = g.per_wave;
      d.n_segs = (int32_t)segs;
      d.n_waves = (int32_t)waves;
      d.n_strips = (int32_t)strips;
    }
  }
  // band b walks rows b RB .. b RB + RB + halo - 1 and needs row b RB + RB + halo
  const int64_t walk = (int64_t)d.band_rows + (1 << (d.levels - 1));
  const int64_t full = d.H - walk - 1 >= 0 ? (d.H - walk - 1) / d.band_rows + 1 : 0;
  d.n_full_bands = (int32_t)std::min<int64_t>(full, d.n_bands);
}

void fill_desc(SeqDesc& d, const tc_seq& q, int dtype, int band_rows) {
  d.frame0 = q.frame0;
  d.frame_stride = q.frame_stride;
  d.row_stride = q.row_stride;
  d.H = q.H;
  d.W = q.W;
  d.n_frames = q.n_frames;
  d.levels = q.levels;
  d.band_rows = band_rows;
  d.n_bands = (q.H + band_rows - 1) / band_rows;
  choose_segments(d);
  d.vec = vector_ok(q, dtype);
}

int persistent_grid(int64_t n_items, int groups_per_cu) {
  const int n_cu = current_cu_count();
  int64_t g = std::min<int64_t>(n_items, (int64_t)n_cu * groups_per_cu);
  if (g >= 8) g -= g % 8;
  return (int)std::max<int64_t>(g, 1);
}

}  // namespace

// (Re)builds the plan's table region for `seqs` in its pinned buffer:
// [SeqDesc per stream | int32 stream of every work item | int32 stream of
// every pair], each part 256-byte aligned, so that a work item or a pair finds
// its stream with one load.
static int plan_fill(tc_ttc_plan* p, const tc_seq* seqs, int32_t n_seqs) {
  std::vector<SeqDesc> descs((size_t)n_seqs);
  int64_t items = 0, pairs = 0, floats = 0;
  for (int i = 0; i < n_seqs; ++i) {
    SeqDesc& d = descs[(size_t)i];
    memset(&d, 0, sizeof d);
    fill_desc(d, seqs[i], p->dtype, p->band_rows);
    d.item_begin = items;
    d.pair_begin = pairs;
    d.partial_begin = floats;
    items += (int64_t)d.n_waves * (d.n_frames - 1);  // one work item per (wave of segments, pair)
    pairs += d.n_frames - 1;
    floats += (int64_t)(d.n_frames - 1) * p->levels * d.n_segs * 10;
  }
  if (items > INT32_MAX || pairs > INT32_MAX) return TC_EINVAL;
  const size_t desc_bytes = align_up(sizeof(SeqDesc) * (size_t)n_seqs);
  const size_t item_bytes = align_up(sizeof(int32_t) * (size_t)items);
  const size_t pair_bytes = align_up(sizeof(int32_t) * (size_t)pairs);
  const size_t bytes = desc_bytes + item_bytes + pair_bytes;
  if (bytes > p->capacity) {
    if (p->table) (void)hipHostFree(p->table);
    p->table = nullptr;
    p->capacity = 0;
    if (hipHostMalloc(reinterpret_cast<void**>(&p->table), bytes, hipHostMallocDefault) != hipSuccess) {
      p->table = nullptr;
      return TC_EDEVICE;
    }
    p->capacity = bytes;
  }
  char* base = reinterpret_cast<char*>(p->table);
  memcpy(base, descs.data(), sizeof(SeqDesc) * (size_t)n_seqs);
  int32_t* item_seq = reinterpret_cast<int32_t*>(base + desc_bytes);
  int32_t* pair_seq = reinterpret_cast<int32_t*>(base + desc_bytes + item_bytes);
  for (int i = 0; i < n_seqs; ++i) {
    const SeqDesc& d = descs[(size_t)i];
    for (int64_t k = 0; k < (int64_t)d.n_waves * (d.n_frames - 1); ++k) item_seq[d.item_begin + k] = i;
    for (int64_t k = 0; k < d.n_frames - 1; ++k) pair_seq[d.pair_begin + k] = i;
  }
  p->n_seqs = n_seqs;
  p->item_index_off = desc_bytes;
  p->pair_index_off = desc_bytes + item_bytes;
  p->table_bytes = bytes;
  p->n_items = items;
  p->n_pairs = pairs;
  p->n_partial_floats = floats;
  p->ws_bytes = p->table_bytes + align_up((size_t)floats * sizeof(float));
  p->grid = persistent_grid(items, p->groups_per_cu);
  return TC_OK;
}

extern "C" int tc_ttc_plan_reset(tc_ttc_plan* plan, const tc_seq* seqs, int32_t n_seqs) {
  if (!plan || !seqs || n_seqs < 1 || n_seqs > (1 << 20)) return TC_EINVAL;
  for (int i = 0; i < n_seqs; ++i) {
    const int st = validate_seq(seqs[i], plan->dtype, plan->levels);
    if (st != TC_OK) return st;
  }
  return plan_fill(plan, seqs, n_seqs);
}

extern "C" int tc_ttc_tuning_default(int32_t dtype, int32_t levels, tc_ttc_tuning* out) {
  if (!out || levels < 1 || levels > TC_MAX_LEVELS) return TC_EINVAL;
  if (dtype != TC_U8 && dtype != TC_F16) return TC_EDTYPE;
  *out = default_tuning(dtype, levels);
  return TC_OK;
}

extern "C" int tc_ttc_plan_create_ex(const tc_seq* seqs, int32_t n_seqs, int32_t dtype, const tc_ttc_tuning* tuning,
                                     tc_ttc_plan** plan) {
  if (!plan) return TC_EINVAL;
  *plan = nullptr;
  if (!seqs || n_seqs < 1 || n_seqs > (1 << 20)) return TC_EINVAL;
  if (dtype != TC_U8 && dtype != TC_F16) return TC_EDTYPE;
  const int levels = seqs[0].levels;
  if (levels < 1 || levels > TC_MAX_LEVELS) return TC_EINVAL;
  for (int i = 0; i < n_seqs; ++i) {
    const int st = validate_seq(seqs[i], dtype, levels);
    if (st != TC_OK) return st;
  }
  const tc_ttc_tuning tn = tuning ? *tuning : default_tuning(dtype, levels);
  if (!tuning_ok(tn, dtype, levels)) return TC_EINVAL;
  const int rh = tn.band_rows;

  tc_ttc_plan* p = new (std::nothrow) tc_ttc_plan();
  if (!p) return TC_ENOMEM;
  p->dtype = dtype;
  p->levels = levels;
  p->band_rows = rh;
  p->groups_per_cu = tn.groups_per_cu;
  const int st = plan_fill(p, seqs, n_seqs);
  if (st != TC_OK) {
    tc_ttc_plan_destroy(p);
    return st;
  }
  *plan = p;
  return TC_OK;
}

extern "C" int tc_ttc_plan_create(const tc_seq* seqs, int32_t n_seqs, int32_t dtype, tc_ttc_plan** plan) {
  return tc_ttc_plan_create_ex(seqs, n_seqs, dtype, nullptr, plan);
}

extern "C" int tc_ttc_plan_info(const tc_ttc_plan* plan, size_t* ws_bytes, int64_t* n_pairs,
                                int64_t* n_level_records) {
  if (!plan) return TC_EINVAL;
  if (ws_bytes) *ws_bytes = plan->ws_bytes;
  if (n_pairs) *n_pairs = plan->n_pairs;
  if (n_level_records) *n_level_records = plan->n_pairs * plan->levels;
  return TC_OK;
}

extern "C" int tc_ttc_plan_upload(const tc_ttc_plan* plan, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || !ws) return TC_EINVAL;
  if (ws_bytes < plan->ws_bytes) return TC_ENOMEM;
  return hip_status(hipMemcpyAsync(ws, plan->table, plan->table_bytes, hipMemcpyHostToDevice,
                                   reinterpret_cast<hipStream_t>(stream)));
}

extern "C" int tc_ttc_plan_run_phase(const tc_ttc_plan* plan, void* ws, size_t ws_bytes, tc_ttc_level* levels_out,
                                     tc_ttc_pick* picks_out, int32_t phase, void* stream) {
  if (!plan || !ws || phase < 1 || phase > 3) return TC_EINVAL;
  if ((phase & TC_PHASE_FINISH) && (!levels_out || !picks_out)) return TC_EINVAL;
  if (ws_bytes < plan->ws_bytes) return TC_ENOMEM;
  FusedLaunch f{};
  f.dt = plan->dtype;
  f.levels = plan->levels;
  f.band_rows = plan->band_rows;
  f.table = reinterpret_cast<const SeqDesc*>(ws);
  f.item_seq = reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(ws) + plan->item_index_off);
  f.pair_seq = reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(ws) + plan->pair_index_off);
  f.n_seqs = plan->n_seqs;
  f.n_items = plan->n_items;
  f.n_pairs = plan->n_pairs;
  f.partials = reinterpret_cast<float*>(reinterpret_cast<char*>(ws) + plan->table_bytes);
  f.grid = plan->grid;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if ((phase & TC_PHASE_FUSED) && launch_ttc_fused(f, s) != hipSuccess) return TC_EDEVICE;
  if ((phase & TC_PHASE_FINISH) && launch_ttc_finish(f, levels_out, picks_out, s) != hipSuccess) return TC_EDEVICE;
  return TC_OK;
}

extern "C" int tc_ttc_plan_run(const tc_ttc_plan* plan, void* ws, size_t ws_bytes, tc_ttc_level* levels_out,
                               tc_ttc_pick* picks_out, void* stream) {
  return tc_ttc_plan_run_phase(plan, ws, ws_bytes, levels_out, picks_out, TC_PHASE_FUSED | TC_PHASE_FINISH, stream);
}

extern "C" void tc_ttc_plan_destroy(tc_ttc_plan* plan) {
  if (!plan) return;
  if (plan->table) {
    (void)hipDeviceSynchronize();
    (void)hipHostFree(plan->table);
  }
  delete plan;
}

extern "C" int tc_ttc_solve_batched(const tc_seq* seqs, int32_t n_seqs, int32_t dtype, void* ws, size_t ws_bytes,
                                    tc_ttc_level* levels_out, tc_ttc_pick* picks_out, void* stream) {
  tc_ttc_plan* p = nullptr;
  int st = tc_ttc_plan_create(seqs, n_seqs, dtype, &p);
  if (st != TC_OK) return st;
  st = tc_ttc_plan_upload(p, ws, ws_bytes, stream);
  if (st == TC_OK) st = tc_ttc_plan_run(p, ws, ws_bytes, levels_out, picks_out, stream);
  if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess && st == TC_OK) st = TC_EDEVICE;
  tc_ttc_plan_destroy(p);
  return st;
}

namespace {

int pair_desc(const tc_tensor* prev, const tc_tensor* next, int32_t levels, SeqDesc& d) {
  int st;
  if ((st = check_tensor(prev, true)) != TC_OK) return st;
  if ((st = check_tensor(next, true)) != TC_OK) return st;
  if (prev->ndim != 2 || next->ndim != 2) return TC_ESHAPE;
  if (prev->dtype != next->dtype) return TC_EDTYPE;
  if (prev->dtype != TC_U8 && prev->dtype != TC_F16) return TC_EDTYPE;
  if (prev->shape[0] != next->shape[0] || prev->shape[1] != next->shape[1]) return TC_ESHAPE;
  if (prev->stride[1] != 1 || next->stride[1] != 1 || prev->stride[0] != next->stride[0]) return TC_ESHAPE;
  if (levels < 1 || levels > TC_MAX_LEVELS) return TC_EINVAL;
  if (prev->shape[0] > (1 << 20) || prev->shape[1] > (1 << 20)) return TC_ESHAPE;
  const int es = elem_size(prev->dtype);
  const int64_t diff = reinterpret_cast<const char*>(next->data) - reinterpret_cast<const char*>(prev->data);
  if (diff % es) return TC_EINVAL;
  tc_seq q;
  q.frame0 = prev->data;
  q.frame_stride = diff / es;
  q.row_stride = prev->stride[0];
  q.H = (int32_t)prev->shape[0];
  q.W = (int32_t)prev->shape[1];
  q.n_frames = 2;
  q.levels = levels;
  if ((st = validate_seq(q, prev->dtype, levels)) != TC_OK) return st;
  fill_desc(d, q, prev->dtype, kPairTuning.band_rows);
  d.item_begin = 0;
  d.pair_begin = 0;
  d.partial_begin = 0;
  return TC_OK;
}

size_t pair_ws_bytes(const SeqDesc& d) { return align_up((size_t)d.levels * d.n_segs * 10 * sizeof(float)); }

}  // namespace

extern "C" int tc_ttc_workspace_size(int64_t H, int64_t W, int32_t levels, size_t* ws_bytes) {
  if (!ws_bytes || H < 2 || W < 2 || H > (1 << 20) || W > (1 << 20) || levels < 1 || levels > TC_MAX_LEVELS)
    return TC_EINVAL;
  size_t best = 0;
  const int dts[2] = {TC_U8, TC_F16};
  for (int dt : dts) {
    tc_seq q{};
    q.H = (int32_t)H;
    q.W = (int32_t)W;
    q.n_frames = 2;
    q.levels = levels;
    // every band height a tuning may use (segment shapes depend on it)
    for (int rb = 16; rb <= 256; rb += 16) {
      SeqDesc d{};
      fill_desc(d, q, dt, rb);
      best = std::max(best, pair_ws_bytes(d));
    }
  }
  *ws_bytes = best;
  return TC_OK;
}

namespace {

// Workspace of the decomposed path: level images 1..levels-1 of both frames
// (FP32, contiguous), one block-mean image for the low-pass filter to read,
// and the per-block partial sums of every level.
struct VariantLayout {
  int64_t Hl[TC_MAX_LEVELS], Wl[TC_MAX_LEVELS];
  size_t level_off[2][TC_MAX_LEVELS];
  size_t tmp_off[2] = {0, 0}, part_off = 0, total = 0;
  VariantLevels lv{};
};

int variant_layout(int64_t H, int64_t W, int32_t levels, int32_t stencil, int32_t lowpass, VariantLayout& L) {
  if (levels < 1 || levels > TC_MAX_LEVELS) return TC_EINVAL;
  if (stencil != TC_STENCIL_FD2 && stencil != TC_STENCIL_PREWITT3 && stencil != TC_STENCIL_SOBEL3) return TC_EINVAL;
  if (lowpass != TC_LOWPASS_NONE && lowpass != TC_LOWPASS_BINOMIAL3) return TC_EINVAL;
  if (H < 1 || W < 1 || H > (1 << 20) || W > (1 << 20)) return TC_ESHAPE;
  const int k = stencil == TC_STENCIL_FD2 ? 2 : 3;
  int64_t parts = 0;
  L.lv.levels = levels;
  for (int l = 0; l < levels; ++l) {
    L.Hl[l] = H >> l;
    L.Wl[l] = W >> l;
    if (L.Hl[l] < k || L.Wl[l] < k) return TC_ESHAPE;
    const int64_t n = (L.Hl[l] - k + 1) * (L.Wl[l] - k + 1);
    L.lv.n[l] = n;
    L.lv.blocks[l] = variant_sum_blocks(n);
    L.lv.part_off[l] = parts;
    parts += L.lv.blocks[l];
  }
  size_t off = 0;
  for (int f = 0; f < 2; ++f)
    for (int l = 1; l < levels; ++l) {
      L.level_off[f][l] = off;
      off += align_up((size_t)(L.Hl[l] * L.Wl[l]) * sizeof(float));
    }
  // the block means before the low-pass, both frames
  for (int f = 0; f < 2; ++f) {
    L.tmp_off[f] = off;
    if (lowpass == TC_LOWPASS_BINOMIAL3 && levels > 1) off += align_up((size_t)(L.Hl[1] * L.Wl[1]) * sizeof(float));
  }
  L.part_off = off;
  off += align_up((size_t)parts * 10 * sizeof(double));
  L.total = off;
  return TC_OK;
}

}  // namespace

extern "C" int tc_ttc_variant_workspace_size(int64_t H, int64_t W, int32_t levels, int32_t stencil, int32_t lowpass,
                                             size_t* ws_bytes) {
  if (!ws_bytes) return TC_EINVAL;
  VariantLayout L;
  const int st = variant_layout(H, W, levels, stencil, lowpass, L);
  if (st != TC_OK) return st;
  *ws_bytes = L.total;
  return TC_OK;
}

extern "C" int tc_ttc_solve_variant(const tc_tensor* prev, const tc_tensor* next, int32_t levels, int32_t stencil,
                                    int32_t lowpass, void* ws, size_t ws_bytes, tc_ttc_level* levels_out,
                                    tc_ttc_pick* pick_out, void* stream) {
  int st;
  if (!ws || !levels_out || !pick_out) return TC_EINVAL;
  if ((st = check_tensor(prev, true)) != TC_OK) return st;
  if ((st = check_tensor(next, true)) != TC_OK) return st;
  if (prev->ndim != 2 || next->ndim != 2) return TC_ESHAPE;
  if (prev->dtype != next->dtype) return TC_EDTYPE;
  if (prev->dtype != TC_U8 && prev->dtype != TC_F16 && prev->dtype != TC_F32) return TC_EDTYPE;
  if (prev->shape[0] != next->shape[0] || prev->shape[1] != next->shape[1]) return TC_ESHAPE;
  const int64_t H = prev->shape[0], W = prev->shape[1];
  VariantLayout L;
  if ((st = variant_layout(H, W, levels, stencil, lowpass, L)) != TC_OK) return st;
  if (ws_bytes < L.total) return TC_ENOMEM;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  double* part = reinterpret_cast<double*>(w + L.part_off);
  // both frames' levels (one launch per level and step), then every level's
  // sums in one launch
  VariantSumLevels ls{};
  VariantPlanes2 cur{{prev->data, next->data}, {prev->stride[0], next->stride[0]}, {prev->stride[1], next->stride[1]}};
  int cur_dt = prev->dtype;
  for (int l = 0; l < levels; ++l) {
    const int Hl = (int)L.Hl[l], Wl = (int)L.Wl[l];
    if (l > 0) {
      VariantPair2 io{};
      for (int f = 0; f < 2; ++f) io.dst[f] = reinterpret_cast<float*>(w + L.level_off[f][l]);
      if (lowpass == TC_LOWPASS_BINOMIAL3) {
        VariantPair2 blk{};
        for (int f = 0; f < 2; ++f) blk.dst[f] = reinterpret_cast<float*>(w + L.tmp_off[f]);
        if (launch_pyramid_pair(cur, cur_dt, blk, Hl, Wl, s) != hipSuccess) return TC_EDEVICE;
        for (int f = 0; f < 2; ++f) io.src[f] = blk.dst[f];
        if (launch_lowpass3_pair(io, Hl, Wl, s) != hipSuccess) return TC_EDEVICE;
      } else if (launch_pyramid_pair(cur, cur_dt, io, Hl, Wl, s) != hipSuccess) {
        return TC_EDEVICE;
      }
      for (int f = 0; f < 2; ++f) {
        cur.p[f] = io.dst[f];
        cur.s0[f] = Wl;
        cur.s1[f] = 1;
      }
      cur_dt = TC_F32;
    }
    ls.a[l] = cur.p[0];
    ls.b[l] = cur.p[1];
    for (int f = 0; f < 2; ++f) {
      ls.s0[f][l] = cur.s0[f];
      ls.s1[f][l] = cur.s1[f];
    }
    ls.Hl[l] = Hl;
    ls.Wl[l] = Wl;
    ls.blocks[l] = L.lv.blocks[l];
    ls.part_off[l] = L.lv.part_off[l];
  }
  if (launch_stencil_sums_levels(stencil, prev->dtype, ls, levels, (int)H, (int)W, part, s) != hipSuccess)
    return TC_EDEVICE;
  return hip_status(launch_variant_finish(part, L.lv, levels_out, pick_out, s));
}

extern "C" int tc_ttc_solve(const tc_tensor* prev, const tc_tensor* next, int32_t levels, void* ws, size_t ws_bytes,
                            tc_ttc_level* levels_out, tc_ttc_pick* pick_out, void* stream) {
  if (!ws || !levels_out || !pick_out) return TC_EINVAL;
  SeqDesc d{};
  int st = pair_desc(prev, next, levels, d);
  if (st != TC_OK) return st;
  if (ws_bytes < pair_ws_bytes(d)) return TC_ENOMEM;
  FusedLaunch f{};
  f.dt = prev->dtype;
  f.levels = levels;
  f.band_rows = d.band_rows;
  f.table = nullptr;
  f.n_seqs = 1;
  f.inl = d;
  f.n_items = d.n_waves;
  f.n_pairs = 1;
  f.partials = reinterpret_cast<float*>(ws);
  f.grid = persistent_grid(f.n_items, kPairTuning.groups_per_cu);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (launch_ttc_fused(f, s) != hipSuccess) return TC_EDEVICE;
  if (launch_ttc_finish(f, levels_out, pick_out, s) != hipSuccess) return TC_EDEVICE;
  return TC_OK;
}
