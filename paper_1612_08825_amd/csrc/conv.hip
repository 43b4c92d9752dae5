// Direct n-D convolution for gfx950.
//
// y[n] = sum_t k[t] * x[n + off - t]  (true convolution; `off` selects the
// output mode: 0 for full, (K-1)/2 for same, min(N,K)-1 for valid), with x read
// as zero outside its extent.  Two kernels:
//   * conv2d_tiled: a 256-thread work-group stages a (64 + KH - 1) x (64 + KW - 1)
//     input tile in LDS (zero-filled at the borders) and every thread keeps a
//     4 x 4 block of outputs in registers; taps are read with scalar loads.
//     For rank 3 the grid's z dimension is the output plane, and the kernel
//     loops over the kernel's planes, re-staging the matching input plane.
//   * conv_generic: one thread per output element of any rank <= 8.
// Taps are visited in kernel-row-major order for every output element.
#include "device_common.hpp"
#include "internal.hpp"

namespace ttc {
namespace {

constexpr int kTX = 16, kTY = 16;   // threads per work-group (x, y)
constexpr int kRX = 4, kRY = 4;     // outputs per thread (x, y)
constexpr int kTileX = kTX * kRX;   // 64 output columns per work-group
constexpr int kTileY = kTY * kRY;   // 64 output rows per work-group

template <typename TX> struct Acc { using type = float; };
template <> struct Acc<uint8_t> { using type = int; };

template <typename TA> __device__ __forceinline__ TA mac(TA acc, TA k, TA v);
template <> __device__ __forceinline__ float mac<float>(float acc, float k, float v) { return fmaf(k, v, acc); }
// u8 pixels times taps of magnitude < 2^23: the 24-bit multiply is exact.
template <> __device__ __forceinline__ int mac<int>(int acc, int k, int v) { return acc + __mul24(k, v); }

// Full 32-bit products, for the generic kernel (taps of any int32 magnitude).
template <typename TA> __device__ __forceinline__ TA mac_full(TA acc, TA k, TA v) { return mac<TA>(acc, k, v); }
template <> __device__ __forceinline__ int mac_full<int>(int acc, int k, int v) { return acc + k * v; }

template <typename TX> __device__ __forceinline__ typename Acc<TX>::type load_x(const TX* x, int64_t i) {
  return (typename Acc<TX>::type)x[i];
}
template <> __device__ __forceinline__ float load_x<_Float16>(const _Float16* x, int64_t i) { return (float)x[i]; }

template <typename TA> __device__ __forceinline__ TA load_k(const void* k, int i) {
  return reinterpret_cast<const TA*>(k)[i];
}

struct Tile2D {
  const void* x;
  int64_t xs0, xs1;
  int H, W;
  const void* k;
  int KH, KW;
  void* y;
  int64_t ys0, ys1;
  int OH, OW;
  int off0, off1;
  // 3-D extension (plane dimension); D == 1 and KD == 1 for plain 2-D.
  int64_t xsd, ysd;
  int D, KD, OD, offd;
};

// Stage the input tile whose top-left corner is (r0, c0) of plane `xp`.
template <typename TX, int PITCH>
__device__ __forceinline__ void stage_tile(typename Acc<TX>::type* lds, const TX* xp, const Tile2D& a, int r0, int c0,
                                           int rows, int cols) {
  using TA = typename Acc<TX>::type;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int lr = ty; lr < rows; lr += kTY) {
    const int gr = r0 + lr;
    const bool rin = (gr >= 0) && (gr < a.H);
    for (int lc = tx; lc < cols; lc += kTX) {
      const int gc = c0 + lc;
      TA v = (TA)0;
      if (rin && gc >= 0 && gc < a.W) v = load_x<TX>(xp, (int64_t)gr * a.xs0 + (int64_t)gc * a.xs1);
      lds[lr * PITCH + lc] = v;
    }
  }
}

// acc += sum over taps of kernel plane `kp` of the staged tile.
template <typename TA, int KWMAX, int PITCH>
__device__ __forceinline__ void tile_fma(TA (&acc)[kRY][kRX], const TA* lds, const void* k, int kp_off, int KH,
                                         int KW) {
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int ky = 0; ky < KH; ++ky) {
    TA kt[KWMAX];
#pragma unroll
    for (int kx = 0; kx < KWMAX; ++kx) kt[kx] = (kx < KW) ? load_k<TA>(k, kp_off + ky * KW + kx) : (TA)0;
#pragma unroll
    for (int ry = 0; ry < kRY; ++ry) {
      const TA* row = lds + (ty * kRY + ry + (KH - 1 - ky)) * PITCH + tx * kRX;
      TA v[kRX + KWMAX - 1];
#pragma unroll
      for (int c = 0; c < kRX + KWMAX - 1; ++c) v[c] = row[c];
#pragma unroll
      for (int kx = 0; kx < KWMAX; ++kx) {
        if (kx < KW) {
#pragma unroll
          for (int rx = 0; rx < kRX; ++rx) acc[ry][rx] = mac<TA>(acc[ry][rx], kt[kx], v[rx + KW - 1 - kx]);
        }
      }
    }
  }
}

template <typename TX, int KWMAX>
__global__ __launch_bounds__(256) void conv2d_tiled(Tile2D a) {
  using TA = typename Acc<TX>::type;
  constexpr int PITCH = ((kTileX + KWMAX - 1 + 3) / 4) * 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TA* lds = reinterpret_cast<TA*>(smem_raw);

  const int o0 = blockIdx.y * kTileY;
  const int p0 = blockIdx.x * kTileX;
  const int od = blockIdx.z;  // output plane (0 for 2-D)
  const int rows = kTileY + a.KH - 1;
  const int cols = kTileX + a.KW - 1;
  const int r0 = o0 + a.off0 - (a.KH - 1);
  const int c0 = p0 + a.off1 - (a.KW - 1);

  TA acc[kRY][kRX];
#pragma unroll
  for (int i = 0; i < kRY; ++i)
#pragma unroll
    for (int j = 0; j < kRX; ++j) acc[i][j] = (TA)0;

  const TX* x = reinterpret_cast<const TX*>(a.x);
  const int nd = od + a.offd;  // full plane index
  for (int kd = 0; kd < a.KD; ++kd) {
    const int xd = nd - kd;
    if (xd < 0 || xd >= a.D) continue;  // uniform across the work-group
    __syncthreads();
    stage_tile<TX, PITCH>(lds, x + (int64_t)xd * a.xsd, a, r0, c0, rows, cols);
    __syncthreads();
    tile_fma<TA, KWMAX, PITCH>(acc, lds, a.k, kd * a.KH * a.KW, a.KH, a.KW);
  }

  TA* y = reinterpret_cast<TA*>(a.y) + (int64_t)od * a.ysd;
#pragma unroll
  for (int ry = 0; ry < kRY; ++ry) {
    const int o = o0 + threadIdx.y * kRY + ry;
    if (o >= a.OH) continue;
#pragma unroll
    for (int rx = 0; rx < kRX; ++rx) {
      const int p = p0 + threadIdx.x * kRX + rx;
      if (p < a.OW) y[(int64_t)o * a.ys0 + (int64_t)p * a.ys1] = acc[ry][rx];
    }
  }
}

struct GenericArgs {
  int ndim;
  const void* x;
  int64_t xshape[TC_MAX_DIMS];
  int64_t xstride[TC_MAX_DIMS];
  const void* k;
  int64_t kshape[TC_MAX_DIMS];
  void* y;
  int64_t yshape[TC_MAX_DIMS];
  int64_t ystride[TC_MAX_DIMS];
  int64_t off[TC_MAX_DIMS];
  int64_t n_out;
  int64_t n_taps;
};

template <typename TX>
__global__ __launch_bounds__(256) void conv_generic(GenericArgs a) {
  using TA = typename Acc<TX>::type;
  const TX* x = reinterpret_cast<const TX*>(a.x);
  const TA* k = reinterpret_cast<const TA*>(a.k);
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < a.n_out;
       o += (int64_t)gridDim.x * blockDim.x) {
    // output coordinates, then full-result coordinates
    int64_t nf[TC_MAX_DIMS];
    int64_t rem = o, yoff = 0;
    for (int d = a.ndim - 1; d >= 0; --d) {
      const int64_t c = rem % a.yshape[d];
      rem /= a.yshape[d];
      yoff += c * a.ystride[d];
      nf[d] = c + a.off[d];
    }
    // walk the taps in row-major order with a multi-index counter
    int64_t t[TC_MAX_DIMS];
    for (int d = 0; d < a.ndim; ++d) t[d] = 0;
    TA acc = (TA)0;
    for (int64_t ti = 0; ti < a.n_taps; ++ti) {
      bool in = true;
      int64_t xoff = 0;
      for (int d = 0; d < a.ndim; ++d) {
        const int64_t xc = nf[d] - t[d];
        in = in && (xc >= 0) && (xc < a.xshape[d]);
        xoff += xc * a.xstride[d];
      }
      if (in) acc = mac_full<TA>(acc, k[ti], load_x<TX>(x, xoff));
      for (int d = a.ndim - 1; d >= 0; --d) {
        if (++t[d] < a.kshape[d]) break;
        t[d] = 0;
      }
    }
    reinterpret_cast<TA*>(a.y)[yoff] = acc;
  }
}

template <typename TX>
hipError_t launch_tiled_t(const Tile2D& t, int kwmax, dim3 grid, hipStream_t s) {
  using TA = typename Acc<TX>::type;
  const dim3 block(kTX, kTY, 1);
  auto go = [&](auto kern, int pitch) {
    const size_t lds = (size_t)(kTileY + t.KH - 1) * pitch * sizeof(TA);
    hipLaunchKernelGGL(kern, grid, block, lds, s, t);
    return hipGetLastError();
  };
  switch (kwmax) {
    case 4: return go(conv2d_tiled<TX, 4>, ((kTileX + 4 - 1 + 3) / 4) * 4);
    case 8: return go(conv2d_tiled<TX, 8>, ((kTileX + 8 - 1 + 3) / 4) * 4);
    case 16: return go(conv2d_tiled<TX, 16>, ((kTileX + 16 - 1 + 3) / 4) * 4);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tiled(int xdt, const Tile2D& t, int kwmax, dim3 grid, hipStream_t s) {
  switch (xdt) {
    case TC_F32: return launch_tiled_t<float>(t, kwmax, grid, s);
    case TC_F16: return launch_tiled_t<_Float16>(t, kwmax, grid, s);
    case TC_U8: return launch_tiled_t<uint8_t>(t, kwmax, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_conv(const ConvND& c, bool small_taps, hipStream_t s) {
  int64_t n_out = 1, n_taps = 1;
  for (int d = 0; d < c.ndim; ++d) {
    n_out *= c.yshape[d];
    n_taps *= c.kshape[d];
  }
  if (n_out == 0) return hipSuccess;

  // 2-D and 3-D: the LDS-tiled kernels, for kernel rows up to 16 taps and
  // kernel heights that keep the staged tile within 64 KiB of LDS.
  const int r = c.ndim;
  const bool tiled_ok = (r == 2 || r == 3) && small_taps && c.kshape[r - 1] <= 16 && c.kshape[r - 2] <= 64 &&
                        c.xshape[r - 1] < (1LL << 30) && c.xshape[r - 2] < (1LL << 30) &&
                        c.yshape[r - 1] < (1LL << 30) && c.yshape[r - 2] < (1LL << 30) &&
                        c.off[r - 1] < (1LL << 30) && c.off[r - 2] < (1LL << 30) &&
                        (r == 2 || (c.xshape[0] < (1LL << 30) && c.yshape[0] < 65536 && c.kshape[0] < (1LL << 20)));
  if (tiled_ok) {
    Tile2D t{};
    t.x = c.x;
    t.xs0 = c.xstride[r - 2];
    t.xs1 = c.xstride[r - 1];
    t.H = (int)c.xshape[r - 2];
    t.W = (int)c.xshape[r - 1];
    t.k = c.k;
    t.KH = (int)c.kshape[r - 2];
    t.KW = (int)c.kshape[r - 1];
    t.y = c.y;
    t.ys0 = c.ystride[r - 2];
    t.ys1 = c.ystride[r - 1];
    t.OH = (int)c.yshape[r - 2];
    t.OW = (int)c.yshape[r - 1];
    t.off0 = (int)c.off[r - 2];
    t.off1 = (int)c.off[r - 1];
    if (r == 3) {
      t.xsd = c.xstride[0];
      t.ysd = c.ystride[0];
      t.D = (int)c.xshape[0];
      t.KD = (int)c.kshape[0];
      t.OD = (int)c.yshape[0];
      t.offd = (int)c.off[0];
    } else {
      t.xsd = 0;
      t.ysd = 0;
      t.D = 1;
      t.KD = 1;
      t.OD = 1;
      t.offd = 0;
    }
    const int kwmax = t.KW <= 4 ? 4 : (t.KW <= 8 ? 8 : 16);
    const dim3 grid((unsigned)((t.OW + kTileX - 1) / kTileX), (unsigned)((t.OH + kTileY - 1) / kTileY),
                    (unsigned)t.OD);
    return launch_tiled(c.xdt, t, kwmax, grid, s);
  }

  GenericArgs g{};
  g.ndim = c.ndim;
  g.x = c.x;
  g.k = c.k;
  g.y = c.y;
  for (int d = 0; d < c.ndim; ++d) {
    g.xshape[d] = c.xshape[d];
    g.xstride[d] = c.xstride[d];
    g.kshape[d] = c.kshape[d];
    g.yshape[d] = c.yshape[d];
    g.ystride[d] = c.ystride[d];
    g.off[d] = c.off[d];
  }
  g.n_out = n_out;
  g.n_taps = n_taps;
  const int64_t blocks64 = (n_out + 255) / 256;
  const unsigned blocks = (unsigned)(blocks64 < 65536 ? blocks64 : 65536);
  switch (c.xdt) {
    case TC_F32: hipLaunchKernelGGL(conv_generic<float>, dim3(blocks), dim3(256), 0, s, g); break;
    case TC_F16: hipLaunchKernelGGL(conv_generic<_Float16>, dim3(blocks), dim3(256), 0, s, g); break;
    case TC_U8: hipLaunchKernelGGL(conv_generic<uint8_t>, dim3(blocks), dim3(256), 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ttc
