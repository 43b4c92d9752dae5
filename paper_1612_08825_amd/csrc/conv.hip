// Direct n-D convolution for gfx950.
//
// y[n] = sum_t k[t] * x[n + off - t]  (true convolution; `off` selects the
// output mode: 0 for full, (K-1)/2 for same, min(N,K)-1 for valid), with x read
// as zero outside its extent.  Three kernels:
//   * conv2d_rows (FP32, contiguous rows, square kernels of 2, 3, 5 or 7
//     taps): one wave per band of output rows, each input row loaded once per
//     wave straight into registers (one 16-byte load per lane, windows
//     assembled across lanes with DPP); described where it is defined.
//   * conv2d_tiled: a 256-thread work-group stages a (64 + KH - 1) x (64 + KW - 1)
//     input tile in LDS (zero-filled at the borders) and every thread keeps a
//     4 x 4 block of outputs in registers; taps are read with scalar loads.
//     For rank 3 the grid's z dimension is the output plane, and the kernel
//     loops over the kernel's planes, re-staging the matching input plane.
//   * conv_generic: one thread per output element of any rank <= 8.
// The generic kernel visits taps in kernel-row-major order for every output
// element, the tiled kernel kernel rows first to last and the taps within a
// row last to first; conv2d_rows visits tap rows from last to first.
#include <algorithm>
#include <type_traits>

#include "conv_common.hpp"
#include "device_common.hpp"
#include "internal.hpp"

namespace ttc {
namespace {

using namespace rows;

constexpr int kTX = 16, kTY = 16;   // threads per work-group (x, y)
constexpr int kRX = 4, kRY = 4;     // outputs per thread (x, y)
constexpr int kTileX = kTX * kRX;   // 64 output columns per work-group
constexpr int kTileY = kTY * kRY;   // 64 output rows per work-group
constexpr int kKernelBlock = 64;     // largest kernel extent one tiled launch takes

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

template <typename TA> __device__ __forceinline__ TA load_k(const void* k, int64_t i) {
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
  // the taps: k[kd * ksd + ky * ks0 + kx] (a block of a larger kernel when
  // ks0 > KW); accumulate: add into y instead of writing it
  int ks0;
  int64_t ksd;
  int accumulate;
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
__device__ __forceinline__ void tile_fma(TA (&acc)[kRY][kRX], const TA* lds, const void* k, int64_t kp_off, int KH,
                                         int KW, int ks0) {
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int ky = 0; ky < KH; ++ky) {
    // the taps of kernel row ky from last to first, kt[j] = k[ky][KW - 1 - j],
    // so that output column rx meets input column rx + j of the window (a
    // static register index for every j)
    TA kt[KWMAX];
#pragma unroll
    for (int j = 0; j < KWMAX; ++j) kt[j] = (j < KW) ? load_k<TA>(k, kp_off + (int64_t)ky * ks0 + (KW - 1 - j)) : (TA)0;
#pragma unroll
    for (int ry = 0; ry < kRY; ++ry) {
      const TA* row = lds + (ty * kRY + ry + (KH - 1 - ky)) * PITCH + tx * kRX;
      TA v[kRX + KWMAX - 1];
#pragma unroll
      for (int c = 0; c < kRX + KWMAX - 1; ++c) v[c] = row[c];
#pragma unroll
      for (int j = 0; j < KWMAX; ++j) {
        if (j < KW) {
#pragma unroll
          for (int rx = 0; rx < kRX; ++rx) acc[ry][rx] = mac<TA>(acc[ry][rx], kt[j], v[rx + j]);
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

  // tiles of output rows in steps of the grid's y extent (at most 65535)
  const int n_ty = (a.OH + kTileY - 1) / kTileY;
  for (int tile_y = blockIdx.y; tile_y < n_ty; tile_y += gridDim.y) {
    const int o0 = tile_y * kTileY;
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
      tile_fma<TA, KWMAX, PITCH>(acc, lds, a.k, kd * a.ksd, a.KH, a.KW, a.ks0);
    }

    TA* y = reinterpret_cast<TA*>(a.y) + (int64_t)od * a.ysd;
#pragma unroll
    for (int ry = 0; ry < kRY; ++ry) {
      const int o = o0 + threadIdx.y * kRY + ry;
      if (o >= a.OH) continue;
#pragma unroll
      for (int rx = 0; rx < kRX; ++rx) {
        const int p = p0 + threadIdx.x * kRX + rx;
        if (p < a.OW) {
          TA& out = y[(int64_t)o * a.ys0 + (int64_t)p * a.ys1];
          out = a.accumulate ? out + acc[ry][rx] : acc[ry][rx];
        }
      }
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
    case 32: return go(conv2d_tiled<TX, 32>, ((kTileX + 32 - 1 + 3) / 4) * 4);
    case 48: return go(conv2d_tiled<TX, 48>, ((kTileX + 48 - 1 + 3) / 4) * 4);
    case 64: return go(conv2d_tiled<TX, 64>, ((kTileX + 64 - 1 + 3) / 4) * 4);
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

// ---------------------------------------------------------------- row-streaming f32 kernel
// FP32 images whose rows are contiguous, for the common kernel sizes (KH and
// KW compile-time).  One wave per item: a band of R (8, or 4 for small
// outputs) output rows by 4 * LO
// output columns of one output plane; lane i < LO holds output columns
// 4i .. 4i+3 of the band in registers.  The wave walks the band's R + KH - 1
// input rows top to bottom and multiplies each into every output row of the
// band it reaches; taps are wave-uniform and come through the scalar cache.
//
// Loads are what bounds this kernel (each vector-memory instruction costs the
// texture addresser about the same whatever its width), so an input row costs
// one 16-byte load per lane: lane i loads 4 consecutive columns ("its chunk"),
// and the KW + 3 columns a lane needs (its window) are its chunk and the chunks
// of the next NC - 1 lanes, moved across the wave with DPP.  The last NC - 1
// lanes only load: their windows would reach past the wave, so LO = 65 - NC.
// The window of lane i starts S columns into its chunk (S = 0..3 is the same
// for every lane and row of a launch and is a template parameter).
//
// In waves whose chunks may leave the image, a lane whose chunk lies wholly
// outside loads nothing, and a lane whose chunk straddles the edge loads it one
// column at a time with buffer loads through a resource limited to the row,
// which read zero left and right of the image; bands whose rows may leave the
// image skip those rows.
// Large square kernels (15 x 15): the unrolled band of conv2d_rows would need
// all KH * KW taps live in scalar registers at once.  Here the band's input
// rows are a runtime loop with a rolling window of KH accumulator rows: at
// input row t, accumulator u holds band output row t - (KH - 1) + u, which
// takes tap row u; after the row, accumulator 0 is complete, is stored, and
// the window moves down one row.  Each input row is loaded once per wave (the
// same chunk + DPP scheme as conv2d_rows, one row ahead) and multiplied into
// all KH rows of the window; the taps are re-read from the scalar cache every
// row (an empty asm keeps the compiler from holding all of them).  Window rows
// outside the band or the output are not updated, so a band of RB rows costs
// RB * KH * KW multiply-adds per lane column, as the convolution itself.
template <int KH, int KW, int RB, int S>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void conv2d_rows_roll(RowArgs a) {
  constexpr int NC = row_chunks<KW, S>();
  constexpr int LO = row_lanes_out<KW, S>();
  constexpr int NW = KW + 3;
  const int lane = threadIdx.x;
  const int64_t G = gridDim.x, g = blockIdx.x;
  const int64_t item = (G % 8 == 0) ? (g % 8) * (G / 8) + g / 8 : g;
  if (item >= a.n_items) return;
  const int64_t per_plane = (int64_t)a.n_bands * a.n_cw;
  const int od = (int)(item / per_plane);
  const int rem = (int)(item - (int64_t)od * per_plane);
  const int band = rem / a.n_cw;
  const int cw = rem - band * a.n_cw;
  const int o0 = band * RB;
  const int p_wave = cw * 4 * LO;
  const int p_lane = p_wave + 4 * lane;
  const int chunk0 = p_wave + a.off1 - (KW - 1) - S;
  const int cc = chunk0 + 4 * lane;  // first column of this lane's chunk
  const bool chunk_in = cc >= 0 && cc + 4 <= a.W;
  const uint32_t row_bytes = (uint32_t)a.W * 4u;
  const int i0 = o0 + a.off0 - (KH - 1);
  const int n_out = RB < a.OH - o0 ? RB : a.OH - o0;  // band rows inside the output
  const int n_rows = n_out + KH - 1;
  const gptr<float> yp = as_global(static_cast<float*>(a.y)) + (int64_t)od * a.ysd;
  const bool store_lane = lane < LO;

  // only one kernel plane per output plane is supported here (2-D)
  const float* plane = static_cast<const float*>(a.x);
  cptr<float> taps = (cptr<float>)(static_cast<const float*>(a.k));

  auto load_chunk = [&](int row, float (&c4)[4]) {
    if (row < 0 || row >= a.H) {  // uniform
      c4[0] = c4[1] = c4[2] = c4[3] = 0.f;
      return;
    }
    const float* rp = plane + (int64_t)row * a.xs0;
    if (chunk_in) {
      const f4u v = *(const __attribute__((address_space(1))) f4u*)(rp + cc);
      c4[0] = v.x;
      c4[1] = v.y;
      c4[2] = v.z;
      c4[3] = v.w;
    } else if (cc >= a.W || cc + 4 <= 0) {
      c4[0] = c4[1] = c4[2] = c4[3] = 0.f;  // wholly outside: no load
    } else {
      const __amdgpu_buffer_rsrc_t rs = make_rsrc(rp, row_bytes);
#pragma unroll
      for (int d = 0; d < 4; ++d)
        c4[d] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (uint32_t)(cc + d) * 4u, 0, 0));
    }
  };

  float acc[KH][4];
#pragma unroll
  for (int u = 0; u < KH; ++u)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[u][c] = 0.f;

  float nxt[4];
  load_chunk(i0, nxt);
  for (int t = 0; t < n_rows; ++t) {
    float ch[4 * NC];
#pragma unroll
    for (int d = 0; d < 4; ++d) ch[d] = nxt[d];
    if (t + 1 < n_rows) load_chunk(i0 + t + 1, nxt);
#pragma unroll
    for (int k = 1; k < NC; ++k)
#pragma unroll
      for (int d = 0; d < 4; ++d) ch[4 * k + d] = from_next_lane(ch[4 * (k - 1) + d]);
    float w[NW];
#pragma unroll
    for (int e = 0; e < NW; ++e) w[e] = ch[S + e];
    asm volatile("" : "+s"(taps));
    // accumulator u is band output row t - (KH - 1) + u: only rows inside the
    // band and the image are worth updating (uniform bounds)
    const int u_lo = (KH - 1 - t) > 0 ? KH - 1 - t : 0;
    const int j_top = (RB < a.OH - o0 ? RB : a.OH - o0) - 1;  // last band row to produce
    const int u_hi = j_top + (KH - 1) - t;
#pragma unroll
    for (int u = 0; u < KH; ++u) {
      if (u < u_lo || u > u_hi) continue;
#pragma unroll
      for (int b = 0; b < KW; ++b) {
        const float kv = taps[u * KW + b];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[u][c] = fmaf(kv, w[c + KW - 1 - b], acc[u][c]);
      }
    }
    // accumulator 0 is band output row t - (KH - 1)
    const int j = t - (KH - 1);
    const int o = o0 + j;
    if (j >= 0 && o < a.OH && store_lane) {
      const gptr<float> yr = yp + (int64_t)o * a.ys0 + p_lane;
      if (p_lane + 3 < a.OW) {
        f4u v;
        v.x = acc[0][0];
        v.y = acc[0][1];
        v.z = acc[0][2];
        v.w = acc[0][3];
        *(__attribute__((address_space(1))) f4u*)yr = v;
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (p_lane + c < a.OW) yr[c] = acc[0][c];
      }
    }
#pragma unroll
    for (int u = 0; u + 1 < KH; ++u)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[u][c] = acc[u + 1][c];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[KH - 1][c] = 0.f;
  }
}

template <int KH, int KW, int RB, int S>
hipError_t launch_roll_s(RowArgs ra, hipStream_t s) {
  constexpr int LO = row_lanes_out<KW, S>();
  ra.n_bands = (ra.OH + RB - 1) / RB;
  ra.n_cw = (ra.OW + 4 * LO - 1) / (4 * LO);
  ra.n_items = (int64_t)ra.OD * ra.n_bands * ra.n_cw;
  const int64_t grid = (ra.n_items + 7) / 8 * 8;
  hipLaunchKernelGGL((conv2d_rows_roll<KH, KW, RB, S>), dim3((unsigned)grid), dim3(64), 0, s, ra);
  return hipGetLastError();
}

template <int KH, int KW, int RB>
hipError_t launch_roll_t(const RowArgs& ra, hipStream_t s) {
  switch ((((ra.off1 - (KW - 1)) % 4) + 4) % 4) {
    case 0: return launch_roll_s<KH, KW, RB, 0>(ra, s);
    case 1: return launch_roll_s<KH, KW, RB, 1>(ra, s);
    case 2: return launch_roll_s<KH, KW, RB, 2>(ra, s);
    default: return launch_roll_s<KH, KW, RB, 3>(ra, s);
  }
}

// Separable kernels k[a][b] = u[a] v[b] (Future Work section: directional
// derivatives, Gaussians, block averages).  The rolling-window walk of
// conv2d_rows_roll with the two factors applied in turn: each input row is
// first convolved along the row with v (K multiply-adds per output column),
// then the K rows of the window take that row times u[a].  2K multiply-adds
// per output instead of K^2, and no intermediate image.
template <int K, int RB, int S>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void conv2d_rows_sep(RowArgs a,
                                                                                             SepTaps tp) {
  constexpr int NC = row_chunks<K, S>();
  constexpr int LO = row_lanes_out<K, S>();
  constexpr int NW = K + 3;
  const int lane = threadIdx.x;
  const int64_t G = gridDim.x, g = blockIdx.x;
  const int64_t item = (G % 8 == 0) ? (g % 8) * (G / 8) + g / 8 : g;
  if (item >= a.n_items) return;
  const int band = (int)(item / a.n_cw);
  const int cw = (int)(item - (int64_t)band * a.n_cw);
  const int o0 = band * RB;
  const int p_wave = cw * 4 * LO;
  const int p_lane = p_wave + 4 * lane;
  const int chunk0 = p_wave + a.off1 - (K - 1) - S;
  const int cc = chunk0 + 4 * lane;
  const bool chunk_in = cc >= 0 && cc + 4 <= a.W;
  const uint32_t row_bytes = (uint32_t)a.W * 4u;
  const int i0 = o0 + a.off0 - (K - 1);
  const int n_out = RB < a.OH - o0 ? RB : a.OH - o0;
  const int n_rows = n_out + K - 1;
  const gptr<float> yp = as_global(static_cast<float*>(a.y));
  const bool store_lane = lane < LO;
  const cptr<float> u = (cptr<float>)tp.u;
  const cptr<float> v = (cptr<float>)tp.v;

  auto load_chunk = [&](int row, float (&c4)[4]) {
    if (row < 0 || row >= a.H) {  // uniform
      c4[0] = c4[1] = c4[2] = c4[3] = 0.f;
      return;
    }
    const float* rp = static_cast<const float*>(a.x) + (int64_t)row * a.xs0;
    if (chunk_in) {
      const f4u q = *(const __attribute__((address_space(1))) f4u*)(rp + cc);
      c4[0] = q.x;
      c4[1] = q.y;
      c4[2] = q.z;
      c4[3] = q.w;
    } else if (cc >= a.W || cc + 4 <= 0) {
      c4[0] = c4[1] = c4[2] = c4[3] = 0.f;
    } else {
      const __amdgpu_buffer_rsrc_t rs = make_rsrc(rp, row_bytes);
#pragma unroll
      for (int d = 0; d < 4; ++d)
        c4[d] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (uint32_t)(cc + d) * 4u, 0, 0));
    }
  };

  float acc[K][4];
#pragma unroll
  for (int t = 0; t < K; ++t)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[t][c] = 0.f;

  float nxt[4];
  load_chunk(i0, nxt);
  for (int t = 0; t < n_rows; ++t) {
    float ch[4 * NC];
#pragma unroll
    for (int d = 0; d < 4; ++d) ch[d] = nxt[d];
    if (t + 1 < n_rows) load_chunk(i0 + t + 1, nxt);
#pragma unroll
    for (int k = 1; k < NC; ++k)
#pragma unroll
      for (int d = 0; d < 4; ++d) ch[4 * k + d] = from_next_lane(ch[4 * (k - 1) + d]);
    // the row pass: r[c] = sum_b v[b] x[row][col_c - b]
    float r[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < K; ++b) {
      const float vb = tp.byval ? tp.vh[b] : v[b];
#pragma unroll
      for (int c = 0; c < 4; ++c) r[c] = fmaf(vb, ch[S + c + K - 1 - b], r[c]);
    }
    // the column pass: window row w (band output row t - (K - 1) + w) takes u[w]
    const int w_lo = (K - 1 - t) > 0 ? K - 1 - t : 0;
    const int w_hi = (n_out - 1) + (K - 1) - t;
#pragma unroll
    for (int w = 0; w < K; ++w) {
      if (w < w_lo || w > w_hi) continue;
      const float uw = tp.byval ? tp.uh[w] : u[w];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[w][c] = fmaf(uw, r[c], acc[w][c]);
    }
    const int j = t - (K - 1);
    const int o = o0 + j;
    if (j >= 0 && store_lane) {
      const gptr<float> yr = yp + (int64_t)o * a.ys0 + p_lane;
      if (p_lane + 3 < a.OW) {
        f4u q;
        q.x = acc[0][0];
        q.y = acc[0][1];
        q.z = acc[0][2];
        q.w = acc[0][3];
        *(__attribute__((address_space(1))) f4u*)yr = q;
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (p_lane + c < a.OW) yr[c] = acc[0][c];
      }
    }
#pragma unroll
    for (int w = 0; w + 1 < K; ++w)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[w][c] = acc[w + 1][c];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[K - 1][c] = 0.f;
  }
}

template <int K, int RB, int S>
hipError_t launch_sep_s(RowArgs ra, const SepTaps& tp, hipStream_t s) {
  constexpr int LO = row_lanes_out<K, S>();
  ra.n_bands = (ra.OH + RB - 1) / RB;
  ra.n_cw = (ra.OW + 4 * LO - 1) / (4 * LO);
  ra.n_items = (int64_t)ra.n_bands * ra.n_cw;
  const int64_t grid = (ra.n_items + 7) / 8 * 8;
  hipLaunchKernelGGL((conv2d_rows_sep<K, RB, S>), dim3((unsigned)grid), dim3(64), 0, s, ra, tp);
  return hipGetLastError();
}

template <int K, int RB>
hipError_t launch_sep_rb(const RowArgs& ra, const SepTaps& tp, hipStream_t s) {
  switch ((((ra.off1 - (K - 1)) % 4) + 4) % 4) {
    case 0: return launch_sep_s<K, RB, 0>(ra, tp, s);
    case 1: return launch_sep_s<K, RB, 1>(ra, tp, s);
    case 2: return launch_sep_s<K, RB, 2>(ra, tp, s);
    default: return launch_sep_s<K, RB, 3>(ra, tp, s);
  }
}

// Bands of 16 output rows when that still gives about two waves per SIMD
// (2048 items), else 8 (timed on 1024^2 .. 4096^2 images with 7 and 15 taps:
// 16 rows beat 32 by 16% at 4096^2, 8 rows win below; 64 rows lose
// everywhere).  The band height never changes a result.
template <int K>
hipError_t launch_sep_k(const RowArgs& ra, const SepTaps& tp, hipStream_t s) {
  constexpr int LO = row_lanes_out<K, 3>();
  const int64_t items16 = (int64_t)((ra.OH + 15) / 16) * ((ra.OW + 4 * LO - 1) / (4 * LO));
  if (items16 >= 2048) return launch_sep_rb<K, 16>(ra, tp, s);
  return launch_sep_rb<K, 8>(ra, tp, s);
}

// The (KH, KW) pairs the row-streaming kernels are built for (15 x 15 only
// for 2-D FP32: the rolling kernel takes one kernel plane).
bool rows_variant(int KH, int KW, int rank, int xdt) {
  if (KH != KW) return false;
  if (KH == 2 || KH == 3 || KH == 5 || KH == 7) return true;
  return KH == 15 && rank == 2 && xdt == TC_F32;
}

// Items (waves) a band height gives; the band height is the tallest that still
// gives about two waves per SIMD (2048 on 256 CUs), else the shortest.
int64_t row_items(const RowArgs& ra, int rb, int lanes_out) {
  return (int64_t)ra.OD * ((ra.OH + rb - 1) / rb) * ((ra.OW + 4 * lanes_out - 1) / (4 * lanes_out));
}
constexpr int64_t kTargetItems = 2048;

hipError_t launch_rows(const RowArgs& ra, int KH, int xdt, int band_rows, hipStream_t s) {
  if (KH == 15) {
    if (row_items(ra, 32, 59) >= kTargetItems) return launch_roll_t<15, 15, 32>(ra, s);
    if (row_items(ra, 16, 59) >= kTargetItems) return launch_roll_t<15, 15, 16>(ra, s);
    return launch_roll_t<15, 15, 8>(ra, s);
  }
  switch (xdt) {
    case TC_F32: return launch_rows_dt0(ra, KH, band_rows, s);
    case TC_F16: return launch_rows_dt1(ra, KH, band_rows, s);
    case TC_U8: return launch_rows_dt2(ra, KH, band_rows, s);
    default: return hipErrorInvalidValue;
  }
}

__global__ __launch_bounds__(256) void fill_zero_words(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

}  // namespace

bool separable_variant(int K) { return K == 3 || K == 5 || K == 7 || K == 9 || K == 11 || K == 15; }

hipError_t launch_conv_separable(const SepConv& c, hipStream_t s) {
  RowArgs ra{};
  ra.x = c.x;
  ra.xs0 = c.xs0;
  ra.H = c.H;
  ra.W = c.W;
  ra.D = 1;
  ra.KD = 1;
  ra.y = c.y;
  ra.ys0 = c.ys0;
  ra.OH = c.OH;
  ra.OW = c.OW;
  ra.OD = 1;
  ra.off0 = c.off0;
  ra.off1 = c.off1;
  switch (c.K) {
    case 3: return launch_sep_k<3>(ra, c.taps, s);
    case 5: return launch_sep_k<5>(ra, c.taps, s);
    case 7: return launch_sep_k<7>(ra, c.taps, s);
    case 9: return launch_sep_k<9>(ra, c.taps, s);
    case 11: return launch_sep_k<11>(ra, c.taps, s);
    case 15: return launch_sep_k<15>(ra, c.taps, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 4);
  if (n == 0) return hipSuccess;
  const int64_t blocks64 = (n + 255) / 256;
  const unsigned blocks = (unsigned)(blocks64 < 4096 ? blocks64 : 4096);
  hipLaunchKernelGGL(fill_zero_words, dim3(blocks), dim3(256), 0, s, static_cast<uint32_t*>(p), n);
  return hipGetLastError();
}

hipError_t launch_conv(const ConvND& c, bool small_taps, hipStream_t s) {
  int64_t n_out = 1, n_taps = 1;
  for (int d = 0; d < c.ndim; ++d) {
    n_out *= c.yshape[d];
    n_taps *= c.kshape[d];
  }
  if (n_out == 0) return hipSuccess;

  const int r = c.ndim;
  // 2-D and 3-D images with contiguous rows and a common kernel size: the
  // row-streaming kernels (FP32; FP16 and u8 when each row's 4-pixel chunks
  // start on 4-byte boundaries; u8 with 24-bit taps only).
  const int es = c.xdt == TC_F32 ? 4 : (c.xdt == TC_F16 ? 2 : 1);
  const bool chunks_aligned = (reinterpret_cast<uintptr_t>(c.x) % 4 == 0) && ((c.xstride[r - 2] * es) % 4 == 0) &&
                              (r == 2 || (c.xstride[0] * es) % 4 == 0);
  const bool rows_type_ok = c.xdt == TC_F32 || (c.xdt == TC_F16 && chunks_aligned) ||
                            (c.xdt == TC_U8 && chunks_aligned && small_taps);
  if ((r == 2 || r == 3) && rows_type_ok && c.xstride[r - 1] == 1 && c.ystride[r - 1] == 1 &&
      rows_variant((int)c.kshape[r - 2], (int)c.kshape[r - 1], r, c.xdt) && c.xshape[r - 1] < (1LL << 28) &&
      c.xshape[r - 2] < (1LL << 30) && c.yshape[r - 1] < (1LL << 30) && c.yshape[r - 2] < (1LL << 30) &&
      c.off[r - 1] < (1LL << 30) && c.off[r - 2] < (1LL << 30) &&
      (r == 2 || (c.xshape[0] < (1LL << 30) && c.yshape[0] < (1LL << 20) && c.kshape[0] < (1LL << 20) &&
                  c.off[0] < (1LL << 30)))) {
    RowArgs ra{};
    ra.x = c.x;
    ra.xs0 = c.xstride[r - 2];
    ra.H = (int)c.xshape[r - 2];
    ra.W = (int)c.xshape[r - 1];
    ra.k = c.k;
    ra.y = c.y;
    ra.ys0 = c.ystride[r - 2];
    ra.OH = (int)c.yshape[r - 2];
    ra.OW = (int)c.yshape[r - 1];
    ra.off0 = (int)c.off[r - 2];
    ra.off1 = (int)c.off[r - 1];
    if (r == 3) {
      ra.xsd = c.xstride[0];
      ra.ysd = c.ystride[0];
      ra.D = (int)c.xshape[0];
      ra.KD = (int)c.kshape[0];
      ra.OD = (int)c.yshape[0];
      ra.offd = (int)c.off[0];
    } else {
      ra.xsd = 0;
      ra.ysd = 0;
      ra.D = 1;
      ra.KD = 1;
      ra.OD = 1;
      ra.offd = 0;
    }
    return launch_rows(ra, (int)c.kshape[r - 2], c.xdt, c.band_rows, s);
  }

  // Other 2-D and 3-D cases: the LDS-tiled kernels, for kernels of up to 64 x 64
  // taps; the staged tile stays within 64 KiB of LDS (at most 127 rows by a
  // pitch of 128 elements: 65,024 bytes).  A kernel of up to 256 x 256 taps is
  // split into blocks of at most 64 x 64: block (bi, bj), taps from
  // (64 bi, 64 bj), contributes conv(x, block) at full index n - (64 bi, 64 bj),
  // so each block runs with its output offset moved back by its origin, the
  // first writing the output and the others adding to it, in a fixed order.
  const int64_t kh = c.kshape[r - 2], kw = c.kshape[r - 1];
  const bool tiled_ok = (r == 2 || r == 3) && small_taps && kw <= 4 * kKernelBlock && kh <= 4 * kKernelBlock &&
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
    t.ks0 = (int)kw;
    t.ksd = kh * kw;
    const int64_t n_ty = (t.OH + kTileY - 1) / kTileY;
    const dim3 grid((unsigned)((t.OW + kTileX - 1) / kTileX), (unsigned)(n_ty < 65535 ? n_ty : 65535),
                    (unsigned)t.OD);
    const int off0 = t.off0, off1 = t.off1;
    for (int bi = 0; bi * kKernelBlock < kh; ++bi) {
      for (int bj = 0; bj * kKernelBlock < kw; ++bj) {
        Tile2D b = t;
        b.KH = (int)std::min<int64_t>(kKernelBlock, kh - bi * kKernelBlock);
        b.KW = (int)std::min<int64_t>(kKernelBlock, kw - bj * kKernelBlock);
        b.k = static_cast<const char*>(c.k) + ((int64_t)bi * kKernelBlock * kw + (int64_t)bj * kKernelBlock) * 4;
        b.off0 = off0 - bi * kKernelBlock;
        b.off1 = off1 - bj * kKernelBlock;
        b.accumulate = (bi | bj) != 0;
        const int kwmax = b.KW <= 4 ? 4 : b.KW <= 8 ? 8 : b.KW <= 16 ? 16 : b.KW <= 32 ? 32 : b.KW <= 48 ? 48 : 64;
        const hipError_t e = launch_tiled(c.xdt, b, kwmax, grid, s);
        if (e != hipSuccess) return e;
      }
    }
    return hipSuccess;
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
