// Row-streaming direct convolution for gfx950, for images whose rows are
// contiguous and square kernels of 2, 3, 5 or 7 taps (Discrete Derivatives,
// the spatial convolution equation; Accelerating Convolutions, the direct
// method):  y[n] = sum_t k[t] x[n + off - t], x read as zero outside.
//
// Built once per input type (-DTC_ROWS_DT=0: FP32 x and taps, FP32 sums;
// 1: FP16 x, FP32 taps and sums; 2: u8 x, int32 taps below 2^23 in magnitude,
// exact int32 sums with 24-bit multiplies).
//
// One wave per item: a band of R (8, or 4 for small outputs) output rows by
// 4 * LO output columns of one output plane; lane i < LO holds output columns
// 4i .. 4i+3 of the band in registers.  The wave walks the band's R + KH - 1
// input rows top to bottom and multiplies each into every output row of the
// band it reaches; taps are wave-uniform and come through the scalar cache.
//
// Loads are what bounds this kernel (each vector-memory instruction costs the
// texture addresser about the same whatever its width), so an input row costs
// one load per lane: lane i loads 4 consecutive columns ("its chunk": 16 bytes
// of FP32, 8 of FP16, 4 of u8), converts them to the accumulation type, and
// the KW + 3 columns a lane needs (its window) are its chunk and the chunks of
// the next NC - 1 lanes, moved across the wave with DPP.  The last NC - 1
// lanes only load: their windows would reach past the wave, so LO = 65 - NC.
// The window of lane i starts S columns into its chunk (S = 0..3 is the same
// for every lane and row of a launch and is a template parameter).
//
// In waves whose chunks may leave the image, a lane whose chunk lies wholly
// outside loads nothing, and a lane whose chunk straddles the edge loads it one
// column at a time with buffer loads through a resource limited to the row,
// which read zero left and right of the image; bands whose rows may leave the
// image skip those rows.  For rank 3 the item is one output plane and the
// kernel planes are walked in turn, each over its input plane.
#include "conv_common.hpp"

#if !defined(TC_ROWS_DT)
#error "conv_rows.hip is built once per input type (TC_ROWS_DT)"
#endif

namespace ttc {
namespace rows {
namespace {

template <int DT> struct Io;

// FP32: one 16-byte load per chunk
template <> struct Io<0> {
  using TX = float;
  using TA = float;
  __device__ static void chunk(const TX* rp, int cc, TA (&c4)[4]) {
    const f4u v = *(const __attribute__((address_space(1))) f4u*)(rp + cc);
    c4[0] = v.x;
    c4[1] = v.y;
    c4[2] = v.z;
    c4[3] = v.w;
  }
  __device__ static TA column(__amdgpu_buffer_rsrc_t rs, int col) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (uint32_t)col * 4u, 0, 0));
  }
  __device__ static TA mac(TA acc, TA k, TA v) { return fmaf(k, v, acc); }
};

// FP16: one 8-byte load per chunk, exact conversion to FP32
typedef unsigned u2a __attribute__((ext_vector_type(2), aligned(4)));
template <> struct Io<1> {
  using TX = _Float16;
  using TA = float;
  __device__ static float half(uint32_t w, int hi) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(hi ? (w >> 16) : (w & 0xffffu)));
  }
  __device__ static void chunk(const TX* rp, int cc, TA (&c4)[4]) {
    const u2a v = *(const __attribute__((address_space(1))) u2a*)(rp + cc);
    c4[0] = half(v.x, 0);
    c4[1] = half(v.x, 1);
    c4[2] = half(v.y, 0);
    c4[3] = half(v.y, 1);
  }
  __device__ static TA column(__amdgpu_buffer_rsrc_t rs, int col) {
    const uint16_t h = __builtin_amdgcn_raw_buffer_load_b16(rs, (uint32_t)col * 2u, 0, 0);
    return (float)__builtin_bit_cast(_Float16, h);
  }
  __device__ static TA mac(TA acc, TA k, TA v) { return fmaf(k, v, acc); }
};

// u8: one 4-byte load per chunk; taps below 2^23 in magnitude times pixels
// below 2^8 are exact 24-bit products
template <> struct Io<2> {
  using TX = uint8_t;
  using TA = int;
  __device__ static void chunk(const TX* rp, int cc, TA (&c4)[4]) {
    const uint32_t v = *(const __attribute__((address_space(1))) uint32_t*)(rp + cc);
    c4[0] = (int)(v & 0xffu);
    c4[1] = (int)((v >> 8) & 0xffu);
    c4[2] = (int)((v >> 16) & 0xffu);
    c4[3] = (int)(v >> 24);
  }
  __device__ static TA column(__amdgpu_buffer_rsrc_t rs, int col) {
    return (int)__builtin_amdgcn_raw_buffer_load_b8(rs, (uint32_t)col, 0, 0);
  }
  __device__ static TA mac(TA acc, TA k, TA v) { return acc + __mul24(k, v); }
};

using IO = Io<TC_ROWS_DT>;
using TX = IO::TX;
using TA = IO::TA;

// acc[j][c] += sum over taps of one kernel plane, for the band's input rows
// i0 .. i0 + R + KH - 2 (output row j of the band takes input rows
// i0 + j .. i0 + j + KH - 1 with tap rows KH - 1 .. 0).  EDGE: some lane's
// chunk may reach outside the image (such a lane loads its chunk one
// range-checked column at a time); ROWCHECK: input rows may lie outside the
// image (uniform across the wave; they are skipped).
template <int KH, int KW, int R, int S, bool EDGE, bool ROWCHECK>
__device__ __forceinline__ void band_accumulate(TA (&acc)[R][4], const TX* plane, int W, int chunk0,
                                                uint32_t lane_col, int64_t xs0, int H, int i0, cptr<TA> taps) {
  constexpr int NW = KW + 3;
  constexpr int NC = row_chunks<KW, S>();
  static_for<0, R + KH - 1>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    const int row = i0 + t;
    if (!ROWCHECK || (row >= 0 && row < H)) {
      const TX* rp = plane + (int64_t)row * xs0;
      // this lane's chunk, then those of the next NC - 1 lanes
      TA ch[4 * NC];
      const int cc = chunk0 + (int)lane_col;  // first column of the chunk
      if (!EDGE || (cc >= 0 && cc + 4 <= W)) {
        TA c4[4];
        IO::chunk(rp, cc, c4);
#pragma unroll
        for (int d = 0; d < 4; ++d) ch[d] = c4[d];
      } else if (cc >= W || cc + 4 <= 0) {
#pragma unroll
        for (int d = 0; d < 4; ++d) ch[d] = (TA)0;  // wholly outside: no load
      } else {
        // a chunk reaching outside the image: one range-checked load per column
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(rp, (uint32_t)W * (uint32_t)sizeof(TX));
#pragma unroll
        for (int d = 0; d < 4; ++d) ch[d] = IO::column(rs, cc + d);
      }
#pragma unroll
      for (int k = 1; k < NC; ++k)
#pragma unroll
        for (int d = 0; d < 4; ++d) ch[4 * k + d] = from_next_lane(ch[4 * (k - 1) + d]);
      TA w[NW];
#pragma unroll
      for (int e = 0; e < NW; ++e) w[e] = ch[S + e];
      static_for<cmax(0, t - KH + 1), cmin(R - 1, t) + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int a = j + KH - 1 - t;  // tap row
#pragma unroll
        for (int b = 0; b < KW; ++b) {
          const TA kv = taps[a * KW + b];
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[j][c] = IO::mac(acc[j][c], kv, w[c + KW - 1 - b]);
        }
      });
    }
  });
}

typedef TA tav4 __attribute__((ext_vector_type(4), aligned(4)));

// At least WPE waves per SIMD (<= 512 / WPE VGPRs): left alone, the compiler
// issues every row load of the unrolled band up front and holds them all.
template <int KH, int KW, int R, int S, int WPE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void conv2d_rows(RowArgs a) {
  constexpr int LO = row_lanes_out<KW, S>();
  const int lane = threadIdx.x;
  const int64_t G = gridDim.x, g = blockIdx.x;
  // XCD-aware order: work-groups are dealt to the 8 XCDs round-robin; give each
  // XCD a contiguous run of items, so vertically adjacent bands (which share
  // KH - 1 input rows) meet in the same L2.  Items run across a band's column
  // strips first, so that concurrent waves read whole row segments.
  const int64_t item = (G % 8 == 0) ? (g % 8) * (G / 8) + g / 8 : g;
  if (item >= a.n_items) return;
  const int64_t per_plane = (int64_t)a.n_bands * a.n_cw;
  const int od = (int)(item / per_plane);
  const int rem = (int)(item - (int64_t)od * per_plane);
  const int band = rem / a.n_cw;
  const int cw = rem - band * a.n_cw;
  const int o0 = band * R;
  const int p_wave = cw * 4 * LO;
  const int p_lane = p_wave + 4 * lane;
  // first column of lane 0's chunk: lane i's window starts S columns into its
  // chunk, at full column p_lane + off1 - (KW - 1)
  const int chunk0 = p_wave + a.off1 - (KW - 1) - S;
  const uint32_t lane_col = 4u * (uint32_t)lane;
  const int i0 = o0 + a.off0 - (KH - 1);  // first input row of the band
  const bool rows_in = i0 >= 0 && i0 + R + KH - 2 < a.H;
  const bool cols_in = chunk0 >= 0 && chunk0 + 256 <= a.W;

  TA acc[R][4];
#pragma unroll
  for (int j = 0; j < R; ++j)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[j][c] = (TA)0;

  const int nd = od + a.offd;  // full-result plane
  for (int kd = 0; kd < a.KD; ++kd) {
    const int xd = nd - kd;
    if (xd < 0 || xd >= a.D) continue;  // uniform
    const TX* plane = static_cast<const TX*>(a.x) + (int64_t)xd * a.xsd;
    const cptr<TA> taps = (cptr<TA>)(static_cast<const TA*>(a.k)) + kd * KH * KW;
    if (rows_in && cols_in)
      band_accumulate<KH, KW, R, S, false, false>(acc, plane, a.W, chunk0, lane_col, a.xs0, a.H, i0, taps);
    else if (cols_in)
      band_accumulate<KH, KW, R, S, false, true>(acc, plane, a.W, chunk0, lane_col, a.xs0, a.H, i0, taps);
    else
      band_accumulate<KH, KW, R, S, true, true>(acc, plane, a.W, chunk0, lane_col, a.xs0, a.H, i0, taps);
  }

  if (lane >= LO) return;
  const gptr<TA> yp = as_global(static_cast<TA*>(a.y)) + (int64_t)od * a.ysd;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int o = o0 + j;
    if (o >= a.OH) break;
    const gptr<TA> yr = yp + (int64_t)o * a.ys0 + p_lane;
    if (p_lane + 3 < a.OW) {
      tav4 v;
      v.x = acc[j][0];
      v.y = acc[j][1];
      v.z = acc[j][2];
      v.w = acc[j][3];
      *(__attribute__((address_space(1))) tav4*)yr = v;
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (p_lane + c < a.OW) yr[c] = acc[j][c];
    }
  }
}

template <int KH, int KW, int R, int S>
hipError_t launch_rows_s(RowArgs ra, hipStream_t s) {
  constexpr int LO = row_lanes_out<KW, S>();
  ra.n_bands = (ra.OH + R - 1) / R;
  ra.n_cw = (ra.OW + 4 * LO - 1) / (4 * LO);
  ra.n_items = (int64_t)ra.OD * ra.n_bands * ra.n_cw;
  const int64_t grid = (ra.n_items + 7) / 8 * 8;
  hipLaunchKernelGGL((conv2d_rows<KH, KW, R, S, 4>), dim3((unsigned)grid), dim3(64), 0, s, ra);
  return hipGetLastError();
}

template <int KH, int KW, int R>
hipError_t launch_rows_t(const RowArgs& ra, hipStream_t s) {
  // the window's offset inside a chunk: (off1 - (KW - 1)) mod 4
  switch ((((ra.off1 - (KW - 1)) % 4) + 4) % 4) {
    case 0: return launch_rows_s<KH, KW, R, 0>(ra, s);
    case 1: return launch_rows_s<KH, KW, R, 1>(ra, s);
    case 2: return launch_rows_s<KH, KW, R, 2>(ra, s);
    default: return launch_rows_s<KH, KW, R, 3>(ra, s);
  }
}

}  // namespace

#define TC_CAT2(a, b) a##b
#define TC_ROWS_LAUNCHER(dt) TC_CAT2(launch_rows_dt, dt)
#define TC_ROWS_LAUNCHER_X(dt) TC_ROWS_LAUNCHER(dt)

// The band height is 8 unless that leaves fewer than about two waves per SIMD
// (2048 items on 256 CUs), then 4.
hipError_t TC_ROWS_LAUNCHER_X(TC_ROWS_DT)(const RowArgs& ra, int KH, hipStream_t s) {
  const int64_t items8 = (int64_t)ra.OD * ((ra.OH + 7) / 8) * ((ra.OW + 4 * 61 - 1) / (4 * 61));
  const bool small = items8 < 2048;
  switch (KH) {
    case 2: return small ? launch_rows_t<2, 2, 4>(ra, s) : launch_rows_t<2, 2, 8>(ra, s);
    case 3: return small ? launch_rows_t<3, 3, 4>(ra, s) : launch_rows_t<3, 3, 8>(ra, s);
    case 5: return small ? launch_rows_t<5, 5, 4>(ra, s) : launch_rows_t<5, 5, 8>(ra, s);
    case 7: return small ? launch_rows_t<7, 7, 4>(ra, s) : launch_rows_t<7, 7, 8>(ra, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rows
}  // namespace ttc
