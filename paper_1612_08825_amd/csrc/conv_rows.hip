// Row-streaming direct convolution for gfx950, for images whose rows are
// contiguous and square kernels of 2, 3, 5 or 7 taps (Discrete Derivatives,
// the spatial convolution equation; Accelerating Convolutions, the direct
// method):  y[n] = sum_t k[t] x[n + off - t], x read as zero outside.
//
// Built once per input type (-DTC_ROWS_DT=0: FP32 x and taps, FP32 sums;
// 1: FP16 x, FP32 taps and sums; 2: u8 x, int32 taps below 2^23 in magnitude,
// exact int32 sums with 24-bit multiplies).
//
// One wave per item: a band of R (2, 4 or 8, from a tuned table) output rows by
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
// kernel planes are walked in turn, each over its input plane -- except for
// 3 x 3 x 3 kernels over images whose rows are a multiple of 4 wide, which
// take conv3d_rows: runs of output planes, each input plane loaded once, and
// waves split into lane groups so that rows just over one wave wide waste
// fewer lanes.
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
  __device__ static TA mul(TA k, TA v) { return k * v; }
  // the chunk at byte offset off of a buffer (zero where out of range)
  __device__ static void chunk_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off, TA (&c4)[4]) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    // element by element through a scalar: a bit_cast of a vector element
    // expression would read element 0 whatever the index
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const uint32_t u = v[d];
      c4[d] = __builtin_bit_cast(float, u);
    }
  }
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
  __device__ static TA mul(TA k, TA v) { return k * v; }
  __device__ static void chunk_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off, TA (&c4)[4]) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
    c4[0] = half(v[0], 0);
    c4[1] = half(v[0], 1);
    c4[2] = half(v[1], 0);
    c4[3] = half(v[1], 1);
  }
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
  __device__ static TA mul(TA k, TA v) { return __mul24(k, v); }
  __device__ static void chunk_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off, TA (&c4)[4]) {
    const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
    c4[0] = (int)(v & 0xffu);
    c4[1] = (int)((v >> 8) & 0xffu);
    c4[2] = (int)((v >> 16) & 0xffu);
    c4[3] = (int)(v >> 24);
  }
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

// The NR rows of one input plane that a band reads, one chunk per lane and
// row, through a buffer resource over the plane: off[t] is the chunk's byte
// offset in the plane, or kOutside for a row or chunk outside the image,
// which the buffer's range check reads as zero.  Loads only: the products
// come after the caller's stores.
constexpr uint32_t kOutside = 0x80000000u;  // beyond any plane taken here (< 2 GiB)
template <int NR>
__device__ __forceinline__ void load_band(TA (&rows)[NR][4], __amdgpu_buffer_rsrc_t plane, const uint32_t (&off)[NR]) {
  static_for<0, NR>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    IO::chunk_buf(plane, off[t], rows[t]);
  });
}

// acc[slot(kd)][j][c] += the band's input rows (one input plane) x taps of
// kernel plane kd, for the kernel planes kd_lo .. kd_hi (those whose output
// planes belong to the run; uniform): each row feeds every output plane it
// contributes to.  The slot of kernel plane kd is (RR + kd + 1) mod K, RR the
// input plane's position in the rotation.  Kernel plane K - 1 starts its
// slot's output plane: the first term of each output row (tap row K - 1,
// column 0) is written, not added, so slots are never cleared.
template <int K, int R, int S, int RR>
__device__ __forceinline__ void band_fma_planes(TA (&acc)[K][R][4], const TA (&rows)[R + K - 1][4],
                                                const TA (&tv)[K * K * K], int kd_lo, int kd_hi) {
  constexpr int NW = K + 3;
  constexpr int NC = row_chunks<K, S>();
  static_for<0, R + K - 1>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    TA ch[4 * NC];
#pragma unroll
    for (int d = 0; d < 4; ++d) ch[d] = rows[t][d];
#pragma unroll
    for (int k = 1; k < NC; ++k)
#pragma unroll
      for (int d = 0; d < 4; ++d) ch[4 * k + d] = from_next_lane(ch[4 * (k - 1) + d]);
    TA w[NW];
#pragma unroll
    for (int e = 0; e < NW; ++e) w[e] = ch[S + e];
    static_for<0, K>([&](auto kc) {
      constexpr int kd = decltype(kc)::value;
      constexpr int slot = (RR + kd + 1) % K;
      if (kd >= kd_lo && kd <= kd_hi) {
        static_for<cmax(0, t - K + 1), cmin(R - 1, t) + 1>([&](auto jc) {
          constexpr int j = decltype(jc)::value;
          constexpr int a = j + K - 1 - t;  // tap row
          static_for<0, K>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
            const TA kv = tv[(kd * K + a) * K + b];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              if constexpr (kd == K - 1 && a == K - 1 && b == 0)
                acc[slot][j][c] = IO::mul(kv, w[c + K - 1 - b]);
              else
                acc[slot][j][c] = IO::mac(acc[slot][j][c], kv, w[c + K - 1 - b]);
            }
          });
        });
      }
    });
  });
}

// Rank 3 with a K x K x K kernel: 2.5-D rolling planes.
//
// An item is a band of R output rows by 4 * LO columns for a run of DZ
// consecutive output planes (the last run may be shorter).  The wave is split
// into 64 / L groups of L lanes (L = 64, 32 or 16; lg = log2 L), one item
// each, consecutive items side by side: for rows a little wider than one
// wave's 4 * (64 - NC + 1) columns this wastes fewer lanes than whole-wave
// strips.  The last NC - 1 lanes of a group only load (their windows would
// reach into the next group), LO = L - NC + 1.
//
// The wave walks the input planes that feed its run once each, in order;
// input plane i (counted from the run's first, od0 + offd - (K - 1)) adds into
// output planes m = i + kd - (K - 1), kd = 0..K-1, held in K accumulator slots
// in rotation (slot of m: m mod K); terms for planes outside the run are not
// formed.  Output plane m has all its terms once plane m + K - 1 is in.  It is
// stored during the step of plane m + K, before that step's products, which
// start the slot afresh.  The loads of all DZ + K - 1 input planes of the run
// are issued first, one row buffer per plane, so the products of a plane run
// while the later planes' rows are still arriving (the compiler waits for one
// plane's rows at a time: vector loads complete in order).  The run is
// unrolled whole: buffers, slots and the first planes' kernel-plane bounds are
// static.  Every plane issues the same loads (a plane past the run or outside
// the image reloads one inside, unused).
//
// Launch shape: bands of 2 rows and runs of 2 planes.  More, smaller waves
// overlap one wave's loads with another's products better than few large ones
// (64 x 256 x 256 by 3^3 on MI355X: 4-row bands and 3-plane runs 14.8 us;
// 2 x 3 13.7; 2 x 1 13.6; 1 x 1..3 14.1-15.7; 2 x 2 13.1).
//
// Rows and chunks outside the image are read through the plane's buffer
// resource at an out-of-range offset, which reads zero (W is a multiple of 4,
// so no chunk straddles the edge; planes are below 2 GiB).  The K^3 taps are
// held in vector registers: wave-uniform, but the scalar registers cannot keep
// them all, and reloading them would stall every step.
template <int K, int R, int S, int DZ>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void conv3d_rows(RowArgs a, int lg) {
  constexpr int NC = row_chunks<K, S>();
  constexpr int NR = R + K - 1;
  const int L = 1 << lg;
  const int LO = L - NC + 1;
  const int lane = threadIdx.x;
  const int gi = lane >> lg, gl = lane & (L - 1);
  const int64_t Gd = gridDim.x, g = blockIdx.x;
  const int64_t wave = (Gd % 8 == 0) ? (g % 8) * (Gd / 8) + g / 8 : g;
  if (wave >= a.n_items) return;
  // waves: run-major; inside a run, item q = (band, strip) with band-major order
  const int per_run = a.n_bands * a.n_cw;
  const int wpr = (per_run + (64 >> lg) - 1) >> (6 - lg);
  const int run = (int)(wave / wpr);
  const int q = (int)(wave - (int64_t)run * wpr) * (64 >> lg) + gi;
  const bool active = q < per_run;
  const int qe = active ? q : per_run - 1;  // an idle group reloads a valid item and stores nothing
  const int band = qe / a.n_cw;
  const int cw = qe - band * a.n_cw;
  const int o0 = band * R;
  const int p_group = cw * 4 * LO;
  const int p_lane = p_group + 4 * gl;
  const int chunk0 = p_group + a.off1 - (K - 1) - S;
  const int cc = chunk0 + 4 * gl;
  const int i0 = o0 + a.off0 - (K - 1);
  const bool chunk_in = cc >= 0 && cc < a.W;
  const int od0 = run * DZ;
  const int nz = DZ < a.OD - od0 ? DZ : a.OD - od0;  // output planes of this run
  const int n_in = nz + K - 1;                          // input planes walked
  const int xd0 = od0 + a.offd - (K - 1);
  const cptr<TA> taps = (cptr<TA>)(static_cast<const TA*>(a.k));
  TA tv[K * K * K];
#pragma unroll
  for (int n = 0; n < K * K * K; ++n) {
    tv[n] = taps[n];
    asm volatile("" : "+v"(tv[n]));
  }

  // this lane's output rows: byte offsets within an output plane, and which
  // exist
  uint32_t yoff[R];
  bool row_ok[R];
  const bool writer = active && gl < LO;
  const bool full4 = p_lane + 3 < a.OW;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    yoff[j] = (uint32_t)(((int64_t)(o0 + j) * a.ys0 + p_lane) * (int64_t)sizeof(TA));
    row_ok[j] = writer && o0 + j < a.OH && p_lane < a.OW;
  }

  TA acc[K][R][4];
  // store output plane m of the run (if it is one) from pl
  auto store_plane = [&](int m, const TA (&pl)[R][4]) {
    if (m >= 0 && m < nz) {  // uniform
      char* yp = reinterpret_cast<char*>(a.y) + (int64_t)(od0 + m) * a.ysd * (int64_t)sizeof(TA);
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (row_ok[j]) {
          if (full4) {
            tav4 v;
            v.x = pl[j][0];
            v.y = pl[j][1];
            v.z = pl[j][2];
            v.w = pl[j][3];
            *(__attribute__((address_space(1))) tav4*)(yp + (uint64_t)yoff[j]) = v;
          } else {
#pragma unroll
            for (int c = 0; c < 4; ++c)
              if (p_lane + c < a.OW)
                *(__attribute__((address_space(1))) TA*)(yp + (uint64_t)(yoff[j] + 4u * c)) = pl[j][c];
          }
        }
      }
    }
  };

  // byte offsets of this lane's chunks in the NR rows of a plane
  uint32_t off[NR];
#pragma unroll
  for (int t = 0; t < NR; ++t) {
    const int row = i0 + t;
    off[t] = (chunk_in && row >= 0 && row < a.H)
                 ? (uint32_t)(((int64_t)row * a.xs0 + cc) * (int64_t)sizeof(TX))
                 : kOutside;
  }
  const uint32_t plane_bytes = (uint32_t)(((int64_t)(a.H - 1) * a.xs0 + a.W) * (int64_t)sizeof(TX));
  // issue the loads of input plane i into dst; false when the plane lies
  // outside the image (the nearest plane inside is read instead)
  auto load_plane = [&](int i, TA (&dst)[NR][4]) -> bool {
    const int xd = xd0 + i;
    const int xc = xd < 0 ? 0 : (xd >= a.D ? a.D - 1 : xd);
    load_band<NR>(dst, make_rsrc(static_cast<const TX*>(a.x) + (int64_t)xc * a.xsd, plane_bytes), off);
    return xd >= 0 && xd < a.D;
  };
  // every input plane of the run has a row buffer, and all their loads are
  // issued first: a wave then waits for memory once, not once per plane
  // (a plane past a shorter last run reloads the run's last plane, unused)
  constexpr int NB = DZ + K - 1;
  TA rows[NB][NR][4];
  bool have[NB];
  static_for<0, NB>([&](auto pc) {
    constexpr int p0 = decltype(pc)::value;
    have[p0] = load_plane(p0 < n_in ? p0 : n_in - 1, rows[p0]);
  });
  static_for<0, NB>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int cur = i % K, nxt = (i + 1) % K;
    if (i < n_in) {                  // uniform: the last run may be shorter
      store_plane(i - K, acc[cur]);  // complete since plane i - 1; slot (i - K) mod K
      if (have[i]) {
        constexpr int kd_lo = K - 1 - i;       // below: planes before the run
        const int kd_hi = nz - 1 - i + K - 1;  // above: planes after it
        band_fma_planes<K, R, S, cur>(acc, rows[i], tv, kd_lo, kd_hi);
      } else {
        // a plane outside the image: its terms are zero, and it would have
        // started output plane i's slot
#pragma unroll
        for (int j = 0; j < R; ++j)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[cur][j][c] = (TA)0;
      }
      if (i == n_in - 1) store_plane(i - (K - 1), acc[nxt]);
    }
  });
}

template <int K, int R, int S>
hipError_t launch_rows3d_s(RowArgs ra, hipStream_t s) {
  constexpr int NC = row_chunks<K, S>();
  ra.n_bands = (ra.OH + R - 1) / R;
  // the group width that needs the fewest waves per plane
  int best_lg = 6, best_cw = 0;
  int64_t best_w = INT64_MAX;
  for (int lg = 6; lg >= 4; --lg) {
    const int LO = (1 << lg) - NC + 1;
    const int n_cw = (ra.OW + 4 * LO - 1) / (4 * LO);
    const int64_t w = ((int64_t)ra.n_bands * n_cw + (64 >> lg) - 1) >> (6 - lg);
    if (w < best_w) best_w = w, best_lg = lg, best_cw = n_cw;
  }
  ra.n_cw = best_cw;
  // runs of 2 output planes
  constexpr int DZ = 2;
  const int n_runs = (ra.OD + DZ - 1) / DZ;
  ra.n_items = (int64_t)n_runs * best_w;  // waves
  const int64_t grid = (ra.n_items + 7) / 8 * 8;
  hipLaunchKernelGGL((conv3d_rows<K, R, S, DZ>), dim3((unsigned)grid), dim3(64), 0, s, ra, best_lg);
  return hipGetLastError();
}

template <int K, int R>
hipError_t launch_rows3d_t(const RowArgs& ra, hipStream_t s) {
  switch ((((ra.off1 - (K - 1)) % 4) + 4) % 4) {
    case 0: return launch_rows3d_s<K, R, 0>(ra, s);
    case 1: return launch_rows3d_s<K, R, 1>(ra, s);
    case 2: return launch_rows3d_s<K, R, 2>(ra, s);
    default: return launch_rows3d_s<K, R, 3>(ra, s);
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

#define TC_CAT2(a, b) a##b
#define TC_ROWS_LAUNCHER(dt) TC_CAT2(launch_rows_dt, dt)
#define TC_ROWS_LAUNCHER_X(dt) TC_ROWS_LAUNCHER(dt)

// Output rows per wave (band height) from the convolution tuning sweep
// (square images, full mode, graph-replayed over buffers rotated past the
// last-level cache), per input type, taps per side (2, 3, 5, 7) and output
// size class (fewer than 2^21 elements, fewer than 2^23, more).  Every height
// sums an output in the same order, so the choice never changes a result; the
// short bands win wherever the output is too small to fill the chip with
// taller ones (more, shorter waves).
constexpr int8_t kBandRows[3][4][3] = {
    {{2, 2, 4}, {2, 2, 4}, {2, 2, 4}, {2, 2, 4}},  // FP32
    {{2, 2, 2}, {2, 2, 2}, {2, 2, 4}, {2, 2, 4}},  // FP16
    {{2, 4, 2}, {2, 2, 4}, {2, 4, 4}, {2, 2, 4}},  // u8
};
int default_band_rows(int KH, int64_t out_elems) {
  const int ki = KH == 2 ? 0 : (KH == 3 ? 1 : (KH == 5 ? 2 : 3));
  const int cls = out_elems < (1LL << 21) ? 0 : (out_elems < (1LL << 23) ? 1 : 2);
  return kBandRows[TC_ROWS_DT][ki][cls];
}

template <int K>
hipError_t launch_rows_k(const RowArgs& ra, int band_rows, hipStream_t s) {
  switch (band_rows) {
    case 2: return launch_rows_t<K, K, 2>(ra, s);
    case 4: return launch_rows_t<K, K, 4>(ra, s);
    default: return launch_rows_t<K, K, 8>(ra, s);
  }
}

}  // namespace

hipError_t TC_ROWS_LAUNCHER_X(TC_ROWS_DT)(const RowArgs& ra, int KH, int band_rows, hipStream_t s) {
  // a 3 x 3 x 3 kernel over several planes: rolling planes, each read once
  // (its band height is fixed)
  if (KH == 3 && ra.KD == 3 && ra.OD > 1 && ra.W % 4 == 0 && ra.W >= 4 &&
      ((int64_t)(ra.H - 1) * ra.xs0 + ra.W) * (int64_t)sizeof(TX) < (1LL << 31) &&
      ((int64_t)(ra.OH - 1) * ra.ys0 + ra.OW) * 4 < (1LL << 31))
    return launch_rows3d_t<3, 2>(ra, s);
  if (band_rows == 0) band_rows = default_band_rows(KH, (int64_t)ra.OD * ra.OH * ra.OW);
  if (band_rows != 2 && band_rows != 4 && band_rows != 8) return hipErrorInvalidValue;
  switch (KH) {
    case 2: return launch_rows_k<2>(ra, band_rows, s);
    case 3: return launch_rows_k<3>(ra, band_rows, s);
    case 5: return launch_rows_k<5>(ra, band_rows, s);
    case 7: return launch_rows_k<7>(ra, band_rows, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rows
}  // namespace ttc
