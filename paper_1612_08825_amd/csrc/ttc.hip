// Fused multi-scale time-to-contact pass for gfx950.
//
// What is computed (Time to Contact, Formulation and Results): for every
// consecutive frame pair of a stream and every pyramid level l < LV, the ten
// sums of the least-squares normal equations over all 2x2x2 first-difference
// cubes of that level; then the FP64 3x3 solve, FOE, TTC and the multi-scale
// level choice.
//
// How (one persistent launch, then a small finishing launch):
//   * A work item is one wave: a band of RH base rows by 480 columns, split in
//     four 16-lane segments; lane i of a segment holds 8 adjacent base columns
//     (one level-3 column).  Lane 15 of each segment only provides its left
//     column to lane 14 (the segment owns 120 columns).
//   * The wave walks the stream's frames in time.  Each row of a new frame is
//     combined with the same row of the previous frame as the temporal sum
//     S = P0 + P1 and difference D = P1 - P0 (for f16 frames one
//     mixed-precision FMA each).  New rows are prefetched a few rows ahead into
//     registers; the previous frame's band stays in LDS in its packed form, so
//     memory sees every frame once.
//   * Rows are walked top to bottom.  Horizontal neighbour sums/differences of
//     S and D give the derivative cube by one more vertical step.  Because the
//     pyramid is linear, the 2x2 sums of S and D at even columns *are* the next
//     level's S and D (times 4), so all levels are built on the fly in
//     registers; nothing is written but the sums.  Values are kept as
//     un-normalised block sums; the powers of two are removed in FP64 at the end.
//   * The walk continues 2^(LV-1) rows past the band (halo) so that the last
//     owned cube row of every level has its lower neighbour.
//   * Per pair each lane sums its cubes in FP32; the wave reduces its lanes
//     (DPP within groups of 8 lanes, then the 8 group totals through LDS) and
//     writes one partial per (pair, level, wave).  The finishing pass
//     combines the partials of a pair in a fixed order with TwoSum (hi, lo)
//     compensation, converts to FP64, solves and selects the level.
//
// Units inside the kernel at level l (U = block sums of 4^l base pixels of S or D):
//   hx = 2^(3l+2) E_x (per base px), hy likewise, ht = 2^(2l+2) E_t,
//   g = x_l hx + y_l hy = 2^(2l+2) G with x_l, y_l the cube centre in level pixels.
#include <math.h>

#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"
#include "solve.hpp"

namespace ttc {
namespace {

struct FusedArgs {
  const SeqDesc* table;
  const int32_t* item_seq;
  const int32_t* pair_seq;
  int n_seqs;
  SeqDesc inl;
  int64_t n_items;
  int64_t n_pairs;
  float* partials;
};

// Every field of a descriptor read by a whole wave is the same in all lanes;
// say so, so that all band geometry lives in scalar registers.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ SeqDesc uniform(const SeqDesc& s) {
  SeqDesc d;
  d.frame0 = reinterpret_cast<const void*>(uni((int64_t)reinterpret_cast<uintptr_t>(s.frame0)));
  d.frame_stride = uni(s.frame_stride);
  d.row_stride = uni(s.row_stride);
  d.H = uni(s.H);
  d.W = uni(s.W);
  d.n_frames = uni(s.n_frames);
  d.levels = uni(s.levels);
  d.band_rows = uni(s.band_rows);
  d.n_bands = uni(s.n_bands);
  d.n_cw = uni(s.n_cw);
  d.item_begin = uni(s.item_begin);
  d.pair_begin = uni(s.pair_begin);
  d.partial_begin = uni(s.partial_begin);
  d.n_witems = uni(s.n_witems);
  d.vec = uni(s.vec);
  d.pad = 0;
  return d;
}

// Copy one table entry through a global pointer, a dword at a time.
__device__ __forceinline__ SeqDesc load_desc(gptr<const SeqDesc> p) {
  static_assert(sizeof(SeqDesc) % 4 == 0, "descriptor must be whole dwords");
  SeqDesc d;
  const gptr<const uint32_t> src = (gptr<const uint32_t>)p;
  uint32_t* dst = reinterpret_cast<uint32_t*>(&d);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(SeqDesc) / 4); ++i) dst[i] = src[i];
  return d;
}

// The stream of a work item or pair: one load from the plan's index arrays.
__device__ __forceinline__ SeqDesc seq_for_item(const FusedArgs& a, int64_t item) {
  if (a.table == nullptr) return a.inl;
  const int32_t i = uni(as_global(a.item_seq)[item]);
  return load_desc(as_global(a.table) + i);
}

__device__ __forceinline__ SeqDesc seq_for_pair(const FusedArgs& a, int64_t pair) {
  if (a.table == nullptr) return a.inl;
  const int32_t i = uni(as_global(a.pair_seq)[pair]);
  return load_desc(as_global(a.table) + i);
}

// Accumulate the cubes of one row of one level.  hd*, hs*, hD* are the horizontal
// quantities of the previous (p) and current level rows.  EDGE: some lane of the
// wave has a partial set of valid columns at this level.
template <int NC, bool EDGE>
__device__ __forceinline__ void cubes(float (&acc)[10], const float (&hdp)[NC], const float (&hd)[NC],
                                      const float (&hsp)[NC], const float (&hs)[NC], const float (&hDp)[NC],
                                      const float (&hD)[NC], int ncv, float xb, float y) {
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (!EDGE || c < ncv) {
      const float ex = hdp[c] + hd[c];
      const float ey = hs[c] - hsp[c];
      const float et = hDp[c] + hD[c];
      const float g = fmaf(y, ey, (xb + (float)c) * ex);
      acc[0] = fmaf(ex, ex, acc[0]);
      acc[1] = fmaf(ex, ey, acc[1]);
      acc[2] = fmaf(ey, ey, acc[2]);
      acc[3] = fmaf(g, ex, acc[3]);
      acc[4] = fmaf(g, ey, acc[4]);
      acc[5] = fmaf(g, g, acc[5]);
      acc[6] = fmaf(ex, et, acc[6]);
      acc[7] = fmaf(ey, et, acc[7]);
      acc[8] = fmaf(g, et, acc[8]);
      acc[9] = fmaf(et, et, acc[9]);
    }
  }
}

template <int NC>
__device__ __forceinline__ void cubes_dispatch(bool edge, float (&acc)[10], const float (&hdp)[NC],
                                               const float (&hd)[NC], const float (&hsp)[NC], const float (&hs)[NC],
                                               const float (&hDp)[NC], const float (&hD)[NC], int ncv, float xb,
                                               float y) {
  if (edge) cubes<NC, true>(acc, hdp, hd, hsp, hs, hDp, hD, ncv, xb, y);
  else cubes<NC, false>(acc, hdp, hd, hsp, hs, hDp, hD, ncv, xb, y);
}

// Value of lane i + 1 of the same 16-lane row (DPP row_shl:1); lane 15 gets 0.
__device__ __forceinline__ float from_right(float v) { return dpp_f32<0x101>(v); }

// Horizontal quantities of one level row of NC columns, given its block sums U
// (of S) and V (of D); the column right of the lane comes from lane + 1.
template <int NC>
__device__ __forceinline__ void horizontals(const float (&U)[NC], const float (&V)[NC], float (&hs)[NC],
                                            float (&hd)[NC], float (&hD)[NC]) {
  const float un = from_right(U[0]);
  const float vn = from_right(V[0]);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const float ur = (c + 1 < NC) ? U[c + 1] : un;
    const float vr = (c + 1 < NC) ? V[c + 1] : vn;
    hs[c] = U[c] + ur;
    hd[c] = ur - U[c];
    hD[c] = V[c] + vr;
  }
}

// The rows of a band are walked in groups of G rows (the depth of the prefetch
// ring: 8 with four levels, else 4).  Rows walked: the band plus the halo of
// 2^(LV-1) rows below it, rounded up to whole groups.
template <int LV> constexpr int row_group() { return LV >= 4 ? 8 : 4; }
template <int LV, int RH> constexpr int walked_rows() {
  return ((RH + (1 << (LV - 1))) + row_group<LV>() - 1) / row_group<LV>() * row_group<LV>();
}

constexpr int kPartialChunk = 16;  // pairs whose partial sums are staged in LDS before the write-out
// s_waitcnt immediate for vmcnt(0) with expcnt and lgkmcnt left at their maxima
// (gfx9 encoding: vmcnt[3:0] and [15:14], expcnt[6:4], lgkmcnt[11:8]).
constexpr int kWaitVmcntZero = 0x0F70;

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// One wave walks one band of one stream through all frames.  CHECK: the band
// touches the bottom of the frame (rows may be missing) or the stream is not
// vector-aligned; otherwise every walked row exists and the 8-pixel vector load
// of a lane may run past column W into rows that exist.
//
// `prev` is this wave's LDS band store, [NR][64] packed rows of the previous
// frame.  Rows of the current frame are prefetched G rows ahead through a
// register ring that crosses frame boundaries: while the last rows of frame k
// are processed, the first rows of frame k+1 are already in flight.
template <typename T, int LV, int RH, bool CHECK>
__device__ __forceinline__ void band_walk(const SeqDesc& d, int row0, int c_lane, int lane, float* part,
                                          int64_t witem, Raw8<T>* prev, float* pbuf, float* red) {
  constexpr int G = row_group<LV>();  // depth of the prefetch ring
  constexpr int NR = walked_rows<LV, RH>();
  const int li = lane & 15;
  const int H = d.H, W = d.W;

  // valid cube columns of this lane per level, and the cube-centre bases
  int ncv[LV];
  float xb[LV], yb[LV];
  bool edge[LV];
#pragma unroll
  for (int l = 0; l < LV; ++l) {
    const int wl = W >> l;
    const int j0 = c_lane >> l;
    int n = wl - 1 - j0;
    n = n < 0 ? 0 : (n > (8 >> l) ? (8 >> l) : n);
    ncv[l] = (li == 15) ? 0 : n;
    xb[l] = (float)(j0 + 1) - (float)W / (float)(2 << l);
    yb[l] = (float)(row0 >> l) - (float)H / (float)(2 << l);
    const bool part_lane = ncv[l] > 0 && ncv[l] < (8 >> l);
    edge[l] = __any(part_lane);
  }

  const int ncols = W - c_lane;  // pixels of this lane inside the image
  // Lanes right of the image read the last aligned chunk of the row instead:
  // every load is unconditional (so the compiler can count loads in flight),
  // and what those lanes hold only reaches cubes that are not valid.
  const int c_load = c_lane < W ? c_lane : ((W - 1) >> 3) << 3;
  const uint32_t coff = (uint32_t)c_load * (uint32_t)sizeof(T);
  const int64_t rs_b = d.row_stride * (int64_t)sizeof(T);
  const int64_t fs_b = d.frame_stride * (int64_t)sizeof(T);
  const char* band0 = reinterpret_cast<const char*>(d.frame0) + (int64_t)row0 * rs_b;

  auto load_row = [&](Raw8<T>& r, const char* frame_band, int w) {
    const T* p = reinterpret_cast<const T*>(frame_band + (int64_t)w * rs_b + coff);
    if constexpr (!CHECK) {
      r.load(p);
    } else {
      const int row = row0 + w;
      if (row < H && ncols > 0) {
        // a vector load may overrun column W only where a next row exists
        if (d.vec && (ncols >= 8 || row < H - 1)) r.load(p);
        else r.load_partial(p, ncols < 8 ? ncols : 8);
      } else {
        r.zero();
      }
    }
  };

  // frame 0 into the band store, the first group of frame 1 into the ring
  for (int w = 0; w < NR; ++w) {
    Raw8<T> r;
    load_row(r, band0, w);
    prev[w * 64 + lane] = r;
  }
  Raw8<T> ahead[G];
#pragma unroll
  for (int i = 0; i < G; ++i) load_row(ahead[i], band0 + fs_b, i);

  for (int k = 1; k < d.n_frames; ++k) {
    const char* fk = band0 + (int64_t)k * fs_b;
    // the frame whose first group is prefetched during this frame's last group
    // (this frame again after the last one: a harmless in-bounds reload)
    const char* fnext = (k + 1 < d.n_frames) ? fk + fs_b : fk;
    float acc[LV][10];
#pragma unroll
    for (int l = 0; l < LV; ++l)
#pragma unroll
      for (int q = 0; q < 10; ++q) acc[l][q] = 0.f;

    float hs0p[8], hd0p[8], hD0p[8];
    float hs1p[4], hd1p[4], hD1p[4];
    float hs2p[2], hd2p[2], hD2p[2];
    float hs3p[1], hd3p[1], hD3p[1];

    // the whole walk of a frame is unrolled: the loads in flight are then only
    // carried across the frame loop's back edge (the compiler cannot keep a
    // partial wait for loads carried across a loop back edge)
    {
      static_for<0, NR>([&](auto wc) {
        constexpr int w = decltype(wc)::value;
        constexpr int i = w % G;
        const Raw8<T> cur = ahead[i];
        if constexpr (w + G < NR) load_row(ahead[i], fk, w + G);
        else load_row(ahead[i], fnext, w + G - NR);
        if (!CHECK || row0 + w < H) {
          const Raw8<T> old = prev[w * 64 + lane];
          prev[w * 64 + lane] = cur;
          float S[8], D[8];
          cur.sum_diff(old, S, D);
          float hs0[8], hd0[8], hD0[8];
          horizontals<8>(S, D, hs0, hd0, hD0);
          if constexpr (w >= 1 && w <= RH)
            cubes_dispatch<8>(edge[0], acc[0], hd0p, hd0, hs0p, hs0, hD0p, hD0, ncv[0], xb[0], yb[0] + (float)w);
          if constexpr (LV >= 2 && (w & 1) == 1) {
            float U1[4], V1[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              U1[c] = hs0p[2 * c] + hs0[2 * c];
              V1[c] = hD0p[2 * c] + hD0[2 * c];
            }
            float hs1[4], hd1[4], hD1[4];
            horizontals<4>(U1, V1, hs1, hd1, hD1);
            constexpr int lr1 = w >> 1;  // level-1 row just formed, counted from the band top
            if constexpr (lr1 >= 1 && lr1 <= (RH >> 1))
              cubes_dispatch<4>(edge[1], acc[1], hd1p, hd1, hs1p, hs1, hD1p, hD1, ncv[1], xb[1], yb[1] + (float)lr1);
            if constexpr (LV >= 3 && (w & 3) == 3) {
              float U2[2], V2[2];
#pragma unroll
              for (int c = 0; c < 2; ++c) {
                U2[c] = hs1p[2 * c] + hs1[2 * c];
                V2[c] = hD1p[2 * c] + hD1[2 * c];
              }
              float hs2[2], hd2[2], hD2[2];
              horizontals<2>(U2, V2, hs2, hd2, hD2);
              constexpr int lr2 = w >> 2;
              if constexpr (lr2 >= 1 && lr2 <= (RH >> 2))
                cubes_dispatch<2>(edge[2], acc[2], hd2p, hd2, hs2p, hs2, hD2p, hD2, ncv[2], xb[2], yb[2] + (float)lr2);
              if constexpr (LV >= 4 && (w & 7) == 7) {
                float U3[1], V3[1];
                U3[0] = hs2p[0] + hs2[0];
                V3[0] = hD2p[0] + hD2[0];
                float hs3[1], hd3[1], hD3[1];
                horizontals<1>(U3, V3, hs3, hd3, hD3);
                constexpr int lr3 = w >> 3;
                if constexpr (lr3 >= 1 && lr3 <= (RH >> 3))
                  cubes_dispatch<1>(edge[3], acc[3], hd3p, hd3, hs3p, hs3, hD3p, hD3, ncv[3], xb[3],
                                    yb[3] + (float)lr3);
                hs3p[0] = hs3[0];
                hd3p[0] = hd3[0];
                hD3p[0] = hD3[0];
              }
#pragma unroll
              for (int c = 0; c < 2; ++c) {
                hs2p[c] = hs2[c];
                hd2p[c] = hd2[c];
                hD2p[c] = hD2[c];
              }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              hs1p[c] = hs1[c];
              hd1p[c] = hd1[c];
              hD1p[c] = hD1[c];
            }
          }
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            hs0p[c] = hs0[c];
            hd0p[c] = hd0[c];
            hD0p[c] = hD0[c];
          }
        }
      });
    }

    // One partial per (pair, level, wave); lanes that own no cube of a level
    // contribute zero.  The 10 LV values are first summed over groups of 8
    // lanes with three DPP steps, the 8 group totals pass through LDS, and lane
    // t < 10 LV adds the 8 totals of value t (= l * 10 + q).  Partials are
    // staged in LDS and written out every kPartialChunk pairs, so that stores
    // are rarely in flight while the next rows are being prefetched.
    const int p = k - 1;
    const int pc = p % kPartialChunk;
    {
      constexpr int NV = LV * 10;
      float v[NV];
#pragma unroll
      for (int l = 0; l < LV; ++l) {
        const bool own = ncv[l] > 0;
#pragma unroll
        for (int q = 0; q < 10; ++q) v[l * 10 + q] = own ? acc[l][q] : 0.f;
      }
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] += dpp_f32<kDppQuadXor1>(v[i]);
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] += dpp_f32<kDppQuadXor2>(v[i]);
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] += dpp_f32<kDppRowHalfMirror>(v[i]);
      if ((lane & 7) == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) red[(lane >> 3) * NV + i] = v[i];
      }
      // the wave's own LDS writes above are complete before its reads below
      // (LDS executes one wave's instructions in order); the fences only keep
      // the compiler from moving the accesses across each other
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (lane < NV) {
        float t = red[lane];
#pragma unroll
        for (int gi = 1; gi < 8; ++gi) t += red[gi * NV + lane];
        pbuf[pc * NV + lane] = t;
      }
    }
    if (pc == kPartialChunk - 1 || k == d.n_frames - 1) {
      __syncthreads();
      const int p0 = p - pc;
      const int n = (pc + 1) * LV * 10;
      for (int idx = lane; idx < n; idx += 64) {
        const int pl = idx / 10;  // (pair in chunk) * LV + level
        const int q = idx - pl * 10;
        as_global(part)[((int64_t)(p0 * LV + pl) * d.n_witems + witem) * 10 + q] = pbuf[idx];
      }
      // Loads and stores share one completion counter and may complete out of
      // order with respect to each other; with a store possibly in flight, every
      // later wait for a prefetched row would have to drain the counter.  Drain
      // it here, once per chunk, so the row loop's waits can stay partial.
      __builtin_amdgcn_s_waitcnt(kWaitVmcntZero);
      __syncthreads();
    }
  }
}

template <typename T, int LV, int RH>
__global__ __launch_bounds__(64) void ttc_fused(FusedArgs a) {
  constexpr int NR = walked_rows<LV, RH>();
  __shared__ Raw8<T> prev[NR * 64];
  __shared__ float pbuf[kPartialChunk * LV * 10];
  __shared__ float red[8 * LV * 10];
  const int lane = threadIdx.x;
  const int li = lane & 15;
  const int seg = lane >> 4;

  const int G = gridDim.x;
  const int g = blockIdx.x;
  // XCD-aware order: work-groups are dealt to the 8 XCDs round-robin, so give
  // each XCD a contiguous run of items (vertically adjacent bands share halos).
  const int64_t slot = (G % 8 == 0) ? (int64_t)(g % 8) * (G / 8) + g / 8 : g;

  for (int64_t t = 0;; ++t) {
    const int64_t item = t * G + slot;
    if (item >= a.n_items) break;
    const SeqDesc d = uniform(seq_for_item(a, item));
    const int64_t local = item - d.item_begin;  // = cw * n_bands + band
    const int cw = (int)(local / d.n_bands);
    const int band = (int)(local % d.n_bands);
    float* part = a.partials + d.partial_begin;
    const int row0 = band * RH;
    const int c_lane = cw * kWaveCols + seg * kSegCols + li * 8;
    // fast path: all walked rows exist and a vector load running up to 7 pixels
    // past column W of the last walked row stays inside the frame
    const int64_t below = (int64_t)d.H - row0 - NR;
    const bool fast = d.vec && below >= 1 && below * d.row_stride >= 8;
    if (fast) band_walk<T, LV, RH, false>(d, row0, c_lane, lane, part, local, prev, pbuf, red);
    else band_walk<T, LV, RH, true>(d, row0, c_lane, lane, part, local, prev, pbuf, red);
  }
}

// ---------------------------------------------------------------- finishing pass
__device__ __forceinline__ int sum_scale_exp(int l, int q) {
  // hx, hy carry 2^(3l+2), g and ht carry 2^(2l+2)
  switch (q) {
    case 0: case 1: case 2: return 6 * l + 4;
    case 3: case 4: case 6: case 7: return 5 * l + 4;
    default: return 4 * l + 4;
  }
}


// The multi-scale choice again, from level records already in device memory:
// rule 0 descends while the TTC keeps decreasing (as ttc_finish does), rule 1
// takes the valid level with the smallest residual per cube (the lower level
// on a tie; level 0 when none is valid).  One thread per pair.
__global__ __launch_bounds__(256) void ttc_reselect(const tc_ttc_level* __restrict__ lv, int64_t n_pairs, int L,
                                                    int rule, tc_ttc_pick* __restrict__ picks) {
  const int64_t gp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gp >= n_pairs) return;
  const tc_ttc_level* r = lv + gp * L;
  int l = 0;
  if (rule == TC_SELECT_DECREASING_TTC) {
    while (l + 1 < L && level_key(r[l + 1]) < level_key(r[l])) ++l;
  } else {
    double best = __builtin_inf();
    for (int k = 0; k < L; ++k) {
      if (!(level_key(r[k]) < __builtin_inf()) || r[k].n <= 0) continue;
      const double v = r[k].resid / (double)r[k].n;
      if (v < best) {
        best = v;
        l = k;
      }
    }
  }
  tc_ttc_pick pk;
  pk.ttc = r[l].ttc;
  pk.x0 = r[l].x0;
  pk.y0 = r[l].y0;
  pk.A = r[l].A;
  pk.B = r[l].B;
  pk.C = r[l].C;
  pk.level = l;
  pk.status = r[l].status;
  picks[gp] = pk;
}

template <int LV>
__global__ __launch_bounds__(256) void ttc_finish(FusedArgs a, tc_ttc_level* __restrict__ out,
                                                  tc_ttc_pick* __restrict__ picks) {
  const int64_t gp = blockIdx.x;
  if (gp >= a.n_pairs) return;
  const SeqDesc d = seq_for_pair(a, gp);
  const int64_t p = gp - d.pair_begin;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double sums[LV][10];
  __shared__ tc_ttc_level res[LV];

  // wave l reduces level l: each lane adds every 64th wave item's partials with
  // TwoSum compensation, then the lanes' (hi, lo) pairs are merged in a fixed
  // butterfly order
  if (wave < LV) {
    const int l = wave;
    float hi[10], lo[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) hi[q] = lo[q] = 0.f;
    const gptr<const float> base =
        as_global(a.partials + d.partial_begin + (p * LV + l) * (int64_t)d.n_witems * 10);
    for (int w = lane; w < d.n_witems; w += 64) {
#pragma unroll
      for (int q = 0; q < 10; ++q) comp_add(hi[q], lo[q], base[(int64_t)w * 10 + q]);
    }
#pragma unroll
    for (int q = 0; q < 10; ++q) {
#pragma unroll
      for (int m = 1; m < 64; m <<= 1) {
        const float h2 = __shfl_xor(hi[q], m, 64);
        const float l2 = __shfl_xor(lo[q], m, 64);
        comp_merge(hi[q], lo[q], h2, l2);
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 10; ++q) sums[l][q] = ldexp((double)hi[q] + (double)lo[q], -sum_scale_exp(l, q));
    }
  }
  __syncthreads();

  if (tid < LV) {
    tc_ttc_level r;
    solve_level(sums[tid], r);
    const int64_t Hl = d.H >> tid, Wl = d.W >> tid;
    r.n = (Hl - 1) * (Wl - 1);
    r.level = tid;
    res[tid] = r;
    out[gp * LV + tid] = r;
  }
  __syncthreads();
  if (tid == 0) {
    int l = 0;
    while (l + 1 < LV && level_key(res[l + 1]) < level_key(res[l])) ++l;
    tc_ttc_pick pk;
    pk.ttc = res[l].ttc;
    pk.x0 = res[l].x0;
    pk.y0 = res[l].y0;
    pk.A = res[l].A;
    pk.B = res[l].B;
    pk.C = res[l].C;
    pk.level = l;
    pk.status = res[l].status;
    picks[gp] = pk;
  }
}

FusedArgs make_args(const FusedLaunch& f) {
  FusedArgs a;
  a.table = f.table;
  a.item_seq = f.item_seq;
  a.pair_seq = f.pair_seq;
  a.n_seqs = f.n_seqs;
  a.inl = f.inl;
  a.n_items = f.n_items;
  a.n_pairs = f.n_pairs;
  a.partials = f.partials;
  return a;
}

template <typename T, int LV>
hipError_t fused_rh(const FusedLaunch& f, hipStream_t s) {
  const FusedArgs a = make_args(f);
  const dim3 grid((unsigned)f.grid), block(64);
  switch (f.band_rows) {
    case 8: hipLaunchKernelGGL((ttc_fused<T, LV, 8>), grid, block, 0, s, a); break;
    case 16: hipLaunchKernelGGL((ttc_fused<T, LV, 16>), grid, block, 0, s, a); break;
    case 32: hipLaunchKernelGGL((ttc_fused<T, LV, 32>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t fused_lv(const FusedLaunch& f, hipStream_t s) {
  switch (f.levels) {
    case 1: return fused_rh<T, 1>(f, s);
    case 2: return fused_rh<T, 2>(f, s);
    case 3: return fused_rh<T, 3>(f, s);
    case 4: return fused_rh<T, 4>(f, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool fused_variant_exists(int dt, int levels, int band_rows) {
  return (dt == TC_U8 || dt == TC_F16) && levels >= 1 && levels <= 4 &&
         (band_rows == 8 || band_rows == 16 || band_rows == 32);
}

hipError_t launch_ttc_fused(const FusedLaunch& f, hipStream_t s) {
  if (f.n_items == 0) return hipSuccess;
  switch (f.dt) {
    case TC_U8: return fused_lv<uint8_t>(f, s);
    case TC_F16: return fused_lv<_Float16>(f, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ttc_reselect(const tc_ttc_level* levels, int64_t n_pairs, int L, int rule, tc_ttc_pick* picks,
                              hipStream_t s) {
  if (n_pairs == 0) return hipSuccess;
  const dim3 grid((unsigned)((n_pairs + 255) / 256)), block(256);
  hipLaunchKernelGGL(ttc_reselect, grid, block, 0, s, levels, n_pairs, L, rule, picks);
  return hipGetLastError();
}

hipError_t launch_ttc_finish(const FusedLaunch& f, tc_ttc_level* out, tc_ttc_pick* picks, hipStream_t s) {
  if (f.n_pairs == 0) return hipSuccess;
  const FusedArgs a = make_args(f);
  const dim3 grid((unsigned)f.n_pairs), block(256);
  switch (f.levels) {
    case 1: hipLaunchKernelGGL(ttc_finish<1>, grid, block, 0, s, a, out, picks); break;
    case 2: hipLaunchKernelGGL(ttc_finish<2>, grid, block, 0, s, a, out, picks); break;
    case 3: hipLaunchKernelGGL(ttc_finish<3>, grid, block, 0, s, a, out, picks); break;
    case 4: hipLaunchKernelGGL(ttc_finish<4>, grid, block, 0, s, a, out, picks); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ttc
