// Fused multi-scale time-to-contact pass for gfx950.
//
// What is computed (Time to Contact, Formulation and Results): for every
// consecutive frame pair of a stream and every pyramid level l < LV, the ten
// sums of the least-squares normal equations over all 2x2x2 first-difference
// cubes of that level.  The FP64 solve, FOE, TTC and the multi-scale choice
// follow in the finishing pass (ttc.hip).
//
// This file is compiled once per frame type and level count
// (-DTC_FUSED_DT=0 for u8 frames, 1 for f16; -DTC_FUSED_LV=1..4), so that the
// kernels build in parallel; each object exports one launcher.
//
// How (one persistent launch):
//   * A segment is a band of RB base rows (RB a multiple of 16, a launch
//     parameter) by a strip of seg_cols base columns (504, 248, 160 or 120,
//     chosen per stream so that a pair takes the fewest waves).  A lane holds 8
//     adjacent base columns (one level-3 column); the column right of its last
//     one comes from the next lane by a whole-wave DPP shift, so a segment
//     takes seg_cols / 8 owning lanes and one more that only lends its columns.
//     A work item is one wave and one frame pair: 1 to 4 segments side by side
//     in its lanes (bands of the same or the next column strip), each lane
//     walking its own segment's rows.
//   * The wave walks the band's rows top to bottom, reading the row of both
//     frames of the pair, and forms the temporal sum S = P0 + P1 and difference
//     D = P1 - P0 (for f16 frames one mixed-precision FMA each).  Rows are
//     prefetched eight ahead through a register ring: row j's registers are
//     refilled with row j + 8 as soon as its S and D are formed.  Work items
//     are numbered pair-minor, so the items of consecutive pairs of one band
//     run side by side on one XCD and the frame they share is fetched from
//     memory about once (the second read is served by the caches).
//   * Horizontal neighbour sums/differences of S and D give the derivative
//     cube by one more vertical step.  Because the pyramid is linear, the 2x2
//     sums of S and D at even columns *are* the next level's S and D (times 4),
//     so all levels are built on the fly in registers; nothing is written but
//     the sums.  Values are kept as un-normalised block sums; the powers of two
//     are removed in FP64 at the end.
//   * Rows go in groups of 8 (one level-3 row): the first group, a loop over
//     the groups inside the band, and the halo past it, 2^(LV-1) rows, so that
//     the last owned cube row of every level has its lower neighbour.
//   * Each lane sums its cubes in FP32 registers and adds the block into its
//     own LDS slots every 16 rows; at the end of the item one lane per
//     (segment, value) adds the segment's owning lanes in a pairwise tree and
//     writes one partial per (pair, level, segment).
//   * After every row's products the ten running sums of each level are tied
//     to that point of the program (an empty asm that reads and writes them),
//     which keeps the compiler from deferring the products of many rows and
//     keeping all their derivatives alive at once.
//
// Units inside the kernel at level l (U = block sums of 4^l base pixels of S or D):
//   hx = 2^(3l+2) E_x (per base px), hy likewise, ht = 2^(2l+2) E_t,
//   g = x_l hx + y_l hy = 2^(2l+2) G with x_l, y_l the cube centre in level pixels.
#include <math.h>

#include <type_traits>

#include "ttc_common.hpp"

#if !defined(TC_FUSED_DT) || !defined(TC_FUSED_LV)
#error "ttc_fused.hip is built once per frame type (TC_FUSED_DT) and level count (TC_FUSED_LV)"
#endif

namespace ttc {
namespace fused {
namespace {

using T = std::conditional_t<TC_FUSED_DT == 0, uint8_t, _Float16>;
constexpr int LV = TC_FUSED_LV;
static_assert(LV >= 1 && LV <= 4, "one to four levels");
constexpr int kGroup = 8;             // rows per unrolled group (one level-3 row)
constexpr int kHalo = 1 << (LV - 1);  // rows walked past the band
constexpr int NV = LV * 10;           // running sums per lane

// Temporal sum and difference of eight pixels of two frames, S = a + b and
// D = b - a in FP32, each one FMA by `one` = 1.0 held in a register, so that
// the multiply is not folded away.  u8: exact byte conversions and exact sums
// (written as plain adds, the compiler turns them into integer adds and then
// converts every value derived from them, several times the conversions).
// f16: one mixed-precision FMA each (both halves converted exactly, one
// rounding).
__device__ __forceinline__ void sum_diff(const Raw8<uint8_t>& a, const Raw8<uint8_t>& b, float (&S)[8],
                                         float (&D)[8], float one) {
  float av[8], bv[8];
  a.unpack(av);
  b.unpack(bv);
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    S[c] = __builtin_fmaf(bv[c], one, av[c]);
    D[c] = __builtin_fmaf(bv[c], one, -av[c]);
  }
}
__device__ __forceinline__ void sum_diff(const Raw8<_Float16>& a, const Raw8<_Float16>& b, float (&S)[8],
                                         float (&D)[8], float one) {
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const uint32_t sh = 16 * (c & 1);
    const float av = (float)__builtin_bit_cast(_Float16, (uint16_t)(a.d[c >> 1] >> sh));
    const float bv = (float)__builtin_bit_cast(_Float16, (uint16_t)(b.d[c >> 1] >> sh));
    S[c] = __builtin_fmaf(bv, one, av);
    D[c] = __builtin_fmaf(bv, one, -av);
  }
}

// Which cube columns of a lane may need masking.  kEdgeNone: every lane owns
// all or none of its columns at every level.  kEdgeLast: a lane with a partial
// set lacks only its last column at each level (always so when W is a multiple
// of 8: its last base column W - 1 has no right neighbour).  kEdgeAny: any other
// partial set.
enum EdgeMode { kEdgeNone = 0, kEdgeLast = 1, kEdgeAny = 2 };

// How rows and lane chunks are loaded.  kCheckNone: every walked row exists
// with one more below it and chunks are aligned (one vector load each, which
// may run up to 7 pixels past column W).  kCheckRows: the segment reaches the
// bottom of the frame, chunks are aligned, W is a multiple of 8 (no chunk
// passes column W) and every segment of the wave walks the same rows: rows
// past the frame are replaced by its last row and skipped.  kCheckAll:
// anything else (every load checked, partial chunks loaded element by element).
enum CheckMode { kCheckNone = 0, kCheckRows = 1, kCheckAll = 2 };

// Accumulate the cubes of one row of one level.  hd*, hs*, hD* are the horizontal
// quantities of the previous (p) and current level rows.  Cubes at columns
// c >= ncv contribute zero (their derivatives are masked), checked at the
// columns the edge mode EM names.
template <int NC, int EM>
__device__ __forceinline__ void cubes(float (&acc)[10], const float (&hdp)[NC], const float (&hd)[NC],
                                      const float (&hsp)[NC], const float (&hs)[NC], const float (&hDp)[NC],
                                      const float (&hD)[NC], int ncv, const float (&xc)[NC], float y) {
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    float ex = hdp[c] + hd[c];
    float ey = hs[c] - hsp[c];
    float et = hDp[c] + hD[c];
    if (EM == kEdgeAny || (EM == kEdgeLast && NC > 1 && c == NC - 1)) {
      const bool ok = c < ncv;
      ex = ok ? ex : 0.f;
      ey = ok ? ey : 0.f;
      et = ok ? et : 0.f;
    }
    const float g = fmaf(y, ey, xc[c] * ex);
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
  // the row's contribution is complete here (see the file comment)
#pragma unroll
  for (int q = 0; q < 10; ++q) asm volatile("" : "+v"(acc[q]));
}

// Value of lane i + 1 of the wave (DPP wave_shl:1); lane 63 receives 0.
__device__ __forceinline__ float from_right(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}

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

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// Which group of the band a row group is: the first (rows 0..7), one inside
// the band, or the halo past it.  It decides, at compile time, which of the
// level rows formed in the group close an owned cube row: a level-l cube row
// lr (between level rows lr - 1 and lr) belongs to the band when
// 1 <= lr <= RB / 2^l.
enum GroupKind { kFirst = 0, kInner = 1, kHaloGroup = 2 };

template <int KIND>
__device__ __forceinline__ constexpr bool owns(int j, int l) {
  // j: row within the group; a level-l row is formed when (j + 1) % 2^l == 0
  if (KIND == kFirst) return (j >> l) >= 1;
  if (KIND == kInner) return true;
  return (j >> l) == 0;  // halo: only the cube row closing on the band's last level row
}

// The walk state of one band: the previous level rows' horizontal quantities,
// the running sums, and the ordinate of the current group's first row per level.
struct Walk {
  float acc[LV][10];
  float hs0p[8], hd0p[8], hD0p[8];
  float hs1p[4], hd1p[4], hD1p[4];
  float hs2p[2], hd2p[2], hD2p[2];
  float hs3p[1], hd3p[1], hD3p[1];
  float y[LV];
};

// One group of NJ (<= 8) rows.  a[j], b[j] hold row j of the pair's two frames;
// refill(a[j], b[j], j) loads row j of the next group into them once row j's S
// and D are formed.  CK != kCheckNone: rows j >= rows_left do not exist (the
// bottom band) and add no cubes.
template <int KIND, int NJ, int EM, int CK, typename REFILL>
__device__ __forceinline__ void walk_group(Walk& s, Raw8<T> (&a)[kGroup], Raw8<T> (&b)[kGroup], REFILL&& refill,
                                           int rows_left, const int (&ncv)[LV], const float (&xc0)[8],
                                           const float (&xc1)[4], const float (&xc2)[2], const float (&xc3)[1],
                                           float one) {
  static_for<0, NJ>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    float S[8], D[8];
    sum_diff(a[j], b[j], S, D, one);
    // the row's registers are free only now: keep the refill behind the reads
    // (a load hoisted above them would need other registers, and a copy back
    // at the loop's back edge that waits for every load in flight)
    asm volatile("" ::"v"(S[7]), "v"(D[7]), "v"(S[6]), "v"(D[6]) : "memory");
    refill(a[j], b[j], j);
    // a row past the frame (and every row after it) adds no cube: only the
    // sums are guarded, the walk state is updated regardless (nothing real
    // reads it afterwards), so the guard costs no copies of that state
    const bool live = CK == kCheckNone || j < rows_left;
    float hs0[8], hd0[8], hD0[8];
    horizontals<8>(S, D, hs0, hd0, hD0);
    if constexpr (owns<KIND>(j, 0))
      if (live) cubes<8, EM>(s.acc[0], s.hd0p, hd0, s.hs0p, hs0, s.hD0p, hD0, ncv[0], xc0, s.y[0] + (float)j);
    if constexpr (LV >= 2 && (j & 1) == 1) {
      float U1[4], V1[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        U1[c] = s.hs0p[2 * c] + hs0[2 * c];
        V1[c] = s.hD0p[2 * c] + hD0[2 * c];
      }
      float hs1[4], hd1[4], hD1[4];
      horizontals<4>(U1, V1, hs1, hd1, hD1);
      if constexpr (owns<KIND>(j, 1))
        if (live) cubes<4, EM>(s.acc[1], s.hd1p, hd1, s.hs1p, hs1, s.hD1p, hD1, ncv[1], xc1, s.y[1] + (float)(j >> 1));
      if constexpr (LV >= 3 && (j & 3) == 3) {
        float U2[2], V2[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          U2[c] = s.hs1p[2 * c] + hs1[2 * c];
          V2[c] = s.hD1p[2 * c] + hD1[2 * c];
        }
        float hs2[2], hd2[2], hD2[2];
        horizontals<2>(U2, V2, hs2, hd2, hD2);
        if constexpr (owns<KIND>(j, 2))
          if (live) cubes<2, EM>(s.acc[2], s.hd2p, hd2, s.hs2p, hs2, s.hD2p, hD2, ncv[2], xc2, s.y[2] + (float)(j >> 2));
        if constexpr (LV >= 4 && (j & 7) == 7) {
          float U3[1], V3[1];
          U3[0] = s.hs2p[0] + hs2[0];
          V3[0] = s.hD2p[0] + hD2[0];
          float hs3[1], hd3[1], hD3[1];
          horizontals<1>(U3, V3, hs3, hd3, hD3);
          if constexpr (owns<KIND>(j, 3))
            if (live) cubes<1, EM>(s.acc[3], s.hd3p, hd3, s.hs3p, hs3, s.hD3p, hD3, ncv[3], xc3, s.y[3]);
          s.hs3p[0] = hs3[0];
          s.hd3p[0] = hd3[0];
          s.hD3p[0] = hD3[0];
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          s.hs2p[c] = hs2[c];
          s.hd2p[c] = hd2[c];
          s.hD2p[c] = hD2[c];
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        s.hs1p[c] = hs1[c];
        s.hd1p[c] = hd1[c];
        s.hD1p[c] = hD1[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      s.hs0p[c] = hs0[c];
      s.hd0p[c] = hd0[c];
      s.hD0p[c] = hD0[c];
    }
  });
  // the next group's first row, per level
#pragma unroll
  for (int l = 0; l < LV; ++l) s.y[l] += (float)(kGroup >> l);
}

// Adds the register block of running sums into the lane's own LDS slots
// (read, FP32 add, write back; no other lane touches them) and clears it, so
// that each FP32 register block holds at most 16 rows of products.
__device__ __forceinline__ void flush(Walk& s, float* tot, int lane) {
  float t[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) t[i] = tot[i * 64 + lane];
#pragma unroll
  for (int i = 0; i < NV; ++i) tot[i * 64 + lane] = t[i] + s.acc[i / 10][i % 10];
#pragma unroll
  for (int l = 0; l < LV; ++l)
#pragma unroll
    for (int q = 0; q < 10; ++q) s.acc[l][q] = 0.f;
}

// One wave, one pair, the lane's own segment: rows row0 .. row0 + RB + kHalo - 1
// (fewer at the bottom of the frame) of columns c_lane .. c_lane + 7; `owner`:
// the lane owns the cubes of its columns (not a lending lane).  EM: the edge
// mode (which cube columns are masked); CK: the check mode of the loads.
// Leaves the lane's sums in tot[(l * 10 + q) * 64 + lane] (zero for a level at
// which the lane owns no cube).
template <int EM, int CK>
__device__ __forceinline__ void band_pair(const SeqDesc& d, int pair, int row0, int RB, int c_lane, bool owner,
                                          int lane, float* tot, float one) {
  const int H = d.H, W = d.W;
  const int NW = RB + kHalo;  // rows walked
  // valid cube columns of this lane per level, and the cube-centre coordinates
  int ncv[LV];
  Walk s;
#pragma unroll
  for (int l = 0; l < LV; ++l) {
    const int j0 = c_lane >> l;
    int n = (W >> l) - 1 - j0;
    n = n < 0 ? 0 : (n > (8 >> l) ? (8 >> l) : n);
    ncv[l] = owner ? n : 0;
    // ordinate of the cube row closing on the band's first level row: the cube
    // between level rows i - 1 and i has its centre at 2^l i - H/2 base pixels
    s.y[l] = (float)(row0 >> l) - (float)H / (float)(2 << l);
  }
  auto xbase = [&](int l) { return (float)((c_lane >> l) + 1) - (float)W / (float)(2 << l); };
  float xc0[8], xc1[4], xc2[2], xc3[1];
#pragma unroll
  for (int c = 0; c < 8; ++c) xc0[c] = xbase(0) + (float)c;
#pragma unroll
  for (int c = 0; c < 4; ++c) xc1[c] = xbase(1) + (float)c;
#pragma unroll
  for (int c = 0; c < 2; ++c) xc2[c] = xbase(2) + (float)c;
  xc3[0] = xbase(3);

  const int ncols = W - c_lane;  // pixels of this lane inside the image
  // Lanes right of the image read the last aligned chunk of the row instead:
  // every load is unconditional, and what those lanes hold only reaches cubes
  // that are not valid.
  const int c_load = c_lane < W ? c_lane : ((W - 1) >> 3) << 3;
  const uint32_t coff = (uint32_t)c_load * (uint32_t)sizeof(T);
  const int64_t rs_b = d.row_stride * (int64_t)sizeof(T);
  // the segment's first row of each frame
  const char* fa = reinterpret_cast<const char*>(d.frame0) +
                   ((int64_t)pair * d.frame_stride + (int64_t)row0 * d.row_stride) * (int64_t)sizeof(T);
  const char* fb = fa + d.frame_stride * (int64_t)sizeof(T);
  // rows of this segment that exist, walked: owned rows plus the halo (the
  // same in every lane of the wave with the rows-only check)
  int n_rows = (H - row0 < NW) ? H - row0 : NW;
  if constexpr (CK == kCheckRows) n_rows = __builtin_amdgcn_readfirstlane(n_rows);

  auto load_row = [&](Raw8<T>& r, const char* base, int w) {
    const T* p = reinterpret_cast<const T*>(base + (int64_t)w * rs_b + coff);
    if constexpr (CK == kCheckNone) {
      r.load(p);
    } else if constexpr (CK == kCheckRows) {
      // rows past the frame repeat its last row (loaded, then skipped)
      r.load(reinterpret_cast<const T*>(base + (int64_t)min(w, n_rows - 1) * rs_b + coff));
    } else {
      const int row = row0 + w;
      if (w < n_rows && ncols > 0) {
        // a vector load may overrun column W only where a next row exists
        if (d.vec && (ncols >= 8 || row < H - 1)) r.load(p);
        else r.load_partial(p, ncols < 8 ? ncols : 8);
      } else {
        r.zero();
      }
    }
  };

#pragma unroll
  for (int l = 0; l < LV; ++l)
#pragma unroll
    for (int q = 0; q < 10; ++q) s.acc[l][q] = 0.f;
#pragma unroll
  for (int i = 0; i < NV; ++i) tot[i * 64 + lane] = 0.f;

  // the ring: rows 0..7, then each row j replaced by row j + 8 once read; the
  // rows refilled in the last inner group are the halo's (a row index past the
  // walk is clamped to its last row: loaded, never used)
  Raw8<T> a[kGroup], b[kGroup];
#pragma unroll
  for (int j = 0; j < kGroup; ++j) {
    load_row(a[j], fa, j);
    load_row(b[j], fb, j);
  }
  int gw = kGroup;  // first row of the next group
  auto refill = [&](Raw8<T>& ra, Raw8<T>& rb, int j) {
    const int w = gw + j < NW ? gw + j : NW - 1;
    load_row(ra, fa, w);
    load_row(rb, fb, w);
  };
  auto none = [&](Raw8<T>&, Raw8<T>&, int) {};

  walk_group<kFirst, kGroup, EM, CK>(s, a, b, refill, n_rows, ncv, xc0, xc1, xc2, xc3, one);
  // groups 1 .. inner_end - 1 lie inside the band, group inner_end is the halo
  const int inner_end = RB / kGroup;
  if constexpr (CK == kCheckRows) {
    // one row count for the wave: the groups inside the frame take the
    // unchecked code, the group holding its last row the checked one, and the
    // walk ends there (the loads it leaves in flight are never read)
    const int g_full = min(inner_end, n_rows / kGroup);
    int g = 1;
    for (; g < g_full; ++g) {
      gw += kGroup;
      walk_group<kInner, kGroup, EM, kCheckNone>(s, a, b, refill, n_rows - g * kGroup, ncv, xc0, xc1, xc2, xc3,
                                                 one);
      if (g & 1) flush(s, tot, lane);
    }
    if (g < inner_end && n_rows > g * kGroup) {
      gw += kGroup;
      walk_group<kInner, kGroup, EM, kCheckRows>(s, a, b, refill, n_rows - g * kGroup, ncv, xc0, xc1, xc2, xc3,
                                                 one);
    }
    if (n_rows > inner_end * kGroup)
      walk_group<kHaloGroup, kHalo, EM, kCheckRows>(s, a, b, none, n_rows - inner_end * kGroup, ncv, xc0, xc1, xc2,
                                                    xc3, one);
  } else {
    for (int g = 1; g < inner_end; ++g) {
      gw += kGroup;
      walk_group<kInner, kGroup, EM, CK>(s, a, b, refill, n_rows - g * kGroup, ncv, xc0, xc1, xc2, xc3, one);
      if (g & 1) flush(s, tot, lane);
    }
    walk_group<kHaloGroup, kHalo, EM, CK>(s, a, b, none, n_rows - inner_end * kGroup, ncv, xc0, xc1, xc2, xc3,
                                          one);
  }
  // lanes that own no cube of a level contribute zero
#pragma unroll
  for (int l = 0; l < LV; ++l) {
    if (ncv[l] == 0) {
#pragma unroll
      for (int q = 0; q < 10; ++q) s.acc[l][q] = 0.f;
    }
  }
  flush(s, tot, lane);
#pragma unroll
  for (int l = 0; l < LV; ++l) {
    if (ncv[l] == 0) {
#pragma unroll
      for (int q = 0; q < 10; ++q) tot[(l * 10 + q) * 64 + lane] = 0.f;
    }
  }
}

// Sums of one segment's owning lanes, for value i: a pairwise tree over S
// slots (S >= the segment's lanes), the slots past its n owning lanes adding 0.
template <int S>
__device__ __forceinline__ float segment_sum(const float* tot, int i, int base, int n) {
  float v[S / 2];
#pragma unroll
  for (int m = 0; m < S / 2; ++m) {
    const float x0 = tot[i * 64 + min(base + 2 * m, 63)];
    const float x1 = tot[i * 64 + min(base + 2 * m + 1, 63)];
    v[m] = (2 * m < n ? x0 : 0.f) + (2 * m + 1 < n ? x1 : 0.f);
  }
#pragma unroll
  for (int w = S / 4; w >= 1; w >>= 1)
#pragma unroll
    for (int m = 0; m < w; ++m) v[m] = v[2 * m] + v[2 * m + 1];
  return v[0];
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void ttc_fused(FusedArgs a, int RB) {
  __shared__ float tot[NV * 64];  // each lane's running sums, [value][lane]
  const int lane = threadIdx.x;

  const int G = gridDim.x;
  const int g = blockIdx.x;
  // XCD-aware order: work-groups are dealt to the 8 XCDs round-robin, so give
  // each XCD a contiguous run of items (the pairs of the same segments, and
  // vertically adjacent bands, which share frames and halo rows).
  const int64_t slot = (G % 8 == 0) ? (int64_t)(g % 8) * (G / 8) + g / 8 : g;

  for (int64_t t = 0;; ++t) {
    const int64_t item = t * G + slot;
    if (item >= a.n_items) break;
    const SeqDesc d = uniform(seq_for_item(a, item));
    const int64_t local = item - d.item_begin;  // = wave * n_pairs + pair
    const int n_pairs = d.n_frames - 1;
    const int wv = (int)(local / n_pairs);
    const int pair = (int)(local - (int64_t)wv * n_pairs);
    // this lane's segment: k-th of the wave, lane li within it (the last lends)
    const int SL = d.seg_lanes, SPW = d.seg_per_wave;
    const int k = lane / SL;
    const int li = lane - k * SL;
    const int sid = wv * SPW + k;
    const bool seg_ok = k < SPW && sid < d.n_segs;
    const int sidc = seg_ok ? sid : wv * SPW;  // lanes past the segments walk the first one's rows
    // the full bands strip-major, then the bottom bands band-major
    const int n_full = d.n_strips * d.n_full_bands;
    int strip, band;
    if (sidc < n_full) {
      strip = sidc / d.n_full_bands;
      band = sidc - strip * d.n_full_bands;
    } else {
      const int r = sidc - n_full;
      const int bb = r / d.n_strips;
      band = d.n_full_bands + bb;
      strip = r - bb * d.n_strips;
    }
    const int row0 = band * RB;
    const int c_lane = strip * d.seg_cols + li * 8;
    const bool owner = seg_ok && li < SL - 1;
    // vector loads are safe when every walked row exists with one more below
    // it (a lane chunk may run up to 7 pixels past column W)
    const int64_t below = (int64_t)d.H - row0 - (RB + kHalo);
    // rows walked by the lane's segment: the rows-only check needs one number
    // for the whole wave (its row skips are then uniform branches)
    const int nr = min(d.H - row0, RB + kHalo);
    const bool same_rows = !__any(nr != __builtin_amdgcn_readfirstlane(nr));
    const int ck = !__any(!(d.vec && below >= 1))          ? kCheckNone
                   : (d.vec && (d.W & 7) == 0 && same_rows) ? kCheckRows
                                                            : kCheckAll;
    // some lane owns a partial set of cube columns at some level; `other`: one
    // that lacks more than its last column there (never when W % 8 == 0)
    bool edge = false, other = false;
#pragma unroll
    for (int l = 0; l < LV; ++l) {
      const int n = (d.W >> l) - 1 - (c_lane >> l);
      const bool part = owner && n > 0 && n < (8 >> l);
      edge = edge || part;
      other = other || (part && n != (8 >> l) - 1);
    }
    const int em = __any(other) ? kEdgeAny : (__any(edge) ? kEdgeLast : kEdgeNone);
#define TC_BAND(E, C) band_pair<E, C>(d, pair, row0, RB, c_lane, owner, lane, tot, a.one)
    if (em == kEdgeNone) {
      if (ck == kCheckNone) TC_BAND(kEdgeNone, kCheckNone);
      else if (ck == kCheckRows) TC_BAND(kEdgeNone, kCheckRows);
      else TC_BAND(kEdgeNone, kCheckAll);
    } else if (em == kEdgeLast) {
      if (ck == kCheckNone) TC_BAND(kEdgeLast, kCheckNone);
      else if (ck == kCheckRows) TC_BAND(kEdgeLast, kCheckRows);
      else TC_BAND(kEdgeLast, kCheckAll);
    } else {
      // W % 8 != 0 here, so the rows-only check never applies
      if (ck == kCheckNone) TC_BAND(kEdgeAny, kCheckNone);
      else TC_BAND(kEdgeAny, kCheckAll);
    }
#undef TC_BAND

    // One partial per (pair, level, segment): reduction lane r takes value
    // i = r mod 10 LV of segment r div 10 LV and adds that segment's owning
    // lanes in a pairwise tree (at most 6 rounded additions deep).
    __syncthreads();  // every lane's slots are written
    float* part = a.partials + d.partial_begin;
    for (int r = lane; r < NV * SPW; r += 64) {
      const int ks = r / NV;
      const int i = r - ks * NV;
      float sum;
      if (SL <= 16) sum = segment_sum<16>(tot, i, ks * SL, SL - 1);
      else if (SL <= 32) sum = segment_sum<32>(tot, i, ks * SL, SL - 1);
      else sum = segment_sum<64>(tot, i, ks * SL, SL - 1);
      const int s2 = wv * SPW + ks;
      if (s2 < d.n_segs) {
        const int l = i / 10, q = i - (i / 10) * 10;
        as_global(part)[((int64_t)(pair * LV + l) * d.n_segs + s2) * 10 + q] = sum;
      }
    }
    __syncthreads();  // the slots are read before the next item clears them
  }
}

}  // namespace

#define TC_CAT3(a, b, c) a##b##c
#define TC_LAUNCHER(dt, lv) TC_CAT3(launch_ttc_fused_dt, dt, _l##lv)
#define TC_LAUNCHER_X(dt, lv) TC_LAUNCHER(dt, lv)

hipError_t TC_LAUNCHER_X(TC_FUSED_DT, TC_FUSED_LV)(const FusedLaunch& f, hipStream_t s) {
  if (f.band_rows < 16 || f.band_rows > 256 || f.band_rows % 16 != 0) return hipErrorInvalidValue;
  const FusedArgs a = make_args(f);
  hipLaunchKernelGGL(ttc_fused, dim3((unsigned)f.grid), dim3(64), 0, s, a, f.band_rows);
  return hipGetLastError();
}

}  // namespace fused
}  // namespace ttc
