// Finishing pass of the multi-scale time-to-contact path for gfx950, and the
// dispatch of the fused pass (ttc_fused.hip, one object per frame type and
// level count).
//
// What is computed (Time to Contact, Formulation and Results): the fused
// pass leaves, for every (pair, level, wave), FP32 partial sums of the ten
// products; here one work-group per pair combines them in a fixed order with
// TwoSum (hi, lo) compensation, converts to FP64, solves the 3x3 normal
// equations, derives FOE and TTC, and takes the multi-scale level choice.
#include <math.h>

#include "solve.hpp"
#include "ttc_common.hpp"

namespace ttc {
namespace {

using namespace fused;

// ---------------------------------------------------------------- finishing pass

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
        as_global(a.partials + d.partial_begin + (p * LV + l) * (int64_t)d.n_segs * 10);
    for (int w = lane; w < d.n_segs; w += 64) {
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

}  // namespace

bool fused_variant_exists(int dt, int levels, int band_rows) {
  return (dt == TC_U8 || dt == TC_F16) && levels >= 1 && levels <= 4 && band_rows >= 16 && band_rows <= 256 &&
         band_rows % 16 == 0;
}

hipError_t launch_ttc_fused(const FusedLaunch& f, hipStream_t s) {
  if (f.n_items == 0) return hipSuccess;
  using namespace fused;
  if (f.dt == TC_U8) {
    switch (f.levels) {
      case 1: return launch_ttc_fused_dt0_l1(f, s);
      case 2: return launch_ttc_fused_dt0_l2(f, s);
      case 3: return launch_ttc_fused_dt0_l3(f, s);
      case 4: return launch_ttc_fused_dt0_l4(f, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (f.dt == TC_F16) {
    switch (f.levels) {
      case 1: return launch_ttc_fused_dt1_l1(f, s);
      case 2: return launch_ttc_fused_dt1_l2(f, s);
      case 3: return launch_ttc_fused_dt1_l3(f, s);
      case 4: return launch_ttc_fused_dt1_l4(f, s);
      default: return hipErrorInvalidValue;
    }
  }
  return hipErrorInvalidValue;
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
