// Pieces shared by the fused time-to-contact pass (ttc_fused.hip) and its
// finishing pass (ttc.hip): the kernel arguments, uniform copies of a stream
// descriptor, and the lookup of a work item's or a pair's stream.
#pragma once

#include "device_common.hpp"
#include "fused.hpp"

namespace ttc {
namespace fused {

struct FusedArgs {
  const SeqDesc* table;
  const int32_t* item_seq;
  const int32_t* pair_seq;
  int n_seqs;
  SeqDesc inl;
  int64_t n_items;
  int64_t n_pairs;
  float* partials;
  float one;  // 1.0, passed in so that mixed-precision FMAs by one are not folded away
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
  d.seg_cols = uni(s.seg_cols);
  d.seg_lanes = uni(s.seg_lanes);
  d.seg_per_wave = uni(s.seg_per_wave);
  d.n_waves = uni(s.n_waves);
  d.n_segs = uni(s.n_segs);
  d.n_strips = uni(s.n_strips);
  d.n_full_bands = uni(s.n_full_bands);
  d.vec = uni(s.vec);
  d.pad = 0;
  d.item_begin = uni(s.item_begin);
  d.pair_begin = uni(s.pair_begin);
  d.partial_begin = uni(s.partial_begin);
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


// Scale exponents of the un-normalised sums of level l: hx, hy carry
// 2^(3l+2), g and ht carry 2^(2l+2).
__device__ __forceinline__ int sum_scale_exp(int l, int q) {
  switch (q) {
    case 0: case 1: case 2: return 6 * l + 4;
    case 3: case 4: case 6: case 7: return 5 * l + 4;
    default: return 4 * l + 4;
  }
}

inline FusedArgs make_args(const FusedLaunch& f) {
  FusedArgs a;
  a.table = f.table;
  a.item_seq = f.item_seq;
  a.pair_seq = f.pair_seq;
  a.n_seqs = f.n_seqs;
  a.inl = f.inl;
  a.n_items = f.n_items;
  a.n_pairs = f.n_pairs;
  a.partials = f.partials;
  a.one = 1.0f;
  return a;
}

}  // namespace fused
}  // namespace ttc
