// Host-side declarations of the fused time-to-contact pass: the device work
// table, the launch description and the launchers.  Shared by the C ABI
// (ttcconv.cpp), the fused pass (ttc_fused.hip) and its finishing pass
// (ttc.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ttcconv.h"

namespace ttc {

// One entry of the device work table: a video stream and where its work and
// results go.  The fused pass covers each frame pair of the stream with
// segments of `band_rows` base rows by `seg_cols` owned base columns; a
// segment occupies seg_cols / 8 lanes that own 8 base columns each and one more
// that only lends its first column to the lane before it.  A work item is one
// wave and one pair: `seg_per_wave` consecutive segments side by side in its
// lanes.  Segments are numbered first over the bands whose walk (owned rows and
// 2^(levels-1) halo rows) has a row of the frame below it, column-strip-major
// and band-minor, then over the remaining bottom bands, band-major, so that the
// waves that reach the bottom of the frame hold segments of one height.  Items
// are numbered wave-major, pair-minor, so that the items of consecutive pairs
// over the same segments are adjacent.
struct SeqDesc {
  const void* frame0;
  int64_t frame_stride;   // elements
  int64_t row_stride;     // elements
  int32_t H, W;
  int32_t n_frames;
  int32_t levels;
  int32_t band_rows;      // owned base rows per segment
  int32_t n_bands;        // ceil(H / band_rows)
  int32_t seg_cols;       // owned base columns per segment (a multiple of 8, at most 504)
  int32_t seg_lanes;      // lanes per segment: seg_cols / 8 + 1
  int32_t seg_per_wave;   // segments per wave: floor(64 / seg_lanes)
  int32_t n_waves;        // work items per pair: ceil(n_segs / seg_per_wave)
  int32_t n_segs;         // segments (column strips x bands): partial sums per (pair, level)
  int32_t n_strips;       // column strips: ceil((W - 1) / seg_cols)
  int32_t n_full_bands;   // leading bands whose walk has a row of the frame below it
  int32_t vec;            // 1: every 8-pixel lane chunk is aligned for one vector load
  int32_t pad;
  int64_t item_begin;     // first work item of this stream (prefix over streams)
  int64_t pair_begin;     // first global pair index of this stream
  int64_t partial_begin;  // first float of this stream's partial sums
};

struct FusedLaunch {
  int dt;           // TC_U8 or TC_F16
  int levels;       // 1..4
  int band_rows;    // 8, 16 or 32
  const SeqDesc* table;  // device table, or nullptr to use `inl`
  const int32_t* item_seq;  // stream of every work item (with `table`)
  const int32_t* pair_seq;  // stream of every pair (with `table`)
  int n_seqs;
  SeqDesc inl;
  int64_t n_items;
  int64_t n_pairs;
  float* partials;
  int grid;         // persistent grid size (work-groups)
};

hipError_t launch_ttc_fused(const FusedLaunch& f, hipStream_t s);
namespace fused {
// One launcher per frame type (dt0 = u8, dt1 = f16) and level count, each built
// from ttc_fused.hip in an object of its own.
hipError_t launch_ttc_fused_dt0_l1(const FusedLaunch& f, hipStream_t s);
hipError_t launch_ttc_fused_dt0_l2(const FusedLaunch& f, hipStream_t s);
hipError_t launch_ttc_fused_dt0_l3(const FusedLaunch& f, hipStream_t s);
hipError_t launch_ttc_fused_dt0_l4(const FusedLaunch& f, hipStream_t s);
hipError_t launch_ttc_fused_dt1_l1(const FusedLaunch& f, hipStream_t s);
hipError_t launch_ttc_fused_dt1_l2(const FusedLaunch& f, hipStream_t s);
hipError_t launch_ttc_fused_dt1_l3(const FusedLaunch& f, hipStream_t s);
hipError_t launch_ttc_fused_dt1_l4(const FusedLaunch& f, hipStream_t s);
}  // namespace fused
hipError_t launch_ttc_finish(const FusedLaunch& f, tc_ttc_level* out, tc_ttc_pick* picks, hipStream_t s);
bool fused_variant_exists(int dt, int levels, int band_rows);
hipError_t launch_ttc_reselect(const tc_ttc_level* levels, int64_t n_pairs, int L, int rule, tc_ttc_pick* picks,
                              hipStream_t s);

}  // namespace ttc
