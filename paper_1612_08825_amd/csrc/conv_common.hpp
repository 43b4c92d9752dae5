// Pieces shared by the row-streaming convolution kernels (conv.hip: the
// rolling-window and separable FP32 kernels; conv_rows.hip: the unrolled band
// kernel for FP32, FP16 and u8 images).
#pragma once

#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"

namespace ttc {
namespace rows {

typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
template <typename T> using cptr = __attribute__((address_space(4))) const T*;

template <int KW, int S> constexpr int row_chunks() { return (S + KW + 3 + 3) / 4; }
template <int KW, int S> constexpr int row_lanes_out() { return 65 - row_chunks<KW, S>(); }

struct RowArgs {
  const void* x;     // FP32, FP16 or u8 (per kernel)
  int64_t xs0, xsd;  // row and plane strides (elements)
  int H, W, D;
  const void* k;     // contiguous [KD][KH][KW], FP32 or int32
  int KD;
  void* y;           // FP32 or int32
  int64_t ys0, ysd;
  int OH, OW, OD;
  int off0, off1, offd;
  int n_bands, n_cw;
  int64_t n_items;   // OD * n_bands * n_cw
};

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int cmin(int a, int b) { return a < b ? a : b; }

// Buffer resource over `bytes` bytes from `base` (gfx9 raw-buffer word 3:
// 32-bit data format, no swizzle).  A buffer load whose offset is outside the
// range returns zero without touching memory (on this chip the scalar offset
// counts toward the range too).  So with the row start as base, W * 4 bytes as
// range and the column (times 4, as an unsigned 32-bit lane value) as the
// vector offset, every load of a column left or right of the image reads zero.
// (Multi-dword buffer loads are not used: they need aligned offsets.)
constexpr int kBufWord3 = 0x00020000;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufWord3);
}

// Value of lane i + 1 (DPP wave_shl:1, whole wave); lane 63 receives 0.
__device__ __forceinline__ float from_next_lane(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ int from_next_lane(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true); }


// Launch entry of the unrolled band kernel for one input type (conv_rows.hip
// is built once per type): x FP32 (dt 0), FP16 (dt 1) or u8 with int32 taps
// whose magnitudes are below 2^23 (dt 2); KH = KW in {2, 3, 5, 7}.
// band_rows: output rows per wave (2, 4 or 8), 0 for the default table.
hipError_t launch_rows_dt0(const RowArgs& ra, int KH, int band_rows, hipStream_t s);
hipError_t launch_rows_dt1(const RowArgs& ra, int KH, int band_rows, hipStream_t s);
hipError_t launch_rows_dt2(const RowArgs& ra, int KH, int band_rows, hipStream_t s);

}  // namespace rows
}  // namespace ttc
