// Host-side declarations shared by the C ABI (ttcconv.cpp) and the kernel
// launchers (*.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ttcconv.h"
#include "fused.hpp"

namespace ttc {

// ---------------------------------------------------------------- convolution
struct ConvND {
  int ndim;
  int xdt;                      // TC_F32, TC_F16 or TC_U8
  const void* x;
  int64_t xshape[TC_MAX_DIMS];
  int64_t xstride[TC_MAX_DIMS];
  const void* k;                // contiguous, F32 or I32
  int64_t kshape[TC_MAX_DIMS];
  void* y;                      // F32 or I32
  int64_t yshape[TC_MAX_DIMS];
  int64_t ystride[TC_MAX_DIMS];
  int64_t off[TC_MAX_DIMS];     // output index n maps to full index n + off
  int band_rows;                // row-streaming kernels: output rows per wave (2, 4, 8; 0 = the default)
};

// Chooses a kernel (2-D tiled, 3-D tiled, or generic rank-n) and launches it.
hipError_t launch_conv(const ConvND& c, bool small_taps, hipStream_t s);

// The two factors of a separable kernel: device arrays, or (byval) the values
// themselves carried in the kernel arguments (at most 16 taps each).
struct SepTaps {
  const float* u;    // K taps along the columns (device)
  const float* v;    // K taps along the rows (device)
  float uh[16];
  float vh[16];
  int byval;
};

// A 2-D FP32 convolution with a separable square kernel u v^T (K taps each).
struct SepConv {
  const float* x;
  int64_t xs0;       // row stride (elements); unit stride along rows
  int H, W;
  SepTaps taps;
  int K;
  float* y;
  int64_t ys0;
  int OH, OW;
  int off0, off1;    // output index n maps to full index n + off
};
bool separable_variant(int K);
hipError_t launch_conv_separable(const SepConv& c, hipStream_t s);

// FFT branch of 2-D and 3-D FP32 convolution: x (strided) and k (contiguous)
// zero-padded to a volume n_0 x .. x n_{d-1} (d = rank, leading axis first)
// whose extents are at most kFftMaxN.  ax[a] is the transform plan of axis a
// (n = product of the stage radices 2, 3, 4, 5), except that the last axis is
// real: its padded extent is 2 ax[d-1].n, transformed as ax[d-1].n complex
// points and stored as ax[d-1].n + 1 frequencies.  Per-axis twiddle tables
// tw[a] (n_a entries; 2 ax[d-1].n for the last axis); A, B and C are complex
// volumes of the stored spectrum (scratch, the spectrum of x, the spectrum of
// k); the output y (strided) is full index n + o.
constexpr int kFftMaxN = 4096;
constexpr int kFftMaxStages = 12;
struct FftAxis {
  int n;
  int n_stages;
  int8_t radix[kFftMaxStages];  // n = product of radix[0 .. n_stages-1]
};
struct FftConv {
  int rank;
  const float* x;
  int64_t xs[3];
  int xn[3];
  const float* k;
  int kn[3];
  FftAxis ax[3];
  float2* tw[3];
  float2 *A, *B, *C;
  float* y;
  int64_t ys[3];
  int yn[3], o[3];
};
hipError_t launch_conv_fft(const FftConv& f, hipStream_t s);

// Zero `bytes` (a multiple of 4) of device memory with a kernel (graph-safe).
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);

// ---------------------------------------------------------------- gradient
struct GradOut {
  float* ex;  int64_t ex0, ex1;  // each output may be null (not written)
  float* ey;  int64_t ey0, ey1;
  float* mag; int64_t mag0, mag1;
  float* dir; int64_t dir0, dir1;
};

// ---------------------------------------------------------------- pyramid / derivatives
struct Image2D {
  const void* p;
  int dt;
  int64_t s0, s1;  // strides (elements)
};

hipError_t launch_gradient(const Image2D& src, int stencil, int Ho, int Wo, const GradOut& o, hipStream_t s);
hipError_t launch_pyramid_level(const Image2D& src, float* dst, int64_t d0, int64_t d1, int Ho, int Wo,
                                hipStream_t s);
// ---------------------------------------------------------------- decomposed TTC (stencil / low-pass variants)
struct VariantLevels {
  int levels;
  int blocks[TC_MAX_LEVELS];        // work-groups of the sums kernel per level
  int64_t part_off[TC_MAX_LEVELS];  // first partial (in units of 10 doubles) per level
  int64_t n[TC_MAX_LEVELS];         // positions summed per level
};
int variant_sum_blocks(int64_t positions);
// The two frames of a pair: sources (any input type, strided) and FP32
// destinations (contiguous rows); [0] the previous frame, [1] the next.
struct VariantPlanes2 {
  const void* p[2];
  int64_t s0[2], s1[2];
};
struct VariantPair2 {
  const float* src[2];
  float* dst[2];
};
// Per level: the two frames' planes (level 0: the frames, input type; above:
// FP32 level images), extents, work-groups and first partial.
struct VariantSumLevels {
  const void* a[TC_MAX_LEVELS];
  const void* b[TC_MAX_LEVELS];
  int64_t s0[2][TC_MAX_LEVELS], s1[2][TC_MAX_LEVELS];
  int Hl[TC_MAX_LEVELS], Wl[TC_MAX_LEVELS], blocks[TC_MAX_LEVELS];
  int64_t part_off[TC_MAX_LEVELS];
};
hipError_t launch_pyramid_pair(const VariantPlanes2& src, int dt, const VariantPair2& io, int Ho, int Wo,
                               hipStream_t s);
hipError_t launch_lowpass3_pair(const VariantPair2& io, int H, int W, hipStream_t s);
hipError_t launch_stencil_sums_levels(int stencil, int dt, const VariantSumLevels& ls, int levels, int H0, int W0,
                                      double* part, hipStream_t s);
hipError_t launch_variant_finish(const double* part, const VariantLevels& lv, tc_ttc_level* out, tc_ttc_pick* pick,
                                 hipStream_t s);

hipError_t launch_horn(const Image2D& prev, const Image2D& next, int H, int W, void* ex, void* ey, void* et,
                       int odt, const int64_t* os0, const int64_t* os1, hipStream_t s);

}  // namespace ttc
