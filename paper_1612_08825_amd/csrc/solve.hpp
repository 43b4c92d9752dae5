// The 3x3 solve of one level's normal equations and the key of the
// multi-scale rule, shared by the fused and the decomposed TTC paths.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/ttcconv.h"

namespace ttc {

// Time to Contact, Formulation: the normal equations
//   [S(ExEx) S(ExEy) S(GEx)] [A]     [S(ExEt)]
//   [S(ExEy) S(EyEy) S(GEy)] [B] = - [S(EyEt)]
//   [S(GEx)  S(GEy)  S(GG) ] [C]     [S(GEt) ]
// solved in FP64 by Gaussian elimination with partial pivoting on the
// equilibrated matrix D M D, D = diag(M_ii^-1/2); singular when a diagonal
// entry is not positive or an equilibrated pivot falls below 1e-6.  FOE
// x0 = -A/C, y0 = -B/C, TTC = 1/C, residual S(EtEt) + A S(ExEt) + B S(EyEt) +
// C S(GEt).  s holds the ten sums in the order of tc_ttc_level.sums.
#pragma clang fp contract(off)
static __device__ void solve_level(const double* s, tc_ttc_level& r) {
  const double nan = __builtin_nan("");
  for (int q = 0; q < TC_NUM_SUMS; ++q) r.sums[q] = s[q];
  r.A = r.B = r.C = r.ttc = r.x0 = r.y0 = r.resid = nan;
  r.status = TC_OK;
  for (int q = 0; q < TC_NUM_SUMS; ++q)
    if (!isfinite(s[q])) {
      r.status = TC_NONFINITE;
      return;
    }
  double M[3][4] = {{s[0], s[1], s[3], -s[6]}, {s[1], s[2], s[4], -s[7]}, {s[3], s[4], s[5], -s[8]}};
  if (M[0][0] <= 0.0 || M[1][1] <= 0.0 || M[2][2] <= 0.0) {
    r.status = TC_SINGULAR;
    return;
  }
  double dg[3];
  for (int i = 0; i < 3; ++i) dg[i] = 1.0 / sqrt(M[i][i]);
  double a[3][4];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) a[i][j] = dg[i] * M[i][j] * dg[j];
    a[i][3] = dg[i] * M[i][3];
  }
  double minpiv = 1e300;
  for (int c = 0; c < 3; ++c) {
    int p = c;
    for (int i = c + 1; i < 3; ++i)
      if (fabs(a[i][c]) > fabs(a[p][c])) p = i;
    if (p != c)
      for (int j = 0; j < 4; ++j) {
        const double t = a[c][j];
        a[c][j] = a[p][j];
        a[p][j] = t;
      }
    const double piv = a[c][c];
    minpiv = fmin(minpiv, fabs(piv));
    if (piv == 0.0) break;
    for (int i = c + 1; i < 3; ++i) {
      const double f = a[i][c] / piv;
      for (int j = c; j < 4; ++j) a[i][j] = a[i][j] - f * a[c][j];
    }
  }
  if (!(minpiv >= 1e-6)) {
    r.status = TC_SINGULAR;
    return;
  }
  double v[3];
  for (int i = 2; i >= 0; --i) {
    double acc = a[i][3];
    for (int j = i + 1; j < 3; ++j) acc = acc - a[i][j] * v[j];
    v[i] = acc / a[i][i];
  }
  const double A = dg[0] * v[0], B = dg[1] * v[1], C = dg[2] * v[2];
  r.A = A;
  r.B = B;
  r.C = C;
  if (C == 0.0) {
    r.ttc = copysign(__builtin_inf(), C);
  } else {
    r.ttc = 1.0 / C;
    r.x0 = -A / C;
    r.y0 = -B / C;
  }
  r.resid = s[9] + A * s[6] + B * s[7] + C * s[8];
}
#pragma clang fp contract(on)

// Multi-scale key: the TTC, or +inf for a level that is singular, non-finite
// or not positive (any valid estimate improves on an invalid one).
__device__ __forceinline__ double level_key(const tc_ttc_level& r) {
  if (r.status != TC_OK || !isfinite(r.ttc) || !(r.ttc > 0.0)) return __builtin_inf();
  return r.ttc;
}

}  // namespace ttc
