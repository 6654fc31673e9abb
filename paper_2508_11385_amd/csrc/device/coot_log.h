// coot_log.h — log(x) for binary32, within half a unit in the last place plus
// about 2^-20 units (so never more than 1 ulp from the exact value).
//
// Method: Tang's table-driven logarithm (ACM TOMS 16(4), 1990), carried in
// float-float (double-word binary32) arithmetic:
//   x = 2^e * m with m in [sqrt(1/2), sqrt(2)), F = 1 + j/128 the table point
//   nearest to m (j = -38 .. 54), f = m - F (exact: F/2 <= m <= 2F), and
//   log(x) = e * ln2 + log(F) + log1p(r),  r = f / F,  |r| < 2^-7.5.
// 1. r = rh + rl: rh = fl(f / F), the remainder f - rh * F exact by FMA, rl its
//    quotient by F (relative error of r about 2^-48).
// 2. log1p(r) = r - r^2/2 + r^3/3 + r^4 (-1/4 + r/5 - r^2/6 + r^3/7): r^2 and r^3
//    from exact products, 1/3 as two words, the r^4 tail (below 2^-30 of r) in
//    working precision; truncation after r^7 leaves 2^-55 of r.
// 3. e * ln2 + log(F): e * L1 exact (L1 has 16 significant bits), e * L2 from an
//    exact product, the table value as three words.
// 4. the two double words are added and rounded once.
// Near x = 1 (e = 0, j = 0) log(F) is 0 and the result is log1p(f) itself, so
// there is no cancellation; the relative error stays about 2^-44 everywhere.
// No binary64 operation is used.  Subnormal inputs are scaled by 2^24 first.
//
// Written without HIP-specific calls so that the same code can be compiled for
// the host (tests define __host__ / __device__ / __forceinline__ as empty).
#pragma once
#pragma clang fp contract(off)

#include "coot_exp.h"
#include "log_tables.h"

namespace coot {

__host__ __device__ __forceinline__ float log_lf(float x) {
  if (!(x == x)) return x + x;                                  // NaN
  if (x < 0.0f) return __builtin_nanf("");
  if (x == 0.0f) return -__builtin_huge_valf();                 // log(+-0) = -inf
  if (x == __builtin_huge_valf()) return x;
  int e;
  float m = x_frexp(x, &e);                                     // x = m * 2^e, m in [0.5, 1) (subnormals too)
  if (m < 0.70710678f) {                                        // m into [sqrt(1/2), sqrt(2))
    m = m * 2.0f;
    e -= 1;
  }
  const float jf = x_rint((m - 1.0f) * 128.0f);                 // m - 1 exact (Sterbenz), * 128 exact
  const int j = (int)jf;
  const float F = 1.0f + jf * 0.0078125f;                       // exact
  const float f = m - F;                                        // exact
  // ---- 1. r = f / F = rh + rl ------------------------------------------------------
  const float rh = f / F;
  const float rl = x_fma(-rh, F, f) / F;                        // remainder exact, then divided
  // ---- 2. log1p(r) = lh + ll ---------------------------------------------------------
  float a_hi, a_lo;
  ef_two_prod(rh, rh, a_hi, a_lo);                              // r^2
  a_lo = a_lo + 2.0f * (rh * rl);
  float c_hi, c_lo;
  ef_two_prod(a_hi, rh, c_hi, c_lo);                            // r^3
  c_lo = c_lo + (a_lo * rh + a_hi * rl);
  float d_hi, d_lo;
  ef_two_prod(c_hi, COOT_LOG_S0F, d_hi, d_lo);                  // r^3 / 3
  d_lo = d_lo + (c_hi * COOT_LOG_S1F + c_lo * COOT_LOG_S0F);
  const float tail =
      (a_hi * a_hi) * (-0.25f + rh * (0.2f + rh * (-0.16666667f + rh * 0.14285715f)));
  float lh, e1, e2;
  ef_two_sum(rh, -0.5f * a_hi, lh, e1);
  ef_two_sum(lh, d_hi, lh, e2);
  float ll = ((((tail + d_lo) - 0.5f * a_lo) + rl) + e2) + e1;
  // ---- 3. e * ln2 + log(F) = kh + kl --------------------------------------------------
  const float ef = (float)e;
  const float p = ef * COOT_LOG_L1F;                            // exact
  float q_hi, q_lo;
  ef_two_prod(ef, COOT_LOG_L2F, q_hi, q_lo);
  const float* T = coot_log_tab_f[j - COOT_LOG_JLO];
  float kh, k1, k2;
  ef_two_sum(p, T[0], kh, k1);
  ef_two_sum(kh, q_hi, kh, k2);
  const float kl = ((((T[2] + ef * COOT_LOG_L3F) + q_lo) + T[1]) + k2) + k1;
  // ---- 4. (kh + kl) + (lh + ll), rounded once -----------------------------------------
  float sh, e3;
  ef_two_sum(kh, lh, sh, e3);
  const float sl = (kl + ll) + e3;
  return sh + sl;
}

}  // namespace coot
