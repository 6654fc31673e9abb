// coot_exp.h — exp(x) rounded correctly to binary32 / binary64.
//
// Method: Tang's table-driven exponential (ACM TOMS 15(2), 1989), carried in
// double-word arithmetic so that the final rounding can be decided exactly:
//   N = rint(x * 128/ln2), k = N >> 7, j = N & 127, r = x - N * ln2/128,
//   exp(x) = 2^k * 2^(j/128) * exp(r),  |r| <= ln2/256 (+ rounding slack).
// 1. r is formed as a double word (rh + rl) with error-free products (FMA) and
//    sums; ln2/128 is split into three words.
// 2. p = exp(r) - 1 is a double word: r + r^2/2 + r^3/6 from exact products,
//    r^4/24 .. r^7/5040 in working precision (they are below 2^-38).
// 3. V = 2^(j/128) * (1 + p) with the table value as three binary32 words
//    (two binary64 words); V = s + u + w with s, u non-overlapping words and w a
//    small correction.
// 4. y = fl(s + u) and the remainder d = s + u - y are exact (TwoSum); y is moved
//    to its neighbour only if d + w passes half the gap to that neighbour, and
//    when the working-precision test lands exactly on the half gap the sign of
//    the exact difference decides.  Subnormal results round once on the
//    subnormal grid (a midpoint reached by the first rounding is resolved by the
//    sign of d + w).
// The only approximation left is in p and the table words (relative error
// around 2^-54 for binary32, 2^-80 for binary64); a result can be misrounded only
// when exp(x) lies within that distance of a rounding boundary.
//
// Written without HIP-specific calls so that the same code can be compiled for
// the host (tests define __host__ / __device__ / __forceinline__ as empty).
#pragma once
#pragma clang fp contract(off)

#include "exp_tables.h"

namespace coot {

// On the device the table's leading words are read from an LDS copy that every
// kernel evaluating exp fills first (exp_table_to_lds): a wavefront's 64 lanes
// index the table at scattered rows, which LDS serves in a few cycles while the
// texture path would spend a cycle per distinct cache line.  Host builds (tests)
// read the global table.
#if defined(__HIP_DEVICE_COMPILE__)
#define COOT_EXP_TABLE_IN_LDS 1
__shared__ float coot_exp_lds_f[128][2];
__shared__ double coot_exp_lds_d[128][2];
#endif

template <typename F> struct ExpConst;

template <> struct ExpConst<float> {
  static __host__ __device__ __forceinline__ float L1() { return COOT_EXP_L1F; }
  static __host__ __device__ __forceinline__ float L2() { return COOT_EXP_L2F; }
  static __host__ __device__ __forceinline__ float L3() { return COOT_EXP_L3F; }
  static __host__ __device__ __forceinline__ float INVL() { return COOT_EXP_INVLF; }
  static __host__ __device__ __forceinline__ float S0() { return COOT_EXP_S0F; }
  static __host__ __device__ __forceinline__ float S1() { return COOT_EXP_S1F; }
  static __host__ __device__ __forceinline__ float OVER() { return 89.0f; }
  static __host__ __device__ __forceinline__ float UNDER() { return -104.0f; }
  static constexpr int KMIN_NORMAL = -126;  // k > KMIN_NORMAL: the result is a normal number
  // fast path: inputs whose result is a normal number, k in [-125, 127]
  static __host__ __device__ __forceinline__ float FAST_LO() { return -86.0f; }
  static __host__ __device__ __forceinline__ float FAST_HI() { return 88.0f; }
  // fast path: half a unit in the last place minus 2^-14 units (>= 4x the error bound)
  static __host__ __device__ __forceinline__ float HALF_LESS_MARGIN() { return 0.5f - 0x1p-14f; }
  static constexpr int SUB = 149;           // subnormal grid 2^-SUB
  static __host__ __device__ __forceinline__ void tab(int j, float& t0, float& t1, float& t2) {
#ifdef COOT_EXP_TABLE_IN_LDS
    t0 = coot_exp_lds_f[j][0];
    t1 = coot_exp_lds_f[j][1];
#else
    t0 = coot_exp_tab_f[j][0];
    t1 = coot_exp_tab_f[j][1];
#endif
    t2 = coot_exp_tab_f[j][2];
  }
};

template <> struct ExpConst<double> {
  static __host__ __device__ __forceinline__ double L1() { return COOT_EXP_M1; }
  static __host__ __device__ __forceinline__ double L2() { return COOT_EXP_M2; }
  static __host__ __device__ __forceinline__ double L3() { return COOT_EXP_M3; }
  static __host__ __device__ __forceinline__ double INVL() { return COOT_EXP_INVL; }
  static __host__ __device__ __forceinline__ double S0() { return 0x1.5555555555555p-3; }
  static __host__ __device__ __forceinline__ double S1() { return 0x1.5555555555555p-57; }
  static __host__ __device__ __forceinline__ double OVER() { return 709.8; }
  static __host__ __device__ __forceinline__ double UNDER() { return -745.2; }
  static constexpr int KMIN_NORMAL = -1022;
  static constexpr int SUB = 1074;
  static __host__ __device__ __forceinline__ double FAST_LO() { return -707.0; }
  static __host__ __device__ __forceinline__ double FAST_HI() { return 709.0; }
  static __host__ __device__ __forceinline__ double HALF_LESS_MARGIN() { return 0.5 - 0x1p-14; }
  static __host__ __device__ __forceinline__ void tab(int j, double& t0, double& t1, double& t2) {
#ifdef COOT_EXP_TABLE_IN_LDS
    t0 = coot_exp_lds_d[j][0];
    t1 = coot_exp_lds_d[j][1];
#else
    t0 = coot_exp_tab_d[j][0];
    t1 = coot_exp_tab_d[j][1];
#endif
    t2 = 0.0;
  }
};

__host__ __device__ __forceinline__ float x_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ __forceinline__ double x_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__host__ __device__ __forceinline__ float x_rint(float a) { return __builtin_rintf(a); }
__host__ __device__ __forceinline__ double x_rint(double a) { return __builtin_rint(a); }
__host__ __device__ __forceinline__ float x_ldexp(float a, int e) { return __builtin_ldexpf(a, e); }
__host__ __device__ __forceinline__ double x_ldexp(double a, int e) { return __builtin_ldexp(a, e); }
__host__ __device__ __forceinline__ float x_frexp(float a, int* e) { return __builtin_frexpf(a, e); }
__host__ __device__ __forceinline__ float x_abs(float a) { return __builtin_fabsf(a); }
__host__ __device__ __forceinline__ double x_abs(double a) { return __builtin_fabs(a); }
__host__ __device__ __forceinline__ double x_frexp(double a, int* e) { return __builtin_frexp(a, e); }

template <typename F>
__host__ __device__ __forceinline__ void ef_two_sum(F a, F b, F& s, F& e) {
  s = a + b;
  F bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}

template <typename F>
__host__ __device__ __forceinline__ void ef_two_prod(F a, F b, F& p, F& e) {
  p = a * b;
  e = x_fma(a, b, -p);
}

template <typename F>
__host__ __device__ __forceinline__ F exp_cr(F x) {
  typedef ExpConst<F> K;
  if (!(x == x)) return x + x;               // NaN
  if (x > K::OVER()) return (F)__builtin_huge_valf();  // +inf (also for x = +inf)
  if (x < K::UNDER()) return (F)0;           // includes -inf
  // ---- 1. reduction: r = x - N * ln2/128 as rh + rl -----------------------------
  const F Nf = x_rint(x * K::INVL());
  const int N = (int)Nf;
  const int k = N >> 7;                      // floor(N / 128)
  const int j = N & 127;
  F p_hi, p_lo, q_hi, q_lo;
  ef_two_prod(Nf, K::L1(), p_hi, p_lo);      // N * L1 exactly
  const F s0 = x - p_hi;                     // exact (Sterbenz, or N = 0)
  ef_two_prod(Nf, K::L2(), q_hi, q_lo);
  F h, t1, t2;
  ef_two_sum(s0, -p_lo, h, t1);
  ef_two_sum(h, -q_hi, h, t2);
  F rl = ((t1 + t2) - q_lo) - Nf * K::L3();
  F rh = h + rl;                             // renormalise
  rl = rl - (rh - h);
  // ---- 2. p = exp(r) - 1 = ph + pl ----------------------------------------------
  F a_hi, a_lo;
  ef_two_prod(rh, rh, a_hi, a_lo);           // rh^2
  F c_hi, c_lo;
  ef_two_prod(a_hi, rh, c_hi, c_lo);         // rh^3 (a_lo * rh added below)
  c_lo = c_lo + a_lo * rh;
  F d_hi, d_lo;
  ef_two_prod(c_hi, K::S0(), d_hi, d_lo);    // rh^3 / 6
  d_lo = d_lo + (c_hi * K::S1() + c_lo * K::S0());
  const F tail = (a_hi * a_hi) *
                 ((F)(1.0 / 24) + rh * ((F)(1.0 / 120) + rh * ((F)(1.0 / 720) + rh * (F)(1.0 / 5040))));
  F ph, e1, e2;
  ef_two_sum(rh, (F)0.5 * a_hi, ph, e1);
  ef_two_sum(ph, d_hi, ph, e2);
  F pl = ((((tail + d_lo) + (F)0.5 * a_hi * rl) + rh * rl) + (F)0.5 * a_lo) + rl;
  pl = (pl + e2) + e1;
  // ---- 3. V = T (1 + p) = s + u + w ----------------------------------------------
  F T0, T1, T2;
  K::tab(j, T0, T1, T2);
  F m_hi, m_lo;
  ef_two_prod(T0, ph, m_hi, m_lo);
  F s, e3;
  ef_two_sum(T0, m_hi, s, e3);
  F u, f1, f2, f3, f4;
  ef_two_sum(e3, T1, u, f1);
  F g_hi, g_lo;
  ef_two_prod(T0, pl, g_hi, g_lo);
  ef_two_sum(u, g_hi, u, f2);
  ef_two_sum(u, m_lo, u, f3);
  ef_two_sum(u, T1 * ph, u, f4);
  const F w = (((T2 + g_lo) + T1 * pl) + (f1 + f2)) + (f3 + f4);
  // ---- 4. exact final rounding ----------------------------------------------------
  F y, d;
  ef_two_sum(s, u, y, d);                    // s + u = y + d exactly; V = y + d + w
  if (k > K::KMIN_NORMAL) {
    int e;
    const F fr = x_frexp(y, &e);             // y = fr * 2^e, fr in [0.5, 1)
    constexpr int P = sizeof(F) == 4 ? 24 : 53;
    const F gap_up = x_ldexp((F)1, e - P);
    const F gap_dn = fr == (F)0.5 ? (F)0.5 * gap_up : gap_up;
    const F hu = (F)0.5 * gap_up, hd = (F)0.5 * gap_dn;
    const F z = d + w;
    if (z > hu) {
      y = y + gap_up;
    } else if (z < -hd) {
      y = y - gap_dn;
    } else if (z == hu || z == -hd) {
      const F t = z > 0 ? (d - hu) + w : (d + hd) + w;   // d -/+ half gap is exact
      if (z > 0 && t > 0) y = y + gap_up;
      else if (z < 0 && t < 0) y = y - gap_dn;
      else if (t == 0) {
        // exact tie: keep y if its significand is even, else move to the neighbour
        const F half_sig = x_ldexp(fr, P - 1);
        if (half_sig != x_rint(half_sig)) y = z > 0 ? y + gap_up : y - gap_dn;
      }
    }
    return x_ldexp(y, k);
  }
  // subnormal (or smallest-binade) result: one rounding on the grid 2^-SUB
  const int m = k + K::SUB;
  if (m < -2) return (F)0;
  const F Y = x_ldexp(y, m);                 // exact scaling, Y < 2^(P-1) * 2
  F n = x_rint(Y);
  const F frac = Y - n;                      // exact
  const F z = d + w;
  if (frac == (F)0.5 || frac == (F)-0.5) {
    // the first rounding (to y) landed on a midpoint of the subnormal grid
    if (z > 0) n = Y + (F)0.5;
    else if (z < 0) n = Y - (F)0.5;
  }
  return x_ldexp(n, -K::SUB);
}


// ---------------------------------------------------------------------------
// Two-level evaluation (Ziv's strategy): a cheaper double-word evaluation with
// relative error about 2^-41 (binary32) / 2^-70 (binary64), then a test whether
// rounding its result is unambiguous, i.e. whether the computed remainder stays
// 2^-14 units in the last place (8x the error bound of 2^-17 units) below half a
// unit.  Only ambiguous lanes (about 1 in 10^4) and inputs outside the
// normal-result range run exp_cr above, out of line.
// ---------------------------------------------------------------------------
template <typename F>
__host__ __device__ __forceinline__ F exp_fast(F x, bool& ok) {
  typedef ExpConst<F> K;
  ok = x > K::FAST_LO() && x < K::FAST_HI();  // false for NaN too
  const F xc = ok ? x : (F)0;
  const F Nf = x_rint(xc * K::INVL());
  const int N = (int)Nf;
  const int k = N >> 7;
  const int j = N & 127;
  F p_hi, p_lo;
  ef_two_prod(Nf, K::L1(), p_hi, p_lo);
  const F s0 = xc - p_hi;                    // exact
  const F c = p_lo + Nf * K::L2();
  F rh, rl;
  ef_two_sum(s0, -c, rh, rl);
  // exp(r) - 1 = rh + [rl + rh*rl + rh^2 (1/2 + rh/6 + ...)]
  F poly;
  if constexpr (sizeof(F) == 4) {
    poly = x_fma(rh, x_fma(rh, (F)(1.0 / 24), (F)(1.0 / 6)), (F)0.5);
  } else {
    poly = x_fma(rh, x_fma(rh, x_fma(rh, x_fma(rh, x_fma(rh, 1.0 / 5040, 1.0 / 720), 1.0 / 120), 1.0 / 24), 1.0 / 6),
                 0.5);
  }
  const F pl = x_fma(rh * rh, poly, x_fma(rh, rl, rl));
  F T0, T1, T2;
  K::tab(j, T0, T1, T2);
  F m_hi, m_lo;
  ef_two_prod(T0, rh, m_hi, m_lo);
  const F s = T0 + m_hi;                     // |T0| >= |m_hi|: fast two-sum
  const F e = m_hi - (s - T0);
  const F u = e + (m_lo + x_fma(T0, pl, x_fma(T1, rh, T1)));
  const F y = s + u;
  const F d = u - (y - s);                   // s + u = y + d exactly, |d| <= half a unit of y
  // y lies in [0.997, 1.995): with P significand bits (24 or 53) the gap between
  // neighbours is 2^-(P-1) above 1 and 2^-P below, and for y = 1 the side d points
  // to decides.  Rounding is unambiguous when |d| plus the error stays under half
  // that gap.
  const bool upper = y > (F)1 || (y == (F)1 && d >= (F)0);
  const F unit_inv_hi = sizeof(F) == 4 ? (F)0x1p23 : (F)0x1p52;   // 2^(P-1)
  const F t = x_abs(d) * (upper ? unit_inv_hi : (F)2 * unit_inv_hi);
  ok = ok && t < K::HALF_LESS_MARGIN();
  return x_ldexp(y, k);
}

#ifdef COOT_EXP_TABLE_IN_LDS
// Copy the table's leading words to LDS; every thread of the workgroup calls it
// before its first exp (it ends with a barrier).
template <typename F>
__device__ __forceinline__ void exp_table_to_lds() {
  for (int k = threadIdx.x; k < 128; k += blockDim.x) {
    if constexpr (sizeof(F) == 4) {
      coot_exp_lds_f[k][0] = coot_exp_tab_f[k][0];
      coot_exp_lds_f[k][1] = coot_exp_tab_f[k][1];
    } else {
      coot_exp_lds_d[k][0] = coot_exp_tab_d[k][0];
      coot_exp_lds_d[k][1] = coot_exp_tab_d[k][1];
    }
  }
  __syncthreads();
}
#else
template <typename F>
__host__ __device__ __forceinline__ void exp_table_to_lds() {}
#endif

template <typename F>
__host__ __device__ __attribute__((noinline)) F exp_slow(F x) {
  return exp_cr<F>(x);
}

template <typename F>
__host__ __device__ __forceinline__ F exp_rn(F x) {
  bool ok;
  F y = exp_fast<F>(x, ok);
  if (!ok) y = exp_slow<F>(x);
  return y;
}

}  // namespace coot
