// coot_dev.h — device side of libcoot for gfx950 (CDNA4, wave64).
//
// This header is embedded in libcoot and handed to hipRTC together with a small
// generated translation unit per expression signature.  The generated part is a
// struct X with
//     typedef <element type> T;
//     NL          number of distinct leaves (operand slot + transpose parity)
//     NP1         number of leaves read transposed (parity 1)
//     slot(k)     operand slot of leaf k
//     par(k)      transpose parity of leaf k (number of trans() above it, mod 2)
//     p1(k)       index of leaf k among the parity-1 leaves (or -1)
//     f(L, sc)    the expression body on one element, leaf values L[NL]
//     f2(L, sc, &a, &b)   for a Schur-product root: its two factors
// and extern "C" kernels that instantiate the templates below.  Everything that
// touches memory is written here by hand: the generated body is straight-line
// arithmetic on registers.
//
// The expression model is the paper's (Section 3): eOp / eGlue nodes are
// element-wise and become the body f; Op<.., op_trans> never becomes a pass of
// its own — it is folded into the index map of the leaves below it, and a leaf
// read transposed is staged through LDS so both its reads and the output writes
// stay coalesced (the implicit transpose Section 3 describes for GEMM, applied to
// element-wise trees).
#pragma once
#pragma clang fp contract(off)

#include "coot_exp.h"
#include "coot_log.h"

typedef unsigned int u32;
typedef int s32;
typedef long long i64;
typedef unsigned long long u64;

#define COOT_MAX_SLOTS 16
#define COOT_MAX_SCALARS 32

// Kernel argument block.  Identical layout on the host (coot_kargs in kargs.h).
struct coot_kargs {
  const void* leaf[COOT_MAX_SLOTS];  // operand base pointers (column-major)
  i64 ld[COOT_MAX_SLOTS];            // leading dimensions (elements)
  u64 sc[COOT_MAX_SCALARS];          // scalars, already converted to the element type (bit pattern)
  void* out;                         // output (eval) / final result (reduce)
  i64 out_ld;
  i64 n_rows, n_cols;                // dimensions of the element-wise result
  void* ws;                          // workspace: per-block / per-tile partials
  void* ws2;                         // second workspace word block (norm rescale control)
  i64 n_part;                        // number of partials written by stage 1
};

namespace coot {

// ---------------------------------------------------------------------------
// element types and scalar unpacking
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T sc_as(u64 bits);
template <> __device__ __forceinline__ float sc_as<float>(u64 b) { return __uint_as_float((u32)b); }
template <> __device__ __forceinline__ double sc_as<double>(u64 b) { return __longlong_as_double((i64)b); }
template <> __device__ __forceinline__ u32 sc_as<u32>(u64 b) { return (u32)b; }
template <> __device__ __forceinline__ s32 sc_as<s32>(u64 b) { return (s32)(u32)b; }

// ---------------------------------------------------------------------------
// 16-bit storage types.  An expression over f16 (IEEE binary16) or bf16
// (bfloat16) operands computes in binary32 and rounds every operator's result to
// the storage type, nearest-even: binary32 carries at least 2p + 2 bits of a p-bit
// type, so the two roundings give the correctly rounded 16-bit result (for bf16,
// while the binary32 result is normal).  Leaves are widened when loaded and
// results narrowed when stored; St<S> maps a storage type to its compute type.
// ---------------------------------------------------------------------------
struct f16 { unsigned short b; };
struct bf16 { unsigned short b; };

template <typename S> struct St {
  typedef S C;
  static __device__ __forceinline__ C in(S x) { return x; }
  static __device__ __forceinline__ S out(C x) { return x; }
  static __device__ __forceinline__ C rnd(C x) { return x; }
};
template <> struct St<f16> {
  typedef float C;
  static __device__ __forceinline__ float in(f16 x) { return (float)__builtin_bit_cast(_Float16, x.b); }
  static __device__ __forceinline__ f16 out(float x) { return f16{__builtin_bit_cast(unsigned short, (_Float16)x)}; }
  // nearest-even binary16 value of x, kept in binary32: the hardware conversions
  // there and back (two instructions).  They are written as one asm statement so
  // that the compiler sees an opaque value between operators: folding the
  // conversions into neighbouring operators has crashed its instruction selection.
  static __device__ __forceinline__ float rnd(float x) {
    float r;
    asm("v_cvt_f16_f32 %0, %1\n\tv_cvt_f32_f16 %0, %0" : "=v"(r) : "v"(x));
    return r;
  }
};
template <> struct St<bf16> {
  typedef float C;
  static __device__ __forceinline__ float in(bf16 x) { return __uint_as_float((u32)x.b << 16); }
  static __device__ __forceinline__ bf16 out(float x) {
    const u32 u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return bf16{(unsigned short)((u >> 16) | 0x40u)};  // NaN: quiet, kept
    return bf16{(unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16)};                  // nearest-even
  }
  // nearest-even bfloat16 value of x, kept in binary32: the packed conversion
  // (both halves from x) and a mask keeping one of them
  static __device__ __forceinline__ float rnd(float x) {
    float r;
    asm("v_cvt_pk_bf16_f32 %0, %1, %1\n\tv_and_b32 %0, 0xffff0000, %0" : "=v"(r) : "v"(x));
    return r;
  }
};

template <typename T> struct is_int_t { static constexpr bool v = false; };
template <> struct is_int_t<u32> { static constexpr bool v = true; };
template <> struct is_int_t<s32> { static constexpr bool v = true; };

// ---------------------------------------------------------------------------
// element-wise operators.  Floating point: IEEE, round-to-nearest-even, no
// contraction (pragma above + -ffp-contract=off), correctly rounded / and sqrt.
// Integers: arithmetic mod 2^32 (s32 computed on the unsigned bit pattern so
// that wrap-around is defined).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float op_add(float a, float b) { return a + b; }
__device__ __forceinline__ float op_sub(float a, float b) { return a - b; }
__device__ __forceinline__ float op_mul(float a, float b) { return a * b; }
__device__ __forceinline__ float op_div(float a, float b) { return a / b; }
__device__ __forceinline__ float op_neg(float a) { return -a; }
__device__ __forceinline__ float op_abs(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ float op_sqrt(float a) { return __builtin_sqrtf(a); }
__device__ __forceinline__ float op_square(float a) { return a * a; }
__device__ __forceinline__ float op_exp(float a) { return exp_rn<float>(a); }  // correctly rounded (coot_exp.h)
__device__ __forceinline__ float op_log(float a) { return log_lf(a); }

__device__ __forceinline__ double op_add(double a, double b) { return a + b; }
__device__ __forceinline__ double op_sub(double a, double b) { return a - b; }
__device__ __forceinline__ double op_mul(double a, double b) { return a * b; }
__device__ __forceinline__ double op_div(double a, double b) { return a / b; }
__device__ __forceinline__ double op_neg(double a) { return -a; }
__device__ __forceinline__ double op_abs(double a) { return __builtin_fabs(a); }
__device__ __forceinline__ double op_sqrt(double a) { return __builtin_sqrt(a); }
__device__ __forceinline__ double op_square(double a) { return a * a; }
__device__ __forceinline__ double op_exp(double a) { return exp_rn<double>(a); }
__device__ __forceinline__ double op_log(double a) { return log(a); }

__device__ __forceinline__ u32 op_add(u32 a, u32 b) { return a + b; }
__device__ __forceinline__ u32 op_sub(u32 a, u32 b) { return a - b; }
__device__ __forceinline__ u32 op_mul(u32 a, u32 b) { return a * b; }
__device__ __forceinline__ u32 op_neg(u32 a) { return 0u - a; }
__device__ __forceinline__ u32 op_abs(u32 a) { return a; }
__device__ __forceinline__ u32 op_square(u32 a) { return a * a; }

__device__ __forceinline__ s32 op_add(s32 a, s32 b) { return (s32)((u32)a + (u32)b); }
__device__ __forceinline__ s32 op_sub(s32 a, s32 b) { return (s32)((u32)a - (u32)b); }
__device__ __forceinline__ s32 op_mul(s32 a, s32 b) { return (s32)((u32)a * (u32)b); }
__device__ __forceinline__ s32 op_neg(s32 a) { return (s32)(0u - (u32)a); }
__device__ __forceinline__ s32 op_abs(s32 a) { return a < 0 ? (s32)(0u - (u32)a) : a; }
__device__ __forceinline__ s32 op_square(s32 a) { return (s32)((u32)a * (u32)a); }

// ---------------------------------------------------------------------------
// vector access: V consecutive elements as one 32/64/128/256-bit access.
// ---------------------------------------------------------------------------
template <typename T, int V> struct vt { T v[V]; };

typedef u32 u32x2 __attribute__((ext_vector_type(2)));
typedef u32 u32x4 __attribute__((ext_vector_type(4)));

// Flat full reductions read every operand once, in order, and write nothing but
// their records: their 8- to 32-byte loads are non-temporal (NT), measured faster
// (accu over 2^28 fp32 172 -> 156 us).  Flat element-wise kernels take NT loads when
// their operands together exceed the Infinity Cache (256 MiB), where no later kernel
// could find them there anyway; below that, plain loads leave them cached for the
// kernels that re-read them next.  The tiled walks read 256-byte column segments and
// keep plain loads (with NT loads the 4096 x 4096 Z tile kernel took 78 instead of
// 53 us).
template <typename T, int V, bool NT = false>
__device__ __forceinline__ vt<T, V> ldv(const T* p) {
  vt<T, V> r;
  constexpr int B = V * (int)sizeof(T);
  if constexpr (B == 2) {
    unsigned short q = *reinterpret_cast<const unsigned short*>(p);
    __builtin_memcpy(&r, &q, 2);
  } else if constexpr (B == 4) {
    u32 q = *reinterpret_cast<const u32*>(p);
    __builtin_memcpy(&r, &q, 4);
  } else if constexpr (B == 8) {
    const u32x2* a = reinterpret_cast<const u32x2*>(p);
    u32x2 q = NT ? __builtin_nontemporal_load(a) : *a;
    __builtin_memcpy(&r, &q, 8);
  } else if constexpr (B == 16) {
    const u32x4* a = reinterpret_cast<const u32x4*>(p);
    u32x4 q = NT ? __builtin_nontemporal_load(a) : *a;
    __builtin_memcpy(&r, &q, 16);
  } else {
    static_assert(B == 32, "vector width");
    const u32x4* a = reinterpret_cast<const u32x4*>(p);
    u32x4 q0 = NT ? __builtin_nontemporal_load(a) : a[0];
    u32x4 q1 = NT ? __builtin_nontemporal_load(a + 1) : a[1];
    __builtin_memcpy(&r, &q0, 16);
    __builtin_memcpy(reinterpret_cast<char*>(&r) + 16, &q1, 16);
  }
  return r;
}

// Results are written with non-temporal stores: an expression's output is streamed
// once, and keeping it out of L2 and the Infinity Cache leaves no dirty lines to be
// written back while the next kernel streams its own operands.  A module generated
// with COOT_PLAIN_STORES (the unfused comparator, whose temporaries the next operator
// reads at once) stores through the caches instead.
template <typename W>
__device__ __forceinline__ void st_word(W* p, W q) {
#ifdef COOT_PLAIN_STORES
  *p = q;
#else
  __builtin_nontemporal_store(q, p);
#endif
}

template <typename T, int V>
__device__ __forceinline__ void stv(T* p, const vt<T, V>& r) {
  constexpr int B = V * (int)sizeof(T);
  if constexpr (B == 2) {
    unsigned short q;
    __builtin_memcpy(&q, &r, 2);
    st_word(reinterpret_cast<unsigned short*>(p), q);
  } else if constexpr (B == 4) {
    u32 q;
    __builtin_memcpy(&q, &r, 4);
    st_word(reinterpret_cast<u32*>(p), q);
  } else if constexpr (B == 8) {
    u32x2 q;
    __builtin_memcpy(&q, &r, 8);
    st_word(reinterpret_cast<u32x2*>(p), q);
  } else if constexpr (B == 16) {
    u32x4 q;
    __builtin_memcpy(&q, &r, 16);
    st_word(reinterpret_cast<u32x4*>(p), q);
  } else {
    u32x4 q0, q1;
    __builtin_memcpy(&q0, &r, 16);
    __builtin_memcpy(&q1, reinterpret_cast<const char*>(&r) + 16, 16);
    st_word(reinterpret_cast<u32x4*>(p), q0);
    st_word(reinterpret_cast<u32x4*>(p) + 1, q1);
  }
}

// V storage elements widened to the compute type / narrowed from it (16-bit types)
template <typename S, int V, bool NT = false>
__device__ __forceinline__ vt<typename St<S>::C, V> ldc(const S* p) {
  if constexpr (sizeof(S) == 2) {
    const vt<S, V> r = ldv<S, V, NT>(p);
    vt<typename St<S>::C, V> c;
#pragma unroll
    for (int q = 0; q < V; ++q) c.v[q] = St<S>::in(r.v[q]);
    return c;
  } else {
    return ldv<S, V, NT>(p);
  }
}
template <typename S, int V>
__device__ __forceinline__ void stc(S* p, const vt<typename St<S>::C, V>& c) {
  if constexpr (sizeof(S) == 2) {
    vt<S, V> r;
#pragma unroll
    for (int q = 0; q < V; ++q) r.v[q] = St<S>::out(c.v[q]);
    stv<S, V>(p, r);
  } else {
    stv<S, V>(p, c);
  }
}

// ---------------------------------------------------------------------------
// Error-free transformations (Knuth's TwoSum, FMA-based TwoProd) and the
// accumulators built from them.  A compensated accumulator keeps (hi, lo) with
// hi + lo the running sum; every addend's rounding error is carried in lo.
// ---------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ void two_sum(F a, F b, F& s, F& e) {
  s = a + b;
  F bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}
__device__ __forceinline__ void two_prod(float a, float b, float& p, float& e) {
  p = a * b;
  e = __builtin_fmaf(a, b, -p);
}
__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = __builtin_fma(a, b, -p);
}

// Double-word sum (hi, lo) + (hi, lo) with renormalisation.
template <typename F>
__device__ __forceinline__ void dw_add(F& h, F& l, F h2, F l2) {
  F s, e;
  two_sum(h, h2, s, e);
  e += l + l2;
  F hs = s + e;
  l = e - (hs - s);
  h = hs;
}

// Reduction kinds
enum { RK_SUM = 0, RK_DOT = 1, RK_SUMSQ = 2, RK_ABSSUM = 3, RK_MAX = 4, RK_MIN = 5, RK_AMAX = 6, RK_MEAN = 7 };
// Variance of all elements in one pass (RK_VAR1): each lane shifts its values by
// its first value K and accumulates the shifted moments sum d and sum d^2, with
// d = v - K and d^2 formed exactly (TwoDiff, TwoProd) and summed float-float; its
// (count, mean, M2) then merge by Chan's formula in binary64 across lanes, waves
// and workgroups.  Stage 2 (RK_VAR / RK_VARN) merges the records and divides M2 by
// N - 1 or N.  The moments about a value of the lane's own data keep M2 free of
// the cancellation of sum v^2 - (sum v)^2 / n however large the mean is next to
// the spread.
enum { RK_VAR1 = 8, RK_VAR = 10, RK_VARN = 11 };

// Extremum kinds keep, per lane and in the compute type, the largest value
// (RK_MAX), the smallest (RK_MIN) or the largest magnitude (RK_AMAX), plus a flag
// for a NaN seen (the result is then NaN: the NaN-propagating extremum of IEEE
// 754-2019).  The lane's value enters the partial record as one binary64 word
// (exact for every type); RK_MIN stores it negated so that records and stage 2
// combine every kind by the same maximum.
template <int RK> __device__ __forceinline__ double ext_identity() {
  return RK == RK_MAX || RK == RK_MIN ? -__builtin_inf() : 0.0;
}
// NaN-propagating maximum of two record words
__device__ __forceinline__ double nmax(double a, double b) { return a != a ? a : (b != b ? b : (a > b ? a : b)); }

template <typename T, int RK>
struct Ext {
  static constexpr bool is_int = is_int_t<T>::v;
  T m;
  bool nan;
  __device__ __forceinline__ void init() {
    nan = false;
    if constexpr (is_int) {
      constexpr bool uns = (T)-1 > (T)0;  // u32: identities 2^32 - 1 (min) and 0 (max)
      m = RK == RK_MIN ? (uns ? (T)0xffffffffu : (T)0x7fffffff) : (uns ? (T)0 : (T)0x80000000u);
    } else {
      m = RK == RK_MAX ? (T)-__builtin_inf() : (RK == RK_MIN ? (T)__builtin_inf() : (T)0);
    }
  }
  __device__ __forceinline__ void add(T v) {
    if constexpr (is_int) {
      m = RK == RK_MIN ? (v < m ? v : m) : (v > m ? v : m);
    } else {
      if (RK == RK_AMAX) v = __builtin_fabs(v);
      nan = nan || v != v;
      m = RK == RK_MIN ? __builtin_fmin(m, v) : __builtin_fmax(m, v);  // NaN-ignoring; the flag keeps it
    }
  }
  __device__ __forceinline__ double word() const {
    const double d = nan ? __builtin_nan("") : (double)m;
    return RK == RK_MIN ? -d : d;
  }
};

// Compensated accumulator for floating T; partial type P carries (hi, lo).
template <typename T>
struct AccComp {
  T hi, lo;
  __device__ __forceinline__ void init() { hi = (T)0; lo = (T)0; }
  __device__ __forceinline__ void add(T x) {
    T s, e;
    two_sum(hi, x, s, e);
    hi = s;
    lo += e;
  }
  __device__ __forceinline__ void add_prod(T a, T b) {
    T p, pe;
    two_prod(a, b, p, pe);
    T s, e;
    two_sum(hi, p, s, e);
    hi = s;
    lo += e + pe;
  }
  __device__ __forceinline__ void merge(T h2, T l2) { dw_add(hi, lo, h2, l2); }
};

template <typename T>
struct AccPlain {
  T s;
  __device__ __forceinline__ void init() { s = (T)0; }
  __device__ __forceinline__ void add(T x) { s = s + x; }
  __device__ __forceinline__ void add_prod(T a, T b) { s = s + a * b; }
};

// ---------------------------------------------------------------------------
// wave / block combination helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float shfl_x(float v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ double shfl_x(double v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ u32 shfl_x(u32 v, int m) { return (u32)__shfl_xor((int)v, m, 64); }
__device__ __forceinline__ s32 shfl_x(s32 v, int m) { return __shfl_xor(v, m, 64); }

// (hi, lo) pairs summed across a whole wavefront with double-word adds.
template <typename F>
__device__ __forceinline__ void wave_dw_sum(F& h, F& l) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    F h2 = shfl_x(h, m), l2 = shfl_x(l, m);
    dw_add(h, l, h2, l2);
  }
}
template <typename F>
__device__ __forceinline__ F wave_sum(F v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = op_add(v, shfl_x(v, m));
  return v;
}

// ---------------------------------------------------------------------------
// Leaf access
// ---------------------------------------------------------------------------
template <class X, int V, bool NT = false>
__device__ __forceinline__ void load_flat(const coot_kargs& a, i64 v, vt<typename X::T, V> (&x)[X::NL]) {
  typedef typename X::S S;
#pragma unroll
  for (int k = 0; k < X::NL; ++k) x[k] = ldc<S, V, NT>((const S*)a.leaf[X::slot(k)] + v * V);
}

// leaf k's element i (scalar tails), widened to the compute type
template <class X>
__device__ __forceinline__ typename X::T leaf_at(const coot_kargs& a, int k, i64 i) {
  typedef typename X::S S;
  return St<S>::in(((const S*)a.leaf[X::slot(k)])[i]);
}

// ===========================================================================
// FLAT family: every leaf untransposed and contiguous; out[i] = f(leaves[i]).
// Grid-stride over V-element groups, E groups in flight per thread per trip,
// then a scalar tail of n mod V elements handled by the last workgroup.
// ===========================================================================
template <class X, int V, int E, bool NT = false>
__device__ __forceinline__ void flat_eval(const coot_kargs& a) {
  typedef typename X::T T;
  const i64 n = a.n_rows * a.n_cols;
  const i64 nv = n / V;
  const int bs = blockDim.x;
  const i64 step = (i64)gridDim.x * bs * E;
  typedef typename X::S S;
  S* out = (S*)a.out;
  for (i64 b = (i64)blockIdx.x * bs * E + threadIdx.x; b < nv; b += step) {
    vt<T, V> x[E][X::NL];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const i64 v = b + (i64)e * bs;
      if (v < nv) load_flat<X, V, NT>(a, v, x[e]);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const i64 v = b + (i64)e * bs;
      if (v < nv) {
        vt<T, V> r;
#pragma unroll
        for (int q = 0; q < V; ++q) {
          T L[X::NL];
#pragma unroll
          for (int k = 0; k < X::NL; ++k) L[k] = x[e][k].v[q];
          r.v[q] = X::f(L, a.sc);
        }
        stc<S, V>(out + v * V, r);
      }
    }
  }
  if (V > 1 && blockIdx.x == gridDim.x - 1) {
    for (i64 i = nv * V + threadIdx.x; i < n; i += bs) {
      T L[X::NL];
#pragma unroll
      for (int k = 0; k < X::NL; ++k) L[k] = leaf_at<X>(a, k, i);
      out[i] = St<S>::out(X::f(L, a.sc));
    }
  }
}

// ===========================================================================
// Element producers.  `Red` selects what a reduction consumes per element:
// RK_SUM the value, RK_DOT the two factors of the Schur-product root, RK_SUMSQ
// the value squared (through the accumulator's product path).
// ===========================================================================
template <class X, int RK, class A>
__device__ __forceinline__ void consume(A& acc, Ext<typename X::T, RK>& ext, const typename X::T* L, const u64* sc) {
  if constexpr (RK == RK_SUM || RK == RK_MEAN) {
    acc.add(X::f(L, sc));
  } else if constexpr (RK == RK_ABSSUM) {
    acc.add(op_abs(X::f(L, sc)));
  } else if constexpr (RK == RK_MAX || RK == RK_MIN || RK == RK_AMAX) {
    ext.add(X::f(L, sc));
  } else if constexpr (RK == RK_DOT) {
    typename X::T p, q;
    X::f2(L, sc, p, q);
    acc.add_prod(p, q);
  } else {
    typename X::T v = X::f(L, sc);
    acc.add_prod(v, v);
  }
}

// What a full reduction's stage 1 does with one element: consume() for most kinds;
// RK_SUMSQ also tracks the largest magnitude and applies the rescaling factor;
// RK_VAR1 feeds the lane's variance state.
template <class X, int RK, class A>
__device__ __forceinline__ void take(A& acc, Ext<typename X::T, RK>& ext, typename X::T& amax, typename X::T scale,
                                     const typename X::T* L, const u64* sc);

// Integer accumulator: plain wrap-around sum.
template <typename T>
struct AccInt {
  T s;
  __device__ __forceinline__ void init() { s = (T)0; }
  __device__ __forceinline__ void add(T x) { s = op_add(s, x); }
  __device__ __forceinline__ void add_prod(T a, T b) { s = op_add(s, op_mul(a, b)); }
};

template <typename T, bool COMP> struct AccSel { typedef AccPlain<T> type; };
template <> struct AccSel<float, true> { typedef AccComp<float> type; };
template <> struct AccSel<double, true> { typedef AccComp<double> type; };
template <> struct AccSel<u32, true> { typedef AccInt<u32> type; };
template <> struct AccSel<u32, false> { typedef AccInt<u32> type; };
template <> struct AccSel<s32, true> { typedef AccInt<s32> type; };
template <> struct AccSel<s32, false> { typedef AccInt<s32> type; };

// Partial record written by stage 1 of a full reduction (one per workgroup) and
// read by stage 2.  Floating compensated: (hi, lo) as binary64 words; fp32
// partials are exact binary64 conversions of the lane's float pair.  Plain:
// hi only.  Integers: the u32 bit pattern in hi.  amax: largest |value| seen
// (sum of squares only, for the rescaling decision).
struct PartRec {
  double hi, lo, amax, pad;
};

template <typename T, bool COMP>
__device__ __forceinline__ void lane_to_words(const typename AccSel<T, COMP>::type& acc, double& h, double& l) {
  if constexpr (is_int_t<T>::v) {
    h = (double)(u32)acc.s;
    l = 0.0;
  } else if constexpr (COMP) {
    if constexpr (sizeof(T) == 4) {
      h = (double)acc.hi + (double)acc.lo;  // exact: the pair spans < 53 bits
      l = 0.0;
    } else {
      h = acc.hi;
      l = acc.lo;
    }
  } else {
    h = (double)acc.s;
    l = 0.0;
  }
}

// Combine one pair of words per lane across the workgroup and write the record.
template <typename T, bool COMP>
__device__ __forceinline__ void block_words_to_record(double h, double l, double amax, PartRec* dst) {
  __shared__ double sh[16], sl[16], sm[16];
  constexpr bool is_int = is_int_t<T>::v;
  if (is_int) {
    u32 v = (u32)h;
    v = wave_sum<u32>(v);
    h = (double)v;
  } else if (COMP) {
    wave_dw_sum<double>(h, l);
  } else if (sizeof(T) == 4) {
    float v = (float)h;
    v = wave_sum<float>(v);
    h = (double)v;
  } else {
    h = wave_sum<double>(h);
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) amax = nmax(amax, __shfl_xor(amax, m, 64));
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[w] = h;
    sl[w] = l;
    sm[w] = amax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double H = sh[0], Lo = sl[0], M = sm[0];
    for (int k = 1; k < nw; ++k) {
      if (is_int) {
        H = (double)((u32)H + (u32)sh[k]);
      } else if (COMP) {
        dw_add<double>(H, Lo, sh[k], sl[k]);
      } else if (sizeof(T) == 4) {
        H = (double)((float)H + (float)sh[k]);
      } else {
        H = H + sh[k];
      }
      M = nmax(M, sm[k]);
    }
    PartRec r;
    r.hi = H;
    r.lo = Lo;
    r.amax = M;
    r.pad = 0.0;
    *dst = r;
  }
}

// a lane's largest magnitude as the record's binary64 word (integers track none)
template <typename T>
__device__ __forceinline__ double mag_word(T m) {
  if constexpr (is_int_t<T>::v) {
    return 0.0;
  } else {
    return (double)m;
  }
}

// amax: the lane's largest magnitude in the compute type (exact: a maximum rounds
// nothing), widened to binary64 once per lane for the record.
template <class X, int RK, class A>
__device__ __forceinline__ void take(A& acc, Ext<typename X::T, RK>& ext, typename X::T& amax, typename X::T scale,
                                     const typename X::T* L, const u64* sc) {
  typedef typename X::T T;
  if constexpr (RK == RK_SUMSQ) {
    T val = X::f(L, sc);
    if constexpr (sizeof(T) == 4)
      amax = __builtin_fmaxf(amax, __builtin_fabsf(val));
    else
      amax = __builtin_fmax(amax, __builtin_fabs(val));
    val = val * scale;
    acc.add_prod(val, val);
  } else if constexpr (RK == RK_VAR1) {
    acc.add(X::f(L, sc));
  } else {
    consume<X, RK>(acc, ext, L, sc);
  }
}

// One lane's variance state (RK_VAR1): shift K (its first value), count, and the
// shifted moments as float-float pairs (plain sums when not compensated).
template <typename T, bool COMP>
struct AccVar {
  T K, s1h, s1l, s2h, s2l;
  u32 n;
  __device__ __forceinline__ void init() {
    K = s1h = s1l = s2h = s2l = (T)0;
    n = 0;
  }
  __device__ __forceinline__ void add(T x) {
    if (n == 0) K = x;
    n += 1;
    T dh, dl;
    two_sum(x, -K, dh, dl);  // d = x - K exactly: dh + dl
    if constexpr (COMP) {
      T p, pe;
      two_prod(dh, dh, p, pe);  // dh^2 exactly: p + pe
      T s, e;
      two_sum(s1h, dh, s, e);
      s1h = s;
      s1l += e + dl;
      two_sum(s2h, p, s, e);
      s2h = s;
      s2l += e + (pe + (T)2 * dh * dl);
    } else {
      s1h += dh;
      s2h += dh * dh;
    }
  }
  // (count, mean, M2) of the lane in binary64
  __device__ __forceinline__ void moments(double& cn, double& mean, double& m2) const {
    cn = (double)n;
    if (n == 0) {
      mean = 0.0;
      m2 = 0.0;
      return;
    }
    const double s1 = (double)s1h + (double)s1l, s2 = (double)s2h + (double)s2l;
    mean = (double)K + s1 / cn;
    m2 = s2 - s1 * (s1 / cn);
  }
};

// Chan's merge of (count, mean, M2) summaries: b into a.
__device__ __forceinline__ void chan_merge(double& na, double& ma, double& qa, double nb, double mb, double qb) {
  if (nb == 0.0) return;
  if (na == 0.0) {
    na = nb;
    ma = mb;
    qa = qb;
    return;
  }
  const double n = na + nb, d = mb - ma;
  ma = ma + d * (nb / n);
  qa = qa + qb + d * d * (na * (nb / n));
  na = n;
}

// A workgroup's lanes merged (wave butterfly, then the waves in order) into one
// record: hi = M2, lo = mean, amax = count.
__device__ __forceinline__ void block_var_to_record(double n, double m, double q, PartRec* dst) {
  __shared__ double sn[16], sm[16], sq[16];
#pragma unroll
  for (int k = 1; k < 64; k <<= 1) {
    const double n2 = __shfl_xor(n, k, 64), m2 = __shfl_xor(m, k, 64), q2 = __shfl_xor(q, k, 64);
    // the lower lane of each pair keeps the order (a, b); both end with the same value
    if ((threadIdx.x & k) == 0) {
      chan_merge(n, m, q, n2, m2, q2);
    } else {
      double nb = n2, mb = m2, qb = q2;
      chan_merge(nb, mb, qb, n, m, q);
      n = nb;
      m = mb;
      q = qb;
    }
  }
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) {
    sn[w] = n;
    sm[w] = m;
    sq[w] = q;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double N = sn[0], M = sm[0], Q = sq[0];
    for (int k = 1; k < nw; ++k) chan_merge(N, M, Q, sn[k], sm[k], sq[k]);
    PartRec r;
    r.hi = Q;
    r.lo = M;
    r.amax = N;
    r.pad = 0.0;
    *dst = r;
  }
}

// ===========================================================================
// Full reduction, FLAT layout: grid-stride over V-groups, one record per block.
// scale: the sum-of-squares rescaling pass multiplies each value by a power of two.
// ===========================================================================
// the accumulator of a full reduction's lane
template <typename T, int RK, bool COMP>
struct RedAcc { typedef typename AccSel<T, COMP>::type type; };
template <typename T, bool COMP>
struct RedAcc<T, RK_VAR1, COMP> { typedef AccVar<T, COMP> type; };

// The lane's accumulator (and extremum / magnitude word) combined across the
// workgroup into its record.
template <typename T, int RK, bool COMP, class Acc>
__device__ __forceinline__ void lane_to_record(const Acc& acc, const Ext<T, RK>& ext, double amax, PartRec* dst) {
  if constexpr (RK == RK_VAR1) {
    double n, m, q;
    acc.moments(n, m, q);
    block_var_to_record(n, m, q, dst);
  } else {
    double h, l;
    lane_to_words<T, COMP>(acc, h, l);
    if constexpr (RK == RK_MAX || RK == RK_MIN || RK == RK_AMAX) amax = ext.word();
    block_words_to_record<T, COMP>(h, l, amax, dst);
  }
}

template <class X, int RK, bool COMP, int V, int E, bool SCALED>
__device__ __forceinline__ void flat_reduce(const coot_kargs& a) {
  typedef typename X::T T;
  typedef typename RedAcc<T, RK, COMP>::type Acc;
  T scale = (T)1;
  if constexpr (SCALED) {
    const double* ctl = (const double*)a.ws2;
    if (ctl[0] == 0.0) return;  // no rescaling requested: the whole grid exits
    scale = (T)ctl[1];
  }
  Acc acc;
  acc.init();
  Ext<T, RK> ext;
  ext.init();
  T amax = (T)0;  // largest magnitude (sum of squares: the rescaling decision)
  const i64 n = a.n_rows * a.n_cols;
  const i64 nv = n / V;
  const int bs = blockDim.x;
  const i64 step = (i64)gridDim.x * bs * E;
  for (i64 b = (i64)blockIdx.x * bs * E + threadIdx.x; b < nv; b += step) {
    vt<T, V> x[E][X::NL];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const i64 v = b + (i64)e * bs;
      if (v < nv) load_flat<X, V, true>(a, v, x[e]);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const i64 v = b + (i64)e * bs;
      if (v < nv) {
#pragma unroll
        for (int q = 0; q < V; ++q) {
          T L[X::NL];
#pragma unroll
          for (int k = 0; k < X::NL; ++k) L[k] = x[e][k].v[q];
          take<X, RK>(acc, ext, amax, scale, L, a.sc);
        }
      }
    }
  }
  if (V > 1 && blockIdx.x == gridDim.x - 1) {
    for (i64 i = nv * V + threadIdx.x; i < n; i += bs) {
      T L[X::NL];
#pragma unroll
      for (int k = 0; k < X::NL; ++k) L[k] = leaf_at<X>(a, k, i);
      take<X, RK>(acc, ext, amax, scale, L, a.sc);
    }
  }
  PartRec* recs = (PartRec*)(SCALED ? (void*)((char*)a.ws2 + 64) : a.ws);
  lane_to_record<T, RK, COMP>(acc, ext, mag_word(amax), recs + blockIdx.x);
}

// ===========================================================================
// Two statements in one pass (multi-statement fusion): out = X, stored in the
// storage type, and the full reduction of Z, whose leaves are X's leaves as
// loaded (before the store) followed by the value just computed (L[X::NL]).
// y = 2.5*x + y then accu(x % y) reads x and y once and writes y once.
// ===========================================================================
template <class X, class Z, int RK, bool COMP, int V, int E>
__device__ __forceinline__ void flat_eval_reduce(const coot_kargs& a) {
  typedef typename X::T T;
  typedef typename X::S S;
  typedef typename AccSel<T, COMP>::type Acc;
  Acc acc;
  acc.init();
  Ext<T, RK> ext;
  ext.init();
  double amax = 0.0;
  const i64 n = a.n_rows * a.n_cols;
  const i64 nv = n / V;
  const int bs = blockDim.x;
  const i64 step = (i64)gridDim.x * bs * E;
  S* out = (S*)a.out;
  for (i64 b = (i64)blockIdx.x * bs * E + threadIdx.x; b < nv; b += step) {
    vt<T, V> x[E][X::NL];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const i64 v = b + (i64)e * bs;
      if (v < nv) load_flat<X, V>(a, v, x[e]);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const i64 v = b + (i64)e * bs;
      if (v < nv) {
        vt<T, V> r;
#pragma unroll
        for (int q = 0; q < V; ++q) {
          T L[X::NL + 1];
#pragma unroll
          for (int k = 0; k < X::NL; ++k) L[k] = x[e][k].v[q];
          L[X::NL] = r.v[q] = X::f(L, a.sc);
          consume<Z, RK>(acc, ext, L, a.sc);
        }
        stc<S, V>(out + v * V, r);
      }
    }
  }
  if (V > 1 && blockIdx.x == gridDim.x - 1) {
    for (i64 i = nv * V + threadIdx.x; i < n; i += bs) {
      T L[X::NL + 1];
#pragma unroll
      for (int k = 0; k < X::NL; ++k) L[k] = leaf_at<X>(a, k, i);
      L[X::NL] = X::f(L, a.sc);
      out[i] = St<S>::out(L[X::NL]);
      consume<Z, RK>(acc, ext, L, a.sc);
    }
  }
  double h, l;
  lane_to_words<T, COMP>(acc, h, l);
  if constexpr (RK == RK_MAX || RK == RK_MIN || RK == RK_AMAX) amax = ext.word();
  block_words_to_record<T, COMP>(h, l, amax, (PartRec*)a.ws + blockIdx.x);
}

// ===========================================================================
// TILED traversal.  TR x TC output tiles (rows x columns), 256 threads.  Parity-1
// leaves (stored n_cols x n_rows) are read along their own contiguous dimension
// into an LDS tile; parity-0 leaves and the output are accessed along output
// columns: TR / V threads cover a column segment of the tile with V-element
// accesses, and the 256 threads cover TC columns in NPASS passes.  A tall tile
// (TR > TC) gives the untransposed operands longer contiguous segments, a wide one
// the transposed operands.  Any leading dimensions and ragged edges; V > 1 only
// when every contiguous extent, leading dimension and base address allows it
// (host-checked).  The parity-0 loads of every pass are issued before the
// transposed leaves are staged (when they fit in NPASS * NL * V <= 64 registers'
// worth), so a tile's two load phases overlap instead of following each other.
// A Sink receives each element (with its leaf values) and each finished group.
// ===========================================================================
template <class X, int V, int TR, int TC>
struct TileGeom {
  static constexpr int NB = 256;
  static constexpr int TPC = TR / V;       // threads along a column segment
  static constexpr int CPP = NB / TPC;     // columns per pass
  static constexpr int NPASS = TC / CPP;   // passes per tile
  static constexpr int TPS = TC / V;       // staging: threads along a stored segment of a transposed leaf
  static constexpr int RPS = NB / TPS;     // staging: stored segments (tile rows) per pass
  static constexpr int NPS = X::NP1 > 0 ? X::NP1 : 1;
  static constexpr int N0 = X::NL - X::NP1;  // parity-0 leaves
  static constexpr bool HOIST = NPASS * (N0 > 0 ? N0 : 1) * V * (int)sizeof(typename X::T) <= 256;
  static_assert(TR % V == 0 && TC % V == 0 && TPC <= NB && TPS <= NB, "vector width must divide the tile");
  static_assert(CPP <= TC && TC % CPP == 0, "a tile's passes must cover its columns");
};

// Stage the transposed leaves of tile (i0, j0) into LDS (lds[p1][il][jl], zero
// outside the matrix).
template <class X, int V, int TR, int TC>
__device__ __forceinline__ void stage_transposed(const coot_kargs& a, typename X::T (*lds)[TR][TC + 1], i64 i0,
                                                 i64 j0) {
  typedef typename X::T T;
  typedef TileGeom<X, V, TR, TC> G;
  const int sc = threadIdx.x % G::TPS, sr = threadIdx.x / G::TPS;
  for (int il = sr; il < TR; il += G::RPS) {
    const i64 i = i0 + il, j = j0 + (i64)sc * V;
    const bool in = (i < a.n_rows) && (j < a.n_cols);
#pragma unroll
    for (int k = 0; k < X::NL; ++k) {
      if (X::par(k) == 0) continue;
      vt<T, V> v;
      if (in) {
        v = ldc<typename X::S, V>((const typename X::S*)a.leaf[X::slot(k)] + j + i * a.ld[X::slot(k)]);
      } else {
#pragma unroll
        for (int q = 0; q < V; ++q) v.v[q] = (T)0;
      }
#pragma unroll
      for (int q = 0; q < V; ++q) lds[X::p1(k) < 0 ? 0 : X::p1(k)][il][sc * V + q] = v.v[q];
    }
  }
}

// The parity-0 leaves of one pass of tile (i0, j0): column j0 + jl, rows i0 + lc * V ...
template <class X, int V>
__device__ __forceinline__ void load_pass(const coot_kargs& a, i64 i, i64 j, bool in, vt<typename X::T, V> (&x)[X::NL]) {
  if (in) {
#pragma unroll
    for (int k = 0; k < X::NL; ++k)
      if (X::par(k) == 0) x[k] = ldc<typename X::S, V>((const typename X::S*)a.leaf[X::slot(k)] + i + j * a.ld[X::slot(k)]);
  }
}

// One pass's elements handed to the sink: leaf values from the registers (parity 0)
// or the staged LDS tile (parity 1).  ELEM(q, in, L) receives element q of the group.
template <class X, int V, int TR, int TC, class F>
__device__ __forceinline__ void pass_elems(typename X::T (*lds)[TR][TC + 1], const vt<typename X::T, V> (&x)[X::NL],
                                           int lc, int jl, bool in, F&& elem) {
  typedef typename X::T T;
#pragma unroll
  for (int q = 0; q < V; ++q) {
    T L[X::NL];
#pragma unroll
    for (int k = 0; k < X::NL; ++k)
      L[k] = X::par(k) ? lds[X::p1(k) < 0 ? 0 : X::p1(k)][lc * V + q][jl] : (in ? x[k].v[q] : (T)0);
    elem(q, in, L);
  }
}

template <class X, int V, int TR, int TC, class Sink>
__device__ __forceinline__ void tiled_walk(const coot_kargs& a, Sink& sink) {
  typedef typename X::T T;
  typedef TileGeom<X, V, TR, TC> G;
  __shared__ T lds[G::NPS][TR][TC + 1];
  const i64 R = a.n_rows, C = a.n_cols;
  const i64 tr = (R + TR - 1) / TR, tc = (C + TC - 1) / TC, nt = tr * tc;
  const int lc = threadIdx.x % G::TPC, lr = threadIdx.x / G::TPC;
  for (i64 t = blockIdx.x; t < nt; t += gridDim.x) {
    const i64 ti = t % tr, tj = t / tr;
    const i64 i0 = ti * TR, j0 = tj * TC;
    const i64 i = i0 + (i64)lc * V;
    sink.begin_tile();
    vt<T, V> x[G::HOIST ? G::NPASS : 1][X::NL];
    if constexpr (G::HOIST) {
#pragma unroll
      for (int p = 0; p < G::NPASS; ++p) {
        const i64 j = j0 + lr + p * G::CPP;
        load_pass<X, V>(a, i, j, (i < R) && (j < C), x[p]);
      }
    }
    if constexpr (X::NP1 > 0) {
      stage_transposed<X, V, TR, TC>(a, lds, i0, j0);
      __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < G::NPASS; ++p) {
      const int jl = lr + p * G::CPP;
      const i64 j = j0 + jl;
      const bool in = (i < R) && (j < C);
      if constexpr (!G::HOIST) load_pass<X, V>(a, i, j, in, x[0]);
      pass_elems<X, V, TR, TC>(lds, x[G::HOIST ? p : 0], lc, jl, in,
                               [&](int q, bool inq, const T* L) { sink.elem(a, q, inq, L); });
      sink.group(a, i, j, jl, lc, in);
    }
    sink.end_tile(a, ti, tj, i0, j0, lr, lc);
    if constexpr (X::NP1 > 0) __syncthreads();
  }
}

template <class X, int V>
struct EvalSink {
  typedef typename X::T T;
  vt<T, V> r;
  __device__ __forceinline__ void begin_tile() {}
  __device__ __forceinline__ void elem(const coot_kargs& a, int q, bool in, const T* L) {
    r.v[q] = in ? X::f(L, a.sc) : (T)0;
  }
  __device__ __forceinline__ void group(const coot_kargs& a, i64 i, i64 j, int, int, bool in) {
    if (in) stc<typename X::S, V>((typename X::S*)a.out + i + j * a.out_ld, r);
  }
  __device__ __forceinline__ void end_tile(const coot_kargs&, i64, i64, i64, i64, int, int) {}
};

template <class X, int V, int TR, int TC>
__device__ __forceinline__ void tiled_eval(const coot_kargs& a) {
  EvalSink<X, V> s;
  tiled_walk<X, V, TR, TC>(a, s);
}

// Full reduction over the tiled traversal (transposed or strided leaves).
template <class X, int RK, bool COMP, bool SCALED>
struct AllSink {
  typedef typename X::T T;
  typedef typename RedAcc<T, RK, COMP>::type Acc;
  Acc acc;
  Ext<T, RK> ext;
  T amax;
  T scale;
  __device__ __forceinline__ void begin_tile() {}
  __device__ __forceinline__ void elem(const coot_kargs& a, int, bool in, const T* L) {
    if (!in) return;
    take<X, RK>(acc, ext, amax, scale, L, a.sc);
  }
  __device__ __forceinline__ void group(const coot_kargs&, i64, i64, int, int, bool) {}
  __device__ __forceinline__ void end_tile(const coot_kargs&, i64, i64, i64, i64, int, int) {}
};

template <class X, int RK, bool COMP, int V, int TR, int TC, bool SCALED>
__device__ __forceinline__ void tiled_reduce(const coot_kargs& a) {
  typedef typename X::T T;
  AllSink<X, RK, COMP, SCALED> s;
  s.acc.init();
  s.ext.init();
  s.amax = (T)0;
  s.scale = (T)1;
  if constexpr (SCALED) {
    const double* ctl = (const double*)a.ws2;
    if (ctl[0] == 0.0) return;
    s.scale = (T)ctl[1];
  }
  tiled_walk<X, V, TR, TC>(a, s);
  PartRec* recs = (PartRec*)(SCALED ? (void*)((char*)a.ws2 + 64) : a.ws);
  lane_to_record<T, RK, COMP>(s.acc, s.ext, mag_word(s.amax), recs + blockIdx.x);
}

// ===========================================================================
// Stage 2 of a full reduction: one workgroup of 256 threads folds the records
// in a fixed order and writes the result in the element type.
//   RK_SUMSQ writes sqrt of the sum (the 2-norm) and decides whether the
//   rescaled pass must run: when the largest magnitude is outside
//   [2^-L, 2^L] the squares may have overflowed or underflowed, so the control
//   block gets flag = 1 and scale = 2^-e (e the exponent of the largest |value|).
// ===========================================================================
// Mean of a binary64 pair sum (h + l) over n elements as a pair (mh, ml) of the
// compute type T: the quotient q = h / n, its remainder by one fused multiply-add
// (exact), and the correction (rem + l) / n, so that mh + ml carries the mean to
// about twice T's precision.
template <typename T>
__device__ __forceinline__ void dd_mean_pair(double h, double l, double n, T& mh, T& ml) {
  const double q = h / n;
  const double ql = (__builtin_fma(-q, n, h) + l) / n;
  mh = (T)q;
  ml = (T)((q - (double)mh) + ql);
}

// Sum of squared deviations -> variance: divided by n - 1 (or n); a count of 1
// gives 0 (the deviation of the single element is 0), NaN when it is NaN; no
// elements give NaN (their mean is 0 / 0).
__device__ __forceinline__ double var_of(double ss, double n, bool by_n) {
  if (n == 0.0) return __builtin_nan("");
  const double den = by_n ? n : n - 1.0;
  return den > 0.0 ? ss / den : ss;
}

// Stage 2 of the one-pass variance: the records' (count, mean, M2) merged by
// Chan's formula in a fixed order (thread-strided, then a tree), M2 / (N - 1) or / N.
template <typename S, bool BY_N>
__device__ __forceinline__ void var_stage2(const coot_kargs& a) {
  typedef typename St<S>::C T;
  __shared__ double sn[256], sm[256], sq[256];
  const PartRec* recs = (const PartRec*)a.ws;
  double N = 0.0, M = 0.0, Q = 0.0;
  for (i64 k = threadIdx.x; k < a.n_part; k += 256) {
    const PartRec r = recs[k];
    chan_merge(N, M, Q, r.amax, r.lo, r.hi);
  }
  sn[threadIdx.x] = N;
  sm[threadIdx.x] = M;
  sq[threadIdx.x] = Q;
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s) {
      double n1 = sn[threadIdx.x], m1 = sm[threadIdx.x], q1 = sq[threadIdx.x];
      chan_merge(n1, m1, q1, sn[threadIdx.x + s], sm[threadIdx.x + s], sq[threadIdx.x + s]);
      sn[threadIdx.x] = n1;
      sm[threadIdx.x] = m1;
      sq[threadIdx.x] = q1;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) ((S*)a.out)[0] = St<S>::out((T)var_of(sq[0], sn[0], BY_N));
}

template <typename S, int RK, bool COMP, bool SCALED>
__device__ __forceinline__ void reduce_stage2(const coot_kargs& a) {
  typedef typename St<S>::C T;  // compute type; the result is stored as S
  if constexpr (RK == RK_VAR || RK == RK_VARN) {
    var_stage2<S, RK == RK_VARN>(a);
    return;
  }
  __shared__ double sh[256], sl[256], sm[256];
  const PartRec* recs = (const PartRec*)(SCALED ? (const void*)((const char*)a.ws2 + 64) : (const void*)a.ws);
  double* ctl = (double*)a.ws2;
  if constexpr (SCALED) {
    if (ctl[0] == 0.0) return;
  }
  constexpr bool is_int = is_int_t<T>::v;
  double H = 0.0, Lo = 0.0, M = ext_identity<RK>();
  for (i64 k = threadIdx.x; k < a.n_part; k += 256) {
    const PartRec r = recs[k];
    if (is_int) {
      H = (double)((u32)H + (u32)r.hi);
    } else if (COMP) {
      dw_add<double>(H, Lo, r.hi, r.lo);
    } else if (sizeof(T) == 4) {
      H = (double)((float)H + (float)r.hi);
    } else {
      H = H + r.hi;
    }
    M = nmax(M, r.amax);
  }
  sh[threadIdx.x] = H;
  sl[threadIdx.x] = Lo;
  sm[threadIdx.x] = M;
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s) {
      double h2 = sh[threadIdx.x + s], l2 = sl[threadIdx.x + s];
      double h1 = sh[threadIdx.x], l1 = sl[threadIdx.x];
      if (is_int) {
        h1 = (double)((u32)h1 + (u32)h2);
      } else if (COMP) {
        dw_add<double>(h1, l1, h2, l2);
      } else if (sizeof(T) == 4) {
        h1 = (double)((float)h1 + (float)h2);
      } else {
        h1 = h1 + h2;
      }
      sh[threadIdx.x] = h1;
      sl[threadIdx.x] = l1;
      sm[threadIdx.x] = nmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    S* out = (S*)a.out;
    const double tot = sh[0] + sl[0];
    if (RK == RK_MAX || RK == RK_AMAX) {
      out[0] = St<S>::out((T)sm[0]);  // an element value (or its magnitude): exact
    } else if (RK == RK_MIN) {
      out[0] = St<S>::out((T)(-sm[0]));
    } else if (is_int) {
      out[0] = St<S>::out((T)(u32)sh[0]);
    } else if (RK == RK_MEAN) {
      out[0] = St<S>::out((T)(tot / (double)(a.n_rows * a.n_cols)));
    } else if (RK != RK_SUMSQ) {
      // one rounding from binary64 (a second one, to a 16-bit type, is innocuous)
      out[0] = St<S>::out((T)tot);
    } else {
      const double mx = sm[0];
      double scale = SCALED ? ctl[1] : 1.0;
      double nrm = __builtin_sqrt(tot) / scale;
      out[0] = St<S>::out((T)nrm);
      if constexpr (!SCALED) {
        const double lim_hi = sizeof(T) == 4 ? 0x1p50 : 0x1p400;
        const double lim_lo = sizeof(T) == 4 ? 0x1p-50 : 0x1p-400;
        const bool risky = mx > 0.0 && (mx > lim_hi || mx < lim_lo || !(tot < 1e300));
        if (risky) {
          int e;
          (void)__builtin_frexp(mx, &e);
          ctl[0] = 1.0;
          ctl[1] = __builtin_ldexp(1.0, -e);
        } else {
          ctl[0] = 0.0;
          ctl[1] = 1.0;
        }
      }
    }
  }
}

// ===========================================================================
// Dimension reductions over the tiled traversal.
//   DIM 0 (per column, 1 x n_cols): each group of TPC lanes owns one column
//     segment; the pair-sum over the segment goes to ws[ti * n_cols + j].
//   DIM 1 (per row, n_rows x 1): each thread keeps V row accumulators across
//     its passes; at the end of the tile they are folded across the CPP column
//     passes through LDS and written to ws[tj * n_rows + i].
// Partials are (hi, lo) pairs of the element type (float-float for fp32).
// ===========================================================================
template <typename T> struct Pair { T hi, lo; };

template <typename T, bool COMP>
__device__ __forceinline__ Pair<T> acc_pair(const typename AccSel<T, COMP>::type& g) {
  Pair<T> p;
  if constexpr (!is_int_t<T>::v && COMP) {
    p.hi = g.hi;
    p.lo = g.lo;
  } else {
    p.hi = g.s;
    p.lo = (T)0;
  }
  return p;
}

template <typename T, bool COMP>
__device__ __forceinline__ void pair_add(T& h, T& l, const Pair<T>& p) {
  if constexpr (is_int_t<T>::v) {
    h = op_add(h, p.hi);
  } else if constexpr (COMP) {
    dw_add<T>(h, l, p.hi, p.lo);
  } else {
    h = h + p.hi;
  }
}

// ===========================================================================
// Dimension reductions over segments.  The tiles along the reduced dimension are
// cut into n_part segments of K = ceil(tiles / n_part) consecutive tiles; one
// workgroup walks a whole segment, each lane accumulating its elements in
// registers (float-float when compensated), and writes one partial per output
// element of the segment, ws[o * n_part + segment], after a single combine of the
// lanes through LDS; dim_stage2 folds each output's partials.  The tile traversal
// (coalesced column segments, transposed leaves staged through LDS) is the one of
// tiled_walk.
// ===========================================================================
template <class X, int V, int TR, int TC, int DIM, class Sink>
__device__ __forceinline__ void tiled_walk_seg(const coot_kargs& a, Sink& sink) {
  typedef typename X::T T;
  typedef TileGeom<X, V, TR, TC> G;
  __shared__ T lds[G::NPS][TR][TC + 1];
  const i64 R = a.n_rows, C = a.n_cols;
  const i64 tr = (R + TR - 1) / TR, tc = (C + TC - 1) / TC;
  const i64 nred = DIM == 0 ? tr : tc, nkeep = DIM == 0 ? tc : tr;
  const i64 K = (nred + a.n_part - 1) / a.n_part;
  const i64 nseg = nkeep * a.n_part;
  const int lc = threadIdx.x % G::TPC, lr = threadIdx.x / G::TPC;
  for (i64 sgi = blockIdx.x; sgi < nseg; sgi += gridDim.x) {
    // neighbouring workgroups take neighbouring output strips of the same segment
    // (measured faster for sum(., 0) than neighbouring segments of one strip)
    const i64 keep = sgi % nkeep, sg = sgi / nkeep;
    sink.begin_seg(a, keep * (DIM == 0 ? TC : TR), lr, lc);
    const i64 r_end = sg * K + K < nred ? sg * K + K : nred;
    for (i64 r = sg * K; r < r_end; ++r) {
      const i64 ti = DIM == 0 ? r : keep, tj = DIM == 0 ? keep : r;
      const i64 i0 = ti * TR, j0 = tj * TC;
      const i64 i = i0 + (i64)lc * V;
      vt<T, V> x[G::HOIST ? G::NPASS : 1][X::NL];
      if constexpr (G::HOIST) {
#pragma unroll
        for (int p = 0; p < G::NPASS; ++p) {
          const i64 j = j0 + lr + p * G::CPP;
          load_pass<X, V>(a, i, j, (i < R) && (j < C), x[p]);
        }
      }
      if constexpr (X::NP1 > 0) {
        stage_transposed<X, V, TR, TC>(a, lds, i0, j0);
        __syncthreads();
      }
#pragma unroll
      for (int p = 0; p < G::NPASS; ++p) {
        const int jl = lr + p * G::CPP;
        const i64 j = j0 + jl;
        const bool in = (i < R) && (j < C);
        if constexpr (!G::HOIST) load_pass<X, V>(a, i, j, in, x[0]);
        pass_elems<X, V, TR, TC>(lds, x[G::HOIST ? p : 0], lc, jl, in,
                                 [&](int q, bool inq, const T* L) { sink.elem(a, p, q, inq, L); });
      }
      if constexpr (X::NP1 > 0) __syncthreads();
    }
    sink.end_seg(a, keep * (DIM == 0 ? TC : TR), sg, lr, lc);
  }
}

// One output's n_part partials folded by one wavefront: lane l takes k = l, l + 64,
// ... in order, then a fixed butterfly combines the lanes (the result does not
// depend on timing).
template <typename T, bool COMP>
__device__ __forceinline__ void fold_pairs(const Pair<T>* ws, i64 o, i64 n_part, int lane, T& h, T& l) {
  h = (T)0;
  l = (T)0;
  for (i64 k = lane; k < n_part; k += 64) pair_add<T, COMP>(h, l, ws[o * n_part + k]);
  if constexpr (is_int_t<T>::v) {
    h = wave_sum<T>(h);
  } else if constexpr (COMP) {
    wave_dw_sum<T>(h, l);
  } else {
    h = wave_sum<T>(h);
  }
}

// Stage 2 of a dimension reduction runs one wavefront per output; MODE says what it
// writes from the folded partials over cnt elements:
//   DM_SUM the sum; DM_MEAN the sum / cnt, rounded once; DM_VAR / DM_VARN the
//   variance from the shifted moments (sum d^2 in ws, sum d in ws2):
//   M2 = S2 - S1^2 / cnt in binary64, divided by cnt - 1 or cnt.
enum { DM_SUM = 0, DM_MEAN = 1, DM_VAR = 3, DM_VARN = 4 };

template <typename S, bool COMP, int MODE>
__device__ __forceinline__ void fold_output(const coot_kargs& a, i64 o, int lane, i64 cnt) {
  typedef typename St<S>::C T;  // partials in the compute type, the result stored as S
  T h, l;
  fold_pairs<T, COMP>((const Pair<T>*)a.ws, o, a.n_part, lane, h, l);
  if constexpr (MODE == DM_VAR || MODE == DM_VARN) {
    T h1, l1;
    fold_pairs<T, COMP>((const Pair<T>*)a.ws2, o, a.n_part, lane, h1, l1);
    if (lane == 0) {
      // the pairs as binary64 words: exact for fp32; for fp64 h + l rounds to h
      const double s2 = (double)h + (double)l, s1 = (double)h1 + (double)l1, n = (double)cnt;
      ((S*)a.out)[o] = St<S>::out((T)var_of(s2 - s1 * (s1 / n), n, MODE == DM_VARN));
    }
    return;
  }
  if (lane == 0) {
    if constexpr (is_int_t<T>::v) {
      ((S*)a.out)[o] = St<S>::out(h);
    } else if constexpr (MODE == DM_SUM) {
      ((S*)a.out)[o] = St<S>::out(h + l);
    } else {
      T mh, ml;
      dd_mean_pair<T>((double)h, (double)l, (double)cnt, mh, ml);
      ((S*)a.out)[o] = St<S>::out((T)((double)mh + (double)ml));
    }
  }
}

// The expression's value at element (i, j), whatever its leaves' layouts (a
// transposed leaf reads its element (j, i); a broadcast leaf has column stride 0).
template <class X>
__device__ __forceinline__ typename X::T value_at(const coot_kargs& a, i64 i, i64 j) {
  typedef typename X::T T;
  T L[X::NL];
#pragma unroll
  for (int k = 0; k < X::NL; ++k) {
    const typename X::S* p = (const typename X::S*)a.leaf[X::slot(k)];
    const i64 ld = a.ld[X::slot(k)];
    L[k] = ldc<typename X::S, 1>(X::par(k) ? p + j + i * ld : p + i + j * ld).v[0];
  }
  return X::f(L, a.sc);
}

// Shifted moments of one output's elements (variance along a dimension, one pass):
// d = v - K exactly (TwoSum), d^2 exactly (TwoProd), sum d and sum d^2 float-float
// (plain sums when not compensated).  K, the output's first element, is the same in
// every segment, so the segments' sums add up and M2 = S2 - S1^2 / n at the end.
template <typename T, bool COMP>
struct AccShift {
  T s1h, s1l, s2h, s2l;
  __device__ __forceinline__ void init() { s1h = s1l = s2h = s2l = (T)0; }
  __device__ __forceinline__ void add(T x, T K) {
    T dh, dl;
    two_sum(x, -K, dh, dl);
    if constexpr (COMP) {
      T p, pe, t, e;
      two_prod(dh, dh, p, pe);
      two_sum(s1h, dh, t, e);
      s1h = t;
      s1l += e + dl;
      two_sum(s2h, p, t, e);
      s2h = t;
      s2l += e + (pe + (T)2 * dh * dl);
    } else {
      s1h += dh;
      s2h += dh * dh;
    }
  }
};

// Per-lane accumulator of a dimension reduction: a sum, or (VAR) shifted moments.
template <typename T, bool COMP, bool VAR>
struct DimAcc {
  typename AccSel<T, COMP>::type g;
  __device__ __forceinline__ void init() { g.init(); }
  __device__ __forceinline__ void add(T x, T) { g.add(x); }
  __device__ __forceinline__ Pair<T> part(int) const { return acc_pair<T, COMP>(g); }
};
template <typename T, bool COMP>
struct DimAcc<T, COMP, true> {
  AccShift<T, COMP> g;
  __device__ __forceinline__ void init() { g.init(); }
  __device__ __forceinline__ void add(T x, T K) { g.add(x, K); }
  // moment m: 1 -> (s1h, s1l), 2 -> (s2h, s2l)
  __device__ __forceinline__ Pair<T> part(int m) const {
    Pair<T> q;
    q.hi = m == 1 ? g.s1h : g.s2h;
    q.lo = m == 1 ? g.s1l : g.s2l;
    return q;
  }
};

// sum(., 0): lane (lr, lc) of pass p covers column lr + p * CPP of the tile, rows
// lc * V .. lc * V + V - 1; it keeps one accumulator per pass.  At the end of the
// segment the TPC lanes of each column are combined in LDS by one thread per column.
// VAR: each accumulator holds the shifted moments of its column about the column's
// first element, evaluated at the segment's start; sum d^2 goes to ws and sum d to
// ws2, one LDS combine each.
template <class X, bool COMP, int V, int TR, int TC, bool VAR>
struct Dim0SegSink {
  typedef typename X::T T;
  static constexpr int TPC = TR / V, CPP = 256 / TPC, NPASS = TC / CPP;
  DimAcc<T, COMP, VAR> g[NPASS];
  T K[VAR ? NPASS : 1];
  __device__ __forceinline__ void begin_seg(const coot_kargs& a, i64 j0, int lr, int) {
#pragma unroll
    for (int p = 0; p < NPASS; ++p) g[p].init();
    if constexpr (VAR) {
#pragma unroll
      for (int p = 0; p < NPASS; ++p) {
        const i64 j = j0 + lr + p * CPP;
        K[p] = (j < a.n_cols && a.n_rows > 0) ? value_at<X>(a, 0, j) : (T)0;
      }
    } else {
      K[0] = (T)0;
    }
  }
  __device__ __forceinline__ void elem(const coot_kargs& a, int p, int, bool in, const T* L) {
    if (in) {
#pragma unroll
      for (int pp = 0; pp < NPASS; ++pp)
        if (pp == p) g[pp].add(X::f(L, a.sc), K[VAR ? pp : 0]);
    }
  }
  __device__ __forceinline__ void end_seg(const coot_kargs& a, i64 j0, i64 sg, int lr, int lc) {
    __shared__ Pair<T> red[TC][TPC + 1];
#pragma unroll
    for (int m = VAR ? 2 : 0; m >= (VAR ? 1 : 0); --m) {
#pragma unroll
      for (int p = 0; p < NPASS; ++p) red[lr + p * CPP][lc] = g[p].part(m);
      __syncthreads();
      if ((int)threadIdx.x < TC) {
        const int jl = threadIdx.x;
        T h = red[jl][0].hi, l = red[jl][0].lo;
        for (int k = 1; k < TPC; ++k) pair_add<T, COMP>(h, l, red[jl][k]);
        const i64 j = j0 + jl;
        if (j < a.n_cols) {
          Pair<T> q;
          q.hi = h;
          q.lo = l;
          ((Pair<T>*)(m == 1 ? a.ws2 : a.ws))[j * a.n_part + sg] = q;
        }
      }
      __syncthreads();
    }
  }
};

// sum(., 1): a lane's rows (lc * V .. lc * V + V - 1 of the row strip) stay fixed over
// the segment; its V accumulators are combined across the CPP lanes of each row in LDS.
// VAR: as for columns, about each row's first element.
template <class X, bool COMP, int V, int TR, int TC, bool VAR>
struct Dim1SegSink {
  typedef typename X::T T;
  static constexpr int TPC = TR / V, CPP = 256 / TPC;
  DimAcc<T, COMP, VAR> r[V];
  T K[VAR ? V : 1];
  __device__ __forceinline__ void begin_seg(const coot_kargs& a, i64 i0, int, int lc) {
#pragma unroll
    for (int q = 0; q < V; ++q) r[q].init();
    if constexpr (VAR) {
#pragma unroll
      for (int q = 0; q < V; ++q) {
        const i64 i = i0 + lc * V + q;
        K[q] = (i < a.n_rows && a.n_cols > 0) ? value_at<X>(a, i, 0) : (T)0;
      }
    } else {
      K[0] = (T)0;
    }
  }
  __device__ __forceinline__ void elem(const coot_kargs& a, int, int q, bool in, const T* L) {
    if (in) {
#pragma unroll
      for (int qq = 0; qq < V; ++qq)
        if (qq == q) r[qq].add(X::f(L, a.sc), K[VAR ? qq : 0]);
    }
  }
  __device__ __forceinline__ void end_seg(const coot_kargs& a, i64 i0, i64 sg, int lr, int lc) {
    __shared__ Pair<T> red[CPP][TR];
#pragma unroll
    for (int m = VAR ? 2 : 0; m >= (VAR ? 1 : 0); --m) {
#pragma unroll
      for (int q = 0; q < V; ++q) red[lr][lc * V + q] = r[q].part(m);
      __syncthreads();
      if ((int)threadIdx.x < TR) {
        const int il = threadIdx.x;
        T h = red[0][il].hi, l = red[0][il].lo;
        for (int k = 1; k < CPP; ++k) pair_add<T, COMP>(h, l, red[k][il]);
        const i64 i = i0 + il;
        if (i < a.n_rows) {
          Pair<T> p;
          p.hi = h;
          p.lo = l;
          ((Pair<T>*)(m == 1 ? a.ws2 : a.ws))[i * a.n_part + sg] = p;
        }
      }
      __syncthreads();
    }
  }
};

// VAR: one-pass variance (shifted moments; sum d^2 partials in ws, sum d in ws2)
template <class X, int DIM, bool COMP, int V, int TR, int TC, bool VAR = false>
__device__ __forceinline__ void tiled_reduce_dim(const coot_kargs& a) {
  if constexpr (DIM == 0) {
    Dim0SegSink<X, COMP, V, TR, TC, VAR> s;
    tiled_walk_seg<X, V, TR, TC, 0>(a, s);
  } else {
    Dim1SegSink<X, COMP, V, TR, TC, VAR> s;
    tiled_walk_seg<X, V, TR, TC, 1>(a, s);
  }
}

// n_out outputs, each over cnt elements (n_rows along dim 0, n_cols along dim 1)
template <typename S, bool COMP, int MODE>
__device__ __forceinline__ void dim_stage2(const coot_kargs& a, i64 n_out, i64 cnt) {
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  for (i64 o = (i64)blockIdx.x * wpb + (threadIdx.x >> 6); o < n_out; o += (i64)gridDim.x * wpb)
    fold_output<S, COMP, MODE>(a, o, lane, cnt);
}

}  // namespace coot
