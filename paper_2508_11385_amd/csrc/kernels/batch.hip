// Persistent interpreter for batches of small independent expressions.
//
// The paper notes that GPUs are ill-suited to small matrices unless enough of
// them keep the device busy (Section 4, second difference).  Here thousands of
// small expressions run in ONE launch: a fixed grid walks a work-list of tiles
// (round-robin, no atomics, so a replayed graph needs no reset), and every tile
// evaluates its expression's bytecode.
//
// Tiles.  An expression whose leaves are all read untransposed and contiguous is
// treated as one flat array: a tile is a chunk of 4 * NT consecutive elements and
// each thread owns 4 consecutive ones (one 128-bit access per leaf when aligned).
// Other expressions use TS x TS output tiles: their transposed leaves are staged
// through LDS along their own contiguous dimension, as in the fused tiled
// kernels, and each thread owns a 4-row column segment (128-bit accesses when the
// layout allows it) or 4 elements in 4 columns.
//
// Bytecode (u32 per instruction): bits 0-5 opcode, 6-8 register b, 9-31 argument,
// emitted in Sethi-Ullman order so registers form a stack:
//   LEAF / SCAL   push into register b (the previous top, register b-1, moves to LDS)
//   binary op     r[b] = op(r[b], r[b+1]); R-variant r[b] = op(r[b+1], r[b])
//   op WITH_LEAF / WITH_SCAL   r[b] = op(r[b], leaf or scalar `argument`)
//   unary op      r[b] = op(r[b])
// The top of the stack stays in VGPRs (`acc`); the entries below it live in a
// per-thread LDS stack indexed by the (wave-uniform) register number, so no
// register file is ever addressed indirectly.  LDS is sized per batch at launch:
// `nstk` stack entries (the deepest expression's need) and `np1` staged tiles
// (the most transposed leaves any expression has, capped); further transposed
// leaves are read from global memory directly.
#include <hip/hip_runtime.h>

#include "device/coot_dev.h"
#include "batch_abi.h"

namespace coot {
namespace batch {

// acc[m] = op(acc[m], x[m]) (R-variants: op(x[m], acc[m])); one dispatch for the E values
template <typename T, int E>
__device__ __forceinline__ void apply_bin(u32 op, T (&acc)[E], const T (&x)[E]) {
  switch (op) {
    case OP_ADD:
#pragma unroll
      for (int q = 0; q < E; ++q) acc[q] = op_add(acc[q], x[q]);
      break;
    case OP_SUB:
#pragma unroll
      for (int q = 0; q < E; ++q) acc[q] = op_sub(acc[q], x[q]);
      break;
    case OP_MUL:
#pragma unroll
      for (int q = 0; q < E; ++q) acc[q] = op_mul(acc[q], x[q]);
      break;
    case OP_DIV:
#pragma unroll
      for (int q = 0; q < E; ++q) acc[q] = op_div(acc[q], x[q]);
      break;
    case OP_RSUB:
#pragma unroll
      for (int q = 0; q < E; ++q) acc[q] = op_sub(x[q], acc[q]);
      break;
    default:  // OP_RDIV
#pragma unroll
      for (int q = 0; q < E; ++q) acc[q] = op_div(x[q], acc[q]);
      break;
  }
}

template <typename T, int E>
__device__ __forceinline__ void apply_un(u32 op, T (&acc)[E]) {
  switch (op) {
    case OP_NEG:
#pragma unroll
      for (int q = 0; q < E; ++q) acc[q] = op_neg(acc[q]);
      break;
    case OP_ABS:
#pragma unroll
      for (int q = 0; q < E; ++q) acc[q] = op_abs(acc[q]);
      break;
    case OP_EXP:
#pragma unroll
      for (int q = 0; q < E; ++q) acc[q] = op_exp(acc[q]);
      break;
    case OP_LOG:
#pragma unroll
      for (int q = 0; q < E; ++q) acc[q] = op_log(acc[q]);
      break;
    case OP_SQRT:
#pragma unroll
      for (int q = 0; q < E; ++q) acc[q] = op_sqrt(acc[q]);
      break;
    default:  // OP_SQUARE
#pragma unroll
      for (int q = 0; q < E; ++q) acc[q] = op_square(acc[q]);
      break;
  }
}

// E values of one thread (E / 4 groups of 4)
template <typename T, int E> struct Vals { T v[E]; };

// transposed leaves staged in LDS per tile (at most): 4 by LDS DMA on one-wave tiles,
// 2 through registers on larger ones (each costs 4 registers per thread in flight)
template <int NT> struct Staged { static constexpr int N = NT == 64 ? 4 : 2; };
constexpr int kXcds = 8;       // accelerator complex dies of an MI355X, each with its own L2

// Raw buffer access.  Every leaf and every output is addressed through a buffer
// resource whose range is the operand's extent (under 2^31 bytes).  A lane that
// must not touch memory (an element past the matrix edge) passes an offset beyond
// every range: the hardware returns 0 for such a load and drops such a store, so
// no access needs a per-lane branch (exec-mask save and restore) around it.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 raw buffer descriptor: 32-bit data format, no swizzle
constexpr int kStoreNt = 2;             // cache policy of result stores: non-temporal

// byte offset o (below 2^31) if the lane's element exists, else an offset outside
// every range (bit 31 set), without a branch
__device__ __forceinline__ u32 masked(u32 o, bool in) { return o | ((u32)!in << 31); }

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, u32 bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kRsrcWord3);
}

template <typename T> struct Buf;
template <> struct Buf<float> {
  static __device__ __forceinline__ float ld1(rsrc_t r, u32 off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  }
  static __device__ __forceinline__ vt<float, 4> ld4(rsrc_t r, u32 off) {
    // (copied whole: a bit cast of one element of a vector value reads element 0)
    const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    vt<float, 4> g;
    __builtin_memcpy(&g, &q, 16);
    return g;
  }
  static __device__ __forceinline__ void st1(rsrc_t r, u32 off, float x) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(u32, x), r, off, 0, kStoreNt);
  }
  static __device__ __forceinline__ void st4(rsrc_t r, u32 off, const float (&x)[4]) {
    u32x4 q;
    __builtin_memcpy(&q, x, 16);
    __builtin_amdgcn_raw_buffer_store_b128(q, r, off, 0, kStoreNt);
  }
};
template <> struct Buf<double> {
  static __device__ __forceinline__ double ld1(rsrc_t r, u32 off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  }
  static __device__ __forceinline__ vt<double, 4> ld4(rsrc_t r, u32 off) {
    const u32x4 q0 = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    const u32x4 q1 = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u, 0, 0);
    vt<double, 4> g;
    __builtin_memcpy(&g.v[0], &q0, 16);
    __builtin_memcpy(&g.v[2], &q1, 16);
    return g;
  }
  static __device__ __forceinline__ void st1(rsrc_t r, u32 off, double x) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, off, 0, kStoreNt);
  }
  static __device__ __forceinline__ void st4(rsrc_t r, u32 off, const double (&x)[4]) {
    u32x4 q0, q1;
    __builtin_memcpy(&q0, &x[0], 16);
    __builtin_memcpy(&q1, &x[2], 16);
    __builtin_amdgcn_raw_buffer_store_b128(q0, r, off, 0, kStoreNt);
    __builtin_amdgcn_raw_buffer_store_b128(q1, r, off + 16u, 0, kStoreNt);
  }
};

// untransposed leaves loaded before the bytecode runs (2-D tiles also hold their
// staged transposed leaves in registers, so they prefetch fewer; threads owning more
// elements prefetch fewer leaves)
template <typename T, bool FLAT, int G> struct Prefetch {
  static constexpr int B = FLAT ? (sizeof(T) == 4 ? 6 : 4) : (sizeof(T) == 4 ? 3 : 2);
  static constexpr int N = B / G > 0 ? B / G : 1;
};

// Occupancy targets (waves per SIMD) that cap the registers the compiler may use:
// fp32 flat chunks of 4 elements fit 64 registers (8 waves).  Threads owning 8 or 16
// elements keep 3 and 2 waves per SIMD: as many elements in flight per CU as 6 - 8
// waves of 4-element threads, without spilling the unrolled exp / log evaluations.
template <typename T, int G, bool FLAT> struct Waves {
  static constexpr int N = G == 1 ? (FLAT && sizeof(T) == 4 ? 8 : 1) : (G == 2 ? 3 : 2);
};

// FLAT: the tile range holds flat chunks only (no staging, no 2-D index maps: fewer
// registers, more waves per SIMD); otherwise 2-D tiles only.
// A tile (TS x TS elements, or a flat chunk of TS * TS) is covered by NT = TS*TS/(4G)
// threads owning E = 4G elements each: G groups of 4 consecutive elements (a flat
// chunk; a 4-row column segment of a 2-D tile when 128-bit accesses are valid) or
// E elements in E columns of one row.  The interpreter's scalar work (tile header,
// decoding and dispatch of every instruction) runs once per wavefront, so larger G
// spreads it over more elements.
template <typename T, int TS, int G, bool FLAT>
__global__ __launch_bounds__(TS * TS / (4 * G)) __attribute__((amdgpu_waves_per_eu(Waves<T, G, FLAT>::N))) void interp(
    const BatchExpr* __restrict__ ex, const u32* __restrict__ tiles, int t_begin, int t_end,
    const u32* __restrict__ code, const T* __restrict__ scal, int nstk, int np1) {
  constexpr int NT = TS * TS / (4 * G);  // threads
  constexpr int E = 4 * G;               // elements per thread
  constexpr int PF = Prefetch<T, FLAT, G>::N;
  constexpr u32 ES = sizeof(T);
  // One-wave 2-D tiles stage their transposed leaves by LDS DMA (buffer loads that
  // write LDS directly): no registers hold them in flight and, the wave being alone
  // in its workgroup, no barrier orders the staging area.  Slot layout: element
  // (row il, column sc) of the tile at il * TS + ((sc + il) mod TS), the rotation
  // spreading a column's reads over the LDS banks.  Larger tiles stage through
  // registers into a padded [TS][TS + 1] layout between two barriers.
  constexpr bool DMA = !FLAT && NT == 64;
  constexpr int kMaxStaged = Staged<NT>::N;
  extern __shared__ __align__(16) unsigned char smem[];
  vt<T, 4>* stk = reinterpret_cast<vt<T, 4>*>(smem);                                  // [nstk][G][NT]
  T* stage = reinterpret_cast<T*>(smem + (size_t)nstk * G * NT * sizeof(vt<T, 4>));  // [np1][TS][TS (+1)]
  const int tid = threadIdx.x;
  exp_table_to_lds<T>();
  // Workgroup i runs on XCD i % 8.  Renumber workgroups so that consecutive logical
  // numbers share an XCD: neighbouring tiles of an expression (whose column segments
  // share cache lines when the leading dimension is not a multiple of the line) then
  // meet in the same L2.
  const int g = (int)gridDim.x, bid = (int)blockIdx.x;
  const int lb = (g % kXcds == 0) ? (bid % kXcds) * (g / kXcds) + bid / kXcds : bid;
  for (int t = t_begin + lb; t < t_end; t += g) {
    const u32 eid = tiles[2 * t], tin = tiles[2 * t + 1];
    const BatchExpr& e = ex[eid];
    const int R = e.n_rows, C = e.n_cols;
    const bool v4 = e.vec4 != 0;
    const u32 p1 = e.p1_mask;
    // this thread's E elements: flat indices fb0 + (m / 4) * 4 * NT + m % 4 (flat chunk), or
    // rows iq(m) and columns jq(m) (2-D tile): 4-row column segments in G columns CPG
    // apart (128-bit accesses valid), else one row, E columns RS apart
    constexpr int TPC = TS / 4, CPG = NT / TPC, RS = NT / TS;
    u32 fb0 = 0;
    u32 n = 0;
    bool full = false;  // flat: every element of the chunk exists (uniform)
    int i0 = 0, j0 = 0, ib = 0, jb = 0;
    Vals<T, E> sv[kMaxStaged];
    if constexpr (FLAT) {
      n = (u32)R * (u32)C;
      const u32 tb = tin * (u32)(TS * TS);
      full = tb + (u32)(TS * TS) <= n;
      fb0 = tb + 4u * (u32)tid;
    } else {
      i0 = (int)(tin & e.tile_mask) * TS;
      j0 = (int)(tin >> e.tile_shift) * TS;
      ib = v4 ? i0 + 4 * (tid % TPC) : i0 + tid % TS;
      jb = v4 ? j0 + tid / TPC : j0 + tid / TS;
      // staged transposed leaves: this thread's E values of each (element idx = tid + m * NT
      // of the tile, read along the leaf's contiguous dimension), loads issued together
      if (DMA && p1 && np1 > 0) {
        // (the previous tile's reads of the staging area are complete: their values were used)
        constexpr int W = sizeof(T) / 4;       // dwords per element
        constexpr int LQ = TS * TS * W / 64;   // dword loads per lane per staged leaf
        u32 rest = p1;
#pragma unroll
        for (int sl = 0; sl < kMaxStaged; ++sl) {
          if (sl < np1 && rest != 0u) {
            const int k = __builtin_ctz(rest);
            rest &= rest - 1u;
            const rsrc_t r = make_rsrc(e.leaf[k], e.nrec[k]);
            const u32 ld = e.ld[k];
#pragma unroll
            for (int q = 0; q < LQ; ++q) {
              // dword p = q * 64 + lane of the slot: element p / W (its half p % W)
              const int el = (q * 64 + tid) / W, half = (q * 64 + tid) % W;
              const int il = el / TS, sc = (el % TS - il) & (TS - 1);
              const int i = i0 + il, j = j0 + sc;
              const u32 off = masked(((u32)j + (u32)i * ld) * ES + 4u * (u32)half, i < R && j < C);
              __builtin_amdgcn_raw_ptr_buffer_load_lds(
                  r, (__attribute__((address_space(3))) void*)(stage + sl * TS * TS + q * 64 / W), 4, off, 0, 0, 0);
            }
          }
        }
      } else if (p1 && np1 > 0) {
        u32 rest = p1;
#pragma unroll
        for (int sl = 0; sl < kMaxStaged; ++sl) {
          if (sl < np1 && rest != 0u) {
            const int k = __builtin_ctz(rest);
            rest &= rest - 1u;
            const rsrc_t r = make_rsrc(e.leaf[k], e.nrec[k]);
            const u32 ld = e.ld[k];
#pragma unroll
            for (int m = 0; m < E; ++m) {
              const int idx = tid + m * NT, i = i0 + idx / TS, j = j0 + idx % TS;
              sv[sl].v[m] = Buf<T>::ld1(r, masked(((u32)j + (u32)i * ld) * ES, i < R && j < C));
            }
          }
        }
      }
    }
    auto iq = [&](int m) __attribute__((always_inline)) { return v4 ? ib + (m & 3) : ib; };
    auto jq = [&](int m) __attribute__((always_inline)) { return v4 ? jb + (m >> 2) * CPG : jb + RS * m; };
    auto inq = [&](int m) __attribute__((always_inline)) {
      return FLAT ? fb0 + (u32)((m >> 2) * 4 * NT + (m & 3)) < n : (iq(m) < R && jq(m) < C);
    };
    auto fbq = [&](int gg) __attribute__((always_inline)) { return fb0 + (u32)(gg * 4 * NT); };
    // an untransposed leaf's E values for this thread (flat chunk or 2-D tile layout)
    auto load_direct = [&](int k) __attribute__((always_inline)) {
      Vals<T, E> v;
      const rsrc_t r = make_rsrc(e.leaf[k], e.nrec[k]);
      if (FLAT) {
#pragma unroll
        for (int gg = 0; gg < G; ++gg) {
          if (v4 && full) {
            const vt<T, 4> x = Buf<T>::ld4(r, fbq(gg) * ES);
#pragma unroll
            for (int q = 0; q < 4; ++q) v.v[4 * gg + q] = x.v[q];
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) v.v[4 * gg + q] = Buf<T>::ld1(r, masked((fbq(gg) + (u32)q) * ES, inq(4 * gg + q)));
          }
        }
      } else {
        const u32 ld = e.ld[k];
        if (v4) {
#pragma unroll
          for (int gg = 0; gg < G; ++gg) {
            const vt<T, 4> x =
                Buf<T>::ld4(r, masked(((u32)iq(4 * gg) + (u32)jq(4 * gg) * ld) * ES, inq(4 * gg)));
#pragma unroll
            for (int q = 0; q < 4; ++q) v.v[4 * gg + q] = x.v[q];
          }
        } else {
#pragma unroll
          for (int m = 0; m < E; ++m) v.v[m] = Buf<T>::ld1(r, masked(((u32)iq(m) + (u32)jq(m) * ld) * ES, inq(m)));
        }
      }
      return v;
    };
    // the first PF untransposed leaves are loaded up front, all in flight together,
    // instead of one round trip per LEAF instruction
    typedef T pfvec __attribute__((ext_vector_type(E * PF)));
    pfvec pf;
#pragma unroll
    for (int k = 0; k < PF; ++k)
      if (k < e.n_leaves && !((p1 >> k) & 1u)) {
        const Vals<T, E> v = load_direct(k);
#pragma unroll
        for (int m = 0; m < E; ++m) pf[E * k + m] = v.v[m];
      }
    // value of leaf k for this thread's E elements (lanes past the edge hold 0 or a
    // value that is never stored)
    auto fetch_leaf = [&](u32 k) __attribute__((always_inline)) {
      Vals<T, E> v;
      if (!FLAT && ((p1 >> k) & 1u)) {
        // transposed leaf: staged in LDS (slot = staged leaves before it) or read directly
        const int slot = __builtin_popcount(p1 & ((1u << k) - 1u));
        if (slot < np1 && DMA) {
          const T* st = stage + slot * TS * TS;
#pragma unroll
          for (int m = 0; m < E; ++m) {
            const int il = iq(m) - i0;
            v.v[m] = st[il * TS + ((jq(m) - j0 + il) & (TS - 1))];
          }
        } else if (slot < np1) {
          const T* st = stage + slot * TS * (TS + 1);
#pragma unroll
          for (int m = 0; m < E; ++m) v.v[m] = st[(iq(m) - i0) * (TS + 1) + (jq(m) - j0)];
        } else {
          const rsrc_t r = make_rsrc(e.leaf[k], e.nrec[k]);
          const u32 ld = e.ld[k];
#pragma unroll
          for (int m = 0; m < E; ++m) v.v[m] = Buf<T>::ld1(r, masked(((u32)jq(m) + (u32)iq(m) * ld) * ES, inq(m)));
        }
      } else if ((int)k < PF) {
        // wave-uniform index into a register vector
#pragma unroll
        for (int m = 0; m < E; ++m) v.v[m] = pf[E * (int)k + m];
      } else {
        v = load_direct((int)k);
      }
      return v;
    };
    if (DMA && p1 && np1 > 0) {
      // the LDS DMA writes land before the staging area is read (the compiler does not
      // track them): vmcnt(0), expcnt and lgkmcnt unconstrained
      __builtin_amdgcn_s_waitcnt(0x0F70);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
    } else if (!FLAT && p1 && np1 > 0) {
      __syncthreads();  // the previous tile's reads of the staging area are done
      u32 rest = p1;
#pragma unroll
      for (int sl = 0; sl < kMaxStaged; ++sl) {
        if (sl < np1 && rest != 0u) {
          rest &= rest - 1u;
#pragma unroll
          for (int m = 0; m < E; ++m) {
            const int idx = tid + m * NT;
            stage[(sl * TS + idx / TS) * (TS + 1) + idx % TS] = sv[sl].v[m];
          }
        }
      }
      __syncthreads();
    }
    T acc[E];
    const u32* prog = code + e.code_off;
    for (int pc = 0; pc < e.code_len; ++pc) {
      const u32 ins = prog[pc];
      const u32 op = ins & 63u, b = (ins >> 6) & 7u, arg = ins >> 9;
      if (op >= OP_WITH_LEAF) {
        // binary op with a leaf or scalar operand taken directly
        T x[E];
        if (op >= OP_WITH_SCAL) {
          const T sv1 = scal[e.sc_off + (int)arg];
#pragma unroll
          for (int m = 0; m < E; ++m) x[m] = sv1;
        } else {
          const Vals<T, E> v = fetch_leaf(arg);
#pragma unroll
          for (int m = 0; m < E; ++m) x[m] = v.v[m];
        }
        apply_bin<T, E>(op & 7u, acc, x);
      } else if (op == OP_LEAF || op == OP_SCAL) {
        if (b > 0) {
#pragma unroll
          for (int gg = 0; gg < G; ++gg) {
            vt<T, 4> s4;
#pragma unroll
            for (int q = 0; q < 4; ++q) s4.v[q] = acc[4 * gg + q];
            stk[((b - 1) * G + gg) * NT + tid] = s4;
          }
        }
        if (op == OP_SCAL) {
          const T sv1 = scal[e.sc_off + (int)arg];
#pragma unroll
          for (int m = 0; m < E; ++m) acc[m] = sv1;
        } else {
          const Vals<T, E> v = fetch_leaf(arg);
#pragma unroll
          for (int m = 0; m < E; ++m) acc[m] = v.v[m];
        }
      } else if (op <= OP_RDIV) {
        // r[b] = op(r[b], r[b+1]): r[b] from the LDS stack, r[b+1] the top
        T top[E];
#pragma unroll
        for (int gg = 0; gg < G; ++gg) {
          const vt<T, 4> a4 = stk[(b * G + gg) * NT + tid];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            top[4 * gg + q] = acc[4 * gg + q];
            acc[4 * gg + q] = a4.v[q];
          }
        }
        apply_bin<T, E>(op, acc, top);
      } else {
        apply_un<T, E>(op, acc);
      }
    }
    const rsrc_t ro = make_rsrc(e.out, e.out_nrec);
    if (FLAT) {
#pragma unroll
      for (int gg = 0; gg < G; ++gg) {
        if (v4 && full) {
          T x4[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) x4[q] = acc[4 * gg + q];
          Buf<T>::st4(ro, fbq(gg) * ES, x4);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            Buf<T>::st1(ro, masked((fbq(gg) + (u32)q) * ES, inq(4 * gg + q)), acc[4 * gg + q]);
        }
      }
    } else {
      const u32 old = e.out_ld;
      if (v4) {
#pragma unroll
        for (int gg = 0; gg < G; ++gg) {
          T x4[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) x4[q] = acc[4 * gg + q];
          Buf<T>::st4(ro, masked(((u32)iq(4 * gg) + (u32)jq(4 * gg) * old) * ES, inq(4 * gg)), x4);
        }
      } else {
#pragma unroll
        for (int m = 0; m < E; ++m)
          Buf<T>::st1(ro, masked(((u32)iq(m) + (u32)jq(m) * old) * ES, inq(m)), acc[m]);
      }
    }
  }
}

template <typename T, int TS, int G>
hipError_t launch_interp(bool flat_only, unsigned grid, size_t shmem, hipStream_t s, const BatchExpr* e, const u32* tl,
                         int t_begin, int t_end, const u32* cd, const T* sc, int nstk, int np1) {
  constexpr int NT = TS * TS / (4 * G);
  if (flat_only)
    hipLaunchKernelGGL((interp<T, TS, G, true>), dim3(grid), dim3(NT), shmem, s, e, tl, t_begin, t_end, cd, sc, nstk, 0);
  else
    hipLaunchKernelGGL((interp<T, TS, G, false>), dim3(grid), dim3(NT), shmem, s, e, tl, t_begin, t_end, cd, sc, nstk,
                       np1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_shape(int ts, int g, bool flat_only, unsigned grid, size_t shmem, hipStream_t s, const BatchExpr* e,
                        const u32* tl, int t_begin, int t_end, const u32* cd, const T* sc, int nstk, int np1) {
  if (ts == 16 && g == 1) return launch_interp<T, 16, 1>(flat_only, grid, shmem, s, e, tl, t_begin, t_end, cd, sc, nstk, np1);
  if (ts == 32 && g == 1) return launch_interp<T, 32, 1>(flat_only, grid, shmem, s, e, tl, t_begin, t_end, cd, sc, nstk, np1);
  if (ts == 32 && g == 2) return launch_interp<T, 32, 2>(flat_only, grid, shmem, s, e, tl, t_begin, t_end, cd, sc, nstk, np1);
  if (ts == 32 && g == 4) return launch_interp<T, 32, 4>(flat_only, grid, shmem, s, e, tl, t_begin, t_end, cd, sc, nstk, np1);
  return hipErrorInvalidValue;
}

}  // namespace batch
}  // namespace coot

// host-side launcher (called from batch.cpp): tile edge ts, g groups of 4 elements per
// thread (ts * ts / (4 g) threads per workgroup)
extern "C" hipError_t coot_batch_launch_kernel(int dtype, int ts, int g, unsigned grid, const void* ex,
                                              const void* tiles, int t_begin, int t_end, const void* code,
                                              const void* scal, int nstk, int np1, int flat_only, hipStream_t s) {
  using namespace coot::batch;
  const size_t es = dtype == COOT_BATCH_F32 ? 4 : 8;
  if ((ts != 16 && ts != 32) || (g != 1 && g != 2 && g != 4) || ts * ts / (4 * g) < 64) return hipErrorInvalidValue;
  const int nt = ts * ts / (4 * g);
  // staging slots: [TS][TS] for the one-wave tiles (LDS DMA), [TS][TS + 1] otherwise
  const size_t slot = (size_t)ts * (nt == 64 ? ts : ts + 1) * es;
  const size_t shmem = (size_t)nstk * ts * ts * es + (size_t)np1 * slot;
  if (nstk < 1 || np1 < 0 || np1 > (nt == 64 ? 4 : 2) || shmem > 65536 - 2048) return hipErrorInvalidValue;  // 2 KB: the exp table
  if (dtype == COOT_BATCH_F32)
    return launch_shape<float>(ts, g, flat_only != 0, grid, shmem, s, (const BatchExpr*)ex, (const u32*)tiles, t_begin,
                               t_end, (const u32*)code, (const float*)scal, nstk, np1);
  return launch_shape<double>(ts, g, flat_only != 0, grid, shmem, s, (const BatchExpr*)ex, (const u32*)tiles, t_begin,
                              t_end, (const u32*)code, (const double*)scal, nstk, np1);
}
