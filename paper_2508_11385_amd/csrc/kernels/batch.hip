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

// acc[q] = op(acc[q], x[q]) (R-variants: op(x[q], acc[q])); one dispatch for the 4 values
template <typename T>
__device__ __forceinline__ void apply_bin(u32 op, T (&acc)[4], const vt<T, 4>& x) {
  switch (op) {
    case OP_ADD:
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = op_add(acc[q], x.v[q]);
      break;
    case OP_SUB:
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = op_sub(acc[q], x.v[q]);
      break;
    case OP_MUL:
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = op_mul(acc[q], x.v[q]);
      break;
    case OP_DIV:
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = op_div(acc[q], x.v[q]);
      break;
    case OP_RSUB:
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = op_sub(x.v[q], acc[q]);
      break;
    default:  // OP_RDIV
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = op_div(x.v[q], acc[q]);
      break;
  }
}

template <typename T>
__device__ __forceinline__ void apply_un(u32 op, T (&acc)[4]) {
  switch (op) {
    case OP_NEG:
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = op_neg(acc[q]);
      break;
    case OP_ABS:
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = op_abs(acc[q]);
      break;
    case OP_EXP:
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = op_exp(acc[q]);
      break;
    case OP_LOG:
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = op_log(acc[q]);
      break;
    case OP_SQRT:
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = op_sqrt(acc[q]);
      break;
    default:  // OP_SQUARE
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = op_square(acc[q]);
      break;
  }
}

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
// staged transposed leaves in registers, so they prefetch fewer)
template <typename T, bool FLAT> struct Prefetch {
  static constexpr int N = FLAT ? (sizeof(T) == 4 ? 6 : 4) : (sizeof(T) == 4 ? 3 : 2);
};

// FLAT: the tile range holds flat chunks only (no staging, no 2-D index maps: fewer
// registers, more waves per SIMD); otherwise 2-D tiles only.
// (fp32 flat chunks fit 64 registers: 8 waves per SIMD)
template <typename T, int TS, bool FLAT>
__global__ __launch_bounds__(TS * TS / 4) __attribute__((amdgpu_waves_per_eu(FLAT && sizeof(T) == 4 ? 8 : 1))) void interp(const BatchExpr* __restrict__ ex, const u32* __restrict__ tiles,
                                                      int t_begin, int t_end, const u32* __restrict__ code,
                                                      const T* __restrict__ scal, int nstk, int np1) {
  constexpr int NT = TS * TS / 4;  // threads: 4 elements each
  constexpr int PF = Prefetch<T, FLAT>::N;
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
  vt<T, 4>* stk = reinterpret_cast<vt<T, 4>*>(smem);                              // [nstk][NT]
  T* stage = reinterpret_cast<T*>(smem + (size_t)nstk * NT * sizeof(vt<T, 4>));  // [np1][TS][TS + 1]
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
    // this thread's 4 elements: rows iq[q], columns jq[q] (2-D) or flat indices fbase + q
    int iq[4], jq[4];
    bool in[4];
    vt<T, 4> sv[kMaxStaged];
    u32 fbase = 0;
    bool full = false;  // flat: every element of the chunk exists (uniform)
    int i0 = 0, j0 = 0;
    if constexpr (FLAT) {
      const u32 n = (u32)R * (u32)C, tb = tin * (u32)(4 * NT);
      fbase = tb + 4u * (u32)tid;
      full = tb + (u32)(4 * NT) <= n;
#pragma unroll
      for (int q = 0; q < 4; ++q) in[q] = fbase + (u32)q < n;
    } else {
      i0 = (int)(tin & e.tile_mask) * TS;
      j0 = (int)(tin >> e.tile_shift) * TS;
      if (v4) {
        const int lc = tid % (TS / 4), lr = tid / (TS / 4);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          iq[q] = i0 + 4 * lc + q;
          jq[q] = j0 + lr;
        }
      } else {
        const int lc = tid % TS, lr = tid / TS;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          iq[q] = i0 + lc;
          jq[q] = j0 + lr + (TS / 4) * q;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) in[q] = iq[q] < R && jq[q] < C;
      // staged transposed leaves: this thread's 4 values of each (element idx = tid + q * NT
      // of the tile, read along the leaf's contiguous dimension), loads issued together
      if (DMA && p1 && np1 > 0) {
        // (the previous tile's reads of the staging area are complete: their values were used)
        constexpr int W = sizeof(T) / 4;  // dwords per element
        u32 rest = p1;
#pragma unroll
        for (int sl = 0; sl < kMaxStaged; ++sl) {
          if (sl < np1 && rest != 0u) {
            const int k = __builtin_ctz(rest);
            rest &= rest - 1u;
            const rsrc_t r = make_rsrc(e.leaf[k], e.nrec[k]);
            const u32 ld = e.ld[k];
#pragma unroll
            for (int q = 0; q < 4 * W; ++q) {
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
            for (int q = 0; q < 4; ++q) {
              const int idx = tid + q * NT, i = i0 + idx / TS, j = j0 + idx % TS;
              sv[sl].v[q] = Buf<T>::ld1(r, masked(((u32)j + (u32)i * ld) * ES, i < R && j < C));
            }
          }
        }
      }
    }
    // an untransposed leaf's 4 values for this thread (flat chunk or 2-D tile layout)
    auto load_direct = [&](int k) __attribute__((always_inline)) {
      vt<T, 4> v;
      const rsrc_t r = make_rsrc(e.leaf[k], e.nrec[k]);
      if (FLAT) {
        if (v4 && full) {
          v = Buf<T>::ld4(r, fbase * ES);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) v.v[q] = Buf<T>::ld1(r, masked((fbase + (u32)q) * ES, in[q]));
        }
      } else {
        const u32 ld = e.ld[k];
        if (v4) {
          v = Buf<T>::ld4(r, masked(((u32)iq[0] + (u32)jq[0] * ld) * ES, in[0]));
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) v.v[q] = Buf<T>::ld1(r, masked(((u32)iq[q] + (u32)jq[q] * ld) * ES, in[q]));
        }
      }
      return v;
    };
    // the first PF untransposed leaves are loaded up front, all in flight together,
    // instead of one round trip per LEAF instruction
    typedef T pfvec __attribute__((ext_vector_type(4 * PF)));
    pfvec pf;
#pragma unroll
    for (int k = 0; k < PF; ++k)
      if (k < e.n_leaves && !((p1 >> k) & 1u)) {
        const vt<T, 4> v = load_direct(k);
#pragma unroll
        for (int q = 0; q < 4; ++q) pf[4 * k + q] = v.v[q];
      }
    // value of leaf k for this thread's 4 elements (lanes past the edge hold 0 or a
    // value that is never stored)
    auto fetch_leaf = [&](u32 k) __attribute__((always_inline)) {
      vt<T, 4> v;
      if (!FLAT && ((p1 >> k) & 1u)) {
        // transposed leaf: staged in LDS (slot = staged leaves before it) or read directly
        const int slot = __builtin_popcount(p1 & ((1u << k) - 1u));
        if (slot < np1 && DMA) {
          const T* st = stage + slot * TS * TS;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int il = iq[q] - i0;
            v.v[q] = st[il * TS + ((jq[q] - j0 + il) & (TS - 1))];
          }
        } else if (slot < np1) {
          const T* st = stage + slot * TS * (TS + 1);
#pragma unroll
          for (int q = 0; q < 4; ++q) v.v[q] = st[(iq[q] - i0) * (TS + 1) + (jq[q] - j0)];
        } else {
          const rsrc_t r = make_rsrc(e.leaf[k], e.nrec[k]);
          const u32 ld = e.ld[k];
#pragma unroll
          for (int q = 0; q < 4; ++q) v.v[q] = Buf<T>::ld1(r, masked(((u32)jq[q] + (u32)iq[q] * ld) * ES, in[q]));
        }
      } else if ((int)k < PF) {
        // wave-uniform index into a register vector
#pragma unroll
        for (int q = 0; q < 4; ++q) v.v[q] = pf[4 * (int)k + q];
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
          for (int q = 0; q < 4; ++q) {
            const int idx = tid + q * NT;
            stage[(sl * TS + idx / TS) * (TS + 1) + idx % TS] = sv[sl].v[q];
          }
        }
      }
      __syncthreads();
    }
    T acc[4];
    const u32* prog = code + e.code_off;
    for (int pc = 0; pc < e.code_len; ++pc) {
      const u32 ins = prog[pc];
      const u32 op = ins & 63u, b = (ins >> 6) & 7u, arg = ins >> 9;
      if (op >= OP_WITH_LEAF) {
        // binary op with a leaf or scalar operand taken directly
        vt<T, 4> x;
        if (op >= OP_WITH_SCAL) {
          const T s = scal[e.sc_off + (int)arg];
#pragma unroll
          for (int q = 0; q < 4; ++q) x.v[q] = s;
        } else {
          x = fetch_leaf(arg);
        }
        apply_bin<T>(op & 7u, acc, x);
      } else if (op == OP_LEAF || op == OP_SCAL) {
        if (b > 0) {
          vt<T, 4> s;
#pragma unroll
          for (int q = 0; q < 4; ++q) s.v[q] = acc[q];
          stk[(b - 1) * NT + tid] = s;
        }
        if (op == OP_SCAL) {
          const T s = scal[e.sc_off + (int)arg];
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] = s;
        } else {
          const vt<T, 4> v = fetch_leaf(arg);
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] = v.v[q];
        }
      } else if (op <= OP_RDIV) {
        // r[b] = op(r[b], r[b+1]): r[b] from the LDS stack, r[b+1] the top
        const vt<T, 4> a = stk[b * NT + tid];
        vt<T, 4> top;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          top.v[q] = acc[q];
          acc[q] = a.v[q];
        }
        apply_bin<T>(op, acc, top);
      } else {
        apply_un<T>(op, acc);
      }
    }
    const rsrc_t ro = make_rsrc(e.out, e.out_nrec);
    if (FLAT) {
      if (v4 && full) {
        Buf<T>::st4(ro, fbase * ES, acc);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) Buf<T>::st1(ro, masked((fbase + (u32)q) * ES, in[q]), acc[q]);
      }
    } else {
      const u32 old = e.out_ld;
      if (v4) {
        Buf<T>::st4(ro, masked(((u32)iq[0] + (u32)jq[0] * old) * ES, in[0]), acc);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) Buf<T>::st1(ro, masked(((u32)iq[q] + (u32)jq[q] * old) * ES, in[q]), acc[q]);
      }
    }
  }
}

}  // namespace batch
}  // namespace coot

// host-side launcher (called from batch.cpp)
extern "C" hipError_t coot_batch_launch_kernel(int dtype, int ts, unsigned grid, const void* ex, const void* tiles,
                                              int t_begin, int t_end, const void* code, const void* scal, int nstk,
                                              int np1, int flat_only, hipStream_t s) {
  using namespace coot::batch;
  const BatchExpr* e = (const BatchExpr*)ex;
  const u32* tl = (const u32*)tiles;
  const u32* cd = (const u32*)code;
  const size_t es = dtype == COOT_BATCH_F32 ? 4 : 8;
  // staging slots: [TS][TS] for the one-wave tiles (LDS DMA), [TS][TS + 1] otherwise
  const size_t slot = (size_t)ts * (ts == 16 ? ts : ts + 1) * es;
  const size_t shmem = (size_t)nstk * (ts * ts / 4) * 4 * es + (size_t)np1 * slot;
  if (nstk < 1 || np1 < 0 || shmem > 65536 - 2048) return hipErrorInvalidValue;  // 2 KB: the exp table
  if (dtype == COOT_BATCH_F32) {
    const float* sc = (const float*)scal;
    switch (ts) {
      case 16:
        if (flat_only)
          hipLaunchKernelGGL((interp<float, 16, true>), dim3(grid), dim3(64), shmem, s, e, tl, t_begin, t_end, cd, sc, nstk, 0);
        else
          hipLaunchKernelGGL((interp<float, 16, false>), dim3(grid), dim3(64), shmem, s, e, tl, t_begin, t_end, cd, sc, nstk, np1);
        break;
      case 32:
        if (flat_only)
          hipLaunchKernelGGL((interp<float, 32, true>), dim3(grid), dim3(256), shmem, s, e, tl, t_begin, t_end, cd, sc, nstk, 0);
        else
          hipLaunchKernelGGL((interp<float, 32, false>), dim3(grid), dim3(256), shmem, s, e, tl, t_begin, t_end, cd, sc, nstk, np1);
        break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const double* sc = (const double*)scal;
    switch (ts) {
      case 16:
        if (flat_only)
          hipLaunchKernelGGL((interp<double, 16, true>), dim3(grid), dim3(64), shmem, s, e, tl, t_begin, t_end, cd, sc, nstk, 0);
        else
          hipLaunchKernelGGL((interp<double, 16, false>), dim3(grid), dim3(64), shmem, s, e, tl, t_begin, t_end, cd, sc, nstk, np1);
        break;
      case 32:
        if (flat_only)
          hipLaunchKernelGGL((interp<double, 32, true>), dim3(grid), dim3(256), shmem, s, e, tl, t_begin, t_end, cd, sc, nstk, 0);
        else
          hipLaunchKernelGGL((interp<double, 32, false>), dim3(grid), dim3(256), shmem, s, e, tl, t_begin, t_end, cd, sc, nstk, np1);
        break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}
