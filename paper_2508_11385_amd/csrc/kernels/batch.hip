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

constexpr int kMaxStaged = 4;  // transposed leaves staged in LDS per tile (at most)
constexpr int kXcds = 8;       // accelerator complex dies of an MI355X, each with its own L2

// untransposed leaves loaded before the bytecode runs (2-D tiles also hold their
// staged transposed leaves in registers, so they prefetch fewer)
template <typename T, bool FLAT> struct Prefetch {
  static constexpr int N = FLAT ? (sizeof(T) == 4 ? 6 : 4) : (sizeof(T) == 4 ? 3 : 2);
};

// FLAT: the tile range holds flat chunks only (no staging, no 2-D index maps: fewer
// registers, more waves per SIMD); otherwise 2-D tiles only.
template <typename T, int TS, bool FLAT>
__global__ __launch_bounds__(TS * TS / 4) void interp(const BatchExpr* __restrict__ ex, const u32* __restrict__ tiles,
                                                      int t_begin, int t_end, const u32* __restrict__ code,
                                                      const T* __restrict__ scal, int nstk, int np1) {
  constexpr int NT = TS * TS / 4;  // threads: 4 elements each
  constexpr int PF = Prefetch<T, FLAT>::N;
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
    constexpr bool flat = FLAT;
    const bool v4 = e.vec4 != 0;
    const u32 p1 = e.p1_mask;
    int iq[4], jq[4];
    bool in[4];
    vt<T, 4> sv[kMaxStaged];
    i64 fbase = 0;
    int i0 = 0, j0 = 0;
    if constexpr (FLAT) {
      const i64 n = (i64)R * C;
      fbase = (i64)tin * (4 * NT) + 4 * tid;
#pragma unroll
      for (int q = 0; q < 4; ++q) in[q] = fbase + q < n;
    } else {
      const int ti = (int)(tin % (u32)e.tiles_r), tj = (int)(tin / (u32)e.tiles_r);
      i0 = ti * TS;
      j0 = tj * TS;
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
      if (p1 && np1 > 0) {
        u32 rest = p1;
#pragma unroll
        for (int sl = 0; sl < kMaxStaged; ++sl) {
          if (sl < np1 && rest != 0u) {
            const int k = __builtin_ctz(rest);
            rest &= rest - 1u;
            const T* src = (const T*)e.leaf[k];
            const i64 ld = e.ld[k];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int idx = tid + q * NT, sc = idx % TS, il = idx / TS;
              const int i = i0 + il, j = j0 + sc;
              sv[sl].v[q] = (i < R && j < C) ? src[(i64)j + (i64)i * ld] : (T)0;
            }
          }
        }
      }
    }
    const bool all_in = in[0] && in[1] && in[2] && in[3];
    // an untransposed leaf's 4 values for this thread (flat chunk or 2-D tile layout)
    auto load_direct = [&](int k) __attribute__((always_inline)) {
      vt<T, 4> g;
      const T* src = (const T*)e.leaf[k];
      if (flat) {
        if (v4 && all_in) {
          g = ldv<T, 4>(src + fbase);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) g.v[q] = in[q] ? src[fbase + q] : (T)0;
        }
      } else {
        const i64 ld = e.ld[k];
        if (v4) {
          if (in[0]) {
            g = ldv<T, 4>(src + (i64)iq[0] + (i64)jq[0] * ld);
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) g.v[q] = (T)0;
          }
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) g.v[q] = in[q] ? src[(i64)iq[q] + (i64)jq[q] * ld] : (T)0;
        }
      }
      return g;
    };
    // the first PF untransposed leaves are loaded up front, all in flight together,
    // instead of one round trip per LEAF instruction
    typedef T pfvec __attribute__((ext_vector_type(4 * PF)));
    pfvec pf;
#pragma unroll
    for (int k = 0; k < PF; ++k)
      if (k < e.n_leaves && !((p1 >> k) & 1u)) {
        const vt<T, 4> g = load_direct(k);
#pragma unroll
        for (int q = 0; q < 4; ++q) pf[4 * k + q] = g.v[q];
      }
    // value of leaf k for this thread's 4 elements
    auto fetch_leaf = [&](u32 k) __attribute__((always_inline)) {
      vt<T, 4> g;
      if (!FLAT && ((p1 >> k) & 1u)) {
        // transposed leaf: staged in LDS (slot = staged leaves before it) or read directly
        const int slot = __builtin_popcount(p1 & ((1u << k) - 1u));
        if (slot < np1) {
          const T* st = stage + slot * TS * (TS + 1);
#pragma unroll
          for (int q = 0; q < 4; ++q) g.v[q] = in[q] ? st[(iq[q] - i0) * (TS + 1) + (jq[q] - j0)] : (T)0;
        } else {
          const T* src = (const T*)e.leaf[k];
          const i64 ld = e.ld[k];
#pragma unroll
          for (int q = 0; q < 4; ++q) g.v[q] = in[q] ? src[(i64)jq[q] + (i64)iq[q] * ld] : (T)0;
        }
      } else if ((int)k < PF) {
        // wave-uniform index into a register vector
#pragma unroll
        for (int q = 0; q < 4; ++q) g.v[q] = pf[4 * (int)k + q];
      } else {
        g = load_direct((int)k);
      }
      return g;
    };
    if (!FLAT && p1 && np1 > 0) {
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
          const T sv = scal[e.sc_off + (int)arg];
#pragma unroll
          for (int q = 0; q < 4; ++q) x.v[q] = sv;
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
          const T sv = scal[e.sc_off + (int)arg];
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] = sv;
        } else {
          const vt<T, 4> g = fetch_leaf(arg);
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] = g.v[q];
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
    T* out = (T*)e.out;
    if (flat) {
      if (v4 && all_in) {
        vt<T, 4> g;
#pragma unroll
        for (int q = 0; q < 4; ++q) g.v[q] = acc[q];
        stv<T, 4>(out + fbase, g);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (in[q]) out[fbase + q] = acc[q];
      }
    } else {
      const i64 old = e.out_ld;
      if (v4) {
        if (in[0]) {
          vt<T, 4> g;
#pragma unroll
          for (int q = 0; q < 4; ++q) g.v[q] = acc[q];
          stv<T, 4>(out + (i64)iq[0] + (i64)jq[0] * old, g);
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (in[q]) out[(i64)iq[q] + (i64)jq[q] * old] = acc[q];
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
  const size_t shmem = (size_t)nstk * (ts * ts / 4) * 4 * es + (size_t)np1 * ts * (ts + 1) * es;
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
