// Persistent interpreter for batches of small independent expressions.
//
// The paper notes that GPUs are ill-suited to small matrices unless enough of
// them keep the device busy (Section 4, second difference).  Here thousands of
// small expressions run in ONE launch: a fixed grid walks a work-list of
// TS x TS output tiles (round-robin, no atomics, so a replayed graph needs no
// reset), and every tile evaluates its expression's bytecode.
//
// Bytecode (u32 per instruction): bits 0-5 opcode, 6-8 register b, 9-31 argument.
// The host orders the tree so that registers form a stack (Sethi-Ullman):
//   LEAF  r[b] = leaf[arg] at the element's coordinates
//   SCAL  r[b] = scalar[arg]
//   binary op       r[b] = op(r[b], r[b+1]);  its R-variant r[b] = op(r[b+1], r[b])
//   unary op        r[b] = op(r[b])
// Every thread owns 4 elements: a 4-row column segment read with one 128-bit
// access when the expression's layout allows it, else 4 elements in 4 columns
// read one by one (consecutive lanes still touch consecutive rows).  Leaves read
// transposed are staged tile-wise through LDS along their own contiguous
// dimension, as in the fused tiled kernels; beyond NP1 of them they are read
// directly from global memory.
#include <hip/hip_runtime.h>

#include "device/coot_dev.h"
#include "batch_abi.h"

namespace coot {
namespace batch {

template <typename T, int TS>
struct Cfg {
  static constexpr int NT = TS * TS / 4;  // threads: 4 elements each
  static constexpr int BYTES = TS * (TS + 1) * (int)sizeof(T);
  static constexpr int NP1 = (49152 / BYTES) < 4 ? (49152 / BYTES) : 4;  // LDS-staged transposed leaves
};

// Register file: eight named 4-element registers.  They are never addressed
// through an index: every (register, operation) pair is its own case below, so
// the registers stay in VGPRs.
template <typename T>
struct Regs {
  T r0[4], r1[4], r2[4], r3[4], r4[4], r5[4], r6[4], r7[4];
};

#define COOT_RB(i) R.r##i
#define COOT_SET(i) \
  case i:           \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) COOT_RB(i)[q] = v[q]; \
    break;

template <typename T>
__device__ __forceinline__ void reg_set(Regs<T>& R, u32 b, const T (&v)[4]) {
  switch (b) {
    COOT_SET(0) COOT_SET(1) COOT_SET(2) COOT_SET(3) COOT_SET(4) COOT_SET(5) COOT_SET(6) COOT_SET(7)
  }
}

// key = op * 8 + register
#define COOT_BIN(OPC, i, j, FN) \
  case OPC * 8 + i:             \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) COOT_RB(i)[q] = FN(COOT_RB(i)[q], COOT_RB(j)[q]); \
    break;
#define COOT_RBIN(OPC, i, j, FN) \
  case OPC * 8 + i:              \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) COOT_RB(i)[q] = FN(COOT_RB(j)[q], COOT_RB(i)[q]); \
    break;
#define COOT_UN(OPC, i, FN) \
  case OPC * 8 + i:         \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) COOT_RB(i)[q] = FN(COOT_RB(i)[q]); \
    break;
#define COOT_BIN_ALL(OPC, FN) \
  COOT_BIN(OPC, 0, 1, FN) COOT_BIN(OPC, 1, 2, FN) COOT_BIN(OPC, 2, 3, FN) COOT_BIN(OPC, 3, 4, FN) \
  COOT_BIN(OPC, 4, 5, FN) COOT_BIN(OPC, 5, 6, FN) COOT_BIN(OPC, 6, 7, FN)
#define COOT_RBIN_ALL(OPC, FN) \
  COOT_RBIN(OPC, 0, 1, FN) COOT_RBIN(OPC, 1, 2, FN) COOT_RBIN(OPC, 2, 3, FN) COOT_RBIN(OPC, 3, 4, FN) \
  COOT_RBIN(OPC, 4, 5, FN) COOT_RBIN(OPC, 5, 6, FN) COOT_RBIN(OPC, 6, 7, FN)
#define COOT_UN_ALL(OPC, FN)                                                                   \
  COOT_UN(OPC, 0, FN) COOT_UN(OPC, 1, FN) COOT_UN(OPC, 2, FN) COOT_UN(OPC, 3, FN) COOT_UN(OPC, 4, FN) \
  COOT_UN(OPC, 5, FN) COOT_UN(OPC, 6, FN) COOT_UN(OPC, 7, FN)

template <typename T>
__device__ __forceinline__ void reg_op(Regs<T>& R, u32 key) {
  switch (key) {
    COOT_BIN_ALL(OP_ADD, op_add)
    COOT_BIN_ALL(OP_SUB, op_sub)
    COOT_BIN_ALL(OP_MUL, op_mul)
    COOT_BIN_ALL(OP_DIV, op_div)
    COOT_RBIN_ALL(OP_RSUB, op_sub)
    COOT_RBIN_ALL(OP_RDIV, op_div)
    COOT_UN_ALL(OP_NEG, op_neg)
    COOT_UN_ALL(OP_ABS, op_abs)
    COOT_UN_ALL(OP_EXP, op_exp)
    COOT_UN_ALL(OP_LOG, op_log)
    COOT_UN_ALL(OP_SQRT, op_sqrt)
    COOT_UN_ALL(OP_SQUARE, op_square)
    default: break;
  }
}

template <typename T, int TS>
__global__ __launch_bounds__(TS * TS / 4) void interp(const BatchExpr* __restrict__ ex, const u32* __restrict__ tiles,
                                                         int t_begin, int t_end, const u32* __restrict__ code,
                                                         const T* __restrict__ scal) {
  typedef Cfg<T, TS> K;
  constexpr int NPS = K::NP1 > 0 ? K::NP1 : 1;
  __shared__ T lds[NPS][TS][TS + 1];
  const int tid = threadIdx.x;
  for (int t = t_begin + (int)blockIdx.x; t < t_end; t += (int)gridDim.x) {
    const u32 eid = tiles[2 * t], tin = tiles[2 * t + 1];
    const BatchExpr& e = ex[eid];
    const int R = e.n_rows, C = e.n_cols;
    const int ti = (int)(tin % (u32)e.tiles_r), tj = (int)(tin / (u32)e.tiles_r);
    const int i0 = ti * TS, j0 = tj * TS;
    const u32 p1 = e.p1_mask;
    if (p1) {
      int slot = 0;
      for (int k = 0; k < COOT_BATCH_MAXL && slot < K::NP1; ++k) {
        if (!((p1 >> k) & 1u)) continue;
        const T* src = (const T*)e.leaf[k];
        const i64 ld = e.ld[k];
        for (int idx = tid; idx < TS * TS; idx += K::NT) {
          const int sc = idx % TS, il = idx / TS;
          const int i = i0 + il, j = j0 + sc;
          lds[slot][il][sc] = (i < R && j < C) ? src[(i64)j + (i64)i * ld] : (T)0;
        }
        ++slot;
      }
      __syncthreads();
    }
    // the 4 elements of this thread
    const bool v4 = e.vec4 != 0;
    int iq[4], jq[4];
    bool in[4];
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
    Regs<T> Rg;
    const u32* prog = code + e.code_off;
    for (int pc = 0; pc < e.code_len; ++pc) {
      const u32 ins = prog[pc];
      const u32 op = ins & 63u, b = (ins >> 6) & 7u, arg = ins >> 9;
      if (op == OP_LEAF) {
        T v[4];
        if ((p1 >> arg) & 1u) {
          // staged transposed leaf (slot = number of staged leaves before it) or direct read
          const int slot = __builtin_popcount(p1 & ((1u << arg) - 1u));
          if (slot < K::NP1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = in[q] ? lds[slot < NPS ? slot : 0][iq[q] - i0][jq[q] - j0] : (T)0;
          } else {
            const T* src = (const T*)e.leaf[arg];
            const i64 ld = e.ld[arg];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = in[q] ? src[(i64)jq[q] + (i64)iq[q] * ld] : (T)0;
          }
        } else {
          const T* src = (const T*)e.leaf[arg];
          const i64 ld = e.ld[arg];
          if (v4) {
            if (in[0]) {
              vt<T, 4> g = ldv<T, 4>(src + (i64)iq[0] + (i64)jq[0] * ld);
#pragma unroll
              for (int q = 0; q < 4; ++q) v[q] = g.v[q];
            } else {
#pragma unroll
              for (int q = 0; q < 4; ++q) v[q] = (T)0;
            }
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = in[q] ? src[(i64)iq[q] + (i64)jq[q] * ld] : (T)0;
          }
        }
        reg_set<T>(Rg, b, v);
      } else if (op == OP_SCAL) {
        const T s = scal[e.sc_off + (int)arg];
        T v[4] = {s, s, s, s};
        reg_set<T>(Rg, b, v);
      } else {
        reg_op<T>(Rg, op * 8u + b);
      }
    }
    T* out = (T*)e.out;
    const i64 old = e.out_ld;
    if (v4) {
      if (in[0]) {
        vt<T, 4> g;
#pragma unroll
        for (int q = 0; q < 4; ++q) g.v[q] = Rg.r0[q];
        stv<T, 4>(out + (i64)iq[0] + (i64)jq[0] * old, g);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (in[q]) out[(i64)iq[q] + (i64)jq[q] * old] = Rg.r0[q];
    }
    if (p1) __syncthreads();  // the next tile restages LDS
  }
}

}  // namespace batch
}  // namespace coot

// host-side launcher (called from batch.cpp)
extern "C" hipError_t coot_batch_launch_kernel(int dtype, int ts, unsigned grid, const void* ex, const void* tiles,
                                              int t_begin, int t_end, const void* code, const void* scal,
                                              hipStream_t s) {
  using namespace coot::batch;
  const BatchExpr* e = (const BatchExpr*)ex;
  const u32* tl = (const u32*)tiles;
  const u32* cd = (const u32*)code;
  if (dtype == COOT_BATCH_F32) {
    const float* sc = (const float*)scal;
    switch (ts) {
      case 16: hipLaunchKernelGGL((interp<float, 16>), dim3(grid), dim3(64), 0, s, e, tl, t_begin, t_end, cd, sc); break;
      case 32: hipLaunchKernelGGL((interp<float, 32>), dim3(grid), dim3(256), 0, s, e, tl, t_begin, t_end, cd, sc); break;
      case 64: hipLaunchKernelGGL((interp<float, 64>), dim3(grid), dim3(1024), 0, s, e, tl, t_begin, t_end, cd, sc); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const double* sc = (const double*)scal;
    switch (ts) {
      case 16: hipLaunchKernelGGL((interp<double, 16>), dim3(grid), dim3(64), 0, s, e, tl, t_begin, t_end, cd, sc); break;
      case 32: hipLaunchKernelGGL((interp<double, 32>), dim3(grid), dim3(256), 0, s, e, tl, t_begin, t_end, cd, sc); break;
      case 64: hipLaunchKernelGGL((interp<double, 64>), dim3(grid), dim3(1024), 0, s, e, tl, t_begin, t_end, cd, sc); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}
