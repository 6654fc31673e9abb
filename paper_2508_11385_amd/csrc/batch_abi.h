// Layout shared by the batch interpreter kernel (kernels/batch.hip) and its host
// side (batch.cpp).
#pragma once
#include <stdint.h>

#define COOT_BATCH_MAXL 12   // distinct (operand, transpose parity) leaves per expression
#define COOT_BATCH_F32 0
#define COOT_BATCH_F64 1

namespace coot {
namespace batch {

enum : uint32_t {
  OP_ADD = 0, OP_SUB = 1, OP_MUL = 2, OP_DIV = 3, OP_RSUB = 4, OP_RDIV = 5,  // binary (R: operands swapped)
  OP_NEG = 6, OP_ABS = 7, OP_EXP = 8, OP_LOG = 9, OP_SQRT = 10, OP_SQUARE = 11,  // unary
  OP_LEAF = 12, OP_SCAL = 13,
  // binary op whose second operand is a leaf / a scalar, taken directly: r[b] = op(r[b], x)
  OP_WITH_LEAF = 16,  // + binary opcode (0..5)
  OP_WITH_SCAL = 24   // + binary opcode (0..5)
};

inline constexpr uint32_t encode(uint32_t op, uint32_t reg, uint32_t arg) { return op | (reg << 6) | (arg << 9); }

// One expression of a batch (device memory, 256-byte records).  Every leaf and the
// output are addressed as raw buffers: offsets are 32-bit byte offsets below the
// operand's extent `nrec`, which the host keeps under 2^31 bytes.
struct BatchExpr {
  const void* leaf[COOT_BATCH_MAXL];  // leaf k: base pointer of its operand
  uint32_t ld[COOT_BATCH_MAXL];       // leading dimension of leaf k's operand (elements)
  uint32_t nrec[COOT_BATCH_MAXL];     // bytes of leaf k's operand from leaf[k] on (its buffer range)
  void* out;
  uint32_t out_ld, out_nrec;          // output leading dimension (elements) and extent (bytes)
  int32_t n_rows, n_cols;             // output dimensions
  int32_t tile_shift;                 // 2-D tile number = ti | tj << tile_shift
  uint32_t tile_mask;                 // (1 << tile_shift) - 1
  int32_t code_off, code_len;         // bytecode range
  int32_t sc_off;                     // first scalar
  uint32_t p1_mask;                   // bit k: leaf k is read transposed
  int32_t vec4;                       // 1: 128-bit accesses are valid
  int32_t flat;                       // 1: untransposed contiguous leaves and output: flat chunks
  int32_t n_leaves;                   // leaves used (leaf[0 .. n_leaves))
  int32_t pad_;
};
static_assert(sizeof(BatchExpr) == 256, "BatchExpr is a 256-byte record");

}  // namespace batch
}  // namespace coot
