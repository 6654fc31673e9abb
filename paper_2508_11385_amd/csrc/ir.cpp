// Expression analysis: validation, transpose-parity push-down, canonical form,
// shape inference and operand checks.
//
// Section 3 of the paper: an expression is a tree of Op (may change dimensions:
// transpose), eOp (element-wise unary / scalar) and eGlue (element-wise binary,
// equal dimensions) nodes, analysed as a whole before any work is issued.  Here
// the tree arrives as a postfix list.  Every trans() is pushed down to the
// leaves: a leaf under an odd number of trans() is read with its index map
// swapped, so transposition never costs a pass of its own.
#include <atomic>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>

#include "core.h"

namespace coot {

size_t dtype_size(int dt) { return dt == COOT_F64 ? 8 : (dtype_is_half(dt) ? 2 : 4); }
const char* dtype_cname(int dt) {
  switch (dt) {
    case COOT_U32: return "u32";
    case COOT_S32: return "s32";
    case COOT_F32: return "float";
    case COOT_F16: return "coot::f16";
    case COOT_BF16: return "coot::bf16";
    default: return "double";
  }
}
bool dtype_is_int(int dt) { return dt == COOT_U32 || dt == COOT_S32; }
bool dtype_is_half(int dt) { return dt == COOT_F16 || dt == COOT_BF16; }

// binary32 value -> nearest-even value of a 16-bit type, returned as binary32
// (the same rounding the kernels apply to every operator's result)
static float round_half(float f, int dt) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t a = u & 0x7fffffffu;
  if (a > 0x7f800000u) return f;  // NaN
  if (dt == COOT_BF16) {
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
  } else {
    // binary16: 11 significant bits, exponents down to 2^-14, subnormal spacing 2^-24
    if (a == 0x7f800000u) return f;  // infinities
    const double ax = std::fabs((double)f);
    int e;
    (void)std::frexp(ax, &e);
    const int q = std::max(e - 11, -24);
    double v = std::ldexp(std::nearbyint(std::ldexp(ax, -q)), q);  // ties to even (default rounding mode)
    if (v >= 65520.0) v = INFINITY;  // 65504 plus half its spacing, and beyond
    const float r = (float)v;
    return std::signbit(f) ? -r : r;
  }
  float r;
  std::memcpy(&r, &u, 4);
  return r;
}

static bool is_binary(int c) { return c >= COOT_OP_ADD && c <= COOT_OP_DIV; }
static bool is_unary(int c) { return c >= COOT_OP_NEG && c <= COOT_OP_SQUARE; }
static bool int_illegal(int c) {
  return c == COOT_OP_DIV || c == COOT_OP_EXP || c == COOT_OP_LOG || c == COOT_OP_SQRT;
}

std::unique_ptr<Expr> analyse(const coot_op* ops, uint32_t n_ops, const coot_slot_type* slots, uint32_t n_slots,
                              uint32_t n_scalars, uint32_t flags) {
  if (!ops || n_ops == 0) fail(COOT_EINVAL, "empty expression");
  if (n_slots > (uint32_t)kMaxSlots) fail(COOT_EINVAL, "more than 16 operand slots");
  if (n_scalars > (uint32_t)kMaxScalars) fail(COOT_EINVAL, "more than 32 scalar slots");
  if (n_slots > 0 && !slots) fail(COOT_EINVAL, "slot types missing");
  if (flags & ~COOT_CF_UNFUSED) fail(COOT_EINVAL, "unknown compile flag");
  auto e = std::make_unique<Expr>();
  static std::atomic<uint64_t> next_uid{1};
  e->uid = next_uid++;
  e->ops.assign(ops, ops + n_ops);
  e->slots.assign(slots, slots + n_slots);
  e->n_scalars = n_scalars;
  e->flags = flags;
  e->dtype = n_slots ? slots[0].dtype : COOT_F32;
  for (uint32_t k = 0; k < n_slots; ++k) {
    if (slots[k].dtype < COOT_U32 || slots[k].dtype > COOT_BF16) fail(COOT_EINVAL, "bad dtype in slot");
    if (slots[k].kind < COOT_MAT || slots[k].kind > COOT_BCAST) fail(COOT_EINVAL, "bad kind in slot");
    if (slots[k].dtype != e->dtype) fail(COOT_ETYPE, "operand slots have different element types");
  }
  // arity and legality
  int depth = 0;
  bool any_load = false;
  for (uint32_t i = 0; i < n_ops; ++i) {
    const int c = ops[i].code;
    if (c == COOT_OP_LOAD) {
      if (ops[i].arg >= n_slots) fail(COOT_EINVAL, "LOAD of a slot out of range");
      any_load = true;
      ++depth;
    } else if (c == COOT_OP_SCALAR) {
      if (ops[i].arg >= n_scalars) fail(COOT_EINVAL, "SCALAR slot out of range");
      ++depth;
    } else if (is_binary(c)) {
      if (depth < 2) fail(COOT_EINVAL, "binary operator needs two operands");
      --depth;
    } else if (is_unary(c) || c == COOT_OP_TRANS) {
      if (depth < 1) fail(COOT_EINVAL, "unary operator needs an operand");
    } else {
      fail(COOT_EINVAL, "unknown opcode " + std::to_string(c));
    }
    if (dtype_is_int(e->dtype) && int_illegal(c)) fail(COOT_ETYPE, "operation not defined for an integer type");
  }
  if (depth != 1) fail(COOT_EINVAL, "expression does not reduce to one value");
  if (!any_load && n_slots == 0) e->dtype = COOT_F32;
  e->scalar_only = !any_load;

  // transpose parity of every op's value, walking from the root down
  e->op_parity.assign(n_ops, 0);
  std::vector<int> pend{0};
  for (int i = (int)n_ops - 1; i >= 0; --i) {
    const int p = pend.back();
    pend.pop_back();
    e->op_parity[i] = p;
    const int c = ops[i].code;
    if (is_binary(c)) {
      pend.push_back(p);
      pend.push_back(p);
    } else if (is_unary(c)) {
      pend.push_back(p);
    } else if (c == COOT_OP_TRANS) {
      pend.push_back(p ^ 1);
    }
  }
  // leaves
  e->op_leaf.assign(n_ops, -1);
  for (uint32_t i = 0; i < n_ops; ++i) {
    if (ops[i].code != COOT_OP_LOAD) continue;
    const uint32_t s = ops[i].arg;
    const uint8_t p = (uint8_t)e->op_parity[i];
    int found = -1;
    for (size_t k = 0; k < e->leaves.size(); ++k)
      if (e->leaves[k].slot == s && e->leaves[k].parity == p) found = (int)k;
    if (found < 0) {
      found = (int)e->leaves.size();
      e->leaves.push_back({s, p});
      if (p) ++e->n_p1;
    }
    e->op_leaf[i] = found;
  }
  e->root_schur = ops[n_ops - 1].code == COOT_OP_SCHUR;
  // canonical text: dtype, operator list with leaf / scalar references, leaf table
  std::ostringstream os;
  os << dtype_cname(e->dtype) << "|";
  for (uint32_t i = 0; i < n_ops; ++i) {
    const int c = ops[i].code;
    if (c == COOT_OP_LOAD) os << "L" << e->op_leaf[i] << " ";
    else if (c == COOT_OP_SCALAR) os << "S" << ops[i].arg << " ";
    else os << "o" << c << " ";
  }
  os << "|";
  for (auto& l : e->leaves) os << l.slot << "/" << (int)l.parity << ",";
  e->canon = os.str();
  return e;
}

void check_operands(const Expr& e, const coot_operand* operands) {
  const size_t n = e.slots.size();
  if (n && !operands) fail(COOT_EINVAL, "operands missing");
  for (size_t k = 0; k < n; ++k) {
    const coot_operand& o = operands[k];
    if (o.dtype != e.slots[k].dtype) fail(COOT_ETYPE, "operand " + std::to_string(k) + " has the wrong element type");
    if (o.kind != e.slots[k].kind) fail(COOT_EINVAL, "operand " + std::to_string(k) + " has the wrong kind");
    if (o.n_rows < 0 || o.n_cols < 0) fail(COOT_ESHAPE, "negative dimension");
    if (o.kind == COOT_COL && o.n_cols != 1) fail(COOT_ESHAPE, "a Col operand must have one column");
    if (o.kind == COOT_ROW && o.n_rows != 1) fail(COOT_ESHAPE, "a Row operand must have one row");
    if (o.kind == COOT_BCAST) {
      if (o.ld != 0) fail(COOT_EINVAL, "a broadcast operand has ld 0 (its columns are one vector)");
    } else {
      const int64_t ld = o.ld ? o.ld : o.n_rows;
      if (ld < o.n_rows) fail(COOT_EINVAL, "leading dimension smaller than the row count");
    }
    if (!o.data && o.n_rows * o.n_cols > 0) fail(COOT_EINVAL, "NULL operand data");
  }
}

void infer_shape(const Expr& e, const coot_operand* operands, int64_t* rows, int64_t* cols) {
  struct Sh {
    bool scalar;
    int64_t r, c;
  };
  std::vector<Sh> st;
  for (size_t i = 0; i < e.ops.size(); ++i) {
    const int c = e.ops[i].code;
    if (c == COOT_OP_LOAD) {
      const coot_operand& o = operands[e.ops[i].arg];
      st.push_back({false, o.n_rows, o.n_cols});
    } else if (c == COOT_OP_SCALAR) {
      st.push_back({true, 1, 1});
    } else if (is_binary(c)) {
      Sh b = st.back();
      st.pop_back();
      Sh a = st.back();
      st.pop_back();
      if (!a.scalar && !b.scalar && (a.r != b.r || a.c != b.c))
        fail(COOT_ESHAPE, "element-wise operands of unequal dimensions: " + std::to_string(a.r) + "x" +
                              std::to_string(a.c) + " vs " + std::to_string(b.r) + "x" + std::to_string(b.c));
      st.push_back(a.scalar ? b : a);
    } else if (c == COOT_OP_TRANS) {
      Sh a = st.back();
      st.pop_back();
      st.push_back({a.scalar, a.c, a.r});
    }
  }
  if (st.back().scalar) fail(COOT_EINVAL, "the expression reads no operand");
  *rows = st.back().r;
  *cols = st.back().c;
}

uint64_t scalar_bits(double v, int dtype) {
  switch (dtype) {
    case COOT_F32: {
      float f = (float)v;  // round to nearest even
      uint32_t b;
      std::memcpy(&b, &f, 4);
      return b;
    }
    case COOT_F64: {
      uint64_t b;
      std::memcpy(&b, &v, 8);
      return b;
    }
    case COOT_F16:
    case COOT_BF16: {
      // the scalar in the 16-bit type, carried as binary32 (the kernels' compute type):
      // binary64 -> binary32 -> 16 bits, nearest-even each time, is one correct rounding
      float f = round_half((float)v, dtype);
      uint32_t b;
      std::memcpy(&b, &f, 4);
      return b;
    }
    default: {
      if (!std::isfinite(v)) fail(COOT_EINVAL, "non-finite scalar for an integer expression");
      double t = std::trunc(v);
      double r = std::fmod(t, 4294967296.0);  // exact
      if (r < 0) r += 4294967296.0;
      return (uint64_t)(uint32_t)r;
    }
  }
}

}  // namespace coot
