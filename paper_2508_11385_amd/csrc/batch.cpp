// Batched evaluation: many small independent expressions in one persistent
// launch, captured once into a HIP graph and replayed.
//
// Each expression's analysed IR (leaves with their transpose parity) becomes
// register bytecode: the tree is emitted in Sethi-Ullman order (the operand that
// needs more registers first), so registers behave as a stack of depth
// need(root) <= 8; a binary op with a leaf or scalar operand takes it directly
// (one instruction, no register).  Every expression is cut into tiles (flat
// chunks or TS x TS output tiles); the tile list holds (expression, tile) pairs
// and a fixed grid walks it round-robin.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>

#include "batch_abi.h"
#include "core.h"

extern "C" hipError_t coot_batch_launch_kernel(int dtype, int ts, int g, unsigned grid, const void* ex,
                                              const void* tiles, int t_begin, int t_end, const void* code,
                                              const void* scal, int nstk, int np1, int flat_only, hipStream_t s);

using namespace coot;
using coot::batch::BatchExpr;

namespace {

struct Node {
  int kind;  // 0 leaf, 1 scalar, 2 unary, 3 binary
  uint32_t op = 0, arg = 0;
  int a = -1, b = -1;
  int need = 1;
};

uint32_t map_op(int code) {
  using namespace coot::batch;
  switch (code) {
    case COOT_OP_ADD: return OP_ADD;
    case COOT_OP_SUB: return OP_SUB;
    case COOT_OP_SCHUR: return OP_MUL;
    case COOT_OP_DIV: return OP_DIV;
    case COOT_OP_NEG: return OP_NEG;
    case COOT_OP_ABS: return OP_ABS;
    case COOT_OP_EXP: return OP_EXP;
    case COOT_OP_LOG: return OP_LOG;
    case COOT_OP_SQRT: return OP_SQRT;
    default: return OP_SQUARE;
  }
}

// Register bytecode of one expression; returns the registers used.
int emit_program(const Expr& e, uint32_t sc_base, std::vector<uint32_t>* code) {
  using namespace coot::batch;
  std::vector<Node> nodes;
  std::vector<int> st;
  for (size_t i = 0; i < e.ops.size(); ++i) {
    const coot_op& o = e.ops[i];
    Node n;
    if (o.code == COOT_OP_LOAD) {
      n.kind = 0;
      n.arg = (uint32_t)e.op_leaf[i];
    } else if (o.code == COOT_OP_SCALAR) {
      n.kind = 1;
      n.arg = sc_base + o.arg;
    } else if (o.code == COOT_OP_TRANS) {
      continue;  // index map folded into the leaves
    } else if (o.code >= COOT_OP_ADD && o.code <= COOT_OP_DIV) {
      n.kind = 3;
      n.op = map_op(o.code);
      n.b = st.back();
      st.pop_back();
      n.a = st.back();
      st.pop_back();
      const int na = nodes[n.a].need, nb = nodes[n.b].need;
      const bool pa = nodes[n.a].kind <= 1, pb = nodes[n.b].kind <= 1;  // plain leaf or scalar
      // a plain operand is taken directly by the op, so only the other one needs registers
      if (pb) n.need = na;
      else if (pa) n.need = nb;
      else n.need = na == nb ? na + 1 : std::max(na, nb);
    } else {
      n.kind = 2;
      n.op = map_op(o.code);
      n.a = st.back();
      st.pop_back();
      n.need = nodes[n.a].need;
    }
    nodes.push_back(n);
    st.push_back((int)nodes.size() - 1);
  }
  const int root = st.back();
  if (nodes[root].need > 8) fail(COOT_EUNSUPPORTED, "expression needs more than 8 registers in the batch interpreter");
  // iterative Sethi-Ullman emission
  struct Frame {
    int node, base, stage;
  };
  std::vector<Frame> fs{{root, 0, 0}};
  int max_reg = 0;
  while (!fs.empty()) {
    Frame& f = fs.back();
    const Node& n = nodes[f.node];
    max_reg = std::max(max_reg, f.base);
    if (n.kind == 0) {
      code->push_back(encode(OP_LEAF, f.base, n.arg));
      fs.pop_back();
    } else if (n.kind == 1) {
      code->push_back(encode(OP_SCAL, f.base, n.arg));
      fs.pop_back();
    } else if (n.kind == 2) {
      if (f.stage == 0) {
        f.stage = 1;
        fs.push_back({n.a, f.base, 0});
      } else {
        code->push_back(encode(n.op, f.base, 0));
        fs.pop_back();
      }
    } else {
      const bool pa = nodes[n.a].kind <= 1, pb = nodes[n.b].kind <= 1;
      // a plain operand (leaf or scalar) goes second and is fused into the op; otherwise
      // the operand needing more registers goes first
      const bool left_first = pb ? true : pa ? false : nodes[n.a].need >= nodes[n.b].need;
      const int first = left_first ? n.a : n.b, second = left_first ? n.b : n.a;
      if (f.stage == 0) {
        f.stage = 1;
        fs.push_back({first, f.base, 0});
      } else if (f.stage == 1 && nodes[second].kind <= 1) {
        uint32_t op = n.op;
        if (!left_first) {  // r[b] holds the b-operand: swap the non-commutative ops
          if (op == OP_SUB) op = OP_RSUB;
          else if (op == OP_DIV) op = OP_RDIV;
        }
        const Node& x = nodes[second];
        code->push_back(encode((x.kind == 0 ? OP_WITH_LEAF : OP_WITH_SCAL) + op, f.base, x.arg));
        fs.pop_back();
      } else if (f.stage == 1) {
        f.stage = 2;
        const int base = f.base;
        fs.push_back({second, base + 1, 0});
      } else {
        uint32_t op = n.op;
        if (!left_first) {  // r[b] holds b-operand: swap for the non-commutative ops
          if (op == OP_SUB) op = OP_RSUB;
          else if (op == OP_DIV) op = OP_RDIV;
        }
        code->push_back(encode(op, f.base, 0));
        fs.pop_back();
      }
    }
  }
  return max_reg + 1;
}

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  void upload(const std::vector<T>& v) {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = v.size();
    if (n == 0) return;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) fail(COOT_ENOMEM, "batch descriptor allocation failed");
    hip_check(hipMemcpy(p, v.data(), n * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

struct coot_batch {
  int dtype = COOT_BATCH_F32;
  std::vector<BatchExpr> ex;
  std::vector<uint32_t> code;
  std::vector<uint64_t> scal_bits;
  std::vector<std::pair<int, int>> ranges;  // per expression: tile range
  int n_flat_tiles = 0;                      // tiles [0, n_flat_tiles) are flat chunks
  std::vector<uint32_t> tiles;
  std::vector<int> vec4_ok, flat_ok;
  DevBuf<BatchExpr> d_ex;
  DevBuf<uint32_t> d_code, d_tiles;
  DevBuf<uint64_t> d_scal32x2;  // scalars packed as the element type
  // launch settings of the two parts: [0] flat chunks, [1] 2-D tiles
  int ts[2] = {32, 32};             // tile edge (a flat chunk holds ts * ts elements)
  int g[2] = {1, 1};                // groups of 4 elements per thread: ts * ts / (4 g) threads per tile
  int gm[2] = {16, 16};             // workgroups per CU
  bool allow_vec[2] = {true, true};  // 128-bit accesses where the layout allows them
  unsigned grid[2] = {1, 1};
  int nstk = 1;    // LDS stack entries: the deepest expression's registers minus the top
  int max_p1 = 0;  // most transposed leaves in one expression
  int64_t bytes = 0;
  bool concurrent = true;  // the graph runs the two parts side by side (fork / join)
  hipStream_t cap = nullptr, cap2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~coot_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (cap2) (void)hipStreamDestroy(cap2);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace {

// each part's persistent grid: gm workgroups per CU, at most one per tile
void set_grids(coot_batch* b) {
  const int n_tiles = (int)(b->tiles.size() / 2);
  const int n_part[2] = {b->n_flat_tiles, n_tiles - b->n_flat_tiles};
  for (int p = 0; p < 2; ++p) b->grid[p] = (unsigned)std::max(1, std::min(n_part[p], b->gm[p] * num_cus()));
}

// The work-list holds the flat-chunk tiles first (one launch of the flat-only
// interpreter), then the 2-D tiles (the general interpreter).
void build_tiles(coot_batch* b) {
  b->tiles.clear();
  b->ranges.assign(b->ex.size(), {0, 0});
  std::vector<size_t> order;
  for (int pass = 0; pass < 2; ++pass)
    for (size_t k = 0; k < b->ex.size(); ++k)
      if ((b->flat_ok[k] != 0) == (pass == 0)) order.push_back(k);
  b->n_flat_tiles = 0;
  for (size_t k : order) {
    BatchExpr& e = b->ex[k];
    e.flat = b->flat_ok[k];
    const int part = e.flat ? 0 : 1, ts = b->ts[part];
    const int tr = (e.n_rows + ts - 1) / ts, tc = (e.n_cols + ts - 1) / ts;
    e.tile_shift = 0;
    while ((1 << e.tile_shift) < tr) ++e.tile_shift;
    e.tile_mask = (1u << e.tile_shift) - 1u;
    e.vec4 = (b->allow_vec[part] && b->vec4_ok[k]) ? 1 : 0;
    const int begin = (int)(b->tiles.size() / 2);
    const int64_t chunk = (int64_t)ts * ts;  // flat tiles: 4 elements per thread, ts*ts/4 threads
    if (e.flat) {
      const int64_t nt = ((int64_t)e.n_rows * e.n_cols + chunk - 1) / chunk;
      for (int64_t t = 0; t < nt; ++t) {
        b->tiles.push_back((uint32_t)k);
        b->tiles.push_back((uint32_t)t);
      }
    } else {  // column-major tile order; the tile coordinates packed, no division on the device
      for (int tj = 0; tj < tc; ++tj)
        for (int ti = 0; ti < tr; ++ti) {
          b->tiles.push_back((uint32_t)k);
          b->tiles.push_back((uint32_t)ti | ((uint32_t)tj << e.tile_shift));
        }
    }
    b->ranges[k] = {begin, (int)(b->tiles.size() / 2)};
    if (e.flat) b->n_flat_tiles = (int)(b->tiles.size() / 2);
  }
  b->d_ex.upload(b->ex);
  b->d_tiles.upload(b->tiles);
  set_grids(b);
}

// Transposed-leaf tiles staged in LDS: as many as an expression needs (at most 4 on
// one-wave tiles, staged by LDS DMA; 2 on larger tiles, staged through registers)
// while the workgroup's LDS stays within 32 KB (several workgroups per CU), and
// always within the 64 KB a workgroup may hold (2 KB of it hold the exp table); the
// rest are read directly.
constexpr size_t kMaxDynLds = 65536 - 2048;
int staged_tiles(const coot_batch* b) {
  const size_t es = b->dtype == COOT_BATCH_F32 ? 4 : 8;
  const int ts = b->ts[1];
  const bool one_wave = ts * ts / (4 * b->g[1]) == 64;
  const size_t stack = (size_t)b->nstk * ts * ts * es;                    // nstk entries of the tile's values
  const size_t slot = (size_t)ts * (one_wave ? ts : ts + 1) * es;         // as the kernel lays them out
  const size_t budget = std::max<size_t>(32768, stack + slot);
  size_t n = std::min<size_t>({(size_t)b->max_p1, one_wave ? 4u : 2u, budget > stack ? (budget - stack) / slot : 0});
  while (n > 0 && stack + n * slot > kMaxDynLds) --n;
  return (int)n;
}

// part 0: the flat-chunk tiles with the flat-only interpreter; part 1: the 2-D tiles
void launch_part(coot_batch* b, int part, hipStream_t s) {
  const int n_tiles = (int)(b->tiles.size() / 2), nf = b->n_flat_tiles;
  const int t0 = part == 0 ? 0 : nf, t1 = part == 0 ? nf : n_tiles;
  if (t1 <= t0) return;
  hip_check(coot_batch_launch_kernel(b->dtype, b->ts[part], b->g[part], b->grid[part], b->d_ex.p, b->d_tiles.p, t0, t1,
                                     b->d_code.p, b->d_scal32x2.p, b->nstk, part == 0 ? 0 : staged_tiles(b),
                                     part == 0 ? 1 : 0, s),
            "batch kernel launch");
}

// Both parts, in stream order or side by side: the 2-D part (latency bound: header,
// staging and leaf loads in a chain per tile) leaves memory bandwidth idle that the
// flat part's workgroups use when they share the CUs.  `s2` is a second stream
// forked from `s` (both captured into the same graph).
void launch_all(coot_batch* b, hipStream_t s, hipStream_t s2) {
  const int nf = b->n_flat_tiles, n = (int)(b->tiles.size() / 2);
  if (!b->concurrent || !s2 || nf == 0 || nf == n) {
    launch_part(b, 0, s);
    launch_part(b, 1, s);
    return;
  }
  hip_check(hipEventRecord(b->fork, s), "hipEventRecord");
  hip_check(hipStreamWaitEvent(s2, b->fork, 0), "hipStreamWaitEvent");
  launch_part(b, 1, s);
  launch_part(b, 0, s2);
  hip_check(hipEventRecord(b->join, s2), "hipEventRecord");
  hip_check(hipStreamWaitEvent(s, b->join, 0), "hipStreamWaitEvent");
}

void capture(coot_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  if (!b->cap) hip_check(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "hipStreamCreate");
  if (!b->cap2) hip_check(hipStreamCreateWithFlags(&b->cap2, hipStreamNonBlocking), "hipStreamCreate");
  if (!b->fork) hip_check(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming), "hipEventCreate");
  if (!b->join) hip_check(hipEventCreateWithFlags(&b->join, hipEventDisableTiming), "hipEventCreate");
  hip_check(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  try {
    launch_all(b, b->cap, b->cap2);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(b->cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hip_check(hipStreamEndCapture(b->cap, &b->graph), "hipStreamEndCapture");
  hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
}

// Every expression of a batch runs concurrently with every other (one persistent
// launch, two captured streams), so no output may overlap another expression's
// output or operand.  Outputs sorted by address: any overlap among them shows
// between neighbours; each operand range is then looked up among the (disjoint,
// sorted) outputs and every output it meets must be its own expression's.
struct Interval {
  uintptr_t lo, hi;  // [lo, hi)
  uint32_t expr;
};

void check_batch_overlaps(std::vector<Interval>& outs, const std::vector<Interval>& ins) {
  std::sort(outs.begin(), outs.end(), [](const Interval& a, const Interval& b) { return a.lo < b.lo; });
  for (size_t i = 1; i < outs.size(); ++i)
    if (outs[i].lo < outs[i - 1].hi)
      fail(COOT_EALIAS, "outputs of batch expressions " + std::to_string(outs[i - 1].expr) + " and " +
                            std::to_string(outs[i].expr) + " overlap");
  for (const Interval& r : ins) {
    // first output whose end lies past the operand's start (ends ascend with starts)
    auto it = std::upper_bound(outs.begin(), outs.end(), r.lo,
                               [](uintptr_t v, const Interval& o) { return v < o.hi; });
    for (; it != outs.end() && it->lo < r.hi; ++it)
      if (it->expr != r.expr)
        fail(COOT_EALIAS, "batch expression " + std::to_string(r.expr) + " reads memory that expression " +
                              std::to_string(it->expr) + " writes");
  }
}

}  // namespace

extern "C" {

coot_status coot_batch_create(uint32_t n, coot_expr* const* exprs, const coot_operand* const* operands,
                              const double* const* scalars, const coot_operand* outs, const coot_launch_cfg* cfg,
                              void* stream, coot_batch** out) {
  (void)stream;
  return guarded([&] {
    if (!out || (n && (!exprs || !operands || !outs))) fail(COOT_EINVAL, "NULL argument");
    *out = nullptr;
    auto b = std::make_unique<coot_batch>();
    if (cfg) {  // the same settings for both parts
      if (cfg->tile_r != cfg->tile_c || (cfg->tile_r && cfg->tile_r != 16 && cfg->tile_r != 32))
        fail(COOT_EINVAL, "batch tiles are 16 x 16 or 32 x 32 elements");
      int ts = 32, g = 1;
      if (cfg->tile_r == 16 || (!cfg->tile_r && cfg->waves == 1)) {
        ts = 16;
        if (cfg->waves > 1) fail(COOT_EINVAL, "a 16 x 16 batch tile is one wavefront");
      } else if (cfg->waves) {
        if (cfg->waves != 1 && cfg->waves != 2 && cfg->waves != 4)
          fail(COOT_EINVAL, "a 32 x 32 batch tile takes 1, 2 or 4 wavefronts");
        g = 4 / cfg->waves;
      }
      for (int p = 0; p < 2; ++p) {
        if (cfg->waves || cfg->tile_r) {
          b->ts[p] = ts;
          b->g[p] = g;
        }
        if (cfg->grid_mult) b->gm[p] = cfg->grid_mult;
        if (cfg->vec == 1) b->allow_vec[p] = false;
      }
    }
    int dtype = -1;
    std::vector<double> scal;
    std::vector<Interval> out_iv, in_iv;  // byte ranges of the outputs and the operands
    for (uint32_t k = 0; k < n; ++k) {
      if (!exprs[k]) fail(COOT_EINVAL, "NULL expression in the batch");
      Expr& e = *exprs[k]->e;
      if (e.dtype != COOT_F32 && e.dtype != COOT_F64) fail(COOT_EUNSUPPORTED, "batch supports f32 and f64 expressions");
      const int dt = e.dtype == COOT_F32 ? COOT_BATCH_F32 : COOT_BATCH_F64;
      if (dtype >= 0 && dt != dtype) fail(COOT_ETYPE, "all expressions of a batch must share one element type");
      dtype = dt;
      if (e.leaves.size() > COOT_BATCH_MAXL) fail(COOT_EUNSUPPORTED, "too many leaves for the batch interpreter");
      const coot_operand* ops = operands[k];
      check_operands(e, ops);
      for (size_t l = 0; l < e.slots.size(); ++l)
        if (ops[l].kind == COOT_BCAST) fail(COOT_EUNSUPPORTED, "broadcast operands are not taken by batches");
      int64_t R = 0, C = 0;
      infer_shape(e, ops, &R, &C);
      const coot_operand& o = outs[k];
      if (o.dtype != e.dtype || o.n_rows != R || o.n_cols != C) fail(COOT_ESHAPE, "batch output has the wrong shape or type");
      BatchExpr be;
      std::memset(&be, 0, sizeof be);
      const size_t es = dtype_size(e.dtype);
      const int64_t old = o.ld ? o.ld : std::max<int64_t>(1, R);
      // the interpreter addresses every operand as a raw buffer with 32-bit byte offsets
      auto extent = [&](int64_t rows, int64_t cols, int64_t ld) -> uint32_t {
        const int64_t bytes = rows > 0 && cols > 0 ? ((cols - 1) * ld + rows) * (int64_t)es : 0;
        if (bytes >= (int64_t(1) << 31) || ld >= (int64_t(1) << 31))
          fail(COOT_EUNSUPPORTED, "batch operands must each span less than 2 GiB");
        return (uint32_t)bytes;
      };
      // 2-D tiles: 4-row column segments need R, every untransposed ld and 16-byte alignment
      bool v4 = R % 4 == 0 && old % 4 == 0 && ((uintptr_t)o.data % 16) == 0;
      // flat chunks: every leaf untransposed and contiguous, like the output
      bool flat = e.n_p1 == 0 && (old == R || C <= 1);
      bool aligned = ((uintptr_t)o.data % 16) == 0;
      for (size_t l = 0; l < e.leaves.size(); ++l) {
        const coot_operand& lo = ops[e.leaves[l].slot];
        const int64_t lld = lo.ld ? lo.ld : std::max<int64_t>(1, lo.n_rows);
        be.leaf[l] = lo.data;
        be.nrec[l] = extent(lo.n_rows, lo.n_cols, lld);
        be.ld[l] = (uint32_t)lld;
        aligned = aligned && ((uintptr_t)lo.data % 16) == 0;
        if (e.leaves[l].parity) {
          be.p1_mask |= 1u << l;
        } else {
          v4 = v4 && lld % 4 == 0 && ((uintptr_t)lo.data % 16) == 0;
          flat = flat && (lld == lo.n_rows || lo.n_cols <= 1);
        }
      }
      // within the expression, the output may only alias an operand read untransposed
      // with its own layout; overlaps across expressions are checked below
      check_alias(e, ops, o, es);
      if (R * C > 0) {
        const uintptr_t ob = (uintptr_t)o.data;
        out_iv.push_back({ob, ob + (uintptr_t)((C - 1) * old + R) * es, k});
        for (size_t l = 0; l < e.slots.size(); ++l) {
          const coot_operand& lo = ops[l];
          if (lo.n_rows * lo.n_cols == 0) continue;
          const uintptr_t lb = (uintptr_t)lo.data;
          in_iv.push_back({lb, lb + (uintptr_t)((lo.n_cols - 1) * ld_of(lo) + lo.n_rows) * es, k});
        }
      }
      if (flat) v4 = aligned;
      be.out = o.data;
      be.out_nrec = extent(R, C, old);
      be.out_ld = (uint32_t)old;
      be.n_rows = (int32_t)R;
      be.n_cols = (int32_t)C;
      be.n_leaves = (int32_t)e.leaves.size();
      be.code_off = (int32_t)b->code.size();
      be.sc_off = 0;
      const int regs = emit_program(e, (uint32_t)scal.size(), &b->code);
      b->nstk = std::max(b->nstk, regs - 1);
      b->max_p1 = std::max(b->max_p1, __builtin_popcount(be.p1_mask));
      be.code_len = (int32_t)(b->code.size() - be.code_off);
      if (e.n_scalars && !scalars) fail(COOT_EINVAL, "scalars missing");
      for (uint32_t s = 0; s < e.n_scalars; ++s) scal.push_back(scalars[k][s]);
      b->ex.push_back(be);
      b->vec4_ok.push_back(v4 ? 1 : 0);
      b->flat_ok.push_back(flat ? 1 : 0);
      // algorithmic bytes: each distinct operand slot read once, the output written once
      std::vector<bool> seen(e.slots.size(), false);
      int64_t elems = R * C;
      for (auto& l : e.leaves)
        if (!seen[l.slot]) {
          seen[l.slot] = true;
          elems += ops[l.slot].n_rows * ops[l.slot].n_cols;
        }
      b->bytes += elems * (int64_t)es;
    }
    check_batch_overlaps(out_iv, in_iv);
    b->dtype = dtype < 0 ? COOT_BATCH_F32 : dtype;
    // scalars in the element type, one 64-bit slot each (fp32 scalars use the low word of a float array)
    if (b->dtype == COOT_BATCH_F32) {
      std::vector<uint64_t> packed((scal.size() + 1) / 2 + 1, 0);
      float* f = reinterpret_cast<float*>(packed.data());
      for (size_t s = 0; s < scal.size(); ++s) f[s] = (float)scal[s];
      b->scal_bits = packed;
    } else {
      b->scal_bits.resize(scal.size() + 1, 0);
      std::memcpy(b->scal_bits.data(), scal.data(), scal.size() * 8);
    }
    b->d_code.upload(b->code.empty() ? std::vector<uint32_t>{0} : b->code);
    b->d_scal32x2.upload(b->scal_bits);
    build_tiles(b.get());
    capture(b.get());
    *out = b.release();
  });
}

coot_status coot_batch_launch(coot_batch* b, void* stream) {
  return guarded([&] {
    if (!b) fail(COOT_EINVAL, "NULL batch");
    if (b->tiles.empty()) return;
    hip_check(hipGraphLaunch(b->exec, (hipStream_t)stream), "hipGraphLaunch");
  });
}

coot_status coot_batch_launch_each(coot_batch* b, void* stream) {
  return guarded([&] {
    if (!b) fail(COOT_EINVAL, "NULL batch");
    for (auto& r : b->ranges) {
      if (r.second == r.first) continue;
      const int fl = r.second <= b->n_flat_tiles ? 1 : 0, part = fl ? 0 : 1;
      const unsigned g = (unsigned)std::min(r.second - r.first, (int)b->grid[part]);
      hip_check(coot_batch_launch_kernel(b->dtype, b->ts[part], b->g[part], g, b->d_ex.p, b->d_tiles.p, r.first, r.second,
                                         b->d_code.p, b->d_scal32x2.p, b->nstk, fl ? 0 : staged_tiles(b), fl,
                                         (hipStream_t)stream),
                "batch kernel launch");
    }
  });
}

coot_status coot_batch_tune(coot_batch* b, void* stream, coot_launch_cfg* best, float* best_us) {
  return guarded([&] {
    if (!b) fail(COOT_EINVAL, "NULL batch");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    float total = 0;
    // median of 5 timed runs of fn (after one warm-up run)
    auto median_ms = [&](auto&& fn) {
      fn();
      std::vector<float> t_ms;
      for (int rep = 0; rep < 5; ++rep) {
        hip_check(hipEventRecord(e0, s), "hipEventRecord");
        fn();
        hip_check(hipEventRecord(e1, s), "hipEventRecord");
        hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        t_ms.push_back(ms);
      }
      std::sort(t_ms.begin(), t_ms.end());
      return t_ms[2];
    };
    try {
      // each part is tuned on its own launch (the other part's settings do not affect it)
      for (int part = 0; part < 2; ++part) {
        float bt = 1e30f;
        int bts = b->ts[part], bg = b->g[part], bgm = b->gm[part];
        bool bvec = b->allow_vec[part];
        // tile shapes: 16 x 16 by one wave, 32 x 32 by four, two or one wave(s)
        for (auto shape : {std::pair<int, int>{16, 1}, {32, 1}, {32, 2}, {32, 4}}) {
          for (bool vec : {true, false}) {
            b->ts[part] = shape.first;
            b->g[part] = shape.second;
            b->allow_vec[part] = vec;
            build_tiles(b);
            for (int gm : {2, 4, 8, 16}) {
              b->gm[part] = gm;
              set_grids(b);
              const float t = median_ms([&] { launch_part(b, part, s); });
              if (t < bt) {
                bt = t;
                bts = shape.first;
                bg = shape.second;
                bgm = gm;
                bvec = vec;
              }
            }
          }
        }
        b->ts[part] = bts;
        b->g[part] = bg;
        b->gm[part] = bgm;
        b->allow_vec[part] = bvec;
      }
      // then the graph: the parts one after the other (each with its own best grid), or
      // side by side.  A persistent grid that alone fills every CU leaves the other part
      // no room until it drains, so side by side also tries smaller grid pairs that let
      // both stay resident together.
      build_tiles(b);
      const int gm_best[2] = {b->gm[0], b->gm[1]};
      bool best_c = false;
      int best_gm[2] = {gm_best[0], gm_best[1]};
      total = 1e30f;
      auto try_graph = [&](bool c, int g0, int g1) {
        b->concurrent = c;
        b->gm[0] = g0;
        b->gm[1] = g1;
        set_grids(b);
        capture(b);
        const float t = median_ms([&] { hip_check(hipGraphLaunch(b->exec, s), "hipGraphLaunch"); });
        if (t < total) {
          total = t;
          best_c = c;
          best_gm[0] = g0;
          best_gm[1] = g1;
        }
      };
      try_graph(false, gm_best[0], gm_best[1]);
      try_graph(true, gm_best[0], gm_best[1]);
      if (b->n_flat_tiles > 0 && b->n_flat_tiles < (int)(b->tiles.size() / 2))
        for (int g1 : {1, 2, 3, 4, 6})
          for (int g0 : {1, 2, 4, 8})
            if (g1 < gm_best[1] || g0 < gm_best[0]) try_graph(true, g0, g1);
      b->concurrent = best_c;
      b->gm[0] = best_gm[0];
      b->gm[1] = best_gm[1];
      set_grids(b);
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    capture(b);
    if (best) {  // the flat part's settings (coot_batch_info reports both parts)
      best->vec = b->allow_vec[0] ? 4 : 1;
      best->ept = 4;
      best->waves = (uint16_t)(b->ts[0] * b->ts[0] / (256 * b->g[0]));
      best->grid_mult = (uint16_t)b->gm[0];
    }
    if (best_us) *best_us = total * 1000.0f;
  });
}

coot_status coot_batch_info(const coot_batch* b, int64_t info[15]) {
  return guarded([&] {
    if (!b || !info) fail(COOT_EINVAL, "NULL argument");
    info[0] = (int64_t)b->ex.size();
    info[1] = (int64_t)(b->tiles.size() / 2);
    info[2] = b->bytes;
    info[3] = b->ts[0];
    info[4] = b->grid[0];
    info[9] = b->ts[1];
    info[10] = b->grid[1];
    info[11] = b->n_flat_tiles;
    info[12] = b->concurrent ? 1 : 0;
    info[13] = b->g[0];
    info[14] = b->g[1];
    int64_t v4 = 0, fl = 0;
    for (auto& e : b->ex) {
      v4 += e.vec4;
      fl += e.flat;
    }
    info[5] = v4;
    info[6] = fl;
    info[7] = b->nstk;
    info[8] = staged_tiles(b);
  });
}

void coot_batch_release(coot_batch* b) { delete b; }

}  // extern "C"
