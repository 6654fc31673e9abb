// Execution: launch planning, fused evaluation, fused reductions, and the
// unfused comparator (one kernel and one temporary per operator).
#include <algorithm>
#include <cstring>
#include <unordered_map>

#include "core.h"

namespace coot {

void fail(coot_status c, const std::string& msg) { throw Error(c, msg); }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(COOT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int num_cus() {
  static int cached_dev = -1, cached = 0;
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (dev != cached_dev) {
    int n = 0;
    hip_check(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
    cached = n > 0 ? n : 1;
    cached_dev = dev;
  }
  return cached;
}

// ---- device memory: the caller's allocator, or hipMalloc ----------------------------
namespace {
DevAllocator& current_allocator() {
  static DevAllocator a;  // all NULL: hipMalloc / hipFree
  return a;
}
}  // namespace

void* dev_alloc(size_t bytes, hipStream_t s, DevAllocator* used) {
  const DevAllocator a = current_allocator();
  void* p = nullptr;
  if (a.alloc) {
    p = a.alloc(bytes, (void*)s, a.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (!p) fail(COOT_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  *used = a;
  return p;
}

void dev_free(void* p, hipStream_t s, const DevAllocator& used) {
  if (!p) return;
  if (used.dealloc) used.dealloc(p, (void*)s, used.ctx);
  else (void)hipFree(p);
}

// ---- workspace and temporaries ------------------------------------------------
namespace {
struct WsKey {
  hipStream_t s;
  int which;
  bool operator==(const WsKey& o) const { return s == o.s && which == o.which; }
};
struct WsHash {
  size_t operator()(const WsKey& k) const { return std::hash<void*>()((void*)k.s) ^ (size_t)k.which; }
};
struct WsBuf {
  void* p = nullptr;
  size_t n = 0;
  DevAllocator al;  // what allocated p
};
std::unordered_map<WsKey, WsBuf, WsHash>& ws_map() {
  static std::unordered_map<WsKey, WsBuf, WsHash> m;
  return m;
}
struct Temp {
  void* p;
  DevAllocator al;
};
std::map<std::pair<void*, size_t>, std::vector<Temp>>& temp_pool() {
  static std::map<std::pair<void*, size_t>, std::vector<Temp>> m;
  return m;
}
// allocator of every temporary handed out and not yet returned to the pool
std::map<void*, DevAllocator>& temps_out() {
  static std::map<void*, DevAllocator> m;
  return m;
}
}  // namespace

void reject_capture(hipStream_t s, const char* call) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  hip_check(hipStreamIsCapturing(s, &st), "hipStreamIsCapturing");
  if (st != hipStreamCaptureStatusNone)
    fail(COOT_EUNSUPPORTED, std::string(call) +
                                " takes library workspace and cannot be recorded into a graph (the stream is capturing)");
}

void* workspace(size_t bytes, hipStream_t s, int which) {
  std::lock_guard<std::mutex> g(global_mutex());
  WsBuf& b = ws_map()[{s, which}];
  if (b.n >= bytes && b.p) return b.p;
  size_t want = std::max<size_t>(bytes, 1 << 16);
  if (b.p) {
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    dev_free(b.p, s, b.al);
    b.p = nullptr;
    b.n = 0;
  }
  b.p = dev_alloc(want, s, &b.al);
  b.n = want;
  return b.p;
}

void* temp_alloc(size_t bytes, hipStream_t s) {
  std::lock_guard<std::mutex> g(global_mutex());
  auto& v = temp_pool()[{(void*)s, bytes}];
  Temp t;
  if (!v.empty()) {
    t = v.back();
    v.pop_back();
  } else {
    t.p = dev_alloc(std::max<size_t>(bytes, 256), s, &t.al);
  }
  temps_out()[t.p] = t.al;
  return t.p;
}

// Stream-ordered reuse: a temporary handed back here is only given out again for
// work queued later on the same stream.
void temp_free(void* p, size_t bytes, hipStream_t s) {
  std::lock_guard<std::mutex> g(global_mutex());
  auto it = temps_out().find(p);
  const DevAllocator al = it != temps_out().end() ? it->second : DevAllocator{};
  if (it != temps_out().end()) temps_out().erase(it);
  temp_pool()[{(void*)s, bytes}].push_back({p, al});
}

// Waits for the device, returns every workspace and pooled temporary to the
// allocator that provided it, and makes `a` the allocator of later ones.
void set_allocator(const DevAllocator& a) {
  std::lock_guard<std::mutex> g(global_mutex());
  if (!temps_out().empty()) fail(COOT_EINVAL, "temporaries are in use");
  hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
  for (auto& kv : ws_map()) dev_free(kv.second.p, kv.first.s, kv.second.al);
  ws_map().clear();
  for (auto& kv : temp_pool())
    for (auto& t : kv.second) dev_free(t.p, (hipStream_t)kv.first.first, t.al);
  temp_pool().clear();
  current_allocator() = a;
}

void launch(hipFunction_t f, unsigned grid, unsigned block, const KArgs& args, hipStream_t s) {
  KArgs copy = args;
  void* params[] = {&copy};
  hip_check(hipModuleLaunchKernel(f, grid, 1, 1, block, 1, 1, 0, s, params, nullptr), "hipModuleLaunchKernel");
  stats().launches += 1;
}

// ---- planning ------------------------------------------------------------------
// column stride in elements: the leading dimension, 0 for a broadcast column (COOT_BCAST)
int64_t ld_of(const coot_operand& o) {
  if (o.kind == COOT_BCAST) return o.n_cols > 1 ? 0 : (o.n_rows > 0 ? o.n_rows : 1);
  return o.ld ? o.ld : (o.n_rows > 0 ? o.n_rows : 1);
}

static bool contiguous(const coot_operand& o) { return ld_of(o) == o.n_rows || o.n_cols <= 1; }

static bool aligned(const void* p, size_t bytes) { return ((uintptr_t)p % bytes) == 0; }

// Library defaults (any field a caller leaves 0), chosen from the autotuner's
// exhaustive tables over 3,000 random signatures on MI355X as the single
// configuration with the lowest geometric-mean time ratio to each signature's best:
//   flat family:   16-byte groups, 1 group per thread per trip, 4 waves, 4 workgroups per CU
//                  (past 2^24 elements: below)
//   tiled family:  2-element groups, 4 waves (fixed), 8 workgroups per CU
//   dimension sums: 16-byte groups (one workgroup per segment)
// (the tables hold 32- and 64-bit types; the 16-bit types' defaults are measured)
coot_launch_cfg default_cfg(int fam, int mode, int dim, int dtype, int64_t n) {
  const uint16_t v16 = dtype == COOT_F64 ? 2 : (dtype_is_half(dtype) ? 8 : 4);  // 16-byte groups
  if (is_dim_kind(mode) && dim >= 0) return {v16, 0, 4, 8, 0, 0};
  // 16-bit types: 16-byte groups, 8 waves and 16 workgroups per CU for element-wise
  // flat launches, 16 workgroups per CU for tiles (measured on the 4096 x 4096 step)
  if (dtype_is_half(dtype) && fam == FAM_FLAT && mode < 0) return {8, 1, 8, 16, 0, 0};
  if (dtype_is_half(dtype) && fam != FAM_FLAT) return {8, 0, 4, 16, 0, 0};
  if (fam == FAM_FLAT) {
    // Past 2^24 elements (the streaming regime).  Reductions: fewer, longer-lived
    // workgroups, the best geomean over the largest signatures of the autotuner's timing
    // tables.  Element-wise: 2-element groups, 8 groups per thread per trip, 16
    // workgroups per CU, the best fixed configuration over 32 signatures of 2^25 to 2^28
    // elements (four types, 1 to 4 operands, exp-heavy and plain) timed one launch after
    // a flush of the caches each (1.05 of each signature's best in geometric mean
    // against 1.11 for the 16-byte groups with 2 workgroups per CU taken from the tables
    // before), and as good on the tables' signatures past 2^24 elements (1.05 against
    // 1.05-1.06): the many loads in flight per thread hide the latency of HBM.
    if (n > kStreamElems) {
      if (mode < 0) return {2, 8, 4, 16, 0, 0};
      return dtype == COOT_F64 ? coot_launch_cfg{2, 4, 8, 8, 0, 0} : coot_launch_cfg{4, 4, 4, 2, 0, 0};
    }
    return {v16, 1, 4, 4, 0, 0};
  }
  return {2, 0, 4, 8, 0, 0};
}

// The library's tile when the caller gives none: 64 x 32 for reductions along a
// dimension (the fastest fixed shape over sums and means of eight shapes from 300 x 170
// to 16384 x 256 in fp32 and fp64: 0.97 of the exhaustive picks' time against 1.04 for
// 64 x 64).  Element-wise evaluation and full reductions: 32 x 32 below 2^22 elements
// and 64 x 64 from there.  Over the autotuner's timing tables of the tiled family (time
// over each signature's best, geometric mean), 32 x 32 takes 1.07 below 2^22 elements
// against 1.41 for 64 x 64 (1.12 against 1.22 from 2^20), and 64 x 64 is ahead from 2^22
// (1.15 against 1.18 up to 2^24, 1.15 against 1.26 beyond); the threshold is the best on
// the training signatures.  Timed one launch after a flush of the caches, 47 signatures
// of 2^24 to 2^26 elements in four types put 64 x 64 at 1.08 against 1.13.  32 x 32
// whenever the staged transposed leaves would not fit.
// 16-bit types keep 64 x 64: their 16-byte groups (8 elements) need tiles of 2048
// elements or more, and the 4096 x 4096 f16 step measured Z 28 against 47 us and the
// sums 24-27 against 45-50 us on 64 x 64 tiles rather than smaller shapes.
void default_tile(const Expr& e, int mode, int dim, int64_t n, int* tr, int* tc) {
  const bool dimk = is_dim_kind(mode) && dim >= 0;
  if (dtype_is_half(e.dtype)) {
    *tr = *tc = 64;
  } else if (dimk) {
    *tr = 64;
    *tc = 32;
  } else {
    *tr = *tc = n >= kTileLargeElems ? 64 : 32;
  }
  if (tile_lds_bytes(e.n_p1, e.dtype, *tr, *tc) > kTileLdsMax) *tr = *tc = 32;
}

coot_launch_cfg resolve_cfg(const coot_launch_cfg* cfg, int fam, int mode, int dim, int dtype, int64_t n) {
  coot_launch_cfg c = default_cfg(fam, mode, dim, dtype, n);
  if (cfg) {
    if (cfg->vec) c.vec = cfg->vec;
    if (cfg->ept) c.ept = cfg->ept;
    if (cfg->waves) c.waves = cfg->waves;
    if (cfg->grid_mult) c.grid_mult = cfg->grid_mult;
    if (cfg->tile_r) c.tile_r = cfg->tile_r;
    if (cfg->tile_c) c.tile_c = cfg->tile_c;
  }
  return c;
}

Request plan(const Expr& e, const coot_operand* ops, const coot_operand* out, int mode, int dim, bool comp,
             const coot_launch_cfg* cfg) {
  Request rq;
  rq.mode = mode;
  rq.dim = dim;
  rq.comp = comp;
  bool flat = e.n_p1 == 0 && !(is_dim_kind(mode) && dim >= 0);
  for (auto& l : e.leaves)
    if (!contiguous(ops[l.slot])) flat = false;
  if (mode < 0 && out && !contiguous(*out)) flat = false;
  rq.fam = flat ? FAM_FLAT : FAM_TILE;
  int64_t R = 0, C = 0;
  infer_shape(e, ops, &R, &C);
  const coot_launch_cfg c = resolve_cfg(cfg, rq.fam, mode, dim, e.dtype, R * C);
  rq.var.vec = c.vec;
  rq.var.ept = c.ept ? c.ept : 1;
  // vec 8 (16-byte groups) for the 16-bit types only
  if (rq.var.vec != 1 && rq.var.vec != 2 && rq.var.vec != 4 && !(rq.var.vec == 8 && dtype_is_half(e.dtype)))
    fail(COOT_EINVAL, "vec must be 1, 2 or 4 (or 8 for 16-bit types)");
  if (rq.var.ept != 1 && rq.var.ept != 2 && rq.var.ept != 4 && rq.var.ept != 8) fail(COOT_EINVAL, "ept must be 1, 2, 4 or 8");
  // tile: the caller's, else the library default (default_tile); the LDS staging of the
  // transposed leaves (held in the compute type: binary32 for 16-bit types) fits 64 KiB
  if ((c.tile_r == 0) != (c.tile_c == 0)) fail(COOT_EINVAL, "give tile_r and tile_c together");
  int tr = c.tile_r, tc = c.tile_c;
  if (tr) {
    if (!tile_shape_ok(tr, tc))
      fail(COOT_EINVAL, "tile edges must be powers of two in [8, 256] with 1024 <= tile_r * tile_c <= 8192");
    if (rq.fam == FAM_TILE && tile_lds_bytes(e.n_p1, e.dtype, tr, tc) > kTileLdsMax)
      fail(COOT_EINVAL, "the staged transposed leaves of a " + std::to_string(tr) + " x " + std::to_string(tc) +
                            " tile exceed 64 KiB of LDS");
  } else {
    default_tile(e, mode, dim, R * C, &tr, &tc);
    if (rq.fam == FAM_TILE && tile_lds_bytes(e.n_p1, e.dtype, tr, tc) > kTileLdsMax)
      fail(COOT_EUNSUPPORTED, std::to_string(e.n_p1) + " transposed leaves: their staged 32 x 32 tiles exceed 64 KiB of LDS");
  }
  rq.var.tr = tr;
  rq.var.tc = tc;
  // a tile's 256 threads cover whole column segments within its columns: V <= tr * tc / 256
  if (rq.fam == FAM_TILE && rq.var.vec > tile_vec_cap(tr, tc)) rq.var.vec = tile_vec_cap(tr, tc);
  if (rq.fam == FAM_FLAT) rq.var.tr = rq.var.tc = 0;
  if (rq.fam == FAM_TILE) rq.var.ept = 0;
  if (rq.fam == FAM_FLAT && mode < 0) {
    // operands larger than the Infinity Cache together: streamed past it (non-temporal loads)
    size_t leaf_bytes = 0;
    for (size_t k = 0; k < e.slots.size(); ++k)
      if (ops[k].kind != COOT_BCAST) leaf_bytes += (size_t)(R * C) * dtype_size(e.dtype);
    rq.stream_ld = leaf_bytes > kStreamLoadBytes;
  }
  return rq;
}

// Can the V-wide kernel run on these operands?  Every access must be aligned to
// V elements: base addresses, leading dimensions and the contiguous extents.
bool vec_ok(const Expr& e, const Request& rq, const coot_operand* ops, const coot_operand* out, int64_t R,
                   int64_t C) {
  const int V = rq.var.vec;
  if (V == 1) return true;
  const size_t vb = V * dtype_size(e.dtype);
  if (rq.fam == FAM_FLAT) {
    for (auto& l : e.leaves)
      if (!aligned(ops[l.slot].data, vb)) return false;
    if (rq.mode < 0 && !aligned(out->data, vb)) return false;
    return true;
  }
  for (auto& l : e.leaves) {
    const coot_operand& o = ops[l.slot];
    if (!aligned(o.data, vb) || ld_of(o) % V) return false;
    if (l.parity == 0 && R % V) return false;
    if (l.parity == 1 && C % V) return false;
  }
  if (R % V) return false;
  if (rq.mode < 0 && (!aligned(out->data, vb) || ld_of(*out) % V)) return false;
  return true;
}

void fill_args(const Expr& e, const coot_operand* ops, const double* scalars, KArgs* a) {
  std::memset(a, 0, sizeof *a);
  for (size_t k = 0; k < e.slots.size(); ++k) {
    a->leaf[k] = ops[k].data;
    a->ld[k] = ld_of(ops[k]);
  }
  if (e.n_scalars && !scalars) fail(COOT_EINVAL, "scalars missing");
  for (uint32_t k = 0; k < e.n_scalars; ++k) a->sc[k] = scalar_bits(scalars[k], e.dtype);
}

void check_alias(const Expr& e, const coot_operand* ops, const coot_operand& out, size_t es) {
  const int64_t oc = out.n_cols, orr = out.n_rows;
  if (orr * oc == 0) return;
  const char* ob = (const char*)out.data;
  const char* oe = ob + (size_t)(ld_of(out) * (oc - 1) + orr) * es;
  for (size_t k = 0; k < e.slots.size(); ++k) {
    const coot_operand& o = ops[k];
    if (o.n_rows * o.n_cols == 0) continue;
    const char* b = (const char*)o.data;
    const char* en = b + (size_t)(ld_of(o) * (o.n_cols - 1) + o.n_rows) * es;
    if (en <= ob || oe <= b) continue;
    bool identity = b == ob && ld_of(o) == ld_of(out) && o.n_rows == orr && o.n_cols == oc;
    for (auto& l : e.leaves)
      if (l.slot == k && l.parity) identity = false;
    if (!identity) fail(COOT_EALIAS, "output overlaps operand " + std::to_string(k) + " with a different index map");
  }
}

unsigned flat_grid(int64_t n, int V, int E, int bs, int gm) {
  const int64_t nv = std::max<int64_t>(1, (n + V - 1) / V);
  const int64_t need = (nv + (int64_t)bs * E - 1) / ((int64_t)bs * E);
  const int64_t cap = (int64_t)gm * num_cus();
  return (unsigned)std::max<int64_t>(1, std::min(need, cap));
}

unsigned tile_grid(int64_t R, int64_t C, int tr, int tc, int gm) {
  const int64_t nt = ((R + tr - 1) / tr) * ((C + tc - 1) / tc);
  const int64_t cap = (int64_t)gm * num_cus();
  return (unsigned)std::max<int64_t>(1, std::min(nt, cap));
}

static bool same_call(const Expr::EvalMemo& m, const Expr& e, const coot_operand* ops, const coot_operand& out,
                      const coot_launch_cfg* cfg, bool plain_store) {
  if (!m.valid || m.plain != plain_store || m.has_cfg != (cfg != nullptr)) return false;
  if (cfg && std::memcmp(cfg, &m.cfg, sizeof *cfg) != 0) return false;
  if (std::memcmp(&out, &m.out, sizeof out) != 0) return false;
  const size_t n = e.slots.size();
  return n == m.ops.size() && (n == 0 || std::memcmp(ops, m.ops.data(), n * sizeof(coot_operand)) == 0);
}

void eval_fused(Expr& e, const coot_operand* ops, const double* scalars, const coot_operand& out,
                const coot_launch_cfg* cfg, hipStream_t s, bool plain_store) {
  if (e.n_scalars && !scalars) fail(COOT_EINVAL, "scalars missing");
  if (!e.slots.empty() && !ops) fail(COOT_EINVAL, "operands missing");
  {
    std::unique_lock<std::mutex> g(e.mu);
    if (same_call(e.memo, e, ops, out, cfg, plain_store)) {
      KArgs a = e.memo.a;
      const hipFunction_t f = e.memo.f;
      const unsigned grid = e.memo.grid, block = e.memo.block;
      g.unlock();
      for (uint32_t k = 0; k < e.n_scalars; ++k) a.sc[k] = scalar_bits(scalars[k], e.dtype);
      launch(f, grid, block, a, s);
      return;
    }
  }
  check_operands(e, ops);
  int64_t R = 0, C = 0;
  infer_shape(e, ops, &R, &C);
  if (out.dtype != e.dtype) fail(COOT_ETYPE, "output element type differs from the expression's");
  if (out.n_rows != R || out.n_cols != C)
    fail(COOT_ESHAPE, "output must be " + std::to_string(R) + "x" + std::to_string(C));
  if (ld_of(out) < R || (!out.data && R * C)) fail(COOT_EINVAL, "bad output operand");
  const size_t es = dtype_size(e.dtype);
  check_alias(e, ops, out, es);
  if (R * C == 0) return;
  Request rq = plan(e, ops, &out, -1, -1, true, cfg);
  rq.plain_store = plain_store;
  auto m = get_module(e, rq, true);
  KArgs a;
  fill_args(e, ops, scalars, &a);
  a.out = out.data;
  a.out_ld = ld_of(out);
  a.n_rows = R;
  a.n_cols = C;
  const bool v = vec_ok(e, rq, ops, &out, R, C);
  const std::string& kn = (v || rq.var.vec == 1) ? m->names.stage1 : m->names.stage1_fallback;
  hipFunction_t f = m->fn(kn);
  const coot_launch_cfg c = resolve_cfg(cfg, rq.fam, -1, -1, e.dtype, R * C);
  unsigned grid, block;
  if (rq.fam == FAM_FLAT) {
    block = 64 * c.waves;
    grid = flat_grid(R * C, v ? rq.var.vec : 1, rq.var.ept, (int)block, c.grid_mult);
  } else {
    block = 256;
    grid = tile_grid(R, C, rq.var.tr, rq.var.tc, c.grid_mult);
  }
  launch(f, grid, block, a, s);
  std::lock_guard<std::mutex> g(e.mu);
  Expr::EvalMemo& mm = e.memo;
  mm.ops.assign(ops, ops + e.slots.size());
  mm.out = out;
  mm.has_cfg = cfg != nullptr;
  if (cfg) mm.cfg = *cfg;
  mm.plain = plain_store;
  mm.f = f;
  mm.grid = grid;
  mm.block = block;
  mm.a = a;
  std::memset(mm.a.sc, 0, sizeof mm.a.sc);
  mm.valid = true;
}

// out = e, then a full reduction of r over e's operands and the result, in one
// pass (see generate_pair).  Both statements must be flat: every leaf untransposed
// and contiguous; r's operand slot k is operand r_src[k] of e, or out for -1.
void eval_reduce(Expr& e, const coot_operand* ops, const double* scalars, const coot_operand& out, Expr& r,
                 const int32_t* r_src, const double* r_scalars, int kind, const coot_operand& r_out,
                 const coot_launch_cfg* cfg, hipStream_t s) {
  if (e.n_scalars && !scalars) fail(COOT_EINVAL, "scalars missing");
  if (r.n_scalars && !r_scalars) fail(COOT_EINVAL, "scalars of the reduced statement missing");
  if (!r.slots.empty() && !r_src) fail(COOT_EINVAL, "operand map of the reduced statement missing");
  if (!e.slots.empty() && !ops) fail(COOT_EINVAL, "operands missing");
  {
    std::unique_lock<std::mutex> g(e.mu);
    const Expr::PairMemo& pm = e.pair_memo;
    const size_t n = e.slots.size(), nr = r.slots.size();
    if (pm.valid && pm.r_uid == r.uid && pm.kind == kind && pm.has_cfg == (cfg != nullptr) &&
        (!cfg || std::memcmp(cfg, &pm.cfg, sizeof *cfg) == 0) && std::memcmp(&out, &pm.out, sizeof out) == 0 &&
        std::memcmp(&r_out, &pm.r_out, sizeof r_out) == 0 && pm.ops.size() == n && pm.r_src.size() == nr &&
        (n == 0 || std::memcmp(ops, pm.ops.data(), n * sizeof(coot_operand)) == 0) &&
        (nr == 0 || std::memcmp(r_src, pm.r_src.data(), nr * sizeof(int32_t)) == 0)) {
      KArgs a = pm.a;
      const hipFunction_t f1 = pm.f1, f2 = pm.f2;
      const unsigned grid = pm.grid, block = pm.block;
      g.unlock();
      for (uint32_t k = 0; k < e.n_scalars; ++k) a.sc[k] = scalar_bits(scalars[k], e.dtype);
      for (uint32_t k = 0; k < r.n_scalars; ++k) a.sc[e.n_scalars + k] = scalar_bits(r_scalars[k], e.dtype);
      a.ws = workspace((size_t)grid * 32, s, 0);
      a.out = out.data;
      launch(f1, grid, block, a, s);
      a.out = r_out.data;
      launch(f2, 1, 256, a, s);
      return;
    }
  }
  check_operands(e, ops);
  int64_t R = 0, C = 0;
  infer_shape(e, ops, &R, &C);
  if (out.dtype != e.dtype || r.dtype != e.dtype || r_out.dtype != e.dtype)
    fail(COOT_ETYPE, "both statements and both outputs take one element type");
  if (out.n_rows != R || out.n_cols != C)
    fail(COOT_ESHAPE, "output must be " + std::to_string(R) + "x" + std::to_string(C));
  if (ld_of(out) < R || (!out.data && R * C)) fail(COOT_EINVAL, "bad output operand");
  const size_t es = dtype_size(e.dtype);
  check_alias(e, ops, out, es);
  check_red_mode(r, kind);
  if (is_dim_kind(kind) || kind == COOT_RED_NORM || kind == COOT_RED_VAR)
    fail(COOT_EUNSUPPORTED, "a fused statement pair closes with accu, dot, min, max, mean, norm1 or norm_inf");
  if (r_out.n_rows * r_out.n_cols != 1 || !r_out.data) fail(COOT_ESHAPE, "the reduction writes one element");
  if (e.n_scalars + r.n_scalars > (uint32_t)kMaxScalars) fail(COOT_EUNSUPPORTED, "more than 32 scalars in the pair");
  if (r.n_scalars && !r_scalars) fail(COOT_EINVAL, "scalars of the reduced statement missing");
  if (!r.slots.empty() && !r_src) fail(COOT_EINVAL, "operand map of the reduced statement missing");
  std::vector<coot_operand> rops(r.slots.size());
  std::vector<int> src(r.slots.size());
  for (size_t k = 0; k < r.slots.size(); ++k) {
    src[k] = r_src[k];
    if (src[k] == -1) {
      rops[k] = out;
      rops[k].kind = r.slots[k].kind;  // the result read as the slot declares it (same layout)
    } else if (src[k] >= 0 && (size_t)src[k] < e.slots.size()) {
      rops[k] = ops[src[k]];
    } else {
      fail(COOT_EINVAL, "operand map entry out of range");
    }
  }
  check_operands(r, rops.data());
  int64_t RR = 0, RC = 0;
  infer_shape(r, rops.data(), &RR, &RC);
  if (RR != R || RC != C) fail(COOT_ESHAPE, "the two statements have different shapes");
  if (r.n_p1 != 0 || e.n_p1 != 0) fail(COOT_EUNSUPPORTED, "a fused statement pair reads every leaf untransposed");
  if ((kind == COOT_RED_MIN || kind == COOT_RED_MAX || kind == COOT_RED_MEAN) && R * C == 0)
    fail(COOT_EINVAL, "min / max / mean of an empty expression");
  Request rq = plan(e, ops, &out, -1, -1, true, cfg);
  if (rq.fam != FAM_FLAT) fail(COOT_EUNSUPPORTED, "a fused statement pair needs contiguous operands and output");
  const int mode = kind == COOT_RED_ACCU && r.root_schur ? COOT_RED_DOT : kind;
  auto m = get_module_pair(e, r, src, mode, rq, true);
  KArgs a;
  fill_args(e, ops, scalars, &a);
  for (uint32_t k = 0; k < r.n_scalars; ++k) a.sc[e.n_scalars + k] = scalar_bits(r_scalars[k], e.dtype);
  a.out = out.data;
  a.out_ld = ld_of(out);
  a.n_rows = R;
  a.n_cols = C;
  const bool v = vec_ok(e, rq, ops, &out, R, C);
  const std::string& kn = (v || rq.var.vec == 1) ? m->names.stage1 : m->names.stage1_fallback;
  const coot_launch_cfg c = resolve_cfg(cfg, FAM_FLAT, -1, -1, e.dtype, R * C);
  const unsigned block = 64u * c.waves;
  const unsigned grid = flat_grid(R * C, v ? rq.var.vec : 1, rq.var.ept, (int)block, c.grid_mult);
  a.n_part = grid;
  a.ws = workspace((size_t)grid * 32, s, 0);
  const hipFunction_t f1 = m->fn(kn), f2 = m->fn(m->names.stage2);
  launch(f1, grid, block, a, s);
  a.out = r_out.data;  // stage 2 writes the reduction's result
  launch(f2, 1, 256, a, s);
  std::lock_guard<std::mutex> g(e.mu);
  Expr::PairMemo& pm = e.pair_memo;
  pm.ops.assign(ops, ops + e.slots.size());
  pm.out = out;
  pm.r_out = r_out;
  pm.r_uid = r.uid;
  pm.r_src.assign(r_src, r_src + r.slots.size());
  pm.kind = kind;
  pm.has_cfg = cfg != nullptr;
  if (cfg) pm.cfg = *cfg;
  pm.f1 = f1;
  pm.f2 = f2;
  pm.grid = grid;
  pm.block = block;
  pm.a = a;
  std::memset(pm.a.sc, 0, sizeof pm.a.sc);
  pm.valid = true;
}

DimPlan dim_plan(int64_t R, int64_t C, int dim, int tile_r, int tile_c, int per_cu, size_t cs) {
  DimPlan p;
  const int64_t tr = (R + tile_r - 1) / tile_r, tc = (C + tile_c - 1) / tile_c;
  // segments of K tiles along the reduced dimension, K growing once there are more
  // than per_cu tiles per CU (at most 16): fewer partials, fewer lane combines
  const int64_t nred = dim == 0 ? tr : tc, nkeep = dim == 0 ? tc : tr;
  const int64_t K =
      std::max<int64_t>(1, std::min<int64_t>({16, nred, (nred * nkeep) / ((int64_t)std::max(1, per_cu) * num_cus())}));
  p.n_out = dim == 0 ? C : R;
  p.n_part = std::max<int64_t>(1, (nred + K - 1) / K);
  p.nseg = nkeep * p.n_part;
  p.part_bytes = (size_t)std::max<int64_t>(1, p.n_part * p.n_out) * 2 * cs;
  return p;
}

void launch_dim(hipFunction_t stage1, hipFunction_t stage2, KArgs& a, const DimPlan& p, hipStream_t s) {
  a.n_part = p.n_part;
  const unsigned g1 = (unsigned)std::min<int64_t>(p.nseg, 1 << 30);
  const unsigned g2 = (unsigned)std::max<int64_t>(1, std::min<int64_t>((p.n_out + 3) / 4, 65536));
  if (p.nseg > 0) launch(stage1, g1, 256, a, s);
  launch(stage2, g2, 256, a, s);
}

void check_red_mode(const Expr& e, int mode) {
  if (mode < COOT_RED_ACCU || mode > COOT_RED_VAR_DIM) fail(COOT_EINVAL, "unknown reduction");
  if (mode == COOT_RED_DOT && !e.root_schur) fail(COOT_EINVAL, "dot needs an expression whose root is a % b");
  const bool float_only = mode == COOT_RED_NORM || mode == COOT_RED_MEAN || mode == COOT_RED_NORM1 ||
                          mode == COOT_RED_NORMINF || mode == COOT_RED_MEAN_DIM || mode == COOT_RED_VAR ||
                          mode == COOT_RED_VAR_DIM;
  if (float_only && dtype_is_int(e.dtype)) fail(COOT_ETYPE, "norm / mean / var of an integer expression");
}

void reduce_fused(Expr& e, const coot_operand* ops, const double* scalars, int kind, int dim, uint32_t flags,
                  const coot_operand& out, const coot_launch_cfg* cfg, hipStream_t s, const Scratch* sc) {
  check_operands(e, ops);
  int64_t R = 0, C = 0;
  infer_shape(e, ops, &R, &C);
  if (out.dtype != e.dtype) fail(COOT_ETYPE, "output element type differs from the expression's");
  int mode = kind;
  if (kind == COOT_RED_ACCU && e.root_schur) mode = COOT_RED_DOT;  // accu(x % y) is dot(x, y)
  check_red_mode(e, kind);
  const bool dimk = is_dim_kind(kind);
  if (dimk && dim != 0 && dim != 1) fail(COOT_EINVAL, "a reduction along a dimension needs dim 0 or 1");
  if ((kind == COOT_RED_MIN || kind == COOT_RED_MAX || kind == COOT_RED_MEAN || kind == COOT_RED_VAR) && R * C == 0)
    fail(COOT_EINVAL, "min / max / mean / var of an empty expression");
  const bool var = kind == COOT_RED_VAR || kind == COOT_RED_VAR_DIM;
  if ((flags & COOT_RF_VAR_N) && !var) fail(COOT_EINVAL, "COOT_RF_VAR_N applies to a variance only");
  int64_t n_out = 1;
  if (dimk) {
    n_out = dim == 0 ? C : R;
    const bool ok = dim == 0 ? (out.n_rows == 1 && out.n_cols == C) : (out.n_rows == R && out.n_cols == 1);
    if (!ok) fail(COOT_ESHAPE, dim == 0 ? "a reduction along dim 0 writes 1 x n_cols" : "a reduction along dim 1 writes n_rows x 1");
    if (out.n_rows * out.n_cols > 1 && !contiguous(out)) fail(COOT_EINVAL, "reduction output must be contiguous");
  } else {
    if (out.n_rows * out.n_cols != 1) fail(COOT_ESHAPE, "a full reduction writes one element");
  }
  if (!out.data && n_out) fail(COOT_EINVAL, "NULL output");
  if (n_out == 0) return;
  const bool comp = !(flags & COOT_RF_PLAIN);
  const bool by_n = (flags & COOT_RF_VAR_N) != 0;
  Request rq = plan(e, ops, nullptr, mode, dimk ? dim : -1, comp, cfg);
  auto m = sc ? find_loaded_module(e, rq) : get_module(e, rq, true);
  // partial results: the library's per-stream workspaces, or the halves of the caller's scratch
  auto part_buf = [&](size_t bytes, int which) -> void* {
    if (!sc) return workspace(bytes, s, which);
    const size_t half = sc->bytes / 2;
    if (bytes > half)
      fail(COOT_EUNSUPPORTED, "the reduction needs " + std::to_string(bytes) + " bytes of partial results; the " +
                                  "allocation-free scratch holds " + std::to_string(half) + " per buffer");
    return (char*)sc->p + (size_t)which * half;
  };
  KArgs a;
  fill_args(e, ops, scalars, &a);
  a.out = out.data;
  a.out_ld = ld_of(out);
  a.n_rows = R;
  a.n_cols = C;
  const bool v = vec_ok(e, rq, ops, nullptr, R, C);
  const std::string& kn = (v || rq.var.vec == 1) ? m->names.stage1 : m->names.stage1_fallback;
  // dimension partials are kept in the compute type (binary32 for 16-bit types)
  const size_t cs = dtype_is_half(e.dtype) ? 4 : dtype_size(e.dtype);
  const coot_launch_cfg c = resolve_cfg(cfg, rq.fam, mode, dimk ? dim : -1, e.dtype, R * C);
  if (dimk) {
    const DimPlan dp = dim_plan(R, C, dim, rq.var.tr, rq.var.tc, c.grid_mult, cs);
    a.ws = part_buf(dp.part_bytes, 0);
    if (var) a.ws2 = part_buf(dp.part_bytes, 1);  // a variance: sum d^2 in ws, sum d in ws2
    launch_dim(m->fn(kn), m->fn(var && by_n ? m->names.stage2_dev_n : m->names.stage2), a, dp, s);
    return;
  }
  unsigned grid;
  unsigned block;
  if (rq.fam == FAM_FLAT) {
    block = 64 * c.waves;
    grid = flat_grid(R * C, v ? rq.var.vec : 1, rq.var.ept, block, c.grid_mult);
  } else {
    block = 256;
    grid = tile_grid(R, C, rq.var.tr, rq.var.tc, c.grid_mult);
  }
  a.n_part = grid;
  a.ws = part_buf((size_t)grid * 32, 0);
  a.ws2 = part_buf(64 + (size_t)grid * 32, 1);
  launch(m->fn(kn), grid, block, a, s);
  // a variance's stage 2 merges the records' (count, mean, M2) and divides by N - 1 or N
  launch(m->fn(var && by_n ? m->names.stage2_dev_n : m->names.stage2), 1, 256, a, s);
  if (mode == COOT_RED_NORM) {
    // runs only when stage 2 found squares that could have overflowed or underflowed
    launch(m->fn(m->names.stage1_rescale), grid, block, a, s);
    launch(m->fn(m->names.stage2_rescale), 1, 256, a, s);
  }
}

// ---- unfused comparator -------------------------------------------------------------
// Each operator runs as its own kernel into a temporary (trans included: it is
// materialised).  Sub-expressions are compiled through the same machinery.
namespace {
std::unordered_map<std::string, std::unique_ptr<Expr>>& sub_cache() {
  static std::unordered_map<std::string, std::unique_ptr<Expr>> m;
  return m;
}

Expr& sub_expr(const std::vector<coot_op>& ops, const std::vector<coot_slot_type>& slots, uint32_t n_sc) {
  std::string k;
  for (auto& o : ops) k += std::to_string(o.code) + "." + std::to_string(o.arg) + " ";
  k += "|";
  for (auto& sl : slots) k += std::to_string(sl.dtype) + "." + std::to_string(sl.kind) + " ";
  k += "|" + std::to_string(n_sc);
  std::lock_guard<std::mutex> g(global_mutex());
  auto& m = sub_cache();
  auto it = m.find(k);
  if (it != m.end()) return *it->second;
  auto e = analyse(ops.data(), (uint32_t)ops.size(), slots.data(), (uint32_t)slots.size(), n_sc, 0);
  Expr& r = *e;
  m[k] = std::move(e);
  return r;
}

struct Val {
  bool scalar = false;
  uint32_t sidx = 0;
  coot_operand op{};
  bool temp = false;
  size_t bytes = 0;
};
}  // namespace

void eval_unfused(Expr& e, const coot_operand* ops, const double* scalars, const coot_operand& out,
                  const coot_launch_cfg* cfg, hipStream_t s) {
  check_operands(e, ops);
  int64_t R = 0, C = 0;
  infer_shape(e, ops, &R, &C);
  if (out.n_rows != R || out.n_cols != C) fail(COOT_ESHAPE, "output has the wrong dimensions");
  if (out.dtype != e.dtype) fail(COOT_ETYPE, "output element type differs from the expression's");
  if (R * C == 0) return;
  const size_t es = dtype_size(e.dtype);
  std::vector<Val> st;
  auto release = [&](Val& v) {
    if (v.temp) temp_free(v.op.data, v.bytes, s);
  };
  const size_t n_ops = e.ops.size();
  if (n_ops == 1) {  // a bare LOAD: a copy
    eval_fused(e, ops, scalars, out, cfg, s, true);
    return;
  }
  for (size_t i = 0; i < n_ops; ++i) {
    const coot_op& o = e.ops[i];
    if (o.code == COOT_OP_LOAD) {
      Val v;
      v.op = ops[o.arg];
      if (!v.op.ld) v.op.ld = v.op.n_rows;
      st.push_back(v);
      continue;
    }
    if (o.code == COOT_OP_SCALAR) {
      Val v;
      v.scalar = true;
      v.sidx = o.arg;
      st.push_back(v);
      continue;
    }
    const bool last = i + 1 == n_ops;
    std::vector<Val> in;
    const bool bin = o.code >= COOT_OP_ADD && o.code <= COOT_OP_DIV;
    if (bin) {
      Val b = st.back();
      st.pop_back();
      Val a = st.back();
      st.pop_back();
      in = {a, b};
    } else {
      in = {st.back()};
      st.pop_back();
    }
    if (o.code == COOT_OP_TRANS && in[0].scalar) {
      st.push_back(in[0]);
      continue;
    }
    bool all_scalar = true;
    for (auto& v : in) all_scalar = all_scalar && v.scalar;
    if (all_scalar) fail(COOT_EUNSUPPORTED, "unfused evaluation of a scalar-only sub-expression");
    std::vector<coot_op> sops;
    std::vector<coot_slot_type> sslots;
    std::vector<coot_operand> sopnds;
    std::vector<double> ssc;
    int64_t r = 0, c = 0;
    for (auto& v : in) {
      if (v.scalar) {
        sops.push_back({COOT_OP_SCALAR, (uint32_t)ssc.size()});
        ssc.push_back(scalars[v.sidx]);
      } else {
        sops.push_back({COOT_OP_LOAD, (uint32_t)sslots.size()});
        sslots.push_back({v.op.dtype, v.op.kind});
        sopnds.push_back(v.op);
        r = v.op.n_rows;
        c = v.op.n_cols;
      }
    }
    sops.push_back({o.code, 0});
    if (o.code == COOT_OP_TRANS) std::swap(r, c);
    Expr& se = sub_expr(sops, sslots, (uint32_t)ssc.size());
    Val res;
    if (last) {
      res.op = out;
    } else {
      res.temp = true;
      res.bytes = (size_t)r * c * es;
      res.op.data = temp_alloc(res.bytes, s);
      res.op.n_rows = r;
      res.op.n_cols = c;
      res.op.ld = r;
      res.op.dtype = e.dtype;
      res.op.kind = c == 1 ? COOT_COL : (r == 1 ? COOT_ROW : COOT_MAT);
      if (r == 1 && c == 1) res.op.kind = COOT_MAT;
    }
    // operand kinds of the temporaries must match the slots just declared
    for (size_t k = 0; k < sopnds.size(); ++k) sslots[k].kind = sopnds[k].kind;
    eval_fused(se, sopnds.data(), ssc.data(), res.op, cfg, s, true);
    for (auto& v : in) release(v);
    st.push_back(res);
  }
}

}  // namespace coot
