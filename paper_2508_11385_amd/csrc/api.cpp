// C ABI of libcoot: argument checks, error mapping, handle ownership.
#include <cstring>
#include <string>

#include "core.h"

using namespace coot;

namespace coot {
std::string& last_error() {
  static thread_local std::string s;
  return s;
}
}  // namespace coot

extern "C" {

coot_status coot_init(int hip_device) {
  return guarded([&] {
    int n = 0;
    hip_check(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (hip_device < 0 || hip_device >= n) fail(COOT_EINVAL, "device index out of range");
    hip_check(hipSetDevice(hip_device), "hipSetDevice");
    (void)num_cus();
    (void)noalloc_scratch();  // this device's address of the allocation-free scratch array
  });
}

coot_status coot_expr_compile(const coot_op* ops, uint32_t n_ops, const coot_slot_type* slots, uint32_t n_slots,
                              uint32_t n_scalars, uint32_t flags, coot_expr** out) {
  return guarded([&] {
    if (!out) fail(COOT_EINVAL, "out handle pointer is NULL");
    *out = nullptr;
    auto h = new coot_expr;
    try {
      h->e = analyse(ops, n_ops, slots, n_slots, n_scalars, flags);
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
  });
}

coot_status coot_set_allocator(coot_alloc_fn alloc, coot_free_fn dealloc, void* ctx) {
  return guarded([&] {
    if ((alloc == nullptr) != (dealloc == nullptr)) fail(COOT_EINVAL, "give both functions or neither");
    DevAllocator a;
    a.alloc = alloc;
    a.dealloc = dealloc;
    a.ctx = ctx;
    set_allocator(a);
  });
}

coot_status coot_expr_prepare(coot_expr* h, int32_t mode, int32_t dim, uint32_t rflags, const coot_launch_cfg* cfg) {
  return guarded([&] {
    if (!h) fail(COOT_EINVAL, "NULL expression");
    Expr& e = *h->e;
    if (mode < -1 || mode > COOT_RED_VAR_DIM) fail(COOT_EINVAL, "bad mode");
    if (rflags & ~(COOT_RF_PLAIN | COOT_RF_VAR_N | COOT_PF_COMPILE_ONLY)) fail(COOT_EINVAL, "unknown prepare flag");
    int m = mode;
    if (mode == COOT_RED_ACCU && e.root_schur) m = COOT_RED_DOT;
    if (mode >= 0) check_red_mode(e, mode);
    // plan with no operands: contiguous untransposed leaves are assumed (the common case)
    std::vector<coot_operand> fake(e.slots.size());
    for (size_t k = 0; k < fake.size(); ++k) {
      fake[k].n_rows = 1;
      fake[k].n_cols = 1;
      fake[k].ld = 1;
      fake[k].dtype = e.slots[k].dtype;
      fake[k].kind = e.slots[k].kind;
    }
    coot_operand o{};
    o.n_rows = o.n_cols = o.ld = 1;
    Request rq = plan(e, fake.data(), &o, m, is_dim_kind(mode) ? dim : -1, !(rflags & COOT_RF_PLAIN), cfg);
    get_module(e, rq, !(rflags & COOT_PF_COMPILE_ONLY));
  });
}

coot_status coot_expr_out_shape(const coot_expr* h, const coot_operand* operands, int64_t* n_rows, int64_t* n_cols) {
  return guarded([&] {
    if (!h || !n_rows || !n_cols) fail(COOT_EINVAL, "NULL argument");
    check_operands(*h->e, operands);
    infer_shape(*h->e, operands, n_rows, n_cols);
  });
}

coot_status coot_expr_eval(coot_expr* h, const coot_operand* operands, const double* scalars, coot_operand* out,
                           const coot_launch_cfg* cfg, void* stream) {
  return guarded([&] {
    if (!h || !out) fail(COOT_EINVAL, "NULL argument");
    if (h->e->flags & COOT_CF_UNFUSED) {
      reject_capture((hipStream_t)stream, "the unfused comparator");
      eval_unfused(*h->e, operands, scalars, *out, cfg, (hipStream_t)stream);
    } else
      eval_fused(*h->e, operands, scalars, *out, cfg, (hipStream_t)stream);
  });
}

coot_status coot_expr_eval_reduce(coot_expr* h, const coot_operand* operands, const double* scalars, coot_operand* out,
                                  coot_expr* r, const int32_t* r_src, const double* r_scalars, int32_t kind,
                                  coot_operand* r_out, const coot_launch_cfg* cfg, void* stream) {
  return guarded([&] {
    if (!h || !out || !r || !r_out) fail(COOT_EINVAL, "NULL argument");
    if ((h->e->flags | r->e->flags) & COOT_CF_UNFUSED) fail(COOT_EUNSUPPORTED, "the comparator has no fused pair");
    reject_capture((hipStream_t)stream, "coot_expr_eval_reduce");
    eval_reduce(*h->e, operands, scalars, *out, *r->e, r_src, r_scalars, kind, *r_out, cfg, (hipStream_t)stream);
  });
}

coot_status coot_reduce(coot_expr* h, const coot_operand* operands, const double* scalars, int32_t kind, int32_t dim,
                        uint32_t flags, coot_operand* out, const coot_launch_cfg* cfg, void* stream) {
  return guarded([&] {
    if (!h || !out) fail(COOT_EINVAL, "NULL argument");
    if (flags & ~(COOT_RF_PLAIN | COOT_RF_VAR_N)) fail(COOT_EINVAL, "unknown reduce flag");
    Expr& e = *h->e;
    hipStream_t s = (hipStream_t)stream;
    reject_capture(s, "coot_reduce");
    if (!(e.flags & COOT_CF_UNFUSED)) {
      reduce_fused(e, operands, scalars, kind, dim, flags, *out, cfg, s);
      return;
    }
    // unfused comparator: materialise the expression, then reduce the temporary
    check_operands(e, operands);
    int64_t R = 0, C = 0;
    infer_shape(e, operands, &R, &C);
    const size_t bytes = (size_t)std::max<int64_t>(1, R * C) * dtype_size(e.dtype);
    coot_operand t{};
    t.data = temp_alloc(bytes, s);
    t.n_rows = R;
    t.n_cols = C;
    t.ld = R ? R : 1;
    t.dtype = e.dtype;
    t.kind = COOT_MAT;
    try {
      eval_unfused(e, operands, scalars, t, cfg, s);
      coot_op op{COOT_OP_LOAD, 0};
      coot_slot_type st{e.dtype, COOT_MAT};
      auto re = analyse(&op, 1, &st, 1, 0, 0);
      const int k = kind == COOT_RED_DOT ? COOT_RED_ACCU : kind;
      if (kind == COOT_RED_DOT && !e.root_schur) fail(COOT_EINVAL, "dot needs a % b at the root");
      reduce_fused(*re, &t, nullptr, k, dim, flags, *out, cfg, s);
      // keep the sub-expression alive until its kernels have been queued; modules are cached globally
    } catch (...) {
      temp_free(t.data, bytes, s);
      throw;
    }
    temp_free(t.data, bytes, s);
  });
}

coot_status coot_reduce_noalloc(coot_expr* h, const coot_operand* operands, const double* scalars, int32_t kind,
                                int32_t dim, uint32_t flags, coot_operand* out, const coot_launch_cfg* cfg,
                                void* stream) {
  return guarded([&] {
    if (!h || !out) fail(COOT_EINVAL, "NULL argument");
    if (flags & ~(COOT_RF_PLAIN | COOT_RF_VAR_N)) fail(COOT_EINVAL, "unknown reduce flag");
    if (h->e->flags & COOT_CF_UNFUSED)
      fail(COOT_EUNSUPPORTED, "the unfused comparator allocates temporaries; use coot_reduce");
    Scratch sc;
    sc.p = noalloc_scratch();
    sc.bytes = kNoallocScratchBytes;
    reduce_fused(*h->e, operands, scalars, kind, dim, flags, *out, cfg, (hipStream_t)stream, &sc);
  });
}

void coot_expr_release(coot_expr* h) { delete h; }

coot_status coot_expr_kernel_name(coot_expr* h, int32_t mode, int32_t dim, const coot_launch_cfg* cfg, char* buf,
                                  size_t cap) {
  return guarded([&] {
    if (!h || !buf || cap == 0) fail(COOT_EINVAL, "NULL argument");
    Expr& e = *h->e;
    std::vector<coot_operand> fake(e.slots.size());
    for (size_t k = 0; k < fake.size(); ++k) {
      fake[k].n_rows = fake[k].n_cols = fake[k].ld = 1;
      fake[k].dtype = e.slots[k].dtype;
      fake[k].kind = e.slots[k].kind;
    }
    coot_operand o{};
    o.n_rows = o.n_cols = o.ld = 1;
    int m = mode;
    if (mode == COOT_RED_ACCU && e.root_schur) m = COOT_RED_DOT;
    Request rq = plan(e, fake.data(), &o, m, is_dim_kind(mode) ? dim : -1, true, cfg);
    KernelNames names;
    generate(e, rq, hex128(e.canon), &names);
    std::strncpy(buf, names.stage1.c_str(), cap - 1);
    buf[cap - 1] = '\0';
  });
}

coot_status coot_cache_info(int64_t out[4]) {
  return guarded([&] {
    if (!out) fail(COOT_EINVAL, "out is NULL");
    cache_info(out);
  });
}

coot_status coot_cache_trim(int64_t* unloaded) {
  return guarded([&] {
    const int64_t n = cache_trim();
    if (unloaded) *unloaded = n;
  });
}

void coot_stats(double out[5]) {
  if (!out) return;
  std::lock_guard<std::mutex> g(global_mutex());
  out[0] = stats().compiles;
  out[1] = stats().mem_hits;
  out[2] = stats().disk_hits;
  out[3] = stats().launches;
  out[4] = stats().compile_ms;
}

const char* coot_last_error(void) { return last_error().c_str(); }

// Diagnostic: the generated source for a request, optionally compiled with
// hipRTC (no device needed).  mode -1 = eval; fam 0 flat / 1 tiled.
coot_status coot_debug_codegen(coot_expr* h, int32_t mode, int32_t dim, uint32_t rflags, int32_t fam, int32_t vec,
                               int32_t ept, int32_t tile_r, int32_t tile_c, int32_t compile, char* buf, size_t cap,
                               size_t* code_size) {
  return guarded([&] {
    if (!h || !buf || cap == 0) fail(COOT_EINVAL, "NULL argument");
    Expr& e = *h->e;
    Request rq;
    rq.mode = mode;
    if (mode == COOT_RED_ACCU && e.root_schur) rq.mode = COOT_RED_DOT;
    rq.dim = is_dim_kind(mode) ? dim : -1;
    rq.comp = !(rflags & COOT_RF_PLAIN);
    rq.fam = fam ? FAM_TILE : FAM_FLAT;
    rq.var.vec = vec;
    rq.var.ept = ept;
    rq.var.tr = tile_r;
    rq.var.tc = tile_c;
    KernelNames names;
    const std::string src = generate(e, rq, hex128(e.canon), &names);
    std::strncpy(buf, src.c_str(), cap - 1);
    buf[cap - 1] = '\0';
    if (code_size) *code_size = 0;
    if (compile) {
      std::vector<char> code;
      compile_source(src, names.stage1, &code);
      if (code_size) *code_size = code.size();
    }
  });
}

}  // extern "C"
