// Autotuning of the fused kernels' launch configuration.
//
// A configuration is (vec, ept, waves, grid_mult, tile_r, tile_c): elements per
// access group, groups in flight per thread, wavefronts per workgroup, workgroups
// per CU and the output tile of the tiled family.  vec, ept and the tile are
// compile-time (one tuning module per signature holds every variant), waves and
// grid_mult are launch parameters.  The tiled family runs 256-thread workgroups, so
// vec, grid_mult and the tile vary there.
// Timing: one warm-up launch per configuration, then `reps` rounds; in each round
// every configuration is timed once with HIP events on the caller's stream around
// enough back-to-back launches to span 40 us (the per-launch time of a repeated
// call, with launch overhead included), or around a single launch after a 512 MiB
// write that evicts L2 and the Infinity Cache.  The median per configuration is
// reported.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "core.h"

extern "C" hipError_t coot_flush_launch(void* buf, size_t bytes, unsigned v, hipStream_t s);

using namespace coot;

namespace {

constexpr size_t kFlushBytes = 512u << 20;
unsigned g_flush_value = 1;  // what each flush folds its reads with (any value; it varies)
constexpr float kSampleUs = 40.0f;  // a timing sample spans at least this many microseconds

bool tune_mode_ok(int mode, int dim) {
  if (mode == -1 || mode == COOT_RED_ACCU) return true;
  return is_dim_kind(mode) && (dim == 0 || dim == 1);
}

struct Prepared {
  Request rq;
  std::shared_ptr<Module> m;
  int64_t R = 0, C = 0;
  int dim = -1;  // reductions along a dimension: 0 or 1
};

Prepared prepare(Expr& e, const coot_operand* ops, const coot_operand* out, int mode, int dim, bool load) {
  if (!tune_mode_ok(mode, dim))
    fail(COOT_EUNSUPPORTED, "tuning covers element-wise evaluation, accu, and sum / mean / var along dim 0 or 1");
  if (mode >= 0) check_red_mode(e, mode);
  Prepared p;
  check_operands(e, ops);
  infer_shape(e, ops, &p.R, &p.C);
  int m = mode;
  if (mode == COOT_RED_ACCU && e.root_schur) m = COOT_RED_DOT;
  p.dim = is_dim_kind(mode) ? dim : -1;
  p.rq = plan(e, ops, mode < 0 ? out : nullptr, m, p.dim, true, nullptr);
  p.rq.all_variants = true;
  p.rq.var.vec = 4;
  p.rq.var.ept = p.rq.fam == FAM_FLAT ? 4 : 0;
  p.m = get_module(e, p.rq, load);
  return p;
}

// The tuning module's request for one configuration: its vector width and, for the
// tiled family, its tile (the library's default tile when the configuration has none).
Request cfg_request(const Prepared& p, const coot_launch_cfg& c) {
  Request rq = p.rq;
  rq.var.vec = c.vec;
  if (rq.fam == FAM_TILE && c.tile_r) {
    rq.var.tr = c.tile_r;
    rq.var.tc = c.tile_c;
  }
  return rq;
}

// Whether a configuration can run on these operands (vector width vs alignment and
// tile, the tile's LDS staging).
bool cfg_runnable(Expr& e, const Prepared& p, const coot_launch_cfg& c, const coot_operand* ops,
                  const coot_operand* out) {
  if (c.vec == 8 && !dtype_is_half(e.dtype)) return false;  // 16-byte groups of 16-bit elements only
  const Request rq = cfg_request(p, c);
  if (rq.fam == FAM_TILE) {
    if (c.vec > tile_vec_cap(rq.var.tr, rq.var.tc)) return false;
    if (tile_lds_bytes(e.n_p1, e.dtype, rq.var.tr, rq.var.tc) > kTileLdsMax) return false;
    bool listed = false;  // the tuning module holds the tile shapes of tile_shapes()
    for (auto& t : tile_shapes()) listed = listed || (t.first == rq.var.tr && t.second == rq.var.tc);
    if (!listed) return false;
  }
  return vec_ok(e, rq, ops, out, p.R, p.C);
}

// Launch one configuration (returns false if it cannot run on these operands).
bool launch_cfg(Expr& e, Prepared& p, const coot_launch_cfg& c, const coot_operand* ops, const double* scalars,
                const coot_operand* out, hipStream_t s) {
  if (!cfg_runnable(e, p, c, ops, out)) return false;
  const Request rq = cfg_request(p, c);
  const int ept = rq.fam == FAM_FLAT ? c.ept : 0;
  hipFunction_t f = p.m->fn(variant_name(e, rq, c.vec, ept));
  KArgs a;
  fill_args(e, ops, scalars, &a);
  a.n_rows = p.R;
  a.n_cols = p.C;
  unsigned grid, block;
  if (rq.fam == FAM_FLAT) {
    block = 64u * c.waves;
    grid = flat_grid(p.R * p.C, c.vec, c.ept, (int)block, c.grid_mult);
  } else {
    block = 256;
    grid = tile_grid(p.R, p.C, rq.var.tr, rq.var.tc, c.grid_mult);
  }
  if (p.dim >= 0) {
    // along a dimension: grid_mult is the number of tiles per CU past which segments grow
    const size_t cs = dtype_is_half(e.dtype) ? 4 : dtype_size(e.dtype);
    const DimPlan dp = dim_plan(p.R, p.C, p.dim, rq.var.tr, rq.var.tc, c.grid_mult, cs);
    a.out = out->data;
    a.out_ld = ld_of(*out);
    a.ws = workspace(dp.part_bytes, s, 2);
    if (rq.mode == COOT_RED_VAR_DIM) a.ws2 = workspace(dp.part_bytes, s, 3);
    launch_dim(f, p.m->fn(p.m->names.stage2), a, dp, s);
  } else if (rq.mode < 0) {
    a.out = out->data;
    a.out_ld = ld_of(*out);
    launch(f, grid, block, a, s);
  } else {
    a.out = out->data;
    a.n_part = grid;
    a.ws = workspace((size_t)grid * 32, s, 2);
    a.ws2 = workspace(64 + (size_t)grid * 32, s, 3);
    launch(f, grid, block, a, s);
    launch(p.m->fn(p.m->names.stage2), 1, 256, a, s);
  }
  return true;
}

bool valid_cfg(const coot_launch_cfg& c) {
  auto pow2 = [](int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; };
  const bool tile = (c.tile_r == 0 && c.tile_c == 0) || tile_shape_ok(c.tile_r, c.tile_c);
  return pow2(c.vec, 1, 8) && pow2(c.ept, 1, 8) && pow2(c.waves, 1, 8) && pow2(c.grid_mult, 1, 16) && tile;
}

}  // namespace

extern "C" {

uint32_t coot_tune_space(int32_t family, coot_launch_cfg* cfgs, uint32_t cap) {
  std::vector<coot_launch_cfg> v;
  if (family == 1) {
    for (auto& t : tile_shapes())
      for (uint16_t vec : {1, 2, 4})
        for (uint16_t gm : {2, 4, 8, 16}) v.push_back({vec, 1, 4, gm, (uint16_t)t.first, (uint16_t)t.second});
  } else {
    for (uint16_t vec : {1, 2, 4})
      for (uint16_t ept : {1, 2, 4, 8})
        for (uint16_t waves : {1, 2, 4, 8})
          for (uint16_t gm : {2, 4, 8, 16}) v.push_back({vec, ept, waves, gm, 0, 0});
  }
  if (cfgs)
    for (uint32_t i = 0; i < std::min<uint32_t>(cap, (uint32_t)v.size()); ++i) cfgs[i] = v[i];
  return (uint32_t)v.size();
}

coot_status coot_tune_prepare(coot_expr* h, const coot_operand* operands, int32_t mode, int32_t dim,
                              int32_t* family) {
  return guarded([&] {
    if (!h) fail(COOT_EINVAL, "NULL expression");
    Prepared p = prepare(*h->e, operands, nullptr, mode, dim, false);
    if (family) *family = p.rq.fam == FAM_FLAT ? 0 : 1;
  });
}

coot_status coot_tune_runnable(coot_expr* h, const coot_operand* operands, const coot_operand* out, int32_t mode,
                               int32_t dim,
                               const coot_launch_cfg* cfgs, uint32_t n_cfgs, int32_t* runnable) {
  return guarded([&] {
    if (!h || (n_cfgs && (!cfgs || !runnable)) || (mode < 0 && !out)) fail(COOT_EINVAL, "NULL argument");
    Prepared p = prepare(*h->e, operands, nullptr, mode, dim, false);
    for (uint32_t k = 0; k < n_cfgs; ++k) {
      if (!valid_cfg(cfgs[k])) fail(COOT_EINVAL, "invalid launch configuration");
      runnable[k] = cfg_runnable(*h->e, p, cfgs[k], operands, mode < 0 ? out : nullptr) ? 1 : 0;
    }
  });
}

coot_status coot_flush_caches(void* stream) {
  return guarded([&] {
    hipStream_t s = (hipStream_t)stream;
    void* buf = workspace(kFlushBytes, s, 4);
    hip_check(coot_flush_launch(buf, kFlushBytes, g_flush_value++, s), "cache flush");
  });
}

coot_status coot_tune_table(coot_expr* h, const coot_operand* operands, const double* scalars, coot_operand* out,
                            int32_t mode, int32_t dim, const coot_launch_cfg* cfgs, uint32_t n_cfgs, uint32_t reps,
                            int32_t flush,
                            float* times_us, void* stream) {
  return guarded([&] {
    if (!h || !out || (n_cfgs && (!cfgs || !times_us))) fail(COOT_EINVAL, "NULL argument");
    if (reps == 0 || reps > 101) fail(COOT_EINVAL, "reps must be 1..101");
    Expr& e = *h->e;
    hipStream_t s = (hipStream_t)stream;
    if (mode < 0) {
      int64_t R, C;
      check_operands(e, operands);
      infer_shape(e, operands, &R, &C);
      if (out->n_rows != R || out->n_cols != C || out->dtype != e.dtype) fail(COOT_ESHAPE, "output shape");
    } else if (is_dim_kind(mode)) {
      int64_t R, C;
      check_operands(e, operands);
      infer_shape(e, operands, &R, &C);
      const bool ok = dim == 0 ? (out->n_rows == 1 && out->n_cols == C) : (out->n_rows == R && out->n_cols == 1);
      if (!ok || out->dtype != e.dtype) fail(COOT_ESHAPE, "a reduction along dim 0 writes 1 x n_cols, along dim 1 n_rows x 1");
      if (out->n_rows * out->n_cols > 1 && !(ld_of(*out) == out->n_rows || out->n_cols <= 1))
        fail(COOT_EINVAL, "reduction output must be contiguous");
    } else if (out->n_rows * out->n_cols != 1 || out->dtype != e.dtype) {
      fail(COOT_ESHAPE, "accu writes one element");
    }
    Prepared p = prepare(e, operands, out, mode, dim, true);
    void* fbuf = flush ? workspace(kFlushBytes, s, 4) : nullptr;
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    unsigned fv = 1;
    auto timed = [&](const coot_launch_cfg& c, uint32_t launches) {
      if (fbuf) hip_check(coot_flush_launch(fbuf, kFlushBytes, fv++, s), "flush");
      hip_check(hipEventRecord(e0, s), "hipEventRecord");
      for (uint32_t l = 0; l < launches; ++l) launch_cfg(e, p, c, operands, scalars, out, s);
      hip_check(hipEventRecord(e1, s), "hipEventRecord");
      hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0;
      hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      return ms * 1000.0f / (float)launches;
    };
    try {
      // warm-up launch of every configuration, which is also its validity test
      std::vector<uint32_t> live;
      for (uint32_t k = 0; k < n_cfgs; ++k) {
        if (!valid_cfg(cfgs[k])) fail(COOT_EINVAL, "invalid launch configuration");
        times_us[k] = NAN;
        if (launch_cfg(e, p, cfgs[k], operands, scalars, out, s)) live.push_back(k);
      }
      if (!live.empty()) {
        // launches per sample: enough back-to-back launches to span kSampleUs (one when flushing)
        uint32_t launches = 1;
        if (!fbuf) {
          const float t1 = std::max(0.5f, timed(cfgs[live[0]], 1));
          launches = (uint32_t)std::min(64.0f, std::max(1.0f, std::ceil(kSampleUs / t1)));
        }
        // rounds over all configurations, so that drift in clocks or temperature spreads evenly
        std::vector<std::vector<float>> t(live.size());
        for (uint32_t r = 0; r < reps; ++r)
          for (size_t i = 0; i < live.size(); ++i) t[i].push_back(timed(cfgs[live[i]], launches));
        for (size_t i = 0; i < live.size(); ++i) {
          std::sort(t[i].begin(), t[i].end());
          times_us[live[i]] = t[i][t[i].size() / 2];
        }
      }
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  });
}

// Launch with an explicit configuration through the tuning module (no extra compile).
coot_status coot_tune_launch(coot_expr* h, const coot_operand* operands, const double* scalars, coot_operand* out,
                             int32_t mode, int32_t dim, const coot_launch_cfg* cfg, void* stream) {
  return guarded([&] {
    if (!h || !out || !cfg) fail(COOT_EINVAL, "NULL argument");
    if (!valid_cfg(*cfg)) fail(COOT_EINVAL, "invalid launch configuration");
    Prepared p = prepare(*h->e, operands, out, mode, dim, true);
    if (!launch_cfg(*h->e, p, *cfg, operands, scalars, out, (hipStream_t)stream))
      fail(COOT_EINVAL, "configuration not valid for these operands");
  });
}

}  // extern "C"
