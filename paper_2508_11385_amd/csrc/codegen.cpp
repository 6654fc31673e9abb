// Code generation: one small HIP translation unit per (expression signature,
// request).  The generated text is the expression body as straight-line SSA on
// registers plus extern "C" wrappers that instantiate the hand-written kernel
// templates of coot_dev.h.  This is the fused-kernel generation the paper's
// conclusion leaves to follow-up work, done at run time (the kernel set of
// Section 4 is also compiled at run time and cached).
#include <functional>
#include <sstream>

#include "core.h"

namespace coot {

struct EmbeddedHeader {
  const char* name;
  const char* text;
};
extern const EmbeddedHeader kDeviceHeaders[];  // embedded device headers (written at build time)
extern const int kNumDeviceHeaders;

const std::vector<std::pair<std::string, std::string>>& device_headers() {
  static const std::vector<std::pair<std::string, std::string>> h = [] {
    std::vector<std::pair<std::string, std::string>> v;
    for (int i = 0; i < kNumDeviceHeaders; ++i) v.emplace_back(kDeviceHeaders[i].name, kDeviceHeaders[i].text);
    return v;
  }();
  return h;
}

// A request's key: its fields as bytes (short enough for the string's inline buffer,
// so a cache lookup on the hot path allocates nothing).
std::string Request::key() const {
  const char b[] = {(char)(mode + 2), (char)(dim + 2), (char)comp,        (char)fam,           (char)var.vec,
                    (char)var.ept,    (char)(var.tr & 0xff), (char)(var.tr >> 8), (char)(var.tc & 0xff),
                    (char)(var.tc >> 8), (char)all_variants, (char)plain_store, (char)stream_ld};
  return std::string(b, sizeof b);
}

bool tile_shape_ok(int tr, int tc) {
  auto pow2 = [](int v) { return v >= 8 && v <= 256 && (v & (v - 1)) == 0; };
  return pow2(tr) && pow2(tc) && tr * tc >= 1024 && tr * tc <= 8192;
}

size_t tile_lds_bytes(int n_p1, int dtype, int tr, int tc) {
  const size_t es = dtype_is_half(dtype) ? 4 : dtype_size(dtype);
  return (size_t)(n_p1 > 0 ? n_p1 : 0) * tr * (tc + 1) * es;
}

const std::vector<std::pair<int, int>>& tile_shapes() {
  static const std::vector<std::pair<int, int>> v = {{64, 64}, {128, 32}, {32, 128}, {256, 16}, {128, 64}, {32, 32},
                                                      {64, 16}, {16, 64},  {128, 8},  {256, 8},  {128, 16}, {64, 32}};
  return v;
}

// tile part of a kernel name: t<rows>x<cols>
static std::string tile_tag(const Request& rq) {
  return "t" + std::to_string(rq.var.tr) + "x" + std::to_string(rq.var.tc);
}

int red_kind(int mode) {
  switch (mode) {
    case COOT_RED_DOT: return RK_DOT;
    case COOT_RED_NORM: return RK_SUMSQ;
    case COOT_RED_MIN: return RK_MIN;
    case COOT_RED_MAX: return RK_MAX;
    case COOT_RED_MEAN: return RK_MEAN;
    case COOT_RED_NORM1: return RK_ABSSUM;
    case COOT_RED_NORMINF: return RK_AMAX;
    case COOT_RED_VAR: return RK_VAR;
    default: return RK_SUM;
  }
}

// Kernels of a tuning module carry a "_tm" suffix, so that profiles tell tuning
// launches from the library's own.
std::string variant_name(const Expr& e, const Request& rq, int V, int E) {
  if (rq.all_variants) {
    Request plain = rq;
    plain.all_variants = false;
    return variant_name(e, plain, V, E) + "_tm";
  }
  const std::string hs = hex128(e.canon).substr(0, 16);
  if (rq.mode < 0) {
    if (rq.fam == FAM_FLAT) return "coot_flat_" + hs + "_v" + std::to_string(V) + "e" + std::to_string(E);
    return "coot_tile_" + hs + "_v" + std::to_string(V) + tile_tag(rq);
  }
  if (is_dim_kind(rq.mode) && rq.dim >= 0) {
    // the sum's stage 1 serves the mean too; a variance has its own
    const char* kind = rq.mode == COOT_RED_SUM ? "" : (rq.mode == COOT_RED_VAR_DIM ? "_var" : "_mean");
    return "coot_rdim_" + hs + "_d" + std::to_string(rq.dim) + "c" + (rq.comp ? "1" : "0") + kind + "_v" +
           std::to_string(V) + tile_tag(rq);
  }
  const std::string tag = "k" + std::to_string(red_kind(rq.mode)) + "c" + (rq.comp ? "1" : "0");
  if (rq.fam == FAM_FLAT) return "coot_rall_" + hs + "_" + tag + "_v" + std::to_string(V) + "e" + std::to_string(E);
  return "coot_rtall_" + hs + "_" + tag + "_v" + std::to_string(V) + tile_tag(rq);
}

static const char* op_fn(int c) {
  switch (c) {
    case COOT_OP_ADD: return "op_add";
    case COOT_OP_SUB: return "op_sub";
    case COOT_OP_SCHUR: return "op_mul";
    case COOT_OP_DIV: return "op_div";
    case COOT_OP_NEG: return "op_neg";
    case COOT_OP_ABS: return "op_abs";
    case COOT_OP_EXP: return "op_exp";
    case COOT_OP_LOG: return "op_log";
    case COOT_OP_SQRT: return "op_sqrt";
    case COOT_OP_SQUARE: return "op_square";
    default: return nullptr;
  }
}

// Emit the SSA statements of the body; returns the names of the last value and,
// for a binary root, of its two operands.
// leaf(i): the index into L of LOAD op i (default: the expression's own leaf
// list); sc_off: where the expression's scalars start in the scalar block.
static void emit_body(const Expr& e, std::ostringstream& os, std::string* root, std::string* lhs, std::string* rhs,
                      const std::function<int(size_t)>& leaf = nullptr, uint32_t sc_off = 0) {
  std::vector<std::string> st;
  // 16-bit storage types: every operator's binary32 result is rounded to the storage type
  const bool half = dtype_is_half(e.dtype);
  const std::string rnd_open = half ? "coot::St<S>::rnd(" : "", rnd_close = half ? ")" : "";
  int t = 0;
  for (size_t i = 0; i < e.ops.size(); ++i) {
    const coot_op& o = e.ops[i];
    std::string name = "t" + std::to_string(t++);
    if (o.code == COOT_OP_LOAD) {
      os << "    const T " << name << " = L[" << (leaf ? leaf(i) : e.op_leaf[i]) << "];\n";
      st.push_back(name);
    } else if (o.code == COOT_OP_SCALAR) {
      os << "    const T " << name << " = sc_as<T>(sc[" << o.arg + sc_off << "]);\n";
      st.push_back(name);
    } else if (o.code == COOT_OP_TRANS) {
      // index map already folded into the leaves
    } else if (o.code >= COOT_OP_ADD && o.code <= COOT_OP_DIV) {
      std::string b = st.back();
      st.pop_back();
      std::string a = st.back();
      st.pop_back();
      if (i + 1 == e.ops.size()) {
        if (lhs) *lhs = a;
        if (rhs) *rhs = b;
      }
      os << "    const T " << name << " = " << rnd_open << op_fn(o.code) << "(" << a << ", " << b << ")" << rnd_close
         << ";\n";
      st.push_back(name);
    } else {
      std::string a = st.back();
      st.pop_back();
      os << "    const T " << name << " = " << rnd_open << op_fn(o.code) << "(" << a << ")" << rnd_close << ";\n";
      st.push_back(name);
    }
  }
  *root = st.back();
}

static std::string meta_fn(const char* fname, const std::vector<int>& v) {
  std::ostringstream os;
  os << "  static constexpr __host__ __device__ int " << fname << "(int k) { return ";
  for (size_t k = 0; k < v.size(); ++k) os << "k == " << k << " ? " << v[k] << " : ";
  os << "0; }\n";
  return os.str();
}

std::string generate(const Expr& e, const Request& rq, const std::string& h, KernelNames* names) {
  std::ostringstream os;
  os << "// generated by libcoot: " << e.canon << "\n";
  if (rq.plain_store) os << "#define COOT_PLAIN_STORES 1\n";
  os << "#include \"coot_dev.h\"\n";
  os << "namespace {\n";
  os << "struct X {\n";
  // S: the storage type of the operands and the result; T: the type every operator
  // computes in (binary32 for the 16-bit types, whose results are rounded back to S)
  os << "  typedef " << dtype_cname(e.dtype) << " S;\n";
  os << "  typedef typename coot::St<S>::C T;\n";
  os << "  static constexpr int NL = " << (e.leaves.empty() ? 1 : e.leaves.size()) << ";\n";
  os << "  static constexpr int NP1 = " << e.n_p1 << ";\n";
  std::vector<int> slot, par, p1;
  int np1 = 0;
  for (auto& l : e.leaves) {
    slot.push_back((int)l.slot);
    par.push_back(l.parity);
    p1.push_back(l.parity ? np1++ : -1);
  }
  if (e.leaves.empty()) {
    slot.push_back(0);
    par.push_back(0);
    p1.push_back(-1);
  }
  os << meta_fn("slot", slot) << meta_fn("par", par) << meta_fn("p1", p1);
  std::string root, lhs, rhs;
  std::ostringstream body;
  emit_body(e, body, &root, &lhs, &rhs);
  os << "  static __device__ __forceinline__ T f(const T* L, const u64* sc) {\n";
  os << "    using namespace coot;\n" << body.str() << "    return " << root << ";\n  }\n";
  os << "  static __device__ __forceinline__ void f2(const T* L, const u64* sc, T& fa, T& fb) {\n";
  os << "    using namespace coot;\n";
  if (e.root_schur) {
    os << body.str() << "    fa = " << lhs << ";\n    fb = " << rhs << ";\n";
  } else {
    os << "    fa = f(L, sc);\n    fb = (T)1;\n";
  }
  os << "  }\n};\n}  // namespace\n";

  const std::string T = dtype_cname(e.dtype);
  const int V = rq.var.vec, E = rq.var.ept;
  const std::string TT = std::to_string(rq.var.tr) + ", " + std::to_string(rq.var.tc);  // template tile args
  const std::string comp = rq.comp ? "true" : "false";
  // kernels of an expression with exp first copy the exp table to LDS
  bool has_exp = false;
  for (auto& o : e.ops) has_exp = has_exp || o.code == COOT_OP_EXP;
  const std::string prologue = has_exp ? "coot::exp_table_to_lds<X::T>(); " : "";
  auto wrap = [&](const std::string& name, const std::string& call, int bounds) {
    os << "extern \"C\" __global__ void __launch_bounds__(" << bounds << ") " << name << "(coot_kargs a) { "
       << prologue << call << "; }\n";
  };
  const std::string hs = h.substr(0, 16);
  if (rq.all_variants) {
    // tuning module: every variant of the family (vec in {1,2,4}, and 8 for 16-bit types;
    // ept in {1,2,4,8} for flat kernels; every tile shape whose staging fits, for tiled ones)
    std::vector<std::pair<int, int>> tiles = {{0, 0}};
    if (rq.fam == FAM_TILE) {
      tiles.clear();
      for (auto& t : tile_shapes())
        if (tile_lds_bytes(e.n_p1, e.dtype, t.first, t.second) <= kTileLdsMax) tiles.push_back(t);
    }
    for (auto& t : tiles) {
      Request rt = rq;
      rt.var.tr = t.first;
      rt.var.tc = t.second;
      const std::string tt = std::to_string(t.first) + ", " + std::to_string(t.second);
      for (int v : {1, 2, 4, 8}) {
        if (v == 8 && !dtype_is_half(e.dtype)) continue;
        for (int ept : {1, 2, 4, 8}) {
          if (rq.fam == FAM_TILE && ept != 1) continue;
          if (rq.fam == FAM_TILE && v > tile_vec_cap(t.first, t.second)) continue;
          const std::string nm = variant_name(e, rt, v, rq.fam == FAM_FLAT ? ept : 0);
          std::string call;
          if (rq.mode < 0) {
            call = rq.fam == FAM_FLAT ? "coot::flat_eval<X, " + std::to_string(v) + ", " + std::to_string(ept) +
                                            (rq.stream_ld ? ", true" : ", false") + ">(a)"
                                      : "coot::tiled_eval<X, " + std::to_string(v) + ", " + tt + ">(a)";
          } else if (is_dim_kind(rq.mode) && rq.dim >= 0) {
            call = "coot::tiled_reduce_dim<X, " + std::to_string(rq.dim) + ", " + comp + ", " + std::to_string(v) +
                   ", " + tt + (rq.mode == COOT_RED_VAR_DIM ? ", true" : ", false") + ">(a)";
          } else {
            const std::string rks2 = std::to_string(red_kind(rq.mode));
            call = rq.fam == FAM_FLAT ? "coot::flat_reduce<X, " + rks2 + ", " + comp + ", " + std::to_string(v) +
                                            ", " + std::to_string(ept) + ", false>(a)"
                                      : "coot::tiled_reduce<X, " + rks2 + ", " + comp + ", " + std::to_string(v) +
                                            ", " + tt + ", false>(a)";
          }
          wrap(nm, call, rq.fam == FAM_FLAT ? 512 : 256);
          if (names->stage1.empty()) names->stage1 = nm;
        }
      }
    }
    if (is_dim_kind(rq.mode) && rq.dim >= 0) {
      // stage 2 of a reduction along dim (a variance: divided by N - 1)
      const std::string d = std::to_string(rq.dim);
      const bool var = rq.mode == COOT_RED_VAR_DIM;
      const std::string fm = rq.mode == COOT_RED_SUM ? "DM_SUM" : (var ? "DM_VAR" : "DM_MEAN");
      names->stage2 = "coot_rdfin_" + hs + "_d" + d + "c" + (rq.comp ? "1" : "0") + "_m" + std::to_string(rq.mode) +
                      "_tm";
      wrap(names->stage2, "coot::dim_stage2<X::S, " + comp + ", coot::" + fm + ">(a, " +
                              (rq.dim == 0 ? "a.n_cols, a.n_rows" : "a.n_rows, a.n_cols") + ")", 256);
    } else if (rq.mode >= 0) {
      const std::string rks2 = std::to_string(red_kind(rq.mode));
      names->stage2 = "coot_rfin_" + hs + "_k" + rks2 + "c" + (rq.comp ? "1" : "0") + "_tm";
      wrap(names->stage2, "coot::reduce_stage2<X::S, " + rks2 + ", " + comp + ", false>(a)", 256);
    }
    return os.str();
  }
  if (rq.mode < 0) {
    if (rq.fam == FAM_FLAT) {
      names->stage1 = "coot_flat_" + hs + "_v" + std::to_string(V) + "e" + std::to_string(E);
      names->stage1_fallback = "coot_flat_" + hs + "_v1e" + std::to_string(E);
      const std::string nt = rq.stream_ld ? ", true" : ", false";
      wrap(names->stage1, "coot::flat_eval<X, " + std::to_string(V) + ", " + std::to_string(E) + nt + ">(a)", 512);
      if (V != 1) wrap(names->stage1_fallback, "coot::flat_eval<X, 1, " + std::to_string(E) + nt + ">(a)", 512);
    } else {
      names->stage1 = "coot_tile_" + hs + "_v" + std::to_string(V) + tile_tag(rq);
      names->stage1_fallback = "coot_tile_" + hs + "_v1" + tile_tag(rq);
      wrap(names->stage1, "coot::tiled_eval<X, " + std::to_string(V) + ", " + TT + ">(a)", 256);
      if (V != 1) wrap(names->stage1_fallback, "coot::tiled_eval<X, 1, " + TT + ">(a)", 256);
    }
    return os.str();
  }
  if (is_dim_kind(rq.mode) && rq.dim >= 0) {
    // sum / mean / variance along dim: one stage 1 (a variance accumulates the shifted
    // moments) and a stage 2 per result (a variance: divided by N - 1, or by N)
    const bool var = rq.mode == COOT_RED_VAR_DIM;
    const std::string d = std::to_string(rq.dim);
    const std::string dc = "_d" + d + "c" + (rq.comp ? "1" : "0");
    const std::string n_out = rq.dim == 0 ? "a.n_cols" : "a.n_rows";
    const std::string cnt = rq.dim == 0 ? "a.n_rows" : "a.n_cols";
    const std::string kind = rq.mode == COOT_RED_SUM ? "" : (var ? "_var" : "_mean");
    auto inst = [&](int v) {
      return "coot::tiled_reduce_dim<X, " + d + ", " + comp + ", " + std::to_string(v) + ", " + TT +
             (var ? ", true" : ", false") + ">(a)";
    };
    auto fin = [&](const std::string& mode) {
      return "coot::dim_stage2<X::S, " + comp + ", coot::" + mode + ">(a, " + n_out + ", " + cnt + ")";
    };
    names->stage1 = "coot_rdim_" + hs + dc + kind + "_v" + std::to_string(V) + tile_tag(rq);
    names->stage1_fallback = "coot_rdim_" + hs + dc + kind + "_v1" + tile_tag(rq);
    wrap(names->stage1, inst(V), 256);
    if (V != 1) wrap(names->stage1_fallback, inst(1), 256);
    names->stage2 = "coot_rdfin_" + hs + dc + kind;
    wrap(names->stage2, fin(rq.mode == COOT_RED_SUM ? "DM_SUM" : (var ? "DM_VAR" : "DM_MEAN")), 256);
    if (var) {
      names->stage2_dev_n = names->stage2 + "n";
      wrap(names->stage2_dev_n, fin("DM_VARN"), 256);
    }
    return os.str();
  }
  // full reductions: accu / dot / norm / min / max / mean / norm1 / norm_inf / var
  const bool var = rq.mode == COOT_RED_VAR;
  const int rk = var ? (int)RK_VAR1 : red_kind(rq.mode);  // what stage 1 accumulates
  const std::string rks = std::to_string(rk);
  const std::string cs = rq.comp ? "1" : "0";
  const std::string tag = "k" + std::to_string(red_kind(rq.mode)) + "c" + cs;
  const bool flat = rq.fam == FAM_FLAT;
  const std::string pre = (flat ? "coot_rall_" : "coot_rtall_") + hs + "_";
  const std::string vs = flat ? "e" + std::to_string(E) : tile_tag(rq);
  auto inst = [&](int k, int v, bool scaled) {
    return (flat ? "coot::flat_reduce<X, " : "coot::tiled_reduce<X, ") + std::to_string(k) + ", " + comp + ", " +
           std::to_string(v) + ", " + (flat ? std::to_string(E) : TT) + ", " + (scaled ? "true" : "false") + ">(a)";
  };
  const int bounds = flat ? 512 : 256;
  auto fin = [&](int k) { return "coot::reduce_stage2<X::S, " + std::to_string(k) + ", " + comp + ", false>(a)"; };
  names->stage1 = pre + tag + "_v" + std::to_string(V) + vs;
  names->stage1_fallback = pre + tag + "_v1" + vs;
  wrap(names->stage1, inst(rk, V, false), bounds);
  if (V != 1) wrap(names->stage1_fallback, inst(rk, 1, false), bounds);
  names->stage2 = "coot_rfin_" + hs + "_" + tag;
  wrap(names->stage2, fin(var ? (int)RK_VAR : rk), 256);
  if (rk == RK_SUMSQ) {
    names->stage1_rescale = pre + tag + "_rescale";
    wrap(names->stage1_rescale, inst(rk, 1, true), bounds);
    names->stage2_rescale = names->stage2 + "_rescale";
    wrap(names->stage2_rescale, "coot::reduce_stage2<X::S, " + rks + ", " + comp + ", true>(a)", 256);
  }
  if (var) {
    // the same records divided by N instead of N - 1
    names->stage2_dev_n = "coot_rfin_" + hs + "_k" + std::to_string((int)RK_VARN) + "c" + cs;
    wrap(names->stage2_dev_n, fin(RK_VARN), 256);
  }
  return os.str();
}

// Two statements in one pass: out = e(leaves) and a full reduction of r, whose
// operand slot k reads e's leaf of operand r_src[k] (the value loaded before the
// store) or, for r_src[k] = -1, the value just computed.  Both are flat (leaves
// untransposed and contiguous).  Struct X is e; struct Z is r over e's leaves with
// the computed value appended (L[X::NL]); r's scalars follow e's.
std::string generate_pair(const Expr& e, const Expr& r, const std::vector<int>& r_src, int kind, const Request& rq,
                          const std::string& h, KernelNames* names) {
  std::ostringstream os;
  os << "// generated by libcoot: " << e.canon << " ; then " << r.canon << "\n";
  os << "#include \"coot_dev.h\"\n";
  os << "namespace {\n";
  auto head = [&](const char* nm, size_t nl) {
    os << "struct " << nm << " {\n";
    os << "  typedef " << dtype_cname(e.dtype) << " S;\n";
    os << "  typedef typename coot::St<S>::C T;\n";
    os << "  static constexpr int NL = " << nl << ";\n";
    os << "  static constexpr int NP1 = 0;\n";
  };
  std::vector<int> slot, par, p1;
  for (auto& l : e.leaves) {
    slot.push_back((int)l.slot);
    par.push_back(0);
    p1.push_back(-1);
  }
  head("X", e.leaves.size());
  os << meta_fn("slot", slot) << meta_fn("par", par) << meta_fn("p1", p1);
  std::string root, lhs, rhs;
  std::ostringstream body;
  emit_body(e, body, &root, &lhs, &rhs);
  os << "  static __device__ __forceinline__ T f(const T* L, const u64* sc) {\n";
  os << "    using namespace coot;\n" << body.str() << "    return " << root << ";\n  }\n};\n";
  // r's LOAD op i reads slot s: e's leaf of operand r_src[s], or the computed value
  auto leaf_of = [&](size_t i) -> int {
    const int src = r_src[r.ops[i].arg];
    if (src < 0) return (int)e.leaves.size();
    for (size_t k = 0; k < e.leaves.size(); ++k)
      if ((int)e.leaves[k].slot == src) return (int)k;
    fail(COOT_EUNSUPPORTED, "the reduction reads an operand the evaluated expression does not read");
  };
  head("Z", e.leaves.size() + 1);
  std::string rroot, rlhs, rrhs;
  std::ostringstream rbody;
  emit_body(r, rbody, &rroot, &rlhs, &rrhs, leaf_of, e.n_scalars);
  os << "  static __device__ __forceinline__ T f(const T* L, const u64* sc) {\n";
  os << "    using namespace coot;\n" << rbody.str() << "    return " << rroot << ";\n  }\n";
  os << "  static __device__ __forceinline__ void f2(const T* L, const u64* sc, T& fa, T& fb) {\n";
  os << "    using namespace coot;\n";
  if (r.root_schur) {
    os << rbody.str() << "    fa = " << rlhs << ";\n    fb = " << rrhs << ";\n";
  } else {
    os << "    fa = f(L, sc);\n    fb = (T)1;\n";
  }
  os << "  }\n};\n}  // namespace\n";
  bool has_exp = false;
  for (auto& o : e.ops) has_exp = has_exp || o.code == COOT_OP_EXP;
  for (auto& o : r.ops) has_exp = has_exp || o.code == COOT_OP_EXP;
  const std::string prologue = has_exp ? "coot::exp_table_to_lds<X::T>(); " : "";
  auto wrap = [&](const std::string& name, const std::string& call, int bounds) {
    os << "extern \"C\" __global__ void __launch_bounds__(" << bounds << ") " << name << "(coot_kargs a) { "
       << prologue << call << "; }\n";
  };
  const int V = rq.var.vec, E = rq.var.ept;
  const std::string comp = rq.comp ? "true" : "false";
  const std::string rks = std::to_string(red_kind(kind));
  const std::string hs = h.substr(0, 16), tag = "k" + rks + "c" + (rq.comp ? "1" : "0");
  auto inst = [&](int v) {
    return "coot::flat_eval_reduce<X, Z, " + rks + ", " + comp + ", " + std::to_string(v) + ", " + std::to_string(E) +
           ">(a)";
  };
  names->stage1 = "coot_fer_" + hs + "_" + tag + "_v" + std::to_string(V) + "e" + std::to_string(E);
  names->stage1_fallback = "coot_fer_" + hs + "_" + tag + "_v1e" + std::to_string(E);
  names->stage2 = "coot_ferfin_" + hs + "_" + tag;
  wrap(names->stage1, inst(V), 512);
  if (V != 1) wrap(names->stage1_fallback, inst(1), 512);
  wrap(names->stage2, "coot::reduce_stage2<X::S, " + rks + ", " + comp + ", false>(a)", 256);
  return os.str();
}

}  // namespace coot
