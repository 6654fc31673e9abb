// Internal declarations of libcoot (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "coot.h"

namespace coot {

constexpr int kMaxSlots = 16;
constexpr int kMaxScalars = 32;

// Host mirror of the device-side coot_kargs (coot_dev.h); layouts must agree.
struct KArgs {
  const void* leaf[kMaxSlots];
  int64_t ld[kMaxSlots];
  uint64_t sc[kMaxScalars];
  void* out;
  int64_t out_ld;
  int64_t n_rows, n_cols;
  void* ws;
  void* ws2;
  int64_t n_part;
};
static_assert(sizeof(KArgs) == 16 * 8 + 16 * 8 + 32 * 8 + 7 * 8, "kernel argument block layout");

struct Error : std::runtime_error {
  coot_status code;
  Error(coot_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};
[[noreturn]] void fail(coot_status c, const std::string& msg);
void hip_check(hipError_t e, const char* what);

size_t dtype_size(int dt);
const char* dtype_cname(int dt);  // C type used in generated code
bool dtype_is_int(int dt);
bool dtype_is_half(int dt);  // f16 / bf16: 16-bit storage, binary32 arithmetic

// A leaf is an (operand slot, transpose parity) pair; repeated loads of the same
// pair share one leaf.
struct Leaf {
  uint32_t slot;
  uint8_t parity;
};

// Validated expression (the analysis of Section 3's whole-expression view).
struct Expr {
  std::vector<coot_op> ops;
  std::vector<coot_slot_type> slots;
  uint32_t n_scalars = 0;
  uint32_t flags = 0;
  int dtype = COOT_F32;
  std::vector<Leaf> leaves;
  std::vector<int> op_leaf;     // per op: leaf index for LOAD, -1 otherwise
  std::vector<int> op_parity;   // per op: transpose parity of the op's value
  int n_p1 = 0;                 // number of parity-1 leaves
  bool root_schur = false;      // root is a Schur product (dot pattern)
  bool scalar_only = false;     // no LOAD at all
  std::string canon;            // canonical text (the signature body)
  uint64_t uid = 0;             // unique per analysed expression (never reused)
  // per-request kernel cache: request key -> module-level kernel handles
  std::mutex mu;
  std::map<std::string, std::shared_ptr<struct Module>> reqs;
  // The last fused evaluation's launch (kernel, grid, block, arguments without the
  // scalars): validation and planning depend only on the operands, the output and the
  // configuration, so a call repeating all three reuses it (under mu).
  struct EvalMemo {
    bool valid = false;
    std::vector<coot_operand> ops;
    coot_operand out{};
    coot_launch_cfg cfg{};
    bool has_cfg = false, plain = false;
    hipFunction_t f = nullptr;
    unsigned grid = 0, block = 0;
    KArgs a{};
  } memo;
  // The same for the last statement pair (eval_reduce) led by this expression: the
  // second statement's uid, operand map, kind and output, and the two launches.
  struct PairMemo {
    bool valid = false;
    std::vector<coot_operand> ops;
    coot_operand out{}, r_out{};
    uint64_t r_uid = 0;
    std::vector<int32_t> r_src;
    int kind = 0;
    coot_launch_cfg cfg{};
    bool has_cfg = false;
    hipFunction_t f1 = nullptr, f2 = nullptr;
    unsigned grid = 0, block = 0;
    KArgs a{};
  } pair_memo;
};

// Analysis
std::unique_ptr<Expr> analyse(const coot_op* ops, uint32_t n_ops, const coot_slot_type* slots, uint32_t n_slots,
                              uint32_t n_scalars, uint32_t flags);
void infer_shape(const Expr& e, const coot_operand* operands, int64_t* rows, int64_t* cols);
void check_operands(const Expr& e, const coot_operand* operands);
uint64_t scalar_bits(double v, int dtype);

// Code generation ------------------------------------------------------------
enum Family { FAM_FLAT = 0, FAM_TILE = 1 };
// reduction kinds of the generated kernels (the same numbers as in coot_dev.h)
enum RedKind {
  RK_SUM = 0, RK_DOT = 1, RK_SUMSQ = 2, RK_ABSSUM = 3, RK_MAX = 4, RK_MIN = 5, RK_AMAX = 6, RK_MEAN = 7,
  RK_VAR1 = 8, RK_VAR = 10, RK_VARN = 11
};
// reductions along a dimension (dim 0 or 1): sum, mean, variance
inline bool is_dim_kind(int kind) { return kind == COOT_RED_SUM || kind == COOT_RED_MEAN_DIM || kind == COOT_RED_VAR_DIM; }
// the kernel kind of a full reduction mode (accu, dot, norm, min, max, mean, norm1, norm_inf)
int red_kind(int mode);
// a reduction mode's arguments are valid for this expression (fails with the reason)
void check_red_mode(const Expr& e, int mode);

// Tiles of the tiled families: tr x tc output elements (rows x columns), 256 threads.
// The tr / V threads of a column segment times tc columns must cover the 256 threads
// (V <= tr * tc / 256); V divides both edges.  Edges are powers of two in [8, 256]
// with 1024 <= tr * tc <= 8192 (4 to 32 elements per thread).
inline int tile_vec_cap(int tr, int tc) { return tr * tc / 256; }
bool tile_shape_ok(int tr, int tc);
// The library's tile (rows x columns) for a request that gives none.
// n: elements of the expression's shape (the output of an element-wise evaluation)
void default_tile(const Expr& e, int mode, int dim, int64_t n, int* tr, int* tc);
// LDS bytes the staged transposed leaves of a tile take (compute-type elements, one
// padded tr x (tc + 1) tile per transposed leaf); the library keeps this <= 64 KiB.
size_t tile_lds_bytes(int n_p1, int dtype, int tr, int tc);
constexpr size_t kTileLdsMax = 65536;
// Flat evaluations whose operands exceed this many bytes together load them
// non-temporally: the MI355X's Infinity Cache holds 256 MiB.
constexpr size_t kStreamLoadBytes = size_t(256) << 20;
// Tile shapes the autotuner tries (those whose staging fits kTileLdsMax).
const std::vector<std::pair<int, int>>& tile_shapes();

struct Variant {  // compile-time parameters of one kernel instance
  int vec = 4;
  int ept = 4;     // flat families
  int tr = 64;     // tiled families: tile rows
  int tc = 64;     //                 tile columns
};

struct Request {
  int mode = -1;      // -1 eval, else coot_red
  int dim = -1;       // dim of SUM / MEAN_DIM / VAR_DIM
  bool comp = true;   // compensated reduction
  Family fam = FAM_FLAT;
  Variant var;
  bool all_variants = false;  // tuning module: every vec x ept (flat) or vec (tiled) variant
  bool plain_store = false;   // results stored with plain (cached) stores: the unfused comparator's temporaries
  bool stream_ld = false;     // flat evaluation: non-temporal leaf loads (operands beyond the Infinity Cache)
  std::string key() const;
};

// Kernel name of one variant (the naming convention codegen uses); the tile is rq.var's.
std::string variant_name(const Expr& e, const Request& rq, int vec, int ept);

struct KernelNames {
  std::string stage1, stage1_fallback, stage2, stage1_rescale, stage2_rescale;
  // a variance's stage 2 dividing by N (stage2 divides by N - 1)
  std::string stage2_dev_n;
};

std::string generate(const Expr& e, const Request& rq, const std::string& hash_hint, KernelNames* names);
// out = e and a full reduction of r in one pass (r_src: r's slots -> e's operands, -1 = the result)
std::string generate_pair(const Expr& e, const Expr& r, const std::vector<int>& r_src, int kind, const Request& rq,
                          const std::string& hash_hint, KernelNames* names);
const std::vector<std::pair<std::string, std::string>>& device_headers();

// JIT + caches -----------------------------------------------------------------
struct Module {
  hipModule_t mod = nullptr;
  std::map<std::string, hipFunction_t> fns;
  KernelNames names;
  std::vector<char> code;   // code object (kept when not loaded, e.g. compile-only)
  bool loaded = false;
  int device = 0;           // the device it is loaded on
  hipFunction_t fn(const std::string& name);
  ~Module();  // hands a loaded module to the unload queue (coot_cache_trim)
};
// Module cache: out[0] modules cached, out[1] the cap, out[2] evictions so far,
// out[3] modules waiting to be unloaded.
void cache_info(int64_t out[4]);
// Synchronises the device and unloads every module no expression holds any more;
// returns how many.
int64_t cache_trim();

// Compile (or fetch) the module for a request; load it on the current device
// unless load == false (compile-only, used where no device exists).
std::shared_ptr<Module> get_module(Expr& e, const Request& rq, bool load);
// The module of a request only if it is loaded on a device already (this expression's
// cache, then the process-wide one); COOT_EINVAL otherwise.  Never compiles or loads.
std::shared_ptr<Module> find_loaded_module(Expr& e, const Request& rq);
std::shared_ptr<Module> get_module_pair(Expr& e, const Expr& r, const std::vector<int>& r_src, int kind,
                                        const Request& rq, bool load);
std::string compile_source(const std::string& src, const std::string& name_hint, std::vector<char>* code);
std::string hex128(const std::string& text);

struct Stats {
  double compiles = 0, mem_hits = 0, disk_hits = 0, launches = 0, compile_ms = 0;
};
Stats& stats();
std::mutex& global_mutex();

// Device / workspace ------------------------------------------------------------
int num_cus();
// Device memory of workspaces and temporaries: the caller's allocator
// (coot_set_allocator) or hipMalloc / hipFree; each buffer remembers which.
struct DevAllocator {
  void* (*alloc)(size_t, void*, void*) = nullptr;
  void (*dealloc)(void*, void*, void*) = nullptr;
  void* ctx = nullptr;
};
void* dev_alloc(size_t bytes, hipStream_t s, DevAllocator* used);
void dev_free(void* p, hipStream_t s, const DevAllocator& used);
void set_allocator(const DevAllocator& a);
void* workspace(size_t bytes, hipStream_t s, int which);
// Calls that take workspace or temporaries refuse a stream under capture: the
// library may free or hand out those buffers again after the call returns, which a
// replayed graph would not see (COOT_EUNSUPPORTED).
void reject_capture(hipStream_t s, const char* call);
void* temp_alloc(size_t bytes, hipStream_t s);
void temp_free(void* p, size_t bytes, hipStream_t s);

// Execution ---------------------------------------------------------------------
void launch(hipFunction_t f, unsigned grid, unsigned block, const KArgs& args, hipStream_t s);
// plain_store: the kernel stores its result with plain stores (kept in L2 and the
// Infinity Cache for a kernel that reads it next), as the unfused comparator does
void eval_fused(Expr& e, const coot_operand* ops, const double* scalars, const coot_operand& out,
                const coot_launch_cfg* cfg, hipStream_t s, bool plain_store = false);
void eval_unfused(Expr& e, const coot_operand* ops, const double* scalars, const coot_operand& out,
                  const coot_launch_cfg* cfg, hipStream_t s);
void eval_reduce(Expr& e, const coot_operand* ops, const double* scalars, const coot_operand& out, Expr& r,
                 const int32_t* r_src, const double* r_scalars, int kind, const coot_operand& r_out,
                 const coot_launch_cfg* cfg, hipStream_t s);
// Launch geometry of a reduction along a dimension: the reduced dimension's tiles cut
// into n_part segments (K tiles each, K growing once there are more than per_cu tiles
// per CU, at most 16), one workgroup per (segment, output strip); part_bytes of
// float-float partials (compute type of cs bytes) per partial array.
struct DimPlan {
  int64_t n_out = 0, n_part = 1, nseg = 0;
  size_t part_bytes = 0;
};
DimPlan dim_plan(int64_t R, int64_t C, int dim, int tile_r, int tile_c, int per_cu, size_t cs);
// Stage 1 over p.nseg workgroups (none when empty), then stage 2, one wavefront per output.
void launch_dim(hipFunction_t stage1, hipFunction_t stage2, KArgs& a, const DimPlan& p, hipStream_t s);
// Partial-result buffers of a reduction given by the caller (the allocation-free entry
// point): two halves of `bytes` / 2, the first in place of workspace 0, the second of
// workspace 1.  With one, reduce_fused allocates nothing and compiles nothing (the
// kernels must be loaded already: COOT_EINVAL otherwise).
struct Scratch {
  void* p = nullptr;
  size_t bytes = 0;
};
void reduce_fused(Expr& e, const coot_operand* ops, const double* scalars, int kind, int dim, uint32_t flags,
                  const coot_operand& out, const coot_launch_cfg* cfg, hipStream_t s, const Scratch* sc = nullptr);
// The device scratch array of coot_reduce_noalloc: kNoallocScratchBytes on every
// device the library runs on, its address looked up once per device (current device).
constexpr size_t kNoallocScratchBytes = COOT_NOALLOC_SCRATCH_BYTES;
void* noalloc_scratch();
// The library's launch configuration for a family when the caller gives none
// (fields 0 there are filled from it); waves and ept are 0/unused where fixed.
constexpr int64_t kStreamElems = int64_t(1) << 24;  // larger flat launches take the streaming defaults
constexpr int64_t kTileLargeElems = int64_t(1) << 22;  // from here tiled launches default to 64 x 64
coot_launch_cfg default_cfg(int fam, int mode, int dim, int dtype, int64_t n);
Request plan(const Expr& e, const coot_operand* ops, const coot_operand* out, int mode, int dim, bool comp,
             const coot_launch_cfg* cfg);

int64_t ld_of(const coot_operand& o);
// COOT_EALIAS unless every operand that overlaps `out` is read untransposed with
// out's own layout (the same base, leading dimension and dims)
void check_alias(const Expr& e, const coot_operand* ops, const coot_operand& out, size_t es);
bool vec_ok(const Expr& e, const Request& rq, const coot_operand* ops, const coot_operand* out, int64_t R, int64_t C);
void fill_args(const Expr& e, const coot_operand* ops, const double* scalars, KArgs* a);
unsigned flat_grid(int64_t n, int V, int E, int bs, int gm);
unsigned tile_grid(int64_t R, int64_t C, int tr, int tc, int gm);

// Thread-local message behind coot_last_error().
std::string& last_error();

// Run f, mapping exceptions to a status and the thread's last-error message.
template <typename F>
coot_status guarded(F&& f) {
  try {
    last_error().clear();
    f();
    return COOT_OK;
  } catch (const Error& e) {
    last_error() = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    last_error() = "host allocation failed";
    return COOT_ENOMEM;
  } catch (const std::exception& e) {
    last_error() = e.what();
    return COOT_EINVAL;
  }
}

}  // namespace coot

// Library-owned expression handle (coot.h's opaque coot_expr).
struct coot_expr {
  std::unique_ptr<coot::Expr> e;
};
