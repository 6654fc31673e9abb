// Runtime compilation and the kernel cache.
//
// Section 4 of the paper: the kernel set is compiled at run time for the device
// found and cached, so the cost is paid once.  Here every (expression
// signature, request) gets its own module: hipRTC compiles the generated source
// for gfx950, the code object is kept in memory (process-wide map keyed by a
// 128-bit hash of source + options + compiler version, least recently used entries
// evicted past a cap) and on disk
// (COOT_CACHE_DIR, default ~/.cache/coot; a header with magic, key and checksum
// guards every file, and a bad file is simply recompiled).
#include <hip/hiprtc.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <list>
#include <unordered_map>

#include "core.h"

namespace coot {

Stats& stats() {
  static Stats s;
  return s;
}
std::mutex& global_mutex() {
  static std::mutex m;
  return m;
}

static uint64_t fnv1a(const std::string& s, uint64_t seed) {
  uint64_t h = 1469598103934665603ull ^ seed;
  for (unsigned char c : s) {
    h ^= c;
    h *= 1099511628211ull;
  }
  return h;
}

std::string hex128(const std::string& text) {
  char buf[40];
  std::snprintf(buf, sizeof buf, "%016llx%016llx", (unsigned long long)fnv1a(text, 0),
                (unsigned long long)fnv1a(text, 0x9e3779b97f4a7c15ull));
  return buf;
}

static const std::vector<std::string>& rtc_options() {
  static const std::vector<std::string> o = {
      "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
      "-fhip-fp32-correctly-rounded-divide-sqrt", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  return o;
}

static std::string rtc_version() {
  int ma = 0, mi = 0;
  hiprtcVersion(&ma, &mi);
  return std::to_string(ma) + "." + std::to_string(mi);
}

std::string compile_source(const std::string& src, const std::string& name_hint, std::vector<char>* code) {
  hiprtcProgram prog;
  std::vector<const char*> hdrs, hdr_names;
  for (auto& h : device_headers()) {
    hdr_names.push_back(h.first.c_str());
    hdrs.push_back(h.second.c_str());
  }
  if (hiprtcCreateProgram(&prog, src.c_str(), (name_hint + ".hip").c_str(), (int)hdrs.size(), hdrs.data(),
                          hdr_names.data()) != HIPRTC_SUCCESS)
    fail(COOT_ECOMPILE, "hiprtcCreateProgram failed");
  std::vector<const char*> opts;
  for (auto& s : rtc_options()) opts.push_back(s.c_str());
  if (const char* extra = std::getenv("COOT_HIPRTC_EXTRA")) opts.push_back(extra);
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
  size_t log_size = 0;
  hiprtcGetProgramLogSize(prog, &log_size);
  std::string log(log_size, '\0');
  if (log_size) hiprtcGetProgramLog(prog, &log[0]);
  if (r != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&prog);
    fail(COOT_ECOMPILE, "hipRTC compilation failed for " + name_hint + ":\n" + log);
  }
  size_t n = 0;
  hiprtcGetCodeSize(prog, &n);
  code->resize(n);
  hiprtcGetCode(prog, code->data());
  hiprtcDestroyProgram(&prog);
  return log;
}

// ---- disk cache ------------------------------------------------------------
static std::string cache_dir() {
  if (const char* d = std::getenv("COOT_CACHE_DIR")) return d;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/coot";
}

static void mkdirs(const std::string& p) {
  std::string cur;
  for (size_t i = 0; i < p.size(); ++i) {
    cur += p[i];
    if (p[i] == '/' && cur.size() > 1) mkdir(cur.c_str(), 0755);
  }
  mkdir(p.c_str(), 0755);
}

struct DiskHeader {
  char magic[8];
  char key[32];
  uint64_t size;
  uint64_t check;
};

static bool disk_load(const std::string& key, std::vector<char>* code) {
  if (std::getenv("COOT_NO_DISK_CACHE")) return false;
  std::ifstream f(cache_dir() + "/" + key + ".co", std::ios::binary);
  if (!f) return false;
  DiskHeader h;
  if (!f.read(reinterpret_cast<char*>(&h), sizeof h)) return false;
  if (std::memcmp(h.magic, "COOTCO1", 8) != 0 || std::memcmp(h.key, key.data(), 32) != 0) return false;
  if (h.size == 0 || h.size > (64u << 20)) return false;
  std::vector<char> buf(h.size);
  if (!f.read(buf.data(), (std::streamsize)h.size)) return false;
  if (fnv1a(std::string(buf.data(), buf.size()), 7) != h.check) return false;
  code->swap(buf);
  return true;
}

static void disk_store(const std::string& key, const std::vector<char>& code) {
  if (std::getenv("COOT_NO_DISK_CACHE")) return;
  const std::string dir = cache_dir();
  mkdirs(dir);
  DiskHeader h;
  std::memcpy(h.magic, "COOTCO1", 8);
  std::memcpy(h.key, key.data(), 32);
  h.size = code.size();
  h.check = fnv1a(std::string(code.data(), code.size()), 7);
  const std::string tmp = dir + "/" + key + ".co.tmp" + std::to_string(getpid());
  {
    std::ofstream f(tmp, std::ios::binary);
    if (!f) return;
    f.write(reinterpret_cast<const char*>(&h), sizeof h);
    f.write(code.data(), (std::streamsize)code.size());
    if (!f) return;
  }
  std::rename(tmp.c_str(), (dir + "/" + key + ".co").c_str());
}

// ---- module cache ------------------------------------------------------------
hipFunction_t Module::fn(const std::string& name) {
  std::lock_guard<std::mutex> g(global_mutex());
  auto it = fns.find(name);
  if (it != fns.end()) return it->second;
  if (!loaded) fail(COOT_EHIP, "module not loaded on a device");
  hipFunction_t f = nullptr;
  hip_check(hipModuleGetFunction(&f, mod, name.c_str()), "hipModuleGetFunction");
  fns[name] = f;
  return f;
}

// Process-wide modules by key, least recently used evicted past `cap` entries
// (COOT_MODULE_CACHE, default 1024).  An evicted module stays alive while an
// expression still holds it; once none does, its device code waits in `graveyard`
// until coot_cache_trim unloads it after a device synchronisation (a kernel of it may
// still be queued when its last holder goes).  Members are used under global_mutex.
struct ModuleCache {
  std::list<std::string> order;  // most recently used first
  std::unordered_map<std::string, std::pair<std::shared_ptr<Module>, std::list<std::string>::iterator>> map;
  size_t cap = 1024;
  double evictions = 0;
};
static ModuleCache& module_cache() {
  static ModuleCache* c = [] {
    auto* mc = new ModuleCache;  // never destroyed: modules may outlive static destruction order
    if (const char* v = std::getenv("COOT_MODULE_CACHE")) {
      const long n = std::strtol(v, nullptr, 10);
      if (n > 0) mc->cap = (size_t)n;
    }
    return mc;
  }();
  return *c;
}
static std::shared_ptr<Module> cache_find(const std::string& key) {
  ModuleCache& c = module_cache();
  auto it = c.map.find(key);
  if (it == c.map.end()) return nullptr;
  c.order.splice(c.order.begin(), c.order, it->second.second);
  return it->second.first;
}
static void cache_put(const std::string& key, const std::shared_ptr<Module>& m) {
  ModuleCache& c = module_cache();
  c.order.push_front(key);
  c.map[key] = {m, c.order.begin()};
  while (c.map.size() > c.cap) {
    c.map.erase(c.order.back());
    c.order.pop_back();
    c.evictions += 1;
  }
}

static std::mutex& graveyard_mutex() {
  static std::mutex* m = new std::mutex;
  return *m;
}
static std::vector<std::pair<int, hipModule_t>>& graveyard() {  // (device, module)
  static auto* v = new std::vector<std::pair<int, hipModule_t>>;
  return *v;
}

Module::~Module() {
  if (loaded && mod) {
    std::lock_guard<std::mutex> g(graveyard_mutex());
    graveyard().push_back({device, mod});
  }
}

void cache_info(int64_t out[4]) {
  std::lock_guard<std::mutex> g(global_mutex());
  const ModuleCache& c = module_cache();
  out[0] = (int64_t)c.map.size();
  out[1] = (int64_t)c.cap;
  out[2] = (int64_t)c.evictions;
  std::lock_guard<std::mutex> g2(graveyard_mutex());
  out[3] = (int64_t)graveyard().size();
}

int64_t cache_trim() {
  std::vector<std::pair<int, hipModule_t>> dead;
  {
    std::lock_guard<std::mutex> g(graveyard_mutex());
    dead.swap(graveyard());
  }
  if (dead.empty()) return 0;
  std::sort(dead.begin(), dead.end());
  int cur = 0;
  hip_check(hipGetDevice(&cur), "hipGetDevice");
  for (size_t i = 0; i < dead.size(); ++i) {
    if (i == 0 || dead[i].first != dead[i - 1].first) {  // each device that holds some: drained first
      hip_check(hipSetDevice(dead[i].first), "hipSetDevice");
      hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    }
    hip_check(hipModuleUnload(dead[i].second), "hipModuleUnload");
  }
  hip_check(hipSetDevice(cur), "hipSetDevice");
  return (int64_t)dead.size();
}

// The module of one generated source, cached under the request key `rk` of `owner`
// (in memory per expression, then by the source's hash process-wide and on disk).
static std::shared_ptr<Module> module_for(Expr& e, const std::string& rk, const std::string& src,
                                          const KernelNames& names, bool load);

std::shared_ptr<Module> get_module(Expr& e, const Request& rq, bool load) {
  const std::string rk = rq.key();
  {
    std::lock_guard<std::mutex> g(e.mu);
    auto it = e.reqs.find(rk);
    if (it != e.reqs.end() && (it->second->loaded || !load)) return it->second;
  }
  KernelNames names;
  const std::string src = generate(e, rq, hex128(e.canon), &names);
  return module_for(e, rk, src, names, load);
}

// Module key of a generated source: the source, the hipRTC options and version, the
// device headers.
static std::string module_key(const std::string& src) {
  std::string opt_text;
  for (auto& o : rtc_options()) opt_text += o + " ";
  if (const char* extra = std::getenv("COOT_HIPRTC_EXTRA")) opt_text += std::string("extra:") + extra;
  std::string hdr_text;
  for (auto& h : device_headers()) hdr_text += h.second;
  return hex128(src + "\n" + opt_text + rtc_version() + hex128(hdr_text));
}

std::shared_ptr<Module> find_loaded_module(Expr& e, const Request& rq) {
  const std::string rk = rq.key();
  {
    std::lock_guard<std::mutex> g(e.mu);
    auto it = e.reqs.find(rk);
    if (it != e.reqs.end() && it->second->loaded) return it->second;
  }
  KernelNames names;
  const std::string key = module_key(generate(e, rq, hex128(e.canon), &names));
  std::shared_ptr<Module> m;
  {
    std::lock_guard<std::mutex> g(global_mutex());
    m = cache_find(key);
    if (m && !m->loaded) m = nullptr;
  }
  if (!m)
    fail(COOT_EINVAL, "the kernels of this reduction are not loaded: run coot_expr_prepare or coot_reduce "
                      "with the same expression, kind and operand layout once first");
  std::lock_guard<std::mutex> g2(e.mu);
  e.reqs[rk] = m;
  return m;
}

std::shared_ptr<Module> get_module_pair(Expr& e, const Expr& r, const std::vector<int>& r_src, int kind,
                                        const Request& rq, bool load) {
  std::string rk = "pair:" + rq.key() + "|" + r.canon + "|" + std::to_string(kind) + "|";
  for (int v : r_src) rk += std::to_string(v) + ",";
  {
    std::lock_guard<std::mutex> g(e.mu);
    auto it = e.reqs.find(rk);
    if (it != e.reqs.end() && (it->second->loaded || !load)) return it->second;
  }
  KernelNames names;
  const std::string src = generate_pair(e, r, r_src, kind, rq, hex128(rk + e.canon), &names);
  return module_for(e, rk, src, names, load);
}

static std::shared_ptr<Module> module_for(Expr& e, const std::string& rk, const std::string& src,
                                          const KernelNames& names, bool load) {
  const std::string key = module_key(src);
  std::shared_ptr<Module> m;
  {
    std::lock_guard<std::mutex> g(global_mutex());
    m = cache_find(key);
    if (m) stats().mem_hits += 1;
  }
  if (!m) {
    // compile without holding the global lock so that several host threads can compile at once
    auto fresh = std::make_shared<Module>();
    fresh->names = names;
    bool from_disk = disk_load(key, &fresh->code);
    double ms = 0;
    if (!from_disk) {
      auto t0 = std::chrono::steady_clock::now();
      compile_source(src, names.stage1, &fresh->code);
      auto t1 = std::chrono::steady_clock::now();
      ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
      disk_store(key, fresh->code);
    }
    std::lock_guard<std::mutex> g(global_mutex());
    m = cache_find(key);  // another thread may have finished first
    if (!m) {
      m = fresh;
      cache_put(key, m);
    }
    if (from_disk) stats().disk_hits += 1;
    else {
      stats().compiles += 1;
      stats().compile_ms += ms;
    }
  }
  if (load) {
    std::lock_guard<std::mutex> g(global_mutex());
    if (!m->loaded) {
      hip_check(hipModuleLoadData(&m->mod, m->code.data()), "hipModuleLoadData");
      hip_check(hipGetDevice(&m->device), "hipGetDevice");
      m->loaded = true;
    }
  }
  std::lock_guard<std::mutex> g2(e.mu);
  e.reqs[rk] = m;
  return m;
}

}  // namespace coot
