// Runtime-generated kernels and their code cache.
//
// The paper compiles each method tree it materialises, caching the compiled
// code under the tree's signature so that later trees of the same shape
// reuse it (Section III-C).  Here a generated HIP source is compiled for the
// device with hipRTC, loaded as a module and kept in memory under its key;
// the code object is also written to a directory (NBGRB_CODE_CACHE, else
// $HOME/.cache/nbgrb) under a hash of the key and the compiler options, so a
// later process loads it without compiling.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <sys/stat.h>
#include <unistd.h>
#include <vector>

#include "runtime.h"

namespace nbgrb {

namespace {

const char* const kOptions[] = {"--offload-arch=gfx950", "-O3", "-ffp-contract=off", "-Xclang", "-target-feature",
                                "-Xclang", "-packed-fp32-ops"};
constexpr int kNumOptions = sizeof(kOptions) / sizeof(kOptions[0]);

struct Loaded {
  hipModule_t module = nullptr;
  hipFunction_t fn = nullptr;
};

std::map<std::string, Loaded>& loaded() {
  static std::map<std::string, Loaded> m;
  return m;
}

uint64_t fnv1a(const std::string& s, uint64_t h = 1469598103934665603ull) {
  for (unsigned char ch : s) {
    h ^= ch;
    h *= 1099511628211ull;
  }
  return h;
}

std::string cache_dir() {
  if (const char* d = std::getenv("NBGRB_CODE_CACHE")) return d;
  if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/nbgrb";
  return "";
}

bool make_dirs(const std::string& path) {
  if (path.empty()) return false;
  std::string cur;
  std::stringstream ss(path);
  std::string part;
  if (path[0] == '/') cur = "/";
  while (std::getline(ss, part, '/')) {
    if (part.empty()) continue;
    cur += part + "/";
    if (mkdir(cur.c_str(), 0755) != 0 && errno != EEXIST) return false;
  }
  return true;
}

std::vector<char> read_file(const std::string& path) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return {};
  return std::vector<char>((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
}

void write_file_atomic(const std::string& path, const std::vector<char>& data) {
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream f(tmp, std::ios::binary);
    if (!f) return;
    f.write(data.data(), (std::streamsize)data.size());
    if (!f) return;
  }
  std::rename(tmp.c_str(), path.c_str());
}

std::vector<char> compile(const std::string& source, const std::string& name) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, source.c_str(), (name + ".hip").c_str(), 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    fail(GrB_PANIC, "hipRTC: cannot create program");
  const hiprtcResult r = hiprtcCompileProgram(prog, kNumOptions, kOptions);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    hiprtcDestroyProgram(&prog);
    fail(GrB_PANIC, "hipRTC compile failed: " + log);
  }
  size_t n = 0;
  hiprtcGetCodeSize(prog, &n);
  std::vector<char> code(n);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  return code;
}

}  // namespace

hipFunction_t jit_kernel(const std::string& key, const std::string& source, const char* name) {
  Ctx& c = ctx();
  auto& m = loaded();
  auto it = m.find(key);
  if (it != m.end()) {
    c.stats.jit_memory_hits++;
    return it->second.fn;
  }
  std::string opts;
  for (int i = 0; i < kNumOptions; ++i) opts += std::string(kOptions[i]) + " ";
  char hex[17];
  std::snprintf(hex, sizeof(hex), "%016llx", (unsigned long long)fnv1a(source, fnv1a(opts + "|" + key)));
  const std::string dir = cache_dir();
  const std::string path = dir.empty() ? "" : dir + "/" + name + "-" + hex + ".co";
  // the cached object is used only if the source stored beside it is this one
  const std::string stamp = opts + "\n" + source;
  std::vector<char> code;
  if (!path.empty()) {
    const std::vector<char> src = read_file(path + ".src");
    if (std::string(src.begin(), src.end()) == stamp) code = read_file(path);
  }
  if (!code.empty()) {
    c.stats.jit_disk_hits++;
  } else {
    code = compile(source, name);
    c.stats.jit_compiles++;
    if (!path.empty() && make_dirs(dir)) {
      write_file_atomic(path, code);
      write_file_atomic(path + ".src", std::vector<char>(stamp.begin(), stamp.end()));
    }
  }
  Loaded l;
  hip_check(hipModuleLoadData(&l.module, code.data()), "load generated module");
  hip_check(hipModuleGetFunction(&l.fn, l.module, name), "generated kernel");
  m[key] = l;
  return l.fn;
}

void jit_clear() {
  for (auto& kv : loaded())
    if (kv.second.module) (void)hipModuleUnload(kv.second.module);
  loaded().clear();
}

}  // namespace nbgrb
