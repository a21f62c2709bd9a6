// Launch-plan cache of the library's autotuner.
//
// A plan is a launch shape that changes no result: the histogram scan's
// particle tile and chunk length (integer counts; only the order of the FP64
// sums of a regression scan), the projection's particle blocks per wave and
// work-group order (every output element is the same MFMA sequence).  Plans
// are measured on the device (hipEvents around each candidate, the fastest
// kept) for a shape class and kept in memory, keyed by the device's
// architecture and the shape class; the cache is read from and written to a
// small JSON file.  Without a plan for a shape the launch takes the fitted
// rule of its kernel.
#include "slm_internal.hpp"

#include <dlfcn.h>

#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

namespace slm {
namespace {

std::mutex g_mu;
std::map<std::string, std::pair<int64_t, int64_t>> g_plans;
int g_mode = -1;               // -1: not initialised
std::string g_path;            // file written by mode 2
uint64_t g_gen = 1;            // bumped whenever the plans in use change

// Directory of this library (the plans file measured on the target ships
// beside it).
std::string lib_dir() {
  Dl_info info{};
  if (dladdr(reinterpret_cast<void *>(&lib_dir), &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    const size_t k = p.rfind('/');
    if (k != std::string::npos) return p.substr(0, k);
  }
  return ".";
}

// {"plans": {"key": [a, b], ...}}; keys hold no quotes.  Anything else in
// the file is ignored; a malformed file loads nothing.
void load_file(const std::string &path) {
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = s.find("\"plans\"");
  if (i == std::string::npos) return;
  i = s.find('{', i);
  while (i != std::string::npos) {
    const size_t k0 = s.find('"', i + 1);
    if (k0 == std::string::npos) break;
    const size_t k1 = s.find('"', k0 + 1);
    const size_t b0 = s.find('[', k1);
    const size_t b1 = s.find(']', b0 == std::string::npos ? k1 : b0);
    if (k1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos) break;
    long long a = 0, b = 0;
    if (sscanf(s.c_str() + b0, "[%lld , %lld]", &a, &b) == 2 ||
        sscanf(s.c_str() + b0, "[%lld,%lld]", &a, &b) == 2)
      g_plans[s.substr(k0 + 1, k1 - k0 - 1)] = {a, b};
    i = s.find_first_of(",}", b1);
    if (i == std::string::npos || s[i] == '}') break;
  }
}

void save_file_locked() {
  if (g_path.empty()) return;
  std::ofstream f(g_path, std::ios::trunc);
  if (!f) return;
  f << "{\n  \"plans\": {";
  bool first = true;
  for (const auto &kv : g_plans) {
    f << (first ? "\n" : ",\n") << "    \"" << kv.first << "\": [" << kv.second.first << ", "
      << kv.second.second << "]";
    first = false;
  }
  f << "\n  }\n}\n";
}

void init_locked() {
  if (g_mode >= 0) return;
  g_mode = 1;
  load_file(lib_dir() + "/plans_" + device_arch() + ".json");
}

}  // namespace

std::string device_arch() {
  static std::string arch = [] {
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      (void)hipGetLastError();
      return std::string("unknown");
    }
    std::string a(prop.gcnArchName);
    const size_t k = a.find(':');
    return k == std::string::npos ? a : a.substr(0, k);
  }();
  return arch;
}

int autotune_mode() {
  std::lock_guard<std::mutex> lk(g_mu);
  init_locked();
  return g_mode;
}

uint64_t autotune_generation() {
  std::lock_guard<std::mutex> lk(g_mu);
  init_locked();
  return g_mode == 0 ? 0 : g_gen;
}

bool plan_lookup(const std::string &key, int64_t *a, int64_t *b) {
  std::lock_guard<std::mutex> lk(g_mu);
  init_locked();
  if (g_mode == 0) return false;
  const auto it = g_plans.find(key);
  if (it == g_plans.end()) return false;
  *a = it->second.first;
  *b = it->second.second;
  return true;
}

bool plan_known(const std::string &key) {
  std::lock_guard<std::mutex> lk(g_mu);
  init_locked();
  return g_plans.count(key) != 0;
}

void plan_store(const std::string &key, int64_t a, int64_t b) {
  std::lock_guard<std::mutex> lk(g_mu);
  init_locked();
  g_plans[key] = {a, b};
  ++g_gen;
  save_file_locked();
}

}  // namespace slm

using namespace slm;

extern "C" {

slm_status slm_autotune_set(int32_t mode, const char *path) {
  clear_error();
  SLM_CHECK(mode >= 0 && mode <= 2, SLM_E_INVALID, "slm_autotune_set: mode %d (0, 1 or 2)", mode);
  SLM_CHECK(mode != 2 || (path && path[0]), SLM_E_INVALID,
            "slm_autotune_set: mode 2 needs a file to write the plans to");
  std::lock_guard<std::mutex> lk(g_mu);
  init_locked();
  if (path && path[0]) {
    g_plans.clear();
    load_file(path);
  } else if (mode == 1) {
    g_plans.clear();
    load_file(lib_dir() + "/plans_" + device_arch() + ".json");
  }
  g_path = mode == 2 ? std::string(path) : std::string();
  g_mode = mode;
  ++g_gen;
  return SLM_OK;
}

int32_t slm_autotune_plans(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  init_locked();
  return (int32_t)g_plans.size();
}

}  // extern "C"
