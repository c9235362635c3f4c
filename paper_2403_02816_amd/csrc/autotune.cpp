#include "autotune.hpp"

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <vector>

namespace cgl {

namespace {

std::mutex g_mu;
std::map<std::string, int>& cache() {
  static std::map<std::string, int> c;
  return c;
}
bool g_loaded = false;

void load_file() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = std::getenv("CGL_AUTOTUNE_CACHE");
  if (!path) return;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string key;
    int v;
    if (ls >> key >> v) cache()[key] = v;
  }
}

void append_file(const std::string& key, int v) {
  const char* path = std::getenv("CGL_AUTOTUNE_CACHE");
  if (!path) return;
  std::ofstream out(path, std::ios::app);
  out << key << " " << v << "\n";
}

}  // namespace

std::string device_tag() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string s = prop.gcnArchName;
  const size_t colon = s.find(':');
  return colon == std::string::npos ? s : s.substr(0, colon);
}

int autotune_pick(const std::string& key, int ncand,
                  const std::function<hipError_t(int)>& launch, hipStream_t s, int reps,
                  const double* weight) {
  {
    std::lock_guard<std::mutex> g(g_mu);
    load_file();
    auto it = cache().find(key);
    if (it != cache().end() && it->second >= 0 && it->second < ncand) return it->second;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 0;
  // two interleaved rounds (A B ... A B ...) after one warm-up launch each;
  // a candidate's time is its better round
  std::vector<float> best_t(ncand, -1.0f);
  for (int c = 0; c < ncand; ++c)
    if (launch(c) != hipSuccess) best_t[c] = -2.0f;  // failed: never chosen
  for (int round = 0; round < 2; ++round) {
    for (int c = 0; c < ncand; ++c) {
      if (best_t[c] == -2.0f) continue;
      bool ok = hipEventRecord(e0, s) == hipSuccess;
      for (int r = 0; r < reps && ok; ++r) ok = launch(c) == hipSuccess;
      ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
      float ms = 0.0f;
      if (!ok || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        best_t[c] = -2.0f;
        continue;
      }
      if (best_t[c] < 0.0f || ms < best_t[c]) best_t[c] = ms;
    }
  }
  if (weight)
    for (int c = 0; c < ncand; ++c)
      if (best_t[c] >= 0.0f) best_t[c] = static_cast<float>(best_t[c] * weight[c]);
  int best = -1;
  for (int c = 0; c < ncand; ++c)
    if (best_t[c] >= 0.0f && (best < 0 || best_t[c] < best_t[best])) best = c;
  if (std::getenv("CGL_AUTOTUNE_VERBOSE")) {
    std::fprintf(stderr, "autotune %s:", key.c_str());
    for (int c = 0; c < ncand; ++c) std::fprintf(stderr, " %.4f", best_t[c] / reps);
    std::fprintf(stderr, " -> %d\n", best);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best < 0) return 0;
  std::lock_guard<std::mutex> g(g_mu);
  cache()[key] = best;
  append_file(key, best);
  return best;
}

}  // namespace cgl
