// Autotuner of the near-sum launch shape (block size, targets per lane, LDS tile), run on the handle's own geometry: every candidate is timed with HIP
// events on the handle's stream; the fastest per precision is kept and optionally
// cached in a text file keyed by device, node count, precision and near set.
#include <algorithm>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>

#include "spm_internal.h"

namespace spm {

void launch_prep_for_timing(spm_handle* h);          // capi.hip

static std::string device_name() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string s = p.gcnArchName;
  for (char& c : s)
    if (c == ' ' || c == ':') c = '_';
  return s;
}

static std::string key_of(spm_handle* h, int prec) {
  std::ostringstream o;
  double work = 0;
  for (const auto& c : h->cells) work += (double)(c.n1 - c.n0) * (double)(c.n1 - c.n0);
  o << device_name() << " N=" << h->geo.N << " C=" << h->geo.C << " W=" << work << " prec=" << (prec == 0 ? "fp64" : "fp32")
    << " set=" << (h->geo.dilated ? "dilated" : "3x3");
  return o.str();
}

static bool cache_lookup(const char* path, const std::string& key, NearConfig& c) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t bar = line.find('|');
    if (bar == std::string::npos || line.substr(0, bar) != key) continue;
    std::istringstream v(line.substr(bar + 1));
    NearConfig t;
    if (v >> t.block >> t.tpt >> t.tile >> t.wg_per_cu && near_config_valid(t)) {
      c = t;
      return true;
    }
  }
  return false;
}

static void cache_store(const char* path, const std::string& key, const NearConfig& c, double ms) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key << "|" << c.block << " " << c.tpt << " " << c.tile << " " << c.wg_per_cu << " " << ms << "\n";
}

double time_near(spm_handle* h, int prec, const NearConfig& c, int reps) {
  NearPlan& P = h->wk.near[prec];
  const NearConfig saved = P.cfg;
  P.cfg = c;
  build_near_plan(h, prec == 0 ? SPM_FP64 : SPM_FP32);
  const bool prof = h->prof;
  h->prof = false;
  hipEvent_t a, b;
  SPM_HIP_CHECK(hipEventCreate(&a));
  SPM_HIP_CHECK(hipEventCreate(&b));
  launch_near(h, prec == 0 ? SPM_FP64 : SPM_FP32);  // warm
  SPM_HIP_CHECK(hipEventRecord(a, h->stream));
  for (int r = 0; r < reps; ++r) launch_near(h, prec == 0 ? SPM_FP64 : SPM_FP32);
  SPM_HIP_CHECK(hipEventRecord(b, h->stream));
  SPM_HIP_CHECK(hipEventSynchronize(b));
  float ms = 0.f;
  SPM_HIP_CHECK(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  P.cfg = saved;
  build_near_plan(h, prec == 0 ? SPM_FP64 : SPM_FP32);
  h->prof = prof;
  return (double)ms / reps;
}

void autotune(spm_handle* h, const char* cache_path, double* best_ms_out) {
  launch_prep_for_timing(h);
  double work = 0;
  for (const auto& c : h->cells) work += (double)(c.n1 - c.n0) * (double)(c.n1 - c.n0);
  for (int prec = 0; prec < 2; ++prec) {
    const std::string key = key_of(h, prec);
    NearConfig best;
    double best_ms = -1.0;
    if (cache_lookup(cache_path, key, best)) {
      h->wk.near[prec].cfg = best;
      build_near_plan(h, prec == 0 ? SPM_FP64 : SPM_FP32);
      if (best_ms_out) best_ms_out[prec] = 0.0;
      continue;
    }
    std::vector<NearConfig> cand;
    for (int block : {64, 128, 256})
      for (int tpt : {1, 2, 4})
        for (int tile : {128, 256, 512}) {
          NearConfig c;
          c.block = block;
          c.tpt = tpt;
          c.tile = tile;
          c.wg_per_cu = 0;
          cand.push_back(c);
        }
    const int reps = work > 4e8 ? 2 : 5;
    for (const auto& c : cand) {
      const double ms = time_near(h, prec, c, reps);
      if (best_ms < 0 || ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    h->wk.near[prec].cfg = best;
    build_near_plan(h, prec == 0 ? SPM_FP64 : SPM_FP32);
    if (best_ms_out) best_ms_out[prec] = best_ms;
    cache_store(cache_path, key, best, best_ms);
  }
  h->wk.tuned = true;
  h->wk.tuned_N = h->geo.N;
}

}  // namespace spm
