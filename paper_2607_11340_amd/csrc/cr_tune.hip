// cr_tune.hip -- the autotune cache: per device and key, the fastest launch
// variant found, and the timings it was chosen from.
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "cr_internal.h"

namespace crk {

namespace {
struct TuneEntry {
  int best;
  float ms[TUNE_NV];
};
using TuneKey = std::tuple<int, int, int, int, int>;  // device, kernel, segments, dtype, log2 work
struct TuneState {
  std::mutex mu;
  bool on = false;
  int force = -1;  // >= 0: every tunable kernel runs this variant
  std::map<TuneKey, TuneEntry> cache;
};
TuneState g_tune;

int work_bucket(int64_t work) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < work) ++b;
  return b;
}

TuneKey make_key(int kernel, int ns, int dtype, int64_t work) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  return TuneKey{dev, kernel, ns, dtype, work_bucket(work)};
}

const char* kernel_name(int k) {
  switch (k) {
    case TK_IK_STAGE1: return "ik_stage1";
    case TK_IK_STAGE1_RAG: return "ik_stage1_ragged";
    case TK_TRAJ_BUILD: return "traj_build";
    case TK_IK_STAGE2: return "ik_stage2";
    case TK_IK_STAGE1_Q: return "ik_stage1_persistent";
  }
  return "?";
}
}  // namespace

bool tune_enabled() {
  std::lock_guard<std::mutex> lk(g_tune.mu);
  return g_tune.on;
}

int tune_forced() {
  std::lock_guard<std::mutex> lk(g_tune.mu);
  return g_tune.force;
}

bool stream_capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return true;  // do not time what cannot be inspected
  return cs != hipStreamCaptureStatusNone;
}

int tune_lookup(int kernel, int ns, int dtype, int64_t work) {
  std::lock_guard<std::mutex> lk(g_tune.mu);
  auto it = g_tune.cache.find(make_key(kernel, ns, dtype, work));
  return it == g_tune.cache.end() ? -1 : it->second.best;
}

void tune_store(int kernel, int ns, int dtype, int64_t work, int best, const float* ms) {
  std::lock_guard<std::mutex> lk(g_tune.mu);
  TuneEntry e;
  e.best = best;
  for (int k = 0; k < TUNE_NV; ++k) e.ms[k] = ms[k];
  g_tune.cache[make_key(kernel, ns, dtype, work)] = e;
}

}  // namespace crk

using namespace crk;

extern "C" {

void cr_autotune_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_tune.mu);
  g_tune.on = on != 0;
}

void cr_autotune_force(int32_t variant) {
  std::lock_guard<std::mutex> lk(g_tune.mu);
  g_tune.force = variant >= 0 && variant < TUNE_NV ? variant : -1;
}

void cr_autotune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune.mu);
  g_tune.cache.clear();
}

int64_t cr_autotune_report(char* buf, int64_t cap) {
  std::string s;
  {
    std::lock_guard<std::mutex> lk(g_tune.mu);
    char line[256];
    for (const auto& kv : g_tune.cache) {
      const TuneKey& k = kv.first;
      const TuneEntry& e = kv.second;
      const int kern = std::get<1>(k);
      const bool lanes = kern == TK_IK_STAGE2;
      std::snprintf(line, sizeof line, "device %d %s n_seg %d %s work<=2^%d: %s %d (ms", std::get<0>(k),
                    kernel_name(kern), std::get<2>(k), std::get<3>(k) == CR_F64 ? "f64" : "f32", std::get<4>(k),
                    lanes ? "lanes per candidate" : "occupancy", tune_occ(kern, e.best));
      s += line;
      for (int v = 0; v < TUNE_NV; ++v) {
        std::snprintf(line, sizeof line, "%s %s%d %.4f", v ? "," : "", lanes ? "lanes" : "occ", tune_occ(kern, v),
                      e.ms[v]);
        s += line;
      }
      s += ")\n";
    }
  }
  const int64_t n = (int64_t)s.size();
  if (buf && cap > 0) {
    const int64_t m = n < cap - 1 ? n : cap - 1;
    s.copy(buf, (size_t)m);
    buf[m] = '\0';
  }
  return n;
}

}  // extern "C"
