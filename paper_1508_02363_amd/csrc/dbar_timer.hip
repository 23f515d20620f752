// Per-stage launch timing with HIP events (measurement support; off unless enabled).
#include <mutex>
#include <string>
#include <vector>

#include "dbar.h"
#include "dbar_launch.h"
#include "dbar_solver.h"

namespace dbar {

namespace {
struct Rec {
  int stage;
  double bytes_per_entry, bytes_once;
  int B;
  int slot;  // -1: all B entries active
  hipEvent_t e0, e1;
};
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
size_t g_pool_next = 0;
DevBuf g_log;
constexpr int kLogSlots = 1 << 20;
int g_slot = 0;

struct StageAgg {
  double ms = 0.0, bytes = 0.0;
  long long launches = 0;
};
std::vector<StageAgg> g_agg;

hipEvent_t next_event() {
  if (g_pool_next == g_pool.size()) {
    hipEvent_t e;
    (void)hipEventCreate(&e);
    g_pool.push_back(e);
  }
  return g_pool[g_pool_next++];
}
}  // namespace

__global__ void k_count_active(const int* act, int B, int* out) {
  int c = 0;
  for (int b = threadIdx.x; b < B; b += 64) c += act[b] != 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if (threadIdx.x == 0) *out = c;
}

const char* stage_name(int stage) {
  static const char* lines[] = {"RowsInvScaled", "ColsInvMoments", "RowsInvRegular", "ColsInvTailFwd",
                                "ColsInvTail",   "RowsFwdEpilogue", "ColsFwdPotential", "ColsFwdPlain",
                                "ColsInvPlain",  "RowsFwdMoments", "ColsFwdRegularInv", "RowsInvTailEpilogue"};
  static std::string names[kNumStages];
  if (stage < 0 || stage >= kNumStages) return "?";
  if (names[stage].empty()) {
    if (stage < kStageDots) {
      const int op = stage / 2;
      names[stage] = std::string("lines.") + (op < 12 ? lines[op] : "?") + (stage % 2 ? ".f32" : ".f64");
    } else if (stage < kStageUpdate) {
      names[stage] = stage == kStageDots ? "krylov.dots.f64" : "krylov.dots.f32";
    } else if (stage < kStageAxpy) {
      names[stage] = stage == kStageUpdate ? "krylov.update.f64" : "krylov.update.f32";
    } else if (stage < kStageReduce) {
      static const char* ax[] = {"krylov.axpy.f64_f64", "krylov.axpy.f64_f32", "krylov.axpy.f32_f32"};
      names[stage] = ax[stage - kStageAxpy];
    } else if (stage == kStageReduce) {
      names[stage] = "reduce";
    } else if (stage == kStageConvert) {
      names[stage] = "convert";
    } else if (stage == kStageMoments) {
      names[stage] = "moments.finish";
    } else {
      names[stage] = "control";
    }
  }
  return names[stage].c_str();
}

bool timer_on() { return g_on; }

static std::mutex g_timer_mutex;

int timer_begin(int stage, double bytes_per_entry, int B, const int* act, hipStream_t s, double bytes_once) {
  std::lock_guard<std::mutex> lock(g_timer_mutex);
  Rec r;
  r.stage = stage;
  r.bytes_per_entry = bytes_per_entry;
  r.bytes_once = bytes_once;
  r.B = B;
  r.slot = -1;
  if (act && g_log.p && g_slot < kLogSlots) {
    r.slot = g_slot++;
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(64), 0, s, act, B, static_cast<int*>(g_log.p) + r.slot);
  }
  r.e0 = next_event();
  r.e1 = next_event();
  (void)hipEventRecord(r.e0, s);
  g_recs.push_back(r);
  return static_cast<int>(g_recs.size()) - 1;
}

void timer_end(int h, hipStream_t s) {
  std::lock_guard<std::mutex> lock(g_timer_mutex);
  (void)hipEventRecord(g_recs[h].e1, s);
}

static int timer_collect() {
  if (hipDeviceSynchronize() != hipSuccess) return fail(DBAR_EDEVICE, "synchronize failed");
  std::vector<int> log(g_slot);
  if (g_slot && hipMemcpy(log.data(), g_log.p, g_slot * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(DBAR_EDEVICE, "timer log copy failed");
  for (const Rec& r : g_recs) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.e0, r.e1);
    const int active = r.slot >= 0 ? log[r.slot] : r.B;
    StageAgg& a = g_agg[r.stage];
    a.ms += ms;
    a.bytes += r.bytes_per_entry * active + (active > 0 ? r.bytes_once : 0.0);
    a.launches += 1;
  }
  g_recs.clear();
  g_pool_next = 0;
  g_slot = 0;
  return DBAR_OK;
}

}  // namespace dbar

using namespace dbar;

extern "C" {

int dbar_timer_enable(int32_t on) {
  if (on) {
    if (g_log.ensure(kLogSlots * sizeof(int))) return DBAR_ENOMEM;
    g_recs.clear();
    g_pool_next = 0;
    g_slot = 0;
    g_agg.assign(kNumStages, StageAgg{});
    g_on = true;
    return DBAR_OK;
  }
  g_on = false;
  return timer_collect();
}

int dbar_timer_stage(int32_t stage, char* name, int32_t name_len, double* total_ms, int64_t* launches,
                     double* bytes) {
  if (stage < 0 || stage >= kNumStages) return fail(DBAR_EINVAL, "stage out of range");
  if (g_on) {
    int rc = timer_collect();
    if (rc) return rc;
  }
  if (g_agg.size() != (size_t)kNumStages) g_agg.assign(kNumStages, StageAgg{});
  if (name && name_len > 0) {
    std::string nm = stage_name(stage);
    std::snprintf(name, name_len, "%s", nm.c_str());
  }
  if (total_ms) *total_ms = g_agg[stage].ms;
  if (launches) *launches = g_agg[stage].launches;
  if (bytes) *bytes = g_agg[stage].bytes;
  return DBAR_OK;
}

int dbar_timer_num_stages(void) { return kNumStages; }

}  // extern "C"
