// timing.hpp -- optional per-kernel-family timing: while enabled, HIP events
// are recorded on the launch stream around every launch of a family; the
// host reads the accumulated time and launch count back (grmhd_timing_read).
#pragma once
#include <hip/hip_runtime.h>

namespace gk {

constexpr int kFamilies = 18;
constexpr int kEventPool = 8192;

// kernel families
enum {
  T_FLUX_X = 0, T_FLUX_Y, T_FLUX_Z, T_FOFC_FLAGS, T_FOFC_FIX, T_CT, T_UPDATE, T_C2P, T_GHOST,
  T_DT, T_BCC, T_C2P_BATCH, T_C2P_LEARNED, T_MLP_TRAIN, T_MLP_BRACKET, T_STAGE_C2P_LEARNED,
  T_MATTER, T_EXCISE
};

struct Timing {
  int on = 0;
  int created = 0;
  int used = 0;
  hipEvent_t ev[kEventPool];
  int fam[kEventPool / 2];
  double ms[kFamilies];
  long long cnt[kFamilies];
};
extern Timing g_tm;

struct TimedScope {
  int slot;
  hipStream_t s;
  TimedScope(int f, hipStream_t st) : slot(-1), s(st) {
    if (g_tm.on && g_tm.used + 2 <= kEventPool) {
      slot = g_tm.used;
      g_tm.used += 2;
      g_tm.fam[slot / 2] = f;
      (void)hipEventRecord(g_tm.ev[slot], s);
    }
  }
  ~TimedScope() {
    if (slot >= 0) (void)hipEventRecord(g_tm.ev[slot + 1], s);
  }
};

}  // namespace gk

#define TIMED(fam, s) gk::TimedScope timed_scope_(fam, s)
