// launch.h -- helpers shared by the engine and the translation units that
// instantiate the sweep launches (launch_*.hip): block size, grid sizes,
// work lists and the launch-timing hook.
#pragma once

#include "engine.h"

#include <string>

namespace fish {

constexpr int kBlock = 256;

inline unsigned grid_for(long long threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(3, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Bracket one kernel launch with events when its class is being timed
// (classes: 1 fluid, 2 field, 8 CFL check).
struct TimedLaunch {
  Engine* e;
  int idx = -1;
  TimedLaunch(Engine* eng, int cls) : e(eng) {
    if ((e->timing_mask & cls) && e->ev_used < e->timing_max) {
      idx = e->ev_used++;
      (void)hipEventRecord(e->ev_start[idx], e->cfg.stream);
    }
  }
  ~TimedLaunch() {
    if (idx >= 0) (void)hipEventRecord(e->ev_stop[idx], e->cfg.stream);
  }
};

inline WorkList make_wl(const Engine* e, int kind) {
  WorkList w;
  w.boxes = static_cast<const BoxDesc*>(e->table.ptr);
  w.wave_box = static_cast<const int*>(e->lists[kind].ptr);
  w.nwaves = e->nwaves[kind];
  w.xcd_remap = e->tuning.remap[kind];
  w.row_groups = e->tuning.groups[kind];
  return w;
}

}  // namespace fish
