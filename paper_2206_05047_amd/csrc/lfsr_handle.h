// Handle state of the C ABI (include/lfsr.h), shared by the solver entry
// points and the serving pool.
#pragma once

#include <string>
#include <vector>

#include "../../include/lfsr.h"
#include "lfsr_internal.h"

namespace lfsr {

// Validated geometry plus the workspace layout of one problem.
struct Plan {
  Geom g;
  size_t off_x, off_dx, off_m, off_vs, off_r, off_pv, off_hp, off_wd, off_ws0, off_ws1, off_lr, off_adj, off_pwzd,
      off_ptv, off_prr0, off_prr1, off_pphp, off_pmax, off_pcnt, off_stats, off_sc, off_taps;
  float taps2d[kMax2DTaps * kMax2DTaps];  // explicit blur kernel (host copy), when g.blur2d
  size_t bytes;
};

// Kernel timing requested through lfsr_profile_begin.
struct Profile {
  bool on = false;
  uint32_t mask = 0;
  std::vector<hipEvent_t> ev;  // pairs
  std::vector<int> kind;
  int used = 0;
};

}  // namespace lfsr

struct lfsr_handle {
  lfsr::Profile prof;
  lfsr_params prm;
  lfsr::Plan plan;
  lfsr::Bufs b;
  char* ws;
  int n_done;
  bool bound;
  bool broken;
  const float* y;
  const float* disp;
  const float* occ;
  std::string err;
};

