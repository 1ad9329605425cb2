// Host-side subgrid plan (partitioning of §3.2 with the A-term cuts of §3.4).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "idg.h"

namespace idg {

constexpr double kSpeedOfLight = 299792458.0;

// One subgrid: a block of one baseline, timesteps [t0, t0 + nt), channels [c0, c0 + nc).
struct SubgridRec {
  int32_t bl, t0, nt, c0, nc, x0, y0, slot, s1, s2, nvis;
  int32_t wlayer;      // W-layer: w offset wlayer * w_step
  int64_t vis_offset;  // first row of this subgrid in HostPlan::samples
};

struct HostPlan {
  idg_params params{};
  std::vector<SubgridRec> subgrids;
  std::vector<uint32_t> samples;    // per planned sample: (t - t0) << 16 | (c - c0)
  std::vector<int64_t> unplanned;   // flat sample ids (bl * nt + t) * nch + c not gridded
  int64_t nr_gridded = 0, nr_dropped = 0, nr_flagged = 0;
  bool uniform_channels = false;    // channel spacings equal to 1e-9 relative (see uniform_spacing)
  int32_t wlayer_min = 0, nr_wlayers = 1;  // W-layers in use: grids [nr_wlayers][4][N][N]
};

// True when every spacing freqs[c + 1] - freqs[c] equals the first one to a
// relative 1e-9: the phase of channel c + j is then the phase of channel c plus
// j times one per-run step, to far below float32 resolution over short runs.
bool uniform_spacing(const double *freqs, int nr_channels);

// Builds the plan; returns IDG_OK or IDG_ENOMEM (inputs are validated by the caller).
int build_plan(const idg_params &p, const int32_t *baselines, const double *uvw, const double *freqs,
               const uint8_t *flags, HostPlan &out, std::string &err);

}  // namespace idg
