// Subgrid planner (host).  Partitions the samples of every baseline into blocks
// whose supports fit an L x L box (§3.2 Partitioning, Fig. 2), never crossing
// an A-term slot so that one Jones matrix per station applies per block (§3.4).
//
// The rule is stated in include/idg.h (idg_plan).  All geometry is float64 and
// must not be contracted into fused multiply-adds: the plan is an integer
// result decided by float comparisons, and it has to be reproducible
// bit-for-bit by any implementation of the same rule.
#pragma STDC FP_CONTRACT OFF

#include "plan.h"

#include <algorithm>
#include <cmath>
#include <new>

namespace idg {
namespace {

struct Box {
  double mnx, mxx, mny, mxy, wpix;
};

inline Box merge(const Box &a, const Box &b) {
  return {std::min(a.mnx, b.mnx), std::max(a.mxx, b.mxx), std::min(a.mny, b.mny), std::max(a.mxy, b.mxy),
          std::max(a.wpix, b.wpix)};
}

struct BaselineGeometry {
  int nt = 0, nch = 0;
  double S = 0.0, w_step = 0.0;
  std::vector<double> x, y, w;  // [t * nch + c]; w in wavelengths

  void compute(const double *uvw_bl, const double *freqs, const idg_params &p) {
    nt = p.nr_timesteps;
    nch = p.nr_channels;
    S = p.image_size;
    w_step = p.w_step;
    x.resize(size_t(nt) * nch);
    y.resize(x.size());
    w.resize(x.size());
    const double half_n = p.grid_size / 2.0;
    for (int t = 0; t < nt; ++t) {
      const double *q = uvw_bl + size_t(t) * 3;
      for (int c = 0; c < nch; ++c) {
        const double s = freqs[c] / kSpeedOfLight;
        const double u = q[0] * s, v = q[1] * s;
        double ux = u * S;
        double vy = v * S;
        const size_t i = size_t(t) * nch + c;
        x[i] = ux + half_n;
        y[i] = vy + half_n;
        w[i] = q[2] * s;
      }
    }
  }

  // W-layer of a block of channels [lo, hi) starting at timestep t: floor(w_mid / w_step + 0.5)
  // of the mid-band w (w is linear in frequency); 0 without layers.
  int layer(int t, int lo, int hi) const {
    if (!(w_step > 0.0)) return 0;
    const size_t base = size_t(t) * nch;
    double mid = w[base + lo] + w[base + hi - 1];
    mid = mid * 0.5;
    mid = mid / w_step;
    return int(std::floor(mid + 0.5));
  }

  // w-support ceil((|w - w0| * S) * S) of one sample
  double wsupport(size_t i, double w0) const {
    double ws = std::fabs(w[i] - w0) * S;
    ws = ws * S;
    return std::ceil(ws);
  }

  Box box(int t, int lo, int hi, double w0) const {
    const size_t base = size_t(t) * nch;
    Box b{x[base + lo], x[base + lo], y[base + lo], y[base + lo], wsupport(base + lo, w0)};
    for (int c = lo + 1; c < hi; ++c) {
      b.mnx = std::min(b.mnx, x[base + c]);
      b.mxx = std::max(b.mxx, x[base + c]);
      b.mny = std::min(b.mny, y[base + c]);
      b.mxy = std::max(b.mxy, y[base + c]);
      b.wpix = std::max(b.wpix, wsupport(base + c, w0));
    }
    return b;
  }

  // the box of timestep t taken alone (with its own layer)
  Box alone(int t, int lo, int hi) const { return box(t, lo, hi, double(layer(t, lo, hi)) * w_step); }
};

inline bool fits(const Box &b, int beta, int L) {
  const double ext = double(beta) + b.wpix;
  const double lim = double(L) - 1.0;
  double sx = b.mxx - b.mnx;
  double sy = b.mxy - b.mny;
  sx = sx + ext;
  sy = sy + ext;
  return sx <= lim && sy <= lim;
}

class Planner {
 public:
  Planner(const idg_params &p, const int32_t *baselines, const double *uvw, const double *freqs,
          const uint8_t *flags, HostPlan &out)
      : p_(p), baselines_(baselines), uvw_(uvw), freqs_(freqs), flags_(flags), out_(out) {}

  void run() {
    const int nbl = p_.nr_baselines, nt = p_.nr_timesteps, nch = p_.nr_channels;
    const int64_t total = int64_t(nbl) * nt * nch;
    planned_.assign(size_t(total), 0);
    if (flags_)
      for (int64_t i = 0; i < total; ++i) out_.nr_flagged += flags_[i] != 0;
    if (nt > 0 && nch > 0) {
      for (int b = 0; b < nbl; ++b) {
        bl_ = b;
        geo_.compute(uvw_ + size_t(b) * nt * 3, freqs_, p_);
        groups_.clear();
        split(0, nch);
        for (auto &g : groups_) scan_group(g.first, g.second);
      }
    }
    for (int64_t i = 0; i < total; ++i)
      if (!planned_[size_t(i)]) out_.unplanned.push_back(i);
  }

 private:
  bool unflagged(int t, int c) const {
    return !flags_ || flags_[(size_t(bl_) * p_.nr_timesteps + t) * p_.nr_channels + c] == 0;
  }

  int count_unflagged(int t0, int t1, int lo, int hi) const {  // timesteps [t0, t1]
    int n = 0;
    for (int t = t0; t <= t1; ++t)
      for (int c = lo; c < hi; ++c) n += unflagged(t, c);
    return n;
  }

  // Channel groups: halve a group while it fails the box fit at some single timestep.
  void split(int lo, int hi) {
    if (hi - lo > 1) {
      for (int t = 0; t < p_.nr_timesteps; ++t) {
        if (!fits(geo_.alone(t, lo, hi), p_.kernel_size, p_.subgrid_size)) {
          const int mid = lo + (hi - lo) / 2;
          split(lo, mid);
          split(mid, hi);
          return;
        }
      }
    }
    groups_.emplace_back(lo, hi);
  }

  void scan_group(int lo, int hi) {
    const int nt = p_.nr_timesteps, L = p_.subgrid_size, beta = p_.kernel_size;
    const int tmax = p_.max_timesteps, aslot = p_.aterm_timesteps;
    bool open = false;
    int t0 = 0, tlast = 0, wl = 0;
    Box cur{};
    for (int t = 0; t < nt; ++t) {
      const int lt = geo_.layer(t, lo, hi);
      const Box bt = geo_.box(t, lo, hi, double(lt) * geo_.w_step);
      if (!fits(bt, beta, L)) {  // this timestep cannot be gridded even on its own
        if (open) close(t0, tlast, lo, hi, cur, wl);
        open = false;
        out_.nr_dropped += count_unflagged(t, t, lo, hi);
        continue;
      }
      if (open) {
        const Box m = merge(cur, geo_.box(t, lo, hi, double(wl) * geo_.w_step));  // the block's own w offset
        if (t - t0 < tmax && t / aslot == t0 / aslot && fits(m, beta, L)) {
          cur = m;
          tlast = t;
          continue;
        }
        close(t0, tlast, lo, hi, cur, wl);
      }
      open = true;
      t0 = tlast = t;
      wl = lt;
      cur = bt;
    }
    if (open) close(t0, tlast, lo, hi, cur, wl);
  }

  void close(int t0, int t1, int lo, int hi, const Box &b, int wlayer) {
    const int kp = count_unflagged(t0, t1, lo, hi);
    if (kp == 0) return;
    const int L = p_.subgrid_size, N = p_.grid_size;
    double cx = b.mnx + b.mxx;
    double cy = b.mny + b.mxy;
    cx = std::floor(cx * 0.5 + 0.5);
    cy = std::floor(cy * 0.5 + 0.5);
    const double x0 = cx - double(L / 2), y0 = cy - double(L / 2);
    if (!(x0 >= 0.0 && x0 + L <= double(N) && y0 >= 0.0 && y0 + L <= double(N))) {
      out_.nr_dropped += kp;
      return;
    }
    SubgridRec r;
    r.bl = bl_;
    r.t0 = t0;
    r.nt = t1 - t0 + 1;
    r.c0 = lo;
    r.nc = hi - lo;
    r.x0 = int32_t(x0);
    r.y0 = int32_t(y0);
    r.slot = t0 / p_.aterm_timesteps;
    r.s1 = baselines_[2 * bl_];
    r.s2 = baselines_[2 * bl_ + 1];
    r.nvis = kp;
    r.wlayer = wlayer;
    r.vis_offset = out_.nr_gridded;
    for (int t = t0; t <= t1; ++t)
      for (int c = lo; c < hi; ++c)
        if (unflagged(t, c)) {
          out_.samples.push_back(uint32_t(t - t0) << 16 | uint32_t(c - lo));
          planned_[(size_t(bl_) * p_.nr_timesteps + t) * p_.nr_channels + c] = 1;
        }
    out_.subgrids.push_back(r);
    out_.nr_gridded += kp;
  }

  const idg_params &p_;
  const int32_t *baselines_;
  const double *uvw_;
  const double *freqs_;
  const uint8_t *flags_;
  HostPlan &out_;
  int bl_ = 0;
  BaselineGeometry geo_;
  std::vector<std::pair<int, int>> groups_;
  std::vector<uint8_t> planned_;
};

}  // namespace

bool uniform_spacing(const double *freqs, int nr_channels) {
  if (nr_channels < 2) return false;
  const double d0 = freqs[1] - freqs[0];
  if (!(d0 > 0.0)) return false;
  for (int c = 1; c + 1 < nr_channels; ++c)
    if (!(std::fabs((freqs[c + 1] - freqs[c]) - d0) <= 1e-9 * d0)) return false;
  return true;
}

int build_plan(const idg_params &p, const int32_t *baselines, const double *uvw, const double *freqs,
               const uint8_t *flags, HostPlan &out, std::string &err) {
  try {
    out = HostPlan{};
    out.params = p;
    out.uniform_channels = uniform_spacing(freqs, p.nr_channels);
    Planner(p, baselines, uvw, freqs, flags, out).run();
    if (!out.subgrids.empty()) {
      int lo = out.subgrids[0].wlayer, hi = lo;
      for (const auto &r : out.subgrids) {
        lo = std::min(lo, r.wlayer);
        hi = std::max(hi, r.wlayer);
      }
      out.wlayer_min = lo;
      out.nr_wlayers = hi - lo + 1;
    }
  } catch (const std::bad_alloc &) {
    err = "idg_plan: out of host memory";
    return IDG_ENOMEM;
  }
  return IDG_OK;
}

}  // namespace idg
