// C ABI of the image-domain gridding library: validation, plan upload, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "idg.h"
#include "internal.h"
#include "plan.h"
#include "taper.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(IDG_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), int(e));
}

#define HIP_TRY(expr, what)                  \
  do {                                       \
    hipError_t e_ = (expr);                  \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

constexpr int64_t kDefaultScratch = int64_t(2) << 30;

// Device-resident plan metadata on one device.
struct Batch {
  int64_t first = 0, count = 0;      // plan subgrids [first, first + count)
  int64_t order_off = 0;             // gridder work list (local indices, costliest first): the subgrids of
  int64_t n_sep = 0;                 // the separable form first (n_sep of them), then those of the direct sum
  int64_t item_off = 0, nitems = 0;  // adder items
  int64_t combine_off = 0, ncombine = 0;
  int64_t nslots = 0;                // partial tiles of this batch
};

struct DevPlan {
  int device = -1;
  int nr_cus = 1;
  idg::DevSubgrid *subgrids = nullptr;
  uint32_t *samples = nullptr;
  int64_t *unplanned = nullptr;
  float4 *lmn = nullptr;
  float2 *twiddle = nullptr;
  float2 *sep = nullptr;   // separable form: (x_q, a_q)
  float *cross = nullptr;  // separable form: c_ij
  int cross_exp = 0;       // max |c_ij| <= 2^cross_exp
  int32_t *grid_order = nullptr, *degrid_order = nullptr, *contrib = nullptr;
  idg::AdderItem *items = nullptr;
  idg::CombineItem *combine = nullptr;
  std::vector<Batch> batches;
  int64_t batch_size = 0, max_slots = 0;
  int64_t degrid_n_sep = 0;    // leading entries of degrid_order in the separable form
  int64_t degrid_n_large = 0;  // then the entries above the small-subgrid threshold
  std::vector<int16_t> order;  // host copy of each subgrid's separable-form order (-1: direct sum)

  ~DevPlan() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != device) (void)hipSetDevice(device);
    void *ptrs[] = {subgrids, samples, unplanned, lmn, twiddle, sep, cross, grid_order, degrid_order, contrib, items,
                    combine};
    for (void *p : ptrs)
      if (p) (void)hipFree(p);
    if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
  }
};

struct TileLists {
  std::vector<int32_t> tile_ids, tile_start, contrib;
};

// Tile ownership for the adder: for every grid tile, the local indices of the
// subgrids that overlap it, ascending; tiles with more work first.
// Tile ids run over the W-layers: (layer - wlayer_min) * ntx^2 + ty * ntx + tx.
void build_tile_lists(const std::vector<idg::SubgridRec> &subs, int64_t first, int64_t count, int N, int L,
                      int wlayer_min, int nr_wlayers, TileLists &out) {
  const int T = idg::kAdderTile;
  const int ntx = (N + T - 1) / T;
  const int64_t ntile = int64_t(ntx) * ntx * nr_wlayers;
  std::vector<int32_t> cnt(size_t(ntile) + 1, 0);
  auto each_tile = [&](const idg::SubgridRec &r, auto &&fn) {
    const int64_t base = int64_t(r.wlayer - wlayer_min) * ntx * ntx;
    for (int ty = r.y0 / T; ty <= (r.y0 + L - 1) / T; ++ty)
      for (int tx = r.x0 / T; tx <= (r.x0 + L - 1) / T; ++tx) fn(base + int64_t(ty) * ntx + tx);
  };
  for (int64_t s = 0; s < count; ++s) each_tile(subs[size_t(first + s)], [&](int64_t t) { cnt[size_t(t)]++; });
  std::vector<int64_t> off(size_t(ntile) + 1, 0);
  for (int64_t t = 0; t < ntile; ++t) off[size_t(t) + 1] = off[size_t(t)] + cnt[size_t(t)];
  std::vector<int32_t> flat(static_cast<size_t>(off[static_cast<size_t>(ntile)]));
  std::vector<int64_t> pos(off.begin(), off.end() - 1);
  for (int64_t s = 0; s < count; ++s)
    each_tile(subs[size_t(first + s)], [&](int64_t t) { flat[size_t(pos[size_t(t)]++)] = int32_t(s); });
  std::vector<int32_t> active;
  for (int64_t t = 0; t < ntile; ++t)
    if (cnt[size_t(t)]) active.push_back(int32_t(t));
  std::stable_sort(active.begin(), active.end(),
                   [&](int32_t a, int32_t b) { return cnt[size_t(a)] > cnt[size_t(b)]; });
  out.tile_ids = active;
  out.tile_start.resize(active.size() + 1);
  out.contrib.clear();
  out.contrib.reserve(flat.size());
  out.tile_start[0] = 0;
  for (size_t i = 0; i < active.size(); ++i) {
    const int64_t t = active[i];
    out.contrib.insert(out.contrib.end(), flat.begin() + off[size_t(t)], flat.begin() + off[size_t(t) + 1]);
    out.tile_start[i + 1] = int32_t(out.contrib.size());
  }
}

// Adder work items for one set of tile lists: runs of at most `chunk`
// contributions; split tiles get partial slots and a combine entry.  Item
// positions are offset by `contrib_base` (position of the lists in the
// concatenated contribution array).
struct AdderPlan {
  std::vector<idg::AdderItem> items;
  std::vector<idg::CombineItem> combine;
  int32_t nslots = 0;
};

void build_adder_plan(const TileLists &tl, int chunk, int64_t contrib_base, AdderPlan &out) {
  out = AdderPlan{};
  for (size_t i = 0; i < tl.tile_ids.size(); ++i) {
    const int32_t b = tl.tile_start[i], e = tl.tile_start[i + 1];
    const int32_t tile = tl.tile_ids[i];
    if (e - b <= chunk) {
      out.items.push_back({tile, int32_t(contrib_base + b), int32_t(contrib_base + e), -1});
      continue;
    }
    const int32_t n = (e - b + chunk - 1) / chunk;
    out.combine.push_back({tile, out.nslots, out.nslots + n, 0});
    for (int32_t j = 0; j < n; ++j) {
      const int32_t cb = b + j * chunk, ce = std::min(e, cb + chunk);
      out.items.push_back({tile, int32_t(contrib_base + cb), int32_t(contrib_base + ce), out.nslots + j});
    }
    out.nslots += n;
  }
}

// Stage timing with HIP events on the launching stream (idg_profile).
struct Profiler {
  struct Rec {
    int stage;
    hipEvent_t start, stop;
  };
  std::mutex mu;
  bool on = false;
  std::vector<Rec> pending;
  double ms[IDG_NR_STAGES] = {};
  int64_t launches[IDG_NR_STAGES] = {};
};

Profiler &profiler() {
  static Profiler p;
  return p;
}

// Brackets one kernel launch when profiling is on.
class StageTimer {
 public:
  StageTimer(int stage, hipStream_t s) : stage_(stage), s_(s) {
    Profiler &p = profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    if (!p.on) return;
    if (hipEventCreate(&a_) != hipSuccess) return;
    if (hipEventCreate(&b_) != hipSuccess) {
      (void)hipEventDestroy(a_);
      return;
    }
    active_ = hipEventRecord(a_, s_) == hipSuccess;
  }
  ~StageTimer() {
    if (!active_) return;
    Profiler &p = profiler();
    if (hipEventRecord(b_, s_) != hipSuccess) {
      (void)hipEventDestroy(a_);
      (void)hipEventDestroy(b_);
      return;
    }
    std::lock_guard<std::mutex> lock(p.mu);
    p.pending.push_back({stage_, a_, b_});
  }

 private:
  int stage_;
  hipStream_t s_;
  hipEvent_t a_{}, b_{};
  bool active_ = false;
};

template <typename T>
int upload(T **dst, const T *src, size_t n, const char *what) {
  *dst = nullptr;
  if (n == 0) return IDG_OK;
  HIP_TRY(hipMalloc(reinterpret_cast<void **>(dst), n * sizeof(T)), what);
  HIP_TRY(hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice), what);
  return IDG_OK;
}

}  // namespace

struct idg_plan_s {
  idg::HostPlan host;
  std::vector<double> wmax;  // per subgrid: largest |w - w_0p| of its samples, wavelengths (float64)
  idg_tuning tuning{};
  std::mutex mu;
  std::map<int, std::unique_ptr<DevPlan>> dev;
};

namespace {

int64_t batch_size_of(const idg_params &p) {
  const int64_t per = int64_t(4) * p.subgrid_size * p.subgrid_size * int64_t(sizeof(idg_cf32));
  const int64_t budget = p.scratch_bytes > 0 ? p.scratch_bytes : kDefaultScratch;
  return std::max<int64_t>(1, std::min<int64_t>(budget / per, int64_t(1) << 30));
}

// Separable form: x_q = (q - L/2) S / L, a_q = sqrt(1 - x_q^2) - 1 and c_ij = n'_ij - a_i - a_j, so that
// n'_ij = a_i + a_j + c_ij exactly in float64.  Returns max |c_ij|.
double separable_tables(int L, double S, std::vector<float2> &sep, std::vector<float> &cross) {
  auto nprime = [](double r2) { return -r2 / (1.0 + std::sqrt(1.0 - r2)); };  // sqrt(1 - r2) - 1, no cancellation
  std::vector<double> x(static_cast<size_t>(L)), av(static_cast<size_t>(L));
  sep.resize(size_t(L));
  for (int q = 0; q < L; ++q) {
    x[size_t(q)] = (q - L / 2) * (S / L);
    av[size_t(q)] = nprime(x[size_t(q)] * x[size_t(q)]);
    sep[size_t(q)] = make_float2(float(x[size_t(q)]), float(av[size_t(q)]));
  }
  cross.resize(size_t(L) * L);
  double cmax = 0.0;
  for (int j = 0; j < L; ++j)
    for (int i = 0; i < L; ++i) {
      const double c = nprime(x[size_t(i)] * x[size_t(i)] + x[size_t(j)] * x[size_t(j)]) - av[size_t(i)] - av[size_t(j)];
      cross[size_t(j) * L + i] = float(c);
      cmax = std::max(cmax, std::fabs(c));
    }
  return cmax;
}

// Expansion order of the separable form's cross term for a subgrid whose largest |w - w_0p| is wmax:
// the smallest N with (2 pi wmax cmax)^(N+1) / (N+1)! <= 1e-6, or -1 when N would exceed max_order.
int separable_order(double wmax, double cmax, int max_order) {
  const double theta = 2.0 * M_PI * wmax * cmax;
  double term = theta, fact = 1.0;
  for (int n = 0; n <= max_order; ++n) {
    fact *= double(n + 1);
    if (term / fact <= 1e-6) return n;
    term *= theta;
  }
  return -1;
}

// Whether the plan's subgrids may take the separable form (subgrid size, precision and tuning).
bool separable_on(const idg_plan_s *plan) {
  const idg_params &p = plan->host.params;
  return idg::separable_supported(p.subgrid_size) && !(p.flags & IDG_PHASE_FP32) &&
         plan->tuning.sum_path == IDG_SUM_AUTO;
}

void lmn_table(int L, double S, std::vector<float4> &lmn, std::vector<float2> &tw) {
  lmn.resize(size_t(L) * L);
  for (int j = 0; j < L; ++j)
    for (int i = 0; i < L; ++i) {
      const double l = (i - L / 2) * (S / L), m = (j - L / 2) * (S / L);
      const double r2 = l * l + m * m;
      const double n = -r2 / (1.0 + std::sqrt(1.0 - r2));  // sqrt(1 - r2) - 1 without cancellation
      lmn[size_t(j) * L + i] = make_float4(float(l), float(m), float(n), 0.0f);
    }
  tw.resize(size_t(L));
  for (int k = 0; k < L; ++k) {
    const double ph = -2.0 * M_PI * k / L;
    tw[size_t(k)] = make_float2(float(std::cos(ph)), float(std::sin(ph)));
  }
}

// The library's stream-ordered memory pool of the current device, created on first use.  Every call's
// scratch comes from it; freed blocks stay in the pool (release threshold: unlimited) so that repeated
// calls do not remap tens of GB, and idg_trim_scratch hands them back.  Being the library's own pool, it
// leaves the device's default pool (torch's and other users') as it is.
hipError_t scratch_pool(hipMemPool_t *out) {
  static std::mutex mu;
  static std::map<int, hipMemPool_t> pools;
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = pools.find(device);
  if (it != pools.end()) {
    *out = it->second;
    return hipSuccess;
  }
  hipMemPoolProps props = {};
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = device;
  hipMemPool_t pool = nullptr;
  e = hipMemPoolCreate(&pool, &props);
  if (e != hipSuccess) return e;
  uint64_t keep = UINT64_MAX;
  e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  if (e != hipSuccess) {
    (void)hipMemPoolDestroy(pool);
    return e;
  }
  pools.emplace(device, pool);
  *out = pool;
  return hipSuccess;
}

// Stream-ordered scratch from the library's pool (released with hipFreeAsync).
hipError_t scratch_alloc(void **p, size_t bytes, hipStream_t s) {
  hipMemPool_t pool = nullptr;
  const hipError_t e = scratch_pool(&pool);
  if (e != hipSuccess) return e;
  return hipMallocFromPoolAsync(p, bytes, pool, s);
}

// Device metadata of `plan` on the current device, uploaded on first use.
int device_plan(idg_plan_t plan, DevPlan **out) {
  int device = 0;
  HIP_TRY(hipGetDevice(&device), "hipGetDevice");
  std::lock_guard<std::mutex> lock(plan->mu);
  auto it = plan->dev.find(device);
  if (it != plan->dev.end()) {
    *out = it->second.get();
    return IDG_OK;
  }
  const idg::HostPlan &h = plan->host;
  const idg_params &p = h.params;
  auto dp = std::make_unique<DevPlan>();
  dp->device = device;
  const int L = p.subgrid_size;
  std::vector<idg::DevSubgrid> subs(h.subgrids.size());
  for (size_t i = 0; i < subs.size(); ++i) {
    const auto &r = h.subgrids[i];
    idg::DevSubgrid &d = subs[i];
    d.bl = r.bl;
    d.t0 = r.t0;
    d.c0 = r.c0;
    d.nvis = r.nvis;
    d.x0 = r.x0;
    d.y0 = r.y0;
    d.a1 = r.slot * p.nr_stations + r.s1;
    d.a2 = r.slot * p.nr_stations + r.s2;
    d.vis_offset = r.vis_offset;
    d.w0 = double(r.wlayer) * p.w_step;
    d.layer = r.wlayer - h.wlayer_min;
    d.order = -1;
    d.wexp = 0;
  }
  std::vector<float4> lmn;
  std::vector<float2> tw;
  lmn_table(L, p.image_size, lmn, tw);
  std::vector<float2> sep;
  std::vector<float> cross;
  const double cmax = separable_tables(L, p.image_size, sep, cross);
  if (cmax > 0.0) (void)std::frexp(cmax, &dp->cross_exp);  // cmax < 2^cross_exp
  // separable form: the expansion order and the power-of-two bound of |w - w_0p| per subgrid
  if (separable_on(plan))
    for (size_t i = 0; i < subs.size(); ++i) {
      const double wm = plan->wmax[i];
      int e = 0;
      if (wm > 0.0) (void)std::frexp(wm, &e);  // wm < 2^e
      subs[i].order = int16_t(separable_order(wm, cmax, idg::separable_max_order()));
      subs[i].wexp = int16_t(std::max(-120, std::min(120, e)));
    }
  dp->order.resize(subs.size());
  for (size_t i = 0; i < subs.size(); ++i) dp->order[i] = subs[i].order;
  int rc;
  if ((rc = upload(&dp->subgrids, subs.data(), subs.size(), "plan upload (subgrids)")) != IDG_OK) return rc;
  if ((rc = upload(&dp->samples, h.samples.data(), h.samples.size(), "plan upload (samples)")) != IDG_OK) return rc;
  if ((rc = upload(&dp->unplanned, h.unplanned.data(), h.unplanned.size(), "plan upload (unplanned)")) != IDG_OK)
    return rc;
  if ((rc = upload(&dp->lmn, lmn.data(), lmn.size(), "plan upload (lmn)")) != IDG_OK) return rc;
  if ((rc = upload(&dp->twiddle, tw.data(), tw.size(), "plan upload (twiddle)")) != IDG_OK) return rc;
  if ((rc = upload(&dp->sep, sep.data(), sep.size(), "plan upload (separable tables)")) != IDG_OK) return rc;
  if ((rc = upload(&dp->cross, cross.data(), cross.size(), "plan upload (separable tables)")) != IDG_OK) return rc;

  // cost-sorted work lists: gridder per batch (local indices), degridder over the plan
  const int64_t P = int64_t(h.subgrids.size());
  auto by_cost = [&](std::vector<int32_t> &ids, int64_t first) {
    std::stable_sort(ids.begin(), ids.end(), [&](int32_t x, int32_t y) {
      return h.subgrids[size_t(first + x)].nvis > h.subgrids[size_t(first + y)].nvis;
    });
  };
  std::vector<int32_t> degrid_order(static_cast<size_t>(P));
  for (int64_t i = 0; i < P; ++i) degrid_order[size_t(i)] = int32_t(i);
  by_cost(degrid_order, 0);
  std::stable_partition(degrid_order.begin(), degrid_order.end(),
                        [&](int32_t x) { return subs[size_t(x)].order >= 0; });
  for (int64_t i = 0; i < P; ++i) {
    const idg::DevSubgrid &r = subs[size_t(degrid_order[size_t(i)])];
    if (r.order >= 0)
      dp->degrid_n_sep++;
    else if (r.nvis > idg::degrid_small_threshold())
      dp->degrid_n_large++;
  }

  // per scratch batch: gridder order and adder items over tile lists
  dp->batch_size = batch_size_of(p);
  const int chunk = plan->tuning.adder_chunk > 0 ? plan->tuning.adder_chunk : 256;
  std::vector<int32_t> grid_order, all_contrib;
  std::vector<idg::AdderItem> all_items;
  std::vector<idg::CombineItem> all_combine;
  for (int64_t f = 0; f < P; f += dp->batch_size) {
    Batch b;
    b.first = f;
    b.count = std::min(dp->batch_size, P - f);
    std::vector<int32_t> ord(static_cast<size_t>(b.count));
    for (int64_t i = 0; i < b.count; ++i) ord[size_t(i)] = int32_t(i);
    by_cost(ord, f);
    // the separable-form subgrids first (each part still costliest first)
    std::stable_partition(ord.begin(), ord.end(), [&](int32_t x) { return subs[size_t(f + x)].order >= 0; });
    for (int32_t x : ord) b.n_sep += subs[size_t(f + x)].order >= 0 ? 1 : 0;
    b.order_off = int64_t(grid_order.size());
    grid_order.insert(grid_order.end(), ord.begin(), ord.end());
    TileLists tl;
    build_tile_lists(h.subgrids, b.first, b.count, p.grid_size, L, h.wlayer_min, h.nr_wlayers, tl);
    AdderPlan ap;
    build_adder_plan(tl, chunk, int64_t(all_contrib.size()), ap);
    all_contrib.insert(all_contrib.end(), tl.contrib.begin(), tl.contrib.end());
    b.item_off = int64_t(all_items.size());
    b.nitems = int64_t(ap.items.size());
    b.combine_off = int64_t(all_combine.size());
    b.ncombine = int64_t(ap.combine.size());
    b.nslots = ap.nslots;
    dp->max_slots = std::max<int64_t>(dp->max_slots, ap.nslots);
    all_items.insert(all_items.end(), ap.items.begin(), ap.items.end());
    all_combine.insert(all_combine.end(), ap.combine.begin(), ap.combine.end());
    dp->batches.push_back(b);
  }
  if ((rc = upload(&dp->grid_order, grid_order.data(), grid_order.size(), "plan upload (order)")) != IDG_OK)
    return rc;
  if ((rc = upload(&dp->degrid_order, degrid_order.data(), degrid_order.size(), "plan upload (order)")) != IDG_OK)
    return rc;
  if ((rc = upload(&dp->contrib, all_contrib.data(), all_contrib.size(), "plan upload (tiles)")) != IDG_OK) return rc;
  if ((rc = upload(&dp->items, all_items.data(), all_items.size(), "plan upload (adder)")) != IDG_OK) return rc;
  if ((rc = upload(&dp->combine, all_combine.data(), all_combine.size(), "plan upload (adder)")) != IDG_OK) return rc;
  HIP_TRY(hipDeviceGetAttribute(&dp->nr_cus, hipDeviceAttributeMultiprocessorCount, device), "CU count");
  *out = dp.get();
  plan->dev.emplace(device, std::move(dp));
  return IDG_OK;
}

// Twiddle table exp(-2 pi i k / L) per (device, L) for the standalone transform; kept for the process.
int device_twiddle(int L, const float2 **out) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, float2 *> cache;
  int device = 0;
  HIP_TRY(hipGetDevice(&device), "hipGetDevice");
  std::lock_guard<std::mutex> lock(mu);
  auto key = std::make_pair(device, L);
  auto it = cache.find(key);
  if (it == cache.end()) {
    std::vector<float4> lmn;
    std::vector<float2> tw;
    lmn_table(L, 1.0, lmn, tw);
    float2 *d = nullptr;
    int rc = upload(&d, tw.data(), tw.size(), "twiddle upload");
    if (rc != IDG_OK) return rc;
    it = cache.emplace(key, d).first;
  }
  *out = it->second;
  return IDG_OK;
}

int validate_params(const idg_params *p) {
  if (!p) return fail(IDG_EINVAL, "idg_plan: params is NULL");
  if (!idg::supported_subgrid_size(p->subgrid_size))
    return fail(IDG_EINVAL, "subgrid_size %d not supported (8, 16, 24, 32, 48 or 64)", p->subgrid_size);
  if (p->grid_size < p->subgrid_size || p->grid_size > 65536 || (p->grid_size & 1))
    return fail(IDG_EINVAL, "grid_size %d must be even and in [subgrid_size, 65536]", p->grid_size);
  if (p->kernel_size < 0 || p->kernel_size >= p->subgrid_size)
    return fail(IDG_EINVAL, "kernel_size %d must be in [0, subgrid_size)", p->kernel_size);
  if (p->max_timesteps < 1 || p->max_timesteps > 65535)
    return fail(IDG_EINVAL, "max_timesteps %d must be in [1, 65535]", p->max_timesteps);
  if (p->aterm_timesteps < 1) return fail(IDG_EINVAL, "aterm_timesteps must be >= 1");
  if (p->nr_stations < 2) return fail(IDG_EINVAL, "nr_stations must be >= 2");
  if (p->nr_baselines < 0 || p->nr_timesteps < 0 || p->nr_channels < 0 || p->nr_channels > 65535)
    return fail(IDG_EINVAL, "negative size or nr_channels > 65535");
  if (!(p->image_size > 0.0) || !(p->image_size <= 1.4))
    return fail(IDG_EINVAL, "image_size must be in (0, 1.4] (direction cosines)");
  if (p->scratch_bytes < 0) return fail(IDG_EINVAL, "scratch_bytes must be >= 0");
  if (!std::isfinite(p->w_step) || p->w_step < 0.0) return fail(IDG_EINVAL, "w_step must be finite and >= 0");
  if (p->flags & ~uint32_t(IDG_STRICT | IDG_PHASE_FP32)) return fail(IDG_EINVAL, "unknown flags 0x%x", p->flags);
  const int64_t total = int64_t(p->nr_baselines) * p->nr_timesteps * p->nr_channels;
  if (total > (int64_t(1) << 40)) return fail(IDG_EINVAL, "too many samples");
  return IDG_OK;
}

}  // namespace

extern "C" {

int idg_version(void) { return 10200; }

const char *idg_last_error(void) { return g_last_error.c_str(); }

int idg_plan(const idg_params *params, const int32_t *baselines, const double *uvw, const double *freqs,
             const uint8_t *flags, idg_plan_t *out) {
  if (!out) return fail(IDG_EINVAL, "idg_plan: out is NULL");
  *out = nullptr;
  int rc = validate_params(params);
  if (rc != IDG_OK) return rc;
  const idg_params &p = *params;
  const int64_t nbt = int64_t(p.nr_baselines) * p.nr_timesteps;
  if (p.nr_baselines > 0 && !baselines) return fail(IDG_EINVAL, "idg_plan: baselines is NULL");
  if (nbt > 0 && !uvw) return fail(IDG_EINVAL, "idg_plan: uvw is NULL");
  if (p.nr_channels > 0 && !freqs) return fail(IDG_EINVAL, "idg_plan: freqs is NULL");
  for (int b = 0; b < p.nr_baselines; ++b) {
    const int s1 = baselines[2 * b], s2 = baselines[2 * b + 1];
    if (s1 < 0 || s2 < 0 || s1 >= p.nr_stations || s2 >= p.nr_stations || s1 == s2)
      return fail(IDG_EINVAL, "idg_plan: baseline %d has invalid stations (%d, %d)", b, s1, s2);
  }
  for (int64_t i = 0; i < nbt * 3; ++i)
    if (!std::isfinite(uvw[i])) return fail(IDG_EINVAL, "idg_plan: uvw[%lld] is not finite", (long long)i);
  for (int c = 0; c < p.nr_channels; ++c)
    if (!std::isfinite(freqs[c]) || !(freqs[c] > 0.0))
      return fail(IDG_EINVAL, "idg_plan: freqs[%d] must be finite and > 0", c);
  if (p.w_step > 0.0 && nbt > 0 && p.nr_channels > 0) {  // layer indices stay far inside int32
    double wmax = 0.0, fmax = 0.0;
    for (int64_t i = 0; i < nbt; ++i) wmax = std::max(wmax, std::fabs(uvw[3 * i + 2]));
    for (int c = 0; c < p.nr_channels; ++c) fmax = std::max(fmax, freqs[c]);
    if (wmax * (fmax / idg::kSpeedOfLight) / p.w_step > 1e6)
      return fail(IDG_EINVAL, "idg_plan: w_step %g gives more than 1e6 W-layers", p.w_step);
  }
  idg_plan_s *plan = new (std::nothrow) idg_plan_s;
  if (!plan) return fail(IDG_ENOMEM, "idg_plan: out of host memory");
  std::string err;
  rc = idg::build_plan(p, baselines, uvw, freqs, flags, plan->host, err);
  if (rc != IDG_OK) {
    delete plan;
    return fail(rc, "%s", err.c_str());
  }
  if (int64_t(plan->host.subgrids.size()) >= (int64_t(1) << 31)) {  // subgrid indices are int32 on the device
    delete plan;
    return fail(IDG_EINVAL, "idg_plan: more than 2^31 - 1 subgrids");
  }
  if (int64_t(plan->host.nr_wlayers) * ((p.grid_size + idg::kAdderTile - 1) / idg::kAdderTile) *
          ((p.grid_size + idg::kAdderTile - 1) / idg::kAdderTile) >= (int64_t(1) << 31)) {
    delete plan;
    return fail(IDG_EINVAL, "idg_plan: W-layers x grid tiles exceed 2^31");
  }
  try {  // per subgrid the largest |w - w_0p| of its samples (separable form), in float64
    const idg::HostPlan &h = plan->host;
    plan->wmax.assign(h.subgrids.size(), 0.0);
    for (size_t i = 0; i < h.subgrids.size(); ++i) {
      const idg::SubgridRec &r = h.subgrids[i];
      const double w0 = double(r.wlayer) * p.w_step;
      double wm = 0.0;
      for (int64_t k = 0; k < r.nvis; ++k) {
        const uint32_t pk = h.samples[size_t(r.vis_offset + k)];
        const int t = r.t0 + int(pk >> 16), c = r.c0 + int(pk & 0xffffu);
        const double w = uvw[(int64_t(r.bl) * p.nr_timesteps + t) * 3 + 2] * (freqs[c] / idg::kSpeedOfLight);
        wm = std::max(wm, std::fabs(w - w0));
      }
      plan->wmax[i] = wm;
    }
  } catch (const std::bad_alloc &) {
    delete plan;
    return fail(IDG_ENOMEM, "idg_plan: out of host memory");
  }
  if ((p.flags & IDG_STRICT) && plan->host.nr_dropped > 0) {
    const long long nd = (long long)plan->host.nr_dropped;
    delete plan;
    return fail(IDG_ERANGE, "idg_plan: %lld unflagged samples do not fit a subgrid (IDG_STRICT)", nd);
  }
  *out = plan;
  return IDG_OK;
}

int idg_plan_stats(idg_plan_t plan, int64_t *nr_subgrids, int64_t *nr_gridded, int64_t *nr_dropped,
                   int64_t *nr_flagged) {
  if (!plan) return fail(IDG_EINVAL, "idg_plan_stats: plan is NULL");
  if (nr_subgrids) *nr_subgrids = int64_t(plan->host.subgrids.size());
  if (nr_gridded) *nr_gridded = plan->host.nr_gridded;
  if (nr_dropped) *nr_dropped = plan->host.nr_dropped;
  if (nr_flagged) *nr_flagged = plan->host.nr_flagged;
  return IDG_OK;
}

int idg_plan_sum_paths(idg_plan_t plan, int64_t *nr_subgrids, int64_t *nr_vis) {
  if (!plan) return fail(IDG_EINVAL, "idg_plan_sum_paths: plan is NULL");
  int64_t ns[3] = {0, 0, 0}, nv[3] = {0, 0, 0};
  const idg::HostPlan &h = plan->host;
  std::lock_guard<std::mutex> lock(plan->mu);
  if (separable_on(plan)) {
    std::vector<float2> sep;
    std::vector<float> cross;
    const double cmax = separable_tables(h.params.subgrid_size, h.params.image_size, sep, cross);
    for (size_t i = 0; i < h.subgrids.size(); ++i) {
      const int n = separable_order(plan->wmax[i], cmax, idg::separable_max_order());
      const int k = n < 0 ? 2 : n;
      ns[k] += 1;
      nv[k] += h.subgrids[i].nvis;
    }
  } else {
    ns[2] = int64_t(h.subgrids.size());
    for (const auto &r : h.subgrids) nv[2] += r.nvis;
  }
  for (int k = 0; k < 3; ++k) {
    if (nr_subgrids) nr_subgrids[k] = ns[k];
    if (nr_vis) nr_vis[k] = nv[k];
  }
  return IDG_OK;
}

int idg_plan_export(idg_plan_t plan, int64_t *subgrids, int32_t *samples) {
  if (!plan) return fail(IDG_EINVAL, "idg_plan_export: plan is NULL");
  const idg::HostPlan &h = plan->host;
  if (subgrids) {
    for (size_t i = 0; i < h.subgrids.size(); ++i) {
      const auto &r = h.subgrids[i];
      int64_t *o = subgrids + i * 13;
      o[0] = r.bl; o[1] = r.t0; o[2] = r.nt; o[3] = r.c0; o[4] = r.nc; o[5] = r.x0;
      o[6] = r.y0; o[7] = r.slot; o[8] = r.s1; o[9] = r.s2; o[10] = r.nvis; o[11] = r.vis_offset;
      o[12] = r.wlayer;
    }
  }
  if (samples) {
    for (const auto &r : h.subgrids)
      for (int64_t k = 0; k < r.nvis; ++k) {
        const uint32_t pk = h.samples[size_t(r.vis_offset + k)];
        samples[2 * (r.vis_offset + k)] = r.t0 + int32_t(pk >> 16);
        samples[2 * (r.vis_offset + k) + 1] = r.c0 + int32_t(pk & 0xffffu);
      }
  }
  return IDG_OK;
}

int idg_plan_wlayers(idg_plan_t plan, int32_t *wlayer_min, int32_t *nr_wlayers) {
  if (!plan) return fail(IDG_EINVAL, "idg_plan_wlayers: plan is NULL");
  if (wlayer_min) *wlayer_min = plan->host.wlayer_min;
  if (nr_wlayers) *nr_wlayers = plan->host.nr_wlayers;
  return IDG_OK;
}

void idg_plan_destroy(idg_plan_t plan) { delete plan; }

static void fill_kernel_args(const idg_plan_s *plan, const DevPlan *dp, idg::KernelArgs &a) {
  const idg_params &p = plan->host.params;
  a = idg::KernelArgs{};
  a.subgrids = dp->subgrids;
  a.samples = dp->samples;
  a.lmn = dp->lmn;
  a.twiddle = dp->twiddle;
  a.sep = dp->sep;
  a.cross = dp->cross;
  a.cross_exp = dp->cross_exp;
  a.nr_timesteps = p.nr_timesteps;
  a.nr_channels = p.nr_channels;
  a.grid_size = p.grid_size;
  a.image_size = p.image_size;
  a.phase_fp32 = (p.flags & IDG_PHASE_FP32) ? 1 : 0;
  a.chan_recur = plan->host.uniform_channels ? 1 : 0;
}

int idg_grid_subgrids(idg_plan_t plan, const double *uvw_d, const double *freqs_d, const idg_cf32 *vis_d,
                      const idg_cf32 *aterms_d, const float *taper_d, int64_t first, int64_t count, int32_t stage,
                      idg_cf32 *out_d, void *stream) {
  if (!plan) return fail(IDG_EINVAL, "idg_grid_subgrids: plan is NULL");
  const int64_t P = int64_t(plan->host.subgrids.size());
  if (first < 0 || count < 0 || first + count > P)
    return fail(IDG_EINVAL, "idg_grid_subgrids: range [%lld, %lld) outside [0, %lld)", (long long)first,
                (long long)(first + count), (long long)P);
  if (stage != 0 && stage != 1) return fail(IDG_EINVAL, "idg_grid_subgrids: stage must be 0 or 1");
  if (count == 0) return IDG_OK;
  if (!uvw_d || !freqs_d || !vis_d || !aterms_d || !taper_d || !out_d)
    return fail(IDG_EINVAL, "idg_grid_subgrids: NULL device pointer");
  DevPlan *dp = nullptr;
  int rc = device_plan(plan, &dp);
  if (rc != IDG_OK) return rc;
  idg::KernelArgs a;
  fill_kernel_args(plan, dp, a);
  a.uvw = uvw_d;
  a.freqs = freqs_d;
  a.vis_in = reinterpret_cast<const float2 *>(vis_d);
  a.aterms = reinterpret_cast<const float2 *>(aterms_d);
  a.taper = taper_d;
  a.subgrids_out = reinterpret_cast<float2 *>(out_d);
  a.stage = stage;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int L = plan->host.params.subgrid_size;
  for (int64_t f = 0; f < count; f += (int64_t(1) << 30)) {
    a.first = first + f;
    const int32_t n = int32_t(std::min<int64_t>(count - f, int64_t(1) << 30));
    a.subgrids_out = reinterpret_cast<float2 *>(out_d) + f * 4 * L * L;
    // as idg_grid: subgrids with an order >= 0 take the separable form, the others the direct sum
    std::vector<int32_t> ord;
    for (int32_t i = 0; i < n; ++i)
      if (dp->order[size_t(a.first + i)] >= 0) ord.push_back(i);
    const int32_t n_sep = int32_t(ord.size());
    if (n_sep == 0) {
      a.count = n;
      HIP_TRY(idg::launch_gridder(L, a, nullptr, s), "gridder launch");
      continue;
    }
    for (int32_t i = 0; i < n; ++i)
      if (dp->order[size_t(a.first + i)] < 0) ord.push_back(i);
    int32_t *ord_d = nullptr;
    HIP_TRY(scratch_alloc(reinterpret_cast<void **>(&ord_d), ord.size() * sizeof(int32_t), s),
            "idg_grid_subgrids: order list");
    hipError_t e = hipMemcpyAsync(ord_d, ord.data(), ord.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host list goes out of scope
    if (e == hipSuccess) {
      a.count = n_sep;
      e = idg::launch_gridder_mfma(L, a, ord_d, s);
    }
    if (e == hipSuccess && n > n_sep) {
      a.count = n - n_sep;
      e = idg::launch_gridder(L, a, ord_d + n_sep, s);
    }
    const hipError_t ef = hipFreeAsync(ord_d, s);
    HIP_TRY(e, "idg_grid_subgrids: gridder launch");
    HIP_TRY(ef, "idg_grid_subgrids: order list release");
  }
  return IDG_OK;
}

// Scratch of one idg_grid call: [queue counter (256 B)][partial tiles][subgrids].
struct GridScratch {
  char *base = nullptr;
  int32_t *counter = nullptr;
  float2 *partials = nullptr;
  float2 *subgrids = nullptr;
};



static bool degrid_wide(const idg_plan_s *plan) {
  return plan->tuning.degrid_shape == IDG_DEGRID_WIDE && !(plan->host.params.flags & IDG_PHASE_FP32);
}

// small: the degridder's kernel for subgrids of few visibilities
static int persistent_blocks(const idg_plan_s *plan, const DevPlan *dp, bool degrid, bool small = false) {
  const int L = plan->host.params.subgrid_size;
  const int want = degrid ? plan->tuning.degrid_blocks_per_cu : plan->tuning.grid_blocks_per_cu;
  const int per_cu =
      want > 0 ? want : idg::persistent_blocks_per_cu(L, degrid, degrid && degrid_wide(plan), degrid && small);
  return std::max(1, per_cu * dp->nr_cus);
}

// Bytes of one idg_grid call's scratch: the queue counter, the partial tiles of split adder lists and the
// transformed subgrids of one batch.
static size_t grid_scratch_bytes(const DevPlan *dp, int64_t nsub, int L) {
  return 256 + size_t(dp->max_slots) * 4 * idg::kAdderTile * idg::kAdderTile * sizeof(float2) +
         size_t(nsub) * 4 * size_t(L) * L * sizeof(float2);
}

static void carve_grid_scratch(char *base, int64_t slots, GridScratch &g) {
  g.base = base;
  g.counter = reinterpret_cast<int32_t *>(base);
  g.partials = reinterpret_cast<float2 *>(base + 256);
  g.subgrids = reinterpret_cast<float2 *>(base + 256 + size_t(slots) * 4 * idg::kAdderTile * idg::kAdderTile *
                                                       sizeof(float2));
}

static int alloc_grid_scratch(const DevPlan *dp, int64_t nsub, int L, hipStream_t s, GridScratch &g) {
  char *base = nullptr;
  HIP_TRY(scratch_alloc(reinterpret_cast<void **>(&base), grid_scratch_bytes(dp, nsub, L), s), "scratch allocation");
  carve_grid_scratch(base, dp->max_slots, g);
  return IDG_OK;
}

// The gridder and adder launches of idg_grid, batch by batch, with scratch g.
static hipError_t grid_launches(idg_plan_t plan, const DevPlan *dp, const double *uvw_d, const double *freqs_d,
                                const idg_cf32 *vis_d, const idg_cf32 *aterms_d, const float *taper_d,
                                idg_cf32 *grid_d, const GridScratch &g, hipStream_t s) {
  const idg_params &p = plan->host.params;
  const int L = p.subgrid_size;
  const bool persistent = plan->tuning.grid_form == IDG_FORM_PERSISTENT;
  const int nblocks = persistent ? persistent_blocks(plan, dp, false) : 0;
  idg::KernelArgs a;
  fill_kernel_args(plan, dp, a);
  a.uvw = uvw_d;
  a.freqs = freqs_d;
  a.vis_in = reinterpret_cast<const float2 *>(vis_d);
  a.aterms = reinterpret_cast<const float2 *>(aterms_d);
  a.taper = taper_d;
  a.subgrids_out = g.subgrids;
  a.stage = 1;
  a.pieces = 1;  // the adder reads each tile's piece of a subgrid as one block
  hipError_t err = hipSuccess;
  const int nblocks_sep = persistent ? std::max(1, (plan->tuning.grid_blocks_per_cu > 0 ? plan->tuning.grid_blocks_per_cu
                                                                                      : idg::mfma_gridder_blocks_per_cu(L)) *
                                                       dp->nr_cus)
                                     : 0;
  for (const Batch &b : dp->batches) {
    a.first = b.first;
    const int32_t *ord = dp->grid_order + b.order_off;
    {
      // separable form (matrix cores) over ord[0 .. n_sep), direct sum over the rest; two queue counters
      StageTimer tm(IDG_STAGE_GRIDDER, s);
      a.count = int32_t(b.n_sep);
      // plain form with every subgrid of the batch separable: plan order (no list to load first)
      err = persistent ? idg::launch_gridder_mfma_persistent(L, a, ord, g.counter, nblocks_sep, s)
                       : idg::launch_gridder_mfma(L, a, b.n_sep == b.count ? nullptr : ord, s);
      if (err == hipSuccess) {
        a.count = int32_t(b.count - b.n_sep);
        err = persistent ? idg::launch_gridder_persistent(L, a, ord + b.n_sep, g.counter + 1, nblocks, s)
                         : idg::launch_gridder(L, a, ord + b.n_sep, s);
      }
    }
    if (err != hipSuccess) break;
    idg::AdderArgs ad{};
    ad.subgrids = dp->subgrids;
    ad.first = b.first;
    ad.items = dp->items + b.item_off;
    ad.combine = dp->combine + b.combine_off;
    ad.contrib = dp->contrib;
    ad.subgrids_in = g.subgrids;
    ad.grid = reinterpret_cast<float2 *>(grid_d);
    ad.partials = g.partials;
    ad.nitems = int32_t(b.nitems);
    ad.ncombine = int32_t(b.ncombine);
    ad.ntx = (p.grid_size + idg::kAdderTile - 1) / idg::kAdderTile;
    ad.grid_size = p.grid_size;
    ad.pieces = 1;
    {
      StageTimer tm(IDG_STAGE_ADDER, s);
      err = idg::launch_adder(L, ad, s);
    }
    if (err != hipSuccess) break;
  }
  return err;
}

int idg_grid(idg_plan_t plan, const double *uvw_d, const double *freqs_d, const idg_cf32 *vis_d,
             const idg_cf32 *aterms_d, const float *taper_d, idg_cf32 *grid_d, void *stream) {
  if (!plan) return fail(IDG_EINVAL, "idg_grid: plan is NULL");
  if (plan->host.subgrids.empty()) return IDG_OK;
  if (!uvw_d || !freqs_d || !vis_d || !aterms_d || !taper_d || !grid_d)
    return fail(IDG_EINVAL, "idg_grid: NULL device pointer");
  DevPlan *dp = nullptr;
  int rc = device_plan(plan, &dp);
  if (rc != IDG_OK) return rc;
  const int L = plan->host.params.subgrid_size;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t nb = std::min<int64_t>(dp->batch_size, int64_t(plan->host.subgrids.size()));
  GridScratch g;
  if ((rc = alloc_grid_scratch(dp, nb, L, s, g)) != IDG_OK) return rc;
  const hipError_t err = grid_launches(plan, dp, uvw_d, freqs_d, vis_d, aterms_d, taper_d, grid_d, g, s);
  hipError_t ef = hipFreeAsync(g.base, s);
  if (err != hipSuccess) return hip_fail(err, "idg_grid: launch");
  HIP_TRY(ef, "idg_grid: scratch release");
  return IDG_OK;
}

// The plan's device metadata on the current device, without uploading it.
static int resident_device_plan(idg_plan_t plan, const char *fn, DevPlan **out) {
  int device = 0;
  HIP_TRY(hipGetDevice(&device), "hipGetDevice");
  std::lock_guard<std::mutex> lock(plan->mu);
  auto it = plan->dev.find(device);
  if (it == plan->dev.end())
    return fail(IDG_ESTATE, "%s: the plan has no device copy on device %d (an idg_grid, idg_degrid or "
                "idg_grid_subgrids call with this plan on this device makes one)", fn, device);
  *out = it->second.get();
  return IDG_OK;
}

int idg_grid_noalloc(idg_plan_t plan, const double *uvw_d, const double *freqs_d, const idg_cf32 *vis_d,
                     const idg_cf32 *aterms_d, const float *taper_d, idg_cf32 *grid_d, void *stream) {
  if (!plan) return fail(IDG_EINVAL, "idg_grid_noalloc: plan is NULL");
  if (plan->host.subgrids.empty()) return IDG_OK;
  if (!uvw_d || !freqs_d || !vis_d || !aterms_d || !taper_d || !grid_d)
    return fail(IDG_EINVAL, "idg_grid_noalloc: NULL device pointer");
  DevPlan *dp = nullptr;
  int rc = resident_device_plan(plan, "idg_grid_noalloc", &dp);
  if (rc != IDG_OK) return rc;
  const int L = plan->host.params.subgrid_size;
  const int64_t nb = std::min<int64_t>(dp->batch_size, int64_t(plan->host.subgrids.size()));
  const size_t need = grid_scratch_bytes(dp, nb, L);
  if (need > idg::kNoAllocScratchBytes)
    return fail(IDG_ERANGE, "idg_grid_noalloc: the plan needs %zu bytes of scratch per call (batches of %lld "
                "subgrids), above the fixed %zu; plan with a smaller scratch_bytes", need, (long long)nb,
                idg::kNoAllocScratchBytes);
  void *base = nullptr;
  HIP_TRY(idg::noalloc_scratch(&base), "idg_grid_noalloc: scratch address");
  GridScratch g;
  carve_grid_scratch(static_cast<char *>(base), dp->max_slots, g);
  const hipError_t err = grid_launches(plan, dp, uvw_d, freqs_d, vis_d, aterms_d, taper_d, grid_d, g,
                                       static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "idg_grid_noalloc: launch");
  return IDG_OK;
}

int idg_degrid(idg_plan_t plan, const double *uvw_d, const double *freqs_d, const idg_cf32 *grid_d,
               const idg_cf32 *aterms_d, const float *taper_d, idg_cf32 *vis_d, void *stream) {
  if (!plan) return fail(IDG_EINVAL, "idg_degrid: plan is NULL");
  const idg::HostPlan &h = plan->host;
  if (h.subgrids.empty() && h.unplanned.empty()) return IDG_OK;
  if (!uvw_d || !freqs_d || !grid_d || !aterms_d || !taper_d || !vis_d)
    return fail(IDG_EINVAL, "idg_degrid: NULL device pointer");
  DevPlan *dp = nullptr;
  int rc = device_plan(plan, &dp);
  if (rc != IDG_OK) return rc;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (!h.unplanned.empty()) {
    StageTimer tm(IDG_STAGE_ZERO, s);
    HIP_TRY(idg::launch_zero_samples(dp->unplanned, int64_t(h.unplanned.size()), reinterpret_cast<float2 *>(vis_d), s),
            "idg_degrid: zero launch");
  }
  idg::KernelArgs a;
  fill_kernel_args(plan, dp, a);
  a.uvw = uvw_d;
  a.freqs = freqs_d;
  a.grid_in = reinterpret_cast<const float2 *>(grid_d);
  a.vis_out = reinterpret_cast<float2 *>(vis_d);
  a.aterms = reinterpret_cast<const float2 *>(aterms_d);
  a.taper = taper_d;
  const int64_t P = int64_t(h.subgrids.size());
  const int L = h.params.subgrid_size;
  if (P == 0) return IDG_OK;
  a.first = 0;
  a.count = int32_t(P);
  if (plan->tuning.degrid_form == IDG_FORM_PERSISTENT) {
    int32_t *counter = nullptr;  // queue counters: large and small subgrids of the direct sum, separable form
    HIP_TRY(scratch_alloc(reinterpret_cast<void **>(&counter), 256, s), "idg_degrid: queue counter");
    hipError_t err;
    {
      StageTimer tm(IDG_STAGE_DEGRIDDER, s);
      const int want = plan->tuning.degrid_blocks_per_cu;
      const int nb_sep = std::max(1, (want > 0 ? want : idg::mfma_degridder_blocks_per_cu(L)) * dp->nr_cus);
      err = idg::launch_degridder_persistent(L, a, degrid_wide(plan), dp->degrid_order, dp->degrid_n_sep,
                                             dp->degrid_n_large, counter, nb_sep, persistent_blocks(plan, dp, true),
                                             persistent_blocks(plan, dp, true, true), s);
    }
    hipError_t ef = hipFreeAsync(counter, s);
    if (err != hipSuccess) return hip_fail(err, "idg_degrid: launch");
    HIP_TRY(ef, "idg_degrid: counter release");
    return IDG_OK;
  }
  StageTimer tm(IDG_STAGE_DEGRIDDER, s);
  HIP_TRY(idg::launch_degridder(L, a, degrid_wide(plan), dp->degrid_order, dp->degrid_n_sep, dp->degrid_n_large, s),
          "idg_degrid: launch");
  return IDG_OK;
}

int idg_plan_set_tuning(idg_plan_t plan, const idg_tuning *t) {
  if (!plan || !t) return fail(IDG_EINVAL, "idg_plan_set_tuning: NULL argument");
  for (int32_t f : {t->grid_form, t->degrid_form})
    if (f != IDG_FORM_PLAIN && f != IDG_FORM_PERSISTENT)
      return fail(IDG_EINVAL, "idg_plan_set_tuning: unknown form %d", f);
  for (int32_t b : {t->grid_blocks_per_cu, t->degrid_blocks_per_cu})
    if (b < 0 || b > 64) return fail(IDG_EINVAL, "idg_plan_set_tuning: blocks_per_cu must be in [0, 64]");
  if (t->adder_chunk < 0) return fail(IDG_EINVAL, "idg_plan_set_tuning: adder_chunk must be >= 0");
  if (t->degrid_shape != IDG_DEGRID_STANDARD && t->degrid_shape != IDG_DEGRID_WIDE)
    return fail(IDG_EINVAL, "idg_plan_set_tuning: unknown degrid_shape %d", t->degrid_shape);
  if (t->sum_path != IDG_SUM_AUTO && t->sum_path != IDG_SUM_DIRECT)
    return fail(IDG_EINVAL, "idg_plan_set_tuning: unknown sum_path %d", t->sum_path);
  if (t->reserved) return fail(IDG_EINVAL, "idg_plan_set_tuning: reserved must be 0");
  std::lock_guard<std::mutex> lock(plan->mu);
  // adder items depend on the chunk length, the gridder work lists on the sum path
  const bool rebuild = t->adder_chunk != plan->tuning.adder_chunk || t->sum_path != plan->tuning.sum_path;
  plan->tuning = *t;
  if (rebuild) plan->dev.clear();  // rebuilt on next use
  return IDG_OK;
}

int idg_plan_get_tuning(idg_plan_t plan, idg_tuning *t) {
  if (!plan || !t) return fail(IDG_EINVAL, "idg_plan_get_tuning: NULL argument");
  std::lock_guard<std::mutex> lock(plan->mu);
  *t = plan->tuning;
  return IDG_OK;
}

// Validation shared by the two image steps.
static int image_args(const char *fn, const void *src, int32_t N, const float *cl, const float *cm, const void *dst) {
  if (!idg::image_size_supported(N)) return fail(IDG_EINVAL, "%s: grid_size %d is not a power of two in [64, 16384]", fn, N);
  if (!src || !dst) return fail(IDG_EINVAL, "%s: NULL device pointer", fn);
  if ((cl == nullptr) != (cm == nullptr)) return fail(IDG_EINVAL, "%s: give both corrections or neither", fn);
  const size_t bytes = size_t(4) * N * N * sizeof(idg_cf32);
  const char *a = static_cast<const char *>(src), *b = static_cast<const char *>(dst);
  if (a != b && a < b + bytes && b < a + bytes) return fail(IDG_EINVAL, "%s: input and output overlap partially", fn);
  return IDG_OK;
}

// The image steps: N/2 twiddles in stream-ordered scratch, two passes.
static int image_transform(const char *fn, bool to_image, const idg_cf32 *src_d, int32_t N, const float *cl,
                           const float *cm, idg_cf32 *dst_d, void *stream) {
  int rc = image_args(fn, src_d, N, cl, cm, dst_d);
  if (rc != IDG_OK) return rc;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const float2 *in = reinterpret_cast<const float2 *>(src_d);
  float2 *out = reinterpret_cast<float2 *>(dst_d);
  // twiddles, plus a [4][N][N] intermediate for in-place calls of the four-step form
  const size_t nscr = idg::image_needs_scratch(N, in, out) ? size_t(4) * N * N : 0;
  float2 *tw = nullptr;
  HIP_TRY(scratch_alloc(reinterpret_cast<void **>(&tw), (size_t(N) / 2 + nscr) * sizeof(float2), s),
          "image scratch");
  float2 *scr = nscr ? tw + N / 2 : nullptr;
  hipError_t e = idg::launch_image_twiddles(tw, N, s);
  if (e == hipSuccess)
    e = to_image ? idg::launch_grid_to_image(in, out, N, cl, cm, tw, scr, s)
                 : idg::launch_image_to_grid(in, out, N, cl, cm, tw, scr, s);
  const hipError_t ef = hipFreeAsync(tw, s);
  if (e != hipSuccess) return hip_fail(e, to_image ? "idg_grid_to_image: launch" : "idg_image_to_grid: launch");
  HIP_TRY(ef, "image twiddles release");
  return IDG_OK;
}

int idg_grid_to_image(const idg_cf32 *grid_d, int32_t grid_size, const float *corr_l_d, const float *corr_m_d,
                      idg_cf32 *image_d, void *stream) {
  return image_transform("idg_grid_to_image", true, grid_d, grid_size, corr_l_d, corr_m_d, image_d, stream);
}

int idg_image_to_grid(const idg_cf32 *image_d, int32_t grid_size, const float *corr_l_d, const float *corr_m_d,
                      idg_cf32 *grid_d, void *stream) {
  return image_transform("idg_image_to_grid", false, image_d, grid_size, corr_l_d, corr_m_d, grid_d, stream);
}

// W-stacked image steps: one layer at a time through a [4][N][N] scratch.
static int wstack_args(const char *fn, const void *image, const void *grids, int32_t N, double S, int32_t nl,
                       const double *w0s, const float *cl, const float *cm) {
  if (!idg::image_size_supported(N)) return fail(IDG_EINVAL, "%s: grid_size %d is not a power of two in [64, 16384]", fn, N);
  if (!(S > 0.0) || !(S <= 1.4)) return fail(IDG_EINVAL, "%s: image_size must be in (0, 1.4]", fn);
  if (nl < 1 || nl > 65536) return fail(IDG_EINVAL, "%s: nr_wlayers %d outside [1, 65536]", fn, nl);
  if (!image || !grids || !w0s) return fail(IDG_EINVAL, "%s: NULL pointer", fn);
  if ((cl == nullptr) != (cm == nullptr)) return fail(IDG_EINVAL, "%s: give both corrections or neither", fn);
  for (int j = 0; j < nl; ++j)
    if (!std::isfinite(w0s[j])) return fail(IDG_EINVAL, "%s: w0s[%d] is not finite", fn, j);
  const size_t layer = size_t(4) * N * N * sizeof(idg_cf32);
  const char *a = static_cast<const char *>(image), *b = static_cast<const char *>(grids);
  if (a < b + layer * size_t(nl) && b < a + layer) return fail(IDG_EINVAL, "%s: image and grids overlap", fn);
  return IDG_OK;
}

int idg_wstack_to_image(const idg_cf32 *grids_d, int32_t nr_wlayers, const double *w0s, int32_t grid_size,
                        double image_size, const float *corr_l_d, const float *corr_m_d, idg_cf32 *image_d,
                        void *stream) {
  int rc = wstack_args("idg_wstack_to_image", image_d, grids_d, grid_size, image_size, nr_wlayers, w0s, corr_l_d,
                       corr_m_d);
  if (rc != IDG_OK) return rc;
  const int N = grid_size;
  const size_t nn = size_t(4) * N * N;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  float2 *scr = nullptr;
  HIP_TRY(scratch_alloc(reinterpret_cast<void **>(&scr), (nn + size_t(N) / 2) * sizeof(float2), s),
          "idg_wstack_to_image: scratch");
  float2 *tw = scr + nn;
  const float2 *g = reinterpret_cast<const float2 *>(grids_d);
  float2 *img = reinterpret_cast<float2 *>(image_d);
  hipError_t e = idg::launch_image_twiddles(tw, N, s);
  for (int j = 0; j < nr_wlayers && e == hipSuccess; ++j)
    e = idg::launch_wlayer_to_image(g + nn * j, img, scr, N, image_size, w0s[j], j > 0, corr_l_d, corr_m_d, tw, s);
  const hipError_t ef = hipFreeAsync(scr, s);
  if (e != hipSuccess) return hip_fail(e, "idg_wstack_to_image: launch");
  HIP_TRY(ef, "idg_wstack_to_image: scratch release");
  return IDG_OK;
}

int idg_image_to_wstack(const idg_cf32 *image_d, int32_t grid_size, double image_size, const float *corr_l_d,
                        const float *corr_m_d, int32_t nr_wlayers, const double *w0s, idg_cf32 *grids_d,
                        void *stream) {
  int rc = wstack_args("idg_image_to_wstack", image_d, grids_d, grid_size, image_size, nr_wlayers, w0s, corr_l_d,
                       corr_m_d);
  if (rc != IDG_OK) return rc;
  const int N = grid_size;
  const size_t nn = size_t(4) * N * N;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  float2 *scr = nullptr;
  HIP_TRY(scratch_alloc(reinterpret_cast<void **>(&scr), (nn + size_t(N) / 2) * sizeof(float2), s),
          "idg_image_to_wstack: scratch");
  float2 *tw = scr + nn;
  const float2 *img = reinterpret_cast<const float2 *>(image_d);
  float2 *g = reinterpret_cast<float2 *>(grids_d);
  hipError_t e = idg::launch_image_twiddles(tw, N, s);
  for (int j = 0; j < nr_wlayers && e == hipSuccess; ++j)
    e = idg::launch_image_to_wlayer(img, g + nn * j, scr, N, image_size, w0s[j], corr_l_d, corr_m_d, tw, s);
  const hipError_t ef = hipFreeAsync(scr, s);
  if (e != hipSuccess) return hip_fail(e, "idg_image_to_wstack: launch");
  HIP_TRY(ef, "idg_image_to_wstack: scratch release");
  return IDG_OK;
}

static int taper_args(const char *fn, int32_t L, double max_shift) {
  if (L < 4 || L > 256) return fail(IDG_EINVAL, "%s: L = %d outside [4, 256]", fn, L);
  if (!std::isfinite(max_shift) || max_shift <= 0.0 || max_shift > 0.5 * double(L))
    return fail(IDG_EINVAL, "%s: max_shift = %g outside (0, L/2]", fn, max_shift);
  return IDG_OK;
}

int idg_taper_optimal(int32_t L, double max_shift, double *taper_out, double *eps_out) {
  int rc = taper_args("idg_taper_optimal", L, max_shift);
  if (rc != IDG_OK) return rc;
  if (!taper_out || !eps_out) return fail(IDG_EINVAL, "idg_taper_optimal: NULL output");
  try {
    rc = idg::optimal_taper(L, max_shift, taper_out, eps_out);
  } catch (const std::bad_alloc &) {
    return fail(IDG_ENOMEM, "idg_taper_optimal: host allocation");
  }
  if (rc == IDG_ERANGE)
    return fail(IDG_ERANGE, "idg_taper_optimal: eps^2 = %.3g is below float64 resolution (L = %d, max_shift = %g)",
                *eps_out * *eps_out, L, max_shift);
  return rc;
}

int idg_taper_correction(int32_t L, double max_shift, const double *taper, int32_t N, float *corr_out) {
  int rc = taper_args("idg_taper_correction", L, max_shift);
  if (rc != IDG_OK) return rc;
  if (N < 2 || N > (1 << 20)) return fail(IDG_EINVAL, "idg_taper_correction: N = %d outside [2, 2^20]", N);
  if (!taper || !corr_out) return fail(IDG_EINVAL, "idg_taper_correction: NULL pointer");
  try {
    idg::taper_correction(L, max_shift, taper, N, corr_out);
  } catch (const std::bad_alloc &) {
    return fail(IDG_ENOMEM, "idg_taper_correction: host allocation");
  }
  return IDG_OK;
}

int idg_subgrid_fft(idg_cf32 *data_d, int64_t count, int32_t subgrid_size, int32_t direction, void *stream) {
  if (!idg::supported_subgrid_size(subgrid_size))
    return fail(IDG_EINVAL, "idg_subgrid_fft: subgrid_size %d not supported", subgrid_size);
  if (direction != -1 && direction != 1) return fail(IDG_EINVAL, "idg_subgrid_fft: direction must be -1 or +1");
  if (count < 0 || count > (int64_t(1) << 31) - 1) return fail(IDG_EINVAL, "idg_subgrid_fft: bad count");
  if (count == 0) return IDG_OK;
  if (!data_d) return fail(IDG_EINVAL, "idg_subgrid_fft: data is NULL");
  const float2 *tw = nullptr;
  int rc = device_twiddle(subgrid_size, &tw);
  if (rc != IDG_OK) return rc;
  HIP_TRY(idg::launch_subgrid_fft(subgrid_size, reinterpret_cast<float2 *>(data_d), count, direction, tw,
                                  static_cast<hipStream_t>(stream)),
          "idg_subgrid_fft: launch");
  return IDG_OK;
}

int idg_add_subgrids(idg_plan_t plan, const idg_cf32 *subgrids_d, int64_t first, int64_t count, idg_cf32 *grid_d,
                     void *stream) {
  if (!plan) return fail(IDG_EINVAL, "idg_add_subgrids: plan is NULL");
  const idg::HostPlan &h = plan->host;
  const int64_t P = int64_t(h.subgrids.size());
  if (first < 0 || count < 0 || first + count > P || count > (int64_t(1) << 31) - 1)
    return fail(IDG_EINVAL, "idg_add_subgrids: bad range");
  if (count == 0) return IDG_OK;
  if (!subgrids_d || !grid_d) return fail(IDG_EINVAL, "idg_add_subgrids: NULL device pointer");
  DevPlan *dp = nullptr;
  int rc = device_plan(plan, &dp);
  if (rc != IDG_OK) return rc;
  const idg_params &p = h.params;
  TileLists tl;
  AdderPlan ap;
  try {
    build_tile_lists(h.subgrids, first, count, p.grid_size, p.subgrid_size, h.wlayer_min, h.nr_wlayers, tl);
    build_adder_plan(tl, plan->tuning.adder_chunk > 0 ? plan->tuning.adder_chunk : 256, 0, ap);
  } catch (const std::bad_alloc &) {
    return fail(IDG_ENOMEM, "idg_add_subgrids: out of host memory");
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t b_items = ap.items.size() * sizeof(idg::AdderItem);
  const size_t b_comb = ap.combine.size() * sizeof(idg::CombineItem);
  const size_t b_con = tl.contrib.size() * sizeof(int32_t);
  const size_t b_part = size_t(ap.nslots) * 4 * idg::kAdderTile * idg::kAdderTile * sizeof(float2);
  auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
  char *buf = nullptr;
  HIP_TRY(scratch_alloc(reinterpret_cast<void **>(&buf), align(b_items) + align(b_comb) + align(b_con) + b_part + 256,
                         s),
          "idg_add_subgrids: allocation");
  char *p_items = buf, *p_comb = p_items + align(b_items), *p_con = p_comb + align(b_comb);
  char *p_part = p_con + align(b_con);
  hipError_t err = hipMemcpyAsync(p_items, ap.items.data(), b_items, hipMemcpyHostToDevice, s);
  if (err == hipSuccess && b_comb) err = hipMemcpyAsync(p_comb, ap.combine.data(), b_comb, hipMemcpyHostToDevice, s);
  if (err == hipSuccess) err = hipMemcpyAsync(p_con, tl.contrib.data(), b_con, hipMemcpyHostToDevice, s);
  if (err == hipSuccess) {
    idg::AdderArgs ad{};
    ad.subgrids = dp->subgrids;
    ad.first = first;
    ad.items = reinterpret_cast<const idg::AdderItem *>(p_items);
    ad.combine = reinterpret_cast<const idg::CombineItem *>(p_comb);
    ad.contrib = reinterpret_cast<const int32_t *>(p_con);
    ad.subgrids_in = reinterpret_cast<const float2 *>(subgrids_d);
    ad.grid = reinterpret_cast<float2 *>(grid_d);
    ad.partials = reinterpret_cast<float2 *>(p_part);
    ad.nitems = int32_t(ap.items.size());
    ad.ncombine = int32_t(ap.combine.size());
    ad.ntx = (p.grid_size + idg::kAdderTile - 1) / idg::kAdderTile;
    ad.grid_size = p.grid_size;
    err = idg::launch_adder(p.subgrid_size, ad, s);
  }
  // the host lists must outlive the copies
  hipError_t es = hipStreamSynchronize(s);
  hipError_t ef = hipFreeAsync(buf, s);
  if (err != hipSuccess) return hip_fail(err, "idg_add_subgrids");
  HIP_TRY(es, "idg_add_subgrids: synchronize");
  HIP_TRY(ef, "idg_add_subgrids: release");
  return IDG_OK;
}

int idg_split_subgrids(idg_plan_t plan, const idg_cf32 *grid_d, int64_t first, int64_t count, idg_cf32 *subgrids_d,
                       void *stream) {
  if (!plan) return fail(IDG_EINVAL, "idg_split_subgrids: plan is NULL");
  const int64_t P = int64_t(plan->host.subgrids.size());
  if (first < 0 || count < 0 || first + count > P || count > (int64_t(1) << 31) - 1)
    return fail(IDG_EINVAL, "idg_split_subgrids: bad range");
  if (count == 0) return IDG_OK;
  if (!subgrids_d || !grid_d) return fail(IDG_EINVAL, "idg_split_subgrids: NULL device pointer");
  DevPlan *dp = nullptr;
  int rc = device_plan(plan, &dp);
  if (rc != IDG_OK) return rc;
  const idg_params &p = plan->host.params;
  HIP_TRY(idg::launch_splitter(p.subgrid_size, dp->subgrids, first, count, reinterpret_cast<const float2 *>(grid_d),
                               p.grid_size, reinterpret_cast<float2 *>(subgrids_d), static_cast<hipStream_t>(stream)),
          "idg_split_subgrids: launch");
  return IDG_OK;
}

int idg_profile(int enable) {
  Profiler &p = profiler();
  std::lock_guard<std::mutex> lock(p.mu);
  p.on = enable != 0;
  return IDG_OK;
}

int idg_profile_read(double *ms, int64_t *launches, int reset) {
  Profiler &p = profiler();
  std::vector<Profiler::Rec> recs;
  {
    std::lock_guard<std::mutex> lock(p.mu);
    recs.swap(p.pending);
  }
  hipError_t err = hipSuccess;
  double add_ms[IDG_NR_STAGES] = {};
  int64_t add_n[IDG_NR_STAGES] = {};
  for (auto &r : recs) {
    float t = 0.0f;
    hipError_t e = hipEventSynchronize(r.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.start, r.stop);
    if (e == hipSuccess) {
      add_ms[r.stage] += t;
      add_n[r.stage] += 1;
    } else if (err == hipSuccess) {
      err = e;
    }
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  std::lock_guard<std::mutex> lock(p.mu);
  for (int i = 0; i < IDG_NR_STAGES; ++i) {
    p.ms[i] += add_ms[i];
    p.launches[i] += add_n[i];
    if (ms) ms[i] = p.ms[i];
    if (launches) launches[i] = p.launches[i];
    if (reset) {
      p.ms[i] = 0.0;
      p.launches[i] = 0;
    }
  }
  if (err != hipSuccess) return hip_fail(err, "idg_profile_read");
  return IDG_OK;
}

int idg_trim_scratch(uint64_t keep_bytes) {
  hipMemPool_t pool = nullptr;
  HIP_TRY(scratch_pool(&pool), "idg_trim_scratch: pool");
  HIP_TRY(hipDeviceSynchronize(), "idg_trim_scratch: synchronise");
  HIP_TRY(hipMemPoolTrimTo(pool, size_t(keep_bytes)), "idg_trim_scratch");
  return IDG_OK;
}

int idg_device_rates(double *fp32_fma_flops, double *sincos_instr, double *fp16_mfma_flops) {
  if (!fp32_fma_flops || !sincos_instr || !fp16_mfma_flops) return fail(IDG_EINVAL, "idg_device_rates: NULL pointer");
  HIP_TRY(idg::measure_device_rates(fp32_fma_flops, sincos_instr, fp16_mfma_flops), "idg_device_rates");
  return IDG_OK;
}

int idg_sync(void *stream) {
  HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "idg_sync");
  HIP_TRY(hipGetLastError(), "idg_sync");
  return IDG_OK;
}

}  // extern "C"
