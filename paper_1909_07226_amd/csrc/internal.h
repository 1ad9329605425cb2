// Shared between the C-ABI implementation (api.cpp) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "idg.h"

namespace idg {

// Device copy of one subgrid record.
struct alignas(16) DevSubgrid {
  int32_t bl, t0, c0, nvis;
  int32_t x0, y0;
  int32_t a1, a2;      // Jones block index (slot * nr_stations + station) of stations s1, s2
  int64_t vis_offset;  // first packed sample of this subgrid
  double w0;           // w offset of the subgrid's W-layer, wavelengths (0 without layers)
  int32_t layer;       // index of that layer's [4][N][N] grid
  int16_t order;       // separable form: expansion order of the cross term (-1: direct sum only)
  int16_t wexp;        // separable form: |w - w0| <= 2^wexp over the subgrid's samples
};
static_assert(sizeof(DevSubgrid) == 64, "DevSubgrid layout");

// Arguments of the gridder / degridder kernels.
struct KernelArgs {
  const DevSubgrid *subgrids;  // plan subgrids (device)
  const uint32_t *samples;     // packed (dt << 16 | dc) per planned sample
  const double *uvw;           // [nbl][nt][3] metres
  const double *freqs;         // [nch] Hz
  const float2 *vis_in;        // gridder: [nbl][nt][nch][4]
  float2 *vis_out;             // degridder: [nbl][nt][nch][4]
  const float2 *aterms;        // [nslot][nst][L*L][4]
  const float *taper;          // [L*L]
  const float4 *lmn;           // [L*L] (l, m, n', 0) float32 from float64
  const float2 *twiddle;       // [L] exp(-2 pi i k / L)
  const float2 *sep;           // [L] (x_q, sqrt(1 - x_q^2) - 1), x_q = (q - L/2) S / L (separable form)
  const float *cross;          // [L*L] n'_ij - a_i - a_j (separable form)
  int32_t cross_exp;           // separable form: max |c_ij| <= 2^cross_exp
  const float2 *grid_in;       // degridder: [4][N][N]
  float2 *subgrids_out;        // gridder: [count][4][L*L]
  int64_t first;               // first plan subgrid of this launch
  int32_t count;               // subgrids in this launch
  int32_t nr_timesteps, nr_channels;
  int32_t grid_size;
  double image_size;
  int32_t stage;       // gridder: 0 = image after A-terms and taper, 1 = after the DFT
  int32_t phase_fp32;  // 1: subgrid offsets in float32 (precision study)
  int32_t chan_recur;  // 1: channel frequencies are uniformly spaced (phasor recurrence over channels)
  int32_t pieces;      // gridder: 1 = store subgrids in the adder's tile-piece layout, 0 = [4][L][L]
};

// Adder tile: TILE x TILE pixels of one polarisation.
constexpr int kAdderTile = 32;

// A run of one tile's contribution list; slot < 0: add into the grid,
// slot >= 0: sum into partial tile `slot` (combined afterwards).
struct AdderItem {
  int32_t tile, begin, end, slot;
};

// A tile whose list was split: partial slots [slot_begin, slot_end) in order.
struct CombineItem {
  int32_t tile, slot_begin, slot_end, pad;
};

struct AdderArgs {
  const DevSubgrid *subgrids;  // plan subgrids (device)
  int64_t first;               // plan index of local subgrid 0
  const AdderItem *items;      // [nitems]
  const CombineItem *combine;  // [ncombine]
  const int32_t *contrib;      // local subgrid indices, ascending per tile
  const float2 *subgrids_in;   // [count][4][L*L]
  float2 *grid;                // [4][N][N]
  float2 *partials;            // [slots][4][TILE*TILE]
  int32_t nitems, ncombine, ntx, grid_size;
  int32_t pieces;              // 1: subgrids_in in the tile-piece layout of the gridder, 0: [4][L][L]
};

bool supported_subgrid_size(int L);

// Gridder, direct sum on the VALU: a.count subgrids, local indices order[0 .. count) (order NULL: 0 .. count).
hipError_t launch_gridder(int L, const KernelArgs &a, const int32_t *order, hipStream_t s);
// Gridder, separable form on the matrix cores (L = 32 only; subgrids with 0 <= order <= separable_max_order()):
// local indices order[0 .. count) (order NULL: 0 .. count).
int separable_max_order();
bool separable_supported(int L);
hipError_t launch_gridder_mfma(int L, const KernelArgs &a, const int32_t *order, hipStream_t s);
hipError_t launch_gridder_mfma_persistent(int L, const KernelArgs &a, const int32_t *order, int32_t *queue_head,
                                          int nblocks, hipStream_t s);
// Degridder: `order` holds a.count global subgrid indices: the n_sep subgrids of the separable form first,
// then the others sorted by visibility count, costliest first; the first n_large of those have more than
// degrid_small_threshold() visibilities (they run the visibility-per-lane kernel, the rest the
// pixel-per-lane kernel).
int degrid_small_threshold();
hipError_t launch_degridder(int L, const KernelArgs &a, bool wide, const int32_t *order, int64_t n_sep,
                            int64_t n_large, hipStream_t s);
// persistent forms: `order` holds a.count items; the gridder's *queue_head (one counter) and the
// degridder's queue_head[0..2] (large, small, separable) are zeroed by the launcher
hipError_t launch_gridder_persistent(int L, const KernelArgs &a, const int32_t *order, int32_t *queue_head,
                                     int nblocks, hipStream_t s);
hipError_t launch_degridder_persistent(int L, const KernelArgs &a, bool wide, const int32_t *order, int64_t n_sep,
                                       int64_t n_large, int32_t *queue_head, int nblocks_sep, int nblocks_large,
                                       int nblocks_small, hipStream_t s);
int persistent_blocks_per_cu(int L, bool degrid, bool wide, bool small);
int mfma_gridder_blocks_per_cu(int L);
int mfma_degridder_blocks_per_cu(int L);
hipError_t launch_adder(int L, const AdderArgs &a, hipStream_t s);
hipError_t launch_splitter(int L, const DevSubgrid *subgrids, int64_t first, int64_t count, const float2 *grid,
                           int grid_size, float2 *out, hipStream_t s);
hipError_t launch_subgrid_fft(int L, float2 *data, int64_t count, int direction, const float2 *twiddle,
                              hipStream_t s);
hipError_t launch_zero_samples(const int64_t *ids, int64_t n, float2 *vis, hipStream_t s);

// Device scratch of idg_grid_noalloc (kernels.hip): kNoAllocScratchBytes on the current device; the address
// is looked up once per device.
constexpr size_t kNoAllocScratchBytes = size_t(IDG_NOALLOC_SCRATCH_BYTES);
hipError_t noalloc_scratch(void **out);

// Device rates (calib.hip): float32 multiply-add flop/s, sine / cosine wave-instructions/s, fp16 matrix-core
// flop/s, each from microkernels over 8 workgroups per compute unit on the current device (synchronous).
hipError_t measure_device_rates(double *fma_flops, double *sincos_instr, double *mfma_flops);

// master grid <-> image (image.hip)
bool image_size_supported(int N);
hipError_t launch_image_twiddles(float2 *tw, int N, hipStream_t s);
// The 2-D transforms of the [4][N][N] array (image.hip), N a power of two in [64, 16384]:
// image = T(grid) / (corr_m[y] corr_l[x]), grid = T^H(image / (corr_m[y] corr_l[x])); corrections
// both NULL or both set; tw from launch_image_twiddles.  In place (image == grid) needs a
// [4][N][N] scratch when image_needs_scratch says so (the four-step form, N >= 2048); scratch is
// otherwise unused and may be NULL.
bool image_needs_scratch(int N, const void *in, const void *out);
hipError_t launch_grid_to_image(const float2 *grid, float2 *image, int N, const float *corr_l, const float *corr_m,
                                const float2 *tw, float2 *scratch, hipStream_t s);
hipError_t launch_image_to_grid(const float2 *image, float2 *grid, int N, const float *corr_l, const float *corr_m,
                                const float2 *tw, float2 *scratch, hipStream_t s);

// out (= or +=) in * exp(sign 2 pi i w0 n'(l, m)) [/ (corr_m[y] corr_l[x])] over [4][N][N]
hipError_t launch_wlayer_phase(const float2 *in, float2 *out, int N, double S, double w0, int sign, bool accumulate,
                               const float *corr_l, const float *corr_m, hipStream_t s);

// One W-layer of the W-stacked image steps: image (= or +=) T(grid) exp(+2 pi i w0 n') / corr, and
// grid = T^H(image exp(-2 pi i w0 n') / corr).  scratch: [4][N][N] (the image direction always uses
// it; the grid direction only below the four-step form).
hipError_t launch_wlayer_to_image(const float2 *grid, float2 *image, float2 *scratch, int N, double S, double w0,
                                  bool accumulate, const float *corr_l, const float *corr_m, const float2 *tw,
                                  hipStream_t s);
hipError_t launch_image_to_wlayer(const float2 *image, float2 *grid, float2 *scratch, int N, double S, double w0,
                                  const float *corr_l, const float *corr_m, const float2 *tw, hipStream_t s);

}  // namespace idg
