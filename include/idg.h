/*
 * idg.h -- C ABI of an MI355X (gfx950) implementation of Image Domain Gridding
 * (van der Tol, Veenboer & Offringa, "Image Domain Gridding: a fast method for
 * convolutional resampling of visibilities", A&A 2018).
 *
 * The library partitions visibilities into subgrids (§3.2), grids each subgrid
 * by a direct image-domain sum with per-pixel A-terms and taper (§3.3 eq.
 * ShiftedDirectImaging, Algorithm 1, §3.4), transforms it to the uv domain and
 * adds it to the master grid; degridding runs the adjoint chain (Algorithm 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - complex numbers are idg_cf32 {re, im} (complex64);
 *  - master grid: grid[4][N][N] complex64, index [pol][y][x], x <-> u, y <-> v;
 *    grid pixel x sits at u = (x - N/2) / S wavelengths (uv cell 1/S);
 *  - visibilities: vis[nr_baselines][nr_timesteps][nr_channels][4] complex64,
 *    polarisations XX, XY, YX, YY, i.e. the 2x2 matrix [[XX, XY], [YX, YY]];
 *  - uvw[nr_baselines][nr_timesteps][3] float64 metres, freqs[nr_channels]
 *    float64 Hz; a sample's uvw in wavelengths is uvw * f / c0 (§2);
 *  - baselines[nr_baselines][2] int32 station pair (s1, s2);
 *  - A-terms: aterms[nr_slots][nr_stations][L][L][4] complex64, a 2x2 Jones
 *    matrix [J00, J01, J10, J11] per (slot, station, subgrid pixel [row m][col l]);
 *    slot = timestep / aterm_timesteps, nr_slots = ceil(nr_timesteps / aterm_timesteps);
 *  - taper: taper[L][L] float32 (the image-domain window c[i,j] of §4.2);
 *  - subgrid image pixel (j, i) is at l = (i - L/2) S / L, m = (j - L/2) S / L,
 *    n' = sqrt(1 - l^2 - m^2) - 1 (§2 pixel positions, §3.3);
 *  - gridding applies c * A_s1^H Y A_s2 per pixel, degridding c * A_s1 B A_s2^H
 *    (the polarised form of §3.4: the scalar kernel c * g_s1^* g_s2 of Algorithm 1
 *    becomes a product of Jones matrices);
 *  - subgrid transform: the centred DFT
 *      V[b][a] = sum_{j,i} I[j][i] exp(-2 pi i ((a-L/2)(i-L/2) + (b-L/2)(j-L/2)) / L),
 *    unnormalised (Algorithm 1 "FFT"); degridding uses its conjugate transpose,
 *    also unnormalised (Algorithm 2 "IFFT"), so idg_degrid is the exact adjoint
 *    of idg_grid on the planned samples.
 *
 * Pointers ending in _d are device pointers (HIP device memory of the current
 * device); the others are host pointers.  The caller owns every data buffer;
 * device buffers must stay valid until the work queued on `stream` has
 * finished.  `stream` is a hipStream_t (NULL = the default stream).  Every
 * function returns IDG_OK (0) or a negative IDG_E* code; arguments are
 * validated before anything is queued, so nothing is written on a validation
 * error.  No C++ exception crosses this interface.  Errors raised by queued
 * device work surface on a later call or through idg_sync().  idg_last_error()
 * describes the last failure of the calling thread.
 */
#ifndef IDG_H
#define IDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  float re, im;
} idg_cf32;

typedef struct idg_plan_s *idg_plan_t; /* opaque; owned by the library */

enum {
  IDG_OK = 0,
  IDG_EINVAL = -1, /* invalid argument or inconsistent sizes */
  IDG_ENOMEM = -2, /* host or device allocation failed */
  IDG_EHIP = -3,   /* HIP runtime or launch error */
  IDG_ERANGE = -4, /* a size beyond a fixed limit, or IDG_STRICT and some samples would be dropped */
  IDG_ESTATE = -5  /* call not valid in the current state */
};

/* idg_params.flags */
#define IDG_STRICT (1u << 0)     /* idg_plan fails with IDG_ERANGE instead of dropping samples */
#define IDG_PHASE_FP32 (1u << 1) /* subgrid phase offsets in float32 instead of float64 (precision study) */

/* Supported subgrid sizes L. */
#define IDG_SUBGRID_SIZES {8, 16, 24, 32, 48, 64}

typedef struct {
  int32_t grid_size;       /* N: even, L <= N <= 65536 */
  int32_t subgrid_size;    /* L: one of IDG_SUBGRID_SIZES */
  int32_t kernel_size;     /* beta: taper support in uv pixels, 0 <= beta < L */
  int32_t max_timesteps;   /* T_max: timesteps per subgrid, 1 .. 65535 */
  int32_t aterm_timesteps; /* A-term slot length in timesteps, >= 1 (blocks never cross a slot) */
  int32_t nr_stations;     /* >= 2 */
  int32_t nr_baselines;    /* >= 0 */
  int32_t nr_timesteps;    /* >= 0 */
  int32_t nr_channels;     /* 0 .. 65535 */
  uint32_t flags;          /* IDG_STRICT | IDG_PHASE_FP32 */
  double image_size;       /* S = N * cell, direction-cosine units (> 0) */
  int64_t scratch_bytes;   /* device budget for transformed subgrids during idg_grid; 0 = 2 GiB.
                              A budget that holds every subgrid of the plan grids it in one launch.
                              The scratch comes from the device's default stream-ordered memory pool,
                              whose release threshold the library raises so freed scratch is reused. */
  double w_step;           /* W-layer spacing in wavelengths (>= 0; 0 = no layers: every subgrid has
                              w offset 0 and the grid is one [4][N][N] array) */
} idg_params;

/*
 * Partition the visibilities into subgrids (§3.2 Partitioning, Fig. 2; blocks
 * cut at A-term slot boundaries as in §3.4 Variations).  Host only: nothing is
 * queued on a device (device metadata is uploaded on first use).
 *
 * Each block holds one baseline, a run of at most T_max timesteps inside one
 * A-term slot, and a contiguous channel group, chosen so that every sample's
 * support (the taper's beta pixels plus ceil(|w| S^2) pixels of w-support)
 * fits the L x L box; its centre lies on the grid lattice.  Rule, in float64
 * without contraction: x = (uvw_u * (f / c0)) * S + N/2 (same for y); a set
 * fits iff (max x - min x) + beta + max ceil((|w| * S) * S) <= L - 1 in both
 * axes; channel groups are split in halves while a group fails at some single
 * timestep; time is scanned greedily; corner x0 = floor((min x + max x) * 0.5
 * + 0.5) - L/2; a block whose box leaves [0, N) is dropped (no wrap-around), as
 * are samples that do not fit alone.  Subgrids are ordered by baseline,
 * channel group, time.
 *
 * W-layers (w_step > 0; the per-subgrid w offset w_0p of Algorithms 1 and 2):
 * a block's layer is j = floor(w_mid / w_step + 0.5), w_mid = (w(t0, c_lo) +
 * w(t0, c_hi)) * 0.5 being the mid-band w of its first timestep; its offset is
 * w_0p = j * w_step and the w-support of a sample becomes ceil((|w - w_0p| * S)
 * * S).  (In the channel-group step a timestep taken alone uses its own
 * layer.)  The grids of idg_grid and idg_degrid then hold one [4][N][N] grid
 * per layer j = wlayer_min .. wlayer_min + nr_wlayers - 1 (idg_plan_wlayers),
 * consecutively; each layer's grid lacks the w-term w_0p n', which the image
 * steps (idg_wstack_to_image, idg_image_to_wstack) put back.
 *
 *   params     sizes and options (copied)
 *   baselines  host int32 [nr_baselines][2], stations in [0, nr_stations), s1 != s2
 *   uvw        host float64 [nr_baselines][nr_timesteps][3], finite
 *   freqs      host float64 [nr_channels], finite and > 0
 *   flags      host uint8 [nr_baselines][nr_timesteps][nr_channels], nonzero =
 *              flagged (not gridded, written as 0 by idg_degrid); NULL = none
 *   out        receives the plan; free it with idg_plan_destroy
 * Errors: IDG_EINVAL (bad sizes or values), IDG_ENOMEM, IDG_ERANGE (IDG_STRICT
 * and some unflagged sample would be dropped).  The arrays are not retained.
 */
int idg_plan(const idg_params *params, const int32_t *baselines, const double *uvw, const double *freqs,
             const uint8_t *flags, idg_plan_t *out);

/* Plan counters; any output pointer may be NULL.  nr_gridded + nr_dropped +
 * nr_flagged = nr_baselines * nr_timesteps * nr_channels. */
int idg_plan_stats(idg_plan_t plan, int64_t *nr_subgrids, int64_t *nr_gridded, int64_t *nr_dropped,
                   int64_t *nr_flagged);

/* How the subgrid sums of the plan are evaluated under its current tuning and
 * precision (either pointer may be NULL; each is int64 [3]):
 *   [0] separable form, cross term to order 0;  [1] separable form, order 1;
 *   [2] direct sum (phasor per sample and pixel, eq. 14 and its adjoint).
 * nr_subgrids counts subgrids, nr_vis their planned samples.  The separable form
 * factors the phasor of eq. 14 into a row factor and a column factor (the
 * phase is linear in the offsets of section 3.1) times a bounded expansion of
 * the non-separable remainder of n'; it applies to 32 x 32 subgrids in
 * float64-offset precision with sum_path IDG_SUM_AUTO. */
int idg_plan_sum_paths(idg_plan_t plan, int64_t *nr_subgrids, int64_t *nr_vis);

/* W-layers of the plan (either pointer may be NULL): the grid passed to
 * idg_grid / idg_degrid is [nr_wlayers][4][N][N], layer index j - wlayer_min.
 * Without layers wlayer_min = 0 and nr_wlayers = 1. */
int idg_plan_wlayers(idg_plan_t plan, int32_t *wlayer_min, int32_t *nr_wlayers);

/* Copy the plan to host arrays (either may be NULL):
 *   subgrids  int64 [nr_subgrids][13]: bl, t0, nt, c0, nc, x0, y0, slot, s1, s2, nvis, vis_offset, wlayer
 *   samples   int32 [nr_gridded][2]: (timestep, channel) of each planned sample,
 *             grouped by subgrid (rows vis_offset .. vis_offset + nvis - 1), t-major. */
int idg_plan_export(idg_plan_t plan, int64_t *subgrids, int32_t *samples);

/* Scheduling knobs of a plan (the path's schedule: every setting but sum_path
 * gives the same result up to float32 summation order; sum_path selects
 * between two evaluations of the subgrid sums that agree to float32 level).
 *   grid_form, degrid_form
 *                  IDG_FORM_PLAIN: one workgroup per subgrid;
 *                  IDG_FORM_PERSISTENT: a fixed set of workgroups takes subgrids
 *                  from a device work queue, costliest (most visibilities)
 *                  first -- for many small or uneven subgrids;
 *   grid_blocks_per_cu, degrid_blocks_per_cu
 *                  persistent form: workgroups per compute unit (0 = as many as fit);
 *   adder_chunk    adder: the longest run of one grid tile's subgrid list handled
 *                  by one workgroup; longer lists are summed in parallel chunks
 *                  whose partial tiles are added in order (0 = 256);
 *   degrid_shape   IDG_DEGRID_STANDARD: degridder lanes own up to 4 visibilities
 *                  each and sum over all pixels of their share;
 *                  IDG_DEGRID_WIDE: subgrids with 64 or more visibilities run
 *                  with 8 visibilities per lane over half the pixels, the two
 *                  halves of a wave adding their sums -- fewer phasor evaluations
 *                  per visibility, more registers; pays for large subgrids.
 *                  Results agree to float32 summation order.  Ignored with
 *                  IDG_PHASE_FP32;
 *   sum_path       IDG_SUM_AUTO: subgrids of 32 x 32 whose w-term allows it run
 *                  the separable form of the subgrid sum on the matrix cores
 *                  (see idg_grid), the others the direct sum; IDG_SUM_DIRECT:
 *                  every subgrid runs the direct sum.  Results agree to float32
 *                  level (the separable form's operands carry 22 significant
 *                  bits and its cross-term expansion is truncated below 1e-6);
 *   reserved       must be 0.
 * idg_plan_set_tuning validates (IDG_EINVAL) and stores the knobs; call it
 * only when no work queued with the plan is pending.  New plans start with
 * all fields 0 (plain forms, default chunk, standard degridder, automatic
 * sum path). */
#define IDG_FORM_PLAIN 0
#define IDG_FORM_PERSISTENT 1
#define IDG_DEGRID_STANDARD 0
#define IDG_DEGRID_WIDE 1
#define IDG_SUM_AUTO 0
#define IDG_SUM_DIRECT 1
typedef struct {
  int32_t grid_form;
  int32_t degrid_form;
  int32_t grid_blocks_per_cu;
  int32_t degrid_blocks_per_cu;
  int32_t adder_chunk;
  int32_t degrid_shape;
  int32_t sum_path;
  int32_t reserved;
} idg_tuning;
int idg_plan_set_tuning(idg_plan_t plan, const idg_tuning *tuning);
int idg_plan_get_tuning(idg_plan_t plan, idg_tuning *tuning);

/* Release the plan and its device metadata.  Work queued with it must have
 * finished.  NULL is ignored. */
void idg_plan_destroy(idg_plan_t plan);

/*
 * Image-domain gridding (Algorithm 1 without its last line, §3.3, §3.4): for
 * every subgrid, the direct sum over its samples of Y_k exp(+2 pi i (du_k l +
 * dv_k m + w_k n')) with du_k = u_k - u_0p computed in float64 and the
 * per-pixel phase in float32; then c * A_s1^H S A_s2 per pixel; the centred
 * DFT; and the sum into grid_d at corner (x0, y0).  grid_d is ACCUMULATED
 * into (the caller zeroes it).  Results are deterministic: for each grid tile
 * the subgrids are added in plan order.  uvw_d and freqs_d must hold the
 * values given to idg_plan.  When idg_plan found the channel frequencies
 * evenly spaced (every spacing equal to the first to 1e-9 relative), the
 * phasors of consecutive channels of one timestep are advanced by one complex
 * multiplication with a per-run step phasor (runs of at most 16 channels)
 * instead of a sin/cos per sample; the result agrees with the per-sample
 * evaluation to float32 rounding.  Subgrids of 32 x 32 may instead run the
 * separable form (tuning sum_path): with n' = a(l) + a(m) + c(l, m),
 * a(x) = sqrt(1 - x^2) - 1, the phasor is U(l) V(m) exp(2 pi i dw c), the
 * last factor expanded to the order (0 or 1) that keeps its truncation
 * below 1e-6 given the subgrid's largest |w - w_0p| (the plan computes it in
 * float64); each order is a dense (32 x K)(K x 32) product per polarisation,
 * on the matrix cores with fp16 high/low operand parts.  Subgrids whose
 * w-term needs a higher order run the direct sum.  Device scratch of at most
 * params.scratch_bytes is allocated stream-ordered for the call.
 *
 *   uvw_d    float64 [nr_baselines][nr_timesteps][3]     freqs_d  float64 [nr_channels]
 *   vis_d    complex64 [nr_baselines][nr_timesteps][nr_channels][4]
 *   aterms_d complex64 [nr_slots][nr_stations][L][L][4]  taper_d  float32 [L][L]
 *   grid_d   complex64 [nr_wlayers][4][N][N] ([4][N][N] without W-layers), read and
 *            written; a subgrid of layer j is added to grid j - wlayer_min
 * With W-layers the phase of sample k in subgrid p uses w_k - w_0p.
 * Errors: IDG_EINVAL (NULL pointer), IDG_ENOMEM, IDG_EHIP.
 */
int idg_grid(idg_plan_t plan, const double *uvw_d, const double *freqs_d, const idg_cf32 *vis_d,
             const idg_cf32 *aterms_d, const float *taper_d, idg_cf32 *grid_d, void *stream);

/*
 * idg_grid without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Arguments, arithmetic and result are those of idg_grid (the
 * same kernels and batches: bitwise the same grid).  Its scratch is a fixed
 * device array of IDG_NOALLOC_SCRATCH_BYTES compiled into the library, one per
 * GPU, held from the first call on that GPU until the process ends.  Every
 * call on a GPU uses that GPU's array: calls that overlap on one GPU (other
 * streams or threads) race and must be ordered by the caller.  Limits:
 *   - one batch of the plan must fit: 256 bytes + the adder's partial tiles +
 *     4 L^2 x 8 bytes per subgrid of a batch (plan with params.scratch_bytes
 *     of at most about 120 MiB); otherwise IDG_ERANGE, nothing launched;
 *   - the plan's device copy must already exist on the current device (an
 *     earlier idg_grid, idg_degrid or idg_grid_subgrids call with the plan on
 *     this device makes it; idg_plan_set_tuning with a new adder_chunk drops
 *     it); otherwise IDG_ESTATE, nothing launched.
 * Errors: IDG_EINVAL (NULL pointer), IDG_ESTATE, IDG_ERANGE, IDG_EHIP.
 */
#define IDG_NOALLOC_SCRATCH_BYTES (128LL << 20)
int idg_grid_noalloc(idg_plan_t plan, const double *uvw_d, const double *freqs_d, const idg_cf32 *vis_d,
                     const idg_cf32 *aterms_d, const float *taper_d, idg_cf32 *grid_d, void *stream);

/*
 * Image-domain degridding (Algorithm 2 after its first two lines): for every
 * subgrid, split it out of grid_d, apply the unnormalised inverse centred DFT,
 * apply c * A_s1 I A_s2^H per pixel, and for every sample compute
 * sum_pix B exp(-2 pi i (du_k l + dv_k m + (w_k - w_0p) n')).  vis_d is OVERWRITTEN:
 * planned samples get their prediction, flagged and dropped samples get 0.
 * Arguments as idg_grid, grid_d read only, vis_d written.
 * Errors: IDG_EINVAL, IDG_ENOMEM, IDG_EHIP.
 */
int idg_degrid(idg_plan_t plan, const double *uvw_d, const double *freqs_d, const idg_cf32 *grid_d,
               const idg_cf32 *aterms_d, const float *taper_d, idg_cf32 *vis_d, void *stream);

/*
 * Stage access for testing and measurement: run the gridder on subgrids
 * first .. first + count - 1 of the plan and write each subgrid to
 * out_d[count][4][L][L] complex64 ([pol][row m / v][col l / u]), either as the
 * image after A-terms and taper (stage 0, before the transform) or as the uv
 * subgrid after the centred DFT (stage 1).  Nothing is added to a grid.  The
 * subgrid sums take the same form as in idg_grid (idg_plan_sum_paths); when
 * some take the separable form, the call uploads a work list and synchronises
 * the stream once.
 * Errors: IDG_EINVAL (range or stage), IDG_ENOMEM, IDG_EHIP.
 */
int idg_grid_subgrids(idg_plan_t plan, const double *uvw_d, const double *freqs_d, const idg_cf32 *vis_d,
                      const idg_cf32 *aterms_d, const float *taper_d, int64_t first, int64_t count, int32_t stage,
                      idg_cf32 *out_d, void *stream);

/*
 * Batched centred subgrid DFT (Algorithm 1 "FFT", Algorithm 2 "IFFT") on
 * data_d[count][4][L][L] complex64, in place, unnormalised; direction -1 is
 * the forward transform (exp(-...)), +1 its conjugate transpose.
 * Errors: IDG_EINVAL (L not supported, direction, count < 0), IDG_EHIP.
 */
int idg_subgrid_fft(idg_cf32 *data_d, int64_t count, int32_t subgrid_size, int32_t direction, void *stream);

/*
 * Adder (Algorithm 1, add subgrid to master grid): grid_d[pol][y0+b][x0+a] +=
 * subgrids_d[s][pol][b][a] for s in 0 .. count-1 taken as plan subgrids
 * first .. first + count - 1.  Tile ownership, deterministic order.
 * Errors: IDG_EINVAL, IDG_ENOMEM, IDG_EHIP.
 */
int idg_add_subgrids(idg_plan_t plan, const idg_cf32 *subgrids_d, int64_t first, int64_t count, idg_cf32 *grid_d,
                     void *stream);

/*
 * Splitter (Algorithm 2, initialise subgrid from master grid):
 * subgrids_d[s][pol][b][a] = grid_d[pol][y0+b][x0+a] for plan subgrids
 * first .. first + count - 1.
 * Errors: IDG_EINVAL, IDG_EHIP.
 */
int idg_split_subgrids(idg_plan_t plan, const idg_cf32 *grid_d, int64_t first, int64_t count, idg_cf32 *subgrids_d,
                       void *stream);

/*
 * Master grid -> image (the last line of Algorithm 1; §3.3: the image is the
 * transform of the grid divided by the taper):
 *   image_d[pol][y][x] = sum_{v,u} grid_d[pol][v][u]
 *                        exp(+2 pi i ((u - N/2)(x - N/2) + (v - N/2)(y - N/2)) / N)
 *                        / (corr_m_d[y] corr_l_d[x]),
 * i.e. the grid's DTFT at the image pixels l_x = (x - N/2) S / N, m_y = (y -
 * N/2) S / N, divided by a separable correction (for subgrids with taper c,
 * corr[x] = L c(l_x) gives the division by L^2 c(l) c(m)).  Unnormalised.
 *   grid_d    device complex64 [4][N][N], read
 *   corr_l_d, corr_m_d  device float32 [N] (both NULL: no division)
 *   image_d   device complex64 [4][N][N], OVERWRITTEN; may be grid_d itself
 *             (in place), must not overlap it otherwise
 * N = grid_size must be a power of two in [64, 16384].  Two passes over the
 * array (three for N >= 2048); N/2 x 8 bytes of twiddles are allocated
 * stream-ordered for the call, and for an in-place call with N >= 2048 also
 * 4 N^2 x 8 bytes of scratch.
 * Errors: IDG_EINVAL (size, NULL or partly overlapping buffers), IDG_ENOMEM,
 * IDG_EHIP.
 */
int idg_grid_to_image(const idg_cf32 *grid_d, int32_t grid_size, const float *corr_l_d, const float *corr_m_d,
                      idg_cf32 *image_d, void *stream);

/*
 * Image -> master grid (the first lines of Algorithm 2, model image divided by
 * the taper and transformed), the adjoint of idg_grid_to_image:
 *   grid_d[pol][v][u] = sum_{y,x} image_d[pol][y][x] / (corr_m_d[y] corr_l_d[x])
 *                       exp(-2 pi i ((u - N/2)(x - N/2) + (v - N/2)(y - N/2)) / N).
 * grid_d is OVERWRITTEN.  Arguments and errors as idg_grid_to_image.
 */
int idg_image_to_grid(const idg_cf32 *image_d, int32_t grid_size, const float *corr_l_d, const float *corr_m_d,
                      idg_cf32 *grid_d, void *stream);

/*
 * W-stacked image steps (the w offsets w_0p of Algorithms 1 and 2): each layer's
 * grid lacks the w-term w_0 n' of its subgrids, which is put back per layer in
 * the image domain,
 *   image_d = sum_j exp(+2 pi i w0s[j] n'(l_x, m_y)) T(grids_d[j]) / (corr_m_d[y] corr_l_d[x]),
 * T being the transform of idg_grid_to_image and n' = sqrt(1 - l^2 - m^2) - 1
 * at l_x = (x - N/2) S / N, m_y = (y - N/2) S / N (0 under the root outside the
 * unit circle).  idg_image_to_wstack is its adjoint (every grid OVERWRITTEN):
 *   grids_d[j] = T^H(image_d exp(-2 pi i w0s[j] n') / (corr_m_d[y] corr_l_d[x])).
 *   grids_d     device complex64 [nr_wlayers][4][N][N]; for a plan, the layer
 *               grids of idg_grid / idg_degrid, w0s[j] = (wlayer_min + j) w_step
 *   w0s         host float64 [nr_wlayers], finite (read during the call)
 *   image_d     device complex64 [4][N][N], must not overlap grids_d
 *   image_size  S in (0, 1.4];  corrections as idg_grid_to_image
 * N = grid_size a power of two in [64, 16384], 1 <= nr_wlayers <= 65536.  One
 * layer at a time through 4 N^2 x 8 bytes of stream-ordered scratch.
 * Errors: IDG_EINVAL, IDG_ENOMEM, IDG_EHIP.
 */
int idg_wstack_to_image(const idg_cf32 *grids_d, int32_t nr_wlayers, const double *w0s, int32_t grid_size,
                        double image_size, const float *corr_l_d, const float *corr_m_d, idg_cf32 *image_d,
                        void *stream);
int idg_image_to_wstack(const idg_cf32 *image_d, int32_t grid_size, double image_size, const float *corr_l_d,
                        const float *corr_m_d, int32_t nr_wlayers, const double *w0s, idg_cf32 *grids_d,
                        void *stream);

/*
 * The optimal window of image domain gridding (§4.3 and Appendix A): the 1-D
 * taper a[0..L-1] (the subgrid taper is c[j][i] = a_j a_i, §4.2) minimising the
 * side-lobe energy of the effective window averaged over the sample shifts
 * |s| <= max_shift (uv pixels from the subgrid centre).  It is the eigenvector
 * of the smallest eigenvalue eps^2 of the L x L matrix Rbar = Qbar o Sbar.
 * Table 1 of the paper uses max_shift = (L - beta + 1)/2 for kernel width beta.
 * The plans of idg_plan with kernel_size beta keep every sample within
 * (L - 1 - beta)/2 of its subgrid centre; design their taper for
 * max_shift = (L - beta)/2, half a pixel more: the window's error rises
 * steeply at the edge of its design range, and samples on the plans' bound
 * would sit there.  Host code, float64; nothing touches the GPU.
 *   L          subgrid size, 4 .. 256
 *   max_shift  0 < max_shift <= L/2
 *   taper_out  host double [L], written; scaled so that taper_out[L/2] = 1
 *   eps_out    host double, written: eps, the rms side-lobe level
 * Errors: IDG_EINVAL (arguments), IDG_ERANGE (eps^2 below 1e-13 of the largest
 * eigenvalue, beyond float64 resolution; the outputs are still written).
 */
int idg_taper_optimal(int32_t L, double max_shift, double *taper_out, double *eps_out);

/*
 * The correction the master-grid image steps divide by for a subgrid taper
 * a[0..L-1] (Algorithms 1 and 2, the inverse rms taper): the effective
 * window's rms over the sample shifts |s| <= max_shift at each image pixel,
 *   corr_out[X] = L sqrt(sum_{k,l} a_k a_l sinc(x - k) sinc(x - l) sinc(2 max_shift (k - l) / L)),
 *   x = L X / N (image pixel X, at l = (X - N/2) S / N, in subgrid index units).
 * Pass it as both corr_l and corr_m, with the max_shift of the plan.  Host code.
 *   taper      host double [L];  corr_out  host float [N], written;  2 <= N <= 2^20
 * Errors: IDG_EINVAL.
 */
int idg_taper_correction(int32_t L, double max_shift, const double *taper, int32_t N, float *corr_out);

/* Stage timing (the library's own tracing).  While enabled, idg_grid and
 * idg_degrid record a pair of HIP events on their stream around every kernel
 * they queue.  idg_profile_read waits for the recorded events and returns the
 * accumulated milliseconds and launch counts per stage (arrays of
 * IDG_NR_STAGES, either may be NULL), then clears them if `reset` is nonzero.
 * Timing adds two event records per launch; it is off by default. */
#define IDG_STAGE_GRIDDER 0
#define IDG_STAGE_ADDER 1
#define IDG_STAGE_DEGRIDDER 2
#define IDG_STAGE_ZERO 3
#define IDG_NR_STAGES 4
int idg_profile(int enable);
int idg_profile_read(double *ms, int64_t *launches, int reset);

/* Scratch memory.  idg_grid, idg_degrid and the image steps take their device
 * scratch stream-ordered from a memory pool the library creates per device
 * (not the device's default pool).  Freed scratch stays in that pool for the
 * next call -- up to the largest scratch any call has used (a plan's
 * params.scratch_bytes plus small work lists) -- so that repeated calls do not
 * map their scratch again.  idg_trim_scratch waits for the current device and
 * returns the pool's unused memory to the driver beyond keep_bytes.
 * Errors: IDG_EHIP. */
int idg_trim_scratch(uint64_t keep_bytes);

/* Measurement aid, not part of the method: the rates this device sustains for
 * the instruction kinds the gridder and degridder issue, from microkernels
 * (8 workgroups per compute unit, best of 3 launches) on the current device:
 * float32 multiply-add flop/s (2 flop each), sine / cosine wave64
 * instructions/s, and fp16 matrix-core flop/s (32 x 32 x 16 products).
 * Synchronous; allocates a small device buffer.  Any pointer may not be NULL.
 * Errors: IDG_EINVAL (NULL pointer), IDG_EHIP. */
int idg_device_rates(double *fp32_fma_flops, double *sincos_instr, double *fp16_mfma_flops);

/* Wait for `stream` and report any error its queued work raised. */
int idg_sync(void *stream);

/* Message describing the last failure of the calling thread ("" if none). */
const char *idg_last_error(void);

/* Interface version (major * 10000 + minor * 100 + patch). */
int idg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IDG_H */
