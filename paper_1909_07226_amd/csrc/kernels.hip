// gfx950 kernels of image-domain gridding.
//
//   gridder    direct image-domain sum of a subgrid's visibilities (§3.3 eq.
//              ShiftedDirectImaging; Algorithm 1 inner loops), A-terms x taper
//              per pixel (§3.4), centred DFT in LDS (Algorithm 1 "FFT")
//   adder      sum of transformed subgrids into the master grid, one
//              workgroup per grid tile and polarisation (Algorithm 1, add)
//   degridder  splitter, inverse centred DFT, A-terms x taper, and the
//              per-visibility sum over pixels (Algorithm 2)
//
// The phasor sum is not a dense contraction (each term has its own phasor), so
// it runs on the VALU: float32 phase per (visibility, pixel) from float64
// per-subgrid offsets, v_sin_f32 / v_cos_f32 on the phase in revolutions, and
// float32 multiply-adds.  When the channel frequencies are evenly spaced, the
// phase is linear in the channel index (u_k = uvw f / c0), so the phasors of a
// run of consecutive channels of one timestep are the run's first phasor times
// powers of one step phasor: one complex multiply per sample replaces sin, cos
// and the phase arithmetic.
#include "internal.h"

#include <algorithm>
#include <atomic>

namespace idg {

constexpr double kC0 = 299792458.0;

template <int L>
struct Cfg;
template <>
struct Cfg<8> {
  static constexpr int NT = 64;
};
template <>
struct Cfg<16> {
  static constexpr int NT = 64;
};
template <>
struct Cfg<24> {
  static constexpr int NT = 192;
};
template <>
struct Cfg<32> {
  static constexpr int NT = 256;
};
template <>
struct Cfg<48> {
  static constexpr int NT = 576;
};
template <>
struct Cfg<64> {
  static constexpr int NT = 512;
};

bool supported_subgrid_size(int L) {
  return L == 8 || L == 16 || L == 24 || L == 32 || L == 48 || L == 64;
}

// ---------------------------------------------------------------------------
// small complex helpers

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cjmul(float2 a, float2 b) {  // conj(a) * b
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
// acc += (xr + i xi) * (c + i s) as four fused multiply-adds
__device__ __forceinline__ void cmac(float2 &acc, float xr, float xi, float c, float s) {
  acc.x = __builtin_fmaf(xr, c, acc.x);
  acc.x = __builtin_fmaf(-xi, s, acc.x);
  acc.y = __builtin_fmaf(xr, s, acc.y);
  acc.y = __builtin_fmaf(xi, c, acc.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// Per-pixel polarised kernel for gridding: c * J1^H S J2 (S = [[s0, s1], [s2, s3]]).
__device__ __forceinline__ void apply_aterms_grid(const float2 *j1, const float2 *j2, float c, float2 s[4]) {
  const float2 t00 = cadd(cmul(s[0], j2[0]), cmul(s[1], j2[2]));
  const float2 t01 = cadd(cmul(s[0], j2[1]), cmul(s[1], j2[3]));
  const float2 t10 = cadd(cmul(s[2], j2[0]), cmul(s[3], j2[2]));
  const float2 t11 = cadd(cmul(s[2], j2[1]), cmul(s[3], j2[3]));
  s[0] = cscale(cadd(cjmul(j1[0], t00), cjmul(j1[2], t10)), c);
  s[1] = cscale(cadd(cjmul(j1[0], t01), cjmul(j1[2], t11)), c);
  s[2] = cscale(cadd(cjmul(j1[1], t00), cjmul(j1[3], t10)), c);
  s[3] = cscale(cadd(cjmul(j1[1], t01), cjmul(j1[3], t11)), c);
}

// Per-pixel polarised kernel for degridding: c * J1 I J2^H.
__device__ __forceinline__ void apply_aterms_degrid(const float2 *j1, const float2 *j2, float c, float2 s[4]) {
  const float2 t00 = cadd(cmulc(s[0], j2[0]), cmulc(s[1], j2[1]));
  const float2 t01 = cadd(cmulc(s[0], j2[2]), cmulc(s[1], j2[3]));
  const float2 t10 = cadd(cmulc(s[2], j2[0]), cmulc(s[3], j2[1]));
  const float2 t11 = cadd(cmulc(s[2], j2[2]), cmulc(s[3], j2[3]));
  s[0] = cscale(cadd(cmul(j1[0], t00), cmul(j1[1], t10)), c);
  s[1] = cscale(cadd(cmul(j1[0], t01), cmul(j1[1], t11)), c);
  s[2] = cscale(cadd(cmul(j1[2], t00), cmul(j1[3], t10)), c);
  s[3] = cscale(cadd(cmul(j1[2], t01), cmul(j1[3], t11)), c);
}

// ---------------------------------------------------------------------------
// Subgrid layout in LDS: [4][L][RS] complex.  Every supported size (2^n and
// 3 x 2^n) is transformed by a register FFT per row / column; the rows are
// padded to RS = L + 1 so that the lanes of a wave, each walking its own row,
// hit different LDS banks.

template <int L>
struct SgLayout {
  static constexpr bool FFT = (L == 8 || L == 16 || L == 24 || L == 32 || L == 48 || L == 64);
  static constexpr int RS = FFT ? L + 1 : L;  // row stride
  static constexpr int POL = L * RS;          // polarisation stride
  static constexpr int SIZE = 4 * POL;        // complex elements
  __device__ static __forceinline__ int idx(int pol, int pix) { return pol * POL + (pix / L) * RS + pix % L; }
};

// exp(-2 pi i k / N), k = 0 .. N-1, evaluated at compile time in double precision
constexpr double kPi = 3.14159265358979323846;
constexpr double cx_sin(double x) {  // |x| <= pi
  double term = x, sum = x;
  for (int n = 1; n < 16; ++n) {
    term *= -x * x / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos(double x) {  // |x| <= pi
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 16; ++n) {
    term *= -x * x / double((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}
template <int N>
struct Twiddles {
  float re[N], im[N];
  constexpr Twiddles() : re(), im() {
    for (int k = 0; k < N; ++k) {
      double a = -2.0 * kPi * k / N;
      if (a < -kPi) a += 2.0 * kPi;
      re[k] = float(cx_cos(a));
      im[k] = float(cx_sin(a));
    }
  }
};
constexpr int bit_reverse(int i, int n) {
  int r = 0;
  for (int b = 1; b < n; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

template <int N, bool INV>
__device__ __forceinline__ void reg_fft(float2 (&x)[N]);

// N = 3M, M a power of two: decimation in time by 3.  With F_r the M-point
// transforms of x[3m + r] and W = exp(-+2 pi i / N),
//   X[k + M q] = sum_r exp(-+2 pi i r q / 3) W^(r k) F_r[k],  k < M, q = 0, 1, 2,
// a radix-3 butterfly per k on (F_0, W^k F_1, W^2k F_2).
template <int N, bool INV>
__device__ __forceinline__ void reg_fft_radix3(float2 (&x)[N]) {
  constexpr int M = N / 3;
  constexpr Twiddles<N> T{};
  constexpr float kS3 = 0.86602540378443865f;  // sin(pi / 3)
  float2 f[3][M];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int m = 0; m < M; ++m) f[r][m] = x[3 * m + r];
    reg_fft<M, INV>(f[r]);
  }
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const float2 a = f[0][k];
    float2 b = f[1][k], c = f[2][k];
    if (k != 0) {
      const float w1r = T.re[k], w1i = INV ? -T.im[k] : T.im[k];
      const float w2r = T.re[2 * k], w2i = INV ? -T.im[2 * k] : T.im[2 * k];
      b = make_float2(b.x * w1r - b.y * w1i, b.x * w1i + b.y * w1r);
      c = make_float2(c.x * w2r - c.y * w2i, c.x * w2i + c.y * w2r);
    }
    // exp(-+2 pi i / 3) = -1/2 -+ i sin(pi / 3):  X1 = a - (b + c) / 2 -+ i s (b - c), X2 = its mirror
    const float2 sum = make_float2(b.x + c.x, b.y + c.y), dif = make_float2(b.x - c.x, b.y - c.y);
    const float2 mid = make_float2(a.x - 0.5f * sum.x, a.y - 0.5f * sum.y);
    const float2 rot = INV ? make_float2(-kS3 * dif.y, kS3 * dif.x) : make_float2(kS3 * dif.y, -kS3 * dif.x);
    x[k] = make_float2(a.x + sum.x, a.y + sum.y);
    x[k + M] = make_float2(mid.x + rot.x, mid.y + rot.y);
    x[k + 2 * M] = make_float2(mid.x - rot.x, mid.y - rot.y);
  }
}

// In-register FFT, X[k] = sum_n x[n] exp(-+2 pi i n k / N) (INV: +), unnormalised: radix 2 for
// N = 2^n, one radix-3 step and then radix 2 for N = 3 x 2^n.
template <int N, bool INV>
__device__ __forceinline__ void reg_fft(float2 (&x)[N]) {
  if constexpr (N % 3 == 0) {
    reg_fft_radix3<N, INV>(x);
    return;
  } else {
  static_assert((N & (N - 1)) == 0, "reg_fft: N = 2^n or 3 x 2^n");
  constexpr Twiddles<N> T{};
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int j = bit_reverse(i, N);
    if (i < j) {
      const float2 t = x[i];
      x[i] = x[j];
      x[j] = t;
    }
  }
#pragma unroll
  for (int len = 2; len <= N; len <<= 1) {
#pragma unroll
    for (int i = 0; i < N; i += len) {
#pragma unroll
      for (int k = 0; k < len / 2; ++k) {
        const int e = k * (N / len);
        const float2 u = x[i + k], v = x[i + k + len / 2];
        float2 vw;
        if (e == 0) {
          vw = v;
        } else if (4 * e == N) {  // exp(-+ i pi / 2)
          vw = INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
        } else {
          const float wr = T.re[e], wi = INV ? -T.im[e] : T.im[e];
          vw = make_float2(v.x * wr - v.y * wi, v.x * wi + v.y * wr);
        }
        x[i + k] = make_float2(u.x + vw.x, u.y + vw.y);
        x[i + k + len / 2] = make_float2(u.x - vw.x, u.y - vw.y);
      }
    }
  }
  }
}

// Centred 2-D DFT of a [4][L][L] subgrid held in LDS, in place:
//   out[b][a] = sum_{j,i} in[j][i] w((a - L/2)(i - L/2)) w((b - L/2)(j - L/2)),
// w(k) = exp(-+2 pi i k / L) (INV: +).  For even L this is
//   out = (-1)^(a+b) FFT2[(-1)^(i+j) in],
// done as register FFTs per (polarisation, row) and then per (polarisation,
// column), two threads per line; `tw` holds exp(-2 pi i k / L), k < L.
template <int L, int NT, bool INV>
__device__ __forceinline__ void lds_centred_dft(float2 *sg, const float2 *tw) {
  using Lay = SgLayout<L>;
  constexpr int NPIX = L * L, PPT = NPIX / NT, H = L / 2;
  const int tid = threadIdx.x;
  static_assert(Lay::FFT, "subgrid transform: L = 2^n or 3 x 2^n");
  {
    // Each line (a row in pass 0, a column in pass 1, of one polarisation) is
    // transformed by two threads: thread h takes the samples n = 2j + h and does
    // an L/2-point FFT in registers; after a barrier, each thread forms half of
    // the radix-2 butterflies X0[k] +- W^k X1[k].  Work item w: the two halves of
    // a wave take the same 32 lines (h = 0, then h = 1), so that the 32 lanes of
    // a half-wave walk 32 different lines, as in a one-thread-per-line layout.
    constexpr int HL = L / 2, QL = L / 4, ROUNDS = (8 * L + NT - 1) / NT;
    static_assert((8 * L) % 64 == 0, "work items fill whole waves");
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
      const int step = pass == 0 ? 1 : Lay::RS;
      for (int w = tid; w < 8 * L; w += NT) {
        const int line = (w >> 6) * 32 + (w & 31), h = (w >> 5) & 1;
        const int pol = line / L, q = line % L;  // q: row (pass 0) or column (pass 1)
        float2 *base = sg + pol * Lay::POL + (pass == 0 ? q * Lay::RS : q);
        float2 x[HL];
#pragma unroll
        for (int j = 0; j < HL; ++j) {
          const int n = 2 * j + h;
          const float2 v = base[n * step];
          const bool flip = pass == 0 && ((n + q) & 1);
          x[j] = flip ? make_float2(-v.x, -v.y) : v;
        }
        reg_fft<HL, INV>(x);
#pragma unroll
        for (int k = 0; k < HL; ++k) base[(2 * k + h) * step] = x[k];  // X_h[k] where sample 2k + h was
      }
      __syncthreads();
      float2 y[ROUNDS][2][QL];
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        const int w = tid + r * NT;
        if (w >= 8 * L) break;
        const int line = (w >> 6) * 32 + (w & 31), h = (w >> 5) & 1;
        const int pol = line / L, q = line % L;
        const float2 *base = sg + pol * Lay::POL + (pass == 0 ? q * Lay::RS : q);
#pragma unroll
        for (int i = 0; i < QL; ++i) {
          const int k = h * QL + i;
          const float2 a0 = base[(2 * k) * step], b0 = base[(2 * k + 1) * step];
          float2 t = tw[k];  // exp(-2 pi i k / L)
          if (INV) t.y = -t.y;
          const float2 bw = make_float2(b0.x * t.x - b0.y * t.y, b0.x * t.y + b0.y * t.x);
          y[r][0][i] = make_float2(a0.x + bw.x, a0.y + bw.y);
          y[r][1][i] = make_float2(a0.x - bw.x, a0.y - bw.y);
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        const int w = tid + r * NT;
        if (w >= 8 * L) break;
        const int line = (w >> 6) * 32 + (w & 31), h = (w >> 5) & 1;
        const int pol = line / L, q = line % L;
        float2 *base = sg + pol * Lay::POL + (pass == 0 ? q * Lay::RS : q);
#pragma unroll
        for (int i = 0; i < QL; ++i) {
          const int k = h * QL + i;  // outputs k and k + L/2; both have the parity of k
          const float2 v0 = y[r][0][i], v1 = y[r][1][i];
          base[k * step] = (k & 1) ? make_float2(-v0.x, -v0.y) : v0;
          base[(k + HL) * step] = ((k + HL) & 1) ? make_float2(-v1.x, -v1.y) : v1;
        }
      }
      __syncthreads();
    }
  }
}

// The same transform with one thread per line (an L-point register FFT each).
// It needs twice the registers per line and leaves half of the threads idle at
// L = 32, but the wide degridder at L <= 32 (the tightest register budget)
// spills less with it and measured faster.
template <int L, int NT, bool INV>
__device__ __forceinline__ void lds_centred_dft_one_thread_per_line(float2 *sg, const float2 *tw) {
  using Lay = SgLayout<L>;
  constexpr int NPIX = L * L, PPT = NPIX / NT, H = L / 2;
  const int tid = threadIdx.x;
  static_assert(Lay::FFT, "subgrid transform: L = 2^n or 3 x 2^n");
  {
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
      for (int line = tid; line < 4 * L; line += NT) {
        const int pol = line / L, q = line % L;  // q: row (pass 0) or column (pass 1)
        float2 *base = sg + pol * Lay::POL + (pass == 0 ? q * Lay::RS : q);
        const int step = pass == 0 ? 1 : Lay::RS;
        float2 x[L];
#pragma unroll
        for (int n = 0; n < L; ++n) {
          const float2 v = base[n * step];
          const bool flip = pass == 0 && ((n + q) & 1);
          x[n] = flip ? make_float2(-v.x, -v.y) : v;
        }
        reg_fft<L, INV>(x);
#pragma unroll
        for (int k = 0; k < L; ++k) base[k * step] = (k & 1) ? make_float2(-x[k].x, -x[k].y) : x[k];
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Tile-piece layout of a transformed subgrid in the gridder's scratch.  The
// adder's tiles (kAdderTile x kAdderTile, aligned to the grid) cut a subgrid
// with corner (x0, y0) into up to 3 x 3 pieces; the subgrid is stored piece by
// piece (row bands top to bottom, pieces left to right, each piece row-major),
// so that the workgroup that owns a tile reads each of its pieces as one
// contiguous block and no cache line is shared by two tiles' pieces except at
// piece ends.  Element (b, a) (row, column) of a subgrid whose corner lies at
// (ox, oy) = (x0, y0) mod kAdderTile:
//   row band  bi = (b + oy) / T, rows [rs, rs + h) of the subgrid;
//   column    ci = (a + ox) / T, columns [cs, cs + w);
//   offset    rs L + h cs + (b - rs) w + (a - cs).
template <int L>
__device__ __forceinline__ int piece_index(int b, int a, int ox, int oy) {
  constexpr int T = kAdderTile;
  const int bi = (b + oy) / T, ci = (a + ox) / T;
  const int rs = bi == 0 ? 0 : bi * T - oy, cs = ci == 0 ? 0 : ci * T - ox;
  const int h = min(L, (bi + 1) * T - oy) - rs, w = min(L, (ci + 1) * T - ox) - cs;
  return rs * L + h * cs + (b - rs) * w + (a - cs);
}

// ---------------------------------------------------------------------------
// Gridder: PPT pixels per thread.  Plain form: one workgroup per subgrid.
// Persistent form: a fixed grid of workgroups pulls subgrids from a work
// queue (a device counter over a cost-sorted list) until the list is empty.

// Longest run of channels whose phasors are advanced by multiplication with a
// per-run step phasor instead of evaluating sin and cos per sample.
constexpr int kChanRun = 16;

template <int L>
struct GridderSmem {
  static constexpr int NT = Cfg<L>::NT;
  static constexpr int CH = NT < 256 ? NT : 256;  // visibilities staged per round
  static constexpr int SG_BYTES = SgLayout<L>::SIZE * 8, STAGE_BYTES = CH * 64;
  static constexpr int RAW = SG_BYTES > STAGE_BYTES ? SG_BYTES : STAGE_BYTES;
  float4 raw[RAW / 16];  // staged samples (offsets, channel steps, visibilities), then the subgrid
  float2 tw[L];
  int next;              // work-queue item of the persistent form
  unsigned ybits;        // separable form: largest |visibility component| of the subgrid (float bits)
};

// Per-thread pixel coordinates (PPT pixels tid + r NT).
template <int L>
struct PixelCoords {
  static constexpr int PPT = L * L / Cfg<L>::NT;
  float l[PPT], m[PPT], n[PPT];
  __device__ __forceinline__ void load(const float4 *lmn) {
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      const float4 q = lmn[threadIdx.x + r * Cfg<L>::NT];
      l[r] = q.x;
      m[r] = q.y;
      n[r] = q.z;
    }
  }
};

// acc[r] += visibility * phasor[r] for the four polarisations, two fused
// multiply-adds per real output.
template <int PPT>
__device__ __forceinline__ void grid_accumulate(float2 (&acc)[PPT][4], const float2 (&ph)[PPT], float4 v01,
                                                float4 v23) {
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    cmac(acc[r][0], v01.x, v01.y, ph[r].x, ph[r].y);
    cmac(acc[r][1], v01.z, v01.w, ph[r].x, ph[r].y);
    cmac(acc[r][2], v23.x, v23.y, ph[r].x, ph[r].y);
    cmac(acc[r][3], v23.z, v23.w, ph[r].x, ph[r].y);
  }
}

// Gridder epilogue: this thread's pixels' sums acc (tid + r NT) -> A-terms x
// taper per pixel -> LDS -> centred DFT (stage 1) -> the subgrid's slot of
// a.subgrids_out.  Starts with s_sg free (all threads past their last read of
// it); the caller synchronises before reusing shared memory.
template <int L>
__device__ __forceinline__ void grid_finish(const KernelArgs &a, const DevSubgrid &d, int local,
                                            float2 (&acc)[L * L / Cfg<L>::NT][4], float2 *s_sg, const float2 *tw) {
  constexpr int NT = Cfg<L>::NT, NPIX = L * L, PPT = NPIX / NT;
  const int tid = threadIdx.x;
  const float2 *j1 = a.aterms + int64_t(d.a1) * NPIX * 4;
  const float2 *j2 = a.aterms + int64_t(d.a2) * NPIX * 4;
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int pix = tid + r * NT;
    float2 J1[4], J2[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      J1[e] = j1[pix * 4 + e];
      J2[e] = j2[pix * 4 + e];
    }
    apply_aterms_grid(J1, J2, a.taper[pix], acc[r]);
#pragma unroll
    for (int pol = 0; pol < 4; ++pol) s_sg[SgLayout<L>::idx(pol, pix)] = acc[r][pol];
  }
  __syncthreads();
  if (a.stage == 1) lds_centred_dft<L, NT, false>(s_sg, tw);

  float2 *out = a.subgrids_out + int64_t(local) * 4 * NPIX;
  const int ox = d.x0 % kAdderTile, oy = d.y0 % kAdderTile;
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int pix = tid + r * NT;
    const int o = a.pieces ? piece_index<L>(pix / L, pix % L, ox, oy) : pix;
#pragma unroll
    for (int pol = 0; pol < 4; ++pol) {
      // streamed past the caches: the adder reads the subgrids back only after the whole launch, by
      // which time tens of GB have gone through; keeping them out leaves L2 and MALL to the Jones blocks
      const float2 v = s_sg[SgLayout<L>::idx(pol, pix)];
      double bits;
      __builtin_memcpy(&bits, &v, 8);
      __builtin_nontemporal_store(bits, reinterpret_cast<double *>(out + pol * NPIX + o));
    }
  }
}

// Grid plan subgrid a.first + local into a.subgrids_out[local].  Starts and ends
// with all threads past a barrier-free point; the caller synchronises before
// reusing shared memory.
template <int L, bool FP32_PHASE>
__device__ __forceinline__ void grid_one(const KernelArgs &a, int local, GridderSmem<L> &sm,
                                         const PixelCoords<L> &pc) {
  constexpr int NT = Cfg<L>::NT, NPIX = L * L, PPT = NPIX / NT, CH = GridderSmem<L>::CH;
  float4 *s_uvw = sm.raw;                        // [CH] offsets (x, y, z) and run length (w)
  float4 *s_step = sm.raw + CH;                  // [CH] channel steps of run starts
  float4 *s_vis = sm.raw + 2 * CH;               // [CH][2]
  float2 *s_sg = reinterpret_cast<float2 *>(sm.raw);
  const int tid = threadIdx.x;
  const DevSubgrid d = a.subgrids[a.first + local];
  const double S = a.image_size;
  const double u0 = double(d.x0 + L / 2 - a.grid_size / 2) / S;
  const double v0 = double(d.y0 + L / 2 - a.grid_size / 2) / S;
  float p0[PPT];
#pragma unroll
  for (int r = 0; r < PPT; ++r)
    p0[r] = FP32_PHASE ? float(u0) * pc.l[r] + float(v0) * pc.m[r] + float(d.w0) * pc.n[r] : 0.0f;
  const bool recur = !FP32_PHASE && a.chan_recur != 0;

  float2 acc[PPT][4];
  float2 ph[PPT], st[PPT];  // current phasor and channel-step phasor per pixel
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    ph[r] = st[r] = make_float2(1.0f, 0.0f);
#pragma unroll
    for (int pol = 0; pol < 4; ++pol) acc[r][pol] = make_float2(0.0f, 0.0f);
  }

  for (int k0 = 0; k0 < d.nvis; k0 += CH) {
    const int nk = min(CH, d.nvis - k0);
    if (tid < nk) {
      const uint32_t *smp = a.samples + d.vis_offset + k0;
      const uint32_t pk = smp[tid];
      const int dc = int(pk & 0xffffu);
      const int t = d.t0 + int(pk >> 16), c = d.c0 + dc;
      const int64_t bt = int64_t(d.bl) * a.nr_timesteps + t;
      const double *q = a.uvw + bt * 3;
      const double s = a.freqs[c] / kC0;
      // Runs: a sample starts a run unless it is the next channel, in the same timestep, of the
      // sample before it.  A run's phasors after the first are the first times powers of one step
      // phasor.  Runs stop at staging chunk ends and every kChanRun channels, which bounds the
      // error of the recurrence.  Run starts store the run length; other samples store 0.
      int len = 0;
      const bool cont_prev = recur && tid > 0 && smp[tid - 1] == pk - 1u && dc % kChanRun != 0;
      if (!cont_prev) {
        len = 1;
        if (recur)
          while (tid + len < nk && smp[tid + len] == pk + uint32_t(len) && (dc + len) % kChanRun != 0) ++len;
      }
      float4 o;
      if (FP32_PHASE) {
        const float sf = float(s);
        o = make_float4(float(q[0]) * sf, float(q[1]) * sf, float(q[2]) * sf, __int_as_float(len));
      } else {
        o = make_float4(float(q[0] * s - u0), float(q[1] * s - v0), float(q[2] * s - d.w0), __int_as_float(len));
      }
      s_uvw[tid] = o;
      if (len > 1) {
        const double ds = (a.freqs[c + 1] - a.freqs[c]) / kC0;
        s_step[tid] = make_float4(float(q[0] * ds), float(q[1] * ds), float(q[2] * ds), 0.0f);
      }
      const float4 *vp = reinterpret_cast<const float4 *>(a.vis_in + (bt * a.nr_channels + c) * 4);
      s_vis[2 * tid] = vp[0];
      s_vis[2 * tid + 1] = vp[1];
    }
    __syncthreads();
    for (int k = 0; k < nk;) {
      const float4 o = s_uvw[k];
      const int len = __builtin_amdgcn_readfirstlane(__float_as_int(o.w));
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        float f = o.x * pc.l[r] + o.y * pc.m[r] + o.z * pc.n[r];
        if (FP32_PHASE) f -= p0[r];
        f = __builtin_amdgcn_fractf(f);
        ph[r] = make_float2(__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f));
      }
      grid_accumulate<PPT>(acc, ph, s_vis[2 * k], s_vis[2 * k + 1]);
      if (len > 1) {
        const float4 q = s_step[k];
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
          const float f = __builtin_amdgcn_fractf(q.x * pc.l[r] + q.y * pc.m[r] + q.z * pc.n[r]);
          st[r] = make_float2(__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f));
        }
        // two channels per trip, alternating between two phasor registers
        int j = 1;
        for (; j + 1 < len; j += 2) {
          float2 pa[PPT];
#pragma unroll
          for (int r = 0; r < PPT; ++r) pa[r] = cmul(ph[r], st[r]);
          grid_accumulate<PPT>(acc, pa, s_vis[2 * (k + j)], s_vis[2 * (k + j) + 1]);
#pragma unroll
          for (int r = 0; r < PPT; ++r) ph[r] = cmul(pa[r], st[r]);
          grid_accumulate<PPT>(acc, ph, s_vis[2 * (k + j + 1)], s_vis[2 * (k + j + 1) + 1]);
        }
        if (j < len) {
#pragma unroll
          for (int r = 0; r < PPT; ++r) ph[r] = cmul(ph[r], st[r]);
          grid_accumulate<PPT>(acc, ph, s_vis[2 * (k + j)], s_vis[2 * (k + j) + 1]);
        }
      }
      k += len > 1 ? len : 1;
    }
    __syncthreads();
  }

  grid_finish<L>(a, d, local, acc, s_sg, sm.tw);
}

// Plain form: one workgroup per subgrid, local index order[blockIdx.x] (or blockIdx.x without a list).
template <int L, bool FP32_PHASE>
__global__ void __launch_bounds__(Cfg<L>::NT) gridder_kernel(KernelArgs a, const int32_t *order) {
  __shared__ GridderSmem<L> sm;
  if (threadIdx.x < L) sm.tw[threadIdx.x] = a.twiddle[threadIdx.x];
  PixelCoords<L> pc;
  pc.load(a.lmn);
  grid_one<L, FP32_PHASE>(a, order ? order[blockIdx.x] : int(blockIdx.x), sm, pc);
}

// Persistent form: items order[0 .. count-1] (local subgrid indices, costliest
// first) are taken one at a time through the counter *queue_head (zero before
// the launch).  Every workgroup leaves once the counter passes the end.  At
// L = 32 it is held to 4 waves per SIMD like the one-subgrid form (which needs
// 120 VGPRs); the persistent loop otherwise takes 150 (3 waves), and 4 waves
// with 18 spilled VGPRs measured faster.
template <int L>
constexpr int grid_persistent_min_waves() {
  return L == 32 ? 4 : 1;
}

template <int L, bool FP32_PHASE>
__global__ void __launch_bounds__(Cfg<L>::NT) __attribute__((amdgpu_waves_per_eu(grid_persistent_min_waves<L>())))
gridder_persistent_kernel(KernelArgs a, const int32_t *order, int32_t *queue_head) {
  __shared__ GridderSmem<L> sm;
  if (threadIdx.x < L) sm.tw[threadIdx.x] = a.twiddle[threadIdx.x];
  PixelCoords<L> pc;
  pc.load(a.lmn);
  for (;;) {
    if (threadIdx.x == 0) sm.next = atomicAdd(queue_head, 1);
    __syncthreads();
    const int item = sm.next;
    if (item >= a.count) break;
    grid_one<L, FP32_PHASE>(a, order[item], sm, pc);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Separable form of the subgrid sum, on the matrix cores (L = 32).
//
// Pixel (j, i) of a subgrid sits at l = x_i, m = x_j.  Writing
// n'_ij = a(x_i) + a(x_j) + c_ij with a(x) = sqrt(1 - x^2) - 1 (an exact split:
// c_ij is whatever of n' is not a sum of a function of l and one of m, about
// -l^2 m^2 / 4, at most about S^4 / 32), the phasor of sample k factors as
//   E_k(i, j) = U_k(i) V_k(j) exp(2 pi i dw_k c_ij),
//   U_k(i) = exp(2 pi i (du_k x_i + dw_k a_i)),  V_k(j) = exp(2 pi i (dv_k x_j + dw_k a_j)),
// and the last factor is expanded to order N, which the plan chooses per
// subgrid from its largest |dw| so that the truncation, below
// (2 pi |dw| max|c|)^(N+1) / (N+1)!, stays under 1e-6:
//   S[j][i] = sum_n (2 pi i c_ij)^n / n! G_n[j][i],  G_n[j][i] = sum_k V_k(j) dw_k^n Y_k U_k(i).
// For each polarisation each G_n is a dense (32 x K)(K x 32) complex matrix
// product: v_mfma_f32_32x32x16_f16 on operands split into fp16 high and low
// parts (22 significant bits), accumulating hi*hi + hi*lo + lo*hi in float32.
// The sines and cosines drop from one pair per (sample, pixel) to two pairs per
// (sample, row or column).  Operands are scaled by powers of two (the largest
// visibility component of the subgrid, the plan's largest |dw|) to stay inside
// the fp16 range; the scales are undone exactly on the float32 sums.

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kSeparableMaxOrder = 1;  // expansion orders the matrix-core kernels carry

// x = hi + lo, both fp16 (truncating conversions: x - hi is exact in float32)
__device__ __forceinline__ void split_half8(const float (&x)[8], half8 &hi, half8 &lo) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const auto h = __builtin_amdgcn_cvt_pkrtz(x[2 * q], x[2 * q + 1]);
    const auto r = __builtin_amdgcn_cvt_pkrtz(x[2 * q] - float(h[0]), x[2 * q + 1] - float(h[1]));
    hi[2 * q] = h[0];
    hi[2 * q + 1] = h[1];
    lo[2 * q] = r[0];
    lo[2 * q + 1] = r[1];
  }
}

// d += (ah + al)(bh + bl) without the lo*lo term
__device__ __forceinline__ floatx16 mfma_split(half8 ah, half8 al, half8 bh, half8 bl, floatx16 d) {
  d = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, d, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bl, d, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, bh, d, 0, 0, 0);
  return d;
}

// Largest of v over the workgroup (v >= 0), through *slot (zeroed by the caller before a barrier).
__device__ __forceinline__ void block_max_into(float v, unsigned *slot) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) atomicMax(slot, __float_as_uint(v));
}

// Matrix-core operands of one block of 16 samples for one lane: A = V (row rc, samples kh .. kh + 7) as fp16
// high/low parts of its real part, its imaginary part and minus its imaginary part; B = Y U for order 0 (high
// and low parts) and dw Y U for order 1 (high parts: that term is scaled by |2 pi dw c| <= 1.5e-3, so fp16
// rounding of it stays below 1e-6 of a phasor).
struct SepOps {
  half8 vrh, vrl, vih, vil, nvih, nvil;
  half8 brh, brl, bih, bil;
  half8 b1rh, b1ih;
};

// s_u, s_v, s_w: staged du, dv, dw; s_yr, s_yi: this polarisation's visibilities; samples kb + kh + (0..7).
__device__ __forceinline__ void sep_operands(const float *s_u, const float *s_v, const float *s_w, const float *s_yr,
                                             const float *s_yi, int k, float2 xa, float yinv, float winv,
                                             bool order1, SepOps &o) {
  float du[8], dv[8], dw[8], yr[8], yi[8];
  *reinterpret_cast<float4 *>(du) = *reinterpret_cast<const float4 *>(s_u + k);
  *reinterpret_cast<float4 *>(du + 4) = *reinterpret_cast<const float4 *>(s_u + k + 4);
  *reinterpret_cast<float4 *>(dv) = *reinterpret_cast<const float4 *>(s_v + k);
  *reinterpret_cast<float4 *>(dv + 4) = *reinterpret_cast<const float4 *>(s_v + k + 4);
  *reinterpret_cast<float4 *>(dw) = *reinterpret_cast<const float4 *>(s_w + k);
  *reinterpret_cast<float4 *>(dw + 4) = *reinterpret_cast<const float4 *>(s_w + k + 4);
  *reinterpret_cast<float4 *>(yr) = *reinterpret_cast<const float4 *>(s_yr + k);
  *reinterpret_cast<float4 *>(yr + 4) = *reinterpret_cast<const float4 *>(s_yr + k + 4);
  *reinterpret_cast<float4 *>(yi) = *reinterpret_cast<const float4 *>(s_yi + k);
  *reinterpret_cast<float4 *>(yi + 4) = *reinterpret_cast<const float4 *>(s_yi + k + 4);
  float vr[8], vi[8], br[8], bi[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const float pv = __builtin_amdgcn_fractf(dv[s] * xa.x + dw[s] * xa.y);
    const float pu = __builtin_amdgcn_fractf(du[s] * xa.x + dw[s] * xa.y);
    vr[s] = __builtin_amdgcn_cosf(pv);
    vi[s] = __builtin_amdgcn_sinf(pv);
    const float ur = __builtin_amdgcn_cosf(pu), ui = __builtin_amdgcn_sinf(pu);
    const float y0 = yr[s] * yinv, y1 = yi[s] * yinv;
    br[s] = y0 * ur - y1 * ui;
    bi[s] = y0 * ui + y1 * ur;
  }
  split_half8(vr, o.vrh, o.vrl);
  split_half8(vi, o.vih, o.vil);
  o.nvih = -o.vih;
  o.nvil = -o.vil;
  split_half8(br, o.brh, o.brl);
  split_half8(bi, o.bih, o.bil);
  if (order1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float w0 = dw[2 * q] * winv, w1 = dw[2 * q + 1] * winv;
      const auto hr = __builtin_amdgcn_cvt_pkrtz(br[2 * q] * w0, br[2 * q + 1] * w1);
      const auto hi = __builtin_amdgcn_cvt_pkrtz(bi[2 * q] * w0, bi[2 * q + 1] * w1);
      o.b1rh[2 * q] = hr[0];
      o.b1rh[2 * q + 1] = hr[1];
      o.b1ih[2 * q] = hi[0];
      o.b1ih[2 * q + 1] = hi[1];
    }
  }
}

// G_0 += V (Y U) with the split products; G_1 += V (dw Y U) with high parts (order 1)
__device__ __forceinline__ void sep_mfma(const SepOps &o, bool order1, floatx16 (&gr)[2], floatx16 (&gi)[2]) {
  // G_r += Vr Br - Vi Bi,  G_i += Vr Bi + Vi Br
  gr[0] = mfma_split(o.vrh, o.vrl, o.brh, o.brl, gr[0]);
  gi[0] = mfma_split(o.vrh, o.vrl, o.bih, o.bil, gi[0]);
  gr[0] = mfma_split(o.nvih, o.nvil, o.bih, o.bil, gr[0]);
  gi[0] = mfma_split(o.vih, o.vil, o.brh, o.brl, gi[0]);
  if (order1) {
    gr[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(o.vrh, o.b1rh, gr[1], 0, 0, 0);
    gi[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(o.vrh, o.b1ih, gi[1], 0, 0, 0);
    gr[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(o.nvih, o.b1ih, gr[1], 0, 0, 0);
    gi[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(o.vih, o.b1rh, gi[1], 0, 0, 0);
  }
}

// Grid plan subgrid a.first + local with the separable form (d.order = N in 0..1).  Four waves, wave w
// accumulates polarisation w.  A, B and D of v_mfma_f32_32x32x16_f16: lane l holds A[l % 32][8 (l / 32) + s]
// and B[8 (l / 32) + s][l % 32] (s = 0..7); D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] is element r of lane l.
// The operands of the next block of samples are formed while the matrix cores work on the current one.
template <int L>
__device__ __forceinline__ void grid_one_mfma(const KernelArgs &a, int local, GridderSmem<L> &sm) {
  static_assert(L == 32 && Cfg<L>::NT == 256, "the matrix-core gridder runs 32 x 32 subgrids on four waves");
  static_assert(kSeparableMaxOrder == 1, "the matrix-core gridder carries orders 0 and 1");
  constexpr int NT = Cfg<L>::NT, NPIX = L * L, PPT = NPIX / NT, CH = GridderSmem<L>::CH;
  float *s_u = reinterpret_cast<float *>(sm.raw);  // [CH] du, then dv, dw, then [4][2][CH] visibilities
  float *s_v = s_u + CH, *s_w = s_u + 2 * CH;
  float *s_y = s_u + 3 * CH;
  float2 *s_sg = reinterpret_cast<float2 *>(sm.raw);
  const int tid = threadIdx.x, lane = tid & 63, pol = tid >> 6;
  const DevSubgrid d = a.subgrids[a.first + local];
  const int K = d.nvis;
  const bool order1 = d.order >= 1;
  const double S = a.image_size;
  const double u0 = double(d.x0 + L / 2 - a.grid_size / 2) / S;
  const double v0 = double(d.y0 + L / 2 - a.grid_size / 2) / S;
  const uint32_t *smp = a.samples + d.vis_offset;
  const float winv = ldexpf(1.0f, -int(d.wexp));
  const int rc = lane & 31, kh = (lane >> 5) * 8;  // row (A) / column (B) of this lane, its first sample slot
  const float2 xa = a.sep[rc];                      // (x, a(x)) of row / column rc
  const float *s_yr = s_y + (2 * pol) * CH, *s_yi = s_y + (2 * pol + 1) * CH;
  floatx16 gr[2], gi[2];
#pragma unroll
  for (int n = 0; n < 2; ++n)
#pragma unroll
    for (int e = 0; e < 16; ++e) gr[n][e] = gi[n][e] = 0.0f;

  // The fp16 operands carry the visibilities divided by 2^yexp >= their largest component so far; when a
  // later staging round holds a larger one, the sums are rescaled by the (exact) power of two first.
  int yexp = -126;
  for (int k0 = 0; k0 < K; k0 += CH) {
    const int nk = min(CH, K - k0), nkp = (nk + 15) & ~15;  // whole blocks of 16; the padding is zero
    float ym = 0.0f;
    if (tid == 0) sm.ybits = 0u;
    if (tid < nkp) {
      float du = 0.0f, dv = 0.0f, dw = 0.0f;
      float4 p0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), p1 = p0;
      if (tid < nk) {
        const uint32_t pk = smp[k0 + tid];
        const int t = d.t0 + int(pk >> 16), c = d.c0 + int(pk & 0xffffu);
        const int64_t bt = int64_t(d.bl) * a.nr_timesteps + t;
        const double *q = a.uvw + bt * 3;
        const double sc = a.freqs[c] / kC0;
        du = float(q[0] * sc - u0);
        dv = float(q[1] * sc - v0);
        dw = float(q[2] * sc - d.w0);
        const float4 *vp = reinterpret_cast<const float4 *>(a.vis_in + (bt * a.nr_channels + c) * 4);
        p0 = vp[0];
        p1 = vp[1];
      }
      s_u[tid] = du;
      s_v[tid] = dv;
      s_w[tid] = dw;
      s_y[0 * CH + tid] = p0.x;
      s_y[1 * CH + tid] = p0.y;
      s_y[2 * CH + tid] = p0.z;
      s_y[3 * CH + tid] = p0.w;
      s_y[4 * CH + tid] = p1.x;
      s_y[5 * CH + tid] = p1.y;
      s_y[6 * CH + tid] = p1.z;
      s_y[7 * CH + tid] = p1.w;
      ym = fmaxf(fmaxf(fmaxf(fabsf(p0.x), fabsf(p0.y)), fmaxf(fabsf(p0.z), fabsf(p0.w))),
                 fmaxf(fmaxf(fabsf(p1.x), fabsf(p1.y)), fmaxf(fabsf(p1.z), fabsf(p1.w))));
    }
    __syncthreads();
    block_max_into(ym, &sm.ybits);
    __syncthreads();
    int e = -126;
    if (sm.ybits) (void)frexpf(__uint_as_float(sm.ybits), &e);  // largest < 2^e
    if (e > yexp) {
      const float r = ldexpf(1.0f, yexp - e);
#pragma unroll
      for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          gr[n][q] *= r;
          gi[n][q] *= r;
        }
      yexp = e;
    }
    const float yinv = ldexpf(1.0f, -yexp);
    for (int kb = 0; kb < nkp; kb += 16) {
      SepOps o;
      sep_operands(s_u, s_v, s_w, s_yr, s_yi, kb + kh, xa, yinv, winv, order1, o);
      sep_mfma(o, order1, gr, gi);
    }
    __syncthreads();  // staging and sm.ybits are reused by the next round
  }

  // S = 2^yexp (G_0 + 2 pi i 2^wexp c G_1), element by element, into LDS
  const float ys = ldexpf(1.0f, yexp), zs = 6.283185307179586f * ldexpf(1.0f, int(d.wexp));
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int j = 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3), i = lane & 31;
    float2 sv = make_float2(gr[0][e], gi[0][e]);
    if (order1) {
      const float z = zs * a.cross[j * L + i];  // i z G_1
      sv = cadd(sv, make_float2(-z * gi[1][e], z * gr[1][e]));
    }
    s_sg[SgLayout<L>::idx(pol, j * L + i)] = make_float2(sv.x * ys, sv.y * ys);
  }
  __syncthreads();
  float2 acc[PPT][4];
#pragma unroll
  for (int r = 0; r < PPT; ++r)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[r][p] = s_sg[SgLayout<L>::idx(p, tid + r * NT)];
  __syncthreads();
  grid_finish<L>(a, d, local, acc, s_sg, sm.tw);
}

// Held to 3 waves per SIMD (144 VGPRs, no spills): three workgroups per compute unit hide the staging
// loads, barriers and epilogue of one subgrid behind the others; measured 20 % faster than the 2 waves the
// compiler picks by itself (on the SKA-low-like share, 58.8 -> 46.9 ms).  4 waves spill 57 VGPRs and lose.
template <int L>
__global__ void __launch_bounds__(Cfg<L>::NT) __attribute__((amdgpu_waves_per_eu(3)))
gridder_mfma_kernel(KernelArgs a, const int32_t *order) {
  __shared__ GridderSmem<L> sm;
  if (threadIdx.x < L) sm.tw[threadIdx.x] = a.twiddle[threadIdx.x];
  grid_one_mfma<L>(a, order ? order[blockIdx.x] : int(blockIdx.x), sm);
}

// Held to 2 waves per SIMD; the loop would otherwise take 1.  At 3 waves it measured slower (SKA-low-like
// share: 63.7 against 54.8 ms).
template <int L>
__global__ void __launch_bounds__(Cfg<L>::NT) __attribute__((amdgpu_waves_per_eu(2)))
gridder_mfma_persistent_kernel(KernelArgs a, const int32_t *order, int32_t *queue_head) {
  __shared__ GridderSmem<L> sm;
  if (threadIdx.x < L) sm.tw[threadIdx.x] = a.twiddle[threadIdx.x];
  for (;;) {
    if (threadIdx.x == 0) sm.next = atomicAdd(queue_head, 1);
    __syncthreads();
    const int item = sm.next;
    if (item >= a.count) break;
    grid_one_mfma<L>(a, order[item], sm);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Degridder: one workgroup per subgrid.  Split + inverse DFT + A-terms into
// LDS, then the visibilities are evaluated in tasks of (64 V visibilities x a
// 1/G share of the pixels): each lane owns V visibilities, so every broadcast
// LDS read of a pixel is used V times.  Pixel shares of one visibility are
// added in LDS at the end.  V and G are chosen per subgrid to fill the waves.

constexpr int kDegridPartCap = 192;  // G * K_p limit of the partial-sum buffer (32 bytes each)
constexpr int kDegridSmallK = 128;  // subgrids with at most this many visibilities take the pixel-owner path
constexpr int kDegridSmallNB = 4;  // visibilities per cross-lane reduction


template <int L, bool SEP = false>
struct DegridderSmem {
  static constexpr bool LMN_LDS = L <= 24;  // larger subgrids read the pixel coordinates through the cache
  // the small-subgrid path reuses sg for its staged offsets and per-wave sums (float2 units); the separable
  // kernels (SEP) for their staged offsets, outputs and phasor tables
  static constexpr int SMALL = (2 * kDegridSmallK * 16 + (Cfg<L>::NT / 64) * kDegridSmallK * 32) / 8;
  static constexpr int SEPT = SEP ? 41728 / 8 : 0;
  static constexpr int SG0 = SgLayout<L>::SIZE > SMALL ? SgLayout<L>::SIZE : SMALL;
  static constexpr int SG = SG0 > SEPT ? SG0 : SEPT;
  float2 sg[SG];                            // SgLayout<L>, then [NPIX][4] after the A-terms
  float4 lmn[LMN_LDS ? L * L : 1];
  float2 tw[L];
  float2 sep[L];                            // separable form: (x_q, a_q)
  float4 part[2 * kDegridPartCap];          // [G][K] partial sums, 4 complex each
  int next;                                 // work-queue item of the persistent form
  unsigned ybits;                           // separable form: largest |image component| (float bits)
};

// Sum over the pixel share [lo, hi) for a lane's V visibilities.  RECUR: the V
// visibilities are consecutive channels of one timestep, and the phasor of
// visibility v is the phasor of visibility 0 times the v-th power of the
// channel-step phasor (offsets du, dv, w of visibility 0; step sx, sy, sz).
template <int L, int V, bool FP32_PHASE, bool RECUR>
__device__ __forceinline__ void degrid_pixels(float2 (&y)[V][4], const float (&du)[V], const float (&dv)[V],
                                              const float (&w)[V], float sx, float sy, float sz,
                                              const KernelArgs &a, const float4 *s_b, const float4 *s_lmn,
                                              int lo, int hi, float u0f, float v0f, float w0f) {
  constexpr bool LMN_LDS = DegridderSmem<L>::LMN_LDS;
  constexpr int UNROLL = V >= 8 ? 1 : 2;
#pragma unroll UNROLL
  for (int pix = lo; pix < hi; ++pix) {
    const float4 q = LMN_LDS ? s_lmn[pix] : a.lmn[pix];
    const float4 b01 = s_b[2 * pix], b23 = s_b[2 * pix + 1];
    if (RECUR) {
      // y += B * exp(-i phase): with E = exp(+i phase), add B * conj(E)
      const float f0 = __builtin_amdgcn_fractf(du[0] * q.x + dv[0] * q.y + w[0] * q.z);
      const float fs = __builtin_amdgcn_fractf(sx * q.x + sy * q.y + sz * q.z);
      float2 e = make_float2(__builtin_amdgcn_cosf(f0), __builtin_amdgcn_sinf(f0));
      const float2 st = make_float2(__builtin_amdgcn_cosf(fs), __builtin_amdgcn_sinf(fs));
#pragma unroll
      for (int v = 0; v < V; ++v) {
        if (v > 0) e = cmul(e, st);
        cmac(y[v][0], b01.x, b01.y, e.x, -e.y);
        cmac(y[v][1], b01.z, b01.w, e.x, -e.y);
        cmac(y[v][2], b23.x, b23.y, e.x, -e.y);
        cmac(y[v][3], b23.z, b23.w, e.x, -e.y);
      }
    } else {
      const float off = FP32_PHASE ? u0f * q.x + v0f * q.y + w0f * q.z : 0.0f;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        float ph = du[v] * q.x + dv[v] * q.y + w[v] * q.z;
        if (FP32_PHASE) ph -= off;
        ph = __builtin_amdgcn_fractf(ph);
        const float sn = __builtin_amdgcn_sinf(ph), cs = __builtin_amdgcn_cosf(ph);
        // y += B * exp(-i phase) = B * (cs - i sn)
        cmac(y[v][0], b01.x, b01.y, cs, -sn);
        cmac(y[v][1], b01.z, b01.w, cs, -sn);
        cmac(y[v][2], b23.x, b23.y, cs, -sn);
        cmac(y[v][3], b23.z, b23.w, cs, -sn);
      }
    }
  }
}

// Output index (into vis_out, in complex units) of sample k of subgrid d.
__device__ __forceinline__ int64_t degrid_out_index(const KernelArgs &a, const DevSubgrid &d, int k) {
  const uint32_t pk = a.samples[d.vis_offset + k];
  const int t = d.t0 + int(pk >> 16), c = d.c0 + int(pk & 0xffffu);
  return ((int64_t(d.bl) * a.nr_timesteps + t) * a.nr_channels + c) * 4;
}

// A wave holds 64/(Q SPLIT) lane groups; each group works on one task: Q x V
// visibilities (lane i of the group owns the V consecutive samples
// (chunk * Q + i) * V + v) over a 1/G share of the pixels.  SPLIT = 2 halves
// that share again between the two 32-lane halves of the wave (Q = 32), whose
// sums are added by a cross-lane exchange: a lane owns twice the visibilities
// for the same number of lanes per task.
template <int L, int V, int SPLIT, bool FP32_PHASE>
__device__ __forceinline__ void degrid_tasks(const KernelArgs &a, const DevSubgrid &d, const float4 *s_b,
                                             const float4 *s_lmn, float4 *s_part, int G, int nchunks, int Q,
                                             double u0, double v0) {
  constexpr int NT = Cfg<L>::NT, NPIX = L * L, W = NT / 64;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int TL = Q * SPLIT;  // lanes per task
  const int R = 64 / TL, lt = lane % TL, lq = lt % Q, half = lt / Q;
  const float u0f = float(u0), v0f = float(v0), w0f = float(d.w0);
  const int K = d.nvis;
  const bool recur = !FP32_PHASE && V > 1 && a.chan_recur != 0;
  for (int task = wave * R + lane / TL; task < nchunks * G; task += W * R) {
    const int chunk = task / G, g = task % G;
    const int kbase = (chunk * Q + lq) * V;
    // this lane's valid samples are consecutive channels of one timestep
    const int nv = min(V, K - kbase);
    const uint32_t pk0 = nv > 0 ? a.samples[d.vis_offset + kbase] : 0u;
    bool run = recur;
    if (nv > 1) run = run && a.samples[d.vis_offset + kbase + nv - 1] == pk0 + uint32_t(nv - 1) &&
                      int(pk0 & 0xffffu) + nv - 1 <= 0xffff;
    const bool wave_runs = __all(run);  // uniform: the recurrence is taken by whole waves
    float du[V], dv[V], w[V];
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int k = kbase + v;
      du[v] = dv[v] = w[v] = 0.0f;
      if (k < K && (v == 0 || !wave_runs)) {
        const uint32_t pk = a.samples[d.vis_offset + k];
        const int t = d.t0 + int(pk >> 16), c = d.c0 + int(pk & 0xffffu);
        const int64_t bt = int64_t(d.bl) * a.nr_timesteps + t;
        const double *q = a.uvw + bt * 3;
        const double s = a.freqs[c] / kC0;
        if (FP32_PHASE) {
          const float sf = float(s);
          du[v] = float(q[0]) * sf;
          dv[v] = float(q[1]) * sf;
          w[v] = float(q[2]) * sf;
        } else {
          du[v] = float(q[0] * s - u0);
          dv[v] = float(q[1] * s - v0);
          w[v] = float(q[2] * s - d.w0);
        }
        if (v == 0 && wave_runs && nv > 1) {  // the step to the next channel
          const double ds = (a.freqs[c + 1] - a.freqs[c]) / kC0;
          sx = float(q[0] * ds);
          sy = float(q[1] * ds);
          sz = float(q[2] * ds);
        }
      }
    }
    float2 y[V][4];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int pol = 0; pol < 4; ++pol) y[v][pol] = make_float2(0.0f, 0.0f);
    const int span = NPIX / G / SPLIT;
    const int lo = g * (NPIX / G) + half * span, hi = lo + span;
    if (wave_runs)
      degrid_pixels<L, V, FP32_PHASE, true>(y, du, dv, w, sx, sy, sz, a, s_b, s_lmn, lo, hi, u0f, v0f, w0f);
    else
      degrid_pixels<L, V, FP32_PHASE, false>(y, du, dv, w, sx, sy, sz, a, s_b, s_lmn, lo, hi, u0f, v0f, w0f);
    if (SPLIT == 2) {
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int pol = 0; pol < 4; ++pol) {
          y[v][pol].x += __shfl_xor(y[v][pol].x, 32);
          y[v][pol].y += __shfl_xor(y[v][pol].y, 32);
        }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int k = kbase + v;
      // with SPLIT = 2 both halves hold the sums: the lower half writes the first V/2 samples
      if (k >= K || (SPLIT == 2 && (v < V / 2) != (half == 0))) continue;
      const float4 r0 = make_float4(y[v][0].x, y[v][0].y, y[v][1].x, y[v][1].y);
      const float4 r1 = make_float4(y[v][2].x, y[v][2].y, y[v][3].x, y[v][3].y);
      if (G == 1) {
        float4 *o = reinterpret_cast<float4 *>(a.vis_out + degrid_out_index(a, d, k));
        o[0] = r0;
        o[1] = r1;
      } else {
        s_part[2 * (g * K + k)] = r0;
        s_part[2 * (g * K + k) + 1] = r1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Small subgrids (few visibilities): lanes own pixels, as in the gridder.  The
// visibilities' offsets are staged in LDS and broadcast; for each visibility
// every lane sums B * conj(E) over its PPT pixels, and each wave adds the
// partial sums of NB visibilities across its 64 lanes with cross-lane moves
// (no LDS); the waves' sums are added in LDS at the end.  Per visibility x
// pixel the LDS traffic is that of the gridder (one staged offset per
// visibility), where the visibility-per-lane tasks read two pixel values and
// the pixel coordinates for every (pixel, lane group) pair.


// Reduce-scatter of M = 32 or 64 values across the 64 lanes of a wave: on return
// lane l holds the sum over all lanes of v[l] (M = 64) or of v[l >> 1] (M = 32).
// Each step halves the values a lane holds: the lane keeps the half selected by
// one bit of its index and adds the same half from the lane that differs in
// that bit (bit 5: lanes 32 apart, permlane32 swap; bit 4: rows of 16,
// permlane16 swap; bits 3, 2, 1 within a row by DPP: rotate by 8, mirror within
// 8, quad permute; bit 0 for M = 32: quad permute, both lanes keep the total).
template <int M>
__device__ __forceinline__ float wave_reduce_scatter(float (&v)[M]) {
  static_assert(M == 32 || M == 64, "32 or 64 values");
  const int lane = threadIdx.x & 63;
  int h = M / 2;
  // bit 5: the swap leaves lanes 0-31 with (x_lo, y_lo) and lanes 32-63 with (x_hi, y_hi) split over the
  // two registers, so one addition gives index i on the lower and i + h on the upper half
#pragma unroll
  for (int i = 0; i < M / 2; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + M / 2]), false,
                                                    false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  h = M / 4;
  // bit 4: the same with rows of 16 lanes (odd rows of the first register swap with even rows of the second)
#pragma unroll
  for (int i = 0; i < M / 4; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + M / 4]), false,
                                                    false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  (void)h;
  // bits 3, 2, 1: DPP within a row of 16 lanes; the partner differs in the step's bit
#define IDG_DPP_STEP(BIT, CTRL, HALF)                                                                     \
  {                                                                                                       \
    const bool up = (lane >> (BIT)) & 1;                                                                  \
    _Pragma("unroll") for (int i = 0; i < (HALF); ++i) {                                                  \
      const float keep = up ? v[i + (HALF)] : v[i];                                                       \
      const float send = up ? v[i] : v[i + (HALF)];                                                       \
      v[i] = keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), (CTRL), 0xf, 0xf, \
                                                               false));                                   \
    }                                                                                                     \
  }
  IDG_DPP_STEP(3, 0x128, M / 8)  // row_ror:8: lane i <-> i ^ 8 within the row
  IDG_DPP_STEP(2, 0x141, M / 16)  // row_half_mirror: lane i <-> 7 - i within 8 (differs in bit 2)
  IDG_DPP_STEP(1, 0x4E, M / 32)   // quad_perm [2, 3, 0, 1]: lane i <-> i ^ 2
#undef IDG_DPP_STEP
  if constexpr (M == 64) {
    const bool up = lane & 1;
    const float keep = up ? v[1] : v[0];
    const float send = up ? v[0] : v[1];
    return keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), 0xB1, 0xf, 0xf, false));
  } else {
    return v[0] + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[0]), 0xB1, 0xf, 0xf, false));
  }
}

// Degrid subgrid d (K <= kDegridSmallK visibilities) with this thread's pixels' polarised values b (after the
// A-terms and taper) in registers.  `smem` is free LDS of at least kDegridSmallK * 32 + W * kDegridSmallK * 32
// bytes.  Starts after a barrier that freed smem; ends with every thread past its last LDS read.
template <int L, bool FP32_PHASE>
__device__ __forceinline__ void degrid_small(const KernelArgs &a, const DevSubgrid &d,
                                             const float2 (&b)[L * L / Cfg<L>::NT][4], float4 *smem, double u0,
                                             double v0) {
  constexpr int NT = Cfg<L>::NT, PPT = L * L / NT, W = NT / 64, NB = kDegridSmallNB, KS = kDegridSmallK;
  float4 *s_uvw = smem;                           // [KS] offsets (x, y, z) and run length (w)
  float4 *s_step = smem + KS;                     // [KS] channel steps of run starts
  float *s_red = reinterpret_cast<float *>(smem + 2 * KS);  // [W][KS][8] per-wave sums
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int K = d.nvis;
  const bool recur = !FP32_PHASE && a.chan_recur != 0;
  for (int k = tid; k < K; k += NT) {
    const uint32_t *smp = a.samples + d.vis_offset;
    const uint32_t pk = smp[k];
    const int dc = int(pk & 0xffffu);
    const int t = d.t0 + int(pk >> 16), c = d.c0 + dc;
    const double *q = a.uvw + (int64_t(d.bl) * a.nr_timesteps + t) * 3;
    const double s = a.freqs[c] / kC0;
    // channel runs as in the gridder: a run continues while the next sample is the next channel of the
    // same timestep, cut every kChanRun channels
    int len = 0;
    const bool cont_prev = recur && k > 0 && smp[k - 1] == pk - 1u && dc % kChanRun != 0;
    if (!cont_prev) {
      len = 1;
      if (recur)
        while (k + len < K && smp[k + len] == pk + uint32_t(len) && (dc + len) % kChanRun != 0) ++len;
    }
    if (FP32_PHASE) {
      const float sf = float(s);
      s_uvw[k] = make_float4(float(q[0]) * sf, float(q[1]) * sf, float(q[2]) * sf, __int_as_float(len));
    } else {
      s_uvw[k] = make_float4(float(q[0] * s - u0), float(q[1] * s - v0), float(q[2] * s - d.w0),
                             __int_as_float(len));
    }
    if (len > 1) {
      const double ds = (a.freqs[c + 1] - a.freqs[c]) / kC0;
      s_step[k] = make_float4(float(q[0] * ds), float(q[1] * ds), float(q[2] * ds), 0.0f);
    }
  }
  float pl[PPT], pm[PPT], pn[PPT], p0[PPT];
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const float4 q = a.lmn[tid + r * NT];
    pl[r] = q.x;
    pm[r] = q.y;
    pn[r] = q.z;
    p0[r] = FP32_PHASE ? float(u0) * q.x + float(v0) * q.y + float(d.w0) * q.z : 0.0f;
  }
  __syncthreads();
  float2 ph[PPT], st[PPT];
#pragma unroll
  for (int r = 0; r < PPT; ++r) ph[r] = st[r] = make_float2(1.0f, 0.0f);
  for (int k0 = 0; k0 < K; k0 += NB) {
    float y[NB * 8];
#pragma unroll
    for (int i = 0; i < NB * 8; ++i) y[i] = 0.0f;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int k = k0 + j;
      if (k < K) {
        const float4 o = s_uvw[k];
        const int len = __builtin_amdgcn_readfirstlane(__float_as_int(o.w));
        if (len > 0) {  // run start (or no run): sin and cos
#pragma unroll
          for (int r = 0; r < PPT; ++r) {
            float f = o.x * pl[r] + o.y * pm[r] + o.z * pn[r];
            if (FP32_PHASE) f -= p0[r];
            f = __builtin_amdgcn_fractf(f);
            ph[r] = make_float2(__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f));
          }
          if (len > 1) {
            const float4 q = s_step[k];
#pragma unroll
            for (int r = 0; r < PPT; ++r) {
              const float f = __builtin_amdgcn_fractf(q.x * pl[r] + q.y * pm[r] + q.z * pn[r]);
              st[r] = make_float2(__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f));
            }
          }
        } else {  // next channel of the run
#pragma unroll
          for (int r = 0; r < PPT; ++r) ph[r] = cmul(ph[r], st[r]);
        }
        // y_k += B * exp(-i phase) = B * conj(E)
#pragma unroll
        for (int r = 0; r < PPT; ++r)
#pragma unroll
          for (int pol = 0; pol < 4; ++pol) {
            float2 acc = make_float2(y[j * 8 + 2 * pol], y[j * 8 + 2 * pol + 1]);
            cmac(acc, b[r][pol].x, b[r][pol].y, ph[r].x, -ph[r].y);
            y[j * 8 + 2 * pol] = acc.x;
            y[j * 8 + 2 * pol + 1] = acc.y;
          }
      }
    }
    const float s = wave_reduce_scatter<NB * 8>(y);
    // lane l holds component (l & 7) of visibility k0 + (l >> 3)  (NB = 8) or (l >> 1): (l >> 4), ((l >> 1) & 7)
    const int idx = NB * 8 == 64 ? lane : lane >> 1;
    const int k = k0 + idx / 8;
    if (k < K && (NB * 8 == 64 || (lane & 1) == 0)) s_red[(wave * KS + k) * 8 + idx % 8] = s;
  }
  __syncthreads();
  for (int e = tid; e < K * 8; e += NT) {
    const int k = e / 8, comp = e % 8;
    float sum = s_red[k * 8 + comp];
#pragma unroll
    for (int w = 1; w < W; ++w) sum += s_red[(w * KS + k) * 8 + comp];
    reinterpret_cast<float *>(a.vis_out + degrid_out_index(a, d, k))[comp] = sum;
  }
}

// Degrid subgrid d (32 x 32, d.order in 0..1) by the separable form (the phasor factors of the gridder's
// separable form, conjugated):
//   Y_k = sum_j conj(V_k(j)) (T_0[j][k] - 2 pi i dw_k T_1[j][k]),  T_n[j][k] = sum_i (c^n B)[j][i] conj(U_k(i)).
// Per polarisation (wave) T_n is a (32 x 32)(32 x K) product on the matrix cores: A = the image B (rows j, fp16
// high/low parts, scaled by a power of two), B = conj(U) of 32 samples (lane l: sample l % 32); then every lane
// forms conj(V_k(j)) for the 16 rows j of its accumulators and the two half-waves add their dot products.
// b: this thread's pixels (tid + r NT) after the A-terms and taper; sm.sg is free and sm.ybits zero on entry.
template <int L, class SM>
__device__ __forceinline__ void degrid_sep(const KernelArgs &a, const DevSubgrid &d, const float2 (&b)[4][4],
                                           SM &sm, double u0, double v0) {
  static_assert(L == 32 && Cfg<L>::NT == 256, "the matrix-core degridder runs 32 x 32 subgrids on four waves");
  constexpr int NT = Cfg<L>::NT, PPT = 4, CH = 64;
  const int tid = threadIdx.x, lane = tid & 63, pol = tid >> 6, hw = lane >> 5, col = lane & 31;
  const bool order1 = d.order >= 1;
  const int K = d.nvis;
  float2 *s_img = sm.sg;
  float bm = 0.0f;
#pragma unroll
  for (int r = 0; r < PPT; ++r)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      bm = fmaxf(bm, fmaxf(fabsf(b[r][e].x), fabsf(b[r][e].y)));
      s_img[SgLayout<L>::idx(e, threadIdx.x + r * NT)] = b[r][e];
    }
  block_max_into(bm, &sm.ybits);
  __syncthreads();
  int bexp = -126;
  if (sm.ybits) (void)frexpf(__uint_as_float(sm.ybits), &bexp);  // largest < 2^bexp
  const float binv = ldexpf(1.0f, -bexp);
  const float cinv = ldexpf(1.0f, -a.cross_exp);
  // A operands of this wave's polarisation: row j = col, columns i = 16 q + 8 hw + s (s = 0..7)
  half8 arh[2], arl[2], aih[2], ail[2], acr[2], aci[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    float xr[8], xi[8];
#pragma unroll
    for (int s8 = 0; s8 < 8; ++s8) {
      const int i = 16 * q + 8 * hw + s8;
      const float2 v = s_img[SgLayout<L>::idx(pol, col * L + i)];
      xr[s8] = v.x * binv;
      xi[s8] = v.y * binv;
    }
    split_half8(xr, arh[q], arl[q]);
    split_half8(xi, aih[q], ail[q]);
    if (order1) {
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int i = 16 * q + 8 * hw + 2 * s2;
        // c_ij scaled by 2^-cross_exp to at most 1: unscaled (|c| ~ 1e-7) its products would underflow fp16
        const float c0 = a.cross[col * L + i] * cinv, c1 = a.cross[col * L + i + 1] * cinv;
        const auto hr = __builtin_amdgcn_cvt_pkrtz(c0 * xr[2 * s2], c1 * xr[2 * s2 + 1]);
        const auto hi = __builtin_amdgcn_cvt_pkrtz(c0 * xi[2 * s2], c1 * xi[2 * s2 + 1]);
        acr[q][2 * s2] = hr[0];
        acr[q][2 * s2 + 1] = hr[1];
        aci[q][2 * s2] = hi[0];
        aci[q][2 * s2 + 1] = hi[1];
      }
    }
  }
  __syncthreads();  // sm.sg holds the staged samples and the phasor tables below
  // Per staging round of CH samples (k < nkp, a multiple of 32), in LDS: du, dv, dw; the outputs [4 pols][2];
  // V_k(j) in float32 (real and imaginary planes [CH][kDegVS]); U_k(i) as fp16 high and low parts of its real
  // and imaginary parts (planes [CH][kDegUS]).  The phasors do not depend on the polarisation: the four waves
  // build them once per round.  Rows are padded by 16 bytes against LDS bank conflicts.
  constexpr int kDegVS = L + 4, kDegUS = L + 8;
  float *s_u = reinterpret_cast<float *>(sm.sg), *s_v = s_u + CH, *s_w = s_u + 2 * CH;
  float *s_out = s_u + 3 * CH;  // [4 pols][2][CH]
  float *t_vr = s_out + 8 * CH, *t_vi = t_vr + CH * kDegVS;
  _Float16 *t_urh = reinterpret_cast<_Float16 *>(t_vi + CH * kDegVS), *t_url = t_urh + CH * kDegUS;
  _Float16 *t_uih = t_url + CH * kDegUS, *t_uil = t_uih + CH * kDegUS;
  static_assert((11 * CH + 2 * CH * kDegVS) * 4 + 4 * CH * kDegUS * 2 <= int(sizeof(sm.sg)), "room for the tables");
  const float bsc = ldexpf(1.0f, bexp), twopi = 6.283185307179586f;
  const int fq = tid & 31, fk = tid >> 5;   // table fill: row q of samples fk + 8 m
  const float2 fxa = sm.sep[fq];
  for (int k0 = 0; k0 < K; k0 += CH) {
    const int nk = min(CH, K - k0), nkp = (nk + 31) & ~31;
    if (tid < nkp) {
      float du = 0.0f, dv = 0.0f, dw = 0.0f;
      if (tid < nk) {
        const uint32_t pk = a.samples[d.vis_offset + k0 + tid];
        const int t = d.t0 + int(pk >> 16), c = d.c0 + int(pk & 0xffffu);
        const double *q = a.uvw + (int64_t(d.bl) * a.nr_timesteps + t) * 3;
        const double sc = a.freqs[c] / kC0;
        du = float(q[0] * sc - u0);
        dv = float(q[1] * sc - v0);
        dw = float(q[2] * sc - d.w0);
      }
      s_u[tid] = du;
      s_v[tid] = dv;
      s_w[tid] = dw;
    }
    __syncthreads();
    for (int k = fk; k < nkp; k += 8) {
      const float du = s_u[k], dv = s_v[k], dw = s_w[k];
      const float pu = __builtin_amdgcn_fractf(du * fxa.x + dw * fxa.y);
      const float pv = __builtin_amdgcn_fractf(dv * fxa.x + dw * fxa.y);
      t_vr[k * kDegVS + fq] = __builtin_amdgcn_cosf(pv);
      t_vi[k * kDegVS + fq] = __builtin_amdgcn_sinf(pv);
      const float ur = __builtin_amdgcn_cosf(pu), ui = __builtin_amdgcn_sinf(pu);
      const auto h = __builtin_amdgcn_cvt_pkrtz(ur, ui);
      const auto l = __builtin_amdgcn_cvt_pkrtz(ur - float(h[0]), ui - float(h[1]));
      t_urh[k * kDegUS + fq] = h[0];
      t_uih[k * kDegUS + fq] = h[1];
      t_url[k * kDegUS + fq] = l[0];
      t_uil[k * kDegUS + fq] = l[1];
    }
    __syncthreads();
    for (int kb = 0; kb < nkp; kb += 32) {
      const int k = kb + col;  // this lane's sample
      const float dw = s_w[k];
      floatx16 t0r, t0i, t1r, t1i;
#pragma unroll
      for (int e = 0; e < 16; ++e) t0r[e] = t0i[e] = t1r[e] = t1i[e] = 0.0f;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        // conj(U_k(i)) = Ur - i Ui for i = 16 q + 8 hw + s
        const int o = k * kDegUS + 16 * q + 8 * hw;
        const half8 urh = *reinterpret_cast<const half8 *>(t_urh + o);
        const half8 url = *reinterpret_cast<const half8 *>(t_url + o);
        const half8 uih = *reinterpret_cast<const half8 *>(t_uih + o);
        const half8 uil = *reinterpret_cast<const half8 *>(t_uil + o);
        const half8 nuih = -uih, nuil = -uil;
        // T_0r += Br Ur + Bi Ui,  T_0i += Bi Ur - Br Ui
        t0r = mfma_split(arh[q], arl[q], urh, url, t0r);
        t0i = mfma_split(aih[q], ail[q], urh, url, t0i);
        t0r = mfma_split(aih[q], ail[q], uih, uil, t0r);
        t0i = mfma_split(arh[q], arl[q], nuih, nuil, t0i);
        if (order1) {
          t1r = __builtin_amdgcn_mfma_f32_32x32x16_f16(acr[q], urh, t1r, 0, 0, 0);
          t1i = __builtin_amdgcn_mfma_f32_32x32x16_f16(aci[q], urh, t1i, 0, 0, 0);
          t1r = __builtin_amdgcn_mfma_f32_32x32x16_f16(aci[q], uih, t1r, 0, 0, 0);
          t1i = __builtin_amdgcn_mfma_f32_32x32x16_f16(acr[q], nuih, t1i, 0, 0, 0);
        }
      }
      // Y_k = sum_j conj(V_k(j)) (T_0 - 2 pi i dw T_1) over this lane's rows j, then the other half-wave's
      float yr = 0.0f, yi = 0.0f;
      const float w2 = twopi * ldexpf(dw, a.cross_exp);  // T_1 carries c 2^-cross_exp
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        // rows j = 8 g + 4 hw + (0 .. 3): accumulator elements e = 4 g .. 4 g + 3
        const float4 vr4 = *reinterpret_cast<const float4 *>(t_vr + k * kDegVS + 8 * g + 4 * hw);
        const float4 vi4 = *reinterpret_cast<const float4 *>(t_vi + k * kDegVS + 8 * g + 4 * hw);
        const float vrs[4] = {vr4.x, vr4.y, vr4.z, vr4.w}, vis[4] = {vi4.x, vi4.y, vi4.z, vi4.w};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = 4 * g + r;
          const float vr = vrs[r], vi = vis[r];
          float tr = t0r[e], ti = t0i[e];
          if (order1) {
            tr = __builtin_fmaf(w2, t1i[e], tr);
            ti = __builtin_fmaf(-w2, t1r[e], ti);
          }
          yr = __builtin_fmaf(vr, tr, __builtin_fmaf(vi, ti, yr));
          yi = __builtin_fmaf(vr, ti, __builtin_fmaf(-vi, tr, yi));
        }
      }
      yr += __shfl_xor(yr, 32);
      yi += __shfl_xor(yi, 32);
      if (hw == 0 && k < nk) {
        s_out[(2 * pol) * CH + k] = yr * bsc;
        s_out[(2 * pol + 1) * CH + k] = yi * bsc;
      }
    }
    __syncthreads();
    if (tid < nk) {
      float4 *o = reinterpret_cast<float4 *>(a.vis_out + degrid_out_index(a, d, k0 + tid));
      o[0] = make_float4(s_out[0 * CH + tid], s_out[1 * CH + tid], s_out[2 * CH + tid], s_out[3 * CH + tid]);
      o[1] = make_float4(s_out[4 * CH + tid], s_out[5 * CH + tid], s_out[6 * CH + tid], s_out[7 * CH + tid]);
    }
    __syncthreads();
  }
}

// Degrid plan subgrid p (global index) into a.vis_out.  The caller has loaded
// sm.tw and sm.lmn and synchronises before reusing shared memory.  WIDE: tasks
// of full-wave lane groups run in the split shape (twice the visibilities per
// lane, two pixel halves per wave), which needs more registers.  SMALL: the
// subgrid has at most kDegridSmallK visibilities and takes the pixel-owner
// path; the two paths are separate kernels, so that each gets its own
// register allocation.
constexpr int kPathLarge = 0, kPathSmall = 1, kPathSep = 2;  // degridder kernels: visibility-per-lane tasks,
                                                              // pixel-per-lane sums, separable form

template <int L, bool FP32_PHASE, bool WIDE, int PATH, class SM>
__device__ __forceinline__ void degrid_one(const KernelArgs &a, int64_t p, SM &sm) {
  constexpr int NT = Cfg<L>::NT, NPIX = L * L, PPT = NPIX / NT, W = NT / 64;
  constexpr bool SMALL = PATH == kPathSmall;
  const int tid = threadIdx.x;
  const DevSubgrid d = a.subgrids[p];
  const int N = a.grid_size;
  if (PATH == kPathSep && tid == 0) sm.ybits = 0u;
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int pix = tid + r * NT;
    const int row = pix / L, col = pix % L;
#pragma unroll
    for (int pol = 0; pol < 4; ++pol)
      sm.sg[SgLayout<L>::idx(pol, pix)] =
          a.grid_in[((int64_t(d.layer) * 4 + pol) * N + d.y0 + row) * N + d.x0 + col];
  }
  __syncthreads();
  // one thread per line for the wide shape and the separable form (measured 3 % faster there, SKA-low-like)
  if constexpr ((WIDE || PATH == kPathSep) && L <= 32) lds_centred_dft_one_thread_per_line<L, NT, true>(sm.sg, sm.tw);
  else lds_centred_dft<L, NT, true>(sm.sg, sm.tw);

  const float2 *j1 = a.aterms + int64_t(d.a1) * NPIX * 4;
  const float2 *j2 = a.aterms + int64_t(d.a2) * NPIX * 4;
  float2 b[PPT][4];
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int pix = tid + r * NT;
    float2 J1[4], J2[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      J1[e] = j1[pix * 4 + e];
      J2[e] = j2[pix * 4 + e];
      b[r][e] = sm.sg[SgLayout<L>::idx(e, pix)];
    }
    apply_aterms_degrid(J1, J2, a.taper[pix], b[r]);
  }
  __syncthreads();
  const int K = d.nvis;
  const double S = a.image_size;
  const double u0 = double(d.x0 + L / 2 - N / 2) / S;
  const double v0 = double(d.y0 + L / 2 - N / 2) / S;
  if constexpr (PATH == kPathSep) {
    if constexpr (L == 32) degrid_sep<L>(a, d, b, sm, u0, v0);
    return;
  } else if constexpr (SMALL) {
    degrid_small<L, FP32_PHASE>(a, d, b, reinterpret_cast<float4 *>(sm.sg), u0, v0);
    return;
  }
  float4 *s_b = reinterpret_cast<float4 *>(sm.sg);  // [NPIX][2] = 4 complex per pixel
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int pix = tid + r * NT;
    s_b[2 * pix] = make_float4(b[r][0].x, b[r][0].y, b[r][1].x, b[r][1].y);
    s_b[2 * pix + 1] = make_float4(b[r][2].x, b[r][2].y, b[r][3].x, b[r][3].y);
  }
  __syncthreads();

  // lane groups of Q lanes (small subgrids use groups of 32 or 16 so that lanes are not idle),
  // visibilities per lane V and pixel shares G (a power of two): fill the W * 64/Q lane groups
  // with tasks first, then prefer the largest V (fewest LDS reads per visibility)
  const int Q = K >= 64 ? 64 : (K > 16 ? 32 : 16);
  const int slots = W * (64 / Q);
  const int nq = (K + Q - 1) / Q;
  int V = 1, G = 1, nchunks = nq, best = -1;
  for (int vc = 4; vc >= 1; vc /= 2) {
    if (vc > 1 && nq < vc) continue;
    const int nc = (nq + vc - 1) / vc;
    int gc = 1;
    while (2 * gc * nc <= slots && 2 * gc * K <= kDegridPartCap && NPIX % (2 * gc) == 0) gc *= 2;
    const int filled = min(nc * gc, slots);
    if (filled > best) {
      best = filled;
      V = vc;
      G = gc;
      nchunks = nc;
    }
  }
  // WIDE: full-wave groups (Q = 64) run as two 32-lane halves over half the pixels each, with
  // twice the visibilities per lane: the same visibilities per task, fewer phasors and pixel
  // reads per visibility
  if (WIDE && Q == 64) {
    if (V == 4)
      degrid_tasks<L, 8, 2, FP32_PHASE>(a, d, s_b, sm.lmn, sm.part, G, nchunks, 32, u0, v0);
    else if (V == 2)
      degrid_tasks<L, 4, 2, FP32_PHASE>(a, d, s_b, sm.lmn, sm.part, G, nchunks, 32, u0, v0);
    else
      degrid_tasks<L, 2, 2, FP32_PHASE>(a, d, s_b, sm.lmn, sm.part, G, nchunks, 32, u0, v0);
  } else if (Q == 32 && nchunks * G <= W) {
    // small subgrids whose tasks fit one per wave: both halves of the wave work on a task
    // (each over half of its pixels), so that twice the lanes are busy
    if (V == 4)
      degrid_tasks<L, 4, 2, FP32_PHASE>(a, d, s_b, sm.lmn, sm.part, G, nchunks, 32, u0, v0);
    else if (V == 2)
      degrid_tasks<L, 2, 2, FP32_PHASE>(a, d, s_b, sm.lmn, sm.part, G, nchunks, 32, u0, v0);
    else
      degrid_tasks<L, 1, 2, FP32_PHASE>(a, d, s_b, sm.lmn, sm.part, G, nchunks, 32, u0, v0);
  } else if (V == 4) {
    degrid_tasks<L, 4, 1, FP32_PHASE>(a, d, s_b, sm.lmn, sm.part, G, nchunks, Q, u0, v0);
  } else if (V == 2) {
    degrid_tasks<L, 2, 1, FP32_PHASE>(a, d, s_b, sm.lmn, sm.part, G, nchunks, Q, u0, v0);
  } else {
    degrid_tasks<L, 1, 1, FP32_PHASE>(a, d, s_b, sm.lmn, sm.part, G, nchunks, Q, u0, v0);
  }
  if (G > 1) {
    __syncthreads();
    for (int k = tid; k < K; k += NT) {
      float4 s0 = sm.part[2 * k], s1 = sm.part[2 * k + 1];
      for (int g = 1; g < G; ++g) {
        const float4 p0 = sm.part[2 * (g * K + k)], p1 = sm.part[2 * (g * K + k) + 1];
        s0.x += p0.x; s0.y += p0.y; s0.z += p0.z; s0.w += p0.w;
        s1.x += p1.x; s1.y += p1.y; s1.z += p1.z; s1.w += p1.w;
      }
      const uint32_t pk = a.samples[d.vis_offset + k];
      const int t = d.t0 + int(pk >> 16), c = d.c0 + int(pk & 0xffffu);
      float4 *o = reinterpret_cast<float4 *>(a.vis_out + ((int64_t(d.bl) * a.nr_timesteps + t) * a.nr_channels + c) * 4);
      o[0] = s0;
      o[1] = s1;
    }
  }
}

template <int L, class SM>
__device__ __forceinline__ void degrid_load_tables(const KernelArgs &a, SM &sm) {
  constexpr int NT = Cfg<L>::NT, NPIX = L * L;
  if (threadIdx.x < L) sm.tw[threadIdx.x] = a.twiddle[threadIdx.x];
  if (threadIdx.x < L && a.sep) sm.sep[threadIdx.x] = a.sep[threadIdx.x];
  if (SM::LMN_LDS)
    for (int pix = threadIdx.x; pix < NPIX; pix += NT) sm.lmn[pix] = a.lmn[pix];
}

// Register budgets at L = 32 (waves per SIMD): the standard degridder 4 (its
// persistent form spills 8 VGPRs, and ran 16 % faster on small subgrids than
// at 3 waves without spills); the wide degridder 3 (spills 22 VGPRs; faster
// than 2 waves without spills).  Other sizes: as the compiler chooses.
template <int L, bool WIDE>
constexpr int degrid_min_waves() {
  return L == 32 ? (WIDE ? 3 : 4) : 1;
}

// Plain form: one workgroup per item order[blockIdx.x] (a.count items).  Subgrids
// with more than kDegridSmallK visibilities run degridder_kernel, the others
// degridder_small_kernel; the host passes each its part of the cost-sorted list.
template <int L, bool FP32_PHASE, bool WIDE>
__global__ void __launch_bounds__(Cfg<L>::NT) __attribute__((amdgpu_waves_per_eu(degrid_min_waves<L, WIDE>())))
degridder_kernel(KernelArgs a, const int32_t *order) {
  __shared__ DegridderSmem<L> sm;
  degrid_load_tables<L>(a, sm);
  degrid_one<L, FP32_PHASE, WIDE, kPathLarge>(a, order[blockIdx.x], sm);
}

template <int L, bool FP32_PHASE>
__global__ void __launch_bounds__(Cfg<L>::NT) __attribute__((amdgpu_waves_per_eu(degrid_min_waves<L, false>())))
degridder_small_kernel(KernelArgs a, const int32_t *order) {
  __shared__ DegridderSmem<L> sm;
  degrid_load_tables<L>(a, sm);
  degrid_one<L, FP32_PHASE, false, kPathSmall>(a, order[blockIdx.x], sm);
}

// Held to 3 waves per SIMD (154 VGPRs, no spills; 3 x 48 KiB of LDS per compute unit): measured 20 % faster
// than 2 waves (SKA-low-like share, 49.2 -> 39.1 ms).
template <int L>
__global__ void __launch_bounds__(Cfg<L>::NT) __attribute__((amdgpu_waves_per_eu(3)))
degridder_sep_kernel(KernelArgs a, const int32_t *order) {
  __shared__ DegridderSmem<L, true> sm;
  degrid_load_tables<L>(a, sm);
  degrid_one<L, false, false, kPathSep>(a, order ? int64_t(order[blockIdx.x]) : int64_t(blockIdx.x), sm);
}

template <int L>
__global__ void __launch_bounds__(Cfg<L>::NT) __attribute__((amdgpu_waves_per_eu(3)))
degridder_sep_persistent_kernel(KernelArgs a, const int32_t *order, int32_t *queue_head) {
  __shared__ DegridderSmem<L, true> sm;
  degrid_load_tables<L>(a, sm);
  for (;;) {
    if (threadIdx.x == 0) sm.next = atomicAdd(queue_head, 1);
    __syncthreads();
    const int item = sm.next;
    if (item >= a.count) break;
    degrid_one<L, false, false, kPathSep>(a, order[item], sm);
    __syncthreads();
  }
}

// Persistent form: items order[0 .. count-1] (global subgrid indices, costliest
// first) through the counter *queue_head (zero before the launch).
template <int L, bool FP32_PHASE, bool WIDE, bool SMALL>
__global__ void __launch_bounds__(Cfg<L>::NT) __attribute__((amdgpu_waves_per_eu(degrid_min_waves<L, WIDE>())))
degridder_persistent_kernel(KernelArgs a, const int32_t *order, int32_t *queue_head) {
  constexpr int PATH = SMALL ? kPathSmall : kPathLarge;
  __shared__ DegridderSmem<L> sm;
  degrid_load_tables<L>(a, sm);
  for (;;) {
    if (threadIdx.x == 0) sm.next = atomicAdd(queue_head, 1);
    __syncthreads();
    const int item = sm.next;
    if (item >= a.count) break;
    degrid_one<L, FP32_PHASE, WIDE, PATH>(a, order[item], sm);
    __syncthreads();
  }
}

int degrid_small_threshold() { return kDegridSmallK; }

// ---------------------------------------------------------------------------
// Adder: one workgroup per (work item, polarisation).  A work item is a grid
// tile with a contiguous run of its contribution list (subgrids overlapping
// it, in plan order).  A tile with a short list is one item that reads the
// tile once, adds every subgrid in order and writes it once.  A long list is
// cut into chunks whose items sum into partial tiles; combine_kernel then adds
// the partials to the grid in chunk order.  Deterministic, no atomics.

template <int L>
__global__ void __launch_bounds__(256) adder_kernel(AdderArgs a) {
  constexpr int T = kAdderTile, ROWS = 256 / T, PER = T / ROWS, NPIX = L * L, U = 4;
  const AdderItem it = a.items[blockIdx.x];
  const int pol = blockIdx.y;
  const int ntile = a.ntx * a.ntx;  // tile ids run over W-layers: layer * ntile + ty * ntx + tx
  const int layer = it.tile / ntile, tile = it.tile % ntile;
  const int tx = tile % a.ntx, ty = tile / a.ntx;
  const int N = a.grid_size;
  const int px = threadIdx.x % T, py = threadIdx.x / T;
  const int x = tx * T + px;
  float2 *gp = a.grid + (int64_t(layer) * 4 + pol) * N * N;
  float2 acc[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int y = ty * T + py + k * ROWS;
    acc[k] = (it.slot < 0 && x < N && y < N) ? gp[int64_t(y) * N + x] : make_float2(0.0f, 0.0f);
  }
  for (int c = it.begin; c < it.end; c += U) {
    float2 v[U][PER];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int k = 0; k < PER; ++k) v[u][k] = make_float2(0.0f, 0.0f);
      if (c + u < it.end) {
        const int s = a.contrib[c + u];
        const DevSubgrid d = a.subgrids[a.first + s];
        const int ia = x - d.x0;
        if (ia >= 0 && ia < L) {
          const float2 *sp = a.subgrids_in + (int64_t(s) * 4 + pol) * NPIX;
          const int ox = d.x0 % T, oy = d.y0 % T;
#pragma unroll
          for (int k = 0; k < PER; ++k) {
            const int jb = ty * T + py + k * ROWS - d.y0;
            if (jb >= 0 && jb < L) {  // read once: streamed
              const double bits = __builtin_nontemporal_load(
                  reinterpret_cast<const double *>(sp + (a.pieces ? piece_index<L>(jb, ia, ox, oy) : jb * L + ia)));
              __builtin_memcpy(&v[u][k], &bits, 8);
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        acc[k].x += v[u][k].x;
        acc[k].y += v[u][k].y;
      }
  }
  if (it.slot < 0) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int y = ty * T + py + k * ROWS;
      if (x < N && y < N) gp[int64_t(y) * N + x] = acc[k];
    }
  } else {
    float2 *pp = a.partials + (int64_t(it.slot) * 4 + pol) * T * T;
#pragma unroll
    for (int k = 0; k < PER; ++k) pp[(py + k * ROWS) * T + px] = acc[k];
  }
}

// Add the partial tiles of split lists to the grid, in chunk order.
__global__ void __launch_bounds__(256) combine_kernel(AdderArgs a) {
  constexpr int T = kAdderTile, ROWS = 256 / T, PER = T / ROWS;
  const CombineItem it = a.combine[blockIdx.x];
  const int pol = blockIdx.y;
  const int ntile = a.ntx * a.ntx;
  const int layer = it.tile / ntile, tile = it.tile % ntile;
  const int tx = tile % a.ntx, ty = tile / a.ntx;
  const int N = a.grid_size;
  const int px = threadIdx.x % T, py = threadIdx.x / T;
  const int x = tx * T + px;
  float2 *gp = a.grid + (int64_t(layer) * 4 + pol) * N * N;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int y = ty * T + py + k * ROWS;
    if (x >= N || y >= N) continue;
    float2 acc = gp[int64_t(y) * N + x];
    for (int sl = it.slot_begin; sl < it.slot_end; ++sl) {
      const float2 v = a.partials[(int64_t(sl) * 4 + pol) * T * T + (py + k * ROWS) * T + px];
      acc.x += v.x;
      acc.y += v.y;
    }
    gp[int64_t(y) * N + x] = acc;
  }
}

__global__ void zero_counter_kernel(int32_t *p) {
  if (threadIdx.x < 4) p[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// Splitter and the standalone transform.

template <int L>
__global__ void __launch_bounds__(Cfg<L>::NT) splitter_kernel(const DevSubgrid *subgrids, int64_t first,
                                                             const float2 *grid, int N, float2 *out) {
  constexpr int NT = Cfg<L>::NT, NPIX = L * L, PPT = NPIX / NT;
  const DevSubgrid d = subgrids[first + blockIdx.x];
  float2 *o = out + int64_t(blockIdx.x) * 4 * NPIX;
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int pix = threadIdx.x + r * NT;
    const int row = pix / L, col = pix % L;
#pragma unroll
    for (int pol = 0; pol < 4; ++pol)
      o[pol * NPIX + pix] = grid[((int64_t(d.layer) * 4 + pol) * N + d.y0 + row) * N + d.x0 + col];
  }
}

template <int L, bool INV>
__global__ void __launch_bounds__(Cfg<L>::NT) subgrid_fft_kernel(float2 *data, const float2 *twiddle) {
  constexpr int NT = Cfg<L>::NT, NPIX = L * L, PPT = NPIX / NT;
  __shared__ float2 s_sg[SgLayout<L>::SIZE];
  __shared__ float2 s_tw[L];
  const int tid = threadIdx.x;
  if (tid < L) s_tw[tid] = twiddle[tid];
  float2 *p = data + int64_t(blockIdx.x) * 4 * NPIX;
#pragma unroll
  for (int r = 0; r < PPT; ++r)
#pragma unroll
    for (int pol = 0; pol < 4; ++pol) s_sg[SgLayout<L>::idx(pol, tid + r * NT)] = p[pol * NPIX + tid + r * NT];
  __syncthreads();
  lds_centred_dft<L, NT, INV>(s_sg, s_tw);
#pragma unroll
  for (int r = 0; r < PPT; ++r)
#pragma unroll
    for (int pol = 0; pol < 4; ++pol) p[pol * NPIX + tid + r * NT] = s_sg[SgLayout<L>::idx(pol, tid + r * NT)];
}

__global__ void zero_samples_kernel(const int64_t *ids, int64_t n, float2 *vis) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    float4 *o = reinterpret_cast<float4 *>(vis + ids[i] * 4);
    o[0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    o[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
}

// ---------------------------------------------------------------------------
// Scratch of idg_grid_noalloc: a fixed device array, one per GPU that loads the
// library, held until the process ends.  Host code never passes `scratch`
// itself to a kernel (on the host the name is a stand-in, not a device
// address): noalloc_scratch() looks up the array's device address once per
// device with hipGetSymbolAddress and returns that.

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void **out) {
  constexpr int kMaxDevices = 64;
  static std::atomic<void *> addr[kMaxDevices];  // zero-initialised: not looked up yet
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  void *p = addr[dev].load(std::memory_order_acquire);
  if (!p) {
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev].store(p, std::memory_order_release);
  }
  *out = p;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// launchers

#define IDG_DISPATCH_L(L, EXPR)   \
  switch (L) {                    \
    case 8: { constexpr int LL = 8; EXPR; break; }   \
    case 16: { constexpr int LL = 16; EXPR; break; } \
    case 24: { constexpr int LL = 24; EXPR; break; } \
    case 32: { constexpr int LL = 32; EXPR; break; } \
    case 48: { constexpr int LL = 48; EXPR; break; } \
    case 64: { constexpr int LL = 64; EXPR; break; } \
    default: return hipErrorInvalidValue;            \
  }

hipError_t launch_gridder(int L, const KernelArgs &a, const int32_t *order, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  IDG_DISPATCH_L(L, {
    if (a.phase_fp32)
      hipLaunchKernelGGL((gridder_kernel<LL, true>), dim3(a.count), dim3(Cfg<LL>::NT), 0, s, a, order);
    else
      hipLaunchKernelGGL((gridder_kernel<LL, false>), dim3(a.count), dim3(Cfg<LL>::NT), 0, s, a, order);
  });
  return hipGetLastError();
}

int separable_max_order() { return kSeparableMaxOrder; }
bool separable_supported(int L) { return L == 32; }

hipError_t launch_gridder_mfma(int L, const KernelArgs &a, const int32_t *order, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  if (L != 32 || a.phase_fp32) return hipErrorInvalidValue;
  hipLaunchKernelGGL((gridder_mfma_kernel<32>), dim3(a.count), dim3(Cfg<32>::NT), 0, s, a, order);
  return hipGetLastError();
}

hipError_t launch_gridder_mfma_persistent(int L, const KernelArgs &a, const int32_t *order, int32_t *queue_head,
                                          int nblocks, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  if (L != 32 || a.phase_fp32) return hipErrorInvalidValue;
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, s, queue_head);
  hipLaunchKernelGGL((gridder_mfma_persistent_kernel<32>), dim3(nblocks), dim3(Cfg<32>::NT), 0, s, a, order,
                     queue_head);
  return hipGetLastError();
}

int mfma_gridder_blocks_per_cu(int L) {
  int n = 0;
  if (L != 32) return 1;
  const hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gridder_mfma_persistent_kernel<32>, Cfg<32>::NT, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_gridder_persistent(int L, const KernelArgs &a, const int32_t *order, int32_t *queue_head,
                                     int nblocks, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, s, queue_head);
  IDG_DISPATCH_L(L, {
    if (a.phase_fp32)
      hipLaunchKernelGGL((gridder_persistent_kernel<LL, true>), dim3(nblocks), dim3(Cfg<LL>::NT), 0, s, a, order,
                         queue_head);
    else
      hipLaunchKernelGGL((gridder_persistent_kernel<LL, false>), dim3(nblocks), dim3(Cfg<LL>::NT), 0, s, a, order,
                         queue_head);
  });
  return hipGetLastError();
}

// The all-float32 phase variant has no wide form.  order: the degridder's work list, order[0 .. n_sep) for the
// separable form, then n_large subgrids with more than kDegridSmallK visibilities, then the rest.
hipError_t launch_degridder(int L, const KernelArgs &a, bool wide, const int32_t *order, int64_t n_sep,
                            int64_t n_large, hipStream_t s) {
  const int64_t n_small = a.count - n_sep - n_large;
  if (n_sep > 0) {
    if (L != 32 || a.phase_fp32) return hipErrorInvalidValue;
    // every subgrid in the separable form: plan order, one dependent load less per workgroup than the list
    hipLaunchKernelGGL((degridder_sep_kernel<32>), dim3(unsigned(n_sep)), dim3(Cfg<32>::NT), 0, s, a,
                       n_sep == a.count ? nullptr : order);
  }
  const int32_t *ol = order + n_sep, *os = order + n_sep + n_large;
  IDG_DISPATCH_L(L, {
    if (n_large > 0) {
      if (a.phase_fp32)
        hipLaunchKernelGGL((degridder_kernel<LL, true, false>), dim3(unsigned(n_large)), dim3(Cfg<LL>::NT), 0, s, a,
                           ol);
      else if (wide)
        hipLaunchKernelGGL((degridder_kernel<LL, false, true>), dim3(unsigned(n_large)), dim3(Cfg<LL>::NT), 0, s, a,
                           ol);
      else
        hipLaunchKernelGGL((degridder_kernel<LL, false, false>), dim3(unsigned(n_large)), dim3(Cfg<LL>::NT), 0, s, a,
                           ol);
    }
    if (n_small > 0) {
      if (a.phase_fp32)
        hipLaunchKernelGGL((degridder_small_kernel<LL, true>), dim3(unsigned(n_small)), dim3(Cfg<LL>::NT), 0, s, a,
                           os);
      else
        hipLaunchKernelGGL((degridder_small_kernel<LL, false>), dim3(unsigned(n_small)), dim3(Cfg<LL>::NT), 0, s, a,
                           os);
    }
  });
  return hipGetLastError();
}

// queue_head: three counters (separable form, large and small subgrids), zeroed here.
hipError_t launch_degridder_persistent(int L, const KernelArgs &a, bool wide, const int32_t *order, int64_t n_sep,
                                       int64_t n_large, int32_t *queue_head, int nblocks_sep, int nblocks_large,
                                       int nblocks_small, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, s, queue_head);
  KernelArgs ap = a, al = a, as = a;
  ap.count = int32_t(n_sep);
  al.count = int32_t(n_large);
  as.count = int32_t(a.count - n_sep - n_large);
  if (ap.count > 0) {
    if (L != 32 || a.phase_fp32) return hipErrorInvalidValue;
    hipLaunchKernelGGL((degridder_sep_persistent_kernel<32>), dim3(nblocks_sep), dim3(Cfg<32>::NT), 0, s, ap, order,
                       queue_head + 2);
  }
  const int32_t *ol = order + n_sep, *os = order + n_sep + n_large;
  IDG_DISPATCH_L(L, {
    if (al.count > 0) {
      if (a.phase_fp32)
        hipLaunchKernelGGL((degridder_persistent_kernel<LL, true, false, false>), dim3(nblocks_large),
                           dim3(Cfg<LL>::NT), 0, s, al, ol, queue_head);
      else if (wide)
        hipLaunchKernelGGL((degridder_persistent_kernel<LL, false, true, false>), dim3(nblocks_large),
                           dim3(Cfg<LL>::NT), 0, s, al, ol, queue_head);
      else
        hipLaunchKernelGGL((degridder_persistent_kernel<LL, false, false, false>), dim3(nblocks_large),
                           dim3(Cfg<LL>::NT), 0, s, al, ol, queue_head);
    }
    if (as.count > 0) {
      if (a.phase_fp32)
        hipLaunchKernelGGL((degridder_persistent_kernel<LL, true, false, true>), dim3(nblocks_small),
                           dim3(Cfg<LL>::NT), 0, s, as, os, queue_head + 1);
      else
        hipLaunchKernelGGL((degridder_persistent_kernel<LL, false, false, true>), dim3(nblocks_small),
                           dim3(Cfg<LL>::NT), 0, s, as, os, queue_head + 1);
    }
  });
  return hipGetLastError();
}

int mfma_degridder_blocks_per_cu(int L) {
  int n = 0;
  if (L != 32) return 1;
  const hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, degridder_sep_persistent_kernel<32>, Cfg<32>::NT, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

int persistent_blocks_per_cu(int L, bool degrid, bool wide, bool small) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (L) {
#define IDG_OCC(LL)                                                                                            \
  case LL:                                                                                                     \
    e = !degrid ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gridder_persistent_kernel<LL, false>,     \
                                                               Cfg<LL>::NT, 0)                               \
        : small ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                                               \
                      &n, degridder_persistent_kernel<LL, false, false, true>, Cfg<LL>::NT, 0)               \
        : wide  ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                                               \
                      &n, degridder_persistent_kernel<LL, false, true, false>, Cfg<LL>::NT, 0)               \
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(                                               \
                      &n, degridder_persistent_kernel<LL, false, false, false>, Cfg<LL>::NT, 0);             \
    break;
    IDG_OCC(8)
    IDG_OCC(16)
    IDG_OCC(24)
    IDG_OCC(32)
    IDG_OCC(48)
    IDG_OCC(64)
#undef IDG_OCC
    default:
      break;
  }
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_adder(int L, const AdderArgs &a, hipStream_t s) {
  if (a.nitems > 0) {
    IDG_DISPATCH_L(L, { hipLaunchKernelGGL((adder_kernel<LL>), dim3(a.nitems, 4), dim3(256), 0, s, a); });
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (a.ncombine > 0) hipLaunchKernelGGL(combine_kernel, dim3(a.ncombine, 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_splitter(int L, const DevSubgrid *subgrids, int64_t first, int64_t count, const float2 *grid,
                           int grid_size, float2 *out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  IDG_DISPATCH_L(L, {
    hipLaunchKernelGGL((splitter_kernel<LL>), dim3(unsigned(count)), dim3(Cfg<LL>::NT), 0, s, subgrids, first,
                       grid, grid_size, out);
  });
  return hipGetLastError();
}

hipError_t launch_subgrid_fft(int L, float2 *data, int64_t count, int direction, const float2 *twiddle,
                              hipStream_t s) {
  if (count <= 0) return hipSuccess;
  IDG_DISPATCH_L(L, {
    if (direction > 0)
      hipLaunchKernelGGL((subgrid_fft_kernel<LL, true>), dim3(unsigned(count)), dim3(Cfg<LL>::NT), 0, s, data, twiddle);
    else
      hipLaunchKernelGGL((subgrid_fft_kernel<LL, false>), dim3(unsigned(count)), dim3(Cfg<LL>::NT), 0, s, data,
                         twiddle);
  });
  return hipGetLastError();
}

hipError_t launch_zero_samples(const int64_t *ids, int64_t n, float2 *vis, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(zero_samples_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, ids, n, vis);
  return hipGetLastError();
}

}  // namespace idg
