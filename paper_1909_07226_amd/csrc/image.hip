// gfx950 kernels of the steps around the hot path: the master grid <-> image
// transform (the last line of Algorithm 1, the first lines of Algorithm 2)
// with the division by a separable taper correction.
//
//   image[y][x] = sum_{v,u} grid[v][u] exp(+2 pi i ((u - N/2)(x - N/2) + (v - N/2)(y - N/2)) / N)
//                 / (corr_m[y] corr_l[x])
//
// and its adjoint.  For N a power of two the centred 1-D transform is
// (-1)^k FFT[(-1)^n x].  Up to N = 1024 the 2-D transform is two passes over
// HBM: one over rows (contiguous), one over blocks of C adjacent columns, each
// workgroup holding whole transforms in LDS.  The column pass reads and writes
// C x 8 bytes per row; its blocks are mapped so that neighbours sharing cache
// lines run on one XCD (one L2).  From N = 2048 on, fewer than 16 whole
// columns fit in LDS, and the column transform takes the four-step form
// (N = N1 N2: length-N1 transforms over runs of consecutive rows, twiddles,
// length-N2 transforms over rows N1 apart), so the 2-D transform is three
// passes: the rows (gathered into the four-step order), step A and step B.
// The division is fused into the last pass (first, in the adjoint).
//
// Inside a workgroup: radix-2 decimation in frequency, three stages at a time
// in registers (a closed set of 8 elements per work item), one LDS round trip
// per three stages; the first three stages read HBM directly; the output is
// un-bit-reversed on its way from LDS to HBM.
#include "internal.h"

#include <cmath>

namespace idg {

constexpr int kXcds = 8;

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }

// tw[m] = exp(-2 pi i m / N), m < N/2, from float64.
__global__ void image_twiddle_kernel(float2 *tw, int N) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N / 2) return;
  double s, c;
  sincospi(2.0 * double(m) / double(N), &s, &c);
  tw[m] = make_float2(float(c), float(-s));
}

__device__ __forceinline__ float2 fmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// a * exp(SIGN 2 pi i k / 8), k < 4 (constant after unrolling)
template <int SIGN>
__device__ __forceinline__ float2 mul_root8(float2 a, int k) {
  constexpr float r = 0.70710678118654752440f;
  constexpr float s = SIGN < 0 ? -1.0f : 1.0f;
  switch (k) {
    case 0: return a;
    case 2: return SIGN < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);  // * (-+ i)
    case 1: return fmul(a, make_float2(r, s * r));
    default: return fmul(a, make_float2(-r, s * r));
  }
}

// R radix-2 decimation-in-frequency stages (half-spans h_min 2^(R-1) down to
// h_min) on the 2^R elements v[m] = x[i_b + m h_min] of one closed set, lo =
// i_b mod h_min.  A stage of half-span h maps (x[i], x[i + h]) with i mod 2h < h
// to (x[i] + x[i + h], (x[i] - x[i + h]) exp(SIGN 2 pi i (i mod h) / (2h))).
template <int N, int R, int SIGN>
__device__ __forceinline__ void dif_set(float2 (&v)[1 << R], int lo, int h_min, const float2 *__restrict__ tw) {
#pragma unroll
  for (int q = R - 1; q >= 0; --q) {
    const int hq = h_min << q;
    float2 base = tw[lo * (N / (2 * hq))];  // exp(-2 pi i lo / (2 hq))
    if (SIGN > 0) base.y = -base.y;
#pragma unroll
    for (int m = 0; m < (1 << R); ++m) {
      if (m & (1 << q)) continue;
      const float2 a = v[m], b = v[m + (1 << q)];
      v[m] = make_float2(a.x + b.x, a.y + b.y);
      // (i mod hq) = lo + r h_min with r = m mod 2^q: the twiddle is base exp(SIGN 2 pi i r / 2^(q+1))
      const float2 w = mul_root8<SIGN>(base, (m & ((1 << q) - 1)) << (2 - q));
      v[m + (1 << q)] = fmul(make_float2(a.x - b.x, a.y - b.y), w);
    }
  }
}

// A workgroup holds C transforms of length N: rows (COLS false: element i of
// transform c at row b0 + c, column i) or columns (COLS true: row i, column
// b0 + c).  LDS indices are padded so that the strided patterns of the
// butterflies and of the bit-reversed read-out spread over the banks.
// threads of a workgroup holding `elems` elements: one per closed set of 8, at most 512
constexpr int fft_threads(int elems) { return elems / 8 < 512 ? elems / 8 : 512; }

template <int N, int C, bool COLS>
struct FftShape {
  static constexpr int n = ilog2c(N);
  static constexpr int NT = fft_threads(N * C);
  static constexpr int RSH = n > 8 ? n - 5 : 3;
  static constexpr int ROW = N + (N >> 3) + (N >> RSH);
  static constexpr int LDS = COLS ? C * (N + N / 8) : C * ROW;
  static __device__ __forceinline__ int lds(int i, int c) {
    if constexpr (COLS)
      return C * (i + (i >> 3)) + c;
    else
      return c * ROW + i + (i >> 3) + (i >> RSH);
  }
};

// Three (or fewer, at the end) stages from LDS to LDS; H is the largest half-span.
template <int N, int C, bool COLS, int SIGN, int H, int R>
__device__ __forceinline__ void lds_group(float2 *s, const float2 *__restrict__ tw, int tid) {
  using S = FftShape<N, C, COLS>;
  constexpr int E = 1 << R, HM = H >> (R - 1), NSET = N / E, PER = NSET * C / S::NT;
  constexpr int LH = ilog2c(H), LHM = ilog2c(HM);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int w = tid + k * S::NT;
    const int c = COLS ? w % C : w / NSET, set = COLS ? w / C : w % NSET;
    const int lo = set & (HM - 1), ib = lo + ((set >> LHM) << (LH + 1));
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = s[S::lds(ib + m * HM, c)];
    dif_set<N, R, SIGN>(v, lo, HM, tw);
#pragma unroll
    for (int m = 0; m < E; ++m) s[S::lds(ib + m * HM, c)] = v[m];
  }
  __syncthreads();
}

template <int N, int C, bool COLS, int SIGN, int H>
__device__ __forceinline__ void lds_groups(float2 *s, const float2 *__restrict__ tw, int tid) {
  if constexpr (H >= 4) {
    lds_group<N, C, COLS, SIGN, H, 3>(s, tw, tid);
    lds_groups<N, C, COLS, SIGN, H / 8>(s, tw, tid);
  } else if constexpr (H == 2) {
    lds_group<N, C, COLS, SIGN, 2, 2>(s, tw, tid);
  } else if constexpr (H == 1) {
    lds_group<N, C, COLS, SIGN, 1, 1>(s, tw, tid);
  }
}

// Centred length-N transforms of 4 N^2 / (N C) workgroups of C rows or columns
// of the [4][N][N] array; out may equal in (a workgroup reads all its elements
// before its first write; workgroups are disjoint).  SCALE 1 divides the input
// by sr[row] sc[col], SCALE 2 the output.
// Four-step split of a column transform: N = N1 N2 with N1 = 2^ceil(log2 N / 2).
template <int N>
constexpr int four_step_n1() {
  return 1 << ((ilog2c(N) + 1) / 2);
}

// GATHER (row pass only): output row p = n1 + N1 n2 takes input row N2 n1 + n2,
// the order the four-step column transform starts from.
template <int N, int C, bool COLS, int SIGN, int SCALE, bool GATHER = false>
__global__ void __launch_bounds__(fft_threads(N * C))
    fft_batch_kernel(const float2 *in, float2 *out, const float2 *__restrict__ tw, const float *__restrict__ sr,
                     const float *__restrict__ sc) {
  using S = FftShape<N, C, COLS>;
  constexpr int NT = S::NT, n = S::n;
  __shared__ float2 s[S::LDS];
  // workgroup i runs on XCD i mod 8: give each XCD a contiguous range of blocks
  const int nb = gridDim.x, bid = blockIdx.x;
  const int lb = (nb % kXcds == 0) ? (bid % kXcds) * (nb / kXcds) + bid / kXcds : bid;
  constexpr int per_plane = N / C;
  const int b0 = (lb % per_plane) * C;
  const int64_t pbase = int64_t(lb / per_plane) * N * N;
  const int tid = threadIdx.x;
  auto gofs = [&](int i, int c) -> int64_t {
    return COLS ? pbase + int64_t(i) * N + b0 + c : pbase + int64_t(b0 + c) * N + i;
  };
  auto gofs_in = [&](int i, int c) -> int64_t {
    if constexpr (GATHER) {
      constexpr int N1 = four_step_n1<N>(), N2 = N / N1;
      const int p = b0 + c;
      return pbase + int64_t(N2 * (p % N1) + p / N1) * N + i;
    } else {
      return gofs(i, c);
    }
  };
  auto inv_corr = [&](int i, int c) -> float {
    return COLS ? 1.0f / (sr[i] * sc[b0 + c]) : 1.0f / (sr[b0 + c] * sc[i]);
  };

  // stages of half-span N/2, N/4, N/8 straight from HBM: loads first, for bytes in flight
  {
    constexpr int HM = N / 8, PER = HM * C / NT;
    float2 v[PER][8];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int w = tid + k * NT;
      const int c = COLS ? w % C : w / HM, lo = COLS ? w / C : w % HM;
#pragma unroll
      for (int m = 0; m < 8; ++m) v[k][m] = in[gofs_in(lo + m * HM, c)];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int w = tid + k * NT;
      const int c = COLS ? w % C : w / HM, lo = COLS ? w / C : w % HM;
      const float sg = (lo & 1) ? -1.0f : 1.0f;  // (-1)^i; i = lo + m N/8 has the parity of lo
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        float f = sg;
        if constexpr (SCALE == 1) f *= inv_corr(lo + m * HM, c);
        v[k][m] = make_float2(v[k][m].x * f, v[k][m].y * f);
      }
      dif_set<N, 3, SIGN>(v[k], lo, HM, tw);
#pragma unroll
      for (int m = 0; m < 8; ++m) s[S::lds(lo + m * HM, c)] = v[k][m];
    }
  }
  __syncthreads();
  lds_groups<N, C, COLS, SIGN, N / 16>(s, tw, tid);

  // element i of LDS holds output k = bitreverse(i); times (-1)^k
  constexpr int PER = N * C / NT;
#pragma unroll 8
  for (int k = 0; k < PER; ++k) {
    const int w = tid + k * NT;
    int i, kk, c;
    if constexpr (COLS) {  // LDS order: each row of the output is still C x 8 contiguous bytes
      c = w % C;
      i = w / C;
      kk = int(__brev(unsigned(i)) >> (32 - n));
    } else {               // output order, contiguous along the row
      c = w / N;
      kk = w % N;
      i = int(__brev(unsigned(kk)) >> (32 - n));
    }
    float2 v = s[S::lds(i, c)];
    float f = (kk & 1) ? -1.0f : 1.0f;
    if constexpr (SCALE == 2) f *= inv_corr(kk, c);
    out[gofs(kk, c)] = make_float2(v.x * f, v.y * f);
  }
}

// ---------------------------------------------------------------------------
// Four-step column transform, N = N1 N2 (N >= 2048).  After the gathered row
// pass, position p = n1 + N1 n2 of a column holds its element N2 n1 + n2.
//   step A: for each n2, the length-N1 DFT over the N1 consecutive rows N1 n2 + n1,
//           times exp(SIGN 2 pi i n2 k1 / N), back into rows N1 n2 + k1;
//   step B: for each k1, the length-N2 DFT over rows k1 + N1 n2, into rows k1 + N1 k2,
//           which is output row k = k1 + N1 k2: natural order, in place.
// The centring signs are (-1)^n = (-1)^n2 (applied on step A's input) and
// (-1)^k = (-1)^k1 (on step B's output).  A workgroup takes 32 adjacent columns
// (256-byte row segments, which DRAM serves better than 128-byte ones) and
// 128 / T sub-transforms of length T: 4096 elements, 36 KiB of LDS.  With GATHER,
// step A reads the element from its natural row N2 n1 + n2 instead (image ->
// grid, whose first pass is the column transform).
// SCALE 1 / 2 divide the input / output by the correction; SCALE 3 applies a
// W-layer's exp(SIGN 2 pi i w0 n'(l, m)) (and the correction, when given) to
// step A's input or step B's output, which then adds into `out` when acc is set.
// The plain passes run 256 threads; SCALE 3 runs 512, because its per-pixel phase
// (float64 square root and range reduction) is ALU work that more waves hide
// better (4 workgroups per CU either way).
constexpr int kSubCols = 32, kSubElems = 128;

template <int SCALE>
constexpr int sub_threads() {
  return SCALE == 3 ? 512 : 256;
}

__device__ __forceinline__ int sub_lds(int i, int c) { return kSubCols * (i + (i >> 3)) + c; }

template <int NTAB, int SIGN, int H, int R, int NT>
__device__ __forceinline__ void sub_group(float2 *s, const float2 *__restrict__ tw, int tid) {
  constexpr int E = 1 << R, HM = H >> (R - 1), NSET = kSubElems / E, PER = NSET * kSubCols / NT;
  constexpr int LH = ilog2c(H), LHM = ilog2c(HM);
  static_assert(PER >= 1, "work split");
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int w = tid + k * NT;
    const int c = w % kSubCols, set = w / kSubCols;
    const int lo = set & (HM - 1), ib = lo + ((set >> LHM) << (LH + 1));
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = s[sub_lds(ib + m * HM, c)];
    dif_set<NTAB, R, SIGN>(v, lo, HM, tw);
#pragma unroll
    for (int m = 0; m < E; ++m) s[sub_lds(ib + m * HM, c)] = v[m];
  }
  __syncthreads();
}

template <int NTAB, int SIGN, int H, int NT>
__device__ __forceinline__ void sub_groups(float2 *s, const float2 *__restrict__ tw, int tid) {
  if constexpr (H >= 4) {
    sub_group<NTAB, SIGN, H, 3, NT>(s, tw, tid);
    sub_groups<NTAB, SIGN, H / 8, NT>(s, tw, tid);
  } else if constexpr (H == 2) {
    sub_group<NTAB, SIGN, 2, 2, NT>(s, tw, tid);
  } else if constexpr (H == 1) {
    sub_group<NTAB, SIGN, 1, 1, NT>(s, tw, tid);
  }
}

// exp(SIGN 2 pi i w0 n'(l_x, m_y)), n' = sqrt(1 - l^2 - m^2) - 1 (0 under the root outside the
// unit circle), l_x = (x - N/2) S / N.  The phase w0 n' (up to thousands of turns) is formed and
// reduced to a fraction of a turn in float64; the sine and cosine of that fraction are taken in
// float32, which is within 2e-7 rad and makes the W-layer passes 2-6 % faster than float64 sincospi.
template <int SIGN>
__device__ __forceinline__ float2 wlayer_phasor(int x, int y, int N, double S, double w0) {
  const double l = double(x - N / 2) * S / double(N), m = double(y - N / 2) * S / double(N);
  double ph = w0 * (sqrt(fmax(0.0, 1.0 - l * l - m * m)) - 1.0);
  ph -= floor(ph);
  float sn, cs;
  sincospif(2.0f * float(ph), &sn, &cs);
  return make_float2(cs, SIGN > 0 ? sn : -sn);
}

template <int N, bool STEP_B, bool GATHER, int SIGN, int SCALE>
__global__ void __launch_bounds__(sub_threads<SCALE>())
    fft_sub_kernel(const float2 *in, float2 *out, const float2 *__restrict__ tw, const float *__restrict__ sr,
                   const float *__restrict__ sc, double S, double w0, int acc) {
  constexpr int N1 = four_step_n1<N>(), N2 = N / N1;
  constexpr int T = STEP_B ? N2 : N1, GB = kSubElems / T, NBLK = STEP_B ? N1 : N2;
  constexpr int NGRP = NBLK / GB, NCG = N / kSubCols;
  constexpr int lt = ilog2c(T);
  static_assert(GB >= 1 && NBLK % GB == 0, "sub-transform grouping");
  __shared__ float2 s[kSubCols * (kSubElems + kSubElems / 8)];
  const int tid = threadIdx.x;
  const int bg = blockIdx.x % NGRP, rest = blockIdx.x / NGRP;
  const int x0 = (rest % NCG) * kSubCols;
  const int64_t pbase = int64_t(rest / NCG) * N * N;
  constexpr int NT = sub_threads<SCALE>(), PER = kSubElems * kSubCols / NT;
  static_assert(PER >= 1 && NT % kSubCols == 0, "work split");
  float2 v[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {  // loads first, for bytes in flight
    const int e = tid + j * NT, c = e % kSubCols, rr = e / kSubCols;
    const int blk = bg * GB + rr / T, i = rr % T;
    const int row = STEP_B ? blk + N1 * i : (GATHER ? N2 * i + blk : N1 * blk + i);
    v[j] = in[pbase + int64_t(row) * N + x0 + c];
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int e = tid + j * NT, c = e % kSubCols, rr = e / kSubCols;
    const int blk = bg * GB + rr / T, i = rr % T;
    float f = (!STEP_B && (blk & 1)) ? -1.0f : 1.0f;
    const int row = STEP_B ? blk + N1 * i : (GATHER ? N2 * i + blk : N1 * blk + i);
    if constexpr (SCALE == 1) f /= sr[row] * sc[x0 + c];
    if constexpr (SCALE == 3 && !STEP_B) {
      if (sr) f /= sr[row] * sc[x0 + c];
      v[j] = fmul(v[j], wlayer_phasor<SIGN>(x0 + c, row, N, S, w0));
    }
    s[sub_lds(rr, c)] = make_float2(v[j].x * f, v[j].y * f);
  }
  __syncthreads();
  sub_groups<N, SIGN, T / 2, NT>(s, tw, tid);
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int e = tid + j * NT, c = e % kSubCols, rr = e / kSubCols;
    const int blk = bg * GB + rr / T, k = int(__brev(unsigned(rr % T)) >> (32 - lt));
    float2 x = s[sub_lds(rr, c)];
    int row;
    if constexpr (STEP_B) {
      row = blk + N1 * k;
      float f = (blk & 1) ? -1.0f : 1.0f;
      if constexpr (SCALE == 2) f /= sr[row] * sc[x0 + c];
      if constexpr (SCALE == 3) {
        if (sr) f /= sr[row] * sc[x0 + c];
        x = fmul(x, wlayer_phasor<SIGN>(x0 + c, row, N, S, w0));
      }
      x = make_float2(x.x * f, x.y * f);
      if (SCALE == 3 && acc) {
        const float2 o = out[pbase + int64_t(row) * N + x0 + c];
        x = make_float2(o.x + x.x, o.y + x.y);
      }
    } else {
      row = N1 * blk + k;
      const int m = (blk * k) & (N - 1);  // exp(SIGN 2 pi i m / N) from the half table
      float2 w = tw[m & (N / 2 - 1)];
      if (m >= N / 2) w = make_float2(-w.x, -w.y);
      if (SIGN > 0) w.y = -w.y;
      x = fmul(x, w);
    }
    out[pbase + int64_t(row) * N + x0 + c] = x;
  }
}

template <int N, bool STEP_B, bool GATHER, int SIGN, int SCALE>
static hipError_t launch_fft_sub(const float2 *in, float2 *out, const float2 *tw, const float *sr, const float *sc,
                                 hipStream_t st, double S = 0.0, double w0 = 0.0, bool acc = false) {
  constexpr int N1 = four_step_n1<N>(), N2 = N / N1, T = STEP_B ? N2 : N1, NBLK = STEP_B ? N1 : N2;
  constexpr int64_t blocks = int64_t(4) * (N / kSubCols) * (NBLK / (kSubElems / T));
  hipLaunchKernelGGL((fft_sub_kernel<N, STEP_B, GATHER, SIGN, SCALE>), dim3(unsigned(blocks)),
                     dim3(sub_threads<SCALE>()), 0, st, in, out, tw, sr, sc, S, w0, int(acc));
  return hipGetLastError();
}

// W-layers: out[pol][y][x] (= or +=) in[pol][y][x] exp(SIGN 2 pi i w0 n'(l_x, m_y)) [/ (cm[y] cl[x])],
// n' = sqrt(1 - l^2 - m^2) - 1 (0 under the root outside the unit circle), l_x = (x - N/2) S / N.
// One thread per pixel: the phasor serves the 4 polarisations.
template <int SIGN, bool ACC>
__global__ void __launch_bounds__(256) wlayer_phase_kernel(const float2 *in, float2 *out, int N, double S, double w0,
                                                           const float *__restrict__ cl,
                                                           const float *__restrict__ cm) {
  const int64_t NN = int64_t(N) * N;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= NN) return;
  const int y = int(i / N), x = int(i % N);
  const double l = double(x - N / 2) * S / double(N), m = double(y - N / 2) * S / double(N);
  const double n1 = sqrt(fmax(0.0, 1.0 - l * l - m * m)) - 1.0;
  double ph = w0 * n1;
  ph -= floor(ph);  // as in wlayer_phasor: reduced in float64, sine and cosine in float32
  float sn, cs;
  sincospif(2.0f * float(ph), &sn, &cs);
  float2 e = make_float2(cs, SIGN > 0 ? sn : -sn);
  if (cl) {
    const float f = 1.0f / (cm[y] * cl[x]);
    e = make_float2(e.x * f, e.y * f);
  }
#pragma unroll
  for (int pol = 0; pol < 4; ++pol) {
    float2 v = fmul(in[pol * NN + i], e);
    if (ACC) {
      const float2 o = out[pol * NN + i];
      v = make_float2(o.x + v.x, o.y + v.y);
    }
    out[pol * NN + i] = v;
  }
}

hipError_t launch_wlayer_phase(const float2 *in, float2 *out, int N, double S, double w0, int sign, bool accumulate,
                               const float *corr_l, const float *corr_m, hipStream_t s) {
  const int64_t NN = int64_t(N) * N;
  const dim3 grid(unsigned((NN + 255) / 256)), block(256);
  if (sign > 0) {
    if (accumulate)
      hipLaunchKernelGGL((wlayer_phase_kernel<1, true>), grid, block, 0, s, in, out, N, S, w0, corr_l, corr_m);
    else
      hipLaunchKernelGGL((wlayer_phase_kernel<1, false>), grid, block, 0, s, in, out, N, S, w0, corr_l, corr_m);
  } else {
    if (accumulate)
      hipLaunchKernelGGL((wlayer_phase_kernel<-1, true>), grid, block, 0, s, in, out, N, S, w0, corr_l, corr_m);
    else
      hipLaunchKernelGGL((wlayer_phase_kernel<-1, false>), grid, block, 0, s, in, out, N, S, w0, corr_l, corr_m);
  }
  return hipGetLastError();
}

bool image_size_supported(int N) { return N >= 64 && N <= 16384 && (N & (N - 1)) == 0; }

// Elements per workgroup: rows, at least kRowElems (whole rows); columns, at
// most kColElems (16384 x 9/8 x 8 bytes = 144 KiB of LDS: one workgroup per CU,
// C = 16384 / N adjacent columns, up to 16 = one 128-byte line per row).
#ifndef IDG_IMAGE_ROW_ELEMS
#define IDG_IMAGE_ROW_ELEMS 2048
#endif
#ifndef IDG_IMAGE_COL_ELEMS
#define IDG_IMAGE_COL_ELEMS 16384
#endif
constexpr int kRowElems = IDG_IMAGE_ROW_ELEMS, kColElems = IDG_IMAGE_COL_ELEMS;

template <int N>
constexpr int row_batch() {
  return N >= kRowElems ? 1 : kRowElems / N;
}
template <int N>
constexpr int col_batch() {
  return kColElems / N < 1 ? 1 : (kColElems / N < 16 ? kColElems / N : 16);
}

template <int N, bool COLS, int SIGN, int SCALE, bool GATHER = false>
static hipError_t launch_fft_batch(const float2 *in, float2 *out, const float2 *tw, const float *sr, const float *sc,
                                   hipStream_t st) {
  constexpr int C = COLS ? col_batch<N>() : row_batch<N>();
  using S = FftShape<N, C, COLS>;
  static_assert(S::LDS * sizeof(float2) <= 160 * 1024, "LDS");
  static_assert((N / 8) * C % S::NT == 0 && (N / 2) * C % S::NT == 0, "work split");
  static_assert(!GATHER || (!COLS && C == 1), "gathered rows: one row per workgroup");
  hipLaunchKernelGGL((fft_batch_kernel<N, C, COLS, SIGN, SCALE, GATHER>), dim3(4 * N / C), dim3(S::NT), 0, st, in,
                     out, tw, sr, sc);
  return hipGetLastError();
}

// The column transform takes the four-step form where whole-column blocks of
// LDS would read fewer than 16 columns (128 bytes) per row.
template <int N>
constexpr bool use_four_step() {
  return col_batch<N>() < 16 && N >= 2048;
}

#define IDG_DISPATCH_N(N, ...)                                    \
  switch (N) {                                                    \
    case 64: { constexpr int NN = 64; __VA_ARGS__; break; }       \
    case 128: { constexpr int NN = 128; __VA_ARGS__; break; }     \
    case 256: { constexpr int NN = 256; __VA_ARGS__; break; }     \
    case 512: { constexpr int NN = 512; __VA_ARGS__; break; }     \
    case 1024: { constexpr int NN = 1024; __VA_ARGS__; break; }   \
    case 2048: { constexpr int NN = 2048; __VA_ARGS__; break; }   \
    case 4096: { constexpr int NN = 4096; __VA_ARGS__; break; }   \
    case 8192: { constexpr int NN = 8192; __VA_ARGS__; break; }   \
    case 16384: { constexpr int NN = 16384; __VA_ARGS__; break; } \
    default: return hipErrorInvalidValue;                         \
  }

hipError_t launch_image_twiddles(float2 *tw, int N, hipStream_t s) {
  if (!image_size_supported(N)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(image_twiddle_kernel, dim3((N / 2 + 255) / 256), dim3(256), 0, s, tw, N);
  return hipGetLastError();
}

bool image_needs_scratch(int N, const void *in, const void *out) {
  bool four = false;
  switch (N) {
    case 2048: four = use_four_step<2048>(); break;
    case 4096: four = use_four_step<4096>(); break;
    case 8192: four = use_four_step<8192>(); break;
    case 16384: four = use_four_step<16384>(); break;
    default: break;
  }
  return four && in == out;
}

hipError_t launch_grid_to_image(const float2 *grid, float2 *image, int N, const float *corr_l, const float *corr_m,
                                const float2 *tw, float2 *scratch, hipStream_t s) {
  hipError_t e = hipSuccess;
  IDG_DISPATCH_N(N, {
    if constexpr (use_four_step<NN>()) {
      // rows gathered into the four-step order (they cross workgroups: in place goes through
      // scratch), step A in place, step B into the image
      float2 *mid = (grid == image) ? scratch : image;
      if (!mid) return hipErrorInvalidValue;
      e = launch_fft_batch<NN, false, 1, 0, true>(grid, mid, tw, nullptr, nullptr, s);
      if (e == hipSuccess) e = launch_fft_sub<NN, false, false, 1, 0>(mid, mid, tw, nullptr, nullptr, s);
      if (e == hipSuccess)
        e = corr_l ? launch_fft_sub<NN, true, false, 1, 2>(mid, image, tw, corr_m, corr_l, s)
                   : launch_fft_sub<NN, true, false, 1, 0>(mid, image, tw, nullptr, nullptr, s);
    } else {
      e = launch_fft_batch<NN, false, 1, 0>(grid, image, tw, nullptr, nullptr, s);
      if (e == hipSuccess)
        e = corr_l ? launch_fft_batch<NN, true, 1, 2>(image, image, tw, corr_m, corr_l, s)
                   : launch_fft_batch<NN, true, 1, 0>(image, image, tw, nullptr, nullptr, s);
    }
  });
  return e;
}

hipError_t launch_image_to_grid(const float2 *image, float2 *grid, int N, const float *corr_l, const float *corr_m,
                                const float2 *tw, float2 *scratch, hipStream_t s) {
  hipError_t e = hipSuccess;
  IDG_DISPATCH_N(N, {
    if constexpr (use_four_step<NN>()) {
      // step A gathering from the image's natural rows (across workgroups: in place goes
      // through scratch), step B in place, then the rows into the grid
      float2 *mid = (grid == image) ? scratch : grid;
      if (!mid) return hipErrorInvalidValue;
      e = corr_l ? launch_fft_sub<NN, false, true, -1, 1>(image, mid, tw, corr_m, corr_l, s)
                 : launch_fft_sub<NN, false, true, -1, 0>(image, mid, tw, nullptr, nullptr, s);
      if (e == hipSuccess) e = launch_fft_sub<NN, true, false, -1, 0>(mid, mid, tw, nullptr, nullptr, s);
      if (e == hipSuccess) e = launch_fft_batch<NN, false, -1, 0>(mid, grid, tw, nullptr, nullptr, s);
    } else {
      e = corr_l ? launch_fft_batch<NN, true, -1, 1>(image, grid, tw, corr_m, corr_l, s)
                 : launch_fft_batch<NN, true, -1, 0>(image, grid, tw, nullptr, nullptr, s);
      if (e == hipSuccess) e = launch_fft_batch<NN, false, -1, 0>(grid, grid, tw, nullptr, nullptr, s);
    }
  });
  return e;
}

hipError_t launch_wlayer_to_image(const float2 *grid, float2 *image, float2 *scratch, int N, double S, double w0,
                                  bool accumulate, const float *corr_l, const float *corr_m, const float2 *tw,
                                  hipStream_t s) {
  hipError_t e = hipSuccess;
  IDG_DISPATCH_N(N, {
    if constexpr (use_four_step<NN>()) {
      // gathered rows and step A in scratch; step B applies the layer's phase and adds into the image
      e = launch_fft_batch<NN, false, 1, 0, true>(grid, scratch, tw, nullptr, nullptr, s);
      if (e == hipSuccess) e = launch_fft_sub<NN, false, false, 1, 0>(scratch, scratch, tw, nullptr, nullptr, s);
      if (e == hipSuccess)
        e = launch_fft_sub<NN, true, false, 1, 3>(scratch, image, tw, corr_m, corr_l, s, S, w0, accumulate);
    } else {
      e = launch_grid_to_image(grid, scratch, N, nullptr, nullptr, tw, nullptr, s);
      if (e == hipSuccess) e = launch_wlayer_phase(scratch, image, N, S, w0, +1, accumulate, corr_l, corr_m, s);
    }
  });
  return e;
}

hipError_t launch_image_to_wlayer(const float2 *image, float2 *grid, float2 *scratch, int N, double S, double w0,
                                  const float *corr_l, const float *corr_m, const float2 *tw, hipStream_t s) {
  hipError_t e = hipSuccess;
  IDG_DISPATCH_N(N, {
    if constexpr (use_four_step<NN>()) {
      // step A gathers from the image with the layer's phase; step B and the rows in the layer grid
      e = launch_fft_sub<NN, false, true, -1, 3>(image, grid, tw, corr_m, corr_l, s, S, w0, false);
      if (e == hipSuccess) e = launch_fft_sub<NN, true, false, -1, 0>(grid, grid, tw, nullptr, nullptr, s);
      if (e == hipSuccess) e = launch_fft_batch<NN, false, -1, 0>(grid, grid, tw, nullptr, nullptr, s);
    } else {
      e = launch_wlayer_phase(image, scratch, N, S, w0, -1, false, corr_l, corr_m, s);
      if (e == hipSuccess) e = launch_image_to_grid(scratch, grid, N, nullptr, nullptr, tw, nullptr, s);
    }
  });
  return e;
}

}  // namespace idg
