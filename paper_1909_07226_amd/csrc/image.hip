// gfx950 kernels of the steps around the hot path: the master grid <-> image
// transform (the last line of Algorithm 1, the first lines of Algorithm 2)
// with the division by a separable taper correction.
//
//   image[y][x] = sum_{v,u} grid[v][u] exp(+2 pi i ((u - N/2)(x - N/2) + (v - N/2)(y - N/2)) / N)
//                 / (corr_m[y] corr_l[x])
//
// and its adjoint.  For N a power of two the centred 1-D transform is
// (-1)^k FFT[(-1)^n x], done per row in LDS (radix-2, decimation in frequency,
// natural order in, bit-reversed order out); the 2-D transform is rows, a tiled
// transpose, rows again and a transpose back.  Every pass reads and writes the
// 4 x N x N complex64 array once: HBM-bound.
#include "internal.h"

#include <cmath>

namespace idg {

constexpr int kImgTile = 32;

// tw[m] = exp(-2 pi i m / N), m < N/2, from float64.
__global__ void image_twiddle_kernel(float2 *tw, int N) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N / 2) return;
  double s, c;
  sincospi(2.0 * double(m) / double(N), &s, &c);
  tw[m] = make_float2(float(c), float(-s));
}

template <int N>
constexpr int fft_threads() {
  return N / 2 < 512 ? N / 2 : 512;
}

template <int N>
__device__ __forceinline__ int bit_reverse_n(int i) {
  return int(__brev(unsigned(i)) >> (32 - __builtin_ctz(N)));
}

// One centred transform of length N per row, rows [0, nrows): out may equal in
// (each workgroup reads its whole row before it writes).  SIGN = +1: exp(+...).
template <int N, int SIGN>
__global__ void __launch_bounds__(fft_threads<N>()) fft_rows_kernel(const float2 *in, float2 *out,
                                                                   const float2 *tw) {
  constexpr int NT = fft_threads<N>();
  __shared__ float2 s[N];
  const int tid = threadIdx.x;
  const int64_t base = int64_t(blockIdx.x) * N;
  for (int i = tid; i < N; i += NT) {
    const float2 v = in[base + i];
    s[i] = (i & 1) ? make_float2(-v.x, -v.y) : v;
  }
  __syncthreads();
  // decimation in frequency: a stage of span 2h combines s[i0] and s[i0 + h]
  for (int h = N / 2; h >= 1; h >>= 1) {
    const int tstride = N / (2 * h);  // twiddle index step: exp(-+2 pi i j / (2h)) = tw[j * N / (2h)]
    for (int b = tid; b < N / 2; b += NT) {
      const int j = b & (h - 1);
      const int i0 = ((b - j) << 1) + j, i1 = i0 + h;
      const float2 a = s[i0], c = s[i1];
      float2 w = tw[j * tstride];
      if (SIGN > 0) w.y = -w.y;
      const float2 d = make_float2(a.x - c.x, a.y - c.y);
      s[i0] = make_float2(a.x + c.x, a.y + c.y);
      s[i1] = make_float2(d.x * w.x - d.y * w.y, d.x * w.y + d.y * w.x);
    }
    __syncthreads();
  }
  for (int k = tid; k < N; k += NT) {
    const float2 v = s[bit_reverse_n<N>(k)];
    out[base + k] = (k & 1) ? make_float2(-v.x, -v.y) : v;
  }
}

// out[p][r][c] = in[p][c][r] / (sr[r] sc[c]) (no division when sr is NULL), N x N
// planes, tiles of 32 x 32 through LDS.  Grid (N/32, N/32, planes).
__global__ void __launch_bounds__(256) transpose_scale_kernel(const float2 *in, float2 *out, int N,
                                                              const float *sr, const float *sc) {
  __shared__ float2 t[kImgTile][kImgTile + 1];
  const int64_t plane = int64_t(blockIdx.z) * N * N;
  const int bx = blockIdx.x * kImgTile, by = blockIdx.y * kImgTile;  // tile of `in`: rows by.., cols bx..
  const int tx = threadIdx.x % kImgTile, ty = threadIdx.x / kImgTile;
  for (int r = ty; r < kImgTile; r += 256 / kImgTile) t[r][tx] = in[plane + int64_t(by + r) * N + bx + tx];
  __syncthreads();
  for (int r = ty; r < kImgTile; r += 256 / kImgTile) {
    const int orow = bx + r, ocol = by + tx;  // out[orow][ocol] = in[ocol][orow]
    float2 v = t[tx][r];
    if (sr) {
      const float f = 1.0f / (sr[orow] * sc[ocol]);
      v = make_float2(v.x * f, v.y * f);
    }
    out[plane + int64_t(orow) * N + ocol] = v;
  }
}

bool image_size_supported(int N) { return N >= 64 && N <= 16384 && (N & (N - 1)) == 0; }

#define IDG_DISPATCH_N(N, EXPR)                            \
  switch (N) {                                             \
    case 64: { constexpr int NN = 64; EXPR; break; }       \
    case 128: { constexpr int NN = 128; EXPR; break; }     \
    case 256: { constexpr int NN = 256; EXPR; break; }     \
    case 512: { constexpr int NN = 512; EXPR; break; }     \
    case 1024: { constexpr int NN = 1024; EXPR; break; }   \
    case 2048: { constexpr int NN = 2048; EXPR; break; }   \
    case 4096: { constexpr int NN = 4096; EXPR; break; }   \
    case 8192: { constexpr int NN = 8192; EXPR; break; }   \
    case 16384: { constexpr int NN = 16384; EXPR; break; } \
    default: return hipErrorInvalidValue;                  \
  }

hipError_t launch_image_twiddles(float2 *tw, int N, hipStream_t s) {
  if (!image_size_supported(N)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(image_twiddle_kernel, dim3((N / 2 + 255) / 256), dim3(256), 0, s, tw, N);
  return hipGetLastError();
}

hipError_t launch_fft_rows(const float2 *in, float2 *out, int N, int64_t nrows, int sign, const float2 *tw,
                           hipStream_t s) {
  if (!image_size_supported(N) || nrows <= 0 || nrows > INT32_MAX) return hipErrorInvalidValue;
  IDG_DISPATCH_N(N, {
    if (sign > 0)
      hipLaunchKernelGGL((fft_rows_kernel<NN, 1>), dim3(unsigned(nrows)), dim3(fft_threads<NN>()), 0, s, in, out, tw);
    else
      hipLaunchKernelGGL((fft_rows_kernel<NN, -1>), dim3(unsigned(nrows)), dim3(fft_threads<NN>()), 0, s, in, out,
                         tw);
  });
  return hipGetLastError();
}

hipError_t launch_transpose_scale(const float2 *in, float2 *out, int N, int planes, const float *sr, const float *sc,
                                  hipStream_t s) {
  if (!image_size_supported(N) || planes <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(transpose_scale_kernel, dim3(N / kImgTile, N / kImgTile, planes), dim3(256), 0, s, in, out, N,
                     sr, sc);
  return hipGetLastError();
}

}  // namespace idg
