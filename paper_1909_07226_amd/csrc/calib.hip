// Device rate microbenchmarks: a measurement aid for expressing the gridder's
// and degridder's times as fractions of what this device sustains for the
// instruction kinds they issue (float32 multiply-adds, the sine / cosine
// instructions, fp16 matrix-core products).  Not part of the method.
#include "internal.h"

namespace idg {

namespace {

typedef _Float16 cal_half8 __attribute__((ext_vector_type(8)));
typedef float cal_floatx16 __attribute__((ext_vector_type(16)));

constexpr int kCalChains = 8;

// 8 independent multiply-add chains per lane.
__global__ void __launch_bounds__(256) cal_fma_kernel(float *out, int iters, float m, float c) {
  float x[kCalChains];
#pragma unroll
  for (int j = 0; j < kCalChains; ++j) x[j] = float(threadIdx.x + j);
  for (int i = 0; i < iters; ++i)
#pragma unroll
    for (int j = 0; j < kCalChains; ++j) x[j] = __builtin_fmaf(x[j], m, c);
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kCalChains; ++j) s += x[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 8 independent chains of sine / cosine instructions (argument in revolutions).
__global__ void __launch_bounds__(256) cal_sincos_kernel(float *out, int iters) {
  float x[kCalChains];
#pragma unroll
  for (int j = 0; j < kCalChains; ++j) x[j] = 1e-3f * float(threadIdx.x + j);
  for (int i = 0; i < iters; ++i)
#pragma unroll
    for (int j = 0; j < kCalChains; ++j)
      x[j] = (j & 1) ? __builtin_amdgcn_cosf(x[j]) : __builtin_amdgcn_sinf(x[j]);
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kCalChains; ++j) s += x[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 4 independent accumulators per wave of 32 x 32 x 16 fp16 products.
__global__ void __launch_bounds__(256) cal_mfma_kernel(float *out, int iters) {
  cal_half8 a, b;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    a[s] = _Float16(1e-3f * float((threadIdx.x + s) & 15));
    b[s] = _Float16(1e-3f * float((threadIdx.x * 3 + s) & 15));
  }
  cal_floatx16 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[j][e] = 0.0f;
  for (int i = 0; i < iters; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[j], 0, 0, 0);
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int e = 0; e < 16; ++e) s += acc[j][e];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

hipError_t measure_device_rates(double *fma_flops, double *sincos_instr, double *mfma_flops) {
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int blocks = 8 * cus, threads = 256;
  float *out = nullptr;
  e = hipMalloc(reinterpret_cast<void **>(&out), size_t(blocks) * threads * sizeof(float));
  if (e != hipSuccess) return e;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  // best of 3 timed launches after one warm-up; returns seconds
  auto time_it = [&](auto launch, double *sec) -> hipError_t {
    hipError_t r = hipSuccess;
    double best = 1e30;
    for (int rep = 0; rep < 4 && r == hipSuccess; ++rep) {
      r = hipEventRecord(t0, nullptr);
      if (r == hipSuccess) launch();
      if (r == hipSuccess) r = hipGetLastError();
      if (r == hipSuccess) r = hipEventRecord(t1, nullptr);
      if (r == hipSuccess) r = hipEventSynchronize(t1);
      float ms = 0.0f;
      if (r == hipSuccess) r = hipEventElapsedTime(&ms, t0, t1);
      if (r == hipSuccess && rep > 0 && ms < best) best = ms;
    }
    *sec = best * 1e-3;
    return r;
  };
  const int it_fma = 4096, it_sc = 1024, it_mfma = 512;
  double s_fma = 0, s_sc = 0, s_mfma = 0;
  if (e == hipSuccess)
    e = time_it([&] { hipLaunchKernelGGL(cal_fma_kernel, dim3(blocks), dim3(threads), 0, nullptr, out, it_fma,
                                         0.999999f, 1e-7f); }, &s_fma);
  if (e == hipSuccess)
    e = time_it([&] { hipLaunchKernelGGL(cal_sincos_kernel, dim3(blocks), dim3(threads), 0, nullptr, out, it_sc); },
                &s_sc);
  if (e == hipSuccess)
    e = time_it([&] { hipLaunchKernelGGL(cal_mfma_kernel, dim3(blocks), dim3(threads), 0, nullptr, out, it_mfma); },
                &s_mfma);
  const double lanes = double(blocks) * threads, waves = lanes / 64.0;
  if (e == hipSuccess) {
    *fma_flops = 2.0 * kCalChains * double(it_fma) * lanes / s_fma;
    *sincos_instr = double(kCalChains) * it_sc * waves / s_sc;
    *mfma_flops = 4.0 * double(it_mfma) * waves * (32.0 * 32.0 * 16.0 * 2.0) / s_mfma;
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  const hipError_t ef = hipFree(out);
  return e != hipSuccess ? e : ef;
}

}  // namespace idg
