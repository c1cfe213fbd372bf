// Self-test kernels for the gfx950 builtins used by the ray-sum kernels (drt_probe.h).
#include <hip/hip_runtime.h>

#include "../../include/drt.h"
#include "drt_probe.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(64) void k_probe_mfma(const float* A, const float* B, float* D) {
  int l = threadIdx.x;
  float a = A[(l % 16) * 4 + l / 16];
  float b = B[(l / 16) * 16 + l % 16];
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  for (int v = 0; v < 4; ++v) D[(4 * (l / 16) + v) * 16 + l % 16] = acc[v];
}

typedef _Float16 half8 __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(64) void k_probe_mfma16(const _Float16* A, const _Float16* B, float* D) {
  int l = threadIdx.x;
  half8 a, b;
  for (int j = 0; j < 8; ++j) {
    a[j] = A[(l % 16) * 32 + 8 * (l / 16) + j];
    b[j] = B[(8 * (l / 16) + j) * 16 + l % 16];
  }
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
  for (int v = 0; v < 4; ++v) D[(4 * (l / 16) + v) * 16 + l % 16] = acc[v];
}

typedef double doublex4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(64) void k_probe_mfma64(const double* A, const double* B, double* D) {
  int l = threadIdx.x;
  double a = A[(l % 16) * 4 + l / 16];
  double b = B[(l / 16) * 16 + l % 16];
  doublex4 acc = {0.0, 0.0, 0.0, 0.0};
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  for (int v = 0; v < 4; ++v) D[(l / 16 + 4 * v) * 16 + l % 16] = acc[v];
}

__global__ __launch_bounds__(256) void k_probe_sincos(const float* x, int n, float* s, float* c) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  s[i] = __builtin_amdgcn_sinf(x[i]);
  c[i] = __builtin_amdgcn_cosf(x[i]);
}

extern "C" int drt_probe_mfma_f32_16x16x4(const float* A, const float* B, float* D) {
  if (!A || !B || !D) return DRT_E_INVAL;
  hipLaunchKernelGGL(k_probe_mfma, dim3(1), dim3(64), 0, 0, A, B, D);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return DRT_E_DEVICE;
  return DRT_OK;
}

extern "C" int drt_probe_mfma_f16_16x16x32(const uint16_t* A, const uint16_t* B, float* D) {
  if (!A || !B || !D) return DRT_E_INVAL;
  hipLaunchKernelGGL(k_probe_mfma16, dim3(1), dim3(64), 0, 0, (const _Float16*)A, (const _Float16*)B, D);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return DRT_E_DEVICE;
  return DRT_OK;
}

extern "C" int drt_probe_mfma_f64_16x16x4(const double* A, const double* B, double* D) {
  if (!A || !B || !D) return DRT_E_INVAL;
  hipLaunchKernelGGL(k_probe_mfma64, dim3(1), dim3(64), 0, 0, A, B, D);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return DRT_E_DEVICE;
  return DRT_OK;
}

extern "C" int drt_probe_sincos_rev(const float* x, int32_t n, float* s, float* c) {
  if (n < 0 || (n > 0 && (!x || !s || !c))) return DRT_E_INVAL;
  if (n == 0) return DRT_OK;
  hipLaunchKernelGGL(k_probe_sincos, dim3((n + 255) / 256), dim3(256), 0, 0, x, n, s, c);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return DRT_E_DEVICE;
  return DRT_OK;
}
