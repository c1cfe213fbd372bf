// Host launchers of the ray sums, the partial-sum reduction and the fill kernels.
#include <algorithm>

#include "dev_cfr.h"

namespace drt {

__global__ __launch_bounds__(256) void k_fill_i32(int32_t* p, size_t n, int32_t v) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_zero(uint32_t* p, size_t n_words) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n_words) p[i] = 0u;
}

hipError_t launch_fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((n + 255) / 256), dim3(256), 0, st, (uint32_t*)p, n);
  return hipGetLastError();
}


hipError_t launch_cfr(const void* rec, const CfrArgs& a, int prec, void* out, hipStream_t st) {
  int grid = ((a.n_blocks + 7) / 8) * 8;
  if (a.path == CFR_MFMA64) {
    const RecM64* r = (const RecM64*)rec;
    double* o = (double*)out;
    if (a.MT == 1 && a.NT == 2)
      hipLaunchKernelGGL((k_cfr_mfma64<1, 2>), dim3(grid), dim3(256), 0, st, r, a, o);
    else if (a.MT == 1 && a.NT == 4)
      hipLaunchKernelGGL((k_cfr_mfma64<1, 4>), dim3(grid), dim3(256), 0, st, r, a, o);
    else if (a.MT == 1 && a.NT == 8)
      hipLaunchKernelGGL((k_cfr_mfma64<1, 8>), dim3(grid), dim3(256), 0, st, r, a, o);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (a.path == CFR_MFMA || a.path == CFR_MFMA16) {
    const RecM* r = (const RecM*)rec;
    float* o = (float*)out;
#define DRT_LAUNCH_MFMA(MT_, NT_)                                                                   \
  if (a.MT == MT_ && a.NT == NT_) {                                                               \
    if (a.path == CFR_MFMA16)                                                                     \
      hipLaunchKernelGGL((k_cfr_mfma16<MT_, NT_>), dim3(grid), dim3(256), 0, st, r, a, o);        \
    else                                                                                          \
      hipLaunchKernelGGL((k_cfr_mfma<MT_, NT_>), dim3(grid), dim3(256), 0, st, r, a, o);          \
    return hipGetLastError();                                                                     \
  }
    DRT_LAUNCH_MFMA(1, 1)
    DRT_LAUNCH_MFMA(1, 2)
    DRT_LAUNCH_MFMA(1, 4)
    DRT_LAUNCH_MFMA(2, 4)
    DRT_LAUNCH_MFMA(4, 4)
#undef DRT_LAUNCH_MFMA
    return hipErrorInvalidValue;
  }
  if (prec == DRT_FP64)
    hipLaunchKernelGGL((k_cfr<DRT_FP64, kNK64>), dim3(grid), dim3(256), 0, st, rec, a, out);
  else if (prec == DRT_SPLIT)
    hipLaunchKernelGGL((k_cfr<DRT_SPLIT, kNK>), dim3(grid), dim3(256), 0, st, rec, a, out);
  else
    hipLaunchKernelGGL((k_cfr<DRT_NAIVE32, kNK>), dim3(grid), dim3(256), 0, st, rec, a, out);
  return hipGetLastError();
}

hipError_t launch_reduce(const void* part, int G, size_t n, int prec, void* H, hipStream_t st) {
  dim3 grid((n + 255) / 256);
  if (prec == DRT_FP64)
    hipLaunchKernelGGL(k_reduce<double2>, grid, dim3(256), 0, st, (const double2*)part, G, n, (double2*)H);
  else
    hipLaunchKernelGGL(k_reduce<float2>, grid, dim3(256), 0, st, (const float2*)part, G, n, (float2*)H);
  return hipGetLastError();
}

}  // namespace drt
