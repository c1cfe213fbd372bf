// H(t, f) by a type-1 non-uniform FFT along the subcarrier grid, in binary64 on gfx950.
//
// For one instant, with tau_r = L_r / c, f_k = f_c + k' df and k' = k - K/2:
//   H[k] = sum_r a_r exp(-j 2 pi f_k tau_r) = sum_r c_r exp(-j 2 pi k' x_r),
//   c_r = a_r exp(-j 2 pi frac(f_c tau_r)),  x_r = frac(df tau_r) in [0, 1),
// a sum of R non-uniform points evaluated at K uniform frequencies.  Each c_r is spread onto
// a periodic grid of M >= 2K points with the "exponential of semicircle" kernel
// phi(u) = exp(beta (sqrt(1 - (2u/w)^2) - 1)), |u| < w/2 grid points; the grid is Fourier
// transformed (G[k'] = sum_m g[m] exp(-j 2 pi k' m / M)), and G[k'] divided by the kernel's
// transform phi_hat(k') = int phi(u) cos(2 pi k' u / M) du gives H[k] to a relative accuracy
// of about 10^-(w-1) of sum_r |a_r| (Poisson summation: the grid sum is M times the kernel
// transform at k' plus its aliases at k' + p M, which the kernel's decay suppresses).
//
//   k_nufft_quad    64-point Gauss-Legendre rule on [0, w/2] (Newton on the Legendre
//                   recurrence), with the kernel folded into the weights
//   k_nufft_tables  twiddles exp(-j 2 pi i / M), i < M/2, and phi_hat(k') for k < K from the
//                   rule (phi is even: phi_hat = 2 int_0^{w/2} phi(u) cos(2 pi k' u / M) du)
//   k_nufft_row     one workgroup per instant: spread every ray of the instant into the LDS
//                   grid with binary64 atomic adds, radix-2 FFT in LDS, deconvolve, write
//
// The grid has M >= 2w points, so a kernel footprint wraps around it at most once.
#include <hip/hip_runtime.h>

#include "drt_kernels.h"

namespace drt {

__device__ __forceinline__ double es_kernel(double u, double half_w, double beta) {
  const double t = u / half_w;
  const double q = 1.0 - t * t;
  return q > 0.0 ? exp(beta * (sqrt(q) - 1.0)) : 0.0;
}

constexpr int kQuad = 64;

__global__ __launch_bounds__(64) void k_nufft_quad(int w, double beta, double2* quad) {
  const int i = threadIdx.x;
  // root i of the Legendre polynomial P_n on (-1, 1), from the classical first guess
  double x = cospi((double(i) + 0.75) / (double(kQuad) + 0.5)), dp = 1.0;
  for (int it = 0; it < 8; ++it) {
    double p0 = 1.0, p1 = x;
    for (int n = 2; n <= kQuad; ++n) {
      const double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
      p0 = p1;
      p1 = p2;
    }
    dp = kQuad * (x * p1 - p0) / (x * x - 1.0);
    x -= p1 / dp;
  }
  const double wt = 2.0 / ((1.0 - x * x) * dp * dp);
  // mapped to [0, w/2]
  const double half_w = 0.5 * double(w), u = 0.5 * half_w * (x + 1.0);
  quad[i] = make_double2(u, 0.5 * half_w * wt * es_kernel(u, half_w, beta));
}

__global__ __launch_bounds__(256) void k_nufft_tables(int M, int K, const double2* quad, double2* tw,
                                                      double* phihat) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < M / 2) {
    double s, c;
    sincospi(-2.0 * double(i) / double(M), &s, &c);
    tw[i] = make_double2(c, s);
  }
  if (i < K) {
    const double kp = double(i - K / 2);
    double acc = 0.0;
    for (int q = 0; q < kQuad; ++q) acc += quad[q].y * cospi(2.0 * kp * quad[q].x / double(M));
    phihat[i] = 2.0 * acc;
  }
}

__global__ __launch_bounds__(256) void k_nufft_row(const RecU* rec, int R, int K, int M, int logM, int w,
                                                   double beta, const double2* tw, const double* phihat,
                                                   double2* H) {
  extern __shared__ double2 g[];
  const int t = blockIdx.x, tid = threadIdx.x;
  for (int m = tid; m < M; m += 256) g[m] = make_double2(0.0, 0.0);
  __syncthreads();
  // spreading: ray r adds c_r phi(m - M x_r) to the w grid points m around M x_r (mod M)
  const RecU* row = rec + size_t(t) * R;
  const double half_w = 0.5 * double(w);
  for (int r = tid; r < R; r += 256) {
    const RecU q = row[r];
    if (q.cr == 0.0 && q.ci == 0.0) continue;
    const double u0 = double(M) * q.x;
    const int m0 = int(ceil(u0 - half_w));
    for (int j = 0; j < w; ++j) {
      const int m = m0 + j;
      const double phi = es_kernel(double(m) - u0, half_w, beta);
      const int idx = m < 0 ? m + M : (m >= M ? m - M : m);
      atomicAdd(&g[idx].x, q.cr * phi);
      atomicAdd(&g[idx].y, q.ci * phi);
    }
  }
  __syncthreads();
  // radix-2 decimation-in-time FFT: bit-reversed order, then log2 M butterfly stages
  for (int i = tid; i < M; i += 256) {
    const int j = int(__brev(unsigned(i)) >> (32 - logM));
    if (i < j) {
      const double2 a = g[i];
      g[i] = g[j];
      g[j] = a;
    }
  }
  __syncthreads();
  for (int s = 0; s < logM; ++s) {
    const int half = 1 << s, stride = M >> (s + 1);
    for (int b = tid; b < M / 2; b += 256) {
      const int pos = b & (half - 1);
      const int i = ((b >> s) << (s + 1)) + pos, j = i + half;
      const double2 wv = tw[pos * stride];
      const double2 y = g[j];
      const double2 x = make_double2(wv.x * y.x - wv.y * y.y, wv.x * y.y + wv.y * y.x);
      const double2 a = g[i];
      g[i] = make_double2(a.x + x.x, a.y + x.y);
      g[j] = make_double2(a.x - x.x, a.y - x.y);
    }
    __syncthreads();
  }
  // deconvolution: H[k] = G[k' mod M] / phi_hat(k'), k' = k - K/2
  double2* out = H + size_t(t) * K;
  for (int k = tid; k < K; k += 256) {
    int kp = k - K / 2;
    if (kp < 0) kp += M;
    const double inv = 1.0 / phihat[k];
    out[k] = make_double2(g[kp].x * inv, g[kp].y * inv);
  }
}

hipError_t launch_nufft(const RecU* rec, int R, int T, int K, int M, int w, double beta, double2* tw,
                        double* phihat, double2* quad, double2* H, hipStream_t st) {
  if (T == 0 || K == 0) return hipSuccess;
  int logM = 0;
  while ((1 << logM) < M) ++logM;
  const int n = (M / 2 > K ? M / 2 : K);
  hipLaunchKernelGGL(k_nufft_quad, dim3(1), dim3(kQuad), 0, st, w, beta, quad);
  hipLaunchKernelGGL(k_nufft_tables, dim3((n + 255) / 256), dim3(256), 0, st, M, K, (const double2*)quad, tw,
                     phihat);
  hipLaunchKernelGGL(k_nufft_row, dim3(T), dim3(256), size_t(M) * sizeof(double2), st, rec, R, K, M, logM, w, beta,
                     (const double2*)tw, (const double*)phihat, H);
  return hipGetLastError();
}

}  // namespace drt
