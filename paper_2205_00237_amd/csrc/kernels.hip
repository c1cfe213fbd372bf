// gfx950 kernels of the DRT hot path.
//
//   k_pose    per (body, instant): sin(theta), 1 - cos(theta) of the body's rotation
//             angle theta = w0*dt + wdot*dt^2/2 (Sec. III-A.1)
//   k_geom    one lane per (ray, instant), one wave per (ray, 64 consecutive instants):
//             interaction points, length, Doppler, angles, field coefficient; writes the
//             caller's per-ray outputs or the per-(ray, instant) anchor records of k_cfr
//   k_cfr     H[t][k] = sum_r a_r(t) exp(-j 2 pi f_k L_r(t)/c): each lane owns one instant
//             and NK consecutive subcarriers, reduces the carrier phase of its first
//             subcarrier modulo one cycle and walks the others with the unit phasor
//             exp(-j 2 pi df L/c); the 4 waves of a workgroup own 4 ray slices of one
//             (instant, subcarrier) tile and are summed in LDS
//   k_reduce  deterministic sum of the per-slice-group partial tiles
#include <hip/hip_runtime.h>

#include "drt_geom.h"
#include "drt_kernels.h"

namespace drt {

template <class F> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// ---------------------------------------------------------------------------------------

template <class F>
__global__ __launch_bounds__(256) void k_pose(const DBody* bodies, int nb, int T, double dt,
                                              typename Vec2<F>::type* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb * T) return;
  int b = i / T, j = i - b * T;
  F d = F(double(j) * dt);
  F th = F(bodies[b].w0) * d + F(0.5) * F(bodies[b].wdot) * d * d;
  F h = msin(th * F(0.5));
  out[i] = {msin(th), F(2) * h * h};   // 1 - cos(theta) without cancellation
}

// ---------------------------------------------------------------------------------------

struct RecS { double L; float gr, gi, zr, zi; };       // split: 24 B
struct RecD { double L, gr, gi, zr, zi; };              // binary64: 40 B
struct RecN { float L, gr, gi, zr, zi, pad; };          // naive binary32: 24 B

template <class F, int MODE, int PREC>
__global__ __launch_bounds__(256) void k_geom(SceneView sc, const typename Vec2<F>::type* pose, int T,
                                              double dt, double f_c, int n_rays, int nchunk,
                                              ExtrapOut eo, void* rec, double df_over_c) {
  int wave = __builtin_amdgcn_readfirstlane(int(blockIdx.x) * 4 + int(threadIdx.x >> 6));
  int lane = threadIdx.x & 63;
  int r = wave / nchunk, chunk = wave - (wave / nchunk) * nchunk;
  if (r >= n_rays) return;
  int t = chunk * 64 + lane;
  bool active = t < T;
  int tq = active ? t : T - 1;
  const DRay& ray = sc.rays[r];
  F dtj = F(double(tq) * dt);
  F half = F(0.5) * dtj * dtj;
  V3<F> TX = ld3<F>(sc.tx_p) + dtj * ld3<F>(sc.tx_v) + half * ld3<F>(sc.tx_a);
  V3<F> RX = ld3<F>(sc.rx_p) + dtj * ld3<F>(sc.rx_v) + half * ld3<F>(sc.rx_a);
  V3<F> VTX = ld3<F>(sc.tx_v) + dtj * ld3<F>(sc.tx_a);
  V3<F> VRX = ld3<F>(sc.rx_v) + dtj * ld3<F>(sc.rx_a);
  Slot<F> sl[DRT_MAX_INT];
  int nint = ray.nint;
#pragma unroll
  for (int i = 0; i < DRT_MAX_INT; ++i) {
    if (i < nint) {
      int b = ray.body[i];
      auto pe = pose[b * T + tq];
      Pose<F> ps = make_pose<F>(sc.bodies[b], dtj, F(pe.x), F(pe.y));
      load_slot<F>(sc, ray.kind[i], ray.prim[i], ps, sl[i]);
    }
  }
  F fc = F(f_c);
  RayResult<F> res = with_signature<F>(ray.code, [&]<int N, int DP, bool SCAT>() {
    return eval_ray<F, N, DP, SCAT>(sc, ray, sl, TX, VTX, RX, VRX, fc);
  });

  if constexpr (MODE == GEOM_EXTRAP) {
    if (!active) return;
    size_t o = size_t(r) * T + t;
    if (eo.L) eo.L[o] = double(res.L);
    if (eo.dop) eo.dop[o] = float(res.dop);
    if (eo.aod_az) eo.aod_az[o] = float(res.aod_az);
    if (eo.aod_el) eo.aod_el[o] = float(res.aod_el);
    if (eo.aoa_az) eo.aoa_az[o] = float(res.aoa_az);
    if (eo.aoa_el) eo.aoa_el[o] = float(res.aoa_el);
    if (eo.gain) {
      if constexpr (PREC == DRT_FP64)
        reinterpret_cast<double2*>(eo.gain)[o] = {double(res.gain.re), double(res.gain.im)};
      else
        reinterpret_cast<float2*>(eo.gain)[o] = {float(res.gain.re), float(res.gain.im)};
    }
    if (eo.valid) eo.valid[o] = res.ok ? 1 : 0;
  } else {
    size_t o = (size_t(chunk) * n_rays + r) * 64 + lane;
    if (!active) res.gain = cx<F>(F(0), F(0));
    if constexpr (PREC == DRT_FP64) {
      double cz = double(res.L) * df_over_c;
      cz -= floor(cz);
      double s, c;
      sincospi(2.0 * cz, &s, &c);
      reinterpret_cast<RecD*>(rec)[o] = {double(res.L), double(res.gain.re), double(res.gain.im), c, -s};
    } else if constexpr (PREC == DRT_SPLIT) {
      double cz = double(res.L) * df_over_c;
      cz -= floor(cz);
      double s, c;
      sincospi(2.0 * cz, &s, &c);
      reinterpret_cast<RecS*>(rec)[o] = {double(res.L), float(res.gain.re), float(res.gain.im),
                                         float(c), float(-s)};
    } else {
      float cz = float(res.L) * float(df_over_c);
      cz -= floorf(cz);
      float s, c;
      sincospif(2.0f * cz, &s, &c);
      reinterpret_cast<RecN*>(rec)[o] = {float(res.L), float(res.gain.re), float(res.gain.im), c, -s, 0.f};
    }
  }
}

// ---------------------------------------------------------------------------------------

// Workgroup -> tile mapping that keeps consecutive logical workgroups on one XCD
// (workgroups are dispatched round-robin over the 8 XCDs); grid padded to a multiple of 8.
__device__ __forceinline__ int xcd_remap(int bid, int grid) {
  int per = grid >> 3;
  return (bid & 7) * per + (bid >> 3);
}

template <class A> struct AccT;
template <> struct AccT<double> { using C = double2; };
template <> struct AccT<float> { using C = float2; };

template <int PREC, int NK>
__global__ __launch_bounds__(256) void k_cfr(const void* rec, CfrArgs a, void* out) {
  using F = typename std::conditional<PREC == DRT_FP64, double, float>::type;
  using C = typename AccT<F>::C;
  __shared__ C red[3][64][NK];
  int bid = xcd_remap(blockIdx.x, gridDim.x);
  if (bid >= a.n_blocks) return;
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int g = bid % a.G, tile = bid / a.G;
  int kt = tile % a.nK, tt = tile / a.nK;
  int slice = g * 4 + wv;
  int r0 = slice * a.slice_len;
  int r1 = min(a.n_rays, r0 + a.slice_len);
  int tl = lane / a.KB, kbl = lane - (lane / a.KB) * a.KB;
  int t = tt * a.TTc + tl;
  int kb = kt * a.KB + kbl;
  int k0 = kb * NK;
  int tq = t < a.T ? t : a.T - 1;
  size_t base = size_t(tq >> 6) * a.n_rays * 64 + (tq & 63);
  const double fb_over_c = (a.f0 + double(k0) * a.df) * (1.0 / 299792458.0);
  F acc_re[NK], acc_im[NK];
#pragma unroll
  for (int i = 0; i < NK; ++i) acc_re[i] = acc_im[i] = F(0);

  for (int r = r0; r < r1; ++r) {
    size_t o = base + size_t(r) * 64;
    F pr, pi, zr, zi;
    if constexpr (PREC == DRT_FP64) {
      RecD q = reinterpret_cast<const RecD*>(rec)[o];
      double cyc = q.L * fb_over_c;
      cyc -= floor(cyc);
      double s, c;
      sincospi(2.0 * cyc, &s, &c);
      pr = q.gr * c + q.gi * s;      // gain * (c - j s)
      pi = q.gi * c - q.gr * s;
      zr = q.zr;
      zi = q.zi;
    } else if constexpr (PREC == DRT_SPLIT) {
      RecS q = reinterpret_cast<const RecS*>(rec)[o];
      double cyc = q.L * fb_over_c;
      cyc -= floor(cyc);
      float ph = float(cyc);
      float s = __builtin_amdgcn_sinf(ph), c = __builtin_amdgcn_cosf(ph);
      pr = q.gr * c + q.gi * s;
      pi = q.gi * c - q.gr * s;
      zr = q.zr;
      zi = q.zi;
    } else {
      RecN q = reinterpret_cast<const RecN*>(rec)[o];
      float cyc = q.L * float(fb_over_c);
      cyc -= floorf(cyc);
      float s = __builtin_amdgcn_sinf(cyc), c = __builtin_amdgcn_cosf(cyc);
      pr = q.gr * c + q.gi * s;
      pi = q.gi * c - q.gr * s;
      zr = q.zr;
      zi = q.zi;
    }
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      acc_re[i] += pr;
      acc_im[i] += pi;
      F nr = pr * zr - pi * zi;
      pi = pr * zi + pi * zr;
      pr = nr;
    }
  }
  // sum the 4 waves' ray slices: waves 1..3 park their partial sums in LDS
  if (wv > 0) {
#pragma unroll
    for (int i = 0; i < NK; ++i) red[wv - 1][lane][i] = C{acc_re[i], acc_im[i]};
  }
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int w = 0; w < 3; ++w) {
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      C v = red[w][lane][i];
      acc_re[i] += v.x;
      acc_im[i] += v.y;
    }
  }
  if (t >= a.T) return;
  C* dst = reinterpret_cast<C*>(out) + (a.G > 1 ? size_t(g) * a.T * a.K : 0) + size_t(t) * a.K;
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    int k = k0 + i;
    if (k < a.K) dst[k] = C{acc_re[i], acc_im[i]};
  }
}

template <class C>
__global__ __launch_bounds__(256) void k_reduce(const C* part, int G, size_t n, C* H) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  C s = part[i];
  for (int g = 1; g < G; ++g) {
    C v = part[size_t(g) * n + i];
    s.x += v.x;
    s.y += v.y;
  }
  H[i] = s;
}

__global__ __launch_bounds__(256) void k_zero(uint32_t* p, size_t n_words) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n_words) p[i] = 0u;
}

// ---------------------------------------------------------------------------------------
// host-side launchers

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((n + 255) / 256), dim3(256), 0, st, (uint32_t*)p, n);
  return hipGetLastError();
}

hipError_t launch_pose(const DBody* bodies, int nb, int T, double dt, int prec, void* out, hipStream_t st) {
  int n = nb * T;
  if (n == 0) return hipSuccess;
  dim3 grid((n + 255) / 256);
  if (prec == DRT_NAIVE32)
    hipLaunchKernelGGL(k_pose<float>, grid, dim3(256), 0, st, bodies, nb, T, dt, (float2*)out);
  else
    hipLaunchKernelGGL(k_pose<double>, grid, dim3(256), 0, st, bodies, nb, T, dt, (double2*)out);
  return hipGetLastError();
}

size_t pose_bytes(int nb, int T, int prec) {
  return size_t(nb) * T * (prec == DRT_NAIVE32 ? sizeof(float2) : sizeof(double2));
}

size_t record_bytes(int n_rays, int T, int prec) {
  size_t per = prec == DRT_FP64 ? sizeof(RecD) : (prec == DRT_SPLIT ? sizeof(RecS) : sizeof(RecN));
  return size_t((T + 63) / 64) * n_rays * 64 * per;
}

template <int MODE>
static hipError_t launch_geom_mode(const SceneView& sc, const void* pose, int T, double dt, double f_c,
                                   int n_rays, int prec, const ExtrapOut& eo, void* rec, double df_over_c,
                                   hipStream_t st) {
  int nchunk = (T + 63) / 64;
  long waves = long(n_rays) * nchunk;
  dim3 grid((waves + 3) / 4);
  if (prec == DRT_FP64)
    hipLaunchKernelGGL((k_geom<double, MODE, DRT_FP64>), grid, dim3(256), 0, st, sc, (const double2*)pose, T,
                       dt, f_c, n_rays, nchunk, eo, rec, df_over_c);
  else if (prec == DRT_SPLIT)
    hipLaunchKernelGGL((k_geom<double, MODE, DRT_SPLIT>), grid, dim3(256), 0, st, sc, (const double2*)pose, T,
                       dt, f_c, n_rays, nchunk, eo, rec, df_over_c);
  else
    hipLaunchKernelGGL((k_geom<float, MODE, DRT_NAIVE32>), grid, dim3(256), 0, st, sc, (const float2*)pose, T,
                       dt, f_c, n_rays, nchunk, eo, rec, df_over_c);
  return hipGetLastError();
}

hipError_t launch_geom(const SceneView& sc, const void* pose, int T, double dt, double f_c, int n_rays, int prec,
                       int mode, const ExtrapOut& eo, void* rec, double df_over_c, hipStream_t st) {
  if (n_rays == 0 || T == 0) return hipSuccess;
  if (mode == GEOM_EXTRAP)
    return launch_geom_mode<GEOM_EXTRAP>(sc, pose, T, dt, f_c, n_rays, prec, eo, rec, df_over_c, st);
  return launch_geom_mode<GEOM_ANCHOR>(sc, pose, T, dt, f_c, n_rays, prec, eo, rec, df_over_c, st);
}

CfrArgs plan_cfr(int n_rays, int T, int K, double f0, double df, int target_waves) {
  CfrArgs a{};
  a.n_rays = n_rays;
  a.T = T;
  a.K = K;
  a.f0 = f0;
  a.df = df;
  int blocks_k = (K + kNK - 1) / kNK;   // subcarrier blocks of kNK
  int kb = 1;
  while (kb < blocks_k && kb < 64) kb <<= 1;
  a.KB = kb;
  a.TTc = 64 / kb;
  a.nT = (T + a.TTc - 1) / a.TTc;
  a.nK = (blocks_k + kb - 1) / kb;
  long tiles = long(a.nT) * a.nK;
  int G = int((target_waves + 4 * tiles - 1) / (4 * tiles));
  int maxG = (n_rays + 4 * kMinSlice - 1) / (4 * kMinSlice);
  if (G > maxG) G = maxG;
  if (G < 1) G = 1;
  a.G = G;
  a.slice_len = (n_rays + 4 * G - 1) / (4 * G);
  a.n_blocks = int(tiles * G);
  return a;
}

hipError_t launch_cfr(const void* rec, const CfrArgs& a, int prec, void* out, hipStream_t st) {
  int grid = ((a.n_blocks + 7) / 8) * 8;
  if (prec == DRT_FP64)
    hipLaunchKernelGGL((k_cfr<DRT_FP64, kNK>), dim3(grid), dim3(256), 0, st, rec, a, out);
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
