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
__device__ __forceinline__ void pose_item(const DBody* bodies, int T, double dt, int i,
                                          typename Vec2<F>::type* out) {
  int b = i / T, j = i - b * T;
  F d = F(double(j) * dt);
  F th = F(bodies[b].w0) * d + F(0.5) * F(bodies[b].wdot) * d * d;
  F h = msin(th * F(0.5));
  out[i] = {msin(th), F(2) * h * h};   // 1 - cos(theta) without cancellation
}

template <class F>
__global__ __launch_bounds__(256) void k_pose(const DBody* bodies, int nb, int T, double dt,
                                              typename Vec2<F>::type* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb * T) pose_item<F>(bodies, T, dt, i, out);
}

// ---------------------------------------------------------------------------------------

struct RecS { double L; float gr, gi, zr, zi; };       // split: 24 B
// split, MFMA path: 32 B.  Phases in cycles, reduced modulo one in binary64: phi0 of the
// first subcarrier (gain argument folded in), phiB per row block of B subcarriers and phi1
// per subcarrier (both kept in binary64, since a lane multiplies them by its row / column
// index 0..15), and p16B, p16_1 their 16-fold multiples (the step between 16-row tiles).
struct RecM {
  float amp, phi0, p16B, p16_1;
  double phiB, phi1;
};
// The same 32 bytes as four 64-bit words (amp | phi0, p16B | p16_1, phiB, phi1).
struct RecW { uint64_t w[4]; };
static_assert(sizeof(RecM) == sizeof(RecW), "RecM is four 64-bit words");
struct RecD { double L, gr, gi, zr, zi; };              // binary64: 40 B
struct RecN { float L, gr, gi, zr, zi, pad; };          // naive binary32: 24 B

// Field-coefficient and angle type of a precision: binary64 only in DRT_FP64.
template <int PREC> struct GainT { using type = float; };
template <> struct GainT<DRT_FP64> { using type = double; };

// Adds each lane's value v to base[key] (lanes with key < 0 add nothing).  Lanes hold
// consecutive instants of one ray, so equal keys come in runs: a segmented inclusive scan
// over the 64 lanes sums each run, and the run's last lane issues one binary64 atomic add.
__device__ __forceinline__ void wave_bin_add(double* base, int key, double v, int lane) {
  const int prev = __shfl_up(key, 1), next = __shfl_down(key, 1);
  const unsigned long long heads = __ballot(lane == 0 || key != prev);
  // first lane of this lane's run: the highest run head at or below the lane
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int start = 63 - __clzll((long long)(heads & upto));
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double u = __shfl_up(v, off);
    if (lane - off >= start) v += u;
  }
  if (key >= 0 && (lane == 63 || key != next)) unsafeAtomicAdd(base + key, v);
}

// One wave: ray order[i] over the 64 instants of chunk c, where wave = 4 (nchunk (i / 4) + c) + i % 4.
template <class F, int MODE, int PREC, int CLS, bool POL = false>
__device__ __forceinline__ void geom_wave(const SceneView& sc, const int32_t* order, int count,
                                          const typename Vec2<F>::type* pose, int T, double dt, double f_c,
                                          int n_rays, int nchunk, const ExtrapOut& eo, void* rec,
                                          const AnchorParams& ap, int wave, int lane) {
  // the 4 waves of a workgroup take 4 consecutive rays of the class at the same 64
  // instants, so their instant-major records of one instant land side by side
  const int blk = wave >> 2;
  const int i = (blk / nchunk) * 4 + (wave & 3), chunk = blk - (blk / nchunk) * nchunk;
  if (i >= count) return;
  int r = __builtin_amdgcn_readfirstlane(order[i]);
  int t = chunk * 64 + lane;
  bool active = t < T;
  int tq = active ? t : T - 1;
  const DRay& ray = sc.rays[r];
  if constexpr (MODE == GEOM_KIN) {
    // the chain as jets in time (binary64): points, velocities, accelerations, L'' (Sec.
    // III-A.1 eqs. ref_point_velo, ref_point_acc; App. B, C); the body angle's jet from the
    // pose table's sin(theta), 1 - cos(theta) and theta' = w0 + wdot t, theta'' = wdot
    using J = J2<double>;
    const double tt = double(tq) * dt;
    const J tj(tt, 1.0, 0.0);
    const J hj = J(0.5) * tj * tj;
    const V3<J> TXj = ld3<J>(sc.tx_p) + tj * ld3<J>(sc.tx_v) + hj * ld3<J>(sc.tx_a);
    const V3<J> RXj = ld3<J>(sc.rx_p) + tj * ld3<J>(sc.rx_v) + hj * ld3<J>(sc.rx_a);
    Slot<J> sj[DRT_MAX_INT];
    const int nint = ray.nint;
#pragma unroll
    for (int i = 0; i < DRT_MAX_INT; ++i) {
      if (i < nint) {
        const int b = ray.body[i];
        const DBody& B = sc.bodies[b];
        const auto pe = pose[b * T + tq];
        const double sn = double(pe.x), c1 = double(pe.y), cs = 1.0 - c1;
        const double w1 = B.w0 + B.wdot * tt, w2 = B.wdot;
        const J sth(sn, cs * w1, -sn * w1 * w1 + cs * w2), cth(c1, sn * w1, cs * w1 * w1 + sn * w2);
        load_slot<J>(sc, ray.kind[i], ray.prim[i], make_pose<J>(B, tj, sth, cth), sj[i]);
      }
    }
    KinResult<J> kr = with_signature_in<J, CLS>(ray.code, [&]<int N, int DP, bool SCAT>() {
      return kin_ray<J, N, DP, SCAT>(sj, TXj, RXj);
    });
    if (!active) return;
    const size_t o = size_t(r) * T + t;
    if (eo.dop_rate) eo.dop_rate[o] = kr.ok ? float(-(f_c / 299792458.0) * kr.L.dd) : 0.f;
#pragma unroll
    for (int i = 0; i < DRT_MAX_INT; ++i) {
      const bool w = kr.ok && i < nint;
      const V3<J> q = kr.Q[i];
      const size_t e = (o * DRT_MAX_INT + i) * 3;
      if (eo.q_pos) {
        eo.q_pos[e] = w ? q.x.v : 0.0;
        eo.q_pos[e + 1] = w ? q.y.v : 0.0;
        eo.q_pos[e + 2] = w ? q.z.v : 0.0;
      }
      if (eo.q_vel) {
        eo.q_vel[e] = w ? q.x.d : 0.0;
        eo.q_vel[e + 1] = w ? q.y.d : 0.0;
        eo.q_vel[e + 2] = w ? q.z.d : 0.0;
      }
      if (eo.q_acc) {
        eo.q_acc[e] = w ? q.x.dd : 0.0;
        eo.q_acc[e + 1] = w ? q.y.dd : 0.0;
        eo.q_acc[e + 2] = w ? q.z.dd : 0.0;
      }
    }
    return;
  }
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
  using G = typename GainT<PREC>::type;
  RayResult<F, G> res = with_signature_in<F, CLS>(ray.code, [&]<int N, int DP, bool SCAT>() {
    return eval_ray<F, G, N, DP, SCAT, false, MODE == GEOM_EXTRAP || MODE == GEOM_POWER, POL>(sc, ray, sl, TX,
                                                                                              VTX, RX, VRX, fc);
  });

  if constexpr (MODE == GEOM_EXTRAP) {
    if (eo.first_out) {
      // first instant of this chunk out of bounds; the ray's minimum over chunks by atomics
      const unsigned long long out = __ballot(active && !res.in_bounds);
      if (out != 0ull && lane == __ffsll((long long)out) - 1) atomicMin(eo.first_out + r, t);
    }
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
    if (eo.in_bounds) eo.in_bounds[o] = res.in_bounds ? 1 : 0;
  } else if constexpr (MODE == GEOM_POWER) {
    // incoherent power sums (Sec. IV-A, IV-B): every lane takes part in the wave scans
    const bool cnt = active && res.ok && (eo.gate == 0 || res.in_bounds);
    const double gr = double(res.gain.re), gi = double(res.gain.im);
    const double p = cnt ? gr * gr + gi * gi : 0.0;
    const int tb = t / eo.spb;
    if (eo.ptotal) wave_bin_add(eo.ptotal, cnt ? tb : -1, p, lane);
    if (eo.pdfp) {
      const double u = floor((double(res.dop) - eo.dop_lo) / eo.dop_step);
      const bool in = cnt && u >= 0.0 && u < double(eo.n_dop);
      wave_bin_add(eo.pdfp, in ? tb * eo.n_dop + int(u) : -1, p, lane);
    }
    if (eo.pdp) {
      const double tau = double(res.L) / 299792458.0;
      const double u = floor((tau - eo.delay_lo) / eo.delay_step);
      const bool in = cnt && u >= 0.0 && u < double(eo.n_delay);
      wave_bin_add(eo.pdp, in ? tb * eo.n_delay + int(u) : -1, p, lane);
    }
  } else if constexpr (MODE == GEOM_NUFFT) {
    // non-uniform FFT record: x = frac(df L / c), c = a exp(-j 2 pi frac(f_c L / c)), both
    // phases reduced modulo one cycle in binary64
    if (!active) return;
    const double L = double(res.L);
    double px = L * ap.f1c, pc = L * ap.f0c;
    px -= floor(px);
    pc -= floor(pc);
    double s, c;
    sincospi(2.0 * pc, &s, &c);
    const double gr = double(res.gain.re), gi = double(res.gain.im);
    reinterpret_cast<RecU*>(rec)[size_t(t) * n_rays + r] = {px, gr * c + gi * s, gi * c - gr * s};
  } else if constexpr (MODE == GEOM_ANCHOR_MFMA) {
    // phases of the first subcarrier, of one row block and of one subcarrier, each reduced
    // modulo one cycle in binary64 before rounding to binary32; the gain enters as its
    // modulus and its argument, the latter folded into the first-subcarrier phase
    // (a e^{-j 2 pi p0} = |a| e^{-j 2 pi (p0 - arg a / 2 pi)})
    if (!active) return;
    size_t o = size_t(t) * n_rays + r;      // instant-major: a ray-sum wave streams its instant
    double L = double(res.L);
    const float gr = float(res.gain.re), gi = float(res.gain.im);
    double p0 = L * ap.f0c - double(atan2f(gi, gr)) * (0.5 / M_PI), pB = L * ap.fBc, p1 = L * ap.f1c;
    p0 -= floor(p0);
    pB -= floor(pB);
    p1 -= floor(p1);
    double q16B = 16.0 * pB, q16_1 = 16.0 * p1;
    q16B -= floor(q16B);
    q16_1 -= floor(q16_1);
    reinterpret_cast<RecM*>(rec)[o] = {sqrtf(gr * gr + gi * gi), float(p0), float(q16B), float(q16_1), pB, p1};
  } else {
    size_t o = (size_t(chunk) * n_rays + r) * 64 + lane;
    if (!active) res.gain = cx<G>(G(0), G(0));
    const double df_over_c = ap.f1c;
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

template <class F, int MODE, int PREC, int CLS, bool POL>
__global__ __launch_bounds__(256) void k_geom(SceneView sc, const int32_t* order, int count,
                                              const typename Vec2<F>::type* pose, int T, double dt, double f_c,
                                              int n_rays, int nchunk, ExtrapOut eo, void* rec, AnchorParams ap) {
  int wave = __builtin_amdgcn_readfirstlane(int(blockIdx.x) * 4 + int(threadIdx.x >> 6));
  geom_wave<F, MODE, PREC, CLS, POL>(sc, order, count, pose, T, dt, f_c, n_rays, nchunk, eo, rec, ap, wave,
                                     int(threadIdx.x & 63));
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

// Three waves per SIMD: the LDS of the slice reduction (48 KiB in binary64) admits three
// workgroups per CU, and capping the registers to match (168) lets all of them run, where
// the unconstrained allocation (256 registers) held two.
template <int PREC, int NK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void k_cfr(const void* rec, CfrArgs a, void* out) {
  using F = typename std::conditional<PREC == DRT_FP64, double, float>::type;
  using C = typename AccT<F>::C;
  constexpr int NH = sizeof(C) * NK > 256 ? NK / 2 : NK;   // subcarriers per LDS pass (48 KiB at most)
  __shared__ C red[3][64][NH];
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

  // first subcarrier's phasor of ray r at this lane's block, times the gain, and the
  // one-subcarrier step
  auto start = [&](int r, F& pr, F& pi, F& zr, F& zi) {
    const size_t o = base + size_t(r) * 64;
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
  };
  // W rays at a time: W independent phasor walks interleave, so each step's latency hides
  // behind the other walks'.  In binary64 a walk takes the three-term form of the unit-phasor
  // power, p_{i+1} = 2 cos(theta) p_i - p_{i-1} (z + 1/z = 2 cos theta for |z| = 1): one FMA per
  // component and step instead of a complex product; its rounding grows like i eps / sin theta,
  // below 1e-12 for the 16 steps at any delay of a metre or more
  constexpr int W = NK > 16 ? 2 : 4;
  int r = r0;
  for (; r + W <= r1; r += W) {
    F pr[W], pi[W], zr[W], zi[W];
#pragma unroll
    for (int u = 0; u < W; ++u) start(r + u, pr[u], pi[u], zr[u], zi[u]);
    if constexpr (PREC == DRT_FP64) {
      F qr[W], qi[W], c2[W];                     // p_{i+1} (q) after p_i (p)
#pragma unroll
      for (int u = 0; u < W; ++u) {
        qr[u] = pr[u] * zr[u] - pi[u] * zi[u];
        qi[u] = pr[u] * zi[u] + pi[u] * zr[u];
        c2[u] = F(2) * zr[u];
      }
#pragma unroll
      for (int i = 0; i < NK; ++i) {
        F sr = pr[0], si = pi[0];
#pragma unroll
        for (int u = 1; u < W; ++u) {
          sr += pr[u];
          si += pi[u];
        }
        acc_re[i] += sr;
        acc_im[i] += si;
#pragma unroll
        for (int u = 0; u < W; ++u) {
          const F nr = c2[u] * qr[u] - pr[u], ni = c2[u] * qi[u] - pi[u];
          pr[u] = qr[u];
          pi[u] = qi[u];
          qr[u] = nr;
          qi[u] = ni;
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < NK; ++i) {
        F sr = pr[0], si = pi[0];
#pragma unroll
        for (int u = 1; u < W; ++u) {
          sr += pr[u];
          si += pi[u];
        }
        acc_re[i] += sr;
        acc_im[i] += si;
#pragma unroll
        for (int u = 0; u < W; ++u) {
          F nr = pr[u] * zr[u] - pi[u] * zi[u];
          pi[u] = pr[u] * zi[u] + pi[u] * zr[u];
          pr[u] = nr;
        }
      }
    }
  }
  for (; r < r1; ++r) {
    F pr, pi, zr, zi;
    start(r, pr, pi, zr, zi);
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      acc_re[i] += pr;
      acc_im[i] += pi;
      F nr = pr * zr - pi * zi;
      pi = pr * zi + pi * zr;
      pr = nr;
    }
  }
  // sum the 4 waves' ray slices: waves 1..3 park their partial sums in LDS, NH subcarriers
  // per pass
#pragma unroll
  for (int h = 0; h < NK; h += NH) {
    if (h > 0) __syncthreads();                  // wave 0 has read the previous pass
    if (wv > 0) {
#pragma unroll
      for (int i = 0; i < NH; ++i) red[wv - 1][lane][i] = C{acc_re[h + i], acc_im[h + i]};
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int w = 0; w < 3; ++w) {
#pragma unroll
        for (int i = 0; i < NH; ++i) {
          C v = red[w][lane][i];
          acc_re[h + i] += v.x;
          acc_im[h + i] += v.y;
        }
      }
    }
  }
  if (wv != 0 || t >= a.T) return;
  C* dst = reinterpret_cast<C*>(out) + (a.G > 1 ? size_t(g) * a.T * a.K : 0) + size_t(t) * a.K;
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    int k = k0 + i;
    if (k < a.K) dst[k] = C{acc_re[i], acc_im[i]};
  }
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

// frac(i * step) + base for a lane's row / column index i < 16: the product and its
// reduction in binary64, so the step's rounding is not multiplied by i; below 2 cycles, as
// v_sin / v_cos take it.
__device__ __forceinline__ float row_phase(int i, double step, float base) {
  return float(__builtin_amdgcn_fract(double(i) * step)) + base;
}

// Split-precision ray sum as complex GEMMs on the matrix cores.  With k = k1 B + k2,
// exp(-j 2 pi f_k L/c) = exp(-j 2 pi (f_0 + k1 B df) L/c) exp(-j 2 pi k2 df L/c), so for one
// instant H[k1 B + k2] = sum_r U[k1][r] V[r][k2] with U = a exp(-j 2 pi (f_0 + k1 B df) L/c)
// and V = exp(-j 2 pi k2 df L/c): each U is reused B times and each V K/B times.  The
// complex product is the real GEMM [U_re U_im] [[V_re V_im], [-V_im V_re]]; one
// v_mfma_f32_16x16x4_f32 takes two rays (4 contraction slots: ray0 re, ray0 im, ray1 re,
// ray1 im).  Lane l supplies A[row l%16][slot l/16] and B[slot l/16][column l%16] and owns
// accumulator rows 4(l/16)..4(l/16)+3 of column l%16.  Rows are k1 (MT tiles of 16), columns
// are [C_re for k2 < B | C_im for k2 < B] (NT tiles of 16, B = 8 NT).  Operands are
// generated on the vector ALU from the record's binary64-reduced phases: with k1 = 16 mt + m
// the U row phase is frac(m phiB) + phi0 + mt p16B and with k2 = 16 h + m the V column phase
// frac(m phi1) + h p16_1 (cycles, below 5), the products m phiB and m phi1 taken in
// binary64; v_sin/v_cos take revolutions and reduce them modulo one exactly.
template <int MT, int NT>
__global__ __launch_bounds__(256) void k_cfr_mfma(const RecM* rec, CfrArgs a, float* out) {
  constexpr int B = 8 * NT;
  __shared__ floatx4 red[3][64][MT * NT];
  int bid = xcd_remap(blockIdx.x, gridDim.x);
  if (bid >= a.n_blocks) return;
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int g = bid % a.G, t = bid / a.G;
  int slice = g * 4 + wv;
  int r0 = slice * a.slice_len;
  int r1 = min(a.n_rays, r0 + a.slice_len);
  const int m = lane & 15, kslot = lane >> 4, rsel = kslot >> 1, part = kslot & 1;
  const RecM* rt = rec + size_t(t) * a.n_rays;
  floatx4 acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  // 64 rays' records per coalesced load (one per lane), the next batch in flight while the
  // current one is consumed pair by pair through cross-lane shuffles
  auto load = [&](int rb) {
    int r = rb + lane;
    return r < r1 ? rt[r] : RecM{0.f, 0.f, 0.f, 0.f, 0.0, 0.0};
  };
  RecM cur = load(r0);
  for (int rb = r0; rb < r1; rb += 64) {
    RecM nxt = load(rb + 64);
    const int npairs = min(32, (r1 - rb + 1) >> 1);
#pragma unroll 2
    for (int p = 0; p < npairs; ++p) {
    const int src = 2 * p + rsel;
    RecM q;
    q.amp = __shfl(cur.amp, src);
    q.phi0 = __shfl(cur.phi0, src);
    q.p16B = __shfl(cur.p16B, src);
    q.p16_1 = __shfl(cur.p16_1, src);
    q.phiB = __shfl(cur.phiB, src);
    q.phi1 = __shfl(cur.phi1, src);
    const float u0 = row_phase(m, q.phiB, q.phi0);
    float av[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      float ph = __builtin_fmaf(float(mt), q.p16B, u0);
      float s = __builtin_amdgcn_sinf(ph), c = __builtin_amdgcn_cosf(ph);
      av[mt] = part == 0 ? q.amp * c : -(q.amp * s);                     // Re / Im of |a| e^{-j 2 pi ph}
    }
    float bv[NT];
    if constexpr (NT == 1) {
      float ph = row_phase(m & 7, q.phi1, 0.f);
      float s = __builtin_amdgcn_sinf(ph), c = __builtin_amdgcn_cosf(ph);
      bv[0] = (m >> 3) == 0 ? (part == 0 ? c : s) : (part == 0 ? -s : c);
    } else {
      const float v0 = row_phase(m, q.phi1, 0.f);
#pragma unroll
      for (int h = 0; h < NT / 2; ++h) {
        float ph = __builtin_fmaf(float(h), q.p16_1, v0);
        float s = __builtin_amdgcn_sinf(ph), c = __builtin_amdgcn_cosf(ph);
        bv[h] = part == 0 ? c : s;                 // C_re columns: V_re, -V_im
        bv[h + NT / 2] = part == 0 ? -s : c;       // C_im columns: V_im, V_re
      }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt], bv[nt], acc[mt][nt], 0, 0, 0);
    }
    cur = nxt;
  }
  if (wv > 0) {
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) red[wv - 1][lane][i * NT + j] = acc[i][j];
  }
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] += red[w][lane][i * NT + j];
  float* dst = out + (a.G > 1 ? size_t(g) * a.T * a.K * 2 : 0) + size_t(t) * a.K * 2;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int k1 = mt * 16 + 4 * kslot + v;
        int col = nt * 16 + m;
        int k2 = col % B, isim = col / B;
        int k = k1 * B + k2;
        if (k1 < a.K1 && k < a.K) dst[size_t(k) * 2 + isim] = acc[mt][nt][v];
      }
}

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __fp16 fp16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// hi + lo binary16 pairs of two binary32 values, each pair packed in one 32-bit word: hi
// rounds toward zero, lo = x - hi is representable to 2^-11 of itself, so hi + lo keeps
// ~22 bits of x.
// The residuals x - hi are exact in binary32 (hi keeps the leading 11 bits of x) and are
// formed by one mixed-precision FMA each, -hi * 1 + x, reading hi straight from its half of
// the packed word; the compiler lowers the plain expression to a conversion and a subtraction.
__device__ __forceinline__ float resid_lo(unsigned h, float x) {
  float r;
  asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(h), "v"(x));
  return r;
}
__device__ __forceinline__ float resid_hi(unsigned h, float x) {
  float r;
  asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(h), "v"(x));
  return r;
}
// Compile-time loop: f(IC<I>{}) for I = B .. E-1.
template <int V> struct IC { static constexpr int value = V; };
template <int B, int E, class Fn>
__device__ __forceinline__ void static_for(Fn&& f) {
  if constexpr (B < E) {
    f(IC<B>{});
    static_for<B + 1, E>(f);
  }
}

// Value of lane 16 (l / 16) + S for lane l: DPP row_newbcast, a vector-ALU move within each
// row of 16 lanes.  Every row and bank is enabled and every lane's source exists, so every
// lane is written and the old value (bound_ctrl set: none is read) needs no initialisation.
template <int S>
__device__ __forceinline__ uint64_t row_bcast(uint64_t x) {
  static_assert(S >= 0 && S < 16, "row position");
  return __builtin_amdgcn_update_dpp(uint64_t(0), x, 0x150 + S, 0xF, 0xF, true);
}

__device__ __forceinline__ unsigned pk16(float x, float y) {
  return __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(x, y));
}

// (x, y) -> hi, lo words of (x, y); with rot, also those of (-y, x): rounding toward zero
// commutes with negation, so the rotated pair splits into the rotated halves
struct Split16 { unsigned hi, lo, rhi, rlo; };
template <bool ROT>
__device__ __forceinline__ Split16 split_pair(float x, float y) {
  Split16 w;
  w.hi = pk16(x, y);
  const float rx = resid_lo(w.hi, x), ry = resid_hi(w.hi, y);
  w.lo = pk16(rx, ry);
  if constexpr (ROT) {
    w.rhi = pk16(-y, x);
    w.rlo = pk16(-ry, rx);
  }
  return w;
}

// Split-precision ray sum on the binary16 matrix cores.  Same factorisation as k_cfr_mfma
// (H[k1 B + k2] = sum_r U[k1][r] V[r][k2]), but each binary32 operand x is carried as
// hi + lo in binary16 and the product as hi.hi + hi.lo + lo.hi (three
// v_mfma_f32_16x16x32_f16 per tile, relative error ~2^-22), accumulated in binary32.
// One instruction contracts 32 slots = 16 rays x (re, im): lane l owns A[row l%16][slots
// 8(l/16)..+7] and B[slots 8(l/16)..+7][column l%16], i.e. rays 4(l/16)..+3 of each block
// of 16, and generates whole complex U and V values for them.  Each wave scales its ray
// slice's gains by a power of two that puts the largest component near 2^13 (binary16
// tops out at 65504 and is normal down to 2^-14) and divides it out of its accumulators
// before the slices are summed.
// Workgroup tile bid = (instant, ray group); red is the workgroup's LDS staging of waves 1..3.
template <int MT, int NT>
__device__ __forceinline__ void cfr16_tile(const RecM* rec, const CfrArgs& a, float* out, int bid,
                                           floatx4 (*red)[64][MT * NT]) {
  constexpr int B = 8 * NT;
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int g = bid % a.G, t = bid / a.G;
  int slice = g * 4 + wv;
  int r0 = slice * a.slice_len;
  int r1 = min(a.n_rays, r0 + a.slice_len);
  const int m = lane & 15, grp = lane >> 4;
  const RecM* rt = rec + size_t(t) * a.n_rays;
  floatx4 acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  // lane 16 g + 4 b + j loads ray 16 b + 4 g + j of each batch of 64 (the same cache lines
  // as a plain load): the four rays of block b that the lanes of row g consume then sit in
  // row g, at positions 4 b .. 4 b + 3, and DPP row broadcasts hand them over without LDS
  const int pl = 16 * ((lane >> 2) & 3) + 4 * grp + (lane & 3);
  const RecW* rw = reinterpret_cast<const RecW*>(rt);
  auto load = [&](int rb) {
    const int r = rb + pl;
    return r < r1 ? rw[r] : RecW{0ull, 0ull, 0ull, 0ull};
  };
  float amax = 0.f;
  for (int rb = r0 + lane; rb < r1; rb += 64) amax = fmaxf(amax, rt[rb].amp);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
  int e2 = 0;
  (void)frexpf(amax, &e2);                       // amax < 2^e2
  const float kScale = amax > 0.f ? ldexpf(1.f, 13 - e2) : 1.f;
  const float kInv = 1.f / kScale;
  RecW cur = load(r0);
  for (int rb = r0; rb < r1; rb += 64) {
    RecW nxt = load(rb + 64);
    const int nblk = min(4, (r1 - rb + 15) >> 4);
    static_for<0, 4>([&](auto BK) {
      constexpr int bk = decltype(BK)::value;
      if (bk >= nblk) return;
      // U operands of the 16 rays (lane: rays 4 grp .. 4 grp + 3 of the block) for every
      // row tile; the V column phases' bases, kept for the column-tile loop below
      u32x4 ahw[MT], alw[MT];
      float vb[4], vs[4];
      static_for<0, 4>([&](auto J) {
        constexpr int j = decltype(J)::value, S = 4 * bk + j;
        const uint64_t w0 = row_bcast<S>(cur.w[0]), w1 = row_bcast<S>(cur.w[1]);
        const double phiB = __builtin_bit_cast(double, row_bcast<S>(cur.w[2]));
        const double phi1 = __builtin_bit_cast(double, row_bcast<S>(cur.w[3]));
        const float amp = __uint_as_float(uint32_t(w0)) * kScale, phi0 = __uint_as_float(uint32_t(w0 >> 32));
        const float p16B = __uint_as_float(uint32_t(w1));
        vs[j] = __uint_as_float(uint32_t(w1 >> 32));
        const float u0 = row_phase(m, phiB, phi0);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const float ph = mt == 0 ? u0 : __builtin_fmaf(float(mt), p16B, u0);
          float sn = __builtin_amdgcn_sinf(ph), c = __builtin_amdgcn_cosf(ph);
          Split16 w = split_pair<false>(amp * c, -(amp * sn));   // U = |a| e^{-j 2 pi ph}
          ahw[mt][j] = w.hi;
          alw[mt][j] = w.lo;
        }
        vb[j] = float(__builtin_amdgcn_fract(double(NT == 1 ? (m & 7) : m) * phi1));
      });
      half8 ah[MT], al[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        ah[mt] = __builtin_bit_cast(half8, ahw[mt]);
        al[mt] = __builtin_bit_cast(half8, alw[mt]);
      }
      // V operands one column-tile pair at a time, each consumed right away (shorter live
      // ranges, and the matrix instructions of one pair overlap the phasors of the next)
#pragma unroll
      for (int hh = 0; hh < (NT + 1) / 2; ++hh) {
        u32x4 h0, l0, h1, l1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float ph = hh == 0 ? vb[j] : __builtin_fmaf(float(hh), vs[j], vb[j]);
          float sn = __builtin_amdgcn_sinf(ph), c = __builtin_amdgcn_cosf(ph);
          if constexpr (NT == 1) {
            // C_re column: (V_re, -V_im) = (c, s); C_im column: (V_im, V_re) = (-s, c)
            Split16 w = (m >> 3) == 0 ? split_pair<false>(c, sn) : split_pair<false>(-sn, c);
            h0[j] = w.hi;
            l0[j] = w.lo;
          } else {
            Split16 w = split_pair<true>(c, sn);
            h0[j] = w.hi;
            l0[j] = w.lo;
            h1[j] = w.rhi;
            l1[j] = w.rlo;
          }
        }
        const half8 bh0 = __builtin_bit_cast(half8, h0), bl0 = __builtin_bit_cast(half8, l0);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          acc[mt][hh] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[mt], bh0, acc[mt][hh], 0, 0, 0);
          acc[mt][hh] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[mt], bl0, acc[mt][hh], 0, 0, 0);
          acc[mt][hh] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[mt], bh0, acc[mt][hh], 0, 0, 0);
        }
        if constexpr (NT > 1) {
          const half8 bh1 = __builtin_bit_cast(half8, h1), bl1 = __builtin_bit_cast(half8, l1);
          constexpr int o = NT / 2;
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            acc[mt][hh + o] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[mt], bh1, acc[mt][hh + o], 0, 0, 0);
            acc[mt][hh + o] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[mt], bl1, acc[mt][hh + o], 0, 0, 0);
            acc[mt][hh + o] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[mt], bh1, acc[mt][hh + o], 0, 0, 0);
          }
        }
      }
    });
    cur = nxt;
  }
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] *= kInv;      // exact: a power of two
  if (wv > 0) {
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) red[wv - 1][lane][i * NT + j] = acc[i][j];
  }
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] += red[w][lane][i * NT + j];
  float* dst = out + (a.G > 1 ? size_t(g) * a.T * a.K * 2 : 0) + size_t(t) * a.K * 2;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int k1 = mt * 16 + 4 * grp + v;
        int col = nt * 16 + m;
        int k2 = col % B, isim = col / B;
        int k = k1 * B + k2;
        if (k1 < a.K1 && k < a.K) dst[size_t(k) * 2 + isim] = acc[mt][nt][v];
      }
}

// Four waves per SIMD for the tile shapes up to 2 x 4 (128 registers): the matrix
// instructions of one wave overlap the phasor arithmetic of the others.
template <int MT, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MT * NT <= 8 ? 4 : 1)))
void k_cfr_mfma16(const RecM* rec, CfrArgs a, float* out) {
  __shared__ floatx4 red[3][64][MT * NT];
  int bid = xcd_remap(blockIdx.x, gridDim.x);
  if (bid < a.n_blocks) cfr16_tile<MT, NT>(rec, a, out, bid, red);
}

template <class C>
__device__ __forceinline__ void reduce_item(const C* part, int G, size_t n, C* H, size_t i) {
  C s = part[i];
  for (int g = 1; g < G; ++g) {
    C v = part[size_t(g) * n + i];
    s.x += v.x;
    s.y += v.y;
  }
  H[i] = s;
}

template <class C>
__global__ __launch_bounds__(256) void k_reduce(const C* part, int G, size_t n, C* H) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) reduce_item<C>(part, G, n, H, i);
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t* p, size_t n, int32_t v) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_zero(uint32_t* p, size_t n_words) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n_words) p[i] = 0u;
}

// ---------------------------------------------------------------------------------------
// batch kernels: one launch per kernel kind covers the work items of every request in the
// batch; the grid is set per batch to the item count (one thread, wave or workgroup per
// item, so the dispatcher balances requests of any size), and the request of an item is
// found from the item prefix sums of its kind

// request j with off[j] <= item < off[j+1] for every lane (n <= 64, item the same on all
// lanes, all lanes active): lane l tests off[l+1] <= item and the ballot counts them
__device__ __forceinline__ int req_of_uniform(const long long* off, int n, long long item) {
  const int lane = threadIdx.x & 63;
  const long long nxt = lane < n ? off[lane + 1] : 0x7fffffffffffffffLL;
  return __popcll(__ballot(nxt <= item));
}

// the same for a per-lane item (binary search)
__device__ __forceinline__ int req_of(const long long* off, int n, long long item) {
  int lo = 0, hi = n;   // off[lo] <= item < off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= item) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void kb_pose(const BatchDesc* bd) {
  const int n = bd->n_req;
  const long long* off = bd->off[BK_POSE];
  const long long it = (long long)blockIdx.x * 256 + threadIdx.x;
  if (it >= off[n]) return;
  const int j = req_of(off, n, it);
  const BatchReq& q = bd->req[j];
  pose_item<double>(q.sc.bodies, q.T, q.dt, int(it - off[j]), (double2*)q.pose);
}

template <int CLS>
__global__ __launch_bounds__(256) void kb_geom(const BatchDesc* bd) {
  const int n = bd->n_req;
  const long long* off = bd->off[BK_GEOM + CLS];
  const long long w = __builtin_amdgcn_readfirstlane(int(blockIdx.x) * 4 + int(threadIdx.x >> 6));
  if (w >= off[n]) return;
  const int j = __builtin_amdgcn_readfirstlane(req_of_uniform(off, n, w));
  const BatchReq& q = bd->req[j];
  geom_wave<double, GEOM_ANCHOR_MFMA, DRT_SPLIT, CLS>(q.sc, q.rc.order[CLS], q.rc.count[CLS], (const double2*)q.pose,
                                                      q.T, q.dt, q.f_c, q.n_rays, q.nchunk, ExtrapOut{}, q.rec, q.ap,
                                                      int(w - off[j]), int(threadIdx.x & 63));
}

template <int MT, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MT * NT <= 8 ? 4 : 1)))
void kb_cfr16(const BatchDesc* bd) {
  __shared__ floatx4 red[3][64][MT * NT];
  const int n = bd->n_req;
  const long long* off = bd->off[BK_CFR + (NT == 1 ? 0 : (NT == 2 ? 1 : (MT == 1 ? 2 : (MT == 2 ? 3 : 4))))];
  const long long it = blockIdx.x;
  if (it >= off[n]) return;
  const int j = __builtin_amdgcn_readfirstlane(req_of_uniform(off, n, it));
  const BatchReq& q = bd->req[j];
  const CfrArgs a = q.a;
  cfr16_tile<MT, NT>((const RecM*)q.rec, a, a.G > 1 ? q.part : q.H, int(it - off[j]), red);
}

__global__ __launch_bounds__(256) void kb_reduce(const BatchDesc* bd) {
  const int n = bd->n_req;
  const long long* off = bd->off[BK_REDUCE];
  const long long it = (long long)blockIdx.x * 256 + threadIdx.x;
  if (it >= off[n]) return;
  const int j = req_of(off, n, it);
  const BatchReq& q = bd->req[j];
  reduce_item<float2>((const float2*)q.part, q.a.G, size_t(q.T) * q.a.K, (float2*)q.H, size_t(it - off[j]));
}

void batch_items(const BatchReq& q, long long items[BK_COUNT]) {
  for (int k = 0; k < BK_COUNT; ++k) items[k] = 0;
  items[BK_POSE] = (long long)q.sc.n_bodies * q.T;
  for (int c = 0; c < CLS_COUNT; ++c) items[BK_GEOM + c] = (long long)((q.rc.count[c] + 3) / 4) * 4 * q.nchunk;
  items[BK_CFR + cfr_shape(q.a.MT, q.a.NT)] = q.a.n_blocks;
  if (q.a.G > 1) items[BK_REDUCE] = (long long)q.T * q.a.K;
}

long long batch_grid(int kind, long long items) {
  if (items <= 0) return 1;
  if (kind == BK_POSE || kind == BK_REDUCE) return (items + 255) / 256;   // a thread per item
  if (kind < BK_CFR) return (items + 3) / 4;                              // a wave per item
  return items;                                                           // a workgroup per item
}

void* batch_kernel(int kind) {
  switch (kind) {
    case BK_POSE: return (void*)kb_pose;
    case BK_GEOM + CLS_R: return (void*)kb_geom<CLS_R>;
    case BK_GEOM + CLS_D: return (void*)kb_geom<CLS_D>;
    case BK_GEOM + CLS_S: return (void*)kb_geom<CLS_S>;
    case BK_CFR + 0: return (void*)kb_cfr16<1, 1>;
    case BK_CFR + 1: return (void*)kb_cfr16<1, 2>;
    case BK_CFR + 2: return (void*)kb_cfr16<1, 4>;
    case BK_CFR + 3: return (void*)kb_cfr16<2, 4>;
    case BK_CFR + 4: return (void*)kb_cfr16<4, 4>;
    case BK_REDUCE: return (void*)kb_reduce;
    default: return nullptr;
  }
}

hipError_t launch_batch(int kind, const BatchDesc* d, int grid, hipStream_t st) {
  dim3 g(grid), b(256);
  switch (kind) {
    case BK_POSE: hipLaunchKernelGGL(kb_pose, g, b, 0, st, d); break;
    case BK_GEOM + CLS_R: hipLaunchKernelGGL(kb_geom<CLS_R>, g, b, 0, st, d); break;
    case BK_GEOM + CLS_D: hipLaunchKernelGGL(kb_geom<CLS_D>, g, b, 0, st, d); break;
    case BK_GEOM + CLS_S: hipLaunchKernelGGL(kb_geom<CLS_S>, g, b, 0, st, d); break;
    case BK_CFR + 0: hipLaunchKernelGGL((kb_cfr16<1, 1>), g, b, 0, st, d); break;
    case BK_CFR + 1: hipLaunchKernelGGL((kb_cfr16<1, 2>), g, b, 0, st, d); break;
    case BK_CFR + 2: hipLaunchKernelGGL((kb_cfr16<1, 4>), g, b, 0, st, d); break;
    case BK_CFR + 3: hipLaunchKernelGGL((kb_cfr16<2, 4>), g, b, 0, st, d); break;
    case BK_CFR + 4: hipLaunchKernelGGL((kb_cfr16<4, 4>), g, b, 0, st, d); break;
    case BK_REDUCE: hipLaunchKernelGGL(kb_reduce, g, b, 0, st, d); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// host-side launchers

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
  size_t per = prec == DRT_FP64 ? sizeof(RecD)
                                : (prec == DRT_SPLIT ? std::max(sizeof(RecS), sizeof(RecM)) : sizeof(RecN));
  return size_t((T + 63) / 64) * n_rays * 64 * per;
}

template <class F, int MODE, int PREC, bool POL>
static void launch_classes(const SceneView& sc, const RayClasses& rc, const void* pose, int T, double dt,
                           double f_c, int n_rays, const ExtrapOut& eo, void* rec, const AnchorParams& ap,
                           hipStream_t st) {
  using P = const typename Vec2<F>::type*;
  int nchunk = (T + 63) / 64;
  for (int c = 0; c < CLS_COUNT; ++c) {
    if (rc.count[c] == 0) continue;
    dim3 grid(unsigned(long((rc.count[c] + 3) / 4) * nchunk));   // 4 rays x 64 instants per workgroup
    if (c == CLS_R)
      hipLaunchKernelGGL((k_geom<F, MODE, PREC, CLS_R, POL>), grid, dim3(256), 0, st, sc, rc.order[c], rc.count[c],
                         (P)pose, T, dt, f_c, n_rays, nchunk, eo, rec, ap);
    else if (c == CLS_D)
      hipLaunchKernelGGL((k_geom<F, MODE, PREC, CLS_D, POL>), grid, dim3(256), 0, st, sc, rc.order[c], rc.count[c],
                         (P)pose, T, dt, f_c, n_rays, nchunk, eo, rec, ap);
    else
      hipLaunchKernelGGL((k_geom<F, MODE, PREC, CLS_S, POL>), grid, dim3(256), 0, st, sc, rc.order[c], rc.count[c],
                         (P)pose, T, dt, f_c, n_rays, nchunk, eo, rec, ap);
  }
}

// The precision instances of one mode; POL: polarimetric field coefficients (dipoles),
// available in binary64 and split precision.
template <int MODE, bool POL>
static void launch_geom_prec(const SceneView& sc, const RayClasses& rc, const void* pose, int T, double dt,
                             double f_c, int n_rays, int prec, const ExtrapOut& eo, void* rec,
                             const AnchorParams& ap, hipStream_t st) {
  if constexpr (MODE == GEOM_ANCHOR_MFMA) {
    launch_classes<double, MODE, DRT_SPLIT, POL>(sc, rc, pose, T, dt, f_c, n_rays, eo, rec, ap, st);
  } else if constexpr (MODE == GEOM_NUFFT) {
    launch_classes<double, MODE, DRT_FP64, POL>(sc, rc, pose, T, dt, f_c, n_rays, eo, rec, ap, st);
  } else if constexpr (MODE == GEOM_KIN) {
    (void)prec;   // jets in binary64 whatever the call's precision (binary64 pose table); no field
    launch_classes<double, MODE, DRT_FP64, false>(sc, rc, pose, T, dt, f_c, n_rays, eo, rec, ap, st);
  } else {
    if (prec == DRT_FP64)
      launch_classes<double, MODE, DRT_FP64, POL>(sc, rc, pose, T, dt, f_c, n_rays, eo, rec, ap, st);
    else if (prec == DRT_SPLIT)
      launch_classes<double, MODE, DRT_SPLIT, POL>(sc, rc, pose, T, dt, f_c, n_rays, eo, rec, ap, st);
    else if constexpr (!POL)
      launch_classes<float, MODE, DRT_NAIVE32, false>(sc, rc, pose, T, dt, f_c, n_rays, eo, rec, ap, st);
  }
}

template <int MODE>
static hipError_t launch_geom_mode(const SceneView& sc, const RayClasses& rc, const void* pose, int T, double dt,
                                   double f_c, int n_rays, int prec, const ExtrapOut& eo, void* rec,
                                   const AnchorParams& ap, hipStream_t st) {
  if (sc.polar && MODE != GEOM_KIN) {
    if (prec == DRT_NAIVE32 && MODE != GEOM_ANCHOR_MFMA && MODE != GEOM_NUFFT) return hipErrorInvalidValue;
    launch_geom_prec<MODE, true>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  } else {
    launch_geom_prec<MODE, false>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  }
  return hipGetLastError();
}

hipError_t launch_geom(const SceneView& sc, const RayClasses& rc, const void* pose, int T, double dt, double f_c,
                       int n_rays, int prec, int mode, const ExtrapOut& eo, void* rec, const AnchorParams& ap,
                       hipStream_t st) {
  if (n_rays == 0 || T == 0) return hipSuccess;
  if (mode == GEOM_EXTRAP)
    return launch_geom_mode<GEOM_EXTRAP>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  if (mode == GEOM_ANCHOR_MFMA)
    return launch_geom_mode<GEOM_ANCHOR_MFMA>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  if (mode == GEOM_KIN)
    return launch_geom_mode<GEOM_KIN>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  if (mode == GEOM_POWER)
    return launch_geom_mode<GEOM_POWER>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  if (mode == GEOM_NUFFT)
    return launch_geom_mode<GEOM_NUFFT>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  return launch_geom_mode<GEOM_ANCHOR>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
}

CfrArgs plan_cfr(int n_rays, int T, int K, double f0, double df, int target_waves, int prec, int split_path) {
  CfrArgs a{};
  a.n_rays = n_rays;
  a.T = T;
  a.K = K;
  a.f0 = f0;
  a.df = df;
  a.path = CFR_VALU;
  if (prec == DRT_SPLIT && K <= 2048 && split_path != CFR_VALU) {
    a.path = split_path;
    a.NT = K <= 64 ? 1 : (K <= 256 ? 2 : 4);
    a.B = 8 * a.NT;
    a.K1 = (K + a.B - 1) / a.B;
    a.MT = (a.K1 + 15) / 16;
    if (a.MT == 3) a.MT = 4;
    long tiles = T;
    int G = int((target_waves + 4 * tiles - 1) / (4 * tiles));
    int maxG = (n_rays + 4 * kMinSlice - 1) / (4 * kMinSlice);
    if (G > maxG) G = maxG;
    if (G < 1) G = 1;
    a.G = G;
    a.slice_len = (n_rays + 4 * G - 1) / (4 * G);
    const int gran = a.path == CFR_MFMA16 ? 16 : 2;   // rays per matrix instruction
    a.slice_len = (a.slice_len + gran - 1) / gran * gran;
    a.n_blocks = int(tiles * G);
    return a;
  }
  const int nk = nk_of(prec);
  int blocks_k = (K + nk - 1) / nk;     // subcarrier blocks of nk
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
