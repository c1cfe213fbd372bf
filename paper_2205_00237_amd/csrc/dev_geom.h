// Device side of the per-(ray, instant) geometry: body poses and the geometry wave
//
//   k_pose    per (body, instant): sin(theta), 1 - cos(theta) of the body's rotation
//             angle theta = w0*dt + wdot*dt^2/2 (Sec. III-A.1)
//   k_geom    one lane per (ray, instant), one wave per (ray, 64 consecutive instants):
//             interaction points, length, Doppler, angles, field coefficient; writes the
//             caller's per-ray outputs or the per-(ray, instant) records of the ray sum
#ifndef DRT_DEV_GEOM_H
#define DRT_DEV_GEOM_H

#include <hip/hip_runtime.h>

#include "drt_geom.h"
#include "drt_kernels.h"
#include "drt_records.h"

namespace drt {

template <class F> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// ---------------------------------------------------------------------------------------

// (sin theta, 1 - cos theta) of body B at instant j.  Not inlined, so that the pose table
// and the geometry waves that compute a pose in place (small merged launches) run the same
// machine code and agree bit for bit.
template <class F>
__device__ __noinline__ typename Vec2<F>::type pose_value(const DBody& B, int j, double dt) {
  F d = F(double(j) * dt);
  F th = F(B.w0) * d + F(0.5) * F(B.wdot) * d * d;
  F h = msin(th * F(0.5));
  return {msin(th), F(2) * h * h};   // 1 - cos(theta) without cancellation
}

template <class F>
__device__ __forceinline__ void pose_item(const DBody* bodies, int T, double dt, int i,
                                          typename Vec2<F>::type* out) {
  int b = i / T, j = i - b * T;
  out[i] = pose_value<F>(bodies[b], j, dt);
}

// The pose of body b at instant j, from the table or computed in place.
template <class F, bool INLINE>
__device__ __forceinline__ typename Vec2<F>::type pose_at(const typename Vec2<F>::type* pose, const DBody* bodies,
                                                          int b, int T, int j, double dt) {
  if constexpr (INLINE) return pose_value<F>(bodies[b], j, dt);
  else return pose[b * T + j];
}

template <class F>
__global__ __launch_bounds__(256) void k_pose(const DBody* bodies, int nb, int T, double dt,
                                              typename Vec2<F>::type* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb * T) pose_item<F>(bodies, T, dt, i, out);
}

// ---------------------------------------------------------------------------------------


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

// Kind of slot i in the chains of signature (N, DP, SCAT): reflections, a diffraction at slot
// DP (at both slots for DP = -2), or one scattering tile.  The loader derives the signature
// code from the kinds, so this is the kind the ray record holds.
template <int N, int DP, bool SCAT> constexpr int slot_kind(int i) {
  return SCAT ? DRT_S : ((DP == -2 || i == DP) ? DRT_D : DRT_R);
}

// One wave: ray order[i] over the 64 instants of chunk c, where wave = 4 (nchunk (i / 4) + c) + i % 4.
template <class F, int MODE, int PREC, int CLS, bool POL = false, bool INLINE_POSE = false>
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
    const int nint = ray.nint;
    KinResult<J> kr = with_signature_in<J, CLS>(ray.code, [&]<int N, int DP, bool SCAT>() {
      // as below: slots of a fixed signature, loaded in straight-line code
      Slot<J> sj[N > 0 ? N : 1];
      typename Vec2<double>::type pe[N > 0 ? N : 1];
#pragma unroll
      for (int i = 0; i < N; ++i) pe[i] = pose[ray.body[i] * T + tq];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const DBody& B = sc.bodies[ray.body[i]];
        const double sn = double(pe[i].x), c1 = double(pe[i].y), cs = 1.0 - c1;
        const double w1 = B.w0 + B.wdot * tt, w2 = B.wdot;
        const J sth(sn, cs * w1, -sn * w1 * w1 + cs * w2), cth(c1, sn * w1, cs * w1 * w1 + sn * w2);
        load_slot<J>(sc, slot_kind<N, DP, SCAT>(i), ray.prim[i], make_pose<J>(B, tj, sth, cth), sj[i]);
      }
      return kin_ray<J, N, DP, SCAT>(sj, TXj, RXj);
    });
    const size_t o = size_t(r) * T + t;
    if (active && eo.dop_rate) eo.dop_rate[o] = kr.ok ? float(-(f_c / 299792458.0) * kr.L.dd) : 0.f;
    // One quantity's 12 values per lane are contiguous in [ray][instant][slot][xyz], so the
    // wave's 64 instants span 6 KB: staged in LDS and written as 16-byte pieces at consecutive
    // addresses, instead of one 24-byte run per lane with the lanes 96 bytes apart.
    constexpr int kPer = DRT_MAX_INT * 3;
    __shared__ double stage[4][64 * kPer];
    double* sw = stage[threadIdx.x >> 6];
    const int nd = max(0, min(64, T - chunk * 64)) * kPer;     // values of the active instants
    const size_t base = (size_t(r) * T + size_t(chunk) * 64) * kPer;
    auto put = [&](double* dst, int which) {
      if (!dst) return;
#pragma unroll
      for (int i = 0; i < DRT_MAX_INT; ++i) {
        const bool w = kr.ok && i < nint;
        const V3<J> q = kr.Q[i];
        const double x = which == 0 ? q.x.v : which == 1 ? q.x.d : q.x.dd;
        const double y = which == 0 ? q.y.v : which == 1 ? q.y.d : q.y.dd;
        const double z = which == 0 ? q.z.v : which == 1 ? q.z.d : q.z.dd;
        sw[lane * kPer + 3 * i] = w ? x : 0.0;
        sw[lane * kPer + 3 * i + 1] = w ? y : 0.0;
        sw[lane * kPer + 3 * i + 2] = w ? z : 0.0;
      }
      // one wave's LDS operations complete in order
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int c = 2 * lane; c < nd; c += 128)
        *reinterpret_cast<double2*>(dst + base + c) = *reinterpret_cast<const double2*>(sw + c);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    put(eo.q_pos, 0);
    put(eo.q_vel, 1);
    put(eo.q_acc, 2);
    return;
  }
  F dtj = F(double(tq) * dt);
  F half = F(0.5) * dtj * dtj;
  V3<F> TX = ld3<F>(sc.tx_p) + dtj * ld3<F>(sc.tx_v) + half * ld3<F>(sc.tx_a);
  V3<F> RX = ld3<F>(sc.rx_p) + dtj * ld3<F>(sc.rx_v) + half * ld3<F>(sc.rx_a);
  V3<F> VTX = ld3<F>(sc.tx_v) + dtj * ld3<F>(sc.tx_a);
  V3<F> VRX = ld3<F>(sc.rx_v) + dtj * ld3<F>(sc.rx_a);
  F fc = F(f_c);
  using G = typename GainT<PREC>::type;
  // a slot's pose rebuilt where the Doppler and the monitor need it, from the instant and the
  // pose table; the empty asm statements keep the compiler from reusing (and so holding
  // through the chain solve) the values computed when the slots were loaded.  They are not
  // volatile: a volatile one counts as a memory access, after which the scene tables are
  // read by vector loads instead of scalar ones, and it keeps the rebuild alive in the
  // record kernels, which never use the Doppler.
  auto pose_of = [&](int i) {
    F d = dtj;
    int j = tq;
    asm("" : "+v"(d), "+v"(j));
    const int b = ray.body[i];
    const auto pe = pose_at<F, INLINE_POSE>(pose, sc.bodies, b, T, j, dt);
    return make_pose<F>(sc.bodies[b], d, F(pe.x), F(pe.y));
  };
  RayResult<F, G> res = with_signature_in<F, CLS>(ray.code, [&]<int N, int DP, bool SCAT>() {
    // slots of a fixed signature: straight-line code, so that the loads of every slot (pose,
    // body, primitive) go out together before the first is used
    Slot<F> sl[N > 0 ? N : 1];
    typename Vec2<F>::type pe[N > 0 ? N : 1];
#pragma unroll
    for (int i = 0; i < N; ++i) pe[i] = pose_at<F, INLINE_POSE>(pose, sc.bodies, ray.body[i], T, tq, dt);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      Pose<F> ps = make_pose<F>(sc.bodies[ray.body[i]], dtj, F(pe[i].x), F(pe[i].y));
      load_slot<F>(sc, slot_kind<N, DP, SCAT>(i), ray.prim[i], ps, sl[i]);
    }
    return eval_ray_with<F, G, N, DP, SCAT, false, MODE == GEOM_EXTRAP || MODE == GEOM_POWER, POL>(
        sc, ray, sl, TX, VTX, RX, VRX, fc, pose_of);
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
  } else if constexpr (MODE == GEOM_ANCHOR_MFMA && PREC == DRT_FP64) {
    // binary64 matrix-core records: the same phases kept in binary64, and the column step
    // exp(-j 2 pi frac(16 df L/c)) of the subcarrier phasors
    if (!active) return;
    const size_t o = size_t(t) * n_rays + r;
    const double L = double(res.L), gr = double(res.gain.re), gi = double(res.gain.im);
    double p0 = L * ap.f0c - atan2(gi, gr) * (0.5 / M_PI), pB = L * ap.fBc, p1 = L * ap.f1c;
    p0 -= floor(p0);
    pB -= floor(pB);
    p1 -= floor(p1);
    double q16 = 16.0 * p1;
    q16 -= floor(q16);
    double fs, fc;
    sincospi(2.0 * q16, &fs, &fc);
    reinterpret_cast<RecM64*>(rec)[o] = {sqrt(gr * gr + gi * gi), p0, pB, p1, fc, -fs};
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

// Waves per SIMD each geometry kernel is compiled for (1: as many as its registers allow).
// Measured per class on the urban workload: the split ray-sum records of reflection chains
// gain from six waves (92 registers unconstrained), the split drt_extrapolate kernels from
// four and three (146 and 169 unconstrained), the power profiles' diffraction kernel from
// three, and the binary64 record kernels with a diffraction from four (158 unconstrained).
// The others measured the same or slower when squeezed and keep their natural allocation.
template <int MODE, int PREC, int CLS> constexpr int geom_waves() {
  if (CLS == CLS_S) return 1;
  if (MODE == GEOM_ANCHOR_MFMA && PREC == DRT_SPLIT && CLS == CLS_R) return 6;
  if (MODE == GEOM_EXTRAP && PREC == DRT_SPLIT) return CLS == CLS_R ? 4 : 3;
  if (MODE == GEOM_POWER && PREC == DRT_SPLIT && CLS == CLS_D) return 3;
  if ((MODE == GEOM_ANCHOR || MODE == GEOM_ANCHOR_MFMA) && PREC == DRT_FP64 && CLS == CLS_D) return 4;
  return 1;
}

template <class F, int MODE, int PREC, int CLS, bool POL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(geom_waves<MODE, PREC, CLS>()))) void k_geom(SceneView sc, const int32_t* order, int count,
                                              const typename Vec2<F>::type* pose, int T, double dt, double f_c,
                                              int n_rays, int nchunk, ExtrapOut eo, void* rec, AnchorParams ap) {
  int wave = __builtin_amdgcn_readfirstlane(int(blockIdx.x) * 4 + int(threadIdx.x >> 6));
  geom_wave<F, MODE, PREC, CLS, POL>(sc, order, count, pose, T, dt, f_c, n_rays, nchunk, eo, rec, ap, wave,
                                     int(threadIdx.x & 63));
}


// The geometry of every signature class in one launch (small calls of the ray-sum record
// modes): workgroups [0, wR) take the reflection class, then the diffraction class, then
// scattering; class boundaries fall on workgroups, so each workgroup runs one class's code.
// Poses are computed in place (pose_value), so such a call needs no pose-table kernel.
template <class F, int MODE, int PREC, bool POL>
__global__ __launch_bounds__(256) void k_geom_merged(SceneView sc, RayClasses rc, const typename Vec2<F>::type* pose,
                                                     int T, double dt, double f_c, int n_rays, int nchunk,
                                                     ExtrapOut eo, void* rec, AnchorParams ap) {
  const int wg = int(blockIdx.x), lane = int(threadIdx.x & 63);
  const int gR = class_workgroups(rc, CLS_R, T), gD = class_workgroups(rc, CLS_D, T);
  const int w = int(threadIdx.x >> 6);
  if (wg < gR) {
    geom_wave<F, MODE, PREC, CLS_R, POL, true>(sc, rc.order[CLS_R], rc.count[CLS_R], pose, T, dt, f_c, n_rays,
                                               nchunk, eo, rec, ap, __builtin_amdgcn_readfirstlane(wg * 4 + w), lane);
  } else if (wg < gR + gD) {
    geom_wave<F, MODE, PREC, CLS_D, POL, true>(sc, rc.order[CLS_D], rc.count[CLS_D], pose, T, dt, f_c, n_rays,
                                               nchunk, eo, rec, ap, __builtin_amdgcn_readfirstlane((wg - gR) * 4 + w), lane);
  } else {
    geom_wave<F, MODE, PREC, CLS_S, POL, true>(sc, rc.order[CLS_S], rc.count[CLS_S], pose, T, dt, f_c, n_rays,
                                               nchunk, eo, rec, ap, __builtin_amdgcn_readfirstlane((wg - gR - gD) * 4 + w), lane);
  }
}

}  // namespace drt

#endif  // DRT_DEV_GEOM_H
