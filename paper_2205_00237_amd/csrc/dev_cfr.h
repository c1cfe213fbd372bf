// Device side of the ray sum H[t][k] = sum_r a_r(t) exp(-j 2 pi f_k L_r(t)/c)
//
//   k_cfr         each lane owns one instant and NK consecutive subcarriers, reduces the
//                 carrier phase of its first subcarrier modulo one cycle and walks the
//                 others with the unit phasor exp(-j 2 pi df L/c); the 4 waves of a
//                 workgroup own 4 ray slices of one (instant, subcarrier) tile, summed in LDS
//   k_cfr_mfma*   the same sum factorised into complex GEMMs per instant on the matrix cores
//   k_reduce      deterministic sum of the per-slice-group partial tiles
#ifndef DRT_DEV_CFR_H
#define DRT_DEV_CFR_H

#include <hip/hip_runtime.h>

#include "drt_geom.h"
#include "drt_kernels.h"
#include "drt_records.h"

namespace drt {
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

typedef double doublex4 __attribute__((ext_vector_type(4)));

// sin(2 pi x) and cos(2 pi x) in binary64 for |x| < 2^30 cycles.  x is reduced exactly to
// r = x - q/4 with q the nearest quarter turn (|r| <= 1/8), the Taylor series of sin and cos
// at theta = 2 pi r (|theta| <= pi/4) are summed through theta^15 and theta^16 (the first
// terms left out are below 5e-17), and the pair is turned by q quarter turns.
__device__ __forceinline__ void sincos_rev64(double x, double& s, double& c) {
  const double q = __builtin_rint(4.0 * x);
  const double th = __builtin_fma(q, -0.25, x) * 6.283185307179586;
  const double t2 = th * th;
  double ps = -7.647163731819816e-13;                   // -1/15!
  ps = __builtin_fma(ps, t2, 1.6059043836821613e-10);   //  1/13!
  ps = __builtin_fma(ps, t2, -2.505210838544172e-08);   // -1/11!
  ps = __builtin_fma(ps, t2, 2.7557319223985893e-06);   //  1/9!
  ps = __builtin_fma(ps, t2, -1.984126984126984e-04);   // -1/7!
  ps = __builtin_fma(ps, t2, 8.333333333333333e-03);    //  1/5!
  ps = __builtin_fma(ps, t2, -1.6666666666666666e-01);  // -1/3!
  const double sn = __builtin_fma(ps * t2, th, th);
  double pc = 4.779477332387385e-14;                    //  1/16!
  pc = __builtin_fma(pc, t2, -1.1470745597729725e-11);  // -1/14!
  pc = __builtin_fma(pc, t2, 2.08767569878681e-09);     //  1/12!
  pc = __builtin_fma(pc, t2, -2.755731922398589e-07);   // -1/10!
  pc = __builtin_fma(pc, t2, 2.48015873015873e-05);     //  1/8!
  pc = __builtin_fma(pc, t2, -1.388888888888889e-03);   // -1/6!
  pc = __builtin_fma(pc, t2, 4.1666666666666664e-02);   //  1/4!
  pc = __builtin_fma(pc, t2, -0.5);
  const double cs = __builtin_fma(pc, t2, 1.0);
  const int iq = int(q) & 3;
  const double s0 = (iq & 1) ? cs : sn, c0 = (iq & 1) ? sn : cs;
  s = (iq & 2) ? -s0 : s0;
  c = ((iq + 1) & 2) ? -c0 : c0;
}

// Binary64 ray sum with the split path's structure: the same factorisation
// H[k1 B + k2] = sum_r U[k1][r] V[r][k2] per instant, as real GEMMs on the binary64 matrix
// cores (v_mfma_f64_16x16x4_f64: two rays x (re, im) per instruction, lane l supplies
// A[row l%16][slot l/16] and B[slot l/16][column l%16] as the binary32 instruction, but owns
// accumulator rows l/16 + 4v, v = 0..3, of column l%16).  Per ray pair a lane forms its
// U row values by a binary64 sincos each (phase p0 + frac(m phiB) + mt frac(16 phiB)) and its
// V column values V(0) = exp(-j 2 pi frac(m phi1)) by one sincos and the next column tiles
// by the record's step exp(-j 2 pi frac(16 phi1)), so K/B + B phasors per (ray, instant).
template <int MT, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void k_cfr_mfma64(const RecM64* rec, CfrArgs a, double* out) {
  constexpr int B = 8 * NT, NH = NT / 2;
  __shared__ doublex4 red[3][64][MT * NT];
  int bid = xcd_remap(blockIdx.x, gridDim.x);
  if (bid >= a.n_blocks) return;
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int g = bid % a.G, t = bid / a.G;
  int slice = g * 4 + wv;
  int r0 = slice * a.slice_len;
  int r1 = min(a.n_rays, r0 + a.slice_len);
  const int m = lane & 15, kslot = lane >> 4, rsel = kslot >> 1, part = kslot & 1;
  const RecM64* rt = rec + size_t(t) * a.n_rays;
  doublex4 acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  const int npair = r1 > r0 ? (r1 - r0 + 1) >> 1 : 0;
  // each lane reads its own ray of the pair (two records per wave, one cache line pair); the
  // next pair's record is in flight while the current one is consumed
  auto load = [&](int p) {
    const int r = r0 + 2 * p + rsel;
    return (p < npair && r < r1) ? rt[r] : RecM64{0.0, 0.0, 0.0, 0.0, 1.0, 0.0};
  };
  RecM64 cur = load(0);
#pragma unroll 1
  for (int p = 0; p < npair; ++p) {
    const RecM64 nxt = load(p + 1);
    const double u0 = cur.p0 + __builtin_amdgcn_fract(double(m) * cur.pB);
    const double u16 = __builtin_amdgcn_fract(16.0 * cur.pB);
    double av[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      double sn, c;
      sincos_rev64(mt == 0 ? u0 : u0 + double(mt) * u16, sn, c);
      av[mt] = part == 0 ? cur.amp * c : -(cur.amp * sn);               // Re / Im of |a| e^{-j 2 pi u}
    }
    double vs, vc;
    sincos_rev64(double(m) * cur.p1, vs, vc);
    double vre = vc, vim = -vs;                                         // V = e^{-j 2 pi k2 phi1}
    double bv[NT];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      bv[h] = part == 0 ? vre : -vim;         // C_re columns: V_re, -V_im
      bv[h + NH] = part == 0 ? vim : vre;     // C_im columns: V_im, V_re
      if (h + 1 < NH) {
        const double nr = vre * cur.fr - vim * cur.fi;
        vim = vre * cur.fi + vim * cur.fr;
        vre = nr;
      }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mt], bv[nt], acc[mt][nt], 0, 0, 0);
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
#pragma unroll 1
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] += red[w][lane][i * NT + j];
  double* dst = out + (a.G > 1 ? size_t(g) * a.T * a.K * 2 : 0) + size_t(t) * a.K * 2;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int k1 = mt * 16 + kslot + 4 * v;
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
// 8(l/16) .. 8(l/16)+7] = rays 4(l/16) .. 4(l/16)+3 of the block, and B likewise.
//
// Operands come from per-ray phasor tables instead of one sine and cosine each.  With the
// tile row or column m = 4a + b (0 <= a, b < 4),
//   U[16 mt + m] = UA[a] UB[b] RU^mt,  UA[a] = |a| e^{-j 2 pi (phi0 + 4 a phiB)},
//                                      UB[b] = e^{-j 2 pi b phiB},  RU = e^{-j 2 pi p16B},
//   V[16 h + m]  = VA[a] VB[b] RV^h,   VA[a] = e^{j 2 pi 4 a phi1},  VB[b] = e^{j 2 pi b phi1},
//                                      RV = e^{j 2 pi p16_1}
// (V is stored as its conjugate, the (cos, sin) pair the C_re columns take).  Each lane builds
// the tables of the ray it loaded (seven sine / cosine pairs, the rest products, the
// products 4 phiB and 4 phi1 reduced in binary64) into LDS, and the lanes of the block take
// one complex product per operand and one per further tile.
struct PhTab {
  float2 ua[4], ub[4], va[4], vb[4];
  float4 rot;      // RU, RV
};

template <bool NEG>
__device__ __forceinline__ float2 cis(float rev) {      // e^{-j 2 pi rev} if NEG, else e^{+j 2 pi rev}
  const float c = __builtin_amdgcn_cosf(rev), s = __builtin_amdgcn_sinf(rev);
  return float2{c, NEG ? -s : s};
}
__device__ __forceinline__ float2 cmul(float2 x, float2 y) {
  return float2{__builtin_fmaf(x.x, y.x, -(x.y * y.y)), __builtin_fmaf(x.x, y.y, x.y * y.x)};
}

template <bool ROT_U, bool ROT_V>
__device__ __forceinline__ void build_tab(const RecW& q, float kScale, PhTab& T) {
  const double phiB = __builtin_bit_cast(double, q.w[2]), phi1 = __builtin_bit_cast(double, q.w[3]);
  const float amp = __uint_as_float(uint32_t(q.w[0])) * kScale, phi0 = __uint_as_float(uint32_t(q.w[0] >> 32));
  const float pB = __uint_as_float(uint32_t(q.w[1])), p1 = __uint_as_float(uint32_t(q.w[1] >> 32));
  const float f4B = float(__builtin_amdgcn_fract(4.0 * phiB)), f41 = float(__builtin_amdgcn_fract(4.0 * phi1));
  const float2 b1 = cis<true>(float(phiB)), e4 = cis<true>(f4B);
  const float2 b2 = cmul(b1, b1), e8 = cmul(e4, e4);
  float2 a0 = cis<true>(phi0);
  a0 = float2{a0.x * amp, a0.y * amp};
  const float2 a1 = cmul(a0, e4);
  T.ua[0] = a0;
  T.ua[1] = a1;
  T.ua[2] = cmul(a0, e8);
  T.ua[3] = cmul(a1, e8);
  T.ub[0] = float2{1.f, 0.f};
  T.ub[1] = b1;
  T.ub[2] = b2;
  T.ub[3] = cmul(b2, b1);
  const float2 v1 = cis<false>(float(phi1)), f4 = cis<false>(f41);
  const float2 v2 = cmul(v1, v1), f8 = cmul(f4, f4);
  T.va[0] = float2{1.f, 0.f};
  T.va[1] = f4;
  T.va[2] = f8;
  T.va[3] = cmul(f8, f4);
  T.vb[0] = float2{1.f, 0.f};
  T.vb[1] = v1;
  T.vb[2] = v2;
  T.vb[3] = cmul(v2, v1);
  float2 ru{1.f, 0.f}, rv{1.f, 0.f};
  if constexpr (ROT_U) ru = cis<true>(pB);
  if constexpr (ROT_V) rv = cis<false>(p1);
  T.rot = float4{ru.x, ru.y, rv.x, rv.y};
}

// LDS of one workgroup of the binary16 ray sum: each wave's phasor tables of its current 64
// rays, and the partial tiles of waves 1-3 for the final sum.  Where the partial tiles fit
// in the tables' space they share it (the tables are dead once every wave has left its loop).
template <int MT, int NT> struct Cfr16Lds {
  static constexpr bool kShare = sizeof(floatx4) * 3 * 64 * MT * NT <= sizeof(PhTab) * 4 * 64;
  struct Split {
    PhTab tab[4][64];
    floatx4 red[3][64][MT * NT];
  };
  union Shared {
    PhTab tab[4][64];
    floatx4 red[3][64][MT * NT];
  };
  using type = typename std::conditional<kShare, Shared, Split>::type;
};

template <int MT, int NT>
__device__ __forceinline__ void cfr16_tile(const RecM* rec, const CfrArgs& a, float* out, int bid,
                                           typename Cfr16Lds<MT, NT>::type& lds) {
  constexpr int B = 8 * NT;
  constexpr bool ROT_U = MT > 1, ROT_V = (NT + 1) / 2 > 1;
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int g = bid % a.G, t = bid / a.G;
  int slice = g * 4 + wv;
  int r0 = slice * a.slice_len;
  int r1 = min(a.n_rays, r0 + a.slice_len);
  const int m = lane & 15, grp = lane >> 4;
  const int ta = NT == 1 ? (m >> 2) & 1 : m >> 2, tb = m & 3;    // table indices of row / column m
  const RecM* rt = rec + size_t(t) * a.n_rays;
  floatx4 acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const RecW* rw = reinterpret_cast<const RecW*>(rt);
  auto load = [&](int rb) {
    const int r = rb + lane;
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
  PhTab (&tab)[64] = lds.tab[wv];
  RecW cur = load(r0);
  for (int rb = r0; rb < r1; rb += 64) {
    // the wave's reads of the previous batch's tables were issued before these stores, and
    // one wave's LDS operations complete in order
    PhTab mine;
    build_tab<ROT_U, ROT_V>(cur, kScale, mine);      // rays past the slice have amplitude 0
    __builtin_amdgcn_wave_barrier();
    tab[lane] = mine;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    RecW nxt = load(rb + 64);
    const int nblk = min(4, (r1 - rb + 15) >> 4);
    static_for<0, 4>([&](auto BK) {
      constexpr int bk = decltype(BK)::value;
      if (bk >= nblk) return;
      // U operands of the 16 rays (lane: rays 4 grp .. 4 grp + 3 of the block) for every
      // row tile, and the first column tile's V, kept for the column-tile loop below
      u32x4 ahw[MT], alw[MT];
      float2 v0[4];
      static_for<0, 4>([&](auto J) {
        constexpr int j = decltype(J)::value;
        const PhTab& T = tab[16 * bk + 4 * grp + j];     // ray 16 bk + 4 grp + j of the batch
        float2 u = cmul(T.ua[ta], T.ub[tb]);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          if (mt > 0) {
            const float4 r = T.rot;
            u = cmul(u, float2{r.x, r.y});
          }
          Split16 w = split_pair<false>(u.x, u.y);
          ahw[mt][j] = w.hi;
          alw[mt][j] = w.lo;
        }
        v0[j] = cmul(T.va[ta], T.vb[tb]);
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
          if (hh > 0) {
            const float4 r = tab[16 * bk + 4 * grp + j].rot;
            v0[j] = cmul(v0[j], float2{r.z, r.w});
          }
          const float c = v0[j].x, sn = v0[j].y;
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
  if constexpr (Cfr16Lds<MT, NT>::kShare) __syncthreads();   // the tables die before the partial tiles land
  if (wv > 0) {
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) lds.red[wv - 1][lane][i * NT + j] = acc[i][j];
  }
  __syncthreads();
  if (wv != 0) return;
#pragma unroll 1
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] += lds.red[w][lane][i * NT + j];
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
  __shared__ typename Cfr16Lds<MT, NT>::type lds;
  int bid = xcd_remap(blockIdx.x, gridDim.x);
  if (bid < a.n_blocks) cfr16_tile<MT, NT>(rec, a, out, bid, lds);
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




}  // namespace drt

#endif  // DRT_DEV_CFR_H
