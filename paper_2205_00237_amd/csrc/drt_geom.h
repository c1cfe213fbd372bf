// Per-(ray, instant) DRT geometry and field coefficient, templated on the real type.
//
// Shared by the gfx950 kernels (one lane per (ray, instant)) and by the host loader's t0
// checks.  Everything is written in the global frame: a rigidly carried point is
// O(t) + R(t)(X0 - O0) with R(t) the rotation by theta(t) = w0*dt + wdot*dt^2/2 about the
// body's fixed axis (Sec. III-A.1; eq. coordinate_transf), which is algebraically the
// paper's local-frame procedure without the explicit change of frame.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "drt_layout.h"

namespace drt {

#define DRT_HD __host__ __device__ __forceinline__

// Square roots.  Device binary64: the library's own sequence (hardware reciprocal square
// root, one Goldschmidt step on the root and its half-reciprocal, two residual corrections)
// without its rescaling of inputs below 2^-767 and its special-value fix-up, so bitwise the
// library's root for every argument the geometry forms (squared lengths: zero or far above
// 2^-767).  Device binary32: the hardware root, within one ulp (the binary32 field
// coefficients are held to 1e-5 relative), not the correctly rounded library sequence.
// Host builds keep the library functions.
DRT_HD double msqrt(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = 0.5 * y;
  const double r = __builtin_fma(-h, s, 0.5);
  s = __builtin_fma(s, r, s);
  h = __builtin_fma(h, r, h);
  double d = __builtin_fma(-s, s, x);
  s = __builtin_fma(d, h, s);
  d = __builtin_fma(-s, s, x);
  s = __builtin_fma(d, h, s);
  return x == 0.0 ? x : s;
#else
  return ::sqrt(x);
#endif
}
DRT_HD float msqrt(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_sqrtf(x);
#else
  return ::sqrtf(x);
#endif
}
DRT_HD double mfloor(double x) { return ::floor(x); }
DRT_HD float mfloor(float x) { return ::floorf(x); }
DRT_HD double matan2(double y, double x) { return ::atan2(y, x); }
DRT_HD float matan2(float y, float x) { return ::atan2f(y, x); }
DRT_HD double mtan(double x) { return ::tan(x); }
DRT_HD float mtan(float x) { return ::tanf(x); }
DRT_HD double mcos(double x) { return ::cos(x); }
DRT_HD float mcos(float x) { return ::cosf(x); }
DRT_HD double msin(double x) { return ::sin(x); }
DRT_HD float msin(float x) { return ::sinf(x); }
DRT_HD double mrint(double x) { return ::rint(x); }
DRT_HD float mrint(float x) { return ::rintf(x); }
DRT_HD double mfabs(double x) { return ::fabs(x); }
DRT_HD float mfabs(float x) { return ::fabsf(x); }
DRT_HD bool mfinite(double x) { return isfinite(x); }
DRT_HD bool mfinite(float x) { return isfinite(x); }

// Reciprocal of the field type: binary32 field coefficients take the hardware's 1-ulp
// reciprocal (their tolerance is 1e-5 relative), binary64 the correctly rounded quotient.
template <class F> DRT_HD F frcp(F x) { return F(1) / x; }
template <> DRT_HD float frcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

// sin and cos of |x| <= 8.  Binary64: the library functions.  Binary32: x = q pi/2 + r
// with q = rint(2x/pi) and r = x - q pi/2 formed by two FMAs against pi/2 split in a
// binary32 head and tail (Cody-Waite), |r| <= pi/4; Taylor polynomials of sin r (through
// r^11) and cos r (through r^12), whose truncation is below 1e-11; quadrant from q mod 4.
// Keeps the relative accuracy of sin near 0 (r carries it) and has no large-argument path.
DRT_HD void sincos_small(double x, double& s, double& c) {
  s = ::sin(x);
  c = ::cos(x);
}
DRT_HD void sincos_small(float x, float& s, float& c) {
  const float q = ::rintf(x * 0.6366197466850281f);
  float r = ::fmaf(q, -1.5707963705062866f, x);
  r = ::fmaf(q, 4.371138828673793e-08f, r);
  const float r2 = r * r;
  float ps = -1.0f / 39916800.0f;
  ps = ::fmaf(ps, r2, 1.0f / 362880.0f);
  ps = ::fmaf(ps, r2, -1.0f / 5040.0f);
  ps = ::fmaf(ps, r2, 1.0f / 120.0f);
  ps = ::fmaf(ps, r2, -1.0f / 6.0f);
  const float sr = ::fmaf(ps * r2, r, r);
  float pc = 1.0f / 479001600.0f;
  pc = ::fmaf(pc, r2, -1.0f / 3628800.0f);
  pc = ::fmaf(pc, r2, 1.0f / 40320.0f);
  pc = ::fmaf(pc, r2, -1.0f / 720.0f);
  pc = ::fmaf(pc, r2, 1.0f / 24.0f);
  pc = ::fmaf(pc, r2, -0.5f);
  const float cr = ::fmaf(pc, r2, 1.0f);
  const int k = int(q) & 3;
  const float a = (k & 1) ? cr : sr, b = (k & 1) ? sr : cr;
  s = (k & 2) ? -a : a;              // sin(r + k pi/2)
  c = ((k + 1) & 2) ? -b : b;        // cos(r + k pi/2)
}

// Second-order jet in time (value, first and second time derivative) for the velocities
// and accelerations of the interaction points (eqs. ref_point_velo, ref_point_acc; App. B,
// C): the geometry templates run on it unchanged and differentiate themselves by the
// product, quotient and square-root rules; comparisons look at the value.
template <class F> struct J2 {
  F v, d, dd;
  J2() = default;
  DRT_HD J2(F x) : v(x), d(F(0)), dd(F(0)) {}
  DRT_HD J2(F x, F x1, F x2) : v(x), d(x1), dd(x2) {}
  friend DRT_HD J2 operator+(J2 a, J2 b) { return {a.v + b.v, a.d + b.d, a.dd + b.dd}; }
  friend DRT_HD J2 operator-(J2 a, J2 b) { return {a.v - b.v, a.d - b.d, a.dd - b.dd}; }
  friend DRT_HD J2 operator-(J2 a) { return {-a.v, -a.d, -a.dd}; }
  friend DRT_HD J2 operator*(J2 a, J2 b) {
    return {a.v * b.v, a.d * b.v + a.v * b.d, a.dd * b.v + F(2) * a.d * b.d + a.v * b.dd};
  }
  friend DRT_HD J2 operator/(J2 a, J2 b) {
    const F q = a.v / b.v, q1 = (a.d - q * b.d) / b.v;
    return {q, q1, (a.dd - F(2) * q1 * b.d - q * b.dd) / b.v};
  }
  friend DRT_HD bool operator<(J2 a, J2 b) { return a.v < b.v; }
  friend DRT_HD bool operator>(J2 a, J2 b) { return a.v > b.v; }
  friend DRT_HD bool operator<=(J2 a, J2 b) { return a.v <= b.v; }
  friend DRT_HD bool operator>=(J2 a, J2 b) { return a.v >= b.v; }
};
template <class F> DRT_HD J2<F> msqrt(J2<F> a) {
  const F r = msqrt(a.v), r1 = a.d / (F(2) * r);
  return {r, r1, (a.dd - F(2) * r1 * r1) / (F(2) * r)};
}
template <class F> DRT_HD bool mfinite(J2<F> a) { return mfinite(a.v) && mfinite(a.d) && mfinite(a.dd); }
template <class F> struct ScalarOf { using type = F; };
template <class F> struct ScalarOf<J2<F>> { using type = F; };

template <class F> struct V3 { F x, y, z; };
template <class F> DRT_HD V3<F> v3(F x, F y, F z) { return V3<F>{x, y, z}; }
template <class F> DRT_HD V3<F> ld3(const double* p) { return V3<F>{F(p[0]), F(p[1]), F(p[2])}; }
template <class F> DRT_HD V3<F> operator+(V3<F> a, V3<F> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class F> DRT_HD V3<F> operator-(V3<F> a, V3<F> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class F> DRT_HD V3<F> operator-(V3<F> a) { return {-a.x, -a.y, -a.z}; }
template <class F> DRT_HD V3<F> operator*(F s, V3<F> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class F> DRT_HD F dot(V3<F> a, V3<F> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class F> DRT_HD V3<F> cross(V3<F> a, V3<F> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class F> DRT_HD F norm(V3<F> a) { return msqrt(dot(a, a)); }

template <class F> struct Cx { F re, im; };
template <class F> DRT_HD Cx<F> cx(F r, F i) { return Cx<F>{r, i}; }
template <class F> DRT_HD Cx<F> operator+(Cx<F> a, Cx<F> b) { return {a.re + b.re, a.im + b.im}; }
template <class F> DRT_HD Cx<F> operator-(Cx<F> a, Cx<F> b) { return {a.re - b.re, a.im - b.im}; }
template <class F> DRT_HD Cx<F> operator*(Cx<F> a, Cx<F> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class F> DRT_HD Cx<F> operator*(F s, Cx<F> a) { return {s * a.re, s * a.im}; }
template <class F> DRT_HD Cx<F> cdiv(Cx<F> a, Cx<F> b) {
  F d = frcp(b.re * b.re + b.im * b.im);
  return {(a.re * b.re + a.im * b.im) * d, (a.im * b.re - a.re * b.im) * d};
}
// principal square root (non-negative real part)
template <class F> DRT_HD Cx<F> csqrt(Cx<F> w) {
  F r = msqrt(w.re * w.re + w.im * w.im);
  if (r == F(0)) return {F(0), F(0)};
  F t = msqrt((r + mfabs(w.re)) * F(0.5));
  F h = frcp(F(2) * t);
  if (w.re >= F(0)) return {t, w.im * h};
  return {mfabs(w.im) * h, w.im >= F(0) ? t : -t};
}

template <class F> struct Consts {
  static constexpr F pi = F(3.14159265358979323846);
  static constexpr F c0 = F(299792458.0);
};

// ---------------------------------------------------------------------------------------
// rigid-body pose of one body at one instant

template <class F> struct Pose {
  V3<F> O, O0, V, k;
  F W, s, c1;       // angular speed, sin(theta), 1 - cos(theta)
  bool moving;
};

template <class F>
DRT_HD Pose<F> make_pose(const DBody& b, F dt, F sin_th, F one_minus_cos) {
  Pose<F> p;
  p.O0 = ld3<F>(b.O0);
  p.k = ld3<F>(b.k);
  V3<F> v0 = ld3<F>(b.v0), a = ld3<F>(b.a);
  p.O = p.O0 + dt * v0 + (F(0.5) * dt * dt) * a;
  p.V = v0 + dt * a;
  p.W = F(b.w0) + F(b.wdot) * dt;
  p.s = sin_th;
  p.c1 = one_minus_cos;
  p.moving = b.moving != 0;
  return p;
}

template <class F> DRT_HD V3<F> rot(const Pose<F>& p, V3<F> v) {
  V3<F> kv = cross(p.k, v);
  return v + p.s * kv + p.c1 * cross(p.k, kv);
}
template <class F> DRT_HD V3<F> place(const Pose<F>& p, V3<F> x0) {
  return p.moving ? p.O + rot(p, x0 - p.O0) : x0;
}
template <class F> DRT_HD V3<F> carry(const Pose<F>& p, V3<F> d0) { return p.moving ? rot(p, d0) : d0; }
template <class F> DRT_HD V3<F> material_velocity(const Pose<F>& p, V3<F> x) {
  if (!p.moving) return v3<F>(0, 0, 0);
  return p.V + p.W * cross(p.k, x - p.O);
}

// ---------------------------------------------------------------------------------------
// one interaction slot moved to the instant

template <class F> struct Slot {
  V3<F> p, n;        // plane point / edge point / tile centroid; normal (plane, tile, 0-face)
  V3<F> e, t;        // edge direction, 0-face tangent
  Pose<F> pose;
};

template <class F> DRT_HD V3<F> mirror(V3<F> x, V3<F> p, V3<F> n) {
  return x - (F(2) * dot(x - p, n)) * n;
}

// Reflection points from src to dst over M walls w[0..M): images forward, then
// back-tracking from dst; ok &= every parameter s in (0, 1).
template <class F, int M>
DRT_HD void reflect_chain(V3<F> src, V3<F> dst, const Slot<F>* w, V3<F>* Q, bool& ok, bool& degen) {
  if constexpr (M > 0) {
    V3<F> A[M];
    V3<F> a = src;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      a = mirror(a, w[m].p, w[m].n);
      A[m] = a;
    }
    V3<F> nxt = dst;
#pragma unroll
    for (int m = M - 1; m >= 0; --m) {
      F num = dot(nxt - w[m].p, w[m].n);
      F den = dot(nxt - A[m], w[m].n);
      F s = num / den;
      bool fin = mfinite(s);
      degen = degen || !fin;
      ok = ok && fin && s > F(0) && s < F(1);
      if (!fin) s = F(0);
      Q[m] = nxt + s * (A[m] - nxt);
      nxt = Q[m];
    }
  }
}

constexpr double kRhoMin = 1e-9;    // diffraction source/receiver this close to the edge: degenerate
constexpr double kUtdEpsD = 1e-8;   // shadow-boundary switch of cot*F (|eps| formed in the geometry type)

template <class F> struct ChainOut {
  V3<F> Q[DRT_MAX_INT];
  V3<F> A, B;         // unfolded image source / receiver of the diffraction
  F rhoA, rhoB;
  F zQ;               // diffraction point along the edge from its reference point
  F zQ2;              // the second edge's point (two-edge chains)
  bool ok, degen;
};

constexpr int kDDIters = 16;        // Newton steps of the two-edge solve

// Points of the shortest path TX -> edge 1 -> edge 2 -> RX (the two-edge extension of
// Sec. III-B; Keller's law at both edges): Newton's method on (z1, z2) from each edge's
// single-edge point, halving a step while it lengthens the path beyond rounding (the length
// is convex in (z1, z2)).  Converged when both stationarity residuals are below tol.
template <class F>
DRT_HD void solve_two_edges(V3<F> TX, V3<F> RX, const Slot<F>& e1, const Slot<F>& e2, ChainOut<F>& c) {
  auto single = [&](const Slot<F>& ed) {
    const F zA = dot(TX - ed.p, ed.e), zB = dot(RX - ed.p, ed.e);
    const F rA = norm((TX - ed.p) - zA * ed.e), rB = norm((RX - ed.p) - zB * ed.e);
    const F z = zB + rB * (zA - zB) / (rA + rB);
    return mfinite(z) ? z : F(0);
  };
  auto length = [&](F a, F b) {
    const V3<F> Q1 = e1.p + a * e1.e, Q2 = e2.p + b * e2.e;
    return norm(Q1 - TX) + norm(Q2 - Q1) + norm(RX - Q2);
  };
  F z1 = single(e1), z2 = single(e2), f = length(z1, z2), g1 = F(1), g2 = F(1);
  const F up = F(1.0 + 1e-12);
  for (int it = 0; it < kDDIters; ++it) {
    const V3<F> Q1 = e1.p + z1 * e1.e, Q2 = e2.p + z2 * e2.e;
    const V3<F> d0 = Q1 - TX, d1 = Q2 - Q1, d2 = RX - Q2;
    const F l0 = norm(d0), l1 = norm(d1), l2 = norm(d2);
    const F c0 = dot(d0, e1.e) / l0, c1a = dot(d1, e1.e) / l1, c1b = dot(d1, e2.e) / l1, c2 = dot(d2, e2.e) / l2;
    g1 = c0 - c1a;
    g2 = c1b - c2;
    const F h11 = (F(1) - c0 * c0) / l0 + (F(1) - c1a * c1a) / l1;
    const F h22 = (F(1) - c1b * c1b) / l1 + (F(1) - c2 * c2) / l2;
    const F h12 = (c1a * c1b - dot(e1.e, e2.e)) / l1;
    const F det = h11 * h22 - h12 * h12;
    F s1 = (h12 * g2 - h22 * g1) / det, s2 = (h12 * g1 - h11 * g2) / det;
    if (!mfinite(s1) || !mfinite(s2)) {
      s1 = -g1;
      s2 = -g2;
    }
    F lam = F(1), fn = length(z1 + s1, z2 + s2);
    for (int h = 0; h < 40 && fn > f * up; ++h) {
      lam = F(0.5) * lam;
      fn = length(z1 + lam * s1, z2 + lam * s2);
    }
    z1 = z1 + lam * s1;
    z2 = z2 + lam * s2;
    f = fn;
  }
  const V3<F> Q1 = e1.p + z1 * e1.e, Q2 = e2.p + z2 * e2.e;
  {   // residuals at the final points
    const V3<F> d0 = Q1 - TX, d1 = Q2 - Q1, d2 = RX - Q2;
    g1 = dot(d0, e1.e) / norm(d0) - dot(d1, e1.e) / norm(d1);
    g2 = dot(d1, e2.e) / norm(d1) - dot(d2, e2.e) / norm(d2);
  }
  auto rho = [](V3<F> X, const Slot<F>& ed) {
    const V3<F> w = X - ed.p;
    return norm(w - dot(w, ed.e) * ed.e);
  };
  const bool far = rho(TX, e1) > F(kRhoMin) && rho(Q2, e1) > F(kRhoMin) && rho(Q1, e2) > F(kRhoMin) &&
                   rho(RX, e2) > F(kRhoMin);
  const F tol = F(sizeof(typename ScalarOf<F>::type) >= 8 ? 1e-12 : 1e-4);
  const bool conv = g1 < tol && g1 > -tol && g2 < tol && g2 > -tol;
  c.Q[0] = Q1;
  c.Q[1] = Q2;
  c.zQ = z1;
  c.zQ2 = z2;
  c.ok = far && conv;
  c.degen = !far;
}

// Interaction points of an N-interaction chain with its diffraction at slot DP (DP = -1:
// reflections only; DP = -2: two diffractions, slots 0 and 1).  Sec. III-A.2 (images and back-tracking), Sec. III-B (eq. diff_point).
template <class F, int N, int DP>
DRT_HD void solve_points(V3<F> TX, V3<F> RX, const Slot<F>* sl, ChainOut<F>& c) {
  c.ok = true;
  c.degen = false;
  if constexpr (DP == -2) {
    solve_two_edges<F>(TX, RX, sl[0], sl[1], c);
  } else if constexpr (DP < 0) {
    reflect_chain<F, N>(TX, RX, sl, c.Q, c.ok, c.degen);
  } else {
    V3<F> A = TX;
#pragma unroll
    for (int i = 0; i < DP; ++i) A = mirror(A, sl[i].p, sl[i].n);
    V3<F> B = RX;
#pragma unroll
    for (int i = N - 1; i > DP; --i) B = mirror(B, sl[i].p, sl[i].n);
    const Slot<F>& ed = sl[DP];
    F zA = dot(A - ed.p, ed.e), zB = dot(B - ed.p, ed.e);
    F rA = norm((A - ed.p) - zA * ed.e), rB = norm((B - ed.p) - zB * ed.e);
    F zQ = zB + rB * (zA - zB) / (rA + rB);
    if (!mfinite(zQ)) zQ = F(0);
    V3<F> QD = ed.p + zQ * ed.e;
    c.Q[DP] = QD;
    reflect_chain<F, DP>(TX, QD, sl, c.Q, c.ok, c.degen);
    reflect_chain<F, N - DP - 1>(QD, RX, sl + DP + 1, c.Q + DP + 1, c.ok, c.degen);
    bool far = rA > F(kRhoMin) && rB > F(kRhoMin);
    c.ok = c.ok && far;
    c.degen = c.degen || !far;
    c.A = A;
    c.B = B;
    c.rhoA = rA;
    c.rhoB = rB;
    c.zQ = zQ;
  }
}

// ---------------------------------------------------------------------------------------
// field coefficients (Fresnel, UTD, Effective Roughness)

template <class F>
DRT_HD Cx<F> fresnel(F cos_t, const DMat& m, F lam, int pol) {
  if (m.pec) return cx<F>(pol == DRT_PAR ? F(1) : F(-1), F(0));
  Cx<F> eps = cx<F>(F(m.eps_r), -F(60) * F(m.sigma) * lam);
  Cx<F> root = csqrt(cx<F>(eps.re - (F(1) - cos_t * cos_t), eps.im));
  if (pol == DRT_PAR) {
    Cx<F> ec = cos_t * eps;
    return cdiv(ec - root, ec + root);
  }
  return cdiv(cx<F>(cos_t, F(0)) - root, cx<F>(cos_t, F(0)) + root);
}

// UTD transition function F(X) = 2j sqrt(X) e^{jX} int_{sqrt X}^inf e^{-j tau^2} d tau.
// Small X: power series of the Fresnel integral from 0 to sqrt(X).  Larger X: the
// tail is (sqrt(pi)/2) e^{-j pi/4} erfc(e^{j pi/4} sqrt X) and the even continued fraction
// of erfc gives F(X) = jX / t with t = z2 + 1/2 - (1*2/4)/(z2 + 5/2 - (3*4/4)/(z2 + 9/2 ...)),
// z2 = jX, evaluated backwards from a fixed depth.
// Series below xs; above it the continued-fraction depth that reaches the type's precision
// shrinks quickly with X (binary64: 28 levels at X = 6, 3 beyond X = 1000).
template <class F> struct FxParams;
template <> struct FxParams<double> {
  static constexpr double xs = 6.0;
  static constexpr int ns = 40;
  static DRT_HD int depth(double X) {
    return X < 8 ? 28 : X < 12 ? 20 : X < 20 ? 14 : X < 40 ? 9 : X < 100 ? 6 : X < 1000 ? 4 : 3;
  }
};
template <> struct FxParams<float> {
  static constexpr float xs = 4.0f;
  static constexpr int ns = 22;
  static DRT_HD int depth(float X) { return X < 12.f ? 8 : X < 40.f ? 4 : 2; }
};

template <class F> DRT_HD Cx<F> utd_transition(F X) {
  if (X <= F(0)) return cx<F>(F(0), F(0));
  if (X < FxParams<F>::xs) {
    F x = msqrt(X);
    F term = x, sr = F(0), si = F(0);
    auto add = [&](int n, F v) {
      switch (n & 3) {         // (-j)^n
        case 0: sr += v; break;
        case 1: si -= v; break;
        case 2: sr -= v; break;
        default: si += v; break;
      }
    };
    if constexpr (sizeof(F) == 4) {
      // unrolled, so the divisions by 2n+1 and n+1 become products with constants
#pragma unroll
      for (int n = 0; n < FxParams<F>::ns; ++n) {
        add(n, term * (F(1) / F(2 * n + 1)));
        term = term * X * (F(1) / F(n + 1));
      }
    } else {
#pragma unroll 4
      for (int n = 0; n < FxParams<F>::ns; ++n) {
        add(n, term / F(2 * n + 1));
        term = term * X / F(n + 1);
      }
    }
    const F h = F(0.62665706865775012);      // sqrt(pi/8) = sqrt(pi)/2 * cos(pi/4)
    Cx<F> tail = cx<F>(h - sr, -h - si);     // sqrt(pi)/2 e^{-j pi/4} - S
    Cx<F> e;
    sincos_small(X, e.im, e.re);
    return (F(2) * x) * (cx<F>(F(0), F(1)) * (e * tail));
  }
  const int depth = FxParams<F>::depth(X);
  Cx<F> t = cx<F>(F(4 * depth + 1) * F(0.5), X);
  for (int n = depth; n >= 1; --n) {
    F c = F((2 * n - 1) * (2 * n)) * F(0.25);
    Cx<F> q = cdiv(cx<F>(c, F(0)), t);
    t = cx<F>(F(4 * n - 3) * F(0.5) - q.re, X - q.im);
  }
  return cdiv(cx<F>(F(0), X), t);
}

// cot((pi + sgn*beta)/(2n)) F(kL a^sgn(beta)) of the Kouyoumjian-Pathak coefficient.  With
// N the integer nearest (beta + sgn*pi)/(2 pi n) and eps = pi + sgn*(beta - 2 pi n N), the
// argument of the cotangent is pi N' + eps/(2n) and a^sgn(beta) = 2 cos^2((2 pi n N - beta)/2)
// = 2 sin^2(eps/2), so both are evaluated from eps (formed in the geometry type F) without
// the cancellation of the textbook form near a shadow or reflection boundary; below
// |eps| = 1e-8 the product is replaced by its small-eps limit.
template <class F, class G> DRT_HD Cx<G> cot_F(F beta, F sgn, F n, F inv_2pin, G kL) {
  const F pi = Consts<F>::pi;
  F N = mrint((beta + sgn * pi) * inv_2pin);
  F epsF = pi + sgn * beta - sgn * F(2) * pi * n * N;
  G eps = G(epsF), nn = G(n);
  if (mfabs(epsF) < F(kUtdEpsD)) {
    G sg = eps > G(0) ? G(1) : (eps < G(0) ? G(-1) : G(0));
    const G r2 = G(0.70710678118654752);
    Cx<G> w = cx<G>(r2, r2);                                // e^{j pi/4}
    Cx<G> inner = cx<G>(msqrt(G(2) * Consts<G>::pi * kL) * sg, G(0)) - (G(2) * kL * eps) * w;
    return nn * (inner * w);
  }
  G h, hc, st, ctn;
  sincos_small(eps * G(0.5), h, hc);                 // |eps| <= n pi <= 2 pi
  sincos_small(eps * frcp(G(2) * nn), st, ctn);      // |eps / 2n| <= pi / 2
  Cx<G> fx = utd_transition(kL * (G(2) * h * h));
  return (ctn * frcp(st)) * fx;
}

// Wedge angle of the edge-normal component u from the 0-face (tangent t towards normal n) in
// [0, 2 pi), except that an angle inside the wedge body within kFaceEps of 2 pi is a
// direction along the 0-face whose sign rounding decided (two edges of one face, a path
// along a roof): it is taken as the tiny negative angle, where the coefficient is
// continuous with the face.
constexpr double kFaceEps = 1e-5;
template <class F>
DRT_HD F utd_angle(const V3<F>& u, const Slot<F>& es, F wn) {
  const F two_pi = F(2) * Consts<F>::pi;
  F phi = matan2(dot(u, es.n), dot(u, es.t));
  if (phi < F(0)) phi += two_pi;
  if (phi > wn * Consts<F>::pi && phi > two_pi - F(kFaceEps)) phi -= two_pi;
  return phi;
}

// Kouyoumjian-Pathak coefficient of a perfectly conducting wedge (soft for pol 0, hard for 1);
// angles in the geometry type F, the rest in the field type G.
template <class F, class G>
DRT_HD Cx<G> utd_coefficient(F phi, F phi_p, G sin_b0, F n, G k, G Ld, int pol) {
  const G pi = Consts<G>::pi;
  F bm = phi - phi_p, bp = phi + phi_p;
  G kL = k * Ld;
  const F inv = F(1) / (F(2) * Consts<F>::pi * n);   // only picks the integer N
  Cx<G> tm = cot_F<F, G>(bm, F(1), n, inv, kL) + cot_F<F, G>(bm, F(-1), n, inv, kL);
  Cx<G> tp = cot_F<F, G>(bp, F(1), n, inv, kL) + cot_F<F, G>(bp, F(-1), n, inv, kL);
  Cx<G> sum = pol == DRT_PAR ? tm + tp : tm - tp;
  const G r2 = G(0.70710678118654752);
  G scale = frcp(G(2) * G(n) * msqrt(G(2) * pi * k) * sin_b0);
  Cx<G> pre = cx<G>(-r2 * scale, r2 * scale);                // -e^{-j pi/4} * scale
  return pre * sum;
}

// integral over the scattering hemisphere of ((1 + cos psi_R)/2)^alpha, integer alpha
template <class F> DRT_HD F er_norm_directive(int alpha, F cos_ti) {
  const F pi = Consts<F>::pi;
  F sin2 = F(1) - cos_ti * cos_ti;
  F total = F(0), binom = F(1);    // C(alpha, j)
  for (int j = 0; j <= alpha; ++j) {
    F Ij;
    if ((j & 1) == 0) {
      Ij = F(2) * pi / F(j + 1);
    } else {
      F acc = F(0), cw = F(1), pw = F(1);   // C(2w, w) / 4^w and sin2^w
      for (int w = 0; w <= (j - 1) / 2; ++w) {
        acc += cw * pw;
        cw = cw * F((2 * w + 1) * (2 * w + 2)) / F((w + 1) * (w + 1)) * F(0.25);
        pw *= sin2;
      }
      Ij = F(2) * pi / F(j + 1) * cos_ti * acc;
    }
    total += binom * Ij;
    binom = binom * F(alpha - j) / F(j + 1);
  }
  F scale = F(1);
  for (int j = 0; j < alpha; ++j) scale *= F(0.5);
  return total * scale;
}

// ---------------------------------------------------------------------------------------
// the whole per-(ray, instant) evaluation

template <class F, class G = F> struct RayResult {
  F L, dop;
  G aod_az, aod_el, aoa_az, aoa_el;
  Cx<G> gain;
  bool ok, degen;
  bool in_bounds;            // validity monitor (with MON)
  V3<F> Q[DRT_MAX_INT];      // interaction points (used by the loader's t0 checks)
};

template <class F> DRT_HD void dir_angles(V3<F> v, F& az, F& el) {
  az = matan2(v.y, v.x);
  el = matan2(v.z, msqrt(v.x * v.x + v.y * v.y));
}

// ---------------------------------------------------------------------------------------
// polarimetric coefficients with half-wave dipoles (vector form of the interactions)

template <class G> struct CV3 { Cx<G> x, y, z; };
template <class G> DRT_HD CV3<G> cv3(Cx<G> s, V3<G> v) { return {v.x * s, v.y * s, v.z * s}; }
template <class G> DRT_HD CV3<G> operator+(CV3<G> a, CV3<G> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class G> DRT_HD Cx<G> cdot(CV3<G> a, V3<G> v) { return v.x * a.x + v.y * a.y + v.z * a.z; }
template <class G> DRT_HD V3<G> unit_or(V3<G> v, V3<G> alt) {
  const G n2 = dot(v, v);
  if (!(n2 > G(1e-24))) { v = alt; }
  return frcp(norm(v)) * v;
}

// Vector pattern of a half-wave dipole along the unit p towards the unit direction k:
// sqrt(1.64) cos((pi/2) cos theta) / sin theta times theta_hat = ((p.k) k - p) / sin theta,
// evaluated as sin((pi/2) s^2 / (1 + |c|)) / s^2 times (c k - p) (no cancellation near the
// axis, where it vanishes with s).
template <class G> DRT_HD V3<G> dipole_pattern(V3<G> p, V3<G> k) {
  const G c = dot(p, k);
  const V3<G> t = c * k - p;
  const G s2 = dot(t, t), ac = c < G(0) ? -c : c;
  const G x = s2 * frcp(G(1) + ac);
  G amp = Consts<G>::pi * G(0.5) * frcp(G(1) + ac);
  if (s2 > G(0)) {
    G sn, cs;
    sincos_small(Consts<G>::pi * G(0.5) * x, sn, cs);
    amp = sn * frcp(s2);
  }
  return (G(1.2806248474865698) * amp) * t;     // sqrt(1.64)
}

// Reflection dyadic: e_perp = k_in x n normalised, e_par = e_perp x k on each side;
// E -> G_perp (E.e_perp) e_perp + G_par (E.e_par_in) e_par_out.
template <class G>
DRT_HD CV3<G> reflect_field(CV3<G> E, V3<G> k_in, V3<G> k_out, V3<G> n, Cx<G> g_perp, Cx<G> g_par) {
  const G az = n.z < G(0) ? -n.z : n.z;
  const V3<G> alt = cross(n, az < G(0.9) ? V3<G>{G(0), G(0), G(1)} : V3<G>{G(1), G(0), G(0)});
  const V3<G> ep = unit_or(cross(k_in, n), alt);
  return cv3(g_perp * cdot(E, ep), ep) + cv3(g_par * cdot(E, cross(ep, k_in)), cross(ep, k_out));
}

// UTD dyadic: e_phi = e x s normalised, e_beta = s x e_phi on each side;
// E -> D_s (E.e_beta_in) e_beta_out + D_h (E.e_phi_in) e_phi_out.
template <class G>
DRT_HD CV3<G> diffract_field(CV3<G> E, V3<G> s_in, V3<G> s_out, V3<G> e, Cx<G> d_soft, Cx<G> d_hard) {
  const V3<G> pi_ = unit_or(cross(e, s_in), cross(e, V3<G>{G(1), G(0), G(0)}));
  const V3<G> po = unit_or(cross(e, s_out), cross(e, V3<G>{G(1), G(0), G(0)}));
  return cv3(d_soft * cdot(E, cross(s_in, pi_)), cross(s_out, po)) + cv3(d_hard * cdot(E, pi_), po);
}

// Evaluate one ray whose N interaction slots are already moved to the instant.  Geometry
// (points, length, Doppler) is computed in F; angles and the field coefficient in G.
// Template parameters fix the signature so that every array stays in registers; the
// interaction points are copied out only with KEEP_Q (the loader's t0 checks), since the
// copy would otherwise survive in private memory behind the signature dispatch.  With MON
// the validity monitor is evaluated too: every reflection point inside its wall's facet
// (tested in the wall body's t0 frame, where the facet is fixed) with both neighbouring
// vertices on the front side, and every diffraction point on its edge segment.
// pose_of(i) gives the pose of slot i for the Doppler and the monitor: the slot's own copy,
// or (on the device) one rebuilt from the instant and the pose table, so that the poses of
// every slot need not stay in registers through the chain solve.
template <class F, class G, int N, int DP, bool SCAT, bool KEEP_Q = false, bool MON = false, bool POL = false,
          class PoseOf>
DRT_HD RayResult<F, G> eval_ray_with(const SceneView& sc, const DRay& ray, const Slot<F>* sl, V3<F> TX,
                                     V3<F> VTX, V3<F> RX, V3<F> VRX, F f_c, PoseOf&& pose_of) {
  RayResult<F, G> res;
  ChainOut<F> ch;
  if constexpr (SCAT) {
    ch.ok = true;
    ch.degen = false;
    ch.Q[0] = sl[0].p;
  } else {
    solve_points<F, N, DP>(TX, RX, sl, ch);
  }
  V3<F> verts[N + 2];
  verts[0] = TX;
#pragma unroll
  for (int i = 0; i < N; ++i) verts[i + 1] = ch.Q[i];
  verts[N + 1] = RX;
  V3<F> kh[N + 1], dv[N + 1];
  F len[N + 1];
  F L = F(0);
#pragma unroll
  for (int i = 0; i <= N; ++i) {
    dv[i] = verts[i + 1] - verts[i];
    len[i] = norm(dv[i]);
    kh[i] = (F(1) / len[i]) * dv[i];     // (only the Doppler, angles and scattering use it)
    L += len[i];
    ch.degen = ch.degen || !(len[i] > F(0));
  }
  // Doppler: f_D = -(f_c/c) sum_i k_i . (u_i - u_{i-1}), u the material velocities
  V3<F> uprev = VTX;
  F dLdt = F(0);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    V3<F> u = material_velocity(pose_of(i), ch.Q[i]);
    dLdt += dot(kh[i], u - uprev);
    uprev = u;
  }
  dLdt += dot(kh[N], VRX - uprev);
  res.dop = -(f_c / Consts<F>::c0) * dLdt;
  auto gv = [](V3<F> v) { return V3<G>{G(v.x), G(v.y), G(v.z)}; };
  dir_angles(gv(kh[0]), res.aod_az, res.aod_el);
  dir_angles(gv(-kh[N]), res.aoa_az, res.aoa_el);
  res.L = L;
  // validity monitor, evaluated while the points, vertices and poses are live and before
  // the field code needs the registers (a scattering chain's monitor is its facing test)
  bool in_bounds = true;
  if constexpr (MON && !SCAT) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (i == DP || DP == -2) {
        const DEdge& ed = sc.edges[ray.prim[i]];
        const F zq = (DP == -2 && i == 1) ? ch.zQ2 : ch.zQ;
        in_bounds = in_bounds && zq >= F(ed.zlo) && zq <= F(ed.zhi);
        continue;
      }
      const V3<F> q = ch.Q[i], nn = sl[i].n;
      in_bounds = in_bounds && dot(verts[i] - q, nn) >= F(0) && dot(verts[i + 2] - q, nn) >= F(0);
      const DPlane& pl = sc.planes[ray.prim[i]];
      if (pl.bounded) {
        // back to the t0 frame of the wall's body: X0 = O0 + R(-theta)(X - O(t))
        const Pose<F> ps = pose_of(i);
        V3<F> x0 = q;
        if (ps.moving) {
          V3<F> w = q - ps.O;
          V3<F> kw = cross(ps.k, w);
          x0 = ps.O0 + (w - ps.s * kw + ps.c1 * cross(ps.k, kw));
        }
        const V3<F> d = x0 - ld3<F>(pl.c0);
        const F su = dot(ld3<F>(pl.du), d), sv = dot(ld3<F>(pl.dv), d);
        in_bounds = in_bounds && su >= F(0) && su <= F(1) && sv >= F(0) && sv <= F(1);
      }
    }
  }

  const G pi = Consts<G>::pi;
  const G lam = G(Consts<F>::c0 / f_c);
  Cx<G> gam = cx<G>(G(1), G(0));
  // with dipoles: the transmitted pattern, carried through the reflections here (and the
  // diffraction below), is projected on the received pattern into gam
  CV3<G> E{};
  if constexpr (POL) {
    const V3<G> pt{G(sc.tx_ant[0]), G(sc.tx_ant[1]), G(sc.tx_ant[2])};
    const V3<G> e0 = dipole_pattern(pt, gv(kh[0]));
    E = CV3<G>{cx<G>(e0.x, G(0)), cx<G>(e0.y, G(0)), cx<G>(e0.z, G(0))};
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (SCAT || i == DP || DP == -2) continue;
    const DPlane& pl = sc.planes[ray.prim[i]];
    G ct = G(mfabs(dot(dv[i], sl[i].n))) * frcp(G(len[i]));
    if constexpr (POL) {
      if (DP >= 0 && i > DP) continue;     // after the edge: applied with the diffraction
      E = reflect_field(E, gv(kh[i]), gv(kh[i + 1]), gv(sl[i].n), fresnel<G>(ct, sc.mats[pl.mat], lam, DRT_PERP),
                        fresnel<G>(ct, sc.mats[pl.mat], lam, DRT_PAR));
    } else {
      gam = gam * fresnel<G>(ct, sc.mats[pl.mat], lam, ray.pol[i]);
    }
  }
  auto receive = [&](CV3<G> Ef) {
    const V3<G> pr{G(sc.rx_ant[0]), G(sc.rx_ant[1]), G(sc.rx_ant[2])};
    return cdot(Ef, dipole_pattern(pr, gv(-kh[N])));
  };
  if constexpr (POL && DP == -1) gam = receive(E);
  bool ok = ch.ok;
  Cx<G> a;
  if constexpr (SCAT) {
    const DTile& tl = sc.tiles[ray.prim[0]];
    V3<F> n = sl[0].n;
    F cti = -dot(kh[0], n), cts = dot(kh[1], n);
    ok = ok && cti > F(0) && cts > F(0);
    V3<F> spec = kh[0] - (F(2) * dot(kh[0], n)) * n;
    G cpsi = G(dot(spec, kh[1]));
    G amp;
    G ci = ok ? G(cti) : G(1), cs = ok ? G(cts) : G(1);
    if (tl.model == 0) {
      amp = G(tl.S) * msqrt(G(tl.area) * ci * cs / pi);
    } else {
      G x = (G(1) + cpsi) * G(0.5);
      if (x < G(0)) x = G(0);
      G lobe = G(1);
      for (int j = 0; j < tl.alpha / 2; ++j) lobe *= x;
      if (tl.alpha & 1) lobe *= msqrt(x);
      amp = G(tl.S) * msqrt(G(tl.area) * ci / er_norm_directive<G>(tl.alpha, ci)) * lobe;
    }
    G ph = G(tl.phase0);
    G sc_ = lam / (G(4) * pi) * amp * frcp(G(len[0]) * G(len[1]));
    G sp_, cp_;
    sincos_small(ph, sp_, cp_);     // tile phase in [0, 2 pi)
    a = cx<G>(sc_ * cp_, sc_ * sp_);
    if constexpr (POL) a = a * gam;   // the tile keeps the field: the two patterns' projection
  } else if constexpr (DP == -2) {
    // two edges: UTD for successive edges (non-slope).  The first edge's field reaches the
    // second as an astigmatic wave with a caustic on the first edge (radius s1) and one at
    // the source's distance s0 + s1; the Kouyoumjian-Pathak distance parameter of that wave
    // is s1 s2 sin^2 b / (s1 + s2) at the second edge (s0 s1 sin^2 b / (s0 + s1) at the
    // first), and the spreading is 1 / sqrt(s0 s1 s2 (s0 + s1 + s2)); exact for parallel
    // edges
    const G k = G(2) * pi / lam;
    const F Lsum = len[0] + len[1] + len[2];
    const F Lpar[2] = {len[0] * len[1] / (len[0] + len[1]), len[1] * len[2] / (len[1] + len[2])};
    Cx<G> Dprod = cx<G>(G(1), G(0));
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const DEdge& ed = sc.edges[ray.prim[j]];
      const Slot<F>& es = sl[j];
      const V3<F> Q = ch.Q[j], dA = verts[j] - Q, dB = verts[j + 2] - Q;
      const F cb = -dot(dA, es.e) / len[j];
      const F sb2 = F(1) - cb * cb;
      const F sb = msqrt(sb2 > F(0) ? sb2 : F(0));
      const V3<F> up = dA - dot(dA, es.e) * es.e, uo = dB - dot(dB, es.e) * es.e;
      const F phi_p = utd_angle(up, es, F(ed.wn)), phi = utd_angle(uo, es, F(ed.wn));
      const G Ld = G(Lpar[j] * sb * sb);
      if constexpr (POL) {
        E = diffract_field(E, gv(kh[j]), gv(kh[j + 1]), gv(es.e),
                           utd_coefficient<F, G>(phi, phi_p, G(sb), F(ed.wn), k, Ld, DRT_PERP),
                           utd_coefficient<F, G>(phi, phi_p, G(sb), F(ed.wn), k, Ld, DRT_PAR));
      } else {
        Dprod = Dprod * utd_coefficient<F, G>(phi, phi_p, G(sb), F(ed.wn), k, Ld, ray.pol[j]);
      }
    }
    const G scale = lam / (G(4) * pi) * frcp(msqrt(G(len[0] * len[1] * len[2] * Lsum)));
    if constexpr (POL) {
      a = scale * receive(E);
    } else {
      a = scale * Dprod;
    }
  } else if constexpr (DP >= 0) {
    const DEdge& ed = sc.edges[ray.prim[DP]];
    const Slot<F>& es = sl[DP];
    V3<F> QD = ch.Q[DP];
    V3<F> dA = ch.A - QD, dB = ch.B - QD;
    F sp = norm(dA), s = norm(dB);
    F cb = -dot(dA, es.e) / sp;
    F sb2 = F(1) - cb * cb;
    F sb = msqrt(sb2 > F(0) ? sb2 : F(0));
    V3<F> up = dA - dot(dA, es.e) * es.e;
    V3<F> uo = dB - dot(dB, es.e) * es.e;
    const F phi_p = utd_angle(up, es, F(ed.wn)), phi = utd_angle(uo, es, F(ed.wn));
    G Ld = G(s * sp * sb * sb) * frcp(G(s + sp));
    G k = G(2) * pi / lam;
    G scale = lam / (G(4) * pi) * frcp(msqrt(G(sp * s * (sp + s))));
    if constexpr (POL) {
      E = diffract_field(E, gv(kh[DP]), gv(kh[DP + 1]), gv(es.e),
                         utd_coefficient<F, G>(phi, phi_p, G(sb), F(ed.wn), k, Ld, DRT_PERP),
                         utd_coefficient<F, G>(phi, phi_p, G(sb), F(ed.wn), k, Ld, DRT_PAR));
#pragma unroll
      for (int i = DP + 1; i < N; ++i) {
        const DPlane& pl = sc.planes[ray.prim[i]];
        G ct = G(mfabs(dot(dv[i], sl[i].n))) * frcp(G(len[i]));
        E = reflect_field(E, gv(kh[i]), gv(kh[i + 1]), gv(sl[i].n),
                          fresnel<G>(ct, sc.mats[pl.mat], lam, DRT_PERP), fresnel<G>(ct, sc.mats[pl.mat], lam, DRT_PAR));
      }
      a = scale * receive(E);
    } else {
      Cx<G> D = utd_coefficient<F, G>(phi, phi_p, G(sb), F(ed.wn), k, Ld, ray.pol[DP]);
      a = scale * (gam * D);
    }
  } else {
    a = (lam * frcp(G(4) * pi * G(L))) * gam;
  }
  if (!ok) {
    res.L = res.dop = F(0);
    res.aod_az = res.aod_el = res.aoa_az = res.aoa_el = G(0);
    a = cx<G>(G(0), G(0));
  }
  res.gain = a;
  res.ok = ok;
  res.degen = ch.degen;
  res.in_bounds = ok && in_bounds;
  if constexpr (KEEP_Q) {
#pragma unroll
    for (int i = 0; i < N; ++i) res.Q[i] = ch.Q[i];
  }
  return res;
}

template <class F, class G, int N, int DP, bool SCAT, bool KEEP_Q = false, bool MON = false, bool POL = false>
DRT_HD RayResult<F, G> eval_ray(const SceneView& sc, const DRay& ray, const Slot<F>* sl, V3<F> TX,
                                V3<F> VTX, V3<F> RX, V3<F> VRX, F f_c) {
  return eval_ray_with<F, G, N, DP, SCAT, KEEP_Q, MON, POL>(sc, ray, sl, TX, VTX, RX, VRX, f_c,
                                                            [&](int i) { return sl[i].pose; });
}

// Interaction points and path length of one ray with its slots moved as jets in time:
// values, velocities and accelerations of the points, L, dL/dt and d2L/dt2.  ok as the
// chain's consistency in eval_ray (reflection parameters in (0, 1), diffraction source and
// receiver off the edge line); a scattering point is always consistent here.
template <class J> struct KinResult {
  V3<J> Q[DRT_MAX_INT];
  J L;
  bool ok;
};
template <class J, int N, int DP, bool SCAT>
DRT_HD KinResult<J> kin_ray(const Slot<J>* sl, V3<J> TX, V3<J> RX) {
  KinResult<J> res;
  ChainOut<J> ch;
  if constexpr (SCAT) {
    ch.ok = true;
    ch.degen = false;
    ch.Q[0] = sl[0].p;
  } else {
    solve_points<J, N, DP>(TX, RX, sl, ch);
  }
  V3<J> prev = TX;
  J L = J(0);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    L = L + norm(ch.Q[i] - prev);
    prev = ch.Q[i];
    res.Q[i] = ch.Q[i];
  }
  L = L + norm(RX - prev);
  res.L = L;
  res.ok = ch.ok && !ch.degen && mfinite(L);
  return res;
}

// Move interaction slot i of `ray` to the instant (poses already evaluated per slot).
template <class F>
DRT_HD void load_slot(const SceneView& sc, int kind, int prim, const Pose<F>& pose, Slot<F>& s) {
  s.pose = pose;
  if (kind == DRT_R) {
    const DPlane& p = sc.planes[prim];
    s.p = place(pose, ld3<F>(p.p0));
    s.n = carry(pose, ld3<F>(p.n0));
  } else if (kind == DRT_D) {
    const DEdge& e = sc.edges[prim];
    s.p = place(pose, ld3<F>(e.a0));
    s.e = carry(pose, ld3<F>(e.e0));
    s.t = carry(pose, ld3<F>(e.t0));
    s.n = carry(pose, ld3<F>(e.n0));
  } else {
    const DTile& t = sc.tiles[prim];
    s.p = place(pose, ld3<F>(t.c0));
    s.n = carry(pose, ld3<F>(t.n0));
  }
}

DRT_HD int prim_body(const SceneView& sc, int kind, int prim) {
  if (kind == DRT_R) return sc.planes[prim].body;
  if (kind == DRT_D) return sc.edges[prim].body;
  return sc.tiles[prim].body;
}

// Dispatch on the signature code within one class.
template <class F, int CLS, class Fn> DRT_HD auto with_signature_in(int code, Fn&& fn) {
  if constexpr (CLS == CLS_R) {
    switch (code) {
      case SIG_LOS: return fn.template operator()<0, -1, false>();
      case SIG_R1: return fn.template operator()<1, -1, false>();
      case SIG_R2: return fn.template operator()<2, -1, false>();
      case SIG_R3: return fn.template operator()<3, -1, false>();
      default: return fn.template operator()<4, -1, false>();
    }
  } else if constexpr (CLS == CLS_D) {
    switch (code) {
      case SIG_D: return fn.template operator()<1, 0, false>();
      case SIG_DR: return fn.template operator()<2, 0, false>();
      case SIG_RD: return fn.template operator()<2, 1, false>();
      case SIG_DRR: return fn.template operator()<3, 0, false>();
      case SIG_RDR: return fn.template operator()<3, 1, false>();
      case SIG_RRD: return fn.template operator()<3, 2, false>();
      case SIG_DRRR: return fn.template operator()<4, 0, false>();
      case SIG_RDRR: return fn.template operator()<4, 1, false>();
      case SIG_RRDR: return fn.template operator()<4, 2, false>();
      case SIG_DD: return fn.template operator()<2, -2, false>();
      default: return fn.template operator()<4, 3, false>();
    }
  } else {
    return fn.template operator()<1, -1, true>();
  }
}

// Dispatch on the signature code (DRay::code) to the matching template instance.
template <class F, class Fn> DRT_HD auto with_signature(int code, Fn&& fn) {
  switch (code) {
    case SIG_LOS: return fn.template operator()<0, -1, false>();
    case SIG_R1: return fn.template operator()<1, -1, false>();
    case SIG_R2: return fn.template operator()<2, -1, false>();
    case SIG_R3: return fn.template operator()<3, -1, false>();
    case SIG_R4: return fn.template operator()<4, -1, false>();
    case SIG_D: return fn.template operator()<1, 0, false>();
    case SIG_DR: return fn.template operator()<2, 0, false>();
    case SIG_RD: return fn.template operator()<2, 1, false>();
    case SIG_DRR: return fn.template operator()<3, 0, false>();
    case SIG_RDR: return fn.template operator()<3, 1, false>();
    case SIG_RRD: return fn.template operator()<3, 2, false>();
    case SIG_DRRR: return fn.template operator()<4, 0, false>();
    case SIG_RDRR: return fn.template operator()<4, 1, false>();
    case SIG_RRDR: return fn.template operator()<4, 2, false>();
    case SIG_RRRD: return fn.template operator()<4, 3, false>();
    case SIG_DD: return fn.template operator()<2, -2, false>();
    default: return fn.template operator()<1, -1, true>();
  }
}

}  // namespace drt
