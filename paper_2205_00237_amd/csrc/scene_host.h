// Host half of the scene loader: the error text of the last failed call, the by-value copy
// of a scene description, its validation and packing into the device tables (with the t0
// solve of every ray), and its carriage to another instant.  Plain C++ over the packed
// layout and the shared geometry header, so it also builds with a host compiler alone.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "drt_geom.h"
#include "drt_layout.h"

namespace drt_host {
using namespace drt;
// ---------------------------------------------------------------------------------------
// errors

static thread_local std::string g_last_error;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

// A scene description held by value (the arrays of drt_scene_desc), kept with each
// resident scene so that it can be carried to another instant and traced again.
struct HostDesc {
  double t0 = 0;
  double tx_p[3]{}, tx_v[3]{}, tx_a[3]{}, rx_p[3]{}, rx_v[3]{}, rx_a[3]{};
  int32_t nb = 0, nm = 0, np = 0, ne = 0, nt = 0, nr = 0;
  std::vector<double> body_O0, body_v0, body_a, body_axis, body_w0, body_wdot;
  std::vector<double> mat_eps_r, mat_sigma;
  std::vector<uint8_t> mat_pec;
  std::vector<int32_t> plane_body, plane_mat;
  std::vector<double> plane_p0, plane_n0, plane_facet;       // facet: empty = every wall unbounded
  std::vector<int32_t> edge_body;
  std::vector<double> edge_a0, edge_e0, edge_t0, edge_n0, edge_wedge_n, edge_zlim;   // zlim may be empty
  std::vector<int32_t> tile_body, tile_alpha;
  std::vector<uint8_t> tile_model;
  std::vector<double> tile_c0, tile_n0, tile_area, tile_S, tile_phase0;
  std::vector<uint8_t> ray_nint, ray_kind, ray_pol;
  std::vector<int32_t> ray_prim;
  std::vector<double> tx_ant, rx_ant;                    // [4] each, or empty
};

// The host side of one packed scene: its description by value, the packed tables and the
// rays of each signature class.  The runtime adds the device copies.
struct PackedScene {
  HostDesc desc;
  SceneView view{};
  std::vector<DBody> bodies;     // host copies of the packed tables
  std::vector<DMat> mats;
  std::vector<DPlane> planes;
  std::vector<DEdge> edges;
  std::vector<DTile> tiles;
  std::vector<DRay> rays;
  std::vector<int32_t> cls_rays[CLS_COUNT];   // ray indices of each signature class, ascending
  // the same lists stable-sorted by signature code: a call over every ray of the scene walks
  // each class signature by signature, so that neighbouring waves run the same code
  std::vector<int32_t> cls_by_sig[CLS_COUNT];
};

// ---------------------------------------------------------------------------------------
// loader

static bool unit(const double* v) {
  double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  return std::fabs(n - 1.0) < 1e-9;
}

template <class K> static int sig_code(int nint, const K* kind, int* dpos) {
  *dpos = 255;
  if (nint == 0) return SIG_LOS;
  if (kind[0] == DRT_S) return SIG_S;
  if (nint == 2 && kind[0] == DRT_D && kind[1] == DRT_D) return SIG_DD;
  int d = -1;
  for (int i = 0; i < nint; ++i)
    if (kind[i] == DRT_D) d = i;
  if (d < 0) return SIG_LOS + nint;
  *dpos = d;
  static const int base[5] = {0, SIG_D, SIG_DR, SIG_DRR, SIG_DRRR};
  return base[nint] + d;
}

template <int N, int DP, bool SCAT>
static RayResult<double> eval_host(const SceneView& sc, const DRay& ray, const Slot<double>* sl) {
  V3<double> TX = ld3<double>(sc.tx_p), RX = ld3<double>(sc.rx_p);
  V3<double> VTX = ld3<double>(sc.tx_v), VRX = ld3<double>(sc.rx_v);
  return eval_ray<double, double, N, DP, SCAT, true>(sc, ray, sl, TX, VTX, RX, VRX, 1e9);
}

static int validate_and_pack(const drt_scene_desc* d, PackedScene& s) {
  if (!d) return fail(DRT_E_INVAL, "null scene description");
  if (d->n_bodies < 1) return fail(DRT_E_INVAL, "n_bodies must be >= 1 (body 0 = static world)");
  if (d->n_mat < 0 || d->n_planes < 0 || d->n_edges < 0 || d->n_tiles < 0 || d->n_rays < 0)
    return fail(DRT_E_INVAL, "negative count");
#define NEED(ptr, cnt) \
  if ((cnt) > 0 && !(ptr)) return fail(DRT_E_INVAL, "%s is NULL with %d entries", #ptr, int(cnt));
  NEED(d->body_O0, d->n_bodies) NEED(d->body_v0, d->n_bodies) NEED(d->body_a, d->n_bodies)
  NEED(d->body_axis, d->n_bodies) NEED(d->body_w0, d->n_bodies) NEED(d->body_wdot, d->n_bodies)
  NEED(d->mat_eps_r, d->n_mat) NEED(d->mat_sigma, d->n_mat) NEED(d->mat_pec, d->n_mat)
  NEED(d->plane_body, d->n_planes) NEED(d->plane_mat, d->n_planes) NEED(d->plane_p0, d->n_planes)
  NEED(d->plane_n0, d->n_planes) NEED(d->edge_body, d->n_edges) NEED(d->edge_a0, d->n_edges)
  NEED(d->edge_e0, d->n_edges) NEED(d->edge_t0, d->n_edges) NEED(d->edge_n0, d->n_edges)
  NEED(d->edge_wedge_n, d->n_edges) NEED(d->tile_body, d->n_tiles) NEED(d->tile_alpha, d->n_tiles)
  NEED(d->tile_model, d->n_tiles) NEED(d->tile_c0, d->n_tiles) NEED(d->tile_n0, d->n_tiles)
  NEED(d->tile_area, d->n_tiles) NEED(d->tile_S, d->n_tiles) NEED(d->tile_phase0, d->n_tiles)
  NEED(d->ray_nint, d->n_rays) NEED(d->ray_kind, d->n_rays) NEED(d->ray_pol, d->n_rays)
  NEED(d->ray_prim, d->n_rays)
#undef NEED
  s.bodies.resize(d->n_bodies);
  for (int b = 0; b < d->n_bodies; ++b) {
    DBody& B = s.bodies[b];
    std::memset(&B, 0, sizeof B);
    std::memcpy(B.O0, d->body_O0 + 3 * b, 24);
    std::memcpy(B.v0, d->body_v0 + 3 * b, 24);
    std::memcpy(B.a, d->body_a + 3 * b, 24);
    std::memcpy(B.k, d->body_axis + 3 * b, 24);
    B.w0 = d->body_w0[b];
    B.wdot = d->body_wdot[b];
    if (!unit(B.k)) return fail(DRT_E_INVAL, "body %d: rotation axis is not a unit vector", b);
    bool mv = B.w0 != 0 || B.wdot != 0;
    for (int i = 0; i < 3; ++i) mv = mv || B.v0[i] != 0 || B.a[i] != 0;
    B.moving = mv ? 1 : 0;
  }
  std::vector<DMat>& mats = s.mats;
  mats.resize(d->n_mat);
  for (int m = 0; m < d->n_mat; ++m) {
    mats[m] = DMat{d->mat_eps_r[m], d->mat_sigma[m], d->mat_pec[m] ? 1 : 0, 0};
    if (!d->mat_pec[m] && !(d->mat_eps_r[m] > 0 && d->mat_sigma[m] >= 0))
      return fail(DRT_E_INVAL, "material %d: need eps_r > 0 and sigma >= 0", m);
  }
  std::vector<DPlane>& planes = s.planes;
  planes.resize(d->n_planes);
  for (int i = 0; i < d->n_planes; ++i) {
    DPlane& P = planes[i];
    std::memset(&P, 0, sizeof P);
    std::memcpy(P.p0, d->plane_p0 + 3 * i, 24);
    std::memcpy(P.n0, d->plane_n0 + 3 * i, 24);
    P.body = d->plane_body[i];
    P.mat = d->plane_mat[i];
    if (P.body < 0 || P.body >= d->n_bodies || P.mat < 0 || P.mat >= d->n_mat)
      return fail(DRT_E_INVAL, "plane %d: body or material index out of range", i);
    if (!unit(P.n0)) return fail(DRT_E_INVAL, "plane %d: normal is not a unit vector", i);
    if (d->plane_facet) {
      const double* f = d->plane_facet + 9 * i;   // corner, u, v
      const double *c = f, *u = f + 3, *v = f + 6;
      auto dt3 = [](const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
      const double uu = dt3(u, u), uv = dt3(u, v), vv = dt3(v, v);
      if (uu == 0 && vv == 0) continue;   // unbounded wall
      const double det = uu * vv - uv * uv;
      if (!(det > 1e-12 * uu * vv) || !std::isfinite(det))
        return fail(DRT_E_INVAL, "plane %d: facet sides are degenerate or parallel", i);
      if (std::fabs(dt3(u, P.n0)) > 1e-9 * std::sqrt(uu) || std::fabs(dt3(v, P.n0)) > 1e-9 * std::sqrt(vv))
        return fail(DRT_E_INVAL, "plane %d: facet sides are not in the plane", i);
      double cp[3] = {c[0] - P.p0[0], c[1] - P.p0[1], c[2] - P.p0[2]};
      if (std::fabs(dt3(cp, P.n0)) > 1e-9 * (1.0 + std::sqrt(dt3(cp, cp))))
        return fail(DRT_E_INVAL, "plane %d: facet corner is not in the plane", i);
      for (int k = 0; k < 3; ++k) {
        P.c0[k] = c[k];
        P.du[k] = (vv * u[k] - uv * v[k]) / det;
        P.dv[k] = (uu * v[k] - uv * u[k]) / det;
      }
      P.bounded = 1;
    }
  }
  std::vector<DEdge>& edges = s.edges;
  edges.resize(d->n_edges);
  for (int i = 0; i < d->n_edges; ++i) {
    DEdge& E = edges[i];
    std::memset(&E, 0, sizeof E);
    std::memcpy(E.a0, d->edge_a0 + 3 * i, 24);
    std::memcpy(E.e0, d->edge_e0 + 3 * i, 24);
    std::memcpy(E.t0, d->edge_t0 + 3 * i, 24);
    std::memcpy(E.n0, d->edge_n0 + 3 * i, 24);
    E.wn = d->edge_wedge_n[i];
    E.body = d->edge_body[i];
    if (E.body < 0 || E.body >= d->n_bodies) return fail(DRT_E_INVAL, "edge %d: body out of range", i);
    if (!unit(E.e0) || !unit(E.t0) || !unit(E.n0))
      return fail(DRT_E_INVAL, "edge %d: direction, tangent or normal is not a unit vector", i);
    if (!(E.wn > 0.5 && E.wn <= 2.0)) return fail(DRT_E_INVAL, "edge %d: wedge index n must be in (0.5, 2]", i);
    E.zlo = -INFINITY;
    E.zhi = INFINITY;
    if (d->edge_zlim) {
      E.zlo = d->edge_zlim[2 * i];
      E.zhi = d->edge_zlim[2 * i + 1];
      if (!(E.zlo <= E.zhi)) return fail(DRT_E_INVAL, "edge %d: segment limits need z_lo <= z_hi", i);
    }
  }
  std::vector<DTile>& tiles = s.tiles;
  tiles.resize(d->n_tiles);
  for (int i = 0; i < d->n_tiles; ++i) {
    DTile& T = tiles[i];
    std::memset(&T, 0, sizeof T);
    std::memcpy(T.c0, d->tile_c0 + 3 * i, 24);
    std::memcpy(T.n0, d->tile_n0 + 3 * i, 24);
    T.area = d->tile_area[i];
    T.S = d->tile_S[i];
    T.phase0 = d->tile_phase0[i];
    T.body = d->tile_body[i];
    T.alpha = d->tile_alpha[i];
    T.model = d->tile_model[i];
    if (T.body < 0 || T.body >= d->n_bodies) return fail(DRT_E_INVAL, "tile %d: body out of range", i);
    if (T.alpha < 0 || T.alpha > 8 || T.model > 1 || !(T.area > 0))
      return fail(DRT_E_INVAL, "tile %d: need alpha in 0..8, model 0/1 and area > 0", i);
    if (!unit(T.n0)) return fail(DRT_E_INVAL, "tile %d: normal is not a unit vector", i);
  }
  s.rays.resize(d->n_rays);
  for (int r = 0; r < d->n_rays; ++r) {
    DRay& R = s.rays[r];
    std::memset(&R, 0, sizeof R);
    int n = d->ray_nint[r];
    if (n > DRT_MAX_INT) return fail(DRT_E_INVAL, "ray %d: %d interactions (max 4)", r, n);
    int nd = 0, ns = 0;
    for (int i = 0; i < n; ++i) {
      int k = d->ray_kind[4 * r + i], p = d->ray_prim[4 * r + i], pol = d->ray_pol[4 * r + i];
      if (pol > 1) return fail(DRT_E_INVAL, "ray %d: polarisation flag %d", r, pol);
      int lim = k == DRT_R ? d->n_planes : k == DRT_D ? d->n_edges : k == DRT_S ? d->n_tiles : -1;
      if (lim < 0) return fail(DRT_E_INVAL, "ray %d: interaction kind %d", r, k);
      if (p < 0 || p >= lim) return fail(DRT_E_INVAL, "ray %d: primitive %d out of range", r, p);
      nd += k == DRT_D;
      ns += k == DRT_S;
      R.kind[i] = k;
      R.pol[i] = pol;
      R.prim[i] = p;
      R.body[i] = k == DRT_R ? planes[p].body : k == DRT_D ? edges[p].body : tiles[p].body;
    }
    if (nd > 1 && !(nd == 2 && n == 2))
      return fail(DRT_E_INVAL, "ray %d: two diffractions only as a two-edge ray, one diffraction otherwise", r);
    if (nd == 2 && R.prim[0] == R.prim[1]) return fail(DRT_E_INVAL, "ray %d: the two edges must differ", r);
    if (ns > 0 && n != 1) return fail(DRT_E_INVAL, "ray %d: scattering must be the only interaction", r);
    R.nint = n;
    int dpos;
    R.code = sig_code(n, R.kind, &dpos);
    R.dpos = dpos;
    s.cls_rays[sig_class(R.code)].push_back(r);
  }
  for (int c = 0; c < CLS_COUNT; ++c) {
    s.cls_by_sig[c] = s.cls_rays[c];
    std::stable_sort(s.cls_by_sig[c].begin(), s.cls_by_sig[c].end(),
                     [&](int32_t a, int32_t b) { return s.rays[a].code < s.rays[b].code; });
  }

  // host view for the t0 checks
  SceneView hv{};
  hv.bodies = s.bodies.data();
  hv.mats = mats.data();
  hv.planes = planes.data();
  hv.edges = edges.data();
  hv.tiles = tiles.data();
  hv.rays = s.rays.data();
  std::memcpy(hv.tx_p, d->tx_p, 24);
  std::memcpy(hv.rx_p, d->rx_p, 24);
  std::memcpy(hv.tx_v, d->tx_v, 24);
  if ((d->tx_ant == nullptr) != (d->rx_ant == nullptr))
    return fail(DRT_E_INVAL, "give both antennas or neither");
  if (d->tx_ant) {
    const double kt = d->tx_ant[3], kr = d->rx_ant[3];
    if (!((kt == 0 || kt == 1) && kt == kr)) return fail(DRT_E_INVAL, "antenna kinds must both be 0 or both be 1");
    if (kt == 1) {
      if (!unit(d->tx_ant) || !unit(d->rx_ant)) return fail(DRT_E_INVAL, "dipole axes must be unit vectors");
      std::memcpy(hv.tx_ant, d->tx_ant, 24);
      std::memcpy(hv.rx_ant, d->rx_ant, 24);
      hv.polar = 1;
    }
  }
  std::memcpy(hv.rx_v, d->rx_v, 24);
  for (int r = 0; r < d->n_rays; ++r) {
    const DRay& R = s.rays[r];
    Slot<double> sl[DRT_MAX_INT];
    for (int i = 0; i < R.nint; ++i) {
      Pose<double> ps = make_pose<double>(s.bodies[R.body[i]], 0.0, 0.0, 0.0);
      load_slot<double>(hv, R.kind[i], R.prim[i], ps, sl[i]);
    }
    RayResult<double> res = with_signature<double>(R.code, [&]<int N, int DP, bool SCAT>() {
      return eval_host<N, DP, SCAT>(hv, R, sl);
    });
    if (res.degen)
      return fail(DRT_E_DEGENERATE, "ray %d is degenerate at t0 (image line parallel to a wall, a "
                  "diffraction source on the edge line, or a zero-length segment)", r);
    if (d->ray_q0) {
      for (int i = 0; i < R.nint; ++i) {
        const double* q = d->ray_q0 + (size_t(r) * 4 + i) * 3;
        double dx = q[0] - res.Q[i].x, dy = q[1] - res.Q[i].y, dz = q[2] - res.Q[i].z;
        if (std::sqrt(dx * dx + dy * dy + dz * dz) > 1e-6)
          return fail(DRT_E_INCONSISTENT, "ray %d interaction %d: ray_q0 is %.3g m from the t0 solve", r, i,
                      std::sqrt(dx * dx + dy * dy + dz * dz));
      }
    }
  }
  s.view = hv;          // device pointers are filled in by device_view()
  s.view.n_bodies = d->n_bodies;
  s.view.n_rays = d->n_rays;
  std::memcpy(s.view.tx_a, d->tx_a, 24);
  std::memcpy(s.view.rx_a, d->rx_a, 24);
  return DRT_OK;
}

// ---------------------------------------------------------------------------------------
// descriptions by value

template <class T>
static std::vector<T> vcopy(const T* p, size_t n) {
  return p ? std::vector<T>(p, p + n) : std::vector<T>();
}
template <class T>
static const T* ptr_or_null(const std::vector<T>& v) {
  return v.empty() ? nullptr : v.data();
}

static HostDesc copy_desc(const drt_scene_desc* d) {
  HostDesc h;
  h.t0 = d->t0;
  std::memcpy(h.tx_p, d->tx_p, 24);
  std::memcpy(h.tx_v, d->tx_v, 24);
  std::memcpy(h.tx_a, d->tx_a, 24);
  std::memcpy(h.rx_p, d->rx_p, 24);
  std::memcpy(h.rx_v, d->rx_v, 24);
  std::memcpy(h.rx_a, d->rx_a, 24);
  h.nb = d->n_bodies;
  h.nm = d->n_mat;
  h.np = d->n_planes;
  h.ne = d->n_edges;
  h.nt = d->n_tiles;
  h.nr = d->n_rays;
  const size_t nb = h.nb, nm = h.nm, np = h.np, ne = h.ne, nt = h.nt, nr = h.nr;
  h.body_O0 = vcopy(d->body_O0, 3 * nb);
  h.body_v0 = vcopy(d->body_v0, 3 * nb);
  h.body_a = vcopy(d->body_a, 3 * nb);
  h.body_axis = vcopy(d->body_axis, 3 * nb);
  h.body_w0 = vcopy(d->body_w0, nb);
  h.body_wdot = vcopy(d->body_wdot, nb);
  h.mat_eps_r = vcopy(d->mat_eps_r, nm);
  h.mat_sigma = vcopy(d->mat_sigma, nm);
  h.mat_pec = vcopy(d->mat_pec, nm);
  h.plane_body = vcopy(d->plane_body, np);
  h.plane_mat = vcopy(d->plane_mat, np);
  h.plane_p0 = vcopy(d->plane_p0, 3 * np);
  h.plane_n0 = vcopy(d->plane_n0, 3 * np);
  h.plane_facet = vcopy(d->plane_facet, 9 * np);
  h.edge_body = vcopy(d->edge_body, ne);
  h.edge_a0 = vcopy(d->edge_a0, 3 * ne);
  h.edge_e0 = vcopy(d->edge_e0, 3 * ne);
  h.edge_t0 = vcopy(d->edge_t0, 3 * ne);
  h.edge_n0 = vcopy(d->edge_n0, 3 * ne);
  h.edge_wedge_n = vcopy(d->edge_wedge_n, ne);
  h.edge_zlim = vcopy(d->edge_zlim, 2 * ne);
  h.tile_body = vcopy(d->tile_body, nt);
  h.tile_alpha = vcopy(d->tile_alpha, nt);
  h.tile_model = vcopy(d->tile_model, nt);
  h.tile_c0 = vcopy(d->tile_c0, 3 * nt);
  h.tile_n0 = vcopy(d->tile_n0, 3 * nt);
  h.tile_area = vcopy(d->tile_area, nt);
  h.tile_S = vcopy(d->tile_S, nt);
  h.tile_phase0 = vcopy(d->tile_phase0, nt);
  h.ray_nint = vcopy(d->ray_nint, nr);
  h.ray_kind = vcopy(d->ray_kind, 4 * nr);
  h.ray_pol = vcopy(d->ray_pol, 4 * nr);
  h.ray_prim = vcopy(d->ray_prim, 4 * nr);
  h.tx_ant = vcopy(d->tx_ant, 4);
  h.rx_ant = vcopy(d->rx_ant, 4);
  return h;
}

static drt_scene_desc desc_view(const HostDesc& h) {
  drt_scene_desc d{};
  d.t0 = h.t0;
  std::memcpy(d.tx_p, h.tx_p, 24);
  std::memcpy(d.tx_v, h.tx_v, 24);
  std::memcpy(d.tx_a, h.tx_a, 24);
  std::memcpy(d.rx_p, h.rx_p, 24);
  std::memcpy(d.rx_v, h.rx_v, 24);
  std::memcpy(d.rx_a, h.rx_a, 24);
  d.n_bodies = h.nb;
  d.body_O0 = ptr_or_null(h.body_O0);
  d.body_v0 = ptr_or_null(h.body_v0);
  d.body_a = ptr_or_null(h.body_a);
  d.body_axis = ptr_or_null(h.body_axis);
  d.body_w0 = ptr_or_null(h.body_w0);
  d.body_wdot = ptr_or_null(h.body_wdot);
  d.n_mat = h.nm;
  d.mat_eps_r = ptr_or_null(h.mat_eps_r);
  d.mat_sigma = ptr_or_null(h.mat_sigma);
  d.mat_pec = ptr_or_null(h.mat_pec);
  d.n_planes = h.np;
  d.plane_body = ptr_or_null(h.plane_body);
  d.plane_mat = ptr_or_null(h.plane_mat);
  d.plane_p0 = ptr_or_null(h.plane_p0);
  d.plane_n0 = ptr_or_null(h.plane_n0);
  d.plane_facet = ptr_or_null(h.plane_facet);
  d.n_edges = h.ne;
  d.edge_body = ptr_or_null(h.edge_body);
  d.edge_a0 = ptr_or_null(h.edge_a0);
  d.edge_e0 = ptr_or_null(h.edge_e0);
  d.edge_t0 = ptr_or_null(h.edge_t0);
  d.edge_n0 = ptr_or_null(h.edge_n0);
  d.edge_wedge_n = ptr_or_null(h.edge_wedge_n);
  d.edge_zlim = ptr_or_null(h.edge_zlim);
  d.n_tiles = h.nt;
  d.tile_body = ptr_or_null(h.tile_body);
  d.tile_alpha = ptr_or_null(h.tile_alpha);
  d.tile_model = ptr_or_null(h.tile_model);
  d.tile_c0 = ptr_or_null(h.tile_c0);
  d.tile_n0 = ptr_or_null(h.tile_n0);
  d.tile_area = ptr_or_null(h.tile_area);
  d.tile_S = ptr_or_null(h.tile_S);
  d.tile_phase0 = ptr_or_null(h.tile_phase0);
  d.n_rays = h.nr;
  d.ray_nint = ptr_or_null(h.ray_nint);
  d.ray_kind = ptr_or_null(h.ray_kind);
  d.ray_pol = ptr_or_null(h.ray_pol);
  d.ray_prim = ptr_or_null(h.ray_prim);
  d.ray_q0 = nullptr;
  d.tx_ant = ptr_or_null(h.tx_ant);
  d.rx_ant = ptr_or_null(h.rx_ant);
  return d;
}

// The description carried to the instant t0 + t: terminals by eq. Taylor; every body's
// reference point, velocity and angular speed advanced (Sec. III-A.1), and the primitives
// of a moving body placed with its pose at t (rotation by theta = w0 t + wdot t^2 / 2 about
// its fixed axis, Rodrigues' formula), so that the new description at its own t0 is the
// old one at t0 + t.
static HostDesc rebase(const HostDesc& d, double t) {
  HostDesc r = d;
  r.t0 = d.t0 + t;
  const double h2 = 0.5 * t * t;
  for (int k = 0; k < 3; ++k) {
    r.tx_p[k] = d.tx_p[k] + d.tx_v[k] * t + d.tx_a[k] * h2;
    r.tx_v[k] = d.tx_v[k] + d.tx_a[k] * t;
    r.rx_p[k] = d.rx_p[k] + d.rx_v[k] * t + d.rx_a[k] * h2;
    r.rx_v[k] = d.rx_v[k] + d.rx_a[k] * t;
  }
  struct BodyPose {
    bool moving;
    double O[3], O0[3], k[3], s, c1;
  };
  std::vector<BodyPose> bp(d.nb);
  for (int b = 0; b < d.nb; ++b) {
    BodyPose& B = bp[b];
    const double *O0 = &d.body_O0[3 * b], *v0 = &d.body_v0[3 * b], *a = &d.body_a[3 * b];
    const double w0 = d.body_w0[b], wd = d.body_wdot[b];
    B.moving = w0 != 0 || wd != 0;
    for (int k = 0; k < 3; ++k) B.moving = B.moving || v0[k] != 0 || a[k] != 0;
    const double th = w0 * t + 0.5 * wd * t * t, hs = std::sin(0.5 * th);
    B.s = std::sin(th);
    B.c1 = 2.0 * hs * hs;
    for (int k = 0; k < 3; ++k) {
      B.O0[k] = O0[k];
      B.k[k] = d.body_axis[3 * b + k];
      B.O[k] = O0[k] + v0[k] * t + a[k] * h2;
      r.body_O0[3 * b + k] = B.O[k];
      r.body_v0[3 * b + k] = v0[k] + a[k] * t;
    }
    r.body_w0[b] = w0 + wd * t;
  }
  auto rot = [](const BodyPose& B, const double* v, double* out) {
    const double kv[3] = {B.k[1] * v[2] - B.k[2] * v[1], B.k[2] * v[0] - B.k[0] * v[2], B.k[0] * v[1] - B.k[1] * v[0]};
    const double kkv[3] = {B.k[1] * kv[2] - B.k[2] * kv[1], B.k[2] * kv[0] - B.k[0] * kv[2],
                           B.k[0] * kv[1] - B.k[1] * kv[0]};
    for (int k = 0; k < 3; ++k) out[k] = v[k] + B.s * kv[k] + B.c1 * kkv[k];
  };
  auto carry = [&](int b, const double* d0, double* out) {
    if (bp[b].moving) rot(bp[b], d0, out);
    else std::memmove(out, d0, 24);
  };
  auto place = [&](int b, const double* x0, double* out) {
    if (!bp[b].moving) {
      std::memmove(out, x0, 24);
      return;
    }
    const double w[3] = {x0[0] - bp[b].O0[0], x0[1] - bp[b].O0[1], x0[2] - bp[b].O0[2]};
    double rw[3];
    rot(bp[b], w, rw);
    for (int k = 0; k < 3; ++k) out[k] = bp[b].O[k] + rw[k];
  };
  for (int i = 0; i < d.np; ++i) {
    const int b = d.plane_body[i];
    place(b, &d.plane_p0[3 * i], &r.plane_p0[3 * i]);
    carry(b, &d.plane_n0[3 * i], &r.plane_n0[3 * i]);
    if (!d.plane_facet.empty()) {
      place(b, &d.plane_facet[9 * i], &r.plane_facet[9 * i]);
      carry(b, &d.plane_facet[9 * i + 3], &r.plane_facet[9 * i + 3]);
      carry(b, &d.plane_facet[9 * i + 6], &r.plane_facet[9 * i + 6]);
    }
  }
  for (int i = 0; i < d.ne; ++i) {
    const int b = d.edge_body[i];
    place(b, &d.edge_a0[3 * i], &r.edge_a0[3 * i]);
    carry(b, &d.edge_e0[3 * i], &r.edge_e0[3 * i]);
    carry(b, &d.edge_t0[3 * i], &r.edge_t0[3 * i]);
    carry(b, &d.edge_n0[3 * i], &r.edge_n0[3 * i]);
  }
  for (int i = 0; i < d.nt; ++i) {
    const int b = d.tile_body[i];
    place(b, &d.tile_c0[3 * i], &r.tile_c0[3 * i]);
    carry(b, &d.tile_n0[3 * i], &r.tile_n0[3 * i]);
  }
  return r;
}

}  // namespace drt_host
