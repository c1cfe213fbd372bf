// Host build of the scene loader (validation, packing, the t0 solve, the copy of a
// description by value and its carriage to another instant) and of the per-ray geometry
// the kernels evaluate, for CPU tests under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// stdin, one item a line:
//   A <name> <count> <v_1 ... v_count>   one array of the scene description, by its field
//                                        name; count -1 leaves the field NULL
//   PACK                                 validate and pack; prints "status <code> <message>"
//   REBASE <t>                           carry the packed description to t0 + t, then pack
//                                        the carried copy again; prints "status ..."
//   EVAL <prec> <n> <t_1 ... t_n>        every ray at each instant t_j after t0 of the last
//                                        packed description, field coefficient in binary64
//                                        (prec 64) or binary32 (32); one line per (ray,
//                                        instant), rays outer: L dop gain_re gain_im aod_az
//                                        aod_el aoa_az aoa_el ok in_bounds degen
//   FC <f_c>                             carrier frequency of EVAL [Hz]
// Arrays are allocated at exactly their given length, so that a read past what the
// description holds is a sanitizer error.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "scene_host.h"

using namespace drt;
using namespace drt_host;

namespace {

std::map<std::string, std::vector<double>> g_arr;   // as read
std::map<std::string, bool> g_null;
std::vector<std::vector<int32_t>> g_i32;             // typed copies the description points into
std::vector<std::vector<uint8_t>> g_u8;
std::vector<std::vector<double>> g_f64;

const double* f64(const char* k) {
  if (g_null[k] || !g_arr.count(k)) return nullptr;
  g_f64.emplace_back(g_arr[k]);
  return g_f64.back().empty() ? nullptr : g_f64.back().data();
}
const int32_t* i32(const char* k) {
  if (g_null[k] || !g_arr.count(k)) return nullptr;
  g_i32.emplace_back(g_arr[k].begin(), g_arr[k].end());
  return g_i32.back().empty() ? nullptr : g_i32.back().data();
}
const uint8_t* u8(const char* k) {
  if (g_null[k] || !g_arr.count(k)) return nullptr;
  g_u8.emplace_back();
  for (double v : g_arr[k]) g_u8.back().push_back(uint8_t(v));
  return g_u8.back().empty() ? nullptr : g_u8.back().data();
}
int32_t count(const char* k, int per) { return g_arr.count(k) ? int32_t(g_arr[k].size() / per) : 0; }
void vec3(const char* k, double* out) {
  for (int i = 0; i < 3; ++i) out[i] = g_arr.count(k) && g_arr[k].size() == 3 ? g_arr[k][i] : 0.0;
}

drt_scene_desc build_desc() {
  drt_scene_desc d{};
  d.t0 = g_arr.count("t0") && !g_arr["t0"].empty() ? g_arr["t0"][0] : 0.0;
  vec3("tx_p", d.tx_p);
  vec3("tx_v", d.tx_v);
  vec3("tx_a", d.tx_a);
  vec3("rx_p", d.rx_p);
  vec3("rx_v", d.rx_v);
  vec3("rx_a", d.rx_a);
  d.n_bodies = count("body_w0", 1);
  d.body_O0 = f64("body_O0");
  d.body_v0 = f64("body_v0");
  d.body_a = f64("body_a");
  d.body_axis = f64("body_axis");
  d.body_w0 = f64("body_w0");
  d.body_wdot = f64("body_wdot");
  d.n_mat = count("mat_eps_r", 1);
  d.mat_eps_r = f64("mat_eps_r");
  d.mat_sigma = f64("mat_sigma");
  d.mat_pec = u8("mat_pec");
  d.n_planes = count("plane_body", 1);
  d.plane_body = i32("plane_body");
  d.plane_mat = i32("plane_mat");
  d.plane_p0 = f64("plane_p0");
  d.plane_n0 = f64("plane_n0");
  d.plane_facet = f64("plane_facet");
  d.n_edges = count("edge_body", 1);
  d.edge_body = i32("edge_body");
  d.edge_a0 = f64("edge_a0");
  d.edge_e0 = f64("edge_e0");
  d.edge_t0 = f64("edge_t0");
  d.edge_n0 = f64("edge_n0");
  d.edge_wedge_n = f64("edge_wedge_n");
  d.edge_zlim = f64("edge_zlim");
  d.n_tiles = count("tile_body", 1);
  d.tile_body = i32("tile_body");
  d.tile_alpha = i32("tile_alpha");
  d.tile_model = u8("tile_model");
  d.tile_c0 = f64("tile_c0");
  d.tile_n0 = f64("tile_n0");
  d.tile_area = f64("tile_area");
  d.tile_S = f64("tile_S");
  d.tile_phase0 = f64("tile_phase0");
  d.n_rays = count("ray_nint", 1);
  d.ray_nint = u8("ray_nint");
  d.ray_kind = u8("ray_kind");
  d.ray_pol = u8("ray_pol");
  d.ray_prim = i32("ray_prim");
  d.ray_q0 = f64("ray_q0");
  d.tx_ant = f64("tx_ant");
  d.rx_ant = f64("rx_ant");
  return d;
}

// One ray at the instant t after t0, as the geometry kernel takes it: terminals by their
// Taylor expansion, every body's pose from sin(theta) and 1 - cos(theta).
template <class G>
RayResult<double, G> eval_at(const PackedScene& s, const DRay& ray, double t, double f_c) {
  const SceneView& sc = s.view;
  const double h = 0.5 * t * t;
  const V3<double> TX = ld3<double>(sc.tx_p) + t * ld3<double>(sc.tx_v) + h * ld3<double>(sc.tx_a);
  const V3<double> RX = ld3<double>(sc.rx_p) + t * ld3<double>(sc.rx_v) + h * ld3<double>(sc.rx_a);
  const V3<double> VTX = ld3<double>(sc.tx_v) + t * ld3<double>(sc.tx_a);
  const V3<double> VRX = ld3<double>(sc.rx_v) + t * ld3<double>(sc.rx_a);
  Slot<double> sl[DRT_MAX_INT];
  for (int i = 0; i < ray.nint; ++i) {
    const DBody& B = sc.bodies[ray.body[i]];
    const double th = B.w0 * t + 0.5 * B.wdot * t * t, hs = std::sin(0.5 * th);
    load_slot<double>(sc, ray.kind[i], ray.prim[i], make_pose<double>(B, t, std::sin(th), 2.0 * hs * hs), sl[i]);
  }
  return with_signature<double>(ray.code, [&]<int N, int DP, bool SCAT>() {
    if (sc.polar) return eval_ray<double, G, N, DP, SCAT, false, true, true>(sc, ray, sl, TX, VTX, RX, VRX, f_c);
    return eval_ray<double, G, N, DP, SCAT, false, true, false>(sc, ray, sl, TX, VTX, RX, VRX, f_c);
  });
}

template <class G>
void eval_all(const PackedScene& s, const std::vector<double>& ts, double f_c) {
  for (const DRay& ray : s.rays)
    for (double t : ts) {
      const RayResult<double, G> r = eval_at<G>(s, ray, t, f_c);
      std::printf("%.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g %d %d %d\n", r.L, r.dop, double(r.gain.re),
                  double(r.gain.im), double(r.aod_az), double(r.aod_el), double(r.aoa_az), double(r.aoa_el),
                  int(r.ok), int(r.in_bounds), int(r.degen));
    }
}

}  // namespace

int main() {
  char cmd[64];
  PackedScene packed;
  bool have = false;
  double f_c = 28e9;
  while (std::scanf("%63s", cmd) == 1) {
    if (!std::strcmp(cmd, "A")) {
      char name[64];
      long n;
      if (std::scanf("%63s %ld", name, &n) != 2) return 2;
      g_null[name] = n < 0;
      std::vector<double> v(n > 0 ? size_t(n) : 0);
      for (double& x : v)
        if (std::scanf("%lf", &x) != 1) return 2;
      g_arr[name] = std::move(v);
    } else if (!std::strcmp(cmd, "FC")) {
      if (std::scanf("%lf", &f_c) != 1) return 2;
    } else if (!std::strcmp(cmd, "PACK")) {
      g_i32.clear();
      g_u8.clear();
      g_f64.clear();
      const drt_scene_desc d = build_desc();
      packed = PackedScene{};
      const int st = validate_and_pack(&d, packed);
      if (st == DRT_OK) packed.desc = copy_desc(&d);
      have = st == DRT_OK;
      std::printf("status %d %s\n", st, st ? g_last_error.c_str() : "ok");
    } else if (!std::strcmp(cmd, "REBASE")) {
      double t;
      if (std::scanf("%lf", &t) != 1 || !have) return 2;
      HostDesc h = rebase(packed.desc, t);
      const drt_scene_desc dv = desc_view(h);
      PackedScene next;
      const int st = validate_and_pack(&dv, next);
      if (st == DRT_OK) {
        next.desc = std::move(h);
        packed = std::move(next);
      }
      have = st == DRT_OK;
      std::printf("status %d %s\n", st, st ? g_last_error.c_str() : "ok");
    } else if (!std::strcmp(cmd, "EVAL")) {
      int prec, n;
      if (std::scanf("%d %d", &prec, &n) != 2 || n < 0 || !have) return 2;
      std::vector<double> ts(n);
      for (double& t : ts)
        if (std::scanf("%lf", &t) != 1) return 2;
      if (prec == 64) eval_all<double>(packed, ts, f_c);
      else eval_all<float>(packed, ts, f_c);
    } else {
      return 2;
    }
    std::fflush(stdout);
  }
  return 0;
}
