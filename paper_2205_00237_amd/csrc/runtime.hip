// Host runtime of libdrt: the C ABI of include/drt.h, the scene loader, scratch management
// and the serving loop (continuous batching of channel-prediction requests).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "drt_geom.h"
#include "drt_kernels.h"

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

#define HIP_OK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(DRT_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

double drt_now_impl() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------------------
// device buffers

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Scene {
  uint32_t id = 0;
  SceneView view{};
  std::vector<DBody> bodies;     // host copies of the packed tables
  std::vector<DMat> mats;
  std::vector<DPlane> planes;
  std::vector<DEdge> edges;
  std::vector<DTile> tiles;
  std::vector<DRay> rays;
  std::vector<int32_t> cls_rays[CLS_COUNT];   // ray indices of each signature class, ascending
  DevBuf d_bodies, d_mats, d_planes, d_edges, d_tiles, d_rays, d_order;
  size_t bytes = 0;
  int inflight = 0;
};

// Scratch of one stream: pose table, anchor records and partial H tiles of one call.
struct Scratch {
  DevBuf buf;
};

struct Request;

// One batch in flight: its stream, the instantiated graph of fused batch kernels, the batch descriptor (pinned host copy and
// device copy; the kernels read only the device copy, so the graph replays with nothing but
// its grid sizes updated), and the scratch arena holding every request's pose table,
// records and partial sums.
struct Slot_ {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t node[BK_COUNT] = {};     // the kernel node of each kind
  hipKernelNodeParams kp[BK_COUNT] = {};  // its launch parameters (grid updated per batch)
  bool on[BK_COUNT] = {};                 // node enabled in exec
  BatchDesc* h_desc = nullptr;
  DevBuf d_desc;
  Scratch scratch;
  std::vector<Request*> reqs;
};

struct Request {
  uint64_t ticket;
  drt_request r;
  Scene* scene;
  size_t footprint;
  int state = 0;   // 0 queued, 1 running, 2 done, < 0 error
  double t_arrive = 0, t_admit = 0, t_done = 0;
};

struct drt_ctx {
  int device = 0;
  uint64_t cap = 0;
  std::atomic<uint64_t> used{0};
  std::mutex mu;
  std::unordered_map<uint32_t, std::unique_ptr<Scene>> scenes;
  uint32_t next_scene = 1;
  std::map<hipStream_t, Scratch> scratch;   // per caller stream (drt_extrapolate / drt_cfr)
  std::mutex scratch_mu;
  int target_waves = 16384;
  int split_path = CFR_MFMA16;               // ray-sum kernel of DRT_SPLIT (DRT_CFR_KERNEL)

  // kernel timing
  struct ProfRec { int kernel, n; hipEvent_t a, b; };   // n kernels back to back between a and b
  std::atomic<bool> prof{false};
  std::mutex prof_mu;
  std::vector<ProfRec> prof_recs;

  // serving
  std::vector<Slot_> slots;
  drt_serving_stats stats{};
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  size_t inflight_bytes = 0;
  std::thread worker;
  std::condition_variable cv;
  bool stop = false;
  bool worker_started = false;
};

static int set_device(drt_ctx* c) {
  HIP_OK(hipSetDevice(c->device));
  return DRT_OK;
}

static int dev_alloc(drt_ctx* c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (c->used.load() + bytes > c->cap)
    return fail(DRT_E_NOMEM, "device memory cap of %llu bytes exceeded (need %zu more)",
                (unsigned long long)c->cap, bytes);
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) return fail(DRT_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  b.bytes = bytes;
  c->used += bytes;
  return DRT_OK;
}

static void dev_free(drt_ctx* c, DevBuf& b) {
  if (b.p) {
    (void)hipFree(b.p);
    c->used -= b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
}

// grow-only scratch; the stream is synchronised first so no kernel still uses the old one
static int ensure_scratch(drt_ctx* c, Scratch& s, size_t bytes, hipStream_t st, size_t limit = SIZE_MAX) {
  if (s.buf.bytes >= bytes) return DRT_OK;
  HIP_OK(hipStreamSynchronize(st));
  dev_free(c, s.buf);
  return dev_alloc(c, s.buf, std::max(bytes, std::min(bytes + bytes / 4, limit)));   // headroom to regrow less
}

// ---------------------------------------------------------------------------------------
// loader

static bool unit(const double* v) {
  double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  return std::fabs(n - 1.0) < 1e-9;
}

static int sig_code(int nint, const uint8_t* kind, int* dpos) {
  *dpos = 255;
  if (nint == 0) return SIG_LOS;
  if (kind[0] == DRT_S) return SIG_S;
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

static int validate_and_pack(const drt_scene_desc* d, Scene& s) {
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
      R.kind[i] = uint8_t(k);
      R.pol[i] = uint8_t(pol);
      R.prim[i] = p;
      R.body[i] = k == DRT_R ? planes[p].body : k == DRT_D ? edges[p].body : tiles[p].body;
    }
    if (nd > 1) return fail(DRT_E_INVAL, "ray %d: more than one diffraction", r);
    if (ns > 0 && n != 1) return fail(DRT_E_INVAL, "ray %d: scattering must be the only interaction", r);
    R.nint = uint8_t(n);
    int dpos;
    R.code = uint8_t(sig_code(n, R.kind, &dpos));
    R.dpos = uint8_t(dpos);
    s.cls_rays[sig_class(R.code)].push_back(r);
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

template <class T>
static int upload(drt_ctx* c, DevBuf& b, const T* host, size_t n) {
  int st = dev_alloc(c, b, n * sizeof(T));
  if (st) return st;
  if (n) HIP_OK(hipMemcpy(b.p, host, n * sizeof(T), hipMemcpyHostToDevice));
  return DRT_OK;
}

static void free_scene(drt_ctx* c, Scene& s) {
  dev_free(c, s.d_bodies);
  dev_free(c, s.d_mats);
  dev_free(c, s.d_planes);
  dev_free(c, s.d_edges);
  dev_free(c, s.d_tiles);
  dev_free(c, s.d_rays);
  dev_free(c, s.d_order);
}

// The rays [0, n_rays) of each signature class for one call.
static RayClasses classes(const Scene& s, int n_rays) {
  RayClasses rc{};
  size_t off = 0;
  for (int c = 0; c < CLS_COUNT; ++c) {
    const auto& v = s.cls_rays[c];
    rc.order[c] = (const int32_t*)s.d_order.p + off;
    rc.count[c] = int(std::lower_bound(v.begin(), v.end(), n_rays) - v.begin());
    off += v.size();
  }
  return rc;
}

// geometry kernels one launch makes (one per non-empty signature class)
static int class_kernels(const RayClasses& rc, int T) {
  int n = 0;
  for (int c = 0; c < CLS_COUNT; ++c) n += rc.count[c] > 0 && T > 0;
  return n;
}

// ---------------------------------------------------------------------------------------
// pipelines

static int check_grid(const drt_time_grid* tg, int32_t n_rays, const Scene& s) {
  if (!tg) return fail(DRT_E_INVAL, "null time grid");
  if (tg->n_steps < 0 || !std::isfinite(tg->dt)) return fail(DRT_E_INVAL, "bad time grid");
  if (n_rays < 0 || n_rays > s.view.n_rays)
    return fail(DRT_E_INVAL, "n_rays %d outside [0, %d]", n_rays, s.view.n_rays);
  return DRT_OK;
}

static SceneView device_view(const Scene& s) {
  SceneView v = s.view;
  v.bodies = (const DBody*)s.d_bodies.p;
  v.mats = (const DMat*)s.d_mats.p;
  v.planes = (const DPlane*)s.d_planes.p;
  v.edges = (const DEdge*)s.d_edges.p;
  v.tiles = (const DTile*)s.d_tiles.p;
  v.rays = (const DRay*)s.d_rays.p;
  return v;
}

// Launch `fn` on stream st, bracketed by a hipEvent pair when kernel timing is on.
template <class Fn>
static hipError_t timed(drt_ctx* c, int kernel, hipStream_t st, Fn&& fn, int n_kernels = 1) {
  if (!c || !c->prof.load()) return fn();
  drt_ctx::ProfRec r{kernel, n_kernels, nullptr, nullptr};
  hipError_t e;
  if ((e = hipEventCreate(&r.a)) != hipSuccess) return e;
  if ((e = hipEventCreate(&r.b)) != hipSuccess) return e;
  if ((e = hipEventRecord(r.a, st)) != hipSuccess) return e;
  if ((e = fn()) != hipSuccess) return e;
  if ((e = hipEventRecord(r.b, st)) != hipSuccess) return e;
  std::lock_guard<std::mutex> g(c->prof_mu);
  c->prof_recs.push_back(r);
  return hipSuccess;
}

struct CfrPlan {
  CfrArgs a;
  size_t pose_off, rec_off, part_off, total;
};

static CfrPlan plan(drt_ctx* c, const Scene& s, int n_rays, int T, const drt_freq_grid* fg, int prec) {
  CfrPlan p{};
  int K = fg->n_sub;
  double df = fg->bandwidth / K;
  double f0 = fg->f_c - double(K / 2) * df;
  p.a = plan_cfr(n_rays, T, K, f0, df, c->target_waves, prec, c->split_path);
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  size_t cbytes = prec == DRT_FP64 ? 16 : 8;
  p.pose_off = 0;
  p.rec_off = al(pose_bytes(s.view.n_bodies, T, prec));
  p.part_off = p.rec_off + al(record_bytes(n_rays, T, prec));
  p.total = p.part_off + (p.a.G > 1 ? al(size_t(p.a.G) * T * K * cbytes) : 0);
  return p;
}

static int run_cfr(drt_ctx* c, const Scene& s, int n_rays, const drt_time_grid* tg, const drt_freq_grid* fg,
                   int prec, void* H, const CfrPlan& p, void* scratch, hipStream_t st) {
  char* base = (char*)scratch;
  int T = tg->n_steps;
  HIP_OK(timed(c, DRT_K_POSE, st, [&] {
    return launch_pose((const DBody*)s.d_bodies.p, s.view.n_bodies, T, tg->dt, prec, base + p.pose_off, st);
  }));
  ExtrapOut none{};
  const double inv_c = 1.0 / 299792458.0;
  AnchorParams ap{p.a.f0 * inv_c, double(p.a.B) * p.a.df * inv_c, p.a.df * inv_c};
  int mode = p.a.path == CFR_VALU ? GEOM_ANCHOR : GEOM_ANCHOR_MFMA;
  const RayClasses rc = classes(s, n_rays);
  HIP_OK(timed(c, DRT_K_GEOM, st, [&] {
    return launch_geom(device_view(s), rc, base + p.pose_off, T, tg->dt, fg->f_c, n_rays, prec,
                       mode, none, base + p.rec_off, ap, st);
  }, class_kernels(rc, T)));
  if (p.a.G > 1) {
    HIP_OK(timed(c, DRT_K_CFR, st, [&] { return launch_cfr(base + p.rec_off, p.a, prec, base + p.part_off, st); }));
    HIP_OK(timed(c, DRT_K_REDUCE, st, [&] {
      return launch_reduce(base + p.part_off, p.a.G, size_t(T) * fg->n_sub, prec, H, st);
    }));
  } else {
    HIP_OK(timed(c, DRT_K_CFR, st, [&] { return launch_cfr(base + p.rec_off, p.a, prec, H, st); }));
  }
  return DRT_OK;
}

static int check_fgrid(const drt_freq_grid* fg) {
  if (!fg) return fail(DRT_E_INVAL, "null frequency grid");
  if (fg->n_sub < 0 || !(fg->f_c > 0) || !(fg->bandwidth >= 0)) return fail(DRT_E_INVAL, "bad frequency grid");
  return DRT_OK;
}

static int check_prec(int prec) {
  if (prec != DRT_FP64 && prec != DRT_SPLIT && prec != DRT_NAIVE32)
    return fail(DRT_E_INVAL, "unknown precision %d", prec);
  return DRT_OK;
}

// ---------------------------------------------------------------------------------------
// serving loop

static void serve_loop(drt_ctx* c);

constexpr int kSlots = 4;
constexpr double kBatchSamples = 4e9;   // work cap of one batch (the first request always fits)

// Capture the batch kernels of one slot into a graph, one chain on the slot's stream: pose,
// the geometry classes, the ray-sum tile shapes, the partial-sum reduction.  The node of
// each launch is taken from the capture as it is recorded, so that its grid can be set
// (and an empty kind switched off) per batch on the instantiated graph.
static int capture_batch_graph(drt_ctx* c, Slot_& sl) {
  (void)c;
  const BatchDesc* d = (const BatchDesc*)sl.d_desc.p;
  hipStream_t m = sl.stream;
  HIP_OK(hipStreamBeginCapture(m, hipStreamCaptureModeThreadLocal));
  hipError_t e1 = hipSuccess;
  for (int kind = 0; kind < BK_COUNT && e1 == hipSuccess; ++kind) {
    if ((e1 = launch_batch(kind, d, 1, m)) != hipSuccess) break;
    hipStreamCaptureStatus cs;
    const hipGraphNode_t* deps = nullptr;
    size_t nd = 0;
    if ((e1 = hipStreamGetCaptureInfo_v2(m, &cs, nullptr, nullptr, &deps, &nd)) != hipSuccess) break;
    if (cs != hipStreamCaptureStatusActive || nd != 1) e1 = hipErrorStreamCaptureInvalidated;
    else sl.node[kind] = deps[0];
  }
  hipError_t e2 = hipStreamEndCapture(m, &sl.graph);
  if (e1 != hipSuccess || e2 != hipSuccess)
    return fail(DRT_E_DEVICE, "graph capture: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  for (int k = 0; k < BK_COUNT; ++k) {
    HIP_OK(hipGraphKernelNodeGetParams(sl.node[k], &sl.kp[k]));
    if (sl.kp[k].func != batch_kernel(k)) return fail(DRT_E_DEVICE, "graph capture: node %d is not its kernel", k);
  }
  HIP_OK(hipGraphInstantiate(&sl.exec, sl.graph, nullptr, nullptr, 0));
  for (int k = 0; k < BK_COUNT; ++k) sl.on[k] = true;
  return DRT_OK;
}

// Size every kernel node of the slot's graph to this batch: grid from the item count,
// nodes of kinds without items switched off.
static int set_batch_grids(Slot_& sl, const BatchDesc& h) {
  for (int k = 0; k < BK_COUNT; ++k) {
    const long long items = h.off[k][h.n_req];
    const bool want = items > 0;
    if (want) {
      const long long g = batch_grid(k, items);
      if (g > 0x7fffffffLL) return fail(DRT_E_INVAL, "batch kernel %d needs %lld workgroups", k, g);
      if (sl.kp[k].gridDim.x != unsigned(g)) {
        sl.kp[k].gridDim = dim3(unsigned(g));
        HIP_OK(hipGraphExecKernelNodeSetParams(sl.exec, sl.node[k], &sl.kp[k]));
      }
    }
    if (want != sl.on[k]) {
      HIP_OK(hipGraphNodeSetEnabled(sl.exec, sl.node[k], want ? 1 : 0));
      sl.on[k] = want;
    }
  }
  return DRT_OK;
}

static void free_slots(drt_ctx* c) {
  for (auto& sl : c->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
    if (sl.graph) (void)hipGraphDestroy(sl.graph);
    dev_free(c, sl.scratch.buf);
    dev_free(c, sl.d_desc);
    if (sl.h_desc) (void)hipHostFree(sl.h_desc);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  c->slots.clear();
}

static int init_slots(drt_ctx* c) {
  c->slots.resize(kSlots);
  for (auto& sl : c->slots) {
    HIP_OK(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    HIP_OK(hipHostMalloc((void**)&sl.h_desc, sizeof(BatchDesc), hipHostMallocDefault));
    int st;
    if ((st = dev_alloc(c, sl.d_desc, sizeof(BatchDesc)))) return st;
    if ((st = capture_batch_graph(c, sl))) return st;
  }
  return DRT_OK;
}

static int start_serving(drt_ctx* c) {
  if (c->worker_started) return DRT_OK;
  int st = init_slots(c);
  if (st != DRT_OK) {
    free_slots(c);
    return st;
  }
  c->worker = std::thread(serve_loop, c);
  c->worker_started = true;
  return DRT_OK;
}

static void finish(drt_ctx* c, Slot_& sl, int state) {
  double now = drt_now_impl();
  for (Request* q : sl.reqs) {
    q->state = state;
    q->t_done = now;
    q->scene->inflight--;
    c->inflight_bytes -= q->footprint;
  }
  sl.reqs.clear();
}

// A request runs in a graph batch when its ray sum is the binary16 matrix-core one.
static bool batchable(drt_ctx* c, const Request* q, CfrPlan* p) {
  if (q->r.precision != DRT_SPLIT) return false;
  *p = plan(c, *q->scene, q->r.n_rays, q->r.tg.n_steps, &q->r.fg, q->r.precision);
  return p->a.path == CFR_MFMA16 && cfr_shape(p->a.MT, p->a.NT) >= 0;
}

// Admit the queue head and, when it is batchable, the batchable requests behind it (FIFO)
// while the batch has room, its work stays under the cap and its arena fits in the HBM
// budget.  Returns false when the head has to wait for memory.
static bool launch_next(drt_ctx* c, Slot_& sl) {
  Request* head = c->queue.front();
  CfrPlan hp;
  const bool batch = batchable(c, head, &hp);
  size_t budget = c->cap > c->used.load() ? c->cap - c->used.load() : 0;
  budget += sl.scratch.buf.bytes;   // the slot's arena is re-used
  std::vector<std::pair<Request*, CfrPlan>> take;
  size_t arena = 0;
  double work = 0;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  if (!batch) {
    if (head->footprint > budget) return false;
    take.push_back({head, plan(c, *head->scene, head->r.n_rays, head->r.tg.n_steps, &head->r.fg, head->r.precision)});
    arena = head->footprint;
  } else {
    for (size_t i = 0; i < c->queue.size() && take.size() < size_t(kMaxBatch); ++i) {
      Request* q = c->queue[i];
      CfrPlan p;
      if (i == 0) p = hp;
      else if (!batchable(c, q, &p)) break;
      double w = double(q->r.n_rays) * q->r.tg.n_steps * q->r.fg.n_sub;
      if (i > 0 && work + w > kBatchSamples) break;
      if (arena + al(p.total) > budget) {
        if (i == 0) return false;
        break;
      }
      take.push_back({q, p});
      arena += al(p.total);
      work += w;
    }
  }
  double now = drt_now_impl();
  for (size_t i = 0; i < take.size(); ++i) {
    Request* q = take[i].first;
    c->queue.pop_front();
    q->state = 1;
    q->t_admit = now;
    c->inflight_bytes += q->footprint;
    sl.reqs.push_back(q);
  }
  int st = ensure_scratch(c, sl.scratch, arena, sl.stream, budget);
  if (st == DRT_OK && !batch) {
    Request* q = take[0].first;
    st = run_cfr(nullptr, *q->scene, q->r.n_rays, &q->r.tg, &q->r.fg, q->r.precision, q->r.H, take[0].second,
                 sl.scratch.buf.p, sl.stream);
    c->stats.single_launches++;
  } else if (st == DRT_OK) {
    BatchDesc* h = sl.h_desc;
    const int n = int(take.size());
    h->n_req = n;
    for (int k = 0; k < BK_COUNT; ++k) h->off[k][0] = 0;
    char* base = (char*)sl.scratch.buf.p;
    size_t cur = 0;
    for (int j = 0; j < n; ++j) {
      Request* q = take[j].first;
      const CfrPlan& p = take[j].second;
      BatchReq& b = h->req[j];
      b.sc = device_view(*q->scene);
      b.rc = classes(*q->scene, q->r.n_rays);
      b.T = q->r.tg.n_steps;
      b.n_rays = q->r.n_rays;
      b.nchunk = (b.T + 63) / 64;
      b.pad = 0;
      b.dt = q->r.tg.dt;
      b.f_c = q->r.fg.f_c;
      const double inv_c = 1.0 / 299792458.0;
      b.ap = AnchorParams{p.a.f0 * inv_c, double(p.a.B) * p.a.df * inv_c, p.a.df * inv_c};
      b.a = p.a;
      b.pose = base + cur + p.pose_off;
      b.rec = base + cur + p.rec_off;
      b.part = (float*)(base + cur + p.part_off);
      b.H = (float*)q->r.H;
      cur += al(p.total);
      long long items[BK_COUNT];
      batch_items(b, items);
      for (int k = 0; k < BK_COUNT; ++k) h->off[k][j + 1] = h->off[k][j] + items[k];
    }
    const size_t bytes = offsetof(BatchDesc, req) + size_t(n) * sizeof(BatchReq);
    st = set_batch_grids(sl, *h);
    if (st == DRT_OK && (hipMemcpyAsync(sl.d_desc.p, h, bytes, hipMemcpyHostToDevice, sl.stream) != hipSuccess ||
                         hipGraphLaunch(sl.exec, sl.stream) != hipSuccess))
      st = fail(DRT_E_DEVICE, "batch launch");
    c->stats.batches++;
    c->stats.batched_requests += n;
    if (n > c->stats.max_batch) c->stats.max_batch = n;
  }
  if (st == DRT_OK && hipEventRecord(sl.done, sl.stream) != hipSuccess) st = DRT_E_DEVICE;
  if (st != DRT_OK) {
    (void)hipStreamSynchronize(sl.stream);
    finish(c, sl, st);
  }
  return true;
}

static void serve_loop(drt_ctx* c) {
  (void)hipSetDevice(c->device);
  std::unique_lock<std::mutex> lk(c->mu);
  while (true) {
    bool progress = false;
    // completions
    for (auto& sl : c->slots) {
      if (sl.reqs.empty()) continue;
      hipError_t e = hipEventQuery(sl.done);
      if (e == hipSuccess) {
        finish(c, sl, 2);
        progress = true;
      } else if (e != hipErrorNotReady) {
        finish(c, sl, DRT_E_DEVICE);
        progress = true;
      }
    }
    // admissions: while a slot is free, batch the queue head with what waits behind it
    while (!c->queue.empty()) {
      Slot_* free_slot = nullptr;
      for (auto& sl : c->slots)
        if (sl.reqs.empty()) {
          free_slot = &sl;
          break;
        }
      if (!free_slot || !launch_next(c, *free_slot)) break;   // no slot, or waiting for memory
      progress = true;
    }
    bool busy = false;
    for (auto& sl : c->slots) busy = busy || !sl.reqs.empty();
    if (c->stop && c->queue.empty() && !busy) break;
    if (!progress) {
      if (busy)
        c->cv.wait_for(lk, std::chrono::microseconds(20));
      else
        c->cv.wait_for(lk, std::chrono::milliseconds(5));
    }
  }
}

// ---------------------------------------------------------------------------------------
// C ABI

extern "C" {

double drt_now(void) { return drt_now_impl(); }

const char* drt_strerror(int status) {
  switch (status) {
    case DRT_OK: return "ok";
    case DRT_E_INVAL: return "invalid argument";
    case DRT_E_DEGENERATE: return "degenerate ray at t0";
    case DRT_E_NOMEM: return "out of device memory or over the HBM cap";
    case DRT_E_ADMISSION: return "request footprint exceeds the admission cap";
    case DRT_E_NOTFOUND: return "unknown scene or ticket";
    case DRT_E_BUSY: return "scene busy";
    case DRT_E_DEVICE: return "HIP runtime error";
    case DRT_E_INCONSISTENT: return "t0 interaction points inconsistent";
    default: return "unknown status";
  }
}

const char* drt_last_error(void) { return g_last_error.c_str(); }

int drt_create(int device, uint64_t hbm_cap_bytes, drt_ctx** out) {
  if (!out) return fail(DRT_E_INVAL, "null out pointer");
  int n = 0;
  HIP_OK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(DRT_E_INVAL, "device %d of %d", device, n);
  HIP_OK(hipSetDevice(device));
  size_t free_b = 0, total_b = 0;
  HIP_OK(hipMemGetInfo(&free_b, &total_b));
  auto c = std::make_unique<drt_ctx>();
  c->device = device;
  c->cap = hbm_cap_bytes ? hbm_cap_bytes : uint64_t(0.9 * double(total_b));
  // tuning / comparison knob: which ray-sum kernel DRT_SPLIT uses
  if (const char* k = std::getenv("DRT_CFR_KERNEL")) {
    if (!std::strcmp(k, "valu")) c->split_path = CFR_VALU;
    else if (!std::strcmp(k, "mfma32")) c->split_path = CFR_MFMA;
    else if (!std::strcmp(k, "mfma16")) c->split_path = CFR_MFMA16;
    else return fail(DRT_E_INVAL, "DRT_CFR_KERNEL=%s: expected valu, mfma32 or mfma16", k);
  }
  *out = c.release();
  return DRT_OK;
}

int drt_destroy(drt_ctx* c) {
  if (!c) return fail(DRT_E_INVAL, "null context");
  if (c->worker_started) {
    {
      std::lock_guard<std::mutex> g(c->mu);
      c->stop = true;
    }
    c->cv.notify_all();
    c->worker.join();
  }
  (void)hipSetDevice(c->device);
  free_slots(c);
  (void)hipDeviceSynchronize();
  for (auto& kv : c->scratch) dev_free(c, kv.second.buf);
  for (auto& kv : c->scenes) free_scene(c, *kv.second);
  delete c;
  return DRT_OK;
}

int drt_load_scene(drt_ctx* c, const drt_scene_desc* d, uint32_t* id) {
  if (!c || !id) return fail(DRT_E_INVAL, "null context or id");
  int st = set_device(c);
  if (st) return st;
  auto s = std::make_unique<Scene>();
  st = validate_and_pack(d, *s);
  if (st) return st;
  if ((st = upload(c, s->d_bodies, s->bodies.data(), s->bodies.size())) ||
      (st = upload(c, s->d_mats, s->mats.data(), s->mats.size())) ||
      (st = upload(c, s->d_planes, s->planes.data(), s->planes.size())) ||
      (st = upload(c, s->d_edges, s->edges.data(), s->edges.size())) ||
      (st = upload(c, s->d_tiles, s->tiles.data(), s->tiles.size())) ||
      (st = upload(c, s->d_rays, s->rays.data(), s->rays.size()))) {
    free_scene(c, *s);
    return st;
  }
  std::vector<int32_t> order;
  for (int k = 0; k < CLS_COUNT; ++k) order.insert(order.end(), s->cls_rays[k].begin(), s->cls_rays[k].end());
  if ((st = upload(c, s->d_order, order.data(), order.size()))) {
    free_scene(c, *s);
    return st;
  }
  s->view.mats = nullptr;
  s->view.planes = nullptr;
  s->view.edges = nullptr;
  s->view.tiles = nullptr;
  s->view.bodies = nullptr;
  s->view.rays = nullptr;
  s->bytes = s->d_bodies.bytes + s->d_mats.bytes + s->d_planes.bytes + s->d_edges.bytes + s->d_tiles.bytes +
             s->d_rays.bytes + s->d_order.bytes;
  std::lock_guard<std::mutex> g(c->mu);
  s->id = c->next_scene++;
  *id = s->id;
  c->scenes[s->id] = std::move(s);
  return DRT_OK;
}

int drt_unload_scene(drt_ctx* c, uint32_t id) {
  if (!c) return fail(DRT_E_INVAL, "null context");
  std::lock_guard<std::mutex> g(c->mu);
  auto it = c->scenes.find(id);
  if (it == c->scenes.end()) return fail(DRT_E_NOTFOUND, "scene %u", id);
  if (it->second->inflight > 0) return fail(DRT_E_BUSY, "scene %u has %d requests in flight", id, it->second->inflight);
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  free_scene(c, *it->second);
  c->scenes.erase(it);
  return DRT_OK;
}

static Scene* find_scene(drt_ctx* c, uint32_t id) {
  std::lock_guard<std::mutex> g(c->mu);
  auto it = c->scenes.find(id);
  return it == c->scenes.end() ? nullptr : it->second.get();
}

int drt_extrapolate(drt_ctx* c, uint32_t scene, int32_t n_rays, const drt_time_grid* tg, double f_c,
                    int32_t prec, const drt_ray_out* out, void* stream) {
  if (!c || !out) return fail(DRT_E_INVAL, "null context or output");
  Scene* s = find_scene(c, scene);
  if (!s) return fail(DRT_E_NOTFOUND, "scene %u", scene);
  int st;
  if ((st = check_grid(tg, n_rays, *s)) || (st = check_prec(prec))) return st;
  if (!(f_c > 0)) return fail(DRT_E_INVAL, "carrier must be > 0");
  if ((st = set_device(c))) return st;
  int T = tg->n_steps;
  hipStream_t hs = (hipStream_t)stream;
  if (n_rays == 0) return DRT_OK;
  if (out->first_out) HIP_OK(launch_fill_i32(out->first_out, size_t(n_rays), T, hs));   // lowered by the kernels
  if (T == 0) return DRT_OK;
  std::lock_guard<std::mutex> g(c->scratch_mu);
  Scratch& sc = c->scratch[hs];
  const bool kin = out->q_pos || out->q_vel || out->q_acc || out->dop_rate;
  const bool ext = out->L || out->dop || out->aod_az || out->aod_el || out->aoa_az || out->aoa_el || out->gain ||
                   out->valid || out->in_bounds || out->first_out;
  // the kinematics outputs are jets in binary64: they need the binary64 pose table
  const size_t pb = pose_bytes(s->view.n_bodies, T, prec), pb64 = pose_bytes(s->view.n_bodies, T, DRT_FP64);
  const bool extra64 = kin && prec == DRT_NAIVE32;
  const size_t off64 = extra64 ? (pb + 255) / 256 * 256 : 0;
  if ((st = ensure_scratch(c, sc, off64 + (extra64 ? pb64 : pb), hs))) return st;
  const RayClasses rc = classes(*s, n_rays);
  const DBody* bodies = (const DBody*)s->d_bodies.p;
  if (ext) {
    HIP_OK(timed(c, DRT_K_POSE, hs, [&] {
      return launch_pose(bodies, s->view.n_bodies, T, tg->dt, prec, sc.buf.p, hs);
    }));
    ExtrapOut eo{out->L,      out->dop,  out->aod_az,    out->aod_el,   out->aoa_az,
                 out->aoa_el, out->gain, out->valid, out->in_bounds, out->first_out,
                 nullptr,     nullptr,   nullptr,    nullptr};
    HIP_OK(timed(c, DRT_K_GEOM, hs, [&] {
      return launch_geom(device_view(*s), rc, sc.buf.p, T, tg->dt, f_c, n_rays, prec, GEOM_EXTRAP,
                         eo, nullptr, AnchorParams{0.0, 0.0, 0.0}, hs);
    }, class_kernels(rc, T)));
  }
  if (kin) {
    char* p64 = (char*)sc.buf.p + off64;
    if (extra64 || !ext)
      HIP_OK(timed(c, DRT_K_POSE, hs, [&] {
        return launch_pose(bodies, s->view.n_bodies, T, tg->dt, DRT_FP64, p64, hs);
      }));
    ExtrapOut ko{};
    ko.q_pos = out->q_pos;
    ko.q_vel = out->q_vel;
    ko.q_acc = out->q_acc;
    ko.dop_rate = out->dop_rate;
    HIP_OK(timed(c, DRT_K_GEOM, hs, [&] {
      return launch_geom(device_view(*s), rc, p64, T, tg->dt, f_c, n_rays, prec, GEOM_KIN, ko, nullptr,
                         AnchorParams{0.0, 0.0, 0.0}, hs);
    }, class_kernels(rc, T)));
  }
  return DRT_OK;
}

int drt_cfr(drt_ctx* c, uint32_t scene, int32_t n_rays, const drt_time_grid* tg, const drt_freq_grid* fg,
            int32_t prec, void* H, void* stream) {
  if (!c) return fail(DRT_E_INVAL, "null context");
  Scene* s = find_scene(c, scene);
  if (!s) return fail(DRT_E_NOTFOUND, "scene %u", scene);
  int st;
  if ((st = check_grid(tg, n_rays, *s)) || (st = check_fgrid(fg)) || (st = check_prec(prec))) return st;
  if (tg->n_steps > 0 && fg->n_sub > 0 && !H) return fail(DRT_E_INVAL, "null H");
  if ((st = set_device(c))) return st;
  int T = tg->n_steps, K = fg->n_sub;
  if (T == 0 || K == 0) return DRT_OK;
  hipStream_t hs = (hipStream_t)stream;
  if (n_rays == 0) {
    HIP_OK(launch_zero(H, size_t(T) * K * (prec == DRT_FP64 ? 16 : 8), hs));
    return DRT_OK;
  }
  CfrPlan p = plan(c, *s, n_rays, T, fg, prec);
  std::lock_guard<std::mutex> g(c->scratch_mu);
  Scratch& sc = c->scratch[hs];
  if ((st = ensure_scratch(c, sc, p.total, hs))) return st;
  return run_cfr(c, *s, n_rays, tg, fg, prec, H, p, sc.buf.p, hs);
}

int drt_profile_enable(drt_ctx* c, int on) {
  if (!c) return fail(DRT_E_INVAL, "null context");
  c->prof.store(on != 0);
  return DRT_OK;
}

int drt_profile_read(drt_ctx* c, drt_profile* out, int reset) {
  if (!c || !out) return fail(DRT_E_INVAL, "null argument");
  std::lock_guard<std::mutex> g(c->prof_mu);
  std::memset(out, 0, sizeof *out);
  for (auto& r : c->prof_recs) {
    HIP_OK(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
    out->ms[r.kernel] += ms;
    out->launches[r.kernel] += r.n;
  }
  if (reset) {
    for (auto& r : c->prof_recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    c->prof_recs.clear();
  }
  return DRT_OK;
}

int drt_submit(drt_ctx* c, const drt_request* r, uint64_t* ticket) {
  if (!c || !r || !ticket) return fail(DRT_E_INVAL, "null argument");
  double now = drt_now_impl();
  int st;
  if ((st = check_prec(r->precision))) return st;
  if (r->precision == DRT_NAIVE32) return fail(DRT_E_INVAL, "serving supports DRT_SPLIT and DRT_FP64");
  if ((st = check_fgrid(&r->fg))) return st;
  if (!r->H && r->tg.n_steps > 0 && r->fg.n_sub > 0) return fail(DRT_E_INVAL, "null H");
  std::unique_lock<std::mutex> lk(c->mu);
  if (!c->worker_started && (st = start_serving(c))) return st;
  auto it = c->scenes.find(r->scene);
  if (it == c->scenes.end()) return fail(DRT_E_NOTFOUND, "scene %u", r->scene);
  Scene* s = it->second.get();
  if ((st = check_grid(&r->tg, r->n_rays, *s))) return st;
  auto q = std::make_unique<Request>();
  q->r = *r;
  q->scene = s;
  q->t_arrive = now;
  q->footprint = (r->tg.n_steps > 0 && r->fg.n_sub > 0 && r->n_rays > 0)
                     ? plan(c, *s, r->n_rays, r->tg.n_steps, &r->fg, r->precision).total
                     : 0;
  size_t resident = 0;
  for (auto& kv : c->scenes) resident += kv.second->bytes;
  if (q->footprint + resident > c->cap)
    return fail(DRT_E_ADMISSION, "request footprint %zu bytes exceeds the cap %llu minus resident scenes",
                q->footprint, (unsigned long long)c->cap);
  q->ticket = c->next_ticket++;
  *ticket = q->ticket;
  s->inflight++;
  if (q->footprint == 0) {   // nothing to compute
    q->state = 2;
    q->t_admit = q->t_done = now;
    s->inflight--;
  } else {
    c->queue.push_back(q.get());
  }
  c->reqs[q->ticket] = std::move(q);
  lk.unlock();
  c->cv.notify_all();
  return DRT_OK;
}

int drt_serving_stats_get(drt_ctx* c, drt_serving_stats* out) {
  if (!c || !out) return fail(DRT_E_INVAL, "null argument");
  std::lock_guard<std::mutex> g(c->mu);
  *out = c->stats;
  out->slots = int32_t(c->slots.size());
  return DRT_OK;
}

int drt_poll(drt_ctx* c, uint64_t ticket, drt_req_stat* out) {
  if (!c || !out) return fail(DRT_E_INVAL, "null argument");
  std::lock_guard<std::mutex> g(c->mu);
  auto it = c->reqs.find(ticket);
  if (it == c->reqs.end()) return fail(DRT_E_NOTFOUND, "ticket %llu", (unsigned long long)ticket);
  Request* q = it->second.get();
  out->state = q->state;
  out->t_arrive = q->t_arrive;
  out->t_admit = q->t_admit;
  out->t_done = q->t_done;
  if (q->state == 2 || q->state < 0) c->reqs.erase(it);
  return DRT_OK;
}

}  // extern "C"
