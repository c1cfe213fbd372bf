// Host runtime of libdrt: the C ABI of include/drt.h, the scene loader, scratch management
// and the serving loop (continuous batching of channel-prediction requests).
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

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

#include <sys/prctl.h>

#include "drt_geom.h"
#include "drt_kernels.h"
#include "scene_host.h"

using namespace drt;
using namespace drt_host;

#define HIP_OK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(DRT_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// A named range on the calling thread for a profiler's marker trace (rocprofv3
// --marker-trace): every entry point that launches work, and every serving batch.  Without
// a profiler attached each push and pop is a cheap no-op.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

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

struct Scene : drt_host::PackedScene {
  uint32_t id = 0;
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
  double batch_samples = 4e9;                // work cap of one serving batch (DRT_BATCH_SAMPLES)
  int split_path = CFR_MFMA16;               // ray-sum kernel of DRT_SPLIT (DRT_CFR_KERNEL)
  int fp64_path = CFR_VALU;                  // ray-sum kernel of DRT_FP64 (DRT_FP64_KERNEL)

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

// ---------------------------------------------------------------------------------------
// Scratch of drt_cfr_noalloc: one file-scope device array per GPU, held until the process
// ends, for callers that cannot allocate.  Host code never passes the array's name to a
// kernel (on the host it only names the symbol): its device address is looked up once per
// device, in drt_create with that device current, and kept in noalloc_ptr.

constexpr size_t kNoAllocBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
static void* noalloc_ptr[kMaxDevices] = {};
static std::mutex noalloc_mu;

static int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(DRT_E_INVAL, "device %d beyond %d", device, kMaxDevices);
  std::lock_guard<std::mutex> g(noalloc_mu);
  if (noalloc_ptr[device]) return DRT_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(DRT_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
  noalloc_ptr[device] = p;
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
// device copies of a packed scene

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

// The rays [0, n_rays) of each signature class for one call: the signature-sorted lists
// (second half of d_order) when the call covers every ray of the scene, else the prefix of
// the ascending lists (first half).
static RayClasses classes(const Scene& s, int n_rays) {
  RayClasses rc{};
  const bool all = size_t(n_rays) >= s.rays.size();
  size_t off = all ? s.rays.size() : 0;
  for (int c = 0; c < CLS_COUNT; ++c) {
    const auto& v = s.cls_rays[c];
    rc.order[c] = (const int32_t*)s.d_order.p + off;
    rc.count[c] = all ? int(v.size()) : int(std::lower_bound(v.begin(), v.end(), n_rays) - v.begin());
    off += v.size();
  }
  return rc;
}

// geometry kernels one launch makes (one per non-empty signature class, or one merged kernel
// for a small ray-sum call)
static int class_kernels(const RayClasses& rc, int T, bool ray_sum = false) {
  int n = 0;
  for (int c = 0; c < CLS_COUNT; ++c) n += rc.count[c] > 0 && T > 0;
  return ray_sum && n > 0 && geom_merged(rc, T) ? 1 : n;
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
  p.a = plan_cfr(n_rays, T, K, f0, df, c->target_waves, prec, c->split_path, c->fp64_path);
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
  const RayClasses rc = classes(s, n_rays);
  if (!geom_merged(rc, T)) {   // a merged geometry launch computes its poses in place
    HIP_OK(timed(c, DRT_K_POSE, st, [&] {
      return launch_pose((const DBody*)s.d_bodies.p, s.view.n_bodies, T, tg->dt, prec, base + p.pose_off, st);
    }));
  }
  ExtrapOut none{};
  const double inv_c = 1.0 / 299792458.0;
  AnchorParams ap{p.a.f0 * inv_c, double(p.a.B) * p.a.df * inv_c, p.a.df * inv_c};
  int mode = p.a.path == CFR_VALU ? GEOM_ANCHOR : GEOM_ANCHOR_MFMA;
  HIP_OK(timed(c, DRT_K_GEOM, st, [&] {
    return launch_geom(device_view(s), rc, base + p.pose_off, T, tg->dt, fg->f_c, n_rays, prec,
                       mode, none, base + p.rec_off, ap, st);
  }, class_kernels(rc, T, true)));
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

static int check_prec(int prec, const Scene* s = nullptr) {
  if (prec != DRT_FP64 && prec != DRT_SPLIT && prec != DRT_NAIVE32)
    return fail(DRT_E_INVAL, "unknown precision %d", prec);
  if (s && s->view.polar && prec == DRT_NAIVE32)
    return fail(DRT_E_INVAL, "dipole antennas need DRT_FP64 or DRT_SPLIT");
  return DRT_OK;
}

// ---------------------------------------------------------------------------------------
// serving loop

static void serve_loop(drt_ctx* c);

constexpr int kSlots = 4;

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
    roctxNameHipStream("drt serving slot", sl.stream);
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
  if (q->r.precision != DRT_SPLIT || q->scene->view.polar) return false;   // batch kernels: scalar model
  if (q->r.n_rays == 0) return false;                                       // served by a zero fill
  *p = plan(c, *q->scene, q->r.n_rays, q->r.tg.n_steps, &q->r.fg, q->r.precision);
  return p->a.path == CFR_MFMA16 && cfr_shape(p->a.MT, p->a.NT) >= 0;
}

// Give back device memory that no running batch uses: the arenas of idle slots other than
// `keep` and, with `callers`, the per-stream scratch buffers of drt_extrapolate / drt_cfr
// and the other stream-ordered calls.  Those streams belong to the callers, so the wait
// before freeing them is device-wide; a caller inside one of those calls holds scratch_mu,
// and then its buffer is left alone this time.
static void reclaim(drt_ctx* c, Slot_* keep, bool callers) {
  for (auto& sl : c->slots)
    if (&sl != keep && sl.reqs.empty() && sl.scratch.buf.p) {
      (void)hipStreamSynchronize(sl.stream);
      dev_free(c, sl.scratch.buf);
    }
  if (!callers) return;
  std::unique_lock<std::mutex> g(c->scratch_mu, std::try_to_lock);
  if (!g.owns_lock() || c->scratch.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto& kv : c->scratch) dev_free(c, kv.second.buf);
  c->scratch.clear();
}

// The queue head needs `need` bytes of arena and the budget of slot `sl` is smaller.  Idle
// arenas are reclaimed at once; while batches run, the head waits for them (false: no
// progress); with nothing running, caller scratch is reclaimed too, and a head that still
// does not fit fails with DRT_E_NOMEM so that the requests behind it can go (true).
static bool head_blocked(drt_ctx* c, Slot_& sl, Request* head, size_t need) {
  bool busy = false;
  for (auto& s : c->slots) busy = busy || !s.reqs.empty();
  reclaim(c, &sl, !busy);
  if (busy) return false;
  const size_t budget = (c->cap > c->used.load() ? c->cap - c->used.load() : 0) + sl.scratch.buf.bytes;
  if (need <= budget) return true;   // fits now: the caller's loop admits it next
  c->queue.pop_front();
  head->state = DRT_E_NOMEM;
  head->t_admit = head->t_done = drt_now_impl();
  head->scene->inflight--;
  c->stats.failed_nomem++;
  return true;
}

// Admit the queue head and, when it is batchable, the batchable requests behind it (FIFO)
// while the batch has room, its work stays under the cap and its arena fits in the HBM
// budget.  Returns false when the head has to wait for memory.
// Admits the queue head (with what can batch behind it) to the free slot sl and launches it.
// Called with c->mu held through lk; the lock is released while the batch is assembled and
// launched (scratch growth, graph update, copies), so that callers of drt_submit and
// drt_poll do not wait on the launch, and taken again before returning.  Only this thread
// touches a slot that holds requests, and their scenes stay resident while they are in flight.
static bool launch_next(drt_ctx* c, Slot_& sl, std::unique_lock<std::mutex>& lk) {
  Range range_("drt serving batch");
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
    if (head->footprint > budget) return head_blocked(c, sl, head, head->footprint);
    CfrPlan p{};
    if (head->r.n_rays > 0) p = plan(c, *head->scene, head->r.n_rays, head->r.tg.n_steps, &head->r.fg, head->r.precision);
    take.push_back({head, p});
    arena = head->footprint;
  } else {
    for (size_t i = 0; i < c->queue.size() && take.size() < size_t(kMaxBatch); ++i) {
      Request* q = c->queue[i];
      CfrPlan p;
      if (i == 0) p = hp;
      else if (!batchable(c, q, &p)) break;
      double w = double(q->r.n_rays) * q->r.tg.n_steps * q->r.fg.n_sub;
      if (i > 0 && work + w > c->batch_samples) break;   // the first request always fits
      if (arena + al(p.total) > budget) {
        if (i == 0) return head_blocked(c, sl, head, al(p.total));
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
  if (batch) {
    c->stats.batches++;
    c->stats.batched_requests += int(take.size());
    if (int(take.size()) > c->stats.max_batch) c->stats.max_batch = int(take.size());
  } else {
    c->stats.single_launches++;
  }
  lk.unlock();
  int st = ensure_scratch(c, sl.scratch, arena, sl.stream, budget);
  if (st == DRT_OK && !batch) {
    Request* q = take[0].first;
    if (q->r.n_rays == 0) {   // no rays: H is zero, as drt_cfr writes it
      const size_t cb = q->r.precision == DRT_FP64 ? 16 : 8;
      if (launch_zero(q->r.H, size_t(q->r.tg.n_steps) * q->r.fg.n_sub * cb, sl.stream) != hipSuccess)
        st = fail(DRT_E_DEVICE, "zero fill");
    } else {
      st = run_cfr(nullptr, *q->scene, q->r.n_rays, &q->r.tg, &q->r.fg, q->r.precision, q->r.H, take[0].second,
                   sl.scratch.buf.p, sl.stream);
    }
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
  }
  if (st == DRT_OK && hipEventRecord(sl.done, sl.stream) != hipSuccess) st = DRT_E_DEVICE;
  if (st != DRT_OK) (void)hipStreamSynchronize(sl.stream);
  lk.lock();
  if (st != DRT_OK) finish(c, sl, st);
  return true;
}

static void serve_loop(drt_ctx* c) {
  (void)hipSetDevice(c->device);
  roctxNameOsThread("drt serving loop");
  // the loop sleeps 5 us between completion checks while batches run; the kernel's default
  // timer slack (50 us) would stretch each of those sleeps, and with them the time from a
  // batch's end to its requests reading done
  (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
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
    // a context being destroyed starts nothing more: queued requests are cancelled
    if (c->stop && !c->queue.empty()) {
      const double now = drt_now_impl();
      for (Request* q : c->queue) {
        q->state = DRT_E_CANCELLED;
        q->t_done = now;
        q->scene->inflight--;
      }
      c->queue.clear();
      progress = true;
    }
    // admissions: while a slot is free, batch the queue head with what waits behind it
    while (!c->queue.empty()) {
      Slot_* free_slot = nullptr;
      for (auto& sl : c->slots)
        if (sl.reqs.empty()) {
          free_slot = &sl;
          break;
        }
      if (!free_slot || !launch_next(c, *free_slot, lk)) break;   // no slot, or waiting for memory
      progress = true;
    }
    bool busy = false;
    for (auto& sl : c->slots) busy = busy || !sl.reqs.empty();
    if (c->stop && c->queue.empty() && !busy) break;
    if (!progress) {
      if (busy)
        c->cv.wait_for(lk, std::chrono::microseconds(5));
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
    case DRT_E_CANCELLED: return "request cancelled: context destroyed";
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
  {
    const int st = noalloc_setup(device);
    if (st != DRT_OK) return st;
  }
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
  // comparison knob: which ray-sum kernel DRT_FP64 uses (the subcarrier walk on the vector
  // ALU, or the split path's GEMM factorisation on the binary64 matrix cores)
  if (const char* k = std::getenv("DRT_FP64_KERNEL")) {
    if (!std::strcmp(k, "valu")) c->fp64_path = CFR_VALU;
    else if (!std::strcmp(k, "mfma64")) c->fp64_path = CFR_MFMA64;
    else return fail(DRT_E_INVAL, "DRT_FP64_KERNEL=%s: expected valu or mfma64", k);
  }
  // tuning knob: waves the ray sum aims for (sets the number of ray groups per instant)
  if (const char* w = std::getenv("DRT_TARGET_WAVES")) {
    char* end = nullptr;
    const long v = std::strtol(w, &end, 10);
    if (end == w || *end != '\0' || v < 64 || v > (1L << 24))
      return fail(DRT_E_INVAL, "DRT_TARGET_WAVES=%s: expected an integer in [64, 16777216]", w);
    c->target_waves = int(v);
  }
  // tuning knob: samples (rays x instants x subcarriers) one serving batch may hold
  if (const char* w = std::getenv("DRT_BATCH_SAMPLES")) {
    char* end = nullptr;
    const double v = std::strtod(w, &end);
    if (end == w || *end != '\0' || !(v >= 1e6 && v <= 1e13))
      return fail(DRT_E_INVAL, "DRT_BATCH_SAMPLES=%s: expected a number in [1e6, 1e13]", w);
    c->batch_samples = v;
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

// Upload a packed scene and make it resident.
static int make_resident(drt_ctx* c, std::unique_ptr<Scene> s, uint32_t* id) {
  int st;
  if ((st = upload(c, s->d_bodies, s->bodies.data(), s->bodies.size())) ||
      (st = upload(c, s->d_mats, s->mats.data(), s->mats.size())) ||
      (st = upload(c, s->d_planes, s->planes.data(), s->planes.size())) ||
      (st = upload(c, s->d_edges, s->edges.data(), s->edges.size())) ||
      (st = upload(c, s->d_tiles, s->tiles.data(), s->tiles.size())) ||
      (st = upload(c, s->d_rays, s->rays.data(), s->rays.size()))) {
    free_scene(c, *s);
    return st;
  }
  std::vector<int32_t> order;    // ascending class lists, then the signature-sorted ones
  for (int k = 0; k < CLS_COUNT; ++k) order.insert(order.end(), s->cls_rays[k].begin(), s->cls_rays[k].end());
  for (int k = 0; k < CLS_COUNT; ++k) order.insert(order.end(), s->cls_by_sig[k].begin(), s->cls_by_sig[k].end());
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

int drt_load_scene(drt_ctx* c, const drt_scene_desc* d, uint32_t* id) {
  Range range_("drt_load_scene");
  if (!c || !id) return fail(DRT_E_INVAL, "null context or id");
  int st = set_device(c);
  if (st) return st;
  auto s = std::make_unique<Scene>();
  st = validate_and_pack(d, *s);
  if (st) return st;
  s->desc = copy_desc(d);
  return make_resident(c, std::move(s), id);
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

// ---------------------------------------------------------------------------------------
// snapshot tracing

// The candidate signatures of a trace, in the order of the new scene's rays: line of sight;
// 1..max_refl reflections; one diffraction with 0..max_refl_diff reflections, the edge at
// every position from first to last; scattering.
static std::vector<TraceSig> trace_signatures(const drt_trace_opts& o, int np, int ne, int nt) {
  std::vector<std::vector<int>> kinds;
  if (o.los) kinds.push_back({});
  for (int n = 1; n <= o.max_refl; ++n) kinds.push_back(std::vector<int>(n, DRT_R));
  for (int n = 0; n <= o.max_refl_diff; ++n)
    for (int d = 0; d <= n; ++d) {
      std::vector<int> k(n + 1, DRT_R);
      k[d] = DRT_D;
      kinds.push_back(k);
    }
  if (o.double_diff) kinds.push_back({DRT_D, DRT_D});
  if (o.scattering) kinds.push_back({DRT_S});
  std::vector<TraceSig> sigs;
  for (const auto& k : kinds) {
    TraceSig g{};
    g.n = int(k.size());
    uint8_t k8[DRT_MAX_INT] = {0, 0, 0, 0};
    g.count = 1;
    for (int i = 0; i < g.n; ++i) {
      g.kind[i] = k[i];
      k8[i] = uint8_t(k[i]);
      const bool repeat = i > 0 && k[i - 1] == k[i];     // consecutive walls (edges) differ
      g.radix[i] = (k[i] == DRT_R ? np : (k[i] == DRT_D ? ne : nt)) - (repeat ? 1 : 0);
      g.count = g.radix[i] > 0 ? g.count * g.radix[i] : 0;
    }
    int dpos;
    g.code = sig_code(g.n, k8, &dpos);
    sigs.push_back(g);
  }
  return sigs;
}

int drt_trace(drt_ctx* c, uint32_t scene, double t, const drt_trace_opts* o, uint32_t* new_scene,
              drt_trace_info* info) {
  Range range_("drt_trace");
  if (!c || !o || !new_scene) return fail(DRT_E_INVAL, "null context, options or output");
  if (!std::isfinite(t)) return fail(DRT_E_INVAL, "trace instant must be finite");
  if (o->max_refl < 0 || o->max_refl > 3 || o->max_refl_diff < -1 || o->max_refl_diff > 2)
    return fail(DRT_E_INVAL, "max_refl must be in 0..3 and max_refl_diff in -1..2");
  Scene* s = find_scene(c, scene);
  if (!s) return fail(DRT_E_NOTFOUND, "scene %u", scene);
  int st = set_device(c);
  if (st) return st;
  HostDesc d = rebase(s->desc, t);
  d.nr = 0;
  d.ray_nint.clear();
  d.ray_kind.clear();
  d.ray_pol.clear();
  d.ray_prim.clear();
  // the primitives at the traced instant, on the device
  Scene prim;
  {
    const drt_scene_desc dv = desc_view(d);
    if ((st = validate_and_pack(&dv, prim))) return st;
  }
  struct Bufs {
    drt_ctx* c;
    DevBuf planes, edges, tiles, sigs, counter, keys, vis, len;
    ~Bufs() {
      for (DevBuf* b : {&planes, &edges, &tiles, &sigs, &counter, &keys, &vis, &len}) dev_free(c, *b);
    }
  } B{c};
  const std::vector<TraceSig> sigs = trace_signatures(*o, d.np, d.ne, d.nt);
  if ((st = upload(c, B.planes, prim.planes.data(), prim.planes.size())) ||
      (st = upload(c, B.edges, prim.edges.data(), prim.edges.size())) ||
      (st = upload(c, B.tiles, prim.tiles.data(), prim.tiles.size())) ||
      (st = upload(c, B.sigs, sigs.data(), sigs.size())) || (st = dev_alloc(c, B.counter, 4)))
    return st;
  SceneView sv = prim.view;
  sv.planes = (const DPlane*)B.planes.p;
  sv.edges = (const DEdge*)B.edges.p;
  sv.tiles = (const DTile*)B.tiles.p;
  int64_t candidates = 0;
  for (const auto& g : sigs) candidates += g.count;
  const hipStream_t hs = nullptr;
  uint32_t cap = uint32_t(std::min<int64_t>(std::max<int64_t>(candidates, 1), int64_t(1) << 20)), n = 0;
  for (int pass = 0; pass < 2; ++pass) {
    dev_free(c, B.keys);
    if ((st = dev_alloc(c, B.keys, size_t(cap) * sizeof(uint64_t)))) return st;
    HIP_OK(launch_fill_i32((int32_t*)B.counter.p, 1, 0, hs));
    for (size_t i = 0; i < sigs.size(); ++i)
      HIP_OK(launch_trace_cand(sv, sigs[i], int(i), (uint64_t*)B.keys.p, cap, (uint32_t*)B.counter.p, hs));
    HIP_OK(hipMemcpy(&n, B.counter.p, 4, hipMemcpyDeviceToHost));
    if (n <= cap) break;
    if (pass == 1) return fail(DRT_E_DEVICE, "survivor count changed between identical passes");
    cap = n;    // rerun with room for every survivor
  }
  if ((st = dev_alloc(c, B.vis, std::max<size_t>(n, 1))) || (st = dev_alloc(c, B.len, std::max<size_t>(n, 1) * 8)))
    return st;
  HIP_OK(launch_trace_vis(sv, (const TraceSig*)B.sigs.p, (const uint64_t*)B.keys.p, n, d.np, (uint8_t*)B.vis.p,
                          (double*)B.len.p, hs));
  std::vector<uint64_t> keys(n);
  std::vector<uint8_t> vis(n);
  if (n) {
    HIP_OK(hipMemcpy(keys.data(), B.keys.p, size_t(n) * 8, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(vis.data(), B.vis.p, n, hipMemcpyDeviceToHost));
  }
  std::vector<uint64_t> found;
  for (uint32_t i = 0; i < n; ++i)
    if (vis[i]) found.push_back(keys[i]);
  std::sort(found.begin(), found.end());
  drt_trace_info inf{};
  inf.candidates = candidates;
  inf.geometric = n;
  d.nr = int32_t(found.size());
  d.ray_nint.assign(found.size(), 0);
  d.ray_kind.assign(4 * found.size(), 0);
  d.ray_pol.assign(4 * found.size(), 0);
  d.ray_prim.assign(4 * found.size(), 0);
  for (size_t r = 0; r < found.size(); ++r) {
    const TraceSig& g = sigs[found[r] >> 40];
    int32_t pr[DRT_MAX_INT];
    trace_decode(g, int64_t(found[r] & ((uint64_t(1) << 40) - 1)), pr);
    d.ray_nint[r] = uint8_t(g.n);
    for (int i = 0; i < g.n; ++i) {
      d.ray_kind[4 * r + i] = uint8_t(g.kind[i]);
      d.ray_prim[4 * r + i] = pr[i];
      int pol = DRT_PERP;
      if (g.kind[i] == DRT_R) pol = std::fabs(d.plane_n0[3 * pr[i] + 2]) > 0.5 ? DRT_PAR : DRT_PERP;
      if (g.kind[i] == DRT_D) pol = std::fabs(d.edge_e0[3 * pr[i] + 2]) > 0.5 ? DRT_PERP : DRT_PAR;
      d.ray_pol[4 * r + i] = uint8_t(pol);
    }
    inf.n_los += g.n == 0;
    inf.n_scat += g.n == 1 && g.kind[0] == DRT_S;
    bool has_d = false;
    for (int i = 0; i < g.n; ++i) has_d = has_d || g.kind[i] == DRT_D;
    inf.n_diff += has_d;
    inf.n_refl += g.n > 0 && g.kind[0] != DRT_S && !has_d;
  }
  inf.n_paths = d.nr;
  auto out = std::make_unique<Scene>();
  {
    const drt_scene_desc dv = desc_view(d);
    if ((st = validate_and_pack(&dv, *out))) return st;
  }
  out->desc = std::move(d);
  if ((st = make_resident(c, std::move(out), new_scene))) return st;
  if (info) *info = inf;
  return DRT_OK;
}

int drt_segments(drt_ctx* c, uint32_t scene, const drt_time_grid* tg, double f_c, const drt_trace_opts* topts,
                 const drt_refresh_opts* ropts, int32_t max_segments, int32_t* seg_start, int32_t* seg_len,
                 uint32_t* seg_scene, int32_t* n_segments) {
  Range range_("drt_segments");
  if (!c || !tg || !topts || !ropts || !n_segments || (max_segments > 0 && (!seg_start || !seg_len || !seg_scene)))
    return fail(DRT_E_INVAL, "null argument");
  if (tg->n_steps < 0 || !(tg->dt > 0) || !std::isfinite(tg->dt)) return fail(DRT_E_INVAL, "bad time grid");
  if (!(f_c > 0)) return fail(DRT_E_INVAL, "carrier must be > 0");
  if (!(ropts->threshold_db >= 0) || ropts->max_steps < 1 || ropts->min_steps < 1 ||
      ropts->min_steps > ropts->max_steps)
    return fail(DRT_E_INVAL, "need threshold_db >= 0 and 1 <= min_steps <= max_steps");
  if (!find_scene(c, scene)) return fail(DRT_E_NOTFOUND, "scene %u", scene);
  int st = set_device(c);
  if (st) return st;
  std::vector<uint32_t> made;
  auto undo = [&](int code) {
    const std::string msg = g_last_error;
    for (uint32_t id : made) (void)drt_unload_scene(c, id);
    g_last_error = msg;
    return code;
  };
  const int T = tg->n_steps;
  int j = 0, k = 0;
  while (j < T) {
    if (k == max_segments) return undo(fail(DRT_E_INVAL, "more than %d segments", max_segments));
    uint32_t sid = 0;
    drt_trace_info inf{};
    if ((st = drt_trace(c, scene, double(j) * tg->dt, topts, &sid, &inf))) return undo(st);
    made.push_back(sid);
    const int m = std::min(ropts->max_steps, T - j);
    int len = m;
    const int R = inf.n_paths;
    if (R > 0) {
      DevBuf gain, fo;
      struct Free {
        drt_ctx* c;
        DevBuf *a, *b;
        ~Free() { dev_free(c, *a), dev_free(c, *b); }
      } fr{c, &gain, &fo};
      if ((st = dev_alloc(c, gain, size_t(R) * 16)) || (st = dev_alloc(c, fo, size_t(R) * 4))) return undo(st);
      drt_ray_out o1{}, om{};
      o1.gain = gain.p;
      om.first_out = (int32_t*)fo.p;
      const drt_time_grid t1{tg->dt, 1}, tm{tg->dt, m};
      if ((st = drt_extrapolate(c, sid, R, &t1, f_c, DRT_FP64, &o1, nullptr)) ||
          (st = drt_extrapolate(c, sid, R, &tm, f_c, DRT_FP64, &om, nullptr)))
        return undo(st);
      std::vector<double> g(2 * size_t(R));
      std::vector<int32_t> f(R);
      if (hipMemcpy(g.data(), gain.p, size_t(R) * 16, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(f.data(), fo.p, size_t(R) * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return undo(fail(DRT_E_DEVICE, "copying the monitor's results"));
      double pmax = 0;
      for (int r = 0; r < R; ++r) pmax = std::max(pmax, g[2 * r] * g[2 * r] + g[2 * r + 1] * g[2 * r + 1]);
      const double floor_p = pmax * std::pow(10.0, -ropts->threshold_db / 10.0);
      int first = m;
      for (int r = 0; r < R; ++r)
        if (g[2 * r] * g[2 * r] + g[2 * r + 1] * g[2 * r + 1] >= floor_p) first = std::min(first, f[r]);
      len = std::min(m, std::max(ropts->min_steps, first));
    }
    seg_start[k] = j;
    seg_len[k] = len;
    seg_scene[k] = sid;
    ++k;
    j += len;
  }
  *n_segments = k;
  return DRT_OK;
}

int drt_scene_rays(drt_ctx* c, uint32_t scene, int32_t cap, int32_t* n_rays, uint8_t* nint, uint8_t* kind,
                   int32_t* prim, uint8_t* pol) {
  if (!c || !n_rays || cap < 0) return fail(DRT_E_INVAL, "null context or count, or negative capacity");
  Scene* s = find_scene(c, scene);
  if (!s) return fail(DRT_E_NOTFOUND, "scene %u", scene);
  const HostDesc& h = s->desc;
  *n_rays = h.nr;
  const size_t m = size_t(std::min(cap, h.nr));
  if (nint && m) std::memcpy(nint, h.ray_nint.data(), m);
  if (kind && m) std::memcpy(kind, h.ray_kind.data(), 4 * m);
  if (prim && m) std::memcpy(prim, h.ray_prim.data(), 16 * m);
  if (pol && m) std::memcpy(pol, h.ray_pol.data(), 4 * m);
  return DRT_OK;
}

int drt_extrapolate(drt_ctx* c, uint32_t scene, int32_t n_rays, const drt_time_grid* tg, double f_c,
                    int32_t prec, const drt_ray_out* out, void* stream) {
  Range range_("drt_extrapolate");
  if (!c || !out) return fail(DRT_E_INVAL, "null context or output");
  Scene* s = find_scene(c, scene);
  if (!s) return fail(DRT_E_NOTFOUND, "scene %u", scene);
  int st;
  if ((st = check_grid(tg, n_rays, *s)) || (st = check_prec(prec, s))) return st;
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

int drt_power_profiles(drt_ctx* c, uint32_t scene, int32_t n_rays, const drt_time_grid* tg, double f_c,
                       int32_t prec, const drt_bins* bins, const drt_power_out* out, void* stream) {
  Range range_("drt_power_profiles");
  if (!c || !bins || !out) return fail(DRT_E_INVAL, "null context, bins or output");
  Scene* s = find_scene(c, scene);
  if (!s) return fail(DRT_E_NOTFOUND, "scene %u", scene);
  int st;
  if ((st = check_grid(tg, n_rays, *s)) || (st = check_prec(prec, s))) return st;
  if (!(f_c > 0)) return fail(DRT_E_INVAL, "carrier must be > 0");
  if (bins->steps_per_bin < 1) return fail(DRT_E_INVAL, "steps_per_bin must be >= 1");
  if (!(bins->dop_step > 0) || !(bins->delay_step > 0) || !std::isfinite(bins->dop_lo) ||
      !std::isfinite(bins->delay_lo) || !std::isfinite(bins->dop_step) || !std::isfinite(bins->delay_step))
    return fail(DRT_E_INVAL, "bin origins must be finite and steps finite and > 0");
  if (bins->n_dop < 0 || bins->n_delay < 0) return fail(DRT_E_INVAL, "negative bin count");
  const int T = tg->n_steps;
  const int64_t n_tb = (int64_t(T) + bins->steps_per_bin - 1) / bins->steps_per_bin;
  if (n_tb * bins->n_dop > INT32_MAX || n_tb * bins->n_delay > INT32_MAX)
    return fail(DRT_E_INVAL, "more than 2^31 - 1 profile bins");
  double* pdfp = bins->n_dop > 0 ? out->pdfp : nullptr;
  double* pdp = bins->n_delay > 0 ? out->pdp : nullptr;
  if (n_tb > 0 && ((bins->n_dop > 0 && !pdfp) || (bins->n_delay > 0 && !pdp)))
    return fail(DRT_E_INVAL, "null profile output with a nonzero bin count");
  if ((st = set_device(c))) return st;
  hipStream_t hs = (hipStream_t)stream;
  if (n_tb == 0) return DRT_OK;
  if (pdfp) HIP_OK(launch_zero(pdfp, size_t(n_tb) * bins->n_dop * sizeof(double), hs));
  if (pdp) HIP_OK(launch_zero(pdp, size_t(n_tb) * bins->n_delay * sizeof(double), hs));
  if (out->total) HIP_OK(launch_zero(out->total, size_t(n_tb) * sizeof(double), hs));
  if (n_rays == 0 || (!pdfp && !pdp && !out->total)) return DRT_OK;
  std::lock_guard<std::mutex> g(c->scratch_mu);
  Scratch& sc = c->scratch[hs];
  if ((st = ensure_scratch(c, sc, pose_bytes(s->view.n_bodies, T, prec), hs))) return st;
  const RayClasses rc = classes(*s, n_rays);
  HIP_OK(timed(c, DRT_K_POSE, hs, [&] {
    return launch_pose((const DBody*)s->d_bodies.p, s->view.n_bodies, T, tg->dt, prec, sc.buf.p, hs);
  }));
  ExtrapOut eo{};
  eo.pdfp = pdfp;
  eo.pdp = pdp;
  eo.ptotal = out->total;
  eo.dop_lo = bins->dop_lo;
  eo.dop_step = bins->dop_step;
  eo.delay_lo = bins->delay_lo;
  eo.delay_step = bins->delay_step;
  eo.spb = bins->steps_per_bin;
  eo.n_dop = bins->n_dop;
  eo.n_delay = bins->n_delay;
  eo.gate = bins->in_bounds_only != 0;
  HIP_OK(timed(c, DRT_K_GEOM, hs, [&] {
    return launch_geom(device_view(*s), rc, sc.buf.p, T, tg->dt, f_c, n_rays, prec, GEOM_POWER, eo, nullptr,
                       AnchorParams{0.0, 0.0, 0.0}, hs);
  }, class_kernels(rc, T)));
  return DRT_OK;
}

int drt_cfr(drt_ctx* c, uint32_t scene, int32_t n_rays, const drt_time_grid* tg, const drt_freq_grid* fg,
            int32_t prec, void* H, void* stream) {
  Range range_("drt_cfr");
  if (!c) return fail(DRT_E_INVAL, "null context");
  Scene* s = find_scene(c, scene);
  if (!s) return fail(DRT_E_NOTFOUND, "scene %u", scene);
  int st;
  if ((st = check_grid(tg, n_rays, *s)) || (st = check_fgrid(fg)) || (st = check_prec(prec, s))) return st;
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

int drt_cfr_noalloc(drt_ctx* c, uint32_t scene, int32_t n_rays, const drt_time_grid* tg,
                    const drt_freq_grid* fg, int32_t prec, void* H, void* stream) {
  Range range_("drt_cfr_noalloc");
  if (!c) return fail(DRT_E_INVAL, "null context");
  Scene* s = find_scene(c, scene);
  if (!s) return fail(DRT_E_NOTFOUND, "scene %u", scene);
  int st;
  if ((st = check_grid(tg, n_rays, *s)) || (st = check_fgrid(fg)) || (st = check_prec(prec, s))) return st;
  if (tg->n_steps > 0 && fg->n_sub > 0 && !H) return fail(DRT_E_INVAL, "null H");
  if ((st = set_device(c))) return st;
  const int T = tg->n_steps, K = fg->n_sub;
  if (T == 0 || K == 0) return DRT_OK;
  hipStream_t hs = (hipStream_t)stream;
  if (n_rays == 0) {
    HIP_OK(launch_zero(H, size_t(T) * K * (prec == DRT_FP64 ? 16 : 8), hs));
    return DRT_OK;
  }
  const CfrPlan p = plan(c, *s, n_rays, T, fg, prec);
  if (p.total > kNoAllocBytes)
    return fail(DRT_E_NOMEM, "drt_cfr_noalloc needs %zu bytes of scratch; its static scratch holds %zu",
                p.total, kNoAllocBytes);
  void* base = noalloc_ptr[c->device];
  if (!base) return fail(DRT_E_DEVICE, "static scratch of device %d not set up", c->device);
  // every scratch byte the kernels read is written first in the same call (pose table,
  // records, partial sums): nothing to clear; no kernel timing (no event creation)
  return run_cfr(nullptr, *s, n_rays, tg, fg, prec, H, p, base, hs);
}

int drt_cfr_nufft(drt_ctx* c, uint32_t scene, int32_t n_rays, const drt_time_grid* tg, const drt_freq_grid* fg,
                  double eps, void* H, void* stream) {
  Range range_("drt_cfr_nufft");
  if (!c) return fail(DRT_E_INVAL, "null context");
  Scene* s = find_scene(c, scene);
  if (!s) return fail(DRT_E_NOTFOUND, "scene %u", scene);
  int st;
  if ((st = check_grid(tg, n_rays, *s)) || (st = check_fgrid(fg))) return st;
  if (!(eps >= 1e-15 && eps <= 1e-1)) return fail(DRT_E_INVAL, "eps must be in [1e-15, 1e-1]");
  if (fg->n_sub > 2048) return fail(DRT_E_INVAL, "n_sub %d above 2048", fg->n_sub);
  const int T = tg->n_steps, K = fg->n_sub;
  if (T == 0 || K == 0) return DRT_OK;
  if (!H) return fail(DRT_E_INVAL, "null H");
  if ((st = set_device(c))) return st;
  hipStream_t hs = (hipStream_t)stream;
  if (n_rays == 0) {
    HIP_OK(launch_zero(H, size_t(T) * K * 16, hs));
    return DRT_OK;
  }
  const int w = std::min(16, std::max(2, int(std::ceil(-std::log10(eps))) + 1));
  int M = 1;
  while (M < 2 * K || M < 2 * w) M *= 2;    // a kernel footprint wraps the grid at most once
  const double beta = 2.30 * w;
  const size_t pb = (pose_bytes(s->view.n_bodies, T, DRT_FP64) + 255) / 256 * 256;
  const size_t rb = (size_t(T) * n_rays * sizeof(RecU) + 255) / 256 * 256;
  const size_t tb = (size_t(M / 2) * 16 + 255) / 256 * 256;
  std::lock_guard<std::mutex> g(c->scratch_mu);
  Scratch& sc = c->scratch[hs];
  const size_t kb = (size_t(K) * 8 + 255) / 256 * 256;
  if ((st = ensure_scratch(c, sc, pb + rb + tb + kb + 64 * 16, hs))) return st;
  char* base = (char*)sc.buf.p;
  HIP_OK(timed(c, DRT_K_POSE, hs, [&] {
    return launch_pose((const DBody*)s->d_bodies.p, s->view.n_bodies, T, tg->dt, DRT_FP64, base, hs);
  }));
  const double inv_c = 1.0 / 299792458.0, df = fg->bandwidth / K;
  const RayClasses rc = classes(*s, n_rays);
  ExtrapOut none{};
  HIP_OK(timed(c, DRT_K_GEOM, hs, [&] {
    return launch_geom(device_view(*s), rc, base, T, tg->dt, fg->f_c, n_rays, DRT_FP64, GEOM_NUFFT, none, base + pb,
                       AnchorParams{fg->f_c * inv_c, 0.0, df * inv_c}, hs);
  }, class_kernels(rc, T)));
  HIP_OK(timed(c, DRT_K_CFR, hs, [&] {
    return launch_nufft((const RecU*)(base + pb), n_rays, T, K, M, w, beta, (double2*)(base + pb + rb),
                        (double*)(base + pb + rb + tb), (double2*)(base + pb + rb + tb + kb), (double2*)H, hs);
  }, 3));
  return DRT_OK;
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
  Range range_("drt_submit");
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
  const bool empty = r->tg.n_steps == 0 || r->fg.n_sub == 0;   // nothing to write
  q->footprint = (!empty && r->n_rays > 0) ? plan(c, *s, r->n_rays, r->tg.n_steps, &r->fg, r->precision).total : 0;
  size_t resident = 0;
  for (auto& kv : c->scenes) resident += kv.second->bytes;
  if (q->footprint + resident > c->cap)
    return fail(DRT_E_ADMISSION, "request footprint %zu bytes exceeds the cap %llu minus resident scenes",
                q->footprint, (unsigned long long)c->cap);
  q->ticket = c->next_ticket++;
  *ticket = q->ticket;
  s->inflight++;
  if (empty) {
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
