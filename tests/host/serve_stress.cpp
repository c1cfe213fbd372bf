// Concurrency stress of the serving loop through the C ABI, for a ThreadSanitizer build of the
// library's host code: submitter threads, a poller, a caller of drt_cfr and drt_extrapolate
// on its own stream and the scheduler thread all run at once; every served H is then compared
// bit for bit with drt_cfr of the same request, and a context is destroyed with requests
// still queued.  Exit status 0 when every check passes.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "drt.h"

namespace {

#define CHECK(cond, ...)                                                        \
  do {                                                                          \
    if (!(cond)) {                                                              \
      std::fprintf(stderr, "check failed at line %d: ", __LINE__);             \
      std::fprintf(stderr, __VA_ARGS__);                                        \
      std::fprintf(stderr, "\n");                                               \
      std::exit(1);                                                             \
    }                                                                           \
  } while (0)

// A street corner: ground, two building walls, a turning and driving truck side; a moving
// transmitter.  Rays: line of sight, four single and two double reflections.
struct Scene {
  std::vector<double> O0, v0, a, axis, w0, wdot, eps, sig, pp, pn;
  std::vector<uint8_t> pec, nint, kind, pol;
  std::vector<int32_t> pbody, pmat, prim;
  drt_scene_desc d{};
  Scene() {
    O0 = {0, 0, 0, 60, 5, 0};
    v0 = {0, 0, 0, -4, 0, 0};
    a = {0, 0, 0, 0, 0, 0};
    axis = {0, 0, 1, 0, 0, 1};
    w0 = {0, 0.05};
    wdot = {0, 0};
    eps = {5.0, 4.0};
    sig = {0.01, 0.02};
    pec = {0, 1};
    // ground z = 0, wall x = 30, wall y = 12, truck side x = 58 (body 1)
    pp = {0, 0, 0, 30, 0, 0, 0, 12, 0, 58, 5, 1};
    pn = {0, 0, 1, -1, 0, 0, 0, -1, 0, -1, 0, 0};
    pbody = {0, 0, 0, 1};
    pmat = {0, 0, 0, 1};
    const int rays[7][3] = {{0, -1, -1}, {1, 0, -1}, {1, 1, -1}, {1, 2, -1}, {1, 3, -1}, {2, 0, 1}, {2, 2, 1}};
    for (auto& r : rays) {
      nint.push_back(uint8_t(r[0]));
      for (int i = 0; i < 4; ++i) {
        const bool used = i < r[0];
        kind.push_back(used ? DRT_R : 0);
        pol.push_back(used ? uint8_t(i & 1) : 0);
        prim.push_back(used ? r[1 + i] : 0);
      }
    }
    const double tx[3] = {0, 0, 1.5}, txv[3] = {10, 0, 0}, rx[3] = {20, 2, 1.5};
    std::memcpy(d.tx_p, tx, 24);
    std::memcpy(d.tx_v, txv, 24);
    std::memcpy(d.rx_p, rx, 24);
    d.n_bodies = 2;
    d.body_O0 = O0.data();
    d.body_v0 = v0.data();
    d.body_a = a.data();
    d.body_axis = axis.data();
    d.body_w0 = w0.data();
    d.body_wdot = wdot.data();
    d.n_mat = 2;
    d.mat_eps_r = eps.data();
    d.mat_sigma = sig.data();
    d.mat_pec = pec.data();
    d.n_planes = 4;
    d.plane_body = pbody.data();
    d.plane_mat = pmat.data();
    d.plane_p0 = pp.data();
    d.plane_n0 = pn.data();
    d.n_rays = int32_t(nint.size());
    d.ray_nint = nint.data();
    d.ray_kind = kind.data();
    d.ray_pol = pol.data();
    d.ray_prim = prim.data();
  }
};

struct Job {
  drt_request r;
  uint64_t ticket = 0;
  int state = 0;
};

size_t h_bytes(const drt_request& r) {
  return size_t(r.tg.n_steps) * r.fg.n_sub * (r.precision == DRT_FP64 ? 16 : 8);
}

drt_request random_request(std::mt19937& g, uint32_t scene, int n_rays) {
  static const int Ks[4] = {64, 200, 512, 1024};
  drt_request r{};
  r.scene = scene;
  r.n_rays = 1 + int(g() % unsigned(n_rays));
  r.tg = drt_time_grid{1e-3, int32_t(10 + g() % 200)};
  r.fg = drt_freq_grid{28e9, 100e6, Ks[g() % 4]};
  r.precision = (g() % 4 == 0) ? DRT_FP64 : DRT_SPLIT;
  CHECK(hipMalloc(&r.H, h_bytes(r)) == hipSuccess, "hipMalloc");
  return r;
}

}  // namespace

int main() {
  Scene sc;
  drt_ctx* ctx = nullptr;
  CHECK(drt_create(0, 0, &ctx) == DRT_OK, "drt_create: %s", drt_last_error());
  uint32_t s1 = 0, s2 = 0;
  CHECK(drt_load_scene(ctx, &sc.d, &s1) == DRT_OK, "load: %s", drt_last_error());
  CHECK(drt_load_scene(ctx, &sc.d, &s2) == DRT_OK, "load: %s", drt_last_error());

  constexpr int kSubmitters = 3, kPerSubmitter = 30;
  std::vector<Job> jobs(kSubmitters * kPerSubmitter);
  std::mutex jobs_mu;
  std::atomic<int> submitted{0};
  std::vector<std::thread> threads;
  for (int s = 0; s < kSubmitters; ++s) {
    threads.emplace_back([&, s] {
      std::mt19937 g(1234 + s);
      for (int i = 0; i < kPerSubmitter; ++i) {
        Job j;
        j.r = random_request(g, (i & 1) ? s1 : s2, sc.d.n_rays);
        CHECK(drt_submit(ctx, &j.r, &j.ticket) == DRT_OK, "submit: %s", drt_last_error());
        {
          std::lock_guard<std::mutex> l(jobs_mu);
          jobs[s * kPerSubmitter + i] = j;
        }
        submitted++;
        std::this_thread::sleep_for(std::chrono::microseconds(g() % 300));
      }
    });
  }
  std::atomic<bool> poll_done{false};
  threads.emplace_back([&] {   // poller
    int done = 0;
    while (done < int(jobs.size())) {
      done = 0;
      for (size_t k = 0; k < jobs.size(); ++k) {
        uint64_t t;
        int st;
        {
          std::lock_guard<std::mutex> l(jobs_mu);
          t = jobs[k].ticket;
          st = jobs[k].state;
        }
        if (t == 0) continue;
        if (st == 2 || st < 0) {
          ++done;
          continue;
        }
        drt_req_stat rs;
        const int p = drt_poll(ctx, t, &rs);
        CHECK(p == DRT_OK, "poll: %s", drt_last_error());
        if (rs.state == 2 || rs.state < 0) {
          std::lock_guard<std::mutex> l(jobs_mu);
          jobs[k].state = rs.state;
        }
      }
      drt_serving_stats stats;
      CHECK(drt_serving_stats_get(ctx, &stats) == DRT_OK, "stats");
      std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    poll_done = true;
  });
  threads.emplace_back([&] {   // a direct caller on its own stream, concurrent with the serving
    hipStream_t st;
    CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess, "stream");
    const drt_time_grid tg{1e-3, 150};
    const drt_freq_grid fg{28e9, 100e6, 256};
    void* H = nullptr;
    double* L = nullptr;
    CHECK(hipMalloc(&H, size_t(tg.n_steps) * fg.n_sub * 8) == hipSuccess, "hipMalloc");
    CHECK(hipMalloc((void**)&L, size_t(tg.n_steps) * sc.d.n_rays * 8) == hipSuccess, "hipMalloc");
    drt_ray_out out{};
    out.L = L;
    for (int i = 0; i < 20; ++i) {
      CHECK(drt_cfr(ctx, s1, sc.d.n_rays, &tg, &fg, DRT_SPLIT, H, st) == DRT_OK, "cfr: %s", drt_last_error());
      CHECK(drt_extrapolate(ctx, s2, sc.d.n_rays, &tg, 28e9, DRT_SPLIT, &out, st) == DRT_OK, "extrapolate: %s",
            drt_last_error());
    }
    CHECK(hipStreamSynchronize(st) == hipSuccess, "sync");
    CHECK(hipFree(H) == hipSuccess && hipFree(L) == hipSuccess, "free");
    CHECK(hipStreamDestroy(st) == hipSuccess, "stream destroy");
  });
  for (auto& t : threads) t.join();
  CHECK(poll_done.load(), "poller did not finish");

  // every served H equals drt_cfr of the same request, bit for bit
  hipStream_t st;
  CHECK(hipStreamCreate(&st) == hipSuccess, "stream");
  int compared = 0;
  for (Job& j : jobs) {
    CHECK(j.state == 2, "ticket %llu ended in state %d", (unsigned long long)j.ticket, j.state);
    const size_t nb = h_bytes(j.r);
    void* ref = nullptr;
    CHECK(hipMalloc(&ref, nb) == hipSuccess, "hipMalloc");
    CHECK(drt_cfr(ctx, j.r.scene, j.r.n_rays, &j.r.tg, &j.r.fg, j.r.precision, ref, st) == DRT_OK, "cfr: %s",
          drt_last_error());
    CHECK(hipStreamSynchronize(st) == hipSuccess, "sync");
    std::vector<unsigned char> a(nb), b(nb);
    CHECK(hipMemcpy(a.data(), j.r.H, nb, hipMemcpyDeviceToHost) == hipSuccess, "copy");
    CHECK(hipMemcpy(b.data(), ref, nb, hipMemcpyDeviceToHost) == hipSuccess, "copy");
    CHECK(std::memcmp(a.data(), b.data(), nb) == 0, "served H differs from drt_cfr (ticket %llu)",
          (unsigned long long)j.ticket);
    CHECK(hipFree(ref) == hipSuccess && hipFree(j.r.H) == hipSuccess, "free");
    ++compared;
  }
  CHECK(hipStreamDestroy(st) == hipSuccess, "stream destroy");

  // a context destroyed with requests queued: they are cancelled and destroy returns
  std::mt19937 g(99);
  std::vector<void*> bufs;
  for (int i = 0; i < 12; ++i) {
    drt_request r = random_request(g, s1, sc.d.n_rays);
    uint64_t t;
    CHECK(drt_submit(ctx, &r, &t) == DRT_OK, "submit: %s", drt_last_error());
    bufs.push_back(r.H);
  }
  CHECK(drt_destroy(ctx) == DRT_OK, "destroy: %s", drt_last_error());
  CHECK(hipDeviceSynchronize() == hipSuccess, "sync");
  for (void* p : bufs) CHECK(hipFree(p) == hipSuccess, "free");
  std::printf("serve_stress: %d served requests equal to drt_cfr; destroy with a queue returned\n", compared);
  return 0;
}
