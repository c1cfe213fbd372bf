// Batched serving kernels: one launch per kernel kind over the work items of every request
// in a batch (poses, geometry per signature class, binary16 ray sum per tile shape, reduction).
#include "dev_cfr.h"
#include "dev_geom.h"

namespace drt {

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
  __shared__ typename Cfr16Lds<MT, NT>::type lds;
  const int n = bd->n_req;
  const long long* off = bd->off[BK_CFR + (NT == 1 ? 0 : (NT == 2 ? 1 : (MT == 1 ? 2 : (MT == 2 ? 3 : 4))))];
  const long long it = blockIdx.x;
  if (it >= off[n]) return;
  const int j = __builtin_amdgcn_readfirstlane(req_of_uniform(off, n, it));
  const BatchReq& q = bd->req[j];
  const CfrArgs a = q.a;
  cfr16_tile<MT, NT>((const RecM*)q.rec, a, a.G > 1 ? q.part : q.H, int(it - off[j]), lds);
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

}  // namespace drt
