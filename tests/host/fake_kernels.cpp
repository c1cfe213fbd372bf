// Host stand-ins for the library's kernel launchers, for the ThreadSanitizer build of the
// host code on a machine without a GPU (with tests/host/fake_hip): launches do no work
// except the fills, and a batch launch on a captured stream records its graph node.
#include <cstring>

#include "drt_kernels.h"

namespace drt {

static char g_batch_kernels[BK_COUNT];   // distinct addresses standing for the batch kernels

void* batch_kernel(int kind) { return kind >= 0 && kind < BK_COUNT ? &g_batch_kernels[kind] : nullptr; }

hipError_t launch_batch(int kind, const BatchDesc*, int, hipStream_t st) {
  fake_capture_launch(st, kind);
  return hipSuccess;
}
hipError_t launch_pose(const DBody*, int, int, double, int, void*, hipStream_t) { return hipSuccess; }
hipError_t launch_geom(const SceneView&, const RayClasses&, const void*, int, double, double, int, int, int,
                       const ExtrapOut&, void*, const AnchorParams&, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_cfr(const void*, const CfrArgs&, int, void*, hipStream_t) { return hipSuccess; }
hipError_t launch_zero(void* p, size_t bytes, hipStream_t) {
  std::memset(p, 0, bytes);
  return hipSuccess;
}
hipError_t launch_fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t) {
  for (size_t i = 0; i < n; ++i) p[i] = v;
  return hipSuccess;
}
hipError_t launch_reduce(const void*, int, size_t, int, void*, hipStream_t) { return hipSuccess; }
hipError_t launch_nufft(const RecU*, int, int, int, int, int, double, double2*, double*, double2*, double2*,
                        hipStream_t) {
  return hipSuccess;
}
hipError_t launch_trace_cand(const SceneView&, const TraceSig&, int, uint64_t*, uint32_t, uint32_t*, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_trace_vis(const SceneView&, const TraceSig*, const uint64_t*, uint32_t, int, uint8_t*, double*,
                            hipStream_t) {
  return hipSuccess;
}

}  // namespace drt

void* fake_batch_kernel_of(int kind) { return drt::batch_kernel(kind); }
