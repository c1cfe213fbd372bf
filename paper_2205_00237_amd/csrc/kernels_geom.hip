// Host launchers of the body poses and of the geometry kernels in the modes the ray sums and
// drt_extrapolate use (extrapolation outputs, ray-sum records); the other modes are
// instantiated in kernels_geom_more.hip.
#include "dev_geom.h"
#include "dev_geom_launch.h"

namespace drt {

hipError_t launch_pose(const DBody* bodies, int nb, int T, double dt, int prec, void* out, hipStream_t st) {
  int n = nb * T;
  if (n == 0) return hipSuccess;
  dim3 grid((n + 255) / 256);
  if (prec == DRT_NAIVE32)
    hipLaunchKernelGGL(k_pose<float>, grid, dim3(256), 0, st, bodies, nb, T, dt, (float2*)out);
  else
    hipLaunchKernelGGL(k_pose<double>, grid, dim3(256), 0, st, bodies, nb, T, dt, (double2*)out);
  return hipGetLastError();
}


hipError_t launch_geom_more(const SceneView& sc, const RayClasses& rc, const void* pose, int T, double dt,
                            double f_c, int n_rays, int prec, int mode, const ExtrapOut& eo, void* rec,
                            const AnchorParams& ap, hipStream_t st);

hipError_t launch_geom(const SceneView& sc, const RayClasses& rc, const void* pose, int T, double dt, double f_c,
                       int n_rays, int prec, int mode, const ExtrapOut& eo, void* rec, const AnchorParams& ap,
                       hipStream_t st) {
  if (n_rays == 0 || T == 0) return hipSuccess;
  if (mode == GEOM_EXTRAP)
    return launch_geom_mode<GEOM_EXTRAP>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  if (mode == GEOM_ANCHOR_MFMA)
    return launch_geom_mode<GEOM_ANCHOR_MFMA>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  if (mode == GEOM_ANCHOR)
    return launch_geom_mode<GEOM_ANCHOR>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  return launch_geom_more(sc, rc, pose, T, dt, f_c, n_rays, prec, mode, eo, rec, ap, st);
}

}  // namespace drt
