// Host launchers of the geometry kernels in the kinematics (second-order jets), power-profile
// and non-uniform-FFT record modes.
#include "dev_geom.h"
#include "dev_geom_launch.h"

namespace drt {

hipError_t launch_geom_more(const SceneView& sc, const RayClasses& rc, const void* pose, int T, double dt,
                            double f_c, int n_rays, int prec, int mode, const ExtrapOut& eo, void* rec,
                            const AnchorParams& ap, hipStream_t st) {
  if (mode == GEOM_KIN)
    return launch_geom_mode<GEOM_KIN>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  if (mode == GEOM_POWER)
    return launch_geom_mode<GEOM_POWER>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  if (mode == GEOM_NUFFT)
    return launch_geom_mode<GEOM_NUFFT>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  return hipErrorInvalidValue;
}

}  // namespace drt
