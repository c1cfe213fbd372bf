// Host-side templates that launch the geometry kernel of one mode for every signature class
// and precision (shared by the translation units that instantiate the modes).
#ifndef DRT_DEV_GEOM_LAUNCH_H
#define DRT_DEV_GEOM_LAUNCH_H

#include "dev_geom.h"

namespace drt {

template <class F, int MODE, int PREC, bool POL>
static void launch_classes(const SceneView& sc, const RayClasses& rc, const void* pose, int T, double dt,
                           double f_c, int n_rays, const ExtrapOut& eo, void* rec, const AnchorParams& ap,
                           hipStream_t st) {
  using P = const typename Vec2<F>::type*;
  int nchunk = (T + 63) / 64;
  if constexpr (MODE == GEOM_ANCHOR || MODE == GEOM_ANCHOR_MFMA) {
    if (geom_merged(rc, T)) {
      int n = 0;
      for (int c = 0; c < CLS_COUNT; ++c) n += class_workgroups(rc, c, T);
      if (n > 0)
        hipLaunchKernelGGL((k_geom_merged<F, MODE, PREC, POL>), dim3(unsigned(n)), dim3(256), 0, st, sc, rc, (P)pose,
                           T, dt, f_c, n_rays, nchunk, eo, rec, ap);
      return;
    }
  }
  for (int c = 0; c < CLS_COUNT; ++c) {
    if (rc.count[c] == 0) continue;
    dim3 grid(unsigned(long((rc.count[c] + 3) / 4) * nchunk));   // 4 rays x 64 instants per workgroup
    if (c == CLS_R)
      hipLaunchKernelGGL((k_geom<F, MODE, PREC, CLS_R, POL>), grid, dim3(256), 0, st, sc, rc.order[c], rc.count[c],
                         (P)pose, T, dt, f_c, n_rays, nchunk, eo, rec, ap);
    else if (c == CLS_D)
      hipLaunchKernelGGL((k_geom<F, MODE, PREC, CLS_D, POL>), grid, dim3(256), 0, st, sc, rc.order[c], rc.count[c],
                         (P)pose, T, dt, f_c, n_rays, nchunk, eo, rec, ap);
    else
      hipLaunchKernelGGL((k_geom<F, MODE, PREC, CLS_S, POL>), grid, dim3(256), 0, st, sc, rc.order[c], rc.count[c],
                         (P)pose, T, dt, f_c, n_rays, nchunk, eo, rec, ap);
  }
}

// The precision instances of one mode; POL: polarimetric field coefficients (dipoles),
// available in binary64 and split precision.
template <int MODE, bool POL>
static void launch_geom_prec(const SceneView& sc, const RayClasses& rc, const void* pose, int T, double dt,
                             double f_c, int n_rays, int prec, const ExtrapOut& eo, void* rec,
                             const AnchorParams& ap, hipStream_t st) {
  if constexpr (MODE == GEOM_ANCHOR_MFMA) {
    if (prec == DRT_FP64)
      launch_classes<double, MODE, DRT_FP64, POL>(sc, rc, pose, T, dt, f_c, n_rays, eo, rec, ap, st);
    else
      launch_classes<double, MODE, DRT_SPLIT, POL>(sc, rc, pose, T, dt, f_c, n_rays, eo, rec, ap, st);
  } else if constexpr (MODE == GEOM_NUFFT) {
    launch_classes<double, MODE, DRT_FP64, POL>(sc, rc, pose, T, dt, f_c, n_rays, eo, rec, ap, st);
  } else if constexpr (MODE == GEOM_KIN) {
    (void)prec;   // jets in binary64 whatever the call's precision (binary64 pose table); no field
    launch_classes<double, MODE, DRT_FP64, false>(sc, rc, pose, T, dt, f_c, n_rays, eo, rec, ap, st);
  } else {
    if (prec == DRT_FP64)
      launch_classes<double, MODE, DRT_FP64, POL>(sc, rc, pose, T, dt, f_c, n_rays, eo, rec, ap, st);
    else if (prec == DRT_SPLIT)
      launch_classes<double, MODE, DRT_SPLIT, POL>(sc, rc, pose, T, dt, f_c, n_rays, eo, rec, ap, st);
    else if constexpr (!POL)
      launch_classes<float, MODE, DRT_NAIVE32, false>(sc, rc, pose, T, dt, f_c, n_rays, eo, rec, ap, st);
  }
}

template <int MODE>
static hipError_t launch_geom_mode(const SceneView& sc, const RayClasses& rc, const void* pose, int T, double dt,
                                   double f_c, int n_rays, int prec, const ExtrapOut& eo, void* rec,
                                   const AnchorParams& ap, hipStream_t st) {
  if (sc.polar && MODE != GEOM_KIN) {
    if (prec == DRT_NAIVE32 && MODE != GEOM_ANCHOR_MFMA && MODE != GEOM_NUFFT) return hipErrorInvalidValue;
    launch_geom_prec<MODE, true>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  } else {
    launch_geom_prec<MODE, false>(sc, rc, pose, T, dt, f_c, n_rays, prec, eo, rec, ap, st);
  }
  return hipGetLastError();
}

}  // namespace drt

#endif  // DRT_DEV_GEOM_LAUNCH_H
