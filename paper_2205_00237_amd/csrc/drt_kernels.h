// Launchers of the gfx950 kernels (kernels.hip) used by the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "drt_layout.h"

namespace drt {

enum GeomMode { GEOM_EXTRAP = 0, GEOM_ANCHOR = 1, GEOM_ANCHOR_MFMA = 2 };
enum CfrPath { CFR_VALU = 0, CFR_MFMA = 1, CFR_MFMA16 = 2 };

constexpr int kNK = 16;          // subcarriers walked by one lane from its phase anchor
constexpr int kMinSlice = 8;     // fewest rays per wave slice of the ray sum

struct ExtrapOut {
  double* L;
  float *dop, *aod_az, *aod_el, *aoa_az, *aoa_el;
  void* gain;
  uint8_t* valid;
};

// Partition of H = sum over rays: a wave owns TTc instants x (KB * kNK) subcarriers of one
// ray slice; a workgroup = 4 waves = 4 consecutive slices of one tile, summed in LDS; G
// slice groups per tile are summed afterwards by k_reduce when G > 1.
struct CfrArgs {
  int n_rays, T, K;
  int KB, TTc, nT, nK, G, slice_len, n_blocks;
  double f0, df;
  int path;          // CfrPath
  int MT, NT, B, K1; // MFMA path: H[t] = U (K1 x R) . V (R x B), 16x16 tiles, B = 8 NT
};

// Per-metre phase factors (cycles per metre of path length) for the anchor records.
struct AnchorParams {
  double f0c;   // f_0 / c: phase of the first subcarrier
  double fBc;   // B df / c: phase step between MFMA row blocks of B subcarriers
  double f1c;   // df / c: phase step between adjacent subcarriers
};

// Rays of each signature class (indices into the scene's ray table, ascending) for one call.
struct RayClasses {
  const int32_t* order[CLS_COUNT];
  int count[CLS_COUNT];
};

size_t pose_bytes(int nb, int T, int prec);
size_t record_bytes(int n_rays, int T, int prec);
CfrArgs plan_cfr(int n_rays, int T, int K, double f0, double df, int target_waves, int prec, int split_path);

hipError_t launch_pose(const DBody* bodies, int nb, int T, double dt, int prec, void* out, hipStream_t st);
hipError_t launch_geom(const SceneView& sc, const RayClasses& rc, const void* pose, int T, double dt, double f_c,
                       int n_rays, int prec, int mode, const ExtrapOut& eo, void* rec, const AnchorParams& ap,
                       hipStream_t st);
hipError_t launch_cfr(const void* rec, const CfrArgs& a, int prec, void* out, hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_reduce(const void* part, int G, size_t n, int prec, void* H, hipStream_t st);

}  // namespace drt
