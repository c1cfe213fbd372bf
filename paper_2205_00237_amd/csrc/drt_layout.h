// Device-resident layout of one scene: array-of-structs tables for the primitives (read
// through the scalar cache: every wave works on one ray, so primitive indices are
// wave-uniform) and a 32-byte record per ray.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/drt.h"

namespace drt {

struct DBody {          // 128 B
  double O0[3], v0[3], a[3], k[3];
  double w0, wdot;
  int32_t moving, pad0;
  int32_t pad1[2];
};
struct DMat {           // 24 B
  double eps_r, sigma;
  int32_t pec, pad;
};
struct DPlane {         // 136 B
  double p0[3], n0[3];
  double c0[3], du[3], dv[3];   // facet at t0: corner and the duals of its sides, so that a
                                // point X of the plane is corner + s u + w v with
                                // s = du . (X - c0), w = dv . (X - c0)
  int32_t body, mat;
  int32_t bounded, pad;         // bounded = 0: the wall has no facet
};
struct DEdge {          // 128 B
  double a0[3], e0[3], t0[3], n0[3];
  double wn;
  double zlo, zhi;              // segment z_lo <= (X - a0) . e0 <= z_hi at t0 (may be infinite)
  int32_t body, pad;
};
struct DTile {          // 88 B
  double c0[3], n0[3];
  double area, S, phase0;
  int32_t body, alpha, model, pad;
};

// interaction signature of a ray (at most one diffraction, scattering only alone)
enum SigCode : uint8_t {
  SIG_LOS = 0, SIG_R1, SIG_R2, SIG_R3, SIG_R4,
  SIG_D, SIG_DR, SIG_RD, SIG_DRR, SIG_RDR, SIG_RRD, SIG_DRRR, SIG_RDRR, SIG_RRDR, SIG_RRRD,
  SIG_S, SIG_DD, SIG_COUNT
};

// Signature classes launched as separate kernels so that each gets its own register budget.
enum SigClass { CLS_R = 0, CLS_D = 1, CLS_S = 2, CLS_COUNT = 3 };
inline __host__ __device__ int sig_class(int code) {
  return code <= SIG_R4 ? CLS_R : (code == SIG_S ? CLS_S : CLS_D);
}

struct DRay {           // 80 B, whole words: a wave reads every field with a scalar load
  int32_t nint, code, dpos, pad;
  int32_t kind[4];
  int32_t pol[4];
  int32_t prim[4];
  int32_t body[4];      // body of each slot's primitive (0 for unused slots)
};
static_assert(sizeof(DRay) == 80, "DRay layout");
static_assert(sizeof(DBody) == 128, "DBody layout");

struct SceneView {
  const DBody* bodies;
  const DMat* mats;
  const DPlane* planes;
  const DEdge* edges;
  const DTile* tiles;
  const DRay* rays;
  double tx_p[3], tx_v[3], tx_a[3];
  double rx_p[3], rx_v[3], rx_a[3];
  double tx_ant[3], rx_ant[3];   // dipole axes (polar = 1)
  int32_t n_bodies, n_rays;
  int32_t polar, pad_;
};

}  // namespace drt
