// Launchers of the gfx950 kernels (kernels_*.hip) used by the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "drt_layout.h"

namespace drt {

enum GeomMode { GEOM_EXTRAP = 0, GEOM_ANCHOR = 1, GEOM_ANCHOR_MFMA = 2, GEOM_KIN = 3, GEOM_POWER = 4, GEOM_NUFFT = 5 };
enum CfrPath { CFR_VALU = 0, CFR_MFMA = 1, CFR_MFMA16 = 2, CFR_MFMA64 = 3 };

constexpr int kNK = 16;          // subcarriers walked by one lane from its phase anchor
constexpr int kNK64 = 32;        // the same in binary64 (its phase anchor costs a binary64 sincos)
inline int nk_of(int prec) { return prec == DRT_FP64 ? kNK64 : kNK; }
constexpr int kMinSlice = 64;    // fewest rays per wave slice of the ray sum (fewer ray groups, and no
                                 // partial sums to reduce, for small calls)

struct ExtrapOut {
  double* L;
  float *dop, *aod_az, *aod_el, *aoa_az, *aoa_el;
  void* gain;
  uint8_t* valid;
  uint8_t* in_bounds;
  int32_t* first_out;   // pre-filled with T; lowered by atomic minimum
  double *q_pos, *q_vel, *q_acc;   // [R][T][4][3] interaction points and their time derivatives
  float* dop_rate;                 // [R][T] Doppler rate at f_c [Hz/s]
  // power profiles (GEOM_POWER): [n_tb][n_dop], [n_tb][n_delay], [n_tb], cleared beforehand
  double *pdfp, *pdp, *ptotal;
  double dop_lo, dop_step, delay_lo, delay_step;
  int spb, n_dop, n_delay, gate;
};

// Partition of H = sum over rays: a wave owns TTc instants x (KB * nk_of(prec)) subcarriers of one
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

// Rays of each signature class (indices into the scene's ray table) for one call.
struct RayClasses {
  const int32_t* order[CLS_COUNT];
  int count[CLS_COUNT];
};

// Geometry workgroups of one class (4 rays x 64 instants each).
__host__ __device__ inline int class_workgroups(const RayClasses& rc, int c, int T) { return (rc.count[c] + 3) / 4 * ((T + 63) / 64); }

// Ray-sum record geometry of a small call runs as one kernel over every class (each workgroup
// takes its class's path) instead of one kernel per class: launches, not work, set its time.
constexpr int kMergedGeomMax = 256;   // most workgroups of a merged launch
inline bool geom_merged(const RayClasses& rc, int T) {
  int n = 0;
  for (int c = 0; c < CLS_COUNT; ++c) n += class_workgroups(rc, c, T);
  return n <= kMergedGeomMax;
}

// ---------------------------------------------------------------------------------------
// Batched serving.  A batch is up to kMaxBatch split-precision requests whose ray sum runs
// on the binary16 matrix cores.  Each kernel kind is one fused launch over the work items of
// every request in the batch (items of request j are [off[kind][j], off[kind][j+1])): pose
// entries, geometry waves per signature class, ray-sum tiles per MFMA tile shape, and
// partial-sum elements.  The launches take only the device-resident descriptor, so a graph
// captured once per slot replays for every batch with just the grid sizes updated.
constexpr int kMaxBatch = 64;
enum BatchKind {
  BK_POSE = 0,
  BK_GEOM = 1,                  // + signature class (CLS_R, CLS_D, CLS_S)
  BK_CFR = BK_GEOM + CLS_COUNT, // + tile shape index of the ray sum
  BK_REDUCE = BK_CFR + 5,
  BK_COUNT
};
// tile shape index of (MT, NT) in the binary16 ray sum, -1 if none
inline int cfr_shape(int MT, int NT) {
  if (NT == 1) return MT == 1 ? 0 : -1;
  if (NT == 2) return MT == 1 ? 1 : -1;
  if (NT == 4) return MT == 1 ? 2 : (MT == 2 ? 3 : (MT == 4 ? 4 : -1));
  return -1;
}

struct BatchReq {
  SceneView sc;
  RayClasses rc;
  int T, n_rays, nchunk, pad;
  double dt, f_c;
  AnchorParams ap;
  CfrArgs a;
  void* pose;      // binary64 pose table [n_bodies][T]
  void* rec;       // ray-sum records [T][n_rays]
  float* part;     // ray-group partial sums [G][T][K] complex (G > 1)
  float* H;        // caller's H [T][K] complex64
};

struct BatchDesc {
  int n_req, pad;
  long long off[BK_COUNT][kMaxBatch + 1];
  BatchReq req[kMaxBatch];   // only the first n_req are copied to the device
};

// work items of one request per kernel kind
void batch_items(const BatchReq& q, long long items[BK_COUNT]);
// workgroups (of 256) a kernel kind needs for `items` work items (1 when empty)
long long batch_grid(int kind, long long items);
// the kernel function of a kind (to recognise graph nodes)
void* batch_kernel(int kind);
hipError_t launch_batch(int kind, const BatchDesc* d, int grid, hipStream_t st);

size_t pose_bytes(int nb, int T, int prec);
size_t record_bytes(int n_rays, int T, int prec);
CfrArgs plan_cfr(int n_rays, int T, int K, double f0, double df, int target_waves, int prec, int split_path,
                 int fp64_path);

hipError_t launch_pose(const DBody* bodies, int nb, int T, double dt, int prec, void* out, hipStream_t st);
hipError_t launch_geom(const SceneView& sc, const RayClasses& rc, const void* pose, int T, double dt, double f_c,
                       int n_rays, int prec, int mode, const ExtrapOut& eo, void* rec, const AnchorParams& ap,
                       hipStream_t st);
hipError_t launch_cfr(const void* rec, const CfrArgs& a, int prec, void* out, hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
// ---------------------------------------------------------------------------------------
// Snapshot tracer.  One signature of candidate interaction sequences: the index of a
// candidate is a mixed-radix number whose digit i (most significant first) picks the
// primitive of interaction i: a wall (radix = walls, or walls - 1 after another wall, the
// previous wall being skipped), an edge (likewise after another edge) or a tile.  Ascending indices are lexicographic
// in the primitive indices.
struct TraceSig {
  int32_t n, code;
  int32_t kind[DRT_MAX_INT];
  int64_t radix[DRT_MAX_INT];
  int64_t count;
};

constexpr double kSegEps = 1e-7;    // an obstruction must cross a segment this far from its ends [m]
constexpr double kFrontEps = 1e-9;  // a path's neighbours must lie this far in front of a wall [m]

__host__ __device__ inline void trace_decode(const TraceSig& g, int64_t c, int32_t* prim) {
  int32_t dig[DRT_MAX_INT] = {0, 0, 0, 0};
  for (int i = g.n - 1; i >= 0; --i) {
    dig[i] = int32_t(c % g.radix[i]);
    c /= g.radix[i];
  }
  for (int i = 0; i < g.n; ++i) {
    int32_t p = dig[i];
    if (i > 0 && g.kind[i] == g.kind[i - 1]) p += (p >= prim[i - 1]) ? 1 : 0;
    prim[i] = p;
  }
}

// Non-uniform-FFT ray sum: per (instant, ray), instant-major, binary64: x = frac(df L / c)
// and c = a exp(-j 2 pi frac(f_c L / c)) (zero for an inconsistent chain).
struct RecU {
  double x, cr, ci;
};

// Binary64 ray-sum record of the matrix-core path, instant-major [instant][ray]: |a|, the
// first subcarrier's phase with arg a folded in, frac(f_0 L/c - arg a / 2 pi), the row-block
// and subcarrier phases frac(B df L/c) and frac(df L/c) (cycles), and the column step
// exp(-j 2 pi frac(16 df L/c)).
struct RecM64 {
  double amp, p0, pB, p1, fr, fi;
};

hipError_t launch_nufft(const RecU* rec, int R, int T, int K, int M, int w, double beta, double2* tw,
                        double* phihat, double2* quad, double2* H, hipStream_t st);

hipError_t launch_trace_cand(const SceneView& sc, const TraceSig& g, int sig_id, uint64_t* keys, uint32_t cap,
                             uint32_t* counter, hipStream_t st);
hipError_t launch_trace_vis(const SceneView& sc, const TraceSig* d_sigs, const uint64_t* keys, uint32_t n,
                            int n_planes, uint8_t* visible, double* length, hipStream_t st);

hipError_t launch_fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t st);
hipError_t launch_reduce(const void* part, int G, size_t n, int prec, void* H, hipStream_t st);

}  // namespace drt
