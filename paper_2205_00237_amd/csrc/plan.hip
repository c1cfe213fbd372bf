// Host-side planning of the kernels: scratch sizes of the pose table and the ray-sum
// records, the ray-sum partition (tile shape, ray groups, workgroups) and the work items
// and grids of the batched serving kernels.  Plain host code, no kernel.
#include <algorithm>

#include "drt_kernels.h"
#include "drt_records.h"

namespace drt {

size_t pose_bytes(int nb, int T, int prec) {
  return size_t(nb) * T * (prec == DRT_NAIVE32 ? sizeof(float2) : sizeof(double2));
}

size_t record_bytes(int n_rays, int T, int prec) {
  size_t per = prec == DRT_FP64 ? std::max(sizeof(RecD), sizeof(RecM64))
                                : (prec == DRT_SPLIT ? std::max(sizeof(RecS), sizeof(RecM)) : sizeof(RecN));
  return size_t((T + 63) / 64) * n_rays * 64 * per;
}

CfrArgs plan_cfr(int n_rays, int T, int K, double f0, double df, int target_waves, int prec, int split_path,
                 int fp64_path) {
  CfrArgs a{};
  a.n_rays = n_rays;
  a.T = T;
  a.K = K;
  a.f0 = f0;
  a.df = df;
  a.path = CFR_VALU;
  const bool mfma64 = prec == DRT_FP64 && fp64_path == CFR_MFMA64 && K > 128 && K <= 1024;
  if ((prec == DRT_SPLIT && K <= 2048 && split_path != CFR_VALU) || mfma64) {
    a.path = mfma64 ? CFR_MFMA64 : split_path;
    if (mfma64) {
      a.NT = K > 512 ? 8 : (K > 256 ? 4 : 2);   // B = 8 NT: one row tile of K / B <= 16
    } else {
      a.NT = K <= 64 ? 1 : (K <= 256 ? 2 : 4);
    }
    a.B = 8 * a.NT;
    a.K1 = (K + a.B - 1) / a.B;
    a.MT = (a.K1 + 15) / 16;
    if (a.MT == 3) a.MT = 4;
    long tiles = T;
    int G = int((target_waves + 4 * tiles - 1) / (4 * tiles));
    int maxG = (n_rays + 4 * kMinSlice - 1) / (4 * kMinSlice);
    if (G > maxG) G = maxG;
    if (G < 1) G = 1;
    a.G = G;
    a.slice_len = (n_rays + 4 * G - 1) / (4 * G);
    const int gran = a.path == CFR_MFMA16 ? 16 : 2;   // rays per matrix instruction
    a.slice_len = (a.slice_len + gran - 1) / gran * gran;
    a.n_blocks = int(tiles * G);
    return a;
  }
  const int nk = nk_of(prec);
  int blocks_k = (K + nk - 1) / nk;     // subcarrier blocks of nk
  int kb = 1;
  while (kb < blocks_k && kb < 64) kb <<= 1;
  a.KB = kb;
  a.TTc = 64 / kb;
  a.nT = (T + a.TTc - 1) / a.TTc;
  a.nK = (blocks_k + kb - 1) / kb;
  long tiles = long(a.nT) * a.nK;
  int G = int((target_waves + 4 * tiles - 1) / (4 * tiles));
  int maxG = (n_rays + 4 * kMinSlice - 1) / (4 * kMinSlice);
  if (G > maxG) G = maxG;
  if (G < 1) G = 1;
  a.G = G;
  a.slice_len = (n_rays + 4 * G - 1) / (4 * G);
  a.n_blocks = int(tiles * G);
  return a;
}

void batch_items(const BatchReq& q, long long items[BK_COUNT]) {
  for (int k = 0; k < BK_COUNT; ++k) items[k] = 0;
  items[BK_POSE] = (long long)q.sc.n_bodies * q.T;
  for (int c = 0; c < CLS_COUNT; ++c) items[BK_GEOM + c] = (long long)((q.rc.count[c] + 3) / 4) * 4 * q.nchunk;
  items[BK_CFR + cfr_shape(q.a.MT, q.a.NT)] = q.a.n_blocks;
  if (q.a.G > 1) items[BK_REDUCE] = (long long)q.T * q.a.K;
}

long long batch_grid(int kind, long long items) {
  if (items <= 0) return 1;
  if (kind == BK_POSE || kind == BK_REDUCE) return (items + 255) / 256;   // a thread per item
  if (kind < BK_CFR) return (items + 3) / 4;                              // a wave per item
  return items;                                                           // a workgroup per item
}

}  // namespace drt
