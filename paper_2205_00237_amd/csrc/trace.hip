// Snapshot ray tracing on gfx950: the conventional image-method RT whose ray set DRT
// extrapolates (Sec. II: the trace at t0 and its refresh at the end of each multipath
// lifetime T_C).  The scene is traced at its own t0 (the host rebases it to the instant
// first), in binary64.
//
//   k_trace_cand  one lane per candidate interaction sequence of one signature: decode the
//                 sequence from the candidate index, solve the interaction points (images
//                 and back-tracking, Sec. III-A.2; eq. diff_point, Sec. III-B), and test the
//                 facets, front sides, edge segment and wedge exterior; survivors are
//                 appended (wave-aggregated atomic) as 64-bit keys signature << 40 | index
//   k_trace_vis   one wave per survivor: rebuild its vertices, each lane tests a strided
//                 subset of the walls against every segment; a ballot gives the verdict
#include <hip/hip_runtime.h>

#include "drt_geom.h"
#include "drt_kernels.h"

namespace drt {

// Slot data at the scene's t0 (no motion): the packed tables as they are.
__device__ __forceinline__ void load_slot_t0(const SceneView& sc, int kind, int prim, Slot<double>& s) {
  if (kind == DRT_R) {
    const DPlane& p = sc.planes[prim];
    s.p = ld3<double>(p.p0);
    s.n = ld3<double>(p.n0);
  } else if (kind == DRT_D) {
    const DEdge& e = sc.edges[prim];
    s.p = ld3<double>(e.a0);
    s.e = ld3<double>(e.e0);
    s.t = ld3<double>(e.t0);
    s.n = ld3<double>(e.n0);
  } else {
    const DTile& t = sc.tiles[prim];
    s.p = ld3<double>(t.c0);
    s.n = ld3<double>(t.n0);
  }
}

// Angle of X about the edge, from the 0-face (tangent t) towards its normal n, in [0, 2 pi).
__device__ __forceinline__ double wedge_angle(const Slot<double>& ed, V3<double> Q, V3<double> X) {
  V3<double> u = X - Q;
  u = u - dot(u, ed.e) * ed.e;
  double phi = atan2(dot(u, ed.n), dot(u, ed.t));
  return phi < 0.0 ? phi + 2.0 * M_PI : phi;
}

// Interaction points of the sequence prim[0..N) (kinds from N, DP, SCAT) and its geometric
// existence: reflection parameters in (0, 1), reflection points in their facets with both
// neighbours more than kFrontEps in front (a wall holding the ray's diffracting edge would
// put the segment between them inside the wall, its side a matter of rounding), the
// diffraction point on its segment with both neighbours in the wedge exterior, a tile
// facing both terminals.  V[0..N+1] = TX, points, RX.
template <int N, int DP, bool SCAT>
__device__ __forceinline__ bool path_geometry(const SceneView& sc, const int32_t* prim, V3<double>* V) {
  const V3<double> TX = ld3<double>(sc.tx_p), RX = ld3<double>(sc.rx_p);
  V[0] = TX;
  V[N + 1] = RX;
  if constexpr (N == 0) {
    return true;
  } else {
    Slot<double> sl[N];
#pragma unroll
    for (int i = 0; i < N; ++i)
      load_slot_t0(sc, SCAT ? DRT_S : ((i == DP || DP == -2) ? DRT_D : DRT_R), prim[i], sl[i]);
    if constexpr (SCAT) {
      V[1] = sl[0].p;
      return dot(TX - sl[0].p, sl[0].n) > 0.0 && dot(RX - sl[0].p, sl[0].n) > 0.0;
    } else {
      ChainOut<double> ch;
      solve_points<double, N, DP>(TX, RX, sl, ch);
      bool ok = ch.ok;
#pragma unroll
      for (int i = 0; i < N; ++i) V[i + 1] = ch.Q[i];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        if (DP == -2) {   // two edges: each point on its segment, neighbours in its exterior
          const DEdge& E = sc.edges[prim[i]];
          const double lim = E.wn * M_PI, zq = i == 0 ? ch.zQ : ch.zQ2;
          ok = ok && zq >= E.zlo && zq <= E.zhi;
          ok = ok && wedge_angle(sl[i], ch.Q[i], V[i]) <= lim && wedge_angle(sl[i], ch.Q[i], V[i + 2]) <= lim;
        } else if (i == DP) {
          const DEdge& E = sc.edges[prim[i]];
          const double lim = E.wn * M_PI;
          ok = ok && ch.zQ >= E.zlo && ch.zQ <= E.zhi;
          ok = ok && wedge_angle(sl[i], ch.Q[i], ch.A) <= lim && wedge_angle(sl[i], ch.Q[i], ch.B) <= lim;
        } else {
          const DPlane& P = sc.planes[prim[i]];
          const V3<double> q = ch.Q[i];
          ok = ok && dot(V[i] - q, sl[i].n) > kFrontEps && dot(V[i + 2] - q, sl[i].n) > kFrontEps;
          if (P.bounded) {
            const V3<double> x = q - ld3<double>(P.c0);
            const double su = dot(ld3<double>(P.du), x), sv = dot(ld3<double>(P.dv), x);
            ok = ok && su >= 0.0 && su <= 1.0 && sv >= 0.0 && sv <= 1.0;
          }
        }
      }
      return ok;
    }
  }
}

template <int N, int DP, bool SCAT>
__global__ __launch_bounds__(256) void k_trace_cand(SceneView sc, TraceSig g, int sig_id, uint64_t* keys,
                                                     uint32_t cap, uint32_t* counter) {
  const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  bool ok = false;
  if (c < g.count) {
    int32_t prim[DRT_MAX_INT];
    trace_decode(g, c, prim);
    V3<double> V[N + 2];
    ok = path_geometry<N, DP, SCAT>(sc, prim, V);
  }
  const unsigned long long m = __ballot(ok);
  if (m == 0ull) return;
  const int leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(counter, uint32_t(__popcll(m)));
  base = __shfl(base, leader);
  const uint32_t idx = base + uint32_t(__popcll(m & ((1ull << lane) - 1ull)));
  if (ok && idx < cap) keys[idx] = (uint64_t(sig_id) << 40) | uint64_t(c);
}

// One wave per survivor key: unobstructed when no wall crosses any segment of the path
// more than kSegEps from both of its ends.
__global__ __launch_bounds__(256) void k_trace_vis(SceneView sc, const TraceSig* sigs, const uint64_t* keys,
                                                    uint32_t n, int n_planes, uint8_t* visible, double* length) {
  const uint32_t k = uint32_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= n) return;
  const uint64_t key = keys[k];
  const TraceSig& g = sigs[key >> 40];
  int32_t prim[DRT_MAX_INT];
  trace_decode(g, int64_t(key & ((1ull << 40) - 1ull)), prim);
  with_signature<double>(g.code, [&]<int N, int DP, bool SCAT>() {
    V3<double> V[N + 2];
    const bool geo = path_geometry<N, DP, SCAT>(sc, prim, V);
    bool hit = false;
    for (int j = lane; j < n_planes; j += 64) {
      const DPlane& P = sc.planes[j];
      const V3<double> p = ld3<double>(P.p0), nn = ld3<double>(P.n0);
#pragma unroll
      for (int s = 0; s <= N; ++s) {
        const V3<double> A = V[s], d = V[s + 1] - V[s];
        const double len = norm(d), den = dot(nn, d);
        if (den == 0.0) continue;
        const double tau = dot(nn, p - A) / den;
        if (!(tau * len > kSegEps && (1.0 - tau) * len > kSegEps)) continue;
        if (!P.bounded) {
          hit = true;
        } else {
          const V3<double> x = (A + tau * d) - ld3<double>(P.c0);
          const double su = dot(ld3<double>(P.du), x), sv = dot(ld3<double>(P.dv), x);
          hit = hit || (su >= 0.0 && su <= 1.0 && sv >= 0.0 && sv <= 1.0);
        }
      }
    }
    const bool blocked = __ballot(hit) != 0ull;
    if (lane == 0) {
      double L = 0.0;
#pragma unroll
      for (int s = 0; s <= N; ++s) L += norm(V[s + 1] - V[s]);
      visible[k] = (geo && !blocked) ? 1 : 0;
      length[k] = L;
    }
    return 0;
  });
}

hipError_t launch_trace_cand(const SceneView& sc, const TraceSig& g, int sig_id, uint64_t* keys, uint32_t cap,
                             uint32_t* counter, hipStream_t st) {
  if (g.count <= 0) return hipSuccess;
  const dim3 grid(unsigned((g.count + 255) / 256));
  switch (g.code) {
#define CAND(CODE, N, DP, SC)                                                                                      \
  case CODE:                                                                                                     \
    hipLaunchKernelGGL((k_trace_cand<N, DP, SC>), grid, dim3(256), 0, st, sc, g, sig_id, keys, cap, counter); \
    break;
    CAND(SIG_LOS, 0, -1, false)
    CAND(SIG_R1, 1, -1, false)
    CAND(SIG_R2, 2, -1, false)
    CAND(SIG_R3, 3, -1, false)
    CAND(SIG_D, 1, 0, false)
    CAND(SIG_DR, 2, 0, false)
    CAND(SIG_RD, 2, 1, false)
    CAND(SIG_DRR, 3, 0, false)
    CAND(SIG_RDR, 3, 1, false)
    CAND(SIG_RRD, 3, 2, false)
    CAND(SIG_S, 1, -1, true)
    CAND(SIG_DD, 2, -2, false)
#undef CAND
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_trace_vis(const SceneView& sc, const TraceSig* d_sigs, const uint64_t* keys, uint32_t n,
                            int n_planes, uint8_t* visible, double* length, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_trace_vis, dim3((n + 3) / 4), dim3(256), 0, st, sc, d_sigs, keys, n, n_planes, visible,
                     length);
  return hipGetLastError();
}

}  // namespace drt
