// CSI tile body (least-squares channel estimate from comb pilots, held over
// the pilot group), shared by the per-stage CSI kernel and the persistent
// batched kernel.
//
// A tile is one antenna and CSI_TILE consecutive subcarriers.  The LS value
// Yf0[q] conj(p[q]) / |p[q]|^2 is formed once per pilot subcarrier q that the
// tile needs and parked in LDS; every thread then writes two subcarriers of
// each user's row of H, so each store instruction of a wave covers 512
// contiguous bytes.
#pragma once

#include "common.h"

namespace rxphy {
namespace csik {

constexpr int CSI_TILE = 512;
constexpr int CSI_WG = 256;
constexpr int CSI_LDS = CSI_TILE + 32;

// Inputs of one tile: the pilot-symbol values and pilots of the pilot
// subcarriers q0 .. q1-1 the tile needs (at most 512 + 2K - 1 < 3 x 256).
struct CsiIn {
  float2 y[3], p[3];
};

__device__ __forceinline__ void csi_range(int K, int n_sc, int i0, int& q0, int& q1) {
  const int G = n_sc / K;
  const int i_last = min(i0 + CSI_TILE, n_sc) - 1;
  q0 = min(i0 / K, G - 1) * K;                               // first pilot subcarrier needed
  q1 = min(i_last / K, G - 1) * K + K;                       // one past the last
}

// y0: the antenna's pilot-symbol row Yf[m][0][:]; pf: the frame's pilot row.
// Issues the tile's loads (lanes past q1 read q0 and are ignored).
__device__ __forceinline__ void csi_load(const float2* __restrict__ y0, const float2* __restrict__ pf,
                                         int K, int n_sc, int i0, CsiIn& in) {
  const int tx = tid_x();
  int q0, q1;
  csi_range(K, n_sc, i0, q0, q1);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int q = q0 + tx + j * CSI_WG;
    const int qc = q < q1 ? q : q0;
    in.y[j] = y0[qc];
    in.p[j] = pf[qc];
  }
}

// hm: H[m][0][0] of the frame ([K][n_sc] rows follow).  The LS values go
// through LDS (ls), then every user's row of the tile is written.
__device__ __forceinline__ void csi_finish(float2* __restrict__ hm, int K, int n_sc, int i0,
                                           const CsiIn& in, float2* ls) {
  const int tx = tid_x();
  int q0, q1;
  csi_range(K, n_sc, i0, q0, q1);
  const int G = n_sc / K;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int q = q0 + tx + j * CSI_WG;
    if (q < q1) ls[q - q0] = ls_estimate(in.y[j], in.p[j]);
  }
  __syncthreads();
  int gq[2];
  bool ok[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int i = i0 + tx + e * CSI_WG;
    ok[e] = i < n_sc;
    gq[e] = ok[e] ? min(i / K, G - 1) * K - q0 : 0;
  }
  float2* hp = hm + i0 + tx;
  for (int u = 0; u < K; ++u) {
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (ok[e]) hp[(int64_t)u * n_sc + e * CSI_WG] = ls[gq[e] + u];
  }
}

__device__ __forceinline__ void csi_tile(const float2* __restrict__ y0, const float2* __restrict__ pf,
                                         float2* __restrict__ hm, int K, int n_sc, int i0,
                                         float2* ls) {
  CsiIn in;
  csi_load(y0, pf, K, n_sc, i0, in);
  csi_finish(hm, K, n_sc, i0, in, ls);
}

}  // namespace csik
}  // namespace rxphy
