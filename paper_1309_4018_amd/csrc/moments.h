// Moment shift of the treecode's upward pass (sec. 2.3, Eq. multexp): the
// moments of a parent cell about its centre c_p from those of its children
// about theirs,
//   M_p[k] = sum_children sum_{j <= k} C(k, j) (c_child - c_p)^(k - j) M_child[j],
// with the multi-index binomial C(k, j) = prod_i C(k_i, j_i), for both halves
// of a moment record [single layer | double layer] (the double-layer moments
// are Taylor moments of a derivative and shift the same way).
#pragma once

#include "taylor.h"

namespace pbtc {

constexpr int kM2MThreads = 256;

// One work-group (kM2MThreads) per parent cell cl (index c) with 1..8
// children in consecutive cells.  The children's moment records and, per
// child and axis, the factors C(k, j) d^(k - j) (k, j <= P) are staged in
// LDS, so the inner loops read LDS only; work items are (coefficient, child)
// pairs, and the children are summed in a fixed order (deterministic).
// The record of cell i (2 N values) is at mom + i * stride.
template <typename real, int P>
__device__ __forceinline__ void m2m_cell(const Cell* __restrict__ cells, const Cell& cl, int c,
                                         real* __restrict__ mom, size_t stride = 2 * ncoef(P)) {
  constexpr int N = ncoef(P);
  constexpr int KPT = (8 * N + kM2MThreads - 1) / kM2MThreads;
  __shared__ real sm[8][2 * N];
  __shared__ real sh[8][3][P + 1][P + 1];
  const int nch = min(cl.nchild, 8);
  const int tid = threadIdx.x;
  for (int i = tid; i < nch * 2 * N; i += kM2MThreads)  // children are consecutive cells
    sm[i / (2 * N)][i % (2 * N)] = mom[(size_t)(cl.child + i / (2 * N)) * stride + i % (2 * N)];
  if (tid < 3 * nch) {
    const int ch = tid / 3, a = tid % 3;
    const Cell& cc = cells[cl.child + ch];
    const double dd = a == 0 ? cc.cx - cl.cx : (a == 1 ? cc.cy - cl.cy : cc.cz - cl.cz);
    const real d = (real)dd;
    real pw[P + 1];
    pw[0] = real(1);
#pragma unroll
    for (int e = 1; e <= P; ++e) pw[e] = pw[e - 1] * d;
#pragma unroll
    for (int k = 0; k <= P; ++k) {
      real cb = real(1);  // C(k, j), exact: C(k, j + 1) = C(k, j) (k - j) / (j + 1)
#pragma unroll
      for (int j = 0; j <= k; ++j) {
        sh[ch][a][k][j] = cb * pw[k - j];
        cb = cb * real(k - j) / real(j + 1);
      }
    }
  }
  __syncthreads();
  real ps[KPT], pd[KPT];
#pragma unroll
  for (int q = 0; q < KPT; ++q) {
    ps[q] = pd[q] = 0;
    const int item = tid + q * kM2MThreads;
    const int ch = item / N, k = item - (item / N) * N;
    if (ch < nch) {
      int k1, k2, k3;
      mindex_inv(k, k1, k2, k3);
      for (int j1 = 0; j1 <= k1; ++j1) {
        const real x1 = sh[ch][0][k1][j1];
        for (int j2 = 0; j2 <= k2; ++j2) {
          const real x12 = x1 * sh[ch][1][k2][j2];
          for (int j3 = 0; j3 <= k3; ++j3) {
            const real coef = x12 * sh[ch][2][k3][j3];
            const int j = mindex(j1, j2, j3);
            ps[q] += coef * sm[ch][j];
            pd[q] += coef * sm[ch][N + j];
          }
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < KPT; ++q) {
    const int item = tid + q * kM2MThreads;
    const int ch = item / N, k = item - (item / N) * N;
    if (ch < nch) {
      sm[ch][k] = ps[q];
      sm[ch][N + k] = pd[q];
    }
  }
  __syncthreads();
  for (int k = tid; k < 2 * N; k += kM2MThreads) {
    real s = 0;
    for (int ch = 0; ch < nch; ++ch) s += sm[ch][k];
    mom[(size_t)c * stride + k] = s;
  }
}

}  // namespace pbtc
