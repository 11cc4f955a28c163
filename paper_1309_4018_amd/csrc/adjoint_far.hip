// Far field and direct pairs of the transposed treecode operator (A^T).
//
// In the transposed product the roles of the two point sets of sec. 2.3 are
// exchanged: the sources are the collocation points x_i with the adjoint
// weights muS_i (single layer) and muD_i (double layer) of one kernel slot,
// and the targets are the Gauss points y with the normal n of their panel.
// Every target accumulates
//   s(y) = sum_i muS_i G(x_i, y),
//   f(y) = sum_i muD_i n . grad_y G(x_i, y)   (double layer, normal at y).
// Near cells go through direct pairs (P2P), far cells through the Cartesian
// Taylor expansion about the cell centre c (Eqs. taylor and multexp with the
// two point sets exchanged): with d = y - c and the coefficients a_k(d) of
// taylor.h,
//   s = sum_{|k|<=P} a_k mS_k,              mS_k = sum_i muS_i (x_i - c)^k,
//   f = -sum_{|k|<=P+1} a_k sum_j n_j G_j,k, G_j,k = k_j mD_{k-e_j},
// because d/dy_j a_k = -(k_j + 1) a_{k+e_j}; the G_j,k are formed once per
// cell by the moment pass.  The coefficients follow the degree-scaled
// recurrences of taylor.h to order P + 1, the contractions are summed per
// degree and the degree factors enter by Horner's rule.
#include <cmath>

#include "device_util.h"
#include "kernel_common.h"
#include "taylor.h"

namespace pbtc {

namespace {

constexpr int kT = 256;
constexpr int kWaves = 4;

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ------------------------------------------------------------------- p2p
// target Gauss point t (position, normal in px..pz) against source s
// (position, weights muS_0, muD_0, muS_1, muD_1 in q, px, py, pz);
// d = x_src - y.  Laplace: muS / r, muD (n . d) / r^3; Yukawa: muS e / r,
// muD (n . d) e (1 + kappa r) / r^3 = muD (n . d) (e / r) (1/r^2 + kappa / r).
// a0, a1 = exp_arg(kappa) of the two kernel slots.
template <typename real, int KS>
__device__ __forceinline__ void adj_pair(real tx, real ty, real tz, real nx, real ny, real nz,
                                         const Src<real>& s, real k0, real k1, real a0, real a1,
                                         real (&acc)[4]) {
  const real dx = s.x - tx, dy = s.y - ty, dz = s.z - tz;
  const real r2 = dx * dx + dy * dy + dz * dz;
  const real rinv = r2 > real(0) ? rsqrt_(r2) : real(0);
  const real dn = nx * dx + ny * dy + nz * dz;
  const real t2 = rinv * rinv;
  if (KS == KS_L || KS == KS_LY) {
    acc[0] += s.q * rinv;
    acc[1] += s.px * (dn * (t2 * rinv));
  }
  if (KS == KS_Y || KS == KS_YY) {
    const real er = exp_scaled(a0 * (r2 * rinv)) * rinv;
    acc[0] += s.q * er;
    acc[1] += s.px * (dn * (er * (k0 * rinv + t2)));
  }
  if (KS == KS_LY || KS == KS_YY) {
    const real er = exp_scaled(a1 * (r2 * rinv)) * rinv;
    acc[2] += s.py * er;
    acc[3] += s.pz * (dn * (er * (k1 * rinv + t2)));
  }
}

template <int KS>
constexpr int nacc2() {
  return KS == KS_L || KS == KS_Y ? 2 : 4;
}

// One wavefront per work unit (a group of 64 target Gauss points and a run
// of its near list); sources through wave-uniform (scalar) loads, four per
// step so that their loads are in flight together.
template <typename real, int KS>
__global__ __launch_bounds__(kT) void k_adj_p2p(UnitArgs a, const Src<real>* __restrict__ gpos,
                                                const Src<real>* __restrict__ asrc,
                                                real* __restrict__ partial) {
  const int u = uni(xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6));
  if (u >= a.nunits) return;
  const int4 un = a.units[u];
  const int item = uni(un.x), e0 = uni(un.y), e1 = uni(un.z);
  const DevBlock& b = a.blocks[uni(a.item_block[item])];
  const long long g = item - b.aitem_off;
  const long long j0 = b.gp_off + g * kAGroup;
  const int nt = (int)min((long long)kAGroup, b.gp_n - g * kAGroup);
  const int lane = threadIdx.x & 63;
  const Src<real> t = gpos[j0 + min(lane, nt - 1)];
  const real k0 = (real)b.kappa0, k1 = (real)b.kappa1;
  const real a0 = exp_arg(k0), a1 = exp_arg(k1);
  const long long soff = b.nf_row - b.tgt_off;
  real acc[4] = {0, 0, 0, 0};
  for (int e = e0; e < e1; ++e) {
    const int c = uni(a.cells_list[e]);
    const int beg = uni(a.cells[c].begin), end = beg + uni(a.cells[c].count);
    const Src<real>* src = asrc + soff;
    int j = beg;
    for (; j + 3 < end; j += 4) {
      const Src<real> s0 = src[j], s1 = src[j + 1], s2 = src[j + 2], s3 = src[j + 3];
      adj_pair<real, KS>(t.x, t.y, t.z, t.px, t.py, t.pz, s0, k0, k1, a0, a1, acc);
      adj_pair<real, KS>(t.x, t.y, t.z, t.px, t.py, t.pz, s1, k0, k1, a0, a1, acc);
      adj_pair<real, KS>(t.x, t.y, t.z, t.px, t.py, t.pz, s2, k0, k1, a0, a1, acc);
      adj_pair<real, KS>(t.x, t.y, t.z, t.px, t.py, t.pz, s3, k0, k1, a0, a1, acc);
    }
    for (; j < end; ++j) {
      const Src<real> s0 = src[j];
      adj_pair<real, KS>(t.x, t.y, t.z, t.px, t.py, t.pz, s0, k0, k1, a0, a1, acc);
    }
  }
#pragma unroll
  for (int q = 0; q < nacc2<KS>(); ++q) partial[((size_t)u * 4 + q) * 64 + lane] = acc[q];
}

// ------------------------------------------------------------------- m2p
// s += sum_{|k|<=P} a_k mS_k and f += -sum_{|k|<=P+1} a_k (n . G_k) for the
// kernel KIND (0 Laplace, 1 Yukawa with e = exp(-kappa R)), M = [mS | G_1 |
// G_2 | G_3] of one cell.  Degree scaling as in taylor_laplace /
// taylor_yukawa, carried to order P + 1: a_k = rho_n alpha_k, with
// rho_0 = 1/R, rho_n = c1(n) rho_{n-1} / R^2, c1(n) = (2n - 1)/n.
template <int P, typename real, int KIND>
__device__ __forceinline__ void taylor_adj(real dx, real dy, real dz, real rinv, real e,
                                           real kappa, real nx, real ny, real nz,
                                           const real* __restrict__ M, real& s, real& f) {
  constexpr int Q = P + 1;  // highest degree
  constexpr int N = MultiIndex<P>::N;
  constexpr int N1 = MultiIndex<Q>::N;
  constexpr MultiIndex<Q> T{};
  const real r2inv = rinv * rinv;
  const real r2 = dx * dx + dy * dy + dz * dz;
  // per-degree factors of the recurrences (taylor.h)
  real A[Q + 1], B[Q + 1], C[Q + 1], V[Q + 1];
  const real R = r2 * rinv;
  const real k2r2 = kappa * kappa * r2;
  const real k2r4 = k2r2 * r2;
  static_for<Q + 1>([&](auto nc) {
    constexpr int n = decltype(nc)::value;
    A[n] = B[n] = C[n] = V[n] = real(0);
    if constexpr (KIND == 0) {
      if constexpr (n >= 2)
        A[n] = (real((n - 1) * (n - 1)) / real((2 * n - 1) * (2 * n - 3))) * r2;
    } else {
      if constexpr (n == 1) B[1] = kappa * e * R;
      if constexpr (n >= 2) {
        constexpr real c1m = real(2 * n - 3) / real(n - 1);
        A[n] = (real(n - 1) / (real(2 * n - 1) * c1m)) * r2;
        V[n] = (real(1) / c1m) * r2;
        B[n] = (real(1) / (real((n - 1) * (2 * n - 1)) * c1m)) * k2r2;
      }
      if constexpr (n == 2) C[2] = kappa * e * R * r2 * (real(1) / real(3));
      if constexpr (n >= 3) {
        constexpr real c1m = real(2 * n - 3) / real(n - 1);
        constexpr real c1mm = real(2 * n - 5) / real(n - 2);
        C[n] = (real(1) / (real((n - 2) * (2 * n - 1)) * c1m * c1mm)) * k2r4;
      }
    }
  });
  real al[N1], be[KIND ? N1 : 1];
  real S[P + 1], F[3][Q + 1];
  static_for<Q + 1>([&](auto nc) {
    constexpr int n = decltype(nc)::value;
    if constexpr (n <= P) S[n] = real(0);
    F[0][n] = F[1][n] = F[2][n] = real(0);
  });
  al[0] = KIND ? e : real(1);
  if constexpr (KIND) be[0] = real(1);
  S[0] = al[0] * M[0];
  static_for<N1 - 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value + 1;
    constexpr int n = T.n[k];
    constexpr int i10 = T.m1[k][0], i11 = T.m1[k][1], i12 = T.m1[k][2];
    constexpr int i20 = T.m2[k][0], i21 = T.m2[k][1], i22 = T.m2[k][2];
    constexpr bool has2 = i20 >= 0 || i21 >= 0 || i22 >= 0;
    real s1a = real(0), s2a = real(0);
    if constexpr (i10 >= 0) s1a += dx * al[i10];
    if constexpr (i11 >= 0) s1a += dy * al[i11];
    if constexpr (i12 >= 0) s1a += dz * al[i12];
    if constexpr (i20 >= 0) s2a += al[i20];
    if constexpr (i21 >= 0) s2a += al[i21];
    if constexpr (i22 >= 0) s2a += al[i22];
    if constexpr (KIND == 0) {
      al[k] = has2 ? s1a - A[n] * s2a : s1a;
    } else {
      real s1b = real(0), s2b = real(0);
      if constexpr (i10 >= 0) s1b += dx * be[i10];
      if constexpr (i11 >= 0) s1b += dy * be[i11];
      if constexpr (i12 >= 0) s1b += dz * be[i12];
      if constexpr (i20 >= 0) s2b += be[i20];
      if constexpr (i21 >= 0) s2b += be[i21];
      if constexpr (i22 >= 0) s2b += be[i22];
      if constexpr (has2) {
        al[k] = s1a - A[n] * s2a + B[n] * s1b - C[n] * s2b;
        if constexpr (n < Q) be[k] = s1a - V[n] * s2a;
      } else {
        al[k] = s1a + B[n] * s1b;
        if constexpr (n < Q) be[k] = s1a;
      }
    }
    if constexpr (n <= P) S[n] += al[k] * M[k];
    if constexpr (T.k1[k] > 0) F[0][n] += al[k] * M[N + k];
    if constexpr (T.k2[k] > 0) F[1][n] += al[k] * M[N + N1 + k];
    if constexpr (T.k3[k] > 0) F[2][n] += al[k] * M[N + 2 * N1 + k];
  });
  // sum_n rho_n X_n = (1/R)(X_0 + g_1 (X_1 + g_2 (X_2 + ...))), g_n = c1(n) / R^2
  real hs = S[P];
  real hf = nx * F[0][Q] + ny * F[1][Q] + nz * F[2][Q];
  static_for<Q>([&](auto nc) {
    constexpr int n = Q - decltype(nc)::value;  // Q .. 1
    constexpr real c1 = real(2 * n - 1) / real(n);
    const real g = c1 * r2inv;
    if constexpr (n <= P) hs = S[n - 1] + g * hs;
    const real fn = nx * F[0][n - 1] + ny * F[1][n - 1] + nz * F[2][n - 1];
    hf = fn + g * hf;
  });
  s += rinv * hs;
  f -= rinv * hf;
}

// One wavefront per work unit (64 target Gauss points and a run of far
// cells); the cell's moments go through a per-wavefront LDS slice (broadcast
// reads); the next cell's moments and centre are loaded into registers while
// the current cell is evaluated.
template <typename real, int P, int KIND>
__global__ __launch_bounds__(kT) void k_adj_m2p(UnitArgs a, const Src<real>* __restrict__ gpos,
                                                const real* __restrict__ mom, int ms, int kslot,
                                                real* __restrict__ partial) {
  constexpr int MS = adj_mom_len(P);
  const int u = uni(xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6));
  if (u >= a.nunits) return;
  const int4 un = a.units[u];
  const int item = uni(un.x), e0 = uni(un.y), e1 = uni(un.z);
  const DevBlock& b = a.blocks[uni(a.item_block[item])];
  const long long g = item - b.aitem_off;
  const long long j0 = b.gp_off + g * kAGroup;
  const int nt = (int)min((long long)kAGroup, b.gp_n - g * kAGroup);
  const int lane = threadIdx.x & 63;
  const Src<real> t = gpos[j0 + min(lane, nt - 1)];
  const real kap = (real)(kslot == 0 ? b.kappa0 : b.kappa1);
  const real* base = mom + (size_t)(b.lslot0 + kslot) * MS;
  constexpr int PER = (MS + 63) / 64;
  __shared__ real smom[kWaves][MS];
  const int wv = uni(threadIdx.x >> 6);
  real* M = smom[wv];
  real pre[PER];
  double pcx = 0, pcy = 0, pcz = 0;
  auto fetch = [&](int e) {
    const int c = uni(a.cells_list[e]);
    const Cell& cl = a.cells[c];
    pcx = cl.cx;
    pcy = cl.cy;
    pcz = cl.cz;
    const real* Mg = base + (size_t)c * ms * MS;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int k = lane + 64 * q;
      pre[q] = k < MS ? Mg[k] : real(0);
    }
  };
  real s = 0, f = 0;
  if (e0 < e1) fetch(e0);
  for (int e = e0; e < e1; ++e) {
    wave_sync();  // the previous cell's reads of M are done
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int k = lane + 64 * q;
      if (k < MS) M[k] = pre[q];
    }
    const real dx = t.x - (real)pcx, dy = t.y - (real)pcy, dz = t.z - (real)pcz;
    wave_sync();  // M is written
    if (e + 1 < e1) fetch(e + 1);
    const real r2 = dx * dx + dy * dy + dz * dz;
    const real rinv = rsqrt_(r2);
    const real ee = KIND ? exp_neg(kap * (r2 * rinv)) : real(1);
    taylor_adj<P, real, KIND>(dx, dy, dz, rinv, ee, kap, t.px, t.py, t.pz, M, s, f);
  }
  partial[((size_t)u * 4 + 0) * 64 + lane] = s;
  partial[((size_t)u * 4 + 1) * 64 + lane] = f;
}

}  // namespace

template <typename real>
void launch_adj_p2p(hipStream_t st, int ks, const UnitArgs& a, int grid, const Src<real>* gpos,
                    const Src<real>* asrc, real* partial) {
  switch (ks) {
    case KS_L: hipLaunchKernelGGL((k_adj_p2p<real, KS_L>), dim3(grid), dim3(kT), 0, st, a, gpos, asrc, partial); break;
    case KS_Y: hipLaunchKernelGGL((k_adj_p2p<real, KS_Y>), dim3(grid), dim3(kT), 0, st, a, gpos, asrc, partial); break;
    case KS_LY: hipLaunchKernelGGL((k_adj_p2p<real, KS_LY>), dim3(grid), dim3(kT), 0, st, a, gpos, asrc, partial); break;
    case KS_YY: hipLaunchKernelGGL((k_adj_p2p<real, KS_YY>), dim3(grid), dim3(kT), 0, st, a, gpos, asrc, partial); break;
    default: break;
  }
}

template <typename real>
void launch_adj_m2p(hipStream_t st, int P, const UnitArgs& a, int grid, const Src<real>* gpos,
                    const real* mom, int ms, int kind, int kslot, real* partial) {
#define PBTC_AM2P(PP)                                                                         \
  case PP:                                                                                    \
    if (kind == 0)                                                                            \
      hipLaunchKernelGGL((k_adj_m2p<real, PP, 0>), dim3(grid), dim3(kT), 0, st, a, gpos, mom, \
                         ms, kslot, partial);                                                 \
    else                                                                                      \
      hipLaunchKernelGGL((k_adj_m2p<real, PP, 1>), dim3(grid), dim3(kT), 0, st, a, gpos, mom, \
                         ms, kslot, partial);                                                 \
    break;
  switch (P) {
    PBTC_AM2P(2)
    PBTC_AM2P(4)
    PBTC_AM2P(6)
    PBTC_AM2P(8)
    PBTC_AM2P(10)
    default:
      break;
  }
#undef PBTC_AM2P
}

template void launch_adj_p2p<float>(hipStream_t, int, const UnitArgs&, int, const Src<float>*,
                                    const Src<float>*, float*);
template void launch_adj_p2p<double>(hipStream_t, int, const UnitArgs&, int, const Src<double>*,
                                     const Src<double>*, double*);
template void launch_adj_m2p<float>(hipStream_t, int, const UnitArgs&, int, const Src<float>*,
                                    const float*, int, int, int, float*);
template void launch_adj_m2p<double>(hipStream_t, int, const UnitArgs&, int, const Src<double>*,
                                     const double*, int, int, int, double*);

}  // namespace pbtc
