// Cartesian Taylor expansions of the treecode (sec. 2.3, Eqs. taylor and
// multexp).
//
// For a source cluster with centre y_c and a target x, with d = x - y_c and
// R = |d|, the Green's function expands in powers of (y - y_c):
//   G(x, y) = sum_{|k| <= P} a_k (y - y_c)^k,   a_k = (1/k!) D_y^k G(x, y_c),
// so that  sum_j q_j G(x, y_j) = sum_k a_k m_k  with moments
// m_k = sum_j q_j (y_j - y_c)^k, and the double layer
// sum_j q_j n_j . grad_y G(x, y_j) = sum_k a_k sum_j q_j n_j . grad (y_j - y_c)^k.
//
// The coefficients follow from the differential identities of the kernels.
// Laplace, 1/R (recurrence after Duan and Krasny): with n = |k|,
//   n R^2 a_k = (2n - 1) sum_i d_i a_{k-e_i} - (n - 1) sum_i a_{k-2e_i},
//   a_0 = 1/R.
// Yukawa, exp(-kappa R)/R (two-sequence recurrence after Li, Johnston and
// Krasny), with b_k the coefficients of exp(-kappa R):
//   n b_k = kappa (sum_i d_i a_{k-e_i} - sum_i a_{k-2e_i}),
//   n R^2 a_k = (2n - 1) sum_i d_i a_{k-e_i} - (n - 1) sum_i a_{k-2e_i}
//               + kappa (sum_i d_i b_{k-e_i} - sum_i b_{k-2e_i}),
//   a_0 = exp(-kappa R)/R, b_0 = exp(-kappa R).
// Both follow from R^2 grad_y g = -(y - x)(...) written for the Taylor
// series in (y - y_c); terms with a negative index are zero.
//
// Multi-indices k = (k1, k2, k3) with |k| <= P are stored by total degree,
// then k1 descending, then k2 descending.
#pragma once

#include <utility>

#include "internal.h"

namespace pbtc {

__host__ __device__ constexpr int mindex(int a, int b, int c) {
  return (a + b + c) * (a + b + c + 1) * (a + b + c + 2) / 6 +
         (b + c) * (b + c + 1) / 2 + c;
}

// Inverse of mindex by arithmetic (no table): total degree n from the
// tetrahedral numbers, then b + c from the triangular numbers.
__host__ __device__ inline void mindex_inv(int k, int& a, int& b, int& c) {
  int n = 0;
  while ((n + 1) * (n + 2) * (n + 3) / 6 <= k) ++n;
  const int r = k - n * (n + 1) * (n + 2) / 6;
  int m = 0;
  while ((m + 1) * (m + 2) / 2 <= r) ++m;
  c = r - m * (m + 1) / 2;
  b = m - c;
  a = n - m;
}

template <int P>
struct MultiIndex {
  static constexpr int N = ncoef(P);
  int n[N], k1[N], k2[N], k3[N];
  int m1[N][3];  // index of k - e_i, or -1
  int m2[N][3];  // index of k - 2 e_i, or -1
  constexpr MultiIndex() : n(), k1(), k2(), k3(), m1(), m2() {
    for (int deg = 0; deg <= P; ++deg)
      for (int a = deg; a >= 0; --a)
        for (int b = deg - a; b >= 0; --b) {
          const int c = deg - a - b;
          const int i = mindex(a, b, c);
          n[i] = deg;
          k1[i] = a;
          k2[i] = b;
          k3[i] = c;
          m1[i][0] = a >= 1 ? mindex(a - 1, b, c) : -1;
          m1[i][1] = b >= 1 ? mindex(a, b - 1, c) : -1;
          m1[i][2] = c >= 1 ? mindex(a, b, c - 1) : -1;
          m2[i][0] = a >= 2 ? mindex(a - 2, b, c) : -1;
          m2[i][1] = b >= 2 ? mindex(a, b - 2, c) : -1;
          m2[i][2] = c >= 2 ? mindex(a, b, c - 2) : -1;
        }
  }
};

// sum_k a_k M[k] and sum_k a_k M[N + k] for the Laplace kernel 1/R.
// Compile-time loop: f(std::integral_constant<int, i>) for i = 0 .. N-1.
// Every coefficient index below is then a constant, so the coefficient
// arrays live in registers whatever the order (a run-time loop over 120+
// terms is not fully unrolled and its arrays go to scratch memory).
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>()), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>());
}

// Coefficient K >= 1 of the table of order PP from those of lower degree
// (the recurrences above): Laplace (YUK = false) fills a, Yukawa fills a
// and b.
template <int PP, int K, bool YUK, typename real>
__device__ __forceinline__ void coef_step(real* a, real* b, real dx, real dy, real dz, real r2inv,
                                          real kappa) {
  constexpr MultiIndex<PP> T{};
  constexpr int n = T.n[K];
  constexpr int i10 = T.m1[K][0], i11 = T.m1[K][1], i12 = T.m1[K][2];
  constexpr int i20 = T.m2[K][0], i21 = T.m2[K][1], i22 = T.m2[K][2];
  real s1 = real(0), s2 = real(0), t1 = real(0), t2 = real(0);
  if constexpr (i10 >= 0) {
    s1 += dx * a[i10];
    if constexpr (YUK) t1 += dx * b[i10];
  }
  if constexpr (i11 >= 0) {
    s1 += dy * a[i11];
    if constexpr (YUK) t1 += dy * b[i11];
  }
  if constexpr (i12 >= 0) {
    s1 += dz * a[i12];
    if constexpr (YUK) t1 += dz * b[i12];
  }
  if constexpr (i20 >= 0) {
    s2 += a[i20];
    if constexpr (YUK) t2 += b[i20];
  }
  if constexpr (i21 >= 0) {
    s2 += a[i21];
    if constexpr (YUK) t2 += b[i21];
  }
  if constexpr (i22 >= 0) {
    s2 += a[i22];
    if constexpr (YUK) t2 += b[i22];
  }
  constexpr real c1 = real(2 * n - 1) / real(n), c2 = real(n - 1) / real(n);
  constexpr real inv_n = real(1) / real(n);
  if constexpr (YUK) {
    b[K] = kappa * inv_n * (s1 - s2);
    a[K] = (c1 * s1 - c2 * s2 + kappa * inv_n * (t1 - t2)) * r2inv;
  } else {
    a[K] = (c1 * s1 - c2 * s2) * r2inv;
  }
}

// sum_k a_k M[k] and sum_k a_k M[N + k] for the Laplace kernel 1/R.
template <int P, typename real>
__device__ __forceinline__ void taylor_laplace(real dx, real dy, real dz, real rinv,
                                               const real* __restrict__ M, real& s, real& d) {
  constexpr int N = MultiIndex<P>::N;
  const real r2inv = rinv * rinv;
  real a[N];
  a[0] = rinv;
  s += a[0] * M[0];
  d += a[0] * M[N];
  static_for<N - 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value + 1;
    coef_step<P, k, false, real>(a, a, dx, dy, dz, r2inv, real(0));
    s += a[k] * M[k];
    d += a[k] * M[N + k];
  });
}

// Same for the Yukawa kernel exp(-kappa R)/R; e = exp(-kappa R).
template <int P, typename real>
__device__ __forceinline__ void taylor_yukawa(real dx, real dy, real dz, real rinv, real e,
                                              real kappa, const real* __restrict__ M, real& s,
                                              real& d) {
  constexpr int N = MultiIndex<P>::N;
  const real r2inv = rinv * rinv;
  real a[N], b[N];
  a[0] = e * rinv;
  b[0] = e;
  s += a[0] * M[0];
  d += a[0] * M[N];
  static_for<N - 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value + 1;
    coef_step<P, k, true, real>(a, b, dx, dy, dz, r2inv, kappa);
    s += a[k] * M[k];
    d += a[k] * M[N + k];
  });
}

// Floating-point operations of one P2P pair as written in the kernel
// (FMA = 2, a transcendental = 1): distance, r^2, rsqrt, n.d and r^-3
// (16), then Laplace single + double layer (4) and Yukawa (12) per kernel.
inline double p2p_flop_per_pair(int ks) {
  switch (ks) {
    case KS_L: return 20.0;
    case KS_Y: return 28.0;
    case KS_LY: return 32.0;
    default: return 40.0;
  }
}

// Floating-point operations of one (target, cell) Taylor evaluation, counted
// from the recurrences above term by term (FMA = 2).
inline double m2p_flop_one(int P, int kind) {
  double f = kind == 0 ? 11.0 : 16.0;  // d, r^2, rsqrt, 1/r^2 [, r, exp]
  for (int deg = 0; deg <= P; ++deg)
    for (int a = deg; a >= 0; --a)
      for (int b = deg - a; b >= 0; --b) {
        const int c = deg - a - b;
        if (deg == 0) {
          f += 4.0 + (kind ? 1.0 : 0.0);
          continue;
        }
        const int nz1 = (a >= 1) + (b >= 1) + (c >= 1);
        const int nz2 = (a >= 2) + (b >= 2) + (c >= 2);
        const double s1 = 2.0 * nz1 - 1.0, s2 = nz2 > 0 ? nz2 - 1.0 : 0.0;
        if (kind == 0)
          f += s1 + s2 + (nz2 ? 4.0 : 2.0) + 4.0;
        else
          f += 2.0 * (s1 + s2) + (nz2 ? 3.0 : 2.0) + (nz2 ? 7.0 : 5.0) + 4.0;
      }
  return f;
}

inline double m2p_flop_per_eval(int P, int ks) {
  switch (ks) {
    case KS_L: return m2p_flop_one(P, 0);
    case KS_Y: return m2p_flop_one(P, 1);
    case KS_LY: return m2p_flop_one(P, 0) + m2p_flop_one(P, 1);
    default: return 2.0 * m2p_flop_one(P, 1);
  }
}

}  // namespace pbtc
