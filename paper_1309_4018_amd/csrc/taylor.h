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

// Inverse of mindex for k < ncoef(kMaxP), by arithmetic and without
// branches: the total degree n counts the tetrahedral numbers <= k, then
// b + c the triangular numbers <= k - T(n).
__host__ __device__ inline void mindex_inv(int k, int& a, int& b, int& c) {
  int n = 0;
#pragma unroll
  for (int i = 1; i <= kMaxP; ++i) n += k >= i * (i + 1) * (i + 2) / 6 ? 1 : 0;
  const int r = k - n * (n + 1) * (n + 2) / 6;
  int m = 0;
#pragma unroll
  for (int i = 1; i <= kMaxP; ++i) m += r >= i * (i + 1) / 2 ? 1 : 0;
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

// sum_k a_k M[k] and sum_k a_k M[N + k] for the Laplace kernel 1/R, with
// the coefficients scaled per degree: a_k = rho_n beta_k for |k| = n, where
// rho_0 = 1/R and rho_n = c1(n) rho_{n-1} / R^2, c1(n) = (2n - 1)/n.  The
// recurrence above then reads
//   beta_k = sum_i d_i beta_{k-e_i} - w_n R^2 sum_i beta_{k-2e_i},
//   w_n = (n - 1)^2 / ((2n - 1)(2n - 3)),   beta_0 = 1,
// one fused multiply-add per coefficient instead of three operations; the
// contraction is summed per degree and the rho_n enter by Horner's rule.
template <int P, typename real>
__device__ __forceinline__ void taylor_laplace(real dx, real dy, real dz, real rinv,
                                               const real* __restrict__ M, real& s, real& d) {
  constexpr int N = MultiIndex<P>::N;
  constexpr MultiIndex<P> T{};
  const real r2inv = rinv * rinv;
  const real r2 = dx * dx + dy * dy + dz * dz;
  real wr[P + 1];
  static_for<P + 1>([&](auto nc) {
    constexpr int n = decltype(nc)::value;
    if constexpr (n >= 2) {
      constexpr real w = real((n - 1) * (n - 1)) / real((2 * n - 1) * (2 * n - 3));
      wr[n] = w * r2;
    } else {
      wr[n] = real(0);
    }
  });
  real beta[N];
  real S[P + 1], D[P + 1];
  static_for<P + 1>([&](auto nc) {
    S[decltype(nc)::value] = real(0);
    D[decltype(nc)::value] = real(0);
  });
  beta[0] = real(1);
  S[0] = M[0];
  D[0] = M[N];
  static_for<N - 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value + 1;
    constexpr int n = T.n[k];
    constexpr int i10 = T.m1[k][0], i11 = T.m1[k][1], i12 = T.m1[k][2];
    constexpr int i20 = T.m2[k][0], i21 = T.m2[k][1], i22 = T.m2[k][2];
    real s1 = real(0), s2 = real(0);
    if constexpr (i10 >= 0) s1 += dx * beta[i10];
    if constexpr (i11 >= 0) s1 += dy * beta[i11];
    if constexpr (i12 >= 0) s1 += dz * beta[i12];
    if constexpr (i20 >= 0) s2 += beta[i20];
    if constexpr (i21 >= 0) s2 += beta[i21];
    if constexpr (i22 >= 0) s2 += beta[i22];
    if constexpr (i20 >= 0 || i21 >= 0 || i22 >= 0)
      beta[k] = s1 - wr[n] * s2;
    else
      beta[k] = s1;
    S[n] += beta[k] * M[k];
    D[n] += beta[k] * M[N + k];
  });
  // sum_n rho_n S_n = (1/R) (S_0 + g_1 (S_1 + g_2 (S_2 + ...))), g_n = c1(n) / R^2
  real hs = S[P], hd = D[P];
  static_for<P>([&](auto nc) {
    constexpr int n = P - decltype(nc)::value;  // P .. 1
    constexpr real c1 = real(2 * n - 1) / real(n);
    const real g = c1 * r2inv;
    hs = S[n - 1] + g * hs;
    hd = D[n - 1] + g * hd;
  });
  s += rinv * hs;
  d += rinv * hd;
}

// Same for the Yukawa kernel exp(-kappa R)/R; e = exp(-kappa R).  Scaled
// per degree like the Laplace form: a_k = rho_n alpha_k and b_k = sigma_n
// beta_k with rho_n as above, sigma_0 = e, sigma_n = kappa rho_{n-1} / n.
// The two-sequence recurrence then reads, for |k| = n >= 1,
//   alpha_k = s1(alpha) - A_n s2(alpha) + B_n s1(beta) - C_n s2(beta),
//   beta_k  = s1(alpha) - V_n s2(alpha),
// with s1(x) = sum_i d_i x_{k-e_i}, s2(x) = sum_i x_{k-2e_i},
// alpha_0 = e, beta_0 = 1, and per-degree factors
//   A_n = (n-1) R^2 / ((2n-1) c1(n-1)),  V_n = R^2 / c1(n-1),
//   B_1 = kappa e R,  B_n = kappa^2 R^2 / ((n-1)(2n-1) c1(n-1))  (n >= 2),
//   C_2 = kappa e R^3 / 3,
//   C_n = kappa^2 R^4 / ((n-2)(2n-1) c1(n-1) c1(n-2))  (n >= 3).
template <int P, typename real>
__device__ __forceinline__ void taylor_yukawa(real dx, real dy, real dz, real rinv, real e,
                                              real kappa, const real* __restrict__ M, real& s,
                                              real& d) {
  constexpr int N = MultiIndex<P>::N;
  constexpr MultiIndex<P> T{};
  const real r2inv = rinv * rinv;
  const real r2 = dx * dx + dy * dy + dz * dz;
  const real R = r2 * rinv;
  const real k2r2 = kappa * kappa * r2;
  const real k2r4 = k2r2 * r2;
  real A[P + 1], B[P + 1], C[P + 1], V[P + 1];
  static_for<P + 1>([&](auto nc) {
    constexpr int n = decltype(nc)::value;
    A[n] = B[n] = C[n] = V[n] = real(0);
    if constexpr (n == 1) B[1] = kappa * e * R;
    if constexpr (n >= 2) {
      constexpr real c1m = real(2 * n - 3) / real(n - 1);  // c1(n - 1)
      A[n] = (real(n - 1) / (real(2 * n - 1) * c1m)) * r2;
      V[n] = (real(1) / c1m) * r2;
      B[n] = (real(1) / (real((n - 1) * (2 * n - 1)) * c1m)) * k2r2;
    }
    if constexpr (n == 2) C[2] = kappa * e * R * r2 * (real(1) / real(3));
    if constexpr (n >= 3) {
      constexpr real c1m = real(2 * n - 3) / real(n - 1);   // c1(n - 1)
      constexpr real c1mm = real(2 * n - 5) / real(n - 2);  // c1(n - 2)
      C[n] = (real(1) / (real((n - 2) * (2 * n - 1)) * c1m * c1mm)) * k2r4;
    }
  });
  real alpha[N], beta[N];
  real S[P + 1], D[P + 1];
  static_for<P + 1>([&](auto nc) {
    S[decltype(nc)::value] = real(0);
    D[decltype(nc)::value] = real(0);
  });
  alpha[0] = e;
  beta[0] = real(1);
  S[0] = e * M[0];
  D[0] = e * M[N];
  static_for<N - 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value + 1;
    constexpr int n = T.n[k];
    constexpr int i10 = T.m1[k][0], i11 = T.m1[k][1], i12 = T.m1[k][2];
    constexpr int i20 = T.m2[k][0], i21 = T.m2[k][1], i22 = T.m2[k][2];
    constexpr bool has2 = i20 >= 0 || i21 >= 0 || i22 >= 0;
    real s1a = real(0), s2a = real(0), s1b = real(0), s2b = real(0);
    if constexpr (i10 >= 0) {
      s1a += dx * alpha[i10];
      s1b += dx * beta[i10];
    }
    if constexpr (i11 >= 0) {
      s1a += dy * alpha[i11];
      s1b += dy * beta[i11];
    }
    if constexpr (i12 >= 0) {
      s1a += dz * alpha[i12];
      s1b += dz * beta[i12];
    }
    if constexpr (i20 >= 0) {
      s2a += alpha[i20];
      s2b += beta[i20];
    }
    if constexpr (i21 >= 0) {
      s2a += alpha[i21];
      s2b += beta[i21];
    }
    if constexpr (i22 >= 0) {
      s2a += alpha[i22];
      s2b += beta[i22];
    }
    if constexpr (has2) {
      alpha[k] = s1a - A[n] * s2a + B[n] * s1b - C[n] * s2b;
      if constexpr (n < P) beta[k] = s1a - V[n] * s2a;
    } else {
      alpha[k] = s1a + B[n] * s1b;
      if constexpr (n < P) beta[k] = s1a;
    }
    S[n] += alpha[k] * M[k];
    D[n] += alpha[k] * M[N + k];
  });
  real hs = S[P], hd = D[P];
  static_for<P>([&](auto nc) {
    constexpr int n = P - decltype(nc)::value;  // P .. 1
    constexpr real c1 = real(2 * n - 1) / real(n);
    const real g = c1 * r2inv;
    hs = S[n - 1] + g * hs;
    hd = D[n - 1] + g * hd;
  });
  s += rinv * hs;
  d += rinv * hd;
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
// Both kernels in the degree-scaled form: set-up (d, r^2, rsqrt, 1/r^2 [, r,
// exp], R^2 again, the per-degree factors), per coefficient the index sums,
// the combination and the two contractions, then Horner over the degrees.
inline double m2p_flop_one(int P, int kind) {
  double f = kind == 0 ? 11.0 + 5.0 + (P - 1) + 5.0 * P + 4.0
                       : 16.0 + 5.0 + 6.0 + 4.0 * P + 5.0 * P + 4.0;
  for (int deg = 0; deg <= P; ++deg)
    for (int a = deg; a >= 0; --a)
      for (int b = deg - a; b >= 0; --b) {
        const int c = deg - a - b;
        if (deg == 0) {
          f += kind ? 2.0 : 0.0;
          continue;
        }
        const int nz1 = (a >= 1) + (b >= 1) + (c >= 1);
        const int nz2 = (a >= 2) + (b >= 2) + (c >= 2);
        const double s1 = 2.0 * nz1 - 1.0, s2 = nz2 > 0 ? nz2 - 1.0 : 0.0;
        if (kind == 0)
          f += s1 + s2 + (nz2 ? 2.0 : 0.0) + 4.0;
        else
          f += 2.0 * (s1 + s2) + (nz2 ? 6.0 : 2.0) + (deg < P ? (nz2 ? 2.0 : 0.0) : 0.0) + 4.0;
      }
  return f;
}

// The same for the transposed operator's pair (target normal n at the
// Gauss point, source weights muS and muD): d, r^2, rsqrt, n.d, 1/r^2 (15),
// Laplace single + double layer (6), Yukawa (12) per kernel.
inline double adj_p2p_flop_per_pair(int ks) {
  switch (ks) {
    case KS_L: return 21.0;
    case KS_Y: return 27.0;
    case KS_LY: return 33.0;
    default: return 39.0;
  }
}

// Operations of one transposed (target Gauss point, cell) evaluation as
// written in the transposed M2P: the degree-scaled recurrence to order
// P + 1, the single-layer contraction to P, the three gradient contractions
// to P + 1 and Horner's rule over the degrees (FMA = 2).
inline double adj_m2p_flop_one(int P, int kind) {
  const int Q = P + 1;
  double f = kind == 0 ? 11.0 + 5.0 + (Q - 1) : 16.0 + 5.0 + 9.0 + 4.0 * (Q - 1);
  f += 1.0;                          // S_0
  f += 5.0 + 4.0;                    // n . F_Q, the two final products
  f += 8.0 * Q + 2.0 * P;            // Horner: g_n, n . F_n, two FMAs (one to P)
  for (int deg = 1; deg <= Q; ++deg)
    for (int a = deg; a >= 0; --a)
      for (int b = deg - a; b >= 0; --b) {
        const int c = deg - a - b;
        const int nz1 = (a >= 1) + (b >= 1) + (c >= 1);
        const int nz2 = (a >= 2) + (b >= 2) + (c >= 2);
        const double s1 = 2.0 * nz1 - 1.0, s2 = nz2 > 0 ? nz2 - 1.0 : 0.0;
        if (kind == 0)
          f += s1 + s2 + (nz2 ? 2.0 : 0.0);
        else
          f += 2.0 * (s1 + s2) + (nz2 ? 6.0 : 2.0) + (deg < Q ? (nz2 ? 2.0 : 0.0) : 0.0);
        f += (deg <= P ? 2.0 : 0.0) + 2.0 * nz1;  // contractions
      }
  return f;
}

inline double adj_m2p_flop_per_eval(int P, int ks) {
  switch (ks) {
    case KS_L: return adj_m2p_flop_one(P, 0);
    case KS_Y: return adj_m2p_flop_one(P, 1);
    case KS_LY: return adj_m2p_flop_one(P, 0) + adj_m2p_flop_one(P, 1);
    default: return 2.0 * adj_m2p_flop_one(P, 1);
  }
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
