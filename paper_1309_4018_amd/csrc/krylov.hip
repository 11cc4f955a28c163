// GMRES on the device (sec. 2.3: a Krylov solver doing one treecode
// evaluation per iteration; the parameter tables give the tolerance).
//
// Restarted GMRES in FP64: Arnoldi by classical Gram-Schmidt applied twice
// (CGS2), Givens rotations on the Hessenberg column, the implicit residual
// |g_{j+1}| / ||b|| read back once per iteration, back substitution and the
// update x += V y on the device.  FP32_REFINED wraps GMRES on the FP32
// operator in FP64 iterative refinement: r = b - A_64 x, solve A_32 d = r,
// x += d, until the FP64 residual meets the tolerance.  The energy is the
// FP64 sum 1/2 * 4 pi k_e * sum_k q_k phi_reac(x_k) (Eq. solv).
#include <algorithm>
#include <chrono>
#include <cmath>

#include "device_util.h"

namespace pbtc {

int apply_operator(pbtc_plan& pl, hipStream_t st, const double* x, double* y, int precision,
                   int phase);
int apply_transpose(pbtc_plan& pl, hipStream_t st, const double* x, double* y, int precision,
                    int phase);

namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 512;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kRedThreads / 64; ++i) t += lds[i];
  return t;
}

// partial[b * nv + i] = sum over block b's slice of V[i] . w  (i < nv)
__global__ __launch_bounds__(kRedThreads) void k_dots(const double* __restrict__ V, int nv,
                                                      int64_t n, const double* __restrict__ w,
                                                      double* __restrict__ partial) {
  __shared__ double lds[kRedThreads / 64];
  const int64_t stride = (int64_t)gridDim.x * kRedThreads;
  for (int i = 0; i < nv; ++i) {
    double s = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; j < n; j += stride)
      s += V[(size_t)i * n + j] * w[j];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * nv + i] = s;
  }
}

// out[i] (+)= sum_b partial[b * nv + i]
__global__ void k_sum_partials(const double* __restrict__ partial, int nb, int nv,
                               double* __restrict__ out, int accumulate) {
  __shared__ double lds[kRedThreads / 64];
  for (int i = 0; i < nv; ++i) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kRedThreads) s += partial[(size_t)b * nv + i];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) out[i] = accumulate ? out[i] + s : s;
  }
}

// w -= sum_i h[i] V[i]
__global__ void k_sub_combo(const double* __restrict__ V, int nv, int64_t n,
                            const double* __restrict__ h, double* __restrict__ w) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = w[j];
  for (int i = 0; i < nv; ++i) s -= h[i] * V[(size_t)i * n + j];
  w[j] = s;
}

// x += sum_i y[i] V[i]
__global__ void k_add_combo(const double* __restrict__ V, int nv, int64_t n,
                            const double* __restrict__ y, double* __restrict__ x) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = x[j];
  for (int i = 0; i < nv; ++i) s += y[i] * V[(size_t)i * n + j];
  x[j] = s;
}

__global__ void k_scale(const double* __restrict__ w, int64_t n, const double* __restrict__ s,
                        int invert, double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double f = invert ? (s[0] > 0.0 ? 1.0 / s[0] : 0.0) : s[0];
  out[j] = w[j] * f;
}

// out = a - b
__global__ void k_sub(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                      double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = a[j] - b[j];
}

__global__ void k_axpy(double alpha, const double* __restrict__ a, int64_t n, double* __restrict__ y) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) y[j] += alpha * a[j];
}

__global__ void k_fill(double* p, int64_t n, double v) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) p[j] = v;
}

__global__ void k_sqrt(double* p) { p[0] = sqrt(fmax(p[0], 0.0)); }

// Givens step for column j: H(:, j) = h (CGS2 sum), H(j+1, j) = hnorm; apply
// the stored rotations, form the new one, update g and the residual estimate.
// H column-major with leading dimension ld.  giv = [cs (m+1), sn (m+1), g (m+2)].
__global__ void k_givens(int j, int ld, const double* __restrict__ h, const double* __restrict__ hn,
                         double* __restrict__ H, double* __restrict__ giv, double bnorm,
                         double* __restrict__ res) {
  double* cs = giv;
  double* sn = giv + ld;
  double* g = giv + 2 * ld;
  double* col = H + (size_t)j * ld;
  for (int i = 0; i <= j; ++i) col[i] = h[i];
  col[j + 1] = hn[0];
  for (int i = 0; i < j; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i] = cs[i] * a + sn[i] * b;
    col[i + 1] = -sn[i] * a + cs[i] * b;
  }
  const double a = col[j], b = col[j + 1];
  const double den = hypot(a, b);
  const double c = den > 0.0 ? a / den : 1.0, s = den > 0.0 ? b / den : 0.0;
  cs[j] = c;
  sn[j] = s;
  col[j] = den;
  col[j + 1] = 0.0;
  g[j + 1] = -s * g[j];
  g[j] = c * g[j];
  res[0] = fabs(g[j + 1]) / bnorm;
}

// y = R^{-1} g (upper triangular, k columns)
__global__ void k_backsolve(int k, int ld, const double* __restrict__ H, const double* __restrict__ giv,
                            double* __restrict__ y) {
  const double* g = giv + 2 * ld;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int c = i + 1; c < k; ++c) s -= H[(size_t)c * ld + i] * y[c];
    const double d = H[(size_t)i * ld + i];
    y[i] = d != 0.0 ? s / d : 0.0;
  }
}

__global__ void k_init_g(double* giv, int ld, const double* beta) {
  double* g = giv + 2 * ld;
  for (int i = 0; i < ld + 1; ++i) g[i] = 0.0;
  g[0] = beta[0];
}

// 1/2 * C * sum_k q_k phi_k  (single block)
__global__ void k_energy(const double* __restrict__ q, const double* __restrict__ phi, int64_t n,
                         double factor, double* __restrict__ out) {
  __shared__ double lds[kRedThreads / 64];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kRedThreads) s += q[i] * phi[i];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) out[0] = factor * s;
}

}  // namespace

struct Krylov {
  pbtc_plan& pl;
  hipStream_t st;
  int64_t n;
  int m;
  double* V;
  double* H;
  double* giv;
  double* scal;  // [0] norm, [1] beta, [2] res, [3..] h and h2
  double* red;
  double* w;
  double* y;
  double* hbuf;
  double* h2buf;

  Krylov(pbtc_plan& p, hipStream_t s) : pl(p), st(s) {
    n = pl.nunk;
    m = pl.prm.restart;
    V = wsp<double>(pl, pl.o_V);
    H = wsp<double>(pl, pl.o_H);
    giv = wsp<double>(pl, pl.o_givens);
    scal = wsp<double>(pl, pl.o_scal);
    red = wsp<double>(pl, pl.o_red);
    w = wsp<double>(pl, pl.o_w);
    y = giv + 3 * (m + 1) + 1;
    hbuf = red + (size_t)kRedBlocks * (m + 2);
    h2buf = hbuf + (m + 2);
  }

  int blocks_for(int64_t len) const { return std::min<int>(kRedBlocks, nblocks(len, kRedThreads)); }

  // out[0..nv) = V[0..nv)^T v  (device)
  int dots(const double* Vb, int nv, const double* v, double* out, int accumulate) {
    const int nb = blocks_for(n);
    hipLaunchKernelGGL(k_dots, dim3(nb), dim3(kRedThreads), 0, st, Vb, nv, n, v, red);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kRedThreads), 0, st, red, nb, nv, out,
                       accumulate);
    PBTC_LAUNCH_CHECK();
    return PBTC_OK;
  }

  int norm(const double* v, double* out) {
    int rc = dots(v, 1, v, out, 0);
    if (rc) return rc;
    hipLaunchKernelGGL(k_sqrt, dim3(1), dim3(1), 0, st, out);
    return PBTC_OK;
  }

  double host_scalar(const double* d) {
    double v = 0.0;
    if (hipMemcpyAsync(&v, d, 8, hipMemcpyDeviceToHost, st) != hipSuccess) return NAN;
    if (hipStreamSynchronize(st) != hipSuccess) return NAN;
    return v;
  }
};

// GMRES for A z = rhs (A applied by `op`), z holds the start vector on entry
// (zero_start: z = 0).  Stops when the implicit residual <= tol * ref_norm.
template <typename Op>
static int gmres(pbtc_plan& pl, hipStream_t st, Op op, const double* rhs, double* z, bool zero_start,
                 double tol, double ref_norm, int max_iter, int* iters, std::vector<double>* hist,
                 bool* converged) {
  Krylov K(pl, st);
  const int T = 256;
  const int64_t n = K.n;
  const int m = K.m;
  const int ld = m + 1;
  double* r = wsp<double>(pl, pl.o_tmp);
  *converged = false;
  bool first = true;
  while (*iters < max_iter) {
    // r = rhs - A z
    if (zero_start && first) {
      hipLaunchKernelGGL(k_fill, dim3(nblocks(n, T)), dim3(T), 0, st, z, n, 0.0);
      PBTC_HIP(hipMemcpyAsync(r, rhs, 8 * n, hipMemcpyDeviceToDevice, st));
    } else {
      int rc = op(z, r);
      if (rc) return rc;
      hipLaunchKernelGGL(k_sub, dim3(nblocks(n, T)), dim3(T), 0, st, rhs, r, n, r);
    }
    first = false;
    int rc = K.norm(r, K.scal + 1);
    if (rc) return rc;
    const double beta = K.host_scalar(K.scal + 1);
    if (!std::isfinite(beta)) {
      pl.err = "GMRES: residual is not finite";
      return PBTC_EDEVICE;
    }
    if (beta <= tol * ref_norm) {
      *converged = true;
      break;
    }
    hipLaunchKernelGGL(k_scale, dim3(nblocks(n, T)), dim3(T), 0, st, r, n, K.scal + 1, 1, K.V);
    hipLaunchKernelGGL(k_init_g, dim3(1), dim3(1), 0, st, K.giv, ld, K.scal + 1);
    int j = 0;
    for (; j < m && *iters < max_iter; ++j) {
      double* vj = K.V + (size_t)j * n;
      double* vn = K.V + (size_t)(j + 1) * n;
      rc = op(vj, K.w);
      if (rc) return rc;
      // CGS2: two passes of classical Gram-Schmidt
      rc = K.dots(K.V, j + 1, K.w, K.hbuf, 0);
      if (rc) return rc;
      hipLaunchKernelGGL(k_sub_combo, dim3(nblocks(n, T)), dim3(T), 0, st, K.V, j + 1, n, K.hbuf,
                         K.w);
      rc = K.dots(K.V, j + 1, K.w, K.h2buf, 0);
      if (rc) return rc;
      hipLaunchKernelGGL(k_sub_combo, dim3(nblocks(n, T)), dim3(T), 0, st, K.V, j + 1, n, K.h2buf,
                         K.w);
      hipLaunchKernelGGL(k_axpy, dim3(1), dim3(T), 0, st, 1.0, K.h2buf, (int64_t)(j + 1), K.hbuf);
      rc = K.norm(K.w, K.scal);
      if (rc) return rc;
      hipLaunchKernelGGL(k_scale, dim3(nblocks(n, T)), dim3(T), 0, st, K.w, n, K.scal, 1, vn);
      hipLaunchKernelGGL(k_givens, dim3(1), dim3(1), 0, st, j, ld, K.hbuf, K.scal, K.H, K.giv,
                         ref_norm, K.scal + 2);
      PBTC_LAUNCH_CHECK();
      const double res = K.host_scalar(K.scal + 2);
      ++*iters;
      if (hist) hist->push_back(res);
      if (!std::isfinite(res)) {
        pl.err = "GMRES: residual estimate is not finite";
        return PBTC_EDEVICE;
      }
      if (res <= tol) {
        ++j;
        *converged = true;
        break;
      }
    }
    const int k = std::min(j, m);
    if (k > 0) {
      hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(1), 0, st, k, ld, K.H, K.giv, K.y);
      hipLaunchKernelGGL(k_add_combo, dim3(nblocks(n, T)), dim3(T), 0, st, K.V, k, n, K.y, z);
      PBTC_LAUNCH_CHECK();
    }
    if (*converged) break;
  }
  return PBTC_OK;
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Solve on a set-up workspace; fills res (timings from t_setup on).
int device_solve(pbtc_plan& pl, hipStream_t st, pbtc_result* res) {
  const int T = 256;
  const int64_t n = pl.nunk;
  double* b = wsp<double>(pl, pl.o_b);
  double* x = wsp<double>(pl, pl.o_x);
  double* r = wsp<double>(pl, pl.o_r);
  double* d = wsp<double>(pl, pl.o_lam);  // correction of a refinement step
  Krylov K(pl, st);
  pl.history.clear();
  int iters = 0, n32 = 0, n64 = 0, nref = 0;
  bool conv = false;
  const double t0 = now_s();
  int rc = K.norm(b, K.scal + 4);
  if (rc) return rc;
  const double bnorm = K.host_scalar(K.scal + 4);
  auto op64 = [&](const double* in, double* out) {
    ++n64;
    return apply_operator(pl, st, in, out, PBTC_FP64, 0);
  };
  auto op32 = [&](const double* in, double* out) {
    ++n32;
    return apply_operator(pl, st, in, out, PBTC_FP32, 0);
  };
  double rel = 1.0;
  if (bnorm == 0.0) {
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n, T)), dim3(T), 0, st, x, n, 0.0);
    conv = true;
    rel = 0.0;
  } else if (pl.prm.precision == PBTC_FP32_REFINED) {
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n, T)), dim3(T), 0, st, x, n, 0.0);
    PBTC_HIP(hipMemcpyAsync(r, b, 8 * n, hipMemcpyDeviceToDevice, st));
    double rnorm = bnorm;
    for (nref = 0; nref < pl.prm.max_refine && iters < pl.prm.max_iter; ++nref) {
      // inner solve of A d = r to a relative tolerance that lands the outer
      // residual below tol, but not below what the FP32 operator resolves
      const double want = 0.5 * pl.prm.tol * bnorm / rnorm;
      const double tin = std::min(0.5, std::max(want, pl.prm.inner_tol));
      bool cin = false;
      rc = gmres(pl, st, op32, r, d, true, tin, rnorm, pl.prm.max_iter, &iters, &pl.history, &cin);
      if (rc) return rc;
      hipLaunchKernelGGL(k_axpy, dim3(nblocks(n, T)), dim3(T), 0, st, 1.0, d, n, x);
      rc = op64(x, r);
      if (rc) return rc;
      hipLaunchKernelGGL(k_sub, dim3(nblocks(n, T)), dim3(T), 0, st, b, r, n, r);
      rc = K.norm(r, K.scal + 5);
      if (rc) return rc;
      rnorm = K.host_scalar(K.scal + 5);
      rel = rnorm / bnorm;
      if (rel <= pl.prm.tol) {
        conv = true;
        ++nref;
        break;
      }
    }
  } else {
    const int prec = pl.prm.precision == PBTC_FP64 ? PBTC_FP64 : PBTC_FP32;
    bool c = false;
    if (prec == PBTC_FP64)
      rc = gmres(pl, st, op64, b, x, true, pl.prm.tol, bnorm, pl.prm.max_iter, &iters, &pl.history, &c);
    else
      rc = gmres(pl, st, op32, b, x, true, pl.prm.tol, bnorm, pl.prm.max_iter, &iters, &pl.history, &c);
    if (rc) return rc;
    // explicit FP64 residual
    rc = op64(x, r);
    if (rc) return rc;
    hipLaunchKernelGGL(k_sub, dim3(nblocks(n, T)), dim3(T), 0, st, b, r, n, r);
    rc = K.norm(r, K.scal + 5);
    if (rc) return rc;
    rel = K.host_scalar(K.scal + 5) / bnorm;
    // FP64: implicit or explicit residual meets tol; FP32 without refinement:
    // the implicit residual of the FP32 operator meets tol (rel is reported)
    conv = c || (prec == PBTC_FP64 && rel <= pl.prm.tol);
  }
  PBTC_HIP(hipStreamSynchronize(st));
  const double t1 = now_s();
  // reaction potential at the charges (FP64 treecode) and the energy
  double* phi = wsp<double>(pl, pl.o_phi_reac);
  rc = apply_operator(pl, st, x, phi, PBTC_FP64, 1);
  if (rc) return rc;
  hipLaunchKernelGGL(k_energy, dim3(1), dim3(kRedThreads), 0, st, wsp<double>(pl, pl.o_q), phi,
                     pl.nq, 0.5 * 4.0 * kPi * kCoulomb, wsp<double>(pl, pl.o_energy));
  PBTC_LAUNCH_CHECK();
  pl.energy = K.host_scalar(wsp<double>(pl, pl.o_energy));
  const double t2 = now_s();
  pl.x_host.resize(n);
  pl.phi_reac_host.resize(pl.nq);
  PBTC_HIP(hipMemcpyAsync(pl.x_host.data(), x, 8 * n, hipMemcpyDeviceToHost, st));
  PBTC_HIP(hipMemcpyAsync(pl.phi_reac_host.data(), phi, 8 * pl.nq, hipMemcpyDeviceToHost, st));
  PBTC_HIP(hipStreamSynchronize(st));
  pl.solved = true;
  if (res) {
    res->energy_kJmol = pl.energy;
    res->n_iter = iters;
    res->converged = conv ? 1 : 0;
    res->final_rel_res = rel;
    res->n_matvec_fp32 = n32;
    res->n_matvec_fp64 = n64;
    res->n_refine = nref;
    res->t_solve_s = t1 - t0;
    res->t_energy_s = t2 - t1;
  }
  if (!conv) {
    pl.err = "GMRES did not reach the tolerance within max_iter";
    return PBTC_ENOCONV;
  }
  return PBTC_OK;
}

double wall_seconds() { return now_s(); }

}  // namespace pbtc
