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
// Optional right preconditioning by the per-panel 2 x 2 diagonal blocks:
// GMRES on A M^-1 (residuals are those of A, so the stopping test is
// unchanged), x += M^-1 V y at the end of each cycle.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "device_util.h"

namespace pbtc {

int apply_operator(pbtc_plan_t& pl, hipStream_t st, const double* x, double* y, int precision,
                   int phase);
int apply_transpose(pbtc_plan_t& pl, hipStream_t st, const double* x, double* y, int precision,
                    int phase);
void prof_collect(pbtc_plan_t& pl);

// per-system scalar arrays of the Krylov state
enum { SC_BNORM = 0, SC_RES, SC_ACTIVE, SC_BETA, SC_HN, SC_TOL, SC_KFIN, SC_REF, SC_NORM, SC_N };

namespace {

constexpr int kRedThreads = 256;

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

// y = M^-1 x or M^-T x for the per-panel 2 x 2 blocks inv (row-major);
// pidx[2p], pidx[2p+1]: the phi and psi entries of panel p (equal to its
// inner- and outer-region rows).  accumulate: y += instead of y =.
__global__ void k_prec_apply(int64_t np, const int* __restrict__ pidx, const double* __restrict__ inv,
                             const double* __restrict__ x, double* __restrict__ y, int transpose,
                             int accumulate) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int i0 = pidx[2 * p], i1 = pidx[2 * p + 1];
  const double a = x[i0], b = x[i1];
  const double m00 = inv[4 * p], m01 = inv[4 * p + 1], m10 = inv[4 * p + 2], m11 = inv[4 * p + 3];
  const double y0 = transpose ? m00 * a + m10 * b : m00 * a + m01 * b;
  const double y1 = transpose ? m01 * a + m11 * b : m10 * a + m11 * b;
  y[i0] = accumulate ? y[i0] + y0 : y0;
  y[i1] = accumulate ? y[i1] + y1 : y1;
}

__global__ void k_fill(double* p, int64_t n, double v) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) p[j] = v;
}

// partial[chunk * ld + i] = <V_i, w> over the chunk; one block per (chunk, i).
// A chunk holds at most kDotChunk entries: each thread's kDotChunk /
// kRedThreads loads are issued together (indices past the chunk read its last
// entry and add nothing), then summed in entry order.
__global__ __launch_bounds__(kRedThreads) void k_dots_seg(const double* __restrict__ V, int nv,
                                                          int64_t n, const double* __restrict__ w,
                                                          const int4* __restrict__ chunks,
                                                          double* __restrict__ partial, int ld) {
  constexpr int kPer = kDotChunk / kRedThreads;
  __shared__ double lds[kRedThreads / 64];
  const int4 ch = chunks[blockIdx.x];
  const int i = blockIdx.y;
  const double* v = V + (size_t)i * n;
  double a[kPer], b[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int64_t j = min((int64_t)ch.y + threadIdx.x + (int64_t)k * kRedThreads, (int64_t)ch.z - 1);
    a[k] = v[j];
    b[k] = w[j];
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    s += (ch.y + (int)threadIdx.x + k * kRedThreads < ch.z ? a[k] : 0.0) * b[k];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) partial[(size_t)blockIdx.x * ld + i] = s;
}

// out[c * ldo + i] = sum of the chunk partials of system c: one wavefront
// per (system c = blockIdx.x, i = blockIdx.y), lanes strided over the chunks,
// then a fixed butterfly; with root set, the square root.
__global__ void k_sum_seg(const double* __restrict__ partial, int pld, const int* __restrict__ chunk0,
                          int ldo, int root, double* __restrict__ out) {
  const int c = blockIdx.x, i = blockIdx.y;
  double s = 0.0;
  for (int b = chunk0[c] + (int)threadIdx.x; b < chunk0[c + 1]; b += 64)
    s += partial[(size_t)b * pld + i];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[(size_t)c * ldo + i] = root ? sqrt(fmax(s, 0.0)) : s;
}

// w -= sum_i h[c, i] V_i on the entries of system c
__global__ void k_sub_combo_seg(const double* __restrict__ V, int nv, int64_t n,
                                const double* __restrict__ h, int ld, const int* __restrict__ comp,
                                double* __restrict__ w) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double* hc = h + (size_t)comp[j] * ld;
  double s = w[j];
  for (int i = 0; i < nv; ++i) s -= hc[i] * V[(size_t)i * n + j];
  w[j] = s;
}

// out[c] = sqrt of the sum of partial[b] over b in [chunk0[c] * per,
// chunk0[c + 1] * per): one wavefront per system, lanes strided, then a fixed
// butterfly.
__global__ void k_norm_seg(const double* __restrict__ partial, const int* __restrict__ chunk0,
                           int per, double* __restrict__ out) {
  const int c = blockIdx.x;
  double s = 0.0;
  for (int b = chunk0[c] * per + (int)threadIdx.x; b < chunk0[c + 1] * per; b += 64) s += partial[b];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[c] = sqrt(fmax(s, 0.0));
}

// Second Gram-Schmidt pass fused with the norm: w -= sum_i h[c, i] V_i, and
// partial[b] = sum of w^2 over block b's part of its chunk (kChunkBlocks
// blocks of kRedThreads entries per chunk; a chunk lies in one system c).
constexpr int kChunkBlocks = kDotChunk / kRedThreads;
static_assert(kChunkBlocks * kRedThreads == kDotChunk, "chunks split into whole blocks");

__global__ __launch_bounds__(kRedThreads) void k_sub_combo_norm_seg(
    const double* __restrict__ V, int nv, int64_t n, const double* __restrict__ h, int ld,
    const int4* __restrict__ chunks, double* __restrict__ w, double* __restrict__ partial) {
  __shared__ double lds[kRedThreads / 64];
  const int4 ch = chunks[blockIdx.x / kChunkBlocks];
  const int64_t j = ch.y + (int64_t)(blockIdx.x % kChunkBlocks) * kRedThreads + threadIdx.x;
  double sq = 0.0;
  if (j < ch.z) {
    const double* hc = h + (size_t)ch.x * ld;
    double s = w[j];
    for (int i = 0; i < nv; ++i) s -= hc[i] * V[(size_t)i * n + j];
    w[j] = s;
    sq = s * s;
  }
  sq = block_sum(sq, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = sq;
}

// One Gram-Schmidt pass with its coefficient sums folded in: every block
// (kChunkBlocks per chunk, a chunk lies in one system c) first forms
// h[c, i] = sum of the chunk partials of system c (thread i adds them in
// chunk order: the same value in every block), the system's first block
// stores it in hout, then w -= sum_i h[c, i] V_i on the block's entries.  The
// first kVecs basis vectors' entries are loaded before the sums, so that both
// sets of loads are in flight together.  With NORM, partial norms of the new
// w per block go to nrm.
template <bool NORM>
__global__ __launch_bounds__(kRedThreads) void k_gs_pass_seg(
    const double* __restrict__ V, int nv, int64_t n, const double* __restrict__ partial, int pld,
    const int4* __restrict__ chunks, const int* __restrict__ chunk0, double* __restrict__ hout,
    int ld, double* __restrict__ w, double* __restrict__ nrm) {
  constexpr int kVecs = 16, kParts = 16;
  extern __shared__ double hl[];  // nv coefficients
  __shared__ double lds[kRedThreads / 64];
  const int4 ch = chunks[blockIdx.x / kChunkBlocks];
  const int c = ch.x;
  const int b0 = chunk0[c], b1 = chunk0[c + 1];
  const bool first = (int)blockIdx.x == b0 * kChunkBlocks;
  const int64_t j = ch.y + (int64_t)(blockIdx.x % kChunkBlocks) * kRedThreads + threadIdx.x;
  const bool in = j < ch.z;
  const int64_t jc = in ? j : (int64_t)ch.z - 1;  // V loads of lanes past the chunk
  // basis vectors past nv: the last one again, with a zero coefficient
  double x[kVecs];
#pragma unroll
  for (int k = 0; k < kVecs; ++k) x[k] = V[(size_t)min(k, nv - 1) * n + jc];
  double s = in ? w[j] : 0.0;  // (w[j] is written below by its own thread only)
  for (int i = threadIdx.x; i < nv; i += kRedThreads) {
    double h = 0.0;
    for (int b = b0; b < b1; b += kParts) {
      double p[kParts];
#pragma unroll
      for (int k = 0; k < kParts; ++k) p[k] = partial[(size_t)min(b + k, b1 - 1) * pld + i];
#pragma unroll
      for (int k = 0; k < kParts; ++k) h += b + k < b1 ? p[k] : 0.0;
    }
    hl[i] = h;
    if (first) hout[(size_t)c * ld + i] = h;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kVecs; ++k) s -= (k < nv ? hl[min(k, nv - 1)] : 0.0) * x[k];
  for (int i0 = kVecs; i0 < nv; i0 += kVecs) {
#pragma unroll
    for (int k = 0; k < kVecs; ++k) x[k] = V[(size_t)min(i0 + k, nv - 1) * n + jc];
#pragma unroll
    for (int k = 0; k < kVecs; ++k) s -= (i0 + k < nv ? hl[min(i0 + k, nv - 1)] : 0.0) * x[k];
  }
  double sq = 0.0;
  if (in) {
    w[j] = s;
    sq = s * s;
  }
  if (NORM) {
    sq = block_sum(sq, lds);
    if (threadIdx.x == 0) nrm[blockIdx.x] = sq;
  }
}

// out = w / s[c] for active systems, 0 for the others (also into out2 if given)
__global__ void k_scale_seg(const double* __restrict__ w, int64_t n, const double* __restrict__ s,
                            const int* __restrict__ comp, const double* __restrict__ active,
                            double* __restrict__ out, double* __restrict__ out2) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int c = comp[j];
  const double v = (active[c] > 0.0 && s[c] > 0.0) ? w[j] / s[c] : 0.0;
  out[j] = v;
  if (out2) out2[j] = v;
}

// start of a restart cycle: g = (beta, 0, ...), kfin = 0
__global__ void k_init_seg(int nc, double* giv, int gstride, int ld, const double* beta,
                           double* kfin) {
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    double* g = giv + (size_t)c * gstride + 2 * ld;
    for (int i = 0; i < ld + 1; ++i) g[i] = 0.0;
    g[0] = beta[c];
    kfin[c] = 0.0;
  }
}

// Givens step for column j of active system c (one work-group): H(:, j) =
// h + h2 (the two Gram-Schmidt passes), H(j+1, j) = hn; apply the stored
// rotations, form the new one, update g, and deactivate the system once
// |g_{j+1}| <= tol * ref (kfin = j + 1).  The column and the rotations pass
// through LDS; the rotations themselves are sequential.  hout (or null):
// pinned host memory that receives [residual estimate, active flag] of every
// system (2 nc values), read by the host behind the event recorded after the
// launch.  Shared by k_givens_seg and k_norm_givens_seg.
__device__ void givens_step(int c, int nc, int j, int ld, const double* __restrict__ h,
                            const double* __restrict__ h2, double* __restrict__ H,
                            double* __restrict__ giv, int gstride, double* __restrict__ sc,
                            double* __restrict__ hout, double hn, double* lds) {
  double* act = sc + (size_t)SC_ACTIVE * nc;
  if (act[c] <= 0.0) {
    if (hout && threadIdx.x == 0) {
      hout[c] = sc[(size_t)SC_RES * nc + c];
      hout[nc + c] = 0.0;
    }
    return;
  }
  double* cs = giv + (size_t)c * gstride;
  double* sn = cs + ld;
  double* g = cs + 2 * ld;
  double* col = H + ((size_t)c * ld + j) * ld;
  const double* hc = h + (size_t)c * ld;
  const double* h2c = h2 + (size_t)c * ld;
  double* lc = lds;
  double* lcs = lds + ld + 1;
  double* lsn = lcs + ld;
  for (int i = threadIdx.x; i <= j; i += blockDim.x) {
    lc[i] = hc[i] + h2c[i];
    if (i < j) {
      lcs[i] = cs[i];
      lsn[i] = sn[i];
    }
  }
  if (threadIdx.x == 0) lc[j + 1] = hn;
  __syncthreads();
  if (threadIdx.x == 0) {
    // rotation i mixes entries i and i + 1; the running entry stays in a
    // register, so only the chain of FMAs is sequential
    double a = lc[0];
#pragma unroll 4
    for (int i = 0; i < j; ++i) {
      const double b = lc[i + 1];
      lc[i] = lcs[i] * a + lsn[i] * b;
      a = -lsn[i] * a + lcs[i] * b;
    }
    const double b = lc[j + 1];
    const double den = hypot(a, b);
    const double cc = den > 0.0 ? a / den : 1.0, ss = den > 0.0 ? b / den : 0.0;
    cs[j] = cc;
    sn[j] = ss;
    lc[j] = den;
    lc[j + 1] = 0.0;
    g[j + 1] = -ss * g[j];
    g[j] = cc * g[j];
    const double ref = sc[(size_t)SC_REF * nc + c];
    const double res = fabs(g[j + 1]) / ref;
    sc[(size_t)SC_RES * nc + c] = res;
    if (res <= sc[(size_t)SC_TOL * nc + c] || den == 0.0) {
      act[c] = 0.0;
      sc[(size_t)SC_KFIN * nc + c] = j + 1;
    }
    if (hout) {
      hout[c] = res;
      hout[nc + c] = act[c];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) col[i] = lc[i];
}

// Givens step of every system (one work-group of 64 per system), H(j+1, j)
// from the norms the second pass stored
__global__ void k_givens_seg(int nc, int j, int ld, const double* __restrict__ h,
                             const double* __restrict__ h2, double* __restrict__ H,
                             double* __restrict__ giv, int gstride, double* __restrict__ sc,
                             double* __restrict__ hout) {
  extern __shared__ double lds[];  // col (ld + 1), cs (ld), sn (ld)
  const int c = blockIdx.x;
  givens_step(c, nc, j, ld, h, h2, H, giv, gstride, sc, hout, sc[(size_t)SC_HN * nc + c], lds);
}

// The second Gram-Schmidt pass's norm of every system, then (one launch,
// after k_gs_pass_seg<true>): work-groups 0 .. nc-1 do the Givens step of
// column j of system c = blockIdx.x exactly as k_givens_seg (with that norm
// as H(j+1, j)), the others write the new basis vector out = w / ||w|| (and
// out2) for every system, active or not (an inactive system's later columns
// are never used).  Each work-group forms the norm itself from the partials
// (lanes strided over the system's partials, then a fixed butterfly).
__global__ __launch_bounds__(kRedThreads) void k_norm_givens_seg(
    int nc, int j, int ld, const double* __restrict__ w, const double* __restrict__ nrm,
    const int4* __restrict__ chunks, const int* __restrict__ chunk0,
    const double* __restrict__ h, const double* __restrict__ h2, double* __restrict__ H,
    double* __restrict__ giv, int gstride, double* __restrict__ sc, double* __restrict__ hout,
    double* __restrict__ out, double* __restrict__ out2) {
  extern __shared__ double lds[];  // Givens: col (ld + 1), cs (ld), sn (ld)
  __shared__ double norm;
  const bool gblock = (int)blockIdx.x < nc;
  const int sb = (int)blockIdx.x - nc;  // scaling work-group
  const int4 ch = gblock ? make_int4(0, 0, 0, 0) : chunks[sb / kChunkBlocks];
  const int c = gblock ? (int)blockIdx.x : ch.x;
  if (threadIdx.x < 64) {
    // lanes strided over the partials, kU of a lane's loads in flight together
    constexpr int kU = 8;
    const int e0 = chunk0[c] * kChunkBlocks, e1 = chunk0[c + 1] * kChunkBlocks;
    double s = 0.0;
    for (int b = e0 + (int)threadIdx.x; b < e1; b += 64 * kU) {
      double p[kU];
#pragma unroll
      for (int k = 0; k < kU; ++k) p[k] = nrm[min(b + 64 * k, e1 - 1)];
#pragma unroll
      for (int k = 0; k < kU; ++k) s += b + 64 * k < e1 ? p[k] : 0.0;
    }
    s = wave_sum(s);
    if (threadIdx.x == 0) norm = sqrt(fmax(s, 0.0));
  }
  __syncthreads();
  if (!gblock) {
    const int64_t i = ch.y + (int64_t)(sb % kChunkBlocks) * kRedThreads + threadIdx.x;
    if (i < ch.z) {
      const double v = norm > 0.0 ? w[i] / norm : 0.0;
      out[i] = v;
      if (out2) out2[i] = v;
    }
    return;
  }
  if (threadIdx.x == 0) sc[(size_t)SC_HN * nc + c] = norm;
  givens_step(c, nc, j, ld, h, h2, H, giv, gstride, sc, hout, norm, lds);
}

// end of a cycle: kfin of still-active systems = columns built; y = R^-1 g
__global__ void k_finish_seg(int nc, int ncol, int ld, const double* __restrict__ H,
                             double* __restrict__ giv, int gstride, double* __restrict__ sc) {
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    double* kf = sc + (size_t)SC_KFIN * nc;
    if (sc[(size_t)SC_ACTIVE * nc + c] > 0.0) kf[c] = ncol;
    const int k = (int)kf[c];
    const double* Hc = H + (size_t)c * ld * ld;
    const double* g = giv + (size_t)c * gstride + 2 * ld;
    double* y = giv + (size_t)c * gstride + 3 * ld + 1;
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int q = i + 1; q < k; ++q) s -= Hc[(size_t)q * ld + i] * y[q];
      const double d = Hc[(size_t)i * ld + i];
      y[i] = d != 0.0 ? s / d : 0.0;
    }
  }
}

// x += sum_{i < kfin[c]} y[c, i] V_i on the entries of system c
__global__ void k_add_combo_seg(const double* __restrict__ V, int64_t n, const double* __restrict__ giv,
                                int gstride, int ld, const double* __restrict__ kfin,
                                const int* __restrict__ comp, double* __restrict__ x) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int c = comp[j];
  const int k = (int)kfin[c];
  const double* y = giv + (size_t)c * gstride + 3 * ld + 1;
  double s = x[j];
  for (int i = 0; i < k; ++i) s += y[i] * V[(size_t)i * n + j];
  x[j] = s;
}

// energy of every system: 1/2 C sum over its charges of q phi
__global__ void k_energy_seg(const double* __restrict__ q, const double* __restrict__ phi,
                             const int* __restrict__ cq, int64_t n, double factor,
                             double* __restrict__ out) {
  __shared__ double lds[kRedThreads / 64];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kRedThreads)
    if (cq[i] == c) s += q[i] * phi[i];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) out[c] = factor * s;
}

// phi_c[i] = sum over the other charges j of i's region of q_j / (eps_r |x_i - x_j|)
__global__ void k_coulomb_pot(int64_t nq, const double* __restrict__ qxyz,
                              const double* __restrict__ q, const int* __restrict__ qreg,
                              const long long* __restrict__ qoff, const double* __restrict__ eps,
                              double* __restrict__ phi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const int r = qreg[i];
  const double x = qxyz[3 * i], y = qxyz[3 * i + 1], z = qxyz[3 * i + 2];
  double s = 0.0;
  for (long long j = qoff[r]; j < qoff[r + 1]; ++j) {
    if (j == i) continue;
    const double dx = x - qxyz[3 * j], dy = y - qxyz[3 * j + 1], dz = z - qxyz[3 * j + 2];
    s += q[j] / sqrt(dx * dx + dy * dy + dz * dz);
  }
  phi[i] = s / eps[r];
}

}  // namespace

// Krylov state of every independent system (a connected component of the
// region graph): H, Givens data and scalars live per system in o_kstate;
// vector operations run over the whole unknown vector, reductions per system.
struct Krylov {
  pbtc_plan_t& pl;
  hipStream_t st;
  int64_t n;
  int m, ld, nc, nchunks;
  double* V;
  double* H;      // nc x ld x ld, column-major per system
  double* giv;    // nc x gstride: cs (ld), sn (ld), g (ld + 1), y (ld + 1)
  int gstride;
  double* sc;     // SC_N x nc
  double* red;    // partials: nchunks x ld
  double* hbuf;   // nc x ld
  double* h2buf;  // nc x ld
  double* nrm;    // norm partials of the fused second pass: nchunks x kChunkBlocks
  double* w;
  bool fuse;      // coefficient sums folded into the Gram-Schmidt passes
  const int4* chunks;
  const int* chunk0;
  const int* comp;

  Krylov(pbtc_plan_t& p, hipStream_t s) : pl(p), st(s) {
    n = pl.nunk;
    m = pl.prm.restart;
    ld = m + 1;
    nc = pl.ncomp;
    nchunks = (int)pl.dot_chunks.size();
    gstride = 4 * (m + 2);
    V = wsp<double>(pl, pl.o_V);
    H = wsp<double>(pl, pl.o_kstate);
    giv = H + (size_t)nc * ld * ld;
    sc = giv + (size_t)nc * gstride;
    red = wsp<double>(pl, pl.o_red);
    hbuf = red + (size_t)nchunks * ld;
    h2buf = hbuf + (size_t)nc * ld;
    nrm = h2buf + (size_t)nc * ld;
    // every block of a fused pass re-reads its system's chunk partials:
    // worth it while systems span few chunks
    int maxch = 0;
    for (int c = 0; c < nc; ++c)
      maxch = std::max(maxch, pl.comp_chunk0[c + 1] - pl.comp_chunk0[c]);
    fuse = maxch <= 256;
    w = wsp<double>(pl, pl.o_w);
    chunks = wsp<int4>(pl, pl.o_chunks);
    chunk0 = reinterpret_cast<const int*>(chunks + nchunks);
    comp = wsp<int>(pl, pl.o_comp_of_unk);
  }
  double* scal(int which) { return sc + (size_t)which * nc; }

  // out[c * ld + i] = <V_i, v> over system c, i < nv
  int dots(const double* Vb, int nv, const double* v, double* out) {
    hipLaunchKernelGGL(k_dots_seg, dim3(nchunks, nv), dim3(kRedThreads), 0, st, Vb, nv, n, v,
                       chunks, red, ld);
    hipLaunchKernelGGL(k_sum_seg, dim3(nc, nv), dim3(64), 0, st, red, ld, chunk0, ld, 0, out);
    PBTC_LAUNCH_CHECK();
    return PBTC_OK;
  }
  // out[c] = ||v|| over system c
  int norm(const double* v, double* out) {
    hipLaunchKernelGGL(k_dots_seg, dim3(nchunks, 1), dim3(kRedThreads), 0, st, v, 1, n, v, chunks,
                       red, ld);
    hipLaunchKernelGGL(k_sum_seg, dim3(nc, 1), dim3(64), 0, st, red, ld, chunk0, 1, 1, out);
    PBTC_LAUNCH_CHECK();
    return PBTC_OK;
  }
  // w -= V h (second pass) and out[c] = ||w|| over system c
  int sub_combo_norm(int nv, const double* h, double* out) {
    hipLaunchKernelGGL(k_sub_combo_norm_seg, dim3(nchunks * kChunkBlocks), dim3(kRedThreads), 0, st,
                       V, nv, n, h, ld, chunks, w, nrm);
    hipLaunchKernelGGL(k_norm_seg, dim3(nc), dim3(64), 0, st, nrm, chunk0, kChunkBlocks, out);
    PBTC_LAUNCH_CHECK();
    return PBTC_OK;
  }
  // one Arnoldi orthogonalisation of w against V_0..V_{nv-1} (CGS2) with
  // coefficients in h1 and h2 (per system), then vn = w / ||w|| and
  // hn = ||w||, and the Givens step of column j = nv - 1 (residual estimates
  // and active flags to hout)
  int arnoldi(int nv, double* h1, double* h2, double* hn, const double* active, double* vn,
              double* vn2, double* hout) {
    const int T = 256;
    const int j = nv - 1;
    if (!fuse) {
      int rc = dots(V, nv, w, h1);
      if (rc) return rc;
      hipLaunchKernelGGL(k_sub_combo_seg, dim3(nblocks(n, T)), dim3(T), 0, st, V, nv, n, h1, ld,
                         comp, w);
      rc = dots(V, nv, w, h2);
      if (rc) return rc;
      rc = sub_combo_norm(nv, h2, hn);
      if (rc) return rc;
      hipLaunchKernelGGL(k_scale_seg, dim3(nblocks(n, T)), dim3(T), 0, st, w, n, hn, comp, active,
                         vn, vn2);
      hipLaunchKernelGGL(k_givens_seg, dim3(nc), dim3(64), 8 * (3 * ld + 1), st, nc, j, ld, h1, h2,
                         H, giv, gstride, sc, hout);
      PBTC_LAUNCH_CHECK();
      return PBTC_OK;
    }
    const dim3 grid(nchunks * kChunkBlocks);
    hipLaunchKernelGGL(k_dots_seg, dim3(nchunks, nv), dim3(kRedThreads), 0, st, V, nv, n, w, chunks,
                       red, ld);
    hipLaunchKernelGGL(k_gs_pass_seg<false>, grid, dim3(kRedThreads), 8 * nv, st, V, nv, n, red, ld,
                       chunks, chunk0, h1, ld, w, nrm);
    hipLaunchKernelGGL(k_dots_seg, dim3(nchunks, nv), dim3(kRedThreads), 0, st, V, nv, n, w, chunks,
                       red, ld);
    hipLaunchKernelGGL(k_gs_pass_seg<true>, grid, dim3(kRedThreads), 8 * nv, st, V, nv, n, red, ld,
                       chunks, chunk0, h2, ld, w, nrm);
    hipLaunchKernelGGL(k_norm_givens_seg, dim3(nc + nchunks * kChunkBlocks), dim3(kRedThreads),
                       8 * (3 * ld + 1), st, nc, j, ld, w, nrm, chunks, chunk0, h1, h2, H, giv,
                       gstride, sc, hout, vn, vn2);
    PBTC_LAUNCH_CHECK();
    return PBTC_OK;
  }
  bool host(const double* d, double* h, int cnt) {
    if (hipMemcpyAsync(h, d, 8 * cnt, hipMemcpyDeviceToHost, st) != hipSuccess) return false;
    return hipStreamSynchronize(st) == hipSuccess;
  }
  // pinned host buffer of 2 slots x cnt values and two events for the
  // residual readback (kept by the plan)
  bool pinned(int cnt) {
    if (pl.res_pin_n < 2 * cnt) {
      if (pl.res_pin) (void)hipHostFree(pl.res_pin);
      pl.res_pin = nullptr;
      pl.res_pin_n = 0;
      if (hipHostMalloc((void**)&pl.res_pin, 8 * 2 * (size_t)cnt) != hipSuccess) return false;
      pl.res_pin_n = 2 * cnt;
    }
    for (int i = 0; i < 2; ++i)
      if (!pl.res_ev[i] && hipEventCreateWithFlags(&pl.res_ev[i], hipEventDisableTiming) != hipSuccess)
        return false;
    return true;
  }
  bool to_dev(double* d, const double* h, int cnt) {
    if (hipMemcpyAsync(d, h, 8 * cnt, hipMemcpyHostToDevice, st) != hipSuccess) return false;
    return hipStreamSynchronize(st) == hipSuccess;
  }
};

int apply_precond(pbtc_plan_t& pl, hipStream_t st, const double* x, double* y, bool transpose,
                  bool accumulate) {
  hipLaunchKernelGGL(k_prec_apply, dim3(nblocks(pl.np_tot, 256)), dim3(256), 0, st, pl.np_tot,
                     wsp<int>(pl, pl.o_pidx), wsp<double>(pl, pl.o_pinv), x, y, transpose ? 1 : 0,
                     accumulate ? 1 : 0);
  PBTC_LAUNCH_CHECK();
  return PBTC_OK;
}

// Restarted GMRES for A z = rhs on every system at once.  System c stops
// when its implicit residual <= tol[c] * ref[c]; its Krylov vectors are zero
// from then on, so further operator applications leave it untouched.
// prec: 0 none, 1 right preconditioning by M^-1, 2 by M^-T (transposed
// system).
// gin, gout (or null): the input and output buffers of the operator's launch
// graph.  The Arnoldi step then writes each new basis vector (or its
// preconditioned image) into gin as well and orthogonalises in gout, so that
// the graph reads and writes them in place (no copies around a replay).
template <typename Op>
static int gmres(pbtc_plan_t& pl, hipStream_t st, Op op, int prec, const double* rhs, double* z,
                 bool zero_start,
                 const std::vector<double>& tol, const std::vector<double>& ref, int max_iter,
                 int* iters, std::vector<double>* hist, std::vector<int>* conv,
                 std::vector<int>* conv_iter, int* discarded, double* gin = nullptr,
                 double* gout = nullptr) {
  Krylov K(pl, st);
  if (gout) K.w = gout;
  double* vin2 = (gin && !prec) ? gin : nullptr;  // second copy of each new basis vector
  const int T = 256;
  const int64_t n = K.n;
  const int m = K.m, nc = K.nc, ld = K.ld;
  double* r = wsp<double>(pl, pl.o_tmp);
  double* pz = wsp<double>(pl, pl.o_ptmp);
  conv->assign(nc, 0);
  if (conv_iter) conv_iter->assign(nc, 0);
  std::vector<double> hbeta(nc), hact(nc), htol(nc), href(nc);
  for (int c = 0; c < nc; ++c) {
    htol[c] = tol[c];
    href[c] = ref[c];
  }
  if (!K.to_dev(K.scal(SC_TOL), htol.data(), nc) || !K.to_dev(K.scal(SC_REF), href.data(), nc)) {
    pl.err = "GMRES: copy failed";
    return PBTC_EDEVICE;
  }
  bool first = true;
  while (*iters < max_iter) {
    if (zero_start && first) {
      hipLaunchKernelGGL(k_fill, dim3(nblocks(n, T)), dim3(T), 0, st, z, n, 0.0);
      PBTC_HIP(hipMemcpyAsync(r, rhs, 8 * n, hipMemcpyDeviceToDevice, st));
    } else {
      int rc = op(z, r);
      if (rc) return rc;
      hipLaunchKernelGGL(k_sub, dim3(nblocks(n, T)), dim3(T), 0, st, rhs, r, n, r);
    }
    first = false;
    int rc = K.norm(r, K.scal(SC_BETA));
    if (rc) return rc;
    if (!K.host(K.scal(SC_BETA), hbeta.data(), nc)) {
      pl.err = "GMRES: copy failed";
      return PBTC_EDEVICE;
    }
    int nact = 0;
    for (int c = 0; c < nc; ++c) {
      if (!std::isfinite(hbeta[c])) {
        pl.err = "GMRES: residual is not finite";
        return PBTC_EDEVICE;
      }
      const bool done = (*conv)[c] || hbeta[c] <= tol[c] * ref[c];
      if (done && !(*conv)[c]) {
        (*conv)[c] = 1;
        if (conv_iter) (*conv_iter)[c] = *iters;
      }
      hact[c] = done ? 0.0 : 1.0;
      nact += !done;
    }
    if (nact == 0) break;
    if (!K.to_dev(K.scal(SC_ACTIVE), hact.data(), nc)) {
      pl.err = "GMRES: copy failed";
      return PBTC_EDEVICE;
    }
    hipLaunchKernelGGL(k_scale_seg, dim3(nblocks(n, T)), dim3(T), 0, st, r, n, K.scal(SC_BETA),
                       K.comp, K.scal(SC_ACTIVE), K.V, vin2);
    hipLaunchKernelGGL(k_init_seg, dim3(1), dim3(64), 0, st, nc, K.giv, K.gstride, ld,
                       K.scal(SC_BETA), K.scal(SC_KFIN));
    // The residual estimates of iteration j are read on the host while
    // iteration j + 1 already runs: each iteration's [residual, active]
    // pair is copied to pinned memory behind its Givens step.  If iteration j
    // turns out to be the last, the queued iteration j + 1 changes nothing
    // that is used (every system is inactive: no Givens update, kfin already
    // fixed, and the basis vector it writes lies past every system's kfin).
    if (!K.pinned(2 * nc)) {
      pl.err = "GMRES: pinned host buffer or event unavailable";
      return PBTC_EDEVICE;
    }
    int j = 0, done = 0, still = nact;
    auto process = [&](int slot) -> int {
      const double* hs = pl.res_pin + (size_t)slot * 2 * nc;
      ++*iters;
      double worst = 0.0;
      int left = 0;
      for (int c = 0; c < nc; ++c) {
        const double res = hs[c];
        if (!std::isfinite(res)) {
          pl.err = "GMRES: residual estimate is not finite";
          return -1;
        }
        if (hact[c] > 0.0) worst = std::max(worst, res);
        if (hact[c] > 0.0 && hs[nc + c] == 0.0) {
          (*conv)[c] = 1;
          if (conv_iter) (*conv_iter)[c] = *iters;
        }
        hact[c] = hs[nc + c];
        left += hact[c] > 0.0;
      }
      if (hist) hist->push_back(worst);
      return left;
    };
    while (true) {
      const bool launch = j < m && *iters + (j - done) < max_iter && still > 0;
      if (launch) {
        double* vj = K.V + (size_t)j * n;
        double* vn = K.V + (size_t)(j + 1) * n;
        if (prec) {
          double* pin = gin ? gin : pz;
          rc = apply_precond(pl, st, vj, pin, prec == 2, false);
          if (!rc) rc = op(pin, K.w);
        } else {
          rc = op(gin ? gin : vj, K.w);
        }
        if (rc) return rc;
        // CGS2 and the Givens step (Hessenberg column = first-pass +
        // second-pass coefficients); the residual estimates and active flags
        // of every system go straight to pinned host memory (no copy)
        rc = K.arnoldi(j + 1, K.hbuf, K.h2buf, K.scal(SC_HN), K.scal(SC_ACTIVE), vn, vin2,
                       pl.res_pin + (size_t)(j & 1) * 2 * nc);
        if (rc) return rc;
        PBTC_HIP(hipEventRecord(pl.res_ev[j & 1], st));
        ++j;
      }
      // process the older iteration once two are queued, or drain
      if (done < j && (j - done > 1 || !launch)) {
        PBTC_HIP(hipEventSynchronize(pl.res_ev[done & 1]));
        still = process(done & 1);
        ++done;
        if (still < 0) return PBTC_EDEVICE;
        if (still == 0) break;
        continue;
      }
      if (!launch) break;
    }
    *discarded += j - done;  // a queued iteration after the last one
    j = done;                // columns formed for the systems still active
    hipLaunchKernelGGL(k_finish_seg, dim3(1), dim3(64), 0, st, nc, std::min(j, m), ld, K.H, K.giv,
                       K.gstride, K.sc);
    if (prec) {
      // z += M^-1 (V y): the combination is formed in w (free at this point)
      hipLaunchKernelGGL(k_fill, dim3(nblocks(n, T)), dim3(T), 0, st, K.w, n, 0.0);
      hipLaunchKernelGGL(k_add_combo_seg, dim3(nblocks(n, T)), dim3(T), 0, st, K.V, n, K.giv,
                         K.gstride, ld, K.scal(SC_KFIN), K.comp, K.w);
      PBTC_LAUNCH_CHECK();
      rc = apply_precond(pl, st, K.w, z, prec == 2, true);
      if (rc) return rc;
    } else {
      hipLaunchKernelGGL(k_add_combo_seg, dim3(nblocks(n, T)), dim3(T), 0, st, K.V, n, K.giv,
                         K.gstride, ld, K.scal(SC_KFIN), K.comp, z);
    }
    PBTC_LAUNCH_CHECK();
    bool all = true;
    for (int c = 0; c < nc; ++c) all &= (*conv)[c] != 0;
    if (all) break;
  }
  return PBTC_OK;
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Solves A x = b (or A^T x = b) for every independent system to the plan's
// tolerance in the plan's precision: FP64 GMRES, FP32 GMRES, or FP32 GMRES
// inside FP64 iterative refinement.  rel = the largest explicit
// ||b_c - (A x)_c|| / ||b_c|| over systems, with the FP64 operator.
int solve_with_ops(pbtc_plan_t& pl, hipStream_t st, bool transpose, const double* b, double* x,
                   int* iters_out, int* n32_out, int* n64_out, int* nref_out, double* rel_out,
                   bool* conv_out, std::vector<double>* hist) {
  const int T = 256;
  const int64_t n = pl.nunk;
  const int nc = pl.ncomp;
  double* r = wsp<double>(pl, pl.o_r);
  double* d = wsp<double>(pl, pl.o_z2);  // correction of a refinement step
  Krylov K(pl, st);
  int iters = 0, n32 = 0, n64 = 0, nref = 0;
  std::vector<double> bnorm(nc), rnorm(nc), rel(nc, 0.0);
  int rc = K.norm(b, K.scal(SC_BNORM));
  if (rc) return rc;
  if (!K.host(K.scal(SC_BNORM), bnorm.data(), nc)) {
    pl.err = "copy failed";
    return PBTC_EDEVICE;
  }
  auto op64 = [&](const double* in, double* out) {
    ++n64;
    return transpose ? apply_transpose(pl, st, in, out, PBTC_FP64, 0)
                     : apply_operator(pl, st, in, out, PBTC_FP64, 0);
  };
  auto op32 = [&](const double* in, double* out) {
    ++n32;
    return transpose ? apply_transpose(pl, st, in, out, PBTC_FP32, 0)
                     : apply_operator(pl, st, in, out, PBTC_FP32, 0);
  };
  const int prec = pl.prm.precond == PBTC_PREC_BLOCK_DIAG ? (transpose ? 2 : 1) : 0;
  // A x through its launch graph: GMRES keeps its operator input and output
  // in the graph's own buffers
  double* gin = (!transpose && pl.prm.op_graph) ? wsp<double>(pl, pl.o_gxin) : nullptr;
  double* gout = (!transpose && pl.prm.op_graph) ? wsp<double>(pl, pl.o_gyout) : nullptr;
  // systems with a zero right-hand side are solved by x = 0
  std::vector<double> ref(nc), tol(nc, pl.prm.tol);
  for (int c = 0; c < nc; ++c) ref[c] = bnorm[c] > 0.0 ? bnorm[c] : 1.0;
  std::vector<int> conv(nc, 0), cit;
  auto explicit_residual = [&]() -> int {
    int e = op64(x, r);
    if (e) return e;
    hipLaunchKernelGGL(k_sub, dim3(nblocks(n, T)), dim3(T), 0, st, b, r, n, r);
    e = K.norm(r, K.scal(SC_NORM));
    if (e) return e;
    if (!K.host(K.scal(SC_NORM), rnorm.data(), nc)) {
      pl.err = "copy failed";
      return PBTC_EDEVICE;
    }
    for (int c = 0; c < nc; ++c) rel[c] = bnorm[c] > 0.0 ? rnorm[c] / bnorm[c] : 0.0;
    return PBTC_OK;
  };
  bool all = false;
  if (pl.prm.precision == PBTC_FP32_REFINED) {
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n, T)), dim3(T), 0, st, x, n, 0.0);
    PBTC_HIP(hipMemcpyAsync(r, b, 8 * n, hipMemcpyDeviceToDevice, st));
    rnorm = bnorm;
    for (int c = 0; c < nc; ++c) rel[c] = bnorm[c] > 0.0 ? 1.0 : 0.0;
    for (nref = 0; nref < pl.prm.max_refine && iters < pl.prm.max_iter; ++nref) {
      // inner solve of A d = r: per system a relative tolerance that lands the
      // outer residual below tol but not below what the FP32 operator resolves;
      // systems already converged take no inner step
      std::vector<double> tin(nc), rref(nc);
      for (int c = 0; c < nc; ++c) {
        rref[c] = rnorm[c] > 0.0 ? rnorm[c] : 1.0;
        if (rel[c] <= pl.prm.tol) {
          tin[c] = 2.0;
        } else {
          const double want = 0.5 * pl.prm.tol * bnorm[c] / rnorm[c];
          tin[c] = std::min(0.5, std::max(want, pl.prm.inner_tol));
        }
      }
      std::vector<int> cin;
      int disc = 0;
      rc = gmres(pl, st, op32, prec, r, d, true, tin, rref, pl.prm.max_iter, &iters, hist, &cin,
                 nullptr, &disc, gin, gout);
      n32 -= disc;  // operator evaluations whose results were not used
      if (rc) return rc;
      hipLaunchKernelGGL(k_axpy, dim3(nblocks(n, T)), dim3(T), 0, st, 1.0, d, n, x);
      rc = explicit_residual();
      if (rc) return rc;
      all = true;
      for (int c = 0; c < nc; ++c) all &= rel[c] <= pl.prm.tol;
      if (all) {
        ++nref;
        break;
      }
    }
    for (int c = 0; c < nc; ++c) conv[c] = rel[c] <= pl.prm.tol;
  } else {
    const int opp = pl.prm.precision == PBTC_FP64 ? PBTC_FP64 : PBTC_FP32;
    int disc = 0;
    if (opp == PBTC_FP64)
      rc = gmres(pl, st, op64, prec, b, x, true, tol, ref, pl.prm.max_iter, &iters, hist, &conv,
                 &cit, &disc, gin, gout);
    else
      rc = gmres(pl, st, op32, prec, b, x, true, tol, ref, pl.prm.max_iter, &iters, hist, &conv,
                 &cit, &disc, gin, gout);
    (opp == PBTC_FP64 ? n64 : n32) -= disc;  // evaluations whose results were not used
    if (rc) return rc;
    rc = explicit_residual();
    if (rc) return rc;
    // FP64: implicit or explicit residual meets tol; FP32 without refinement:
    // the implicit residual of the FP32 operator meets tol (rel is reported)
    for (int c = 0; c < nc; ++c) conv[c] = conv[c] || (opp == PBTC_FP64 && rel[c] <= pl.prm.tol);
  }
  all = true;
  double worst = 0.0;
  for (int c = 0; c < nc; ++c) {
    all &= conv[c] != 0;
    worst = std::max(worst, rel[c]);
  }
  if (!transpose) {  // per-system results of the forward solve
    pl.comp_rel = rel;
    pl.comp_conv = conv;
  }
  *iters_out = iters;
  *n32_out = n32;
  *n64_out = n64;
  *nref_out = nref;
  *rel_out = worst;
  *conv_out = all;
  return PBTC_OK;
}

// Solve on a set-up workspace; fills res (timings from t_setup on).
int device_solve(pbtc_plan_t& pl, hipStream_t st, pbtc_result* res) {
  const int64_t n = pl.nunk;
  double* b = wsp<double>(pl, pl.o_b);
  double* x = wsp<double>(pl, pl.o_x);
  Krylov K(pl, st);
  pl.history.clear();
  pl.n_graph_launch = 0;
  prof_collect(pl);
  for (int i = 0; i < kProfKinds; ++i) pl.prof_t[i] = pl.prof_flop[i] = 0.0, pl.prof_n[i] = 0;
  int iters = 0, n32 = 0, n64 = 0, nref = 0;
  bool conv = false;
  double rel = 0.0;
  const double t0 = now_s();
  int rc = solve_with_ops(pl, st, false, b, x, &iters, &n32, &n64, &nref, &rel, &conv, &pl.history);
  if (rc) return rc;
  PBTC_HIP(hipStreamSynchronize(st));
  const double t1 = now_s();
  // reaction potential at the charges (FP64 treecode) and the energy of
  // every system (Eq. solv)
  double* phi = wsp<double>(pl, pl.o_phi_reac);
  rc = apply_operator(pl, st, x, phi, PBTC_FP64, 1);
  if (rc) return rc;
  double* e = wsp<double>(pl, pl.o_energy);
  hipLaunchKernelGGL(k_energy_seg, dim3(pl.ncomp), dim3(kRedThreads), 0, st, wsp<double>(pl, pl.o_q),
                     phi, wsp<int>(pl, pl.o_comp_q), pl.nq, 0.5 * 4.0 * kPi * kCoulomb, e);
  PBTC_LAUNCH_CHECK();
  pl.comp_energy.assign(pl.ncomp, 0.0);
  if (!K.host(e, pl.comp_energy.data(), pl.ncomp)) {
    pl.err = "copy failed";
    return PBTC_EDEVICE;
  }
  pl.energy = 0.0;
  for (double v : pl.comp_energy) pl.energy += v;
  const double t2 = now_s();
  pl.x_host.resize(n);
  pl.phi_reac_host.resize(pl.nq);
  PBTC_HIP(hipMemcpyAsync(pl.x_host.data(), x, 8 * n, hipMemcpyDeviceToHost, st));
  PBTC_HIP(hipMemcpyAsync(pl.phi_reac_host.data(), phi, 8 * pl.nq, hipMemcpyDeviceToHost, st));
  PBTC_HIP(hipStreamSynchronize(st));
  pl.solved = true;
  pl.dev_solved = true;
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
    prof_collect(pl);
    res->t_p2p_s = pl.prof_t[0];
    res->t_m2p_s = pl.prof_t[1] + pl.prof_t[2] + pl.prof_t[kProfM2PPair];
    res->n_p2p_launch = pl.prof_n[0];
    res->n_m2p_launch = pl.prof_n[1] + pl.prof_n[2] + pl.prof_n[kProfM2PPair];
    res->p2p_flop = pl.prof_flop[0];
    res->m2p_flop = pl.prof_flop[1] + pl.prof_flop[2] + pl.prof_flop[kProfM2PPair];
    res->t_m2p_yuk_s = pl.prof_t[2];
    res->n_m2p_yuk_launch = pl.prof_n[2];
    res->m2p_yuk_flop = pl.prof_flop[2];
    res->op_kernels = pl.op_kernels[1][0];
    res->op_graph_launches = (int)pl.n_graph_launch;
    static_assert(kProfKinds == PBTC_KERNEL_KINDS, "timed kernel kinds of pbtc_result");
    for (int k = 0; k < kProfKinds; ++k) {
      res->t_kernel_s[k] = pl.prof_t[k];
      res->n_kernel_launch[k] = pl.prof_n[k];
      res->kernel_flop[k] = pl.prof_flop[k];
    }
  }
  if (!conv) {
    pl.err = "GMRES did not reach the tolerance within max_iter";
    return PBTC_ENOCONV;
  }
  return PBTC_OK;
}

// Coulomb energy of every system: 1/2 k_e sum_i q_i phi_c[i].
int device_coulomb(pbtc_plan_t& pl, hipStream_t st, double* total, double* per_system) {
  // table: nreg + 1 first-charge offsets (int64), then nreg permittivities
  std::vector<double>& tab = pl.qtab_host;
  tab.assign(2 * pl.nreg + 1, 0.0);
  for (int r = 0; r <= pl.nreg; ++r) {
    const long long o = pl.q_off_region[r];
    std::memcpy(&tab[r], &o, 8);
  }
  for (int r = 0; r < pl.nreg; ++r) tab[pl.nreg + 1 + r] = pl.prob.regions[r].eps;
  double* dtab = wsp<double>(pl, pl.o_qtab);
  PBTC_HIP(hipMemcpyAsync(dtab, tab.data(), 8 * tab.size(), hipMemcpyHostToDevice, st));
  double* phi = wsp<double>(pl, pl.o_z2);
  std::vector<double> e(pl.ncomp, 0.0);
  if (pl.nq > 0) {
    hipLaunchKernelGGL(k_coulomb_pot, dim3(nblocks(pl.nq, 256)), dim3(256), 0, st, pl.nq,
                       wsp<double>(pl, pl.o_qxyz), wsp<double>(pl, pl.o_q), wsp<int>(pl, pl.o_qreg),
                       reinterpret_cast<const long long*>(dtab), dtab + pl.nreg + 1, phi);
    double* out = wsp<double>(pl, pl.o_coul);
    hipLaunchKernelGGL(k_energy_seg, dim3(pl.ncomp), dim3(kRedThreads), 0, st,
                       wsp<double>(pl, pl.o_q), phi, wsp<int>(pl, pl.o_comp_q), pl.nq, 0.5 * kCoulomb,
                       out);
    PBTC_LAUNCH_CHECK();
    PBTC_HIP(hipMemcpyAsync(e.data(), out, 8 * pl.ncomp, hipMemcpyDeviceToHost, st));
  }
  PBTC_HIP(hipStreamSynchronize(st));
  double t = 0.0;
  for (int c = 0; c < pl.ncomp; ++c) {
    if (!std::isfinite(e[c])) {
      pl.err = "Coulomb energy is not finite (coincident charges in one region)";
      return PBTC_EINVAL;
    }
    t += e[c];
    if (per_system) per_system[c] = e[c];
  }
  *total = t;
  return PBTC_OK;
}

double wall_seconds() { return now_s(); }

// ---------------------------------------------------------------------------
// Allocation-free variant of the Coulomb energy for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops):
// its scratch -- the Coulomb potential at every charge, the per-system sums and
// the region table -- lives in this file-scope device array instead of the
// plan's workspace.  Each GPU holds its own copy until the process ends; its
// device address is taken once per device with hipGetSymbolAddress (the
// array's name in host code is not a device address).  Calls that overlap on
// one GPU share the array and race; every value a call reads is written by
// that call first, so nothing needs clearing.
constexpr int64_t kScratchCharges = int64_t(1) << 20;  // phi: one double per charge
constexpr int64_t kScratchTable = int64_t(1) << 16;    // region table + per-system sums
constexpr size_t kScratchBytes = 8 * (size_t)(kScratchCharges + kScratchTable);
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device (looked up once per device).
static int scratch_address(pbtc_plan_t& pl, char** out) {
  int dev = 0;
  PBTC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    pl.err = "device index beyond the scratch table";
    return PBTC_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    PBTC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return PBTC_OK;
}

int device_coulomb_noalloc(pbtc_plan_t& pl, hipStream_t st, double* total, double* per_system) {
  const int64_t ntab = 2 * (int64_t)pl.nreg + 1, nout = pl.ncomp;
  if (pl.nq > kScratchCharges || ntab + nout > kScratchTable) {
    pl.err = "allocation-free Coulomb energy: at most " + std::to_string(kScratchCharges) +
             " charges and " + std::to_string(kScratchTable) +
             " values of region table plus systems (2 regions + 1 + systems)";
    return PBTC_EINVAL;
  }
  char* base = nullptr;
  int rc = scratch_address(pl, &base);
  if (rc) return rc;
  double* phi = reinterpret_cast<double*>(base);
  double* dtab = phi + kScratchCharges;
  double* out = dtab + ntab;
  // host tables sized when the plan was made: no allocation here
  double* tab = pl.coul_host.data();
  for (int r = 0; r <= pl.nreg; ++r) {
    const long long o = pl.q_off_region[r];
    std::memcpy(&tab[r], &o, 8);
  }
  for (int r = 0; r < pl.nreg; ++r) tab[pl.nreg + 1 + r] = pl.prob.regions[r].eps;
  double* e = tab + ntab;
  for (int64_t c = 0; c < nout; ++c) e[c] = 0.0;
  PBTC_HIP(hipMemcpyAsync(dtab, tab, 8 * ntab, hipMemcpyHostToDevice, st));
  if (pl.nq > 0) {
    hipLaunchKernelGGL(k_coulomb_pot, dim3(nblocks(pl.nq, 256)), dim3(256), 0, st, pl.nq,
                       wsp<double>(pl, pl.o_qxyz), wsp<double>(pl, pl.o_q), wsp<int>(pl, pl.o_qreg),
                       reinterpret_cast<const long long*>(dtab), dtab + pl.nreg + 1, phi);
    hipLaunchKernelGGL(k_energy_seg, dim3(pl.ncomp), dim3(kRedThreads), 0, st,
                       wsp<double>(pl, pl.o_q), phi, wsp<int>(pl, pl.o_comp_q), pl.nq, 0.5 * kCoulomb,
                       out);
    PBTC_LAUNCH_CHECK();
    PBTC_HIP(hipMemcpyAsync(e, out, 8 * nout, hipMemcpyDeviceToHost, st));
  }
  PBTC_HIP(hipStreamSynchronize(st));
  double t = 0.0;
  for (int64_t c = 0; c < nout; ++c) {
    if (!std::isfinite(e[c])) {
      pl.err = "Coulomb energy is not finite (coincident charges in one region)";
      return PBTC_EINVAL;
    }
    t += e[c];
    if (per_system) per_system[c] = e[c];
  }
  *total = t;
  return PBTC_OK;
}

}  // namespace pbtc
