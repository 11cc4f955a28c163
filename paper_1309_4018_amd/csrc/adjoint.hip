// Transposed operator and gradients of the solvation energy.
//
// With A x = B q (Eq. matrix, multi-surface form) and dG = 1/2 C q^T S x
// (Eqs. reac_integral and solv, C = 4 pi k_e), the adjoint lambda solves
// A^T lambda = S^T q, and
//   dG/dq_k   = 1/2 C (S x + B^T lambda)_k
//   dG/dp     = 1/2 C [q^T S'_p x - lambda^T A'_p x + lambda^T B'_p q]
// for p = eps_r, kappa_r.
//
// A^T applied to lambda: the phi-columns of A carry 1/2 I and sigma K, the
// psi-columns -sigma c V, so A^T lambda has the phi part
// 1/2 (lambda_I + lambda_O) + sum sigma K^T lambda and the psi part
// sum -sigma c V^T lambda.  For a panel j and weights mu on the targets x_i,
//   (V^T mu)_j = sum_g W_jg sum_i mu_i G(x_i, y_jg)       + near-field terms
//   (K^T mu)_j = sum_g W_jg n_j . sum_i mu_i grad_y G(x_i, y_jg) + near terms
// i.e. a potential and a gradient at the Gauss points y (the adjoint double
// layer takes the normal at the target).  These sums are evaluated by a
// treecode with the roles swapped: sources at the collocation points
// (octree per target set, moments of mu), targets at the Gauss points
// (groups of kAGroup consecutive Morton-sorted points), P2P near, and M2P far with
// Taylor coefficients to order P+1 for the gradient:
//   grad_y a_k(y; x_c) = -(k_d + 1) a_{k+e_d}(y; x_c).
// The near-field corrections are applied through the transpose (CSC) of the
// forward table.  With the direct operator (no far field) this is the exact
// transpose of the forward operator; with the treecode it agrees with it to
// the truncation error of the expansion.
//
// kappa enters through the Yukawa kernels and the near-field tables; dG/dkappa
// uses a central difference of the FP64 operator in kappa (step 1e-4 kappa),
// applied to x against lambda.  eps enters only through c_rs and 1/eps_r and
// is differentiated exactly.
#include <algorithm>
#include <cmath>

#include "device_util.h"
#include "kernel_common.h"
#include "traverse.h"
#include "taylor.h"

namespace pbtc {

int build_octree(pbtc_plan_t& pl, hipStream_t st, Cell* cells, int64_t cap,
                 const std::vector<Cell>& roots, const uint64_t* key, const double* px,
                 const double* py, const double* pz, int ncrit, long long* cnt,
                 long long* scan_scratch, int64_t* n_cells, std::vector<int>* level_begin,
                 int64_t* need);
int apply_operator(pbtc_plan_t& pl, hipStream_t st, const double* x, double* y, int precision,
                   int phase);
int recompute_near_values(pbtc_plan_t& pl, hipStream_t st);
int recompute_rhs(pbtc_plan_t& pl, hipStream_t st);
int upload_coulomb_rows(pbtc_plan_t& pl, hipStream_t st);
int upload_descriptors(pbtc_plan_t& pl, hipStream_t st);
template <typename Op>
int krylov_solve(pbtc_plan_t& pl, hipStream_t st, Op op32, Op op64, const double* b, double* x,
                 int precision, double tol, int* iters, int* n32, int* n64, int* nref,
                 double* rel, bool* conv, std::vector<double>* hist);
int solve_with_ops(pbtc_plan_t& pl, hipStream_t st, bool transpose, const double* b, double* x,
                   int* iters, int* n32, int* n64, int* nref, double* rel, bool* conv,
                   std::vector<double>* hist);

namespace {

constexpr int kT = 256;
constexpr int kWaves = 4;

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ------------------------------------------------------------- setup kernels
// Gauss points as adjoint targets: position, panel normal, weight.
template <typename real>
__global__ void k_gpos(int64_t ngp, const double* __restrict__ gx, const double* __restrict__ gy,
                       const double* __restrict__ gz, const double* __restrict__ gw,
                       const int* __restrict__ gpid, const int* __restrict__ gidx,
                       const double* __restrict__ nx, const double* __restrict__ ny,
                       const double* __restrict__ nz, Src<real>* __restrict__ out,
                       int* __restrict__ pos) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ngp) return;
  const int p = gpid[j];
  Src<real> s;
  s.x = (real)gx[j];
  s.y = (real)gy[j];
  s.z = (real)gz[j];
  s.q = (real)gw[j];
  s.px = (real)nx[p];
  s.py = (real)ny[p];
  s.pz = (real)nz[p];
  s.pad = 0;
  out[j] = s;
  if (pos) pos[gidx[j]] = (int)j;
}

// bounding sphere of Gauss-point group G (kAGroup consecutive sorted points of one surface)
__global__ void k_gp_groups(int64_t ngrp, int nsurf, const long long* __restrict__ tab,
                            const double* __restrict__ gx, const double* __restrict__ gy,
                            const double* __restrict__ gz, double* __restrict__ grp) {
  const int64_t G = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (G >= ngrp) return;
  const long long* grp_off = tab;           // nsurf + 1
  const long long* gp_off = tab + nsurf + 1;  // nsurf + 1
  int s = 0;
  while (s + 1 < nsurf && G >= grp_off[s + 1]) ++s;
  const long long o = gp_off[s] + (G - grp_off[s]) * kAGroup;
  const int n = (int)min((long long)kAGroup, gp_off[s + 1] - o);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int i = 0; i < n; ++i) {
    lo[0] = fmin(lo[0], gx[o + i]);
    hi[0] = fmax(hi[0], gx[o + i]);
    lo[1] = fmin(lo[1], gy[o + i]);
    hi[1] = fmax(hi[1], gy[o + i]);
    lo[2] = fmin(lo[2], gz[o + i]);
    hi[2] = fmax(hi[2], gz[o + i]);
  }
  const double c[3] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])};
  double r2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double dx = gx[o + i] - c[0], dy = gy[o + i] - c[1], dz = gz[o + i] - c[2];
    r2 = fmax(r2, dx * dx + dy * dy + dz * dz);
  }
  grp[4 * G] = c[0];
  grp[4 * G + 1] = c[1];
  grp[4 * G + 2] = c[2];
  grp[4 * G + 3] = sqrt(r2) * (1.0 + 1e-12);
}


// one thread per adjoint item (block, Gauss-point group); mode 0 count, 1 fill
__global__ __launch_bounds__(64 * kTravWaves) void k_adj_lists(
    int64_t nitems, const int* __restrict__ item_block, const DevBlock* __restrict__ blocks,
    const Cell* __restrict__ cells, const double* __restrict__ grp, double theta, int direct,
    int direct_below, int mode, long long* __restrict__ near_ptr, long long* __restrict__ far_ptr,
    int* __restrict__ near, int* __restrict__ far, long long cap_near, long long cap_far,
    int* __restrict__ overflow) {
  __shared__ int stk[kTravWaves][kTravStack];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t it = (int64_t)blockIdx.x * kTravWaves + w;
  if (it >= nitems) return;
  const DevBlock& b = blocks[item_block[it]];
  const int64_t g = b.gpgrp_off + (it - b.aitem_off);
  long long pn = 0, pf = 0, nn = 0, nf = 0;
  if (mode == 1) {
    pn = near_ptr[it];
    pf = far_ptr[it];
  }
  if (direct) {
    if (mode == 1 && lane == 0 && pn < cap_near) near[pn] = b.troot;
    nn = 1;
  } else {
    wave_lists(cells, b.troot, grp[4 * g], grp[4 * g + 1], grp[4 * g + 2], grp[4 * g + 3], theta,
               b.direct_below, mode, pn, pf, near, far, cap_near, cap_far, stk[w], &nn, &nf,
               overflow);
  }
  if (mode == 0 && lane == 0) {
    near_ptr[it] = nn;
    far_ptr[it] = nf;
  }
}

// Transposed near-field table: column slot = (block, panel of its source
// surface).  mode 0 counts, mode 1 fills (unordered), then columns are sorted.
__global__ void k_csc_count(int64_t nrows, const int* __restrict__ row_block,
                            const DevBlock* __restrict__ blocks, const long long* __restrict__ ptr,
                            const int* __restrict__ col, long long* __restrict__ cnt,
                            long long* __restrict__ csc_ptr, int* __restrict__ ent,
                            int* __restrict__ ent_row, int mode) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nrows) return;
  const DevBlock b = blocks[row_block[row]];
  for (long long e = ptr[row]; e < ptr[row + 1]; ++e) {
    const long long slot = b.csc_off + (col[e] - b.pan_off);
    const long long k = atomicAdd((unsigned long long*)&cnt[slot], 1ull);
    if (mode == 1) {
      ent[csc_ptr[slot] + k] = (int)e;
      ent_row[csc_ptr[slot] + k] = (int)row;
    }
  }
}

__global__ void k_csc_sort(int64_t ncol, const long long* __restrict__ csc_ptr,
                           int* __restrict__ ent, int* __restrict__ ent_row) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const long long a = csc_ptr[c], b = csc_ptr[c + 1];
  for (long long i = a + 1; i < b; ++i) {
    const int e = ent[i], r = ent_row[i];
    long long j = i - 1;
    while (j >= a && ent[j] > e) {
      ent[j + 1] = ent[j];
      ent_row[j + 1] = ent_row[j];
      --j;
    }
    ent[j + 1] = e;
    ent_row[j + 1] = r;
  }
}

__global__ void k_zero_ll(long long* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_zero_i32(int* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_zero_f64(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void k_ones_f64(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 1.0;
}

// --------------------------------------------------------------- per apply
// mu weights of every kernel slot from the row weights lambda
__global__ void k_adj_mu(const DevSlot* __restrict__ slots, const double* __restrict__ lam,
                         double* __restrict__ muS, double* __restrict__ muD) {
  const DevSlot s = slots[blockIdx.y];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  double vs = 0.0, vd = 0.0;
  for (int c = 0; c < s.ncontrib; ++c) {
    const double l = lam[s.lam_off[c] + i];
    vs += s.cS[c] * l;
    vd += s.cD[c] * l;
  }
  muS[s.out + i] = vs;
  muD[s.out + i] = vd;
}

// adjoint source records of one block in sorted target order:
// (x, y, z, muS_0, muD_0, muS_1, muD_1)
template <typename real>
__global__ void k_adj_src(const int* __restrict__ blist, const DevBlock* __restrict__ blocks,
                          const real* __restrict__ tx, const real* __restrict__ ty,
                          const real* __restrict__ tz, const int* __restrict__ tidx,
                          const double* __restrict__ muS, const double* __restrict__ muD,
                          Src<real>* __restrict__ asrc) {
  const DevBlock b = blocks[blist[blockIdx.y]];
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= b.ntgt) return;
  const long long g = b.tgt_off + j;
  const long long i = tidx[g] - b.tgt_off;
  Src<real> s;
  s.x = tx[g];
  s.y = ty[g];
  s.z = tz[g];
  s.q = (real)muS[b.out0 + i];
  s.px = (real)muD[b.out0 + i];
  s.py = b.nk == 2 ? (real)muS[b.out1 + i] : real(0);
  s.pz = b.nk == 2 ? (real)muD[b.out1 + i] : real(0);
  s.pad = 0;
  asrc[b.nf_row + j] = s;
}

// Moments of mu about the centre of every cell of a block's target tree,
// all levels at once: mS[k] = sum muS (x - c)^k and mD[k] = sum muD (x - c)^k
// over the collocation points x of the cell, for one kernel slot.  One block
// per chunk (cell, first source, count <= kMomSpan, slot), sources staged
// through LDS kMomChunk at a time; a second launch sums each (cell, slot)
// pair's chunks in chunk order into mom[(cell * nrec + local slot) * 2 N].
constexpr int kAMomThreads = 256;

template <typename real, int P>
__global__ __launch_bounds__(kAMomThreads) void k_adj_p2m_chunk(
    const int4* __restrict__ chunks, const Cell* __restrict__ cells,
    const int* __restrict__ slot_block, const int* __restrict__ slot_kidx,
    const DevBlock* __restrict__ blocks, const Src<real>* __restrict__ asrc,
    real* __restrict__ part) {
  constexpr int N = ncoef(P);
  constexpr int G = N <= kAMomThreads ? kAMomThreads / N : 1;
  constexpr int KPT = (N + kAMomThreads - 1) / kAMomThreads;
  static_assert(kMomChunk <= kAMomThreads, "one source per thread while staging");
  __shared__ real pw[kMomChunk][3][P + 1];
  __shared__ real sw[kMomChunk][2];
  __shared__ real red[G][2 * N];
  const int4 ch = chunks[blockIdx.x];
  const Cell& cl = cells[ch.x];
  const DevBlock& b = blocks[slot_block[ch.w]];
  const int kid = slot_kidx[ch.w];
  const real cx = (real)cl.cx, cy = (real)cl.cy, cz = (real)cl.cz;
  const int tid = threadIdx.x;
  const int g = N <= kAMomThreads ? tid / N : 0;
  int kk[KPT][3];
  bool on[KPT];
  real ms[KPT], md[KPT];
#pragma unroll
  for (int q = 0; q < KPT; ++q) {
    const int k = N <= kAMomThreads ? tid - g * N : tid + q * kAMomThreads;
    on[q] = N <= kAMomThreads ? tid < G * N : k < N;
    mindex_inv(on[q] ? k : 0, kk[q][0], kk[q][1], kk[q][2]);
    ms[q] = md[q] = 0;
  }
  for (int b0 = 0; b0 < ch.z; b0 += kMomChunk) {
    const int nj = min(kMomChunk, ch.z - b0);
    if (tid < nj) {
      const Src<real> s = asrc[b.nf_row + (ch.y + b0 + tid - b.tgt_off)];
      const real d[3] = {s.x - cx, s.y - cy, s.z - cz};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        real v = 1;
#pragma unroll
        for (int e = 0; e <= P; ++e) {
          pw[tid][a][e] = v;
          v *= d[a];
        }
      }
      sw[tid][0] = kid == 0 ? s.q : s.py;
      sw[tid][1] = kid == 0 ? s.px : s.pz;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      if (!on[q]) continue;
      const int k1 = kk[q][0], k2 = kk[q][1], k3 = kk[q][2];
      for (int t = g; t < nj; t += G) {
        const real m = pw[t][0][k1] * pw[t][1][k2] * pw[t][2][k3];
        ms[q] += sw[t][0] * m;
        md[q] += sw[t][1] * m;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < KPT; ++q) {
    if (!on[q]) continue;
    const int k = N <= kAMomThreads ? tid - g * N : tid + q * kAMomThreads;
    red[g][k] = ms[q];
    red[g][N + k] = md[q];
  }
  __syncthreads();
  for (int k = tid; k < 2 * N; k += kAMomThreads) {
    real v = 0;
#pragma unroll
    for (int gg = 0; gg < G; ++gg) v += red[gg][k];
    part[(size_t)blockIdx.x * 2 * N + k] = v;
  }
}

// mom[pair.x] = sum of the pair's chunks [pair.y, pair.z), in order, in the
// layout the transposed M2P reads: [mS_k (|k| <= P) | G_1,k | G_2,k | G_3,k
// (|k| <= P + 1)] with G_j,k = k_j mD_{k - e_j} (0 where k_j = 0)
template <typename real, int P>
__global__ __launch_bounds__(256) void k_adj_mom_sum(const int4* __restrict__ pairs,
                                                     const real* __restrict__ part,
                                                     real* __restrict__ mom) {
  constexpr int N = ncoef(P), N2 = 2 * N, N1 = ncoef(P + 1), MS = adj_mom_len(P);
  __shared__ real sm[N2];
  const int4 pr = pairs[blockIdx.x];
  for (int k = threadIdx.x; k < N2; k += 256) {
    real v = 0;
    int j = pr.y;
    for (; j + 4 <= pr.z; j += 4) {
      real a[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = part[(size_t)(j + i) * N2 + k];
      v += (a[0] + a[1]) + (a[2] + a[3]);
    }
    for (; j < pr.z; ++j) v += part[(size_t)j * N2 + k];
    sm[k] = v;
  }
  __syncthreads();
  real* out = mom + (size_t)pr.x * MS;
  for (int k = threadIdx.x; k < N; k += 256) out[k] = sm[k];
  for (int i = threadIdx.x; i < 3 * N1; i += 256) {
    const int d = i / N1, k = i - d * N1;
    int c[3];
    mindex_inv(k, c[0], c[1], c[2]);
    real v = 0;
    if (c[d] > 0) {
      c[d] -= 1;
      v = real(c[d] + 1) * sm[N + mindex(c[0], c[1], c[2])];
    }
    out[N + i] = v;
  }
}

// per Gauss point of the item's group: aout[slot] (+)= sum over units / (4 pi)
template <typename real, int NQ>
__global__ __launch_bounds__(256) void k_adj_reduce(
    const int* __restrict__ list, const int* __restrict__ uptr, const int* __restrict__ item_block,
    const DevBlock* __restrict__ blocks, const real* __restrict__ partial, double* __restrict__ aS,
    double* __restrict__ aD, int mode, int first_slot) {
  // four waves take the item's units round-robin; their sums are added in
  // wave order (deterministic)
  __shared__ double lds[3][NQ][64];
  const int l = blockIdx.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  for (int u = uptr[l] + w; u < uptr[l + 1]; u += 4)
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] += (double)partial[((size_t)u * 4 + q) * 64 + lane];
  if (w > 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds[w - 1][q][lane] = v[q];
  __syncthreads();
  if (w > 0) return;
  const int item = list[l];
  const DevBlock& b = blocks[item_block[item]];
  const long long g = item - b.aitem_off;
  const int nt = (int)min((long long)kAGroup, b.gp_n - g * kAGroup);
  if (lane >= nt) return;
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] += lds[k][q][lane];
  const long long i = g * kAGroup + lane;  // sorted position within the surface
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const long long out = (first_slot + (q >> 1) == 0 ? b.aout0 : b.aout1) + i;
    double* dst = (q & 1) ? aD : aS;
    const double val = v[q] * kInv4Pi;
    if (mode == 0)
      dst[out] = val;
    else
      dst[out] += val;
  }
}

// z for every panel: Gauss-point sums of every slot of its surface, the
// transposed near-field terms and (rows of A) 1/2 (lambda_I + lambda_O).
template <typename real>
__global__ void k_adj_gather(int64_t np, int K, const int* __restrict__ pan_surf,
                             const long long* __restrict__ pan_off_tab,
                             const long long* __restrict__ gp_off_tab,
                             const DevGather* __restrict__ gathers, const int* __restrict__ gslots,
                             const int* __restrict__ slot_block, const int* __restrict__ slot_kidx,
                             const DevBlock* __restrict__ blocks, const int* __restrict__ gp_pos,
                             const double* __restrict__ gw, const double* __restrict__ aS,
                             const double* __restrict__ aD, const long long* __restrict__ csc_ptr,
                             const int* __restrict__ csc_ent, const int* __restrict__ csc_row,
                             const real* __restrict__ nfv, const double* __restrict__ muS,
                             const double* __restrict__ muD, const int* __restrict__ pidx,
                             const double* __restrict__ lam, int add_identity,
                             double* __restrict__ z) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int s = pan_surf[p];
  const DevGather gg = gathers[s];
  double zs = 0.0, zd = 0.0;
  for (int q = 0; q < gg.nslots; ++q) {
    const int slot = gslots[gg.slot_off + q];
    const DevBlock b = blocks[slot_block[slot]];
    const int kid = slot_kidx[slot];
    const long long ao = kid == 0 ? b.aout0 : b.aout1;
    for (int g = 0; g < K; ++g) {
      const int j = gp_pos[p * K + g];  // global sorted index
      const long long i = j - gp_off_tab[s];
      zs += gw[j] * aS[ao + i];
      zd += gw[j] * aD[ao + i];
    }
    const long long cs = b.csc_off + (p - pan_off_tab[s]);
    const long long mo = kid == 0 ? b.out0 : b.out1;
    for (long long e = csc_ptr[cs]; e < csc_ptr[cs + 1]; ++e) {
      const long long row = csc_row[e];
      const long long ent = csc_ent[e];
      const long long i = row - b.nf_row;
      zs += (double)nfv[4 * ent + 2 * kid] * muS[mo + i];
      zd += (double)nfv[4 * ent + 2 * kid + 1] * muD[mo + i];
    }
  }
  const int ip = pidx[2 * p], is = pidx[2 * p + 1];
  if (add_identity) zd += 0.5 * (lam[ip] + lam[is]);
  z[ip] = zd;
  z[is] = zs;
}

// (B^T lam)_k = sum over rows of the charge's region lam_i G(x_i, x_k) / eps
// Transposed Coulomb term: out[k] += sum over the row blocks of charge k's
// region of sum_i lam_i G(c_i - x_k) / eps (one wavefront per charge; lanes
// stride over the rows, a fixed butterfly combines them).
__global__ void k_coulomb_t_rows(long long nq, const DevCoulRow* __restrict__ rows,
                                 const int* __restrict__ reg_ptr, const int* __restrict__ reg_rows,
                                 const int* __restrict__ qreg, const double* __restrict__ qxyz,
                                 const double* __restrict__ cx, const double* __restrict__ cy,
                                 const double* __restrict__ cz, const double* __restrict__ lam,
                                 double* __restrict__ out) {
  const long long k = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (k >= nq) return;
  const int lane = threadIdx.x & 63;
  const int r = qreg[k];
  const double x = qxyz[3 * k], y = qxyz[3 * k + 1], zq = qxyz[3 * k + 2];
  double s = 0.0, inv_eps = 0.0;
  for (int e = reg_ptr[r]; e < reg_ptr[r + 1]; ++e) {
    const DevCoulRow rb = rows[reg_rows[e]];
    inv_eps = rb.inv_eps;
    for (long long i = lane; i < rb.n; i += 64) {
      const long long p = rb.pan_first + i;
      const double dx = cx[p] - x, dy = cy[p] - y, dz = cz[p] - zq;
      const double d = sqrt(dx * dx + dy * dy + dz * dz);
      s += lam[rb.row_off + i] * (rb.kappa == 0.0 ? 1.0 : exp(-rb.kappa * d)) / d;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) out[k] += s * inv_eps * kInv4Pi;
}

// dots[t] = sum_i a[offa_t + i] b[offb_t + i]   (one block per pair)
__global__ void k_pair_dots(const long long* __restrict__ tab, const double* __restrict__ A,
                            const double* __restrict__ B, double* __restrict__ dots) {
  __shared__ double lds[kT / 64];
  const long long oa = tab[3 * blockIdx.x], ob = tab[3 * blockIdx.x + 1], n = tab[3 * blockIdx.x + 2];
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += kT) s += A[oa + i] * B[ob + i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kT / 64; ++w) t += lds[w];
    dots[blockIdx.x] = t;
  }
}

}  // namespace

// ---------------------------------------------------------------- host side
namespace {

struct AdjTables {
  std::vector<int> slot_block, slot_kidx, slot_ids[2], blist[2];
};

}  // namespace

static int adj_upload_small(pbtc_plan_t& pl, hipStream_t st);

// One-off set-up of the transposed operator on the plan's workspace.
int adjoint_setup(pbtc_plan_t& pl, hipStream_t st, int* need_retry) {
  *need_retry = 0;
  const int T = 256;
  // Gauss points as targets, and the inverse of their Morton permutation
  hipLaunchKernelGGL(k_gpos<float>, dim3(nblocks(pl.ngp, T)), dim3(T), 0, st, pl.ngp,
                     wsp<double>(pl, pl.o_gx), wsp<double>(pl, pl.o_gy), wsp<double>(pl, pl.o_gz),
                     wsp<double>(pl, pl.o_gw), wsp<int>(pl, pl.o_gpid), wsp<int>(pl, pl.o_gidx),
                     wsp<double>(pl, pl.o_nx), wsp<double>(pl, pl.o_ny), wsp<double>(pl, pl.o_nz),
                     wsp<Src<float>>(pl, pl.o_gpos32), wsp<int>(pl, pl.o_gp_pos));
  hipLaunchKernelGGL(k_gpos<double>, dim3(nblocks(pl.ngp, T)), dim3(T), 0, st, pl.ngp,
                     wsp<double>(pl, pl.o_gx), wsp<double>(pl, pl.o_gy), wsp<double>(pl, pl.o_gz),
                     wsp<double>(pl, pl.o_gw), wsp<int>(pl, pl.o_gpid), wsp<int>(pl, pl.o_gidx),
                     wsp<double>(pl, pl.o_nx), wsp<double>(pl, pl.o_ny), wsp<double>(pl, pl.o_nz),
                     wsp<Src<double>>(pl, pl.o_gpos64), (int*)nullptr);
  PBTC_LAUNCH_CHECK();
  // Gauss-point groups
  {
    std::vector<long long> tab(2 * (pl.nsurf + 1));
    for (int s = 0; s <= pl.nsurf; ++s) {
      tab[s] = pl.gpgrp_off[s];
      tab[pl.nsurf + 1 + s] = pl.gp_off[s];
    }
    long long* dtab = wsp<long long>(pl, pl.o_dots);
    PBTC_HIP(hipMemcpyAsync(dtab, tab.data(), 8 * tab.size(), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_gp_groups, dim3(nblocks(pl.ngpgrp, T)), dim3(T), 0, st, pl.ngpgrp,
                       pl.nsurf, dtab, wsp<double>(pl, pl.o_gx), wsp<double>(pl, pl.o_gy),
                       wsp<double>(pl, pl.o_gz), wsp<double>(pl, pl.o_gpgrp));
    PBTC_LAUNCH_CHECK();
    PBTC_HIP(hipStreamSynchronize(st));
  }
  // octree over every target set (collocation points of a surface or charges)
  long long* scan_scratch = wsp<long long>(pl, pl.o_red);
  {
    std::vector<Cell> roots(pl.tsets.size());
    for (size_t ti = 0; ti < pl.tsets.size(); ++ti) {
      Cell& c = roots[ti];
      c.cx = pl.tcube[4 * ti];
      c.cy = pl.tcube[4 * ti + 1];
      c.cz = pl.tcube[4 * ti + 2];
      c.h = pl.tcube[4 * ti + 3];
      c.rb = 0.0;
      c.begin = (int)pl.tsets[ti].off;
      c.count = (int)pl.tsets[ti].n;
      c.child = c.nchild = 0;
      c.level = 0;
      c.surf = (int)ti;
    }
    int64_t need = 0;
    const int rc = build_octree(pl, st, wsp<Cell>(pl, pl.o_tcells), pl.cap_tcells, roots,
                                wsp<uint64_t>(pl, pl.o_tkey_sorted), wsp<double>(pl, pl.o_tx),
                                wsp<double>(pl, pl.o_ty), wsp<double>(pl, pl.o_tz), pl.ncrit,
                                wsp<long long>(pl, pl.o_tcnt), scan_scratch, &pl.n_tcells,
                                &pl.tlevel_begin, &need);
    if (rc == PBTC_EWORKSPACE) {
      pl.cap_tcells = 2 * need + 1024;
      *need_retry = 1;
      pl.err = "target trees larger than the workspace estimate";
    }
    if (rc) return rc;
    pl.n_tlevels = (int)pl.tlevel_begin.size() - 1;
  }
  int rc = adj_upload_small(pl, st);
  if (rc) return rc;
  // lists
  const int direct = pl.prm.op == PBTC_OP_DIRECT;
  long long* near_ptr = wsp<long long>(pl, pl.o_anear_ptr);
  long long* far_ptr = wsp<long long>(pl, pl.o_afar_ptr);
  int* flags = wsp<int>(pl, pl.o_flags);
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, flags, (int64_t)16);
  hipLaunchKernelGGL(k_adj_lists, dim3(nblocks(pl.nitems_adj, kTravWaves)), dim3(64 * kTravWaves),
                     0, st, pl.nitems_adj, wsp<int>(pl, pl.o_aitems), wsp<DevBlock>(pl, pl.o_blocks),
                     wsp<Cell>(pl, pl.o_tcells), wsp<double>(pl, pl.o_gpgrp), pl.prm.theta, direct,
                     pl.direct_below, 0, near_ptr, far_ptr, (int*)nullptr, (int*)nullptr,
                     (long long)0, (long long)0, flags);
  PBTC_LAUNCH_CHECK();
  scan_exclusive<long long>(near_ptr, pl.nitems_adj, scan_scratch, st);
  scan_exclusive<long long>(far_ptr, pl.nitems_adj, scan_scratch, st);
  long long tot[2] = {0, 0};
  PBTC_HIP(hipMemcpyAsync(&tot[0], near_ptr + pl.nitems_adj, 8, hipMemcpyDeviceToHost, st));
  PBTC_HIP(hipMemcpyAsync(&tot[1], far_ptr + pl.nitems_adj, 8, hipMemcpyDeviceToHost, st));
  PBTC_HIP(hipStreamSynchronize(st));
  if (tot[0] > pl.cap_anear || tot[1] > pl.cap_afar) {
    pl.cap_anear = std::max<int64_t>(pl.cap_anear, tot[0] + tot[0] / 8 + 1024);
    pl.cap_afar = std::max<int64_t>(pl.cap_afar, tot[1] + tot[1] / 8 + 1024);
    *need_retry = 1;
    pl.err = "adjoint lists larger than the workspace estimate";
    return PBTC_EWORKSPACE;
  }
  pl.n_anear = tot[0];
  pl.n_afar = tot[1];
  hipLaunchKernelGGL(k_adj_lists, dim3(nblocks(pl.nitems_adj, kTravWaves)), dim3(64 * kTravWaves),
                     0, st, pl.nitems_adj, wsp<int>(pl, pl.o_aitems), wsp<DevBlock>(pl, pl.o_blocks),
                     wsp<Cell>(pl, pl.o_tcells), wsp<double>(pl, pl.o_gpgrp), pl.prm.theta, direct,
                     pl.direct_below, 1, near_ptr, far_ptr, wsp<int>(pl, pl.o_anear),
                     wsp<int>(pl, pl.o_afar), (long long)pl.cap_anear, (long long)pl.cap_afar, flags);
  PBTC_LAUNCH_CHECK();
  {
    int hflag = 0;
    PBTC_HIP(hipMemcpyAsync(&hflag, flags, 4, hipMemcpyDeviceToHost, st));
    PBTC_HIP(hipStreamSynchronize(st));
    if (hflag) {
      pl.err = "tree traversal stack exhausted (octree too deep)";
      return PBTC_EDEVICE;
    }
  }
  // work units
  {
    std::vector<long long> np_(pl.nitems_adj + 1), fp_(pl.nitems_adj + 1);
    std::vector<int> nl(std::max<int64_t>(pl.n_anear, 1));
    std::vector<Cell> hc(pl.n_tcells);
    PBTC_HIP(hipMemcpy(np_.data(), near_ptr, 8 * (pl.nitems_adj + 1), hipMemcpyDeviceToHost));
    PBTC_HIP(hipMemcpy(fp_.data(), far_ptr, 8 * (pl.nitems_adj + 1), hipMemcpyDeviceToHost));
    if (pl.n_anear)
      PBTC_HIP(hipMemcpy(nl.data(), wsp<int>(pl, pl.o_anear), 4 * pl.n_anear, hipMemcpyDeviceToHost));
    PBTC_HIP(hipMemcpy(hc.data(), wsp<Cell>(pl, pl.o_tcells), sizeof(Cell) * pl.n_tcells,
                       hipMemcpyDeviceToHost));
    // the forward operator's tiles (chosen at set-up for the same lists' sizes)
    // the forward tiles are per 16-target group (four lanes per target); a
    // transposed unit has one lane per Gauss point of a 64-point group
    const int kUnitSources = std::max(64, pl.tile_sources / kQuarters);
    const int kUnitCells = std::max(1, pl.tile_cells / kQuarters);
    std::vector<int4> units;
    std::vector<int> uptr;
    const bool tree = pl.prm.op == PBTC_OP_TREECODE;
    // algorithmic operations of each launch (kernel timing)
    for (int ph = 0; ph < 2; ++ph)
      for (int ks = 0; ks < KS_COUNT; ++ks) {
        double fp = 0.0, fm = 0.0;
        for (int item : pl.aitem_list[ph][ks]) {
          const int bi = pl.aitem_block[item];
          const int s_ = pl.blocks[bi].s;
          const int64_t g = item - pl.blk_aitem_off[bi];
          const int64_t ngs = pl.gp_off[s_ + 1] - pl.gp_off[s_];
          const double ntg = (double)std::min<int64_t>(kAGroup, ngs - g * kAGroup);
          double src = 0.0;
          for (long long e = np_[item]; e < np_[item + 1]; ++e) src += hc[nl[e]].count;
          fp += ntg * src * adj_p2p_flop_per_pair(ks);
          if (tree) fm += ntg * (double)(fp_[item + 1] - fp_[item]) * adj_m2p_flop_per_eval(pl.P, ks);
        }
        pl.alaunch_flop_p2p[ph][ks] = fp;
        pl.alaunch_flop_m2p[ph][ks] = fm;
      }
    for (int ph = 0; ph < 2; ++ph)
      for (int ks = 0; ks < KS_COUNT; ++ks)
        for (int kind = 0; kind < 2; ++kind) {
          UnitSet& us = pl.aunits[ph][ks][kind];
          us.off = (int64_t)units.size();
          us.ptr_off = (int64_t)uptr.size();
          for (int item : pl.aitem_list[ph][ks]) {
            uptr.push_back((int)(units.size() - us.off));
            if (kind == 0) {
              long long e = np_[item], acc = 0, start = e;
              for (; e < np_[item + 1]; ++e) {
                const int cnt = hc[nl[e]].count;
                if (acc > 0 && acc + cnt > kUnitSources) {
                  units.push_back(make_int4(item, (int)start, (int)e, 0));
                  start = e;
                  acc = 0;
                }
                acc += cnt;
              }
              if (e > start) units.push_back(make_int4(item, (int)start, (int)e, 0));
            } else if (tree) {
              for (long long e = fp_[item]; e < fp_[item + 1]; e += kUnitCells)
                units.push_back(make_int4(item, (int)e,
                                          (int)std::min<long long>(e + kUnitCells, fp_[item + 1]), 0));
            }
          }
          uptr.push_back((int)(units.size() - us.off));
          us.n = (int64_t)units.size() - us.off;
        }
    if ((int64_t)units.size() > pl.cap_aunits || (int64_t)uptr.size() > pl.cap_auptr) {
      pl.cap_aunits = (int64_t)units.size() + 1024;
      pl.cap_auptr = (int64_t)uptr.size() + 64;
      *need_retry = 1;
      pl.err = "adjoint work units exceed the workspace estimate";
      return PBTC_EWORKSPACE;
    }
    PBTC_HIP(hipMemcpy(wsp<int4>(pl, pl.o_aunits), units.data(), 16 * units.size(), hipMemcpyHostToDevice));
    PBTC_HIP(hipMemcpy(wsp<int>(pl, pl.o_auptr), uptr.data(), 4 * uptr.size(), hipMemcpyHostToDevice));

    // direct moment pass: per phase, every (cell, slot of its tree) pair's
    // sources in chunks of at most kMomSpan
    std::vector<int4> amch, amp;
    const int ms = pl.adj_ms;
    for (int ph = 0; ph < 2; ++ph) {
      pl.am_chunk_off[ph] = (int64_t)amch.size();
      pl.am_pair_off[ph] = (int64_t)amp.size();
      const std::vector<int>& ts = pl.adj_tslot_host[ph];
      for (int64_t c = 0; c < pl.n_tcells; ++c) {
        if (hc[c].count == 0) continue;
        for (int l = 0; l < ms; ++l) {
          const int slot = ts[(size_t)hc[c].surf * ms + l];
          if (slot < 0) continue;
          const int first = (int)amch.size();
          for (int o = 0; o < hc[c].count; o += kMomSpan)
            amch.push_back(make_int4((int)c, hc[c].begin + o, std::min(kMomSpan, hc[c].count - o), slot));
          amp.push_back(make_int4((int)(c * ms + l), first, (int)amch.size(), 0));
        }
      }
    }
    pl.am_chunk_off[2] = (int64_t)amch.size();
    pl.am_pair_off[2] = (int64_t)amp.size();
    if ((int64_t)amch.size() > pl.cap_amchunks || (int64_t)amp.size() > pl.cap_ampairs) {
      pl.cap_amchunks = std::max<int64_t>(pl.cap_amchunks, (int64_t)amch.size() + 1024);
      pl.cap_ampairs = std::max<int64_t>(pl.cap_ampairs, (int64_t)amp.size() + 64);
      *need_retry = 1;
      pl.err = "adjoint moment chunks exceed the workspace estimate";
      return PBTC_EWORKSPACE;
    }
    if (!amch.empty())
      PBTC_HIP(hipMemcpy(wsp<int4>(pl, pl.o_amchunks), amch.data(), 16 * amch.size(), hipMemcpyHostToDevice));
    if (!amp.empty())
      PBTC_HIP(hipMemcpy(wsp<int4>(pl, pl.o_ampairs), amp.data(), 16 * amp.size(), hipMemcpyHostToDevice));
  }
  // transposed near-field table (CSC by (block, panel)), deterministic order
  {
    long long* cnt = wsp<long long>(pl, pl.o_csc_fill);
    long long* cptr = wsp<long long>(pl, pl.o_csc_ptr);
    hipLaunchKernelGGL(k_zero_ll, dim3(nblocks(pl.ncsc + 1, T)), dim3(T), 0, st, cnt, pl.ncsc + 1);
    hipLaunchKernelGGL(k_csc_count, dim3(nblocks(pl.nf_rows, T)), dim3(T), 0, st, pl.nf_rows,
                       wsp<int>(pl, pl.o_nf_rowblk), wsp<DevBlock>(pl, pl.o_blocks),
                       wsp<long long>(pl, pl.o_nf_ptr), wsp<int>(pl, pl.o_nf_col), cnt, cptr,
                       (int*)nullptr, (int*)nullptr, 0);
    PBTC_HIP(hipMemcpyAsync(cptr, cnt, 8 * pl.ncsc, hipMemcpyDeviceToDevice, st));
    scan_exclusive<long long>(cptr, pl.ncsc, scan_scratch, st);
    hipLaunchKernelGGL(k_zero_ll, dim3(nblocks(pl.ncsc + 1, T)), dim3(T), 0, st, cnt, pl.ncsc + 1);
    hipLaunchKernelGGL(k_csc_count, dim3(nblocks(pl.nf_rows, T)), dim3(T), 0, st, pl.nf_rows,
                       wsp<int>(pl, pl.o_nf_rowblk), wsp<DevBlock>(pl, pl.o_blocks),
                       wsp<long long>(pl, pl.o_nf_ptr), wsp<int>(pl, pl.o_nf_col), cnt, cptr,
                       wsp<int>(pl, pl.o_csc_ent), wsp<int>(pl, pl.o_csc_row), 1);
    hipLaunchKernelGGL(k_csc_sort, dim3(nblocks(pl.ncsc, T)), dim3(T), 0, st, pl.ncsc, cptr,
                       wsp<int>(pl, pl.o_csc_ent), wsp<int>(pl, pl.o_csc_row));
    PBTC_LAUNCH_CHECK();
    PBTC_HIP(hipStreamSynchronize(st));
  }
  pl.adj_done = true;
  return PBTC_OK;
}

// slot tables, item lists and gather tables of the transposed operator
static int adj_upload_small(pbtc_plan_t& pl, hipStream_t st) {
  PBTC_HIP(hipMemcpyAsync(wsp<int>(pl, pl.o_aitems), pl.aitem_block.data(),
                          4 * pl.aitem_block.size(), hipMemcpyHostToDevice, st));
  for (int ph = 0; ph < 2; ++ph) {
    for (int ks = 0; ks < KS_COUNT; ++ks)
      if (!pl.aitem_list[ph][ks].empty())
        PBTC_HIP(hipMemcpyAsync(wsp<int>(pl, pl.o_aitem_list[ph][ks]), pl.aitem_list[ph][ks].data(),
                                4 * pl.aitem_list[ph][ks].size(), hipMemcpyHostToDevice, st));
    if (!pl.slots[ph].empty())
      PBTC_HIP(hipMemcpyAsync(wsp<DevSlot>(pl, pl.o_slots[ph]), pl.slots[ph].data(),
                              sizeof(DevSlot) * pl.slots[ph].size(), hipMemcpyHostToDevice, st));
    PBTC_HIP(hipMemcpyAsync(wsp<DevGather>(pl, pl.o_gather[ph]), pl.gathers[ph].data(),
                            sizeof(DevGather) * pl.gathers[ph].size(), hipMemcpyHostToDevice, st));
    if (!pl.gather_slots[ph].empty())
      PBTC_HIP(hipMemcpyAsync(wsp<int>(pl, pl.o_gather_slots[ph]), pl.gather_slots[ph].data(),
                              4 * pl.gather_slots[ph].size(), hipMemcpyHostToDevice, st));
  }
  // slot -> block, kernel index; per phase: slot ids and block ids
  std::vector<int> sb, sk, blk[2], sid[2];
  for (size_t bi = 0; bi < pl.blocks.size(); ++bi) {
    const Block& b = pl.blocks[bi];
    for (int k = 0; k < b.nk; ++k) {
      sb.push_back((int)bi);
      sk.push_back(k);
      sid[b.reaction ? 1 : 0].push_back((int)(pl.blk_slot0[bi] + k));
    }
    blk[b.reaction ? 1 : 0].push_back((int)bi);
  }
  pl.adj_blist[0] = blk[0];
  pl.adj_blist[1] = blk[1];
  pl.adj_sids[0] = sid[0];
  pl.adj_sids[1] = sid[1];
  PBTC_HIP(hipMemcpyAsync(wsp<int>(pl, pl.o_slot_block), sb.data(), 4 * sb.size(), hipMemcpyHostToDevice, st));
  PBTC_HIP(hipMemcpyAsync(wsp<int>(pl, pl.o_slot_kidx), sk.data(), 4 * sk.size(), hipMemcpyHostToDevice, st));
  for (int ph = 0; ph < 2; ++ph) {
    // the slots of each target-set tree, by local slot number
    std::vector<int>& ts = pl.adj_tslot_host[ph];
    ts.assign(std::max<size_t>(pl.tsets.size() * pl.adj_ms, 1), -1);
    for (size_t bi = 0; bi < pl.blocks.size(); ++bi) {
      const Block& b = pl.blocks[bi];
      if ((b.reaction ? 1 : 0) != ph) continue;
      for (int k = 0; k < b.nk; ++k)
        ts[(size_t)b.t * pl.adj_ms + pl.blk_lslot0[bi] + k] = (int)(pl.blk_slot0[bi] + k);
    }
    PBTC_HIP(hipMemcpyAsync(wsp<int>(pl, pl.o_adj_tslot[ph]), ts.data(), 4 * ts.size(),
                            hipMemcpyHostToDevice, st));
    if (!blk[ph].empty())
      PBTC_HIP(hipMemcpyAsync(wsp<int>(pl, pl.o_adj_blist[ph]), blk[ph].data(), 4 * blk[ph].size(),
                              hipMemcpyHostToDevice, st));
    if (!sid[ph].empty())
      PBTC_HIP(hipMemcpyAsync(wsp<int>(pl, pl.o_adj_sids[ph]), sid[ph].data(), 4 * sid[ph].size(),
                              hipMemcpyHostToDevice, st));
  }
  std::vector<long long> tab(2 * (pl.nsurf + 1));
  for (int s = 0; s <= pl.nsurf; ++s) {
    tab[s] = pl.pan_off[s];
    tab[pl.nsurf + 1 + s] = pl.gp_off[s];
  }
  PBTC_HIP(hipMemcpyAsync(wsp<long long>(pl, pl.o_adj_tab), tab.data(), 8 * tab.size(),
                          hipMemcpyHostToDevice, st));
  PBTC_HIP(hipStreamSynchronize(st));
  return PBTC_OK;
}

void prof_mark(pbtc_plan_t& pl, hipStream_t st, bool on, int kind, double flop, bool begin);
void prof_collect(pbtc_plan_t& pl);

template <typename real>
void launch_adj_p2p(hipStream_t st, int ks, const UnitArgs& a, int grid, const Src<real>* gpos,
                    const Src<real>* asrc, real* partial);
template <typename real>
void launch_adj_m2p(hipStream_t st, int P, const UnitArgs& a, int grid, const Src<real>* gpos,
                    const real* mom, int ms, int kind, int kslot, real* partial);

template <typename real>
static int adj_moments(pbtc_plan_t& pl, hipStream_t st, int phase, real* mom) {
  const int64_t c0 = pl.am_chunk_off[phase], c1 = pl.am_chunk_off[phase + 1];
  const int64_t p0 = pl.am_pair_off[phase], p1 = pl.am_pair_off[phase + 1];
  if (p1 == p0) return PBTC_OK;
  const Cell* cells = wsp<Cell>(pl, pl.o_tcells);
  const int4* chunks = wsp<int4>(pl, pl.o_amchunks) + c0;
  const int4* pairs = wsp<int4>(pl, pl.o_ampairs) + p0;
  const int* sb = wsp<int>(pl, pl.o_slot_block);
  const int* sk = wsp<int>(pl, pl.o_slot_kidx);
  const DevBlock* blocks = wsp<DevBlock>(pl, pl.o_blocks);
  const Src<real>* asrc = wsp<Src<real>>(pl, sizeof(real) == 4 ? pl.o_asrc32 : pl.o_asrc64);
  // partial moments of this phase's chunks (chunk ids are global; the
  // pairs' ranges index the same global table)
  real* part = wsp<real>(pl, pl.o_ampart);
#define PBTC_AMOM(PP)                                                                           \
  case PP:                                                                                      \
    if (c1 > c0)                                                                                \
      hipLaunchKernelGGL((k_adj_p2m_chunk<real, PP>), dim3((unsigned)(c1 - c0)),                \
                         dim3(kAMomThreads), 0, st, chunks, cells, sb, sk, blocks, asrc,        \
                         part + (size_t)c0 * 2 * ncoef(PP));                                    \
    hipLaunchKernelGGL((k_adj_mom_sum<real, PP>), dim3((unsigned)(p1 - p0)), dim3(256), 0, st,  \
                       pairs, part, mom);                                                       \
    break;
  switch (pl.P) {
    PBTC_AMOM(2)
    PBTC_AMOM(4)
    PBTC_AMOM(6)
    PBTC_AMOM(8)
    PBTC_AMOM(10)
    default:
      pl.err = "unsupported P";
      return PBTC_EINVAL;
  }
#undef PBTC_AMOM
  PBTC_LAUNCH_CHECK();
  return PBTC_OK;
}

// z = A^T lam (phase 0) or z = S^T lam (phase 1, lam = charge weights)
template <typename real>
static int transpose_impl(pbtc_plan_t& pl, hipStream_t st, const double* lam, double* z, int phase) {
  const int T = 256;
  const bool tree = pl.prm.op == PBTC_OP_TREECODE;
  // every profile-th FP32 evaluation of A^T x times its P2P and M2P launches
  const bool timed = sizeof(real) == 4 && phase == 0 && pl.prm.profile > 0 &&
                     pl.aprof_count++ % pl.prm.profile == 0;
  double* muS = wsp<double>(pl, pl.o_mu_s);
  double* muD = wsp<double>(pl, pl.o_mu_d);
  const auto& slots = pl.slots[phase];
  if (slots.empty()) {
    hipLaunchKernelGGL(k_zero_f64, dim3(nblocks(pl.nunk, 256)), dim3(256), 0, st, z,
                       (int64_t)pl.nunk);
    PBTC_LAUNCH_CHECK();
    return PBTC_OK;
  }
  {
    int64_t nmax = 0;
    for (const DevSlot& s : slots) nmax = std::max<int64_t>(nmax, s.n);
    hipLaunchKernelGGL(k_adj_mu, dim3(nblocks(nmax, T), (unsigned)slots.size()), dim3(T), 0, st,
                       wsp<DevSlot>(pl, pl.o_slots[phase]), lam, muS, muD);
  }
  const real* tx = wsp<real>(pl, sizeof(real) == 4 ? pl.o_txf : pl.o_tx);
  const real* ty = wsp<real>(pl, sizeof(real) == 4 ? pl.o_tyf : pl.o_ty);
  const real* tz = wsp<real>(pl, sizeof(real) == 4 ? pl.o_tzf : pl.o_tz);
  Src<real>* asrc = wsp<Src<real>>(pl, sizeof(real) == 4 ? pl.o_asrc32 : pl.o_asrc64);
  {
    int64_t nmax = 0;
    for (int bi : pl.adj_blist[phase]) nmax = std::max<int64_t>(nmax, pl.tsets[pl.blocks[bi].t].n);
    hipLaunchKernelGGL(k_adj_src<real>, dim3(nblocks(nmax, T), (unsigned)pl.adj_blist[phase].size()),
                       dim3(T), 0, st, wsp<int>(pl, pl.o_adj_blist[phase]),
                       wsp<DevBlock>(pl, pl.o_blocks), tx, ty, tz, wsp<int>(pl, pl.o_tidx), muS,
                       muD, asrc);
  }
  PBTC_LAUNCH_CHECK();
  real* mom = wsp<real>(pl, sizeof(real) == 4 ? pl.o_amom32 : pl.o_amom64);
  if (tree) {
    const int rc = adj_moments<real>(pl, st, phase, mom);
    if (rc) return rc;
  }
  const Src<real>* gpos = wsp<Src<real>>(pl, sizeof(real) == 4 ? pl.o_gpos32 : pl.o_gpos64);
  real* partial = wsp<real>(pl, pl.o_partial);
  double* aS = wsp<double>(pl, pl.o_aout_s);
  double* aD = wsp<double>(pl, pl.o_aout_d);
  UnitArgs a;
  a.item_block = wsp<int>(pl, pl.o_aitems);
  a.blocks = wsp<DevBlock>(pl, pl.o_blocks);
  a.cells = wsp<Cell>(pl, pl.o_tcells);
  for (int ks = 0; ks < KS_COUNT; ++ks) {
    const int n = (int)pl.aitem_list[phase][ks].size();
    if (n == 0) continue;
    const int* list = wsp<int>(pl, pl.o_aitem_list[phase][ks]);
    const bool two = ks == KS_LY || ks == KS_YY;
    {
      const UnitSet& us = pl.aunits[phase][ks][0];
      a.units = wsp<int4>(pl, pl.o_aunits + 16 * us.off);
      a.nunits = (int)us.n;
      a.cells_list = wsp<int>(pl, pl.o_anear);
      const int grid = nblocks(us.n, kWaves);
      if (us.n > 0) {
        prof_mark(pl, st, timed, 3, pl.alaunch_flop_p2p[phase][ks], true);
        launch_adj_p2p<real>(st, ks, a, grid, gpos, asrc, partial);
        prof_mark(pl, st, timed, 3, 0.0, false);
      }
      const int* uptr = wsp<int>(pl, pl.o_auptr + 4 * us.ptr_off);
      if (two)
        hipLaunchKernelGGL((k_adj_reduce<real, 4>), dim3(n), dim3(256), 0, st, list, uptr, a.item_block,
                           a.blocks, partial, aS, aD, 0, 0);
      else
        hipLaunchKernelGGL((k_adj_reduce<real, 2>), dim3(n), dim3(256), 0, st, list, uptr, a.item_block,
                           a.blocks, partial, aS, aD, 0, 0);
      PBTC_LAUNCH_CHECK();
    }
    if (tree && pl.n_afar > 0) {
      const UnitSet& us = pl.aunits[phase][ks][1];
      if (us.n == 0) continue;
      a.units = wsp<int4>(pl, pl.o_aunits + 16 * us.off);
      a.nunits = (int)us.n;
      a.cells_list = wsp<int>(pl, pl.o_afar);
      const int grid = nblocks(us.n, kWaves);
      const int* uptr = wsp<int>(pl, pl.o_auptr + 4 * us.ptr_off);
      const int kind0 = (ks == KS_L || ks == KS_LY) ? 0 : 1;
      for (int slot = 0; slot < (two ? 2 : 1); ++slot) {
        const int kind = slot == 0 ? kind0 : 1;
        const double fl = pl.alaunch_flop_m2p[phase][ks] * adj_m2p_flop_one(pl.P, kind) /
                          adj_m2p_flop_per_eval(pl.P, ks);
        prof_mark(pl, st, timed, 4 + kind, fl, true);
        launch_adj_m2p<real>(st, pl.P, a, grid, gpos, mom, pl.adj_ms, kind, slot, partial);
        prof_mark(pl, st, timed, 4 + kind, 0.0, false);
        hipLaunchKernelGGL((k_adj_reduce<real, 2>), dim3(n), dim3(256), 0, st, list, uptr,
                           a.item_block, a.blocks, partial, aS, aD, 1, slot);
      }
      PBTC_LAUNCH_CHECK();
    }
  }
  const long long* tab = wsp<long long>(pl, pl.o_adj_tab);
  hipLaunchKernelGGL(k_adj_gather<real>, dim3(nblocks(pl.np_tot, T)), dim3(T), 0, st, pl.np_tot,
                     pl.prm.K, wsp<int>(pl, pl.o_pan_surf), tab, tab + pl.nsurf + 1,
                     wsp<DevGather>(pl, pl.o_gather[phase]), wsp<int>(pl, pl.o_gather_slots[phase]),
                     wsp<int>(pl, pl.o_slot_block), wsp<int>(pl, pl.o_slot_kidx),
                     wsp<DevBlock>(pl, pl.o_blocks), wsp<int>(pl, pl.o_gp_pos),
                     wsp<double>(pl, pl.o_gw), aS, aD, wsp<long long>(pl, pl.o_csc_ptr),
                     wsp<int>(pl, pl.o_csc_ent), wsp<int>(pl, pl.o_csc_row),
                     wsp<real>(pl, sizeof(real) == 4 ? pl.o_nf_v32 : pl.o_nf_v64), muS, muD,
                     wsp<int>(pl, pl.o_pidx), lam, phase == 0 ? 1 : 0, z);
  PBTC_LAUNCH_CHECK();
  return PBTC_OK;
}

void compute_layout(pbtc_plan_t& pl);

static int ensure_adjoint(pbtc_plan_t& pl, hipStream_t st) {
  if (pl.adj_done) return PBTC_OK;
  int retry = 0;
  const int rc = adjoint_setup(pl, st, &retry);
  if (rc == PBTC_EWORKSPACE && retry) {
    // the grown capacities move every array: the workspace must be set up
    // (and the forward system solved) again at the new size
    compute_layout(pl);
    pl.setup_done = false;
    pl.dev_solved = false;
    pl.err = "workspace too small for the transposed operator: " + pl.err +
             " (grow it to pbtc_result.workspace_needed, solve again and call again)";
  }
  return rc;
}

int apply_transpose(pbtc_plan_t& pl, hipStream_t st, const double* x, double* y, int precision,
                    int phase) {
  const int rc = ensure_adjoint(pl, st);
  if (rc) return rc;
  if (precision == PBTC_FP64) return transpose_impl<double>(pl, st, x, y, phase);
  return transpose_impl<float>(pl, st, x, y, phase);
}

// sum over the listed (a offset, b offset, n) triples of a . b (device dots ->
// host).  Long triples are cut into pieces of at most kDotPiece elements, one
// work-group each, whose dots the host adds in piece order.
static int pair_dots(pbtc_plan_t& pl, hipStream_t st, const std::vector<long long>& tab,
                     const double* A, const double* B, std::vector<double>* out) {
  constexpr long long kDotPiece = 16384;
  out->assign(tab.size() / 3, 0.0);
  if (tab.empty()) return PBTC_OK;
  std::vector<long long> pieces;
  std::vector<int> owner;
  for (size_t t = 0; t < tab.size() / 3; ++t) {
    const long long oa = tab[3 * t], ob = tab[3 * t + 1], n = tab[3 * t + 2];
    for (long long o = 0; o < n; o += kDotPiece) {
      pieces.insert(pieces.end(), {oa + o, ob + o, std::min(kDotPiece, n - o)});
      owner.push_back((int)t);
    }
  }
  long long* dtab = wsp<long long>(pl, pl.o_dots);
  double* dres = reinterpret_cast<double*>(dtab + 3 * 1024);
  std::vector<double> part(owner.size());
  for (size_t base = 0; base < owner.size(); base += 1024) {
    const size_t cnt = std::min<size_t>(1024, owner.size() - base);
    PBTC_HIP(hipMemcpyAsync(dtab, pieces.data() + 3 * base, 8 * 3 * cnt, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_pair_dots, dim3((unsigned)cnt), dim3(kT), 0, st, dtab, A, B, dres);
    PBTC_LAUNCH_CHECK();
    PBTC_HIP(hipMemcpyAsync(part.data() + base, dres, 8 * cnt, hipMemcpyDeviceToHost, st));
    PBTC_HIP(hipStreamSynchronize(st));
  }
  for (size_t i = 0; i < owner.size(); ++i) (*out)[owner[i]] += part[i];
  return PBTC_OK;
}

int launch_dk0_diag(pbtc_plan_t& pl, hipStream_t st, const double* x, double* e);

int device_backward(pbtc_plan_t& pl, hipStream_t st, double gE, double* dq, double* dk, double* de,
                    pbtc_result* res) {
  int rc = ensure_adjoint(pl, st);
  if (rc) {
    if (res) res->workspace_needed = pl.ws_bytes;
    return rc;
  }
  const int T = 256;
  const double C = 4.0 * kPi * kCoulomb;
  prof_collect(pl);
  for (int i = 0; i < kProfKinds; ++i) pl.prof_t[i] = pl.prof_flop[i] = 0.0, pl.prof_n[i] = 0;
  double* x = wsp<double>(pl, pl.o_x);
  double* lam = wsp<double>(pl, pl.o_lam);
  double* rhs = wsp<double>(pl, pl.o_adj_rhs);
  double* q = wsp<double>(pl, pl.o_q);
  // adjoint right-hand side S^T q (FP64)
  rc = transpose_impl<double>(pl, st, q, rhs, 1);
  if (rc) return rc;
  int iters = 0, n32 = 0, n64 = 0, nref = 0;
  double rel = 0.0;
  bool conv = false;
  std::vector<double> hist;
  rc = solve_with_ops(pl, st, true, rhs, lam, &iters, &n32, &n64, &nref, &rel, &conv, &hist);
  if (rc) return rc;
  // dG/dq = 1/2 C (phi_reac + B^T lam)
  double* g = wsp<double>(pl, pl.o_z2);
  PBTC_HIP(hipMemcpyAsync(g, wsp<double>(pl, pl.o_phi_reac), 8 * pl.nq, hipMemcpyDeviceToDevice, st));
  rc = upload_coulomb_rows(pl, st);
  if (rc) return rc;
  if (pl.nq > 0) {
    const char* ct = wsp<char>(pl, pl.o_crows);
    const int* reg_ptr = reinterpret_cast<const int*>(ct + sizeof(DevCoulRow) * pl.rows.size());
    hipLaunchKernelGGL(k_coulomb_t_rows, dim3(nblocks(pl.nq, T / 64)), dim3(T), 0, st,
                       (long long)pl.nq, reinterpret_cast<const DevCoulRow*>(ct), reg_ptr,
                       reg_ptr + pl.nreg + 1, wsp<int>(pl, pl.o_qreg), wsp<double>(pl, pl.o_qxyz),
                       wsp<double>(pl, pl.o_cx), wsp<double>(pl, pl.o_cy), wsp<double>(pl, pl.o_cz),
                       lam, g);
  }
  PBTC_LAUNCH_CHECK();
  std::vector<double> gq(pl.nq);
  PBTC_HIP(hipMemcpyAsync(gq.data(), g, 8 * pl.nq, hipMemcpyDeviceToHost, st));
  PBTC_HIP(hipStreamSynchronize(st));
  if (dq)
    for (int64_t k = 0; k < pl.nq; ++k) dq[k] = gE * 0.5 * C * gq[k];

  // eps: forward FP64 block outputs at x (A and S), then dot products
  double* y = wsp<double>(pl, pl.o_r);
  std::vector<double> deps(pl.nreg, 0.0);
  {
    // reaction blocks first (phase 1 leaves S of the reaction blocks), then A
    rc = apply_operator(pl, st, x, wsp<double>(pl, pl.o_phi_reac), PBTC_FP64, 1);
    if (rc) return rc;
    rc = apply_operator(pl, st, x, y, PBTC_FP64, 0);
    if (rc) return rc;
    const pbtc_problem& P = pl.prob;
    auto dratio = [&](int r, int s, int p) {
      const int i = P.surfaces[s].inner;
      if (i == r) return 0.0;
      return (p == i ? 1.0 : 0.0) / P.regions[r].eps -
             (p == r ? P.regions[i].eps / (P.regions[r].eps * P.regions[r].eps) : 0.0);
    };
    auto sigma = [&](int r, int s) { return P.surfaces[s].inner == r ? 1.0 : -1.0; };
    // <lam_(t,r), S_(b,k)> for every forward term, <q_r, S_(b)> for every reaction term,
    // <lam_(t,r), b_(t,r)> for every row block
    std::vector<long long> tA, tS, tB;
    for (const RowBlock& rb : pl.rows)
      for (const RowTerm& t : rb.terms)
        tA.insert(tA.end(), {(long long)rb.row_off, (long long)pl.blocks[t.block].out[t.kidx],
                             (long long)rb.n});
    for (const RowBlock& rb : pl.reac_rows)
      for (const RowTerm& t : rb.terms)
        tS.insert(tS.end(), {(long long)rb.row_off, (long long)pl.blocks[t.block].out[t.kidx],
                             (long long)rb.n});
    for (const RowBlock& rb : pl.rows)
      tB.insert(tB.end(), {(long long)rb.row_off, (long long)rb.row_off, (long long)rb.n});
    std::vector<double> dA, dS, dB;
    rc = pair_dots(pl, st, tA, lam, wsp<double>(pl, pl.o_S), &dA);
    if (rc) return rc;
    rc = pair_dots(pl, st, tS, q, wsp<double>(pl, pl.o_S), &dS);
    if (rc) return rc;
    rc = pair_dots(pl, st, tB, lam, wsp<double>(pl, pl.o_b), &dB);
    if (rc) return rc;
    for (int p = 0; p < pl.nreg; ++p) {
      double vA = 0.0, vS = 0.0, vB = 0.0;
      size_t i = 0;
      for (const RowBlock& rb : pl.rows)
        for (const RowTerm& t : rb.terms) {
          const int s = pl.blocks[t.block].s;
          vA += -sigma(rb.r, s) * dratio(rb.r, s, p) * dA[i++];
        }
      i = 0;
      for (const RowBlock& rb : pl.reac_rows)
        for (const RowTerm& t : rb.terms) {
          const int s = pl.blocks[t.block].s;
          vS += sigma(rb.r, s) * dratio(rb.r, s, p) * dS[i++];
        }
      i = 0;
      for (const RowBlock& rb : pl.rows) {
        if (rb.r == p) vB += -dB[i] / P.regions[p].eps;
        ++i;
      }
      deps[p] = 0.5 * C * (vS - vA + vB);
    }
  }
  // kappa: central difference of the FP64 Lagrangian in kappa_p.  Only the
  // rows of region p (forward rows, their Coulomb terms, the reaction rows of
  // its charges) depend on kappa_p, so the difference quotient of each region
  // reads those rows alone.  All regions that share one kappa value are then
  // perturbed together (their kernels are shared between blocks), and one
  // pair of operator evaluations serves all of them (every molecule of a
  // batch at once).
  std::vector<double> dkap(pl.nreg, 0.0);
  std::vector<double> kvals;
  for (int p = 0; p < pl.nreg; ++p) {
    const double k0 = pl.prob.regions[p].kappa;
    if (k0 != 0.0 && std::find(kvals.begin(), kvals.end(), k0) == kvals.end())
      kvals.push_back(k0);
  }
  for (const double k0 : kvals) {
    std::vector<int> group;
    for (int p = 0; p < pl.nreg; ++p)
      if (pl.prob.regions[p].kappa == k0) group.push_back(p);
    std::vector<std::pair<int, int>> kern;  // (block, kernel) pairs evaluated with k0
    for (size_t bi = 0; bi < pl.blocks.size(); ++bi)
      for (int k = 0; k < pl.blocks[bi].nk; ++k)
        if (pl.blocks[bi].kappa[k] == k0) kern.emplace_back((int)bi, k);
    // restricted dots: q . phi over region p's charges, lam . (A x) and
    // lam . b over region p's forward rows; owner = index into group
    std::vector<long long> tq, tr;
    std::vector<int> oq, orow;
    for (size_t gi = 0; gi < group.size(); ++gi) {
      const int p = group[gi];
      const int64_t nqp = pl.prob.charges[p].n();
      if (nqp > 0) {
        tq.insert(tq.end(), {(long long)pl.q_off_region[p], (long long)pl.q_off_region[p],
                             (long long)nqp});
        oq.push_back((int)gi);
      }
      for (const RowBlock& rb : pl.rows)
        if (rb.r == p) {
          tr.insert(tr.end(), {(long long)rb.row_off, (long long)rb.row_off, (long long)rb.n});
          orow.push_back((int)gi);
        }
    }
    const double h = 1e-4 * k0;
    std::vector<double> val[2];
    auto set_kappa = [&](double kv) -> int {
      for (int p : group) pl.prob.regions[p].kappa = kv;
      for (const auto& bk : kern) pl.blocks[bk.first].kappa[bk.second] = kv;
      int r2 = upload_descriptors(pl, st);
      if (!r2) r2 = recompute_near_values(pl, st);
      if (!r2) r2 = recompute_rhs(pl, st);
      return r2;
    };
    for (int side = 0; side < 2; ++side) {
      rc = set_kappa(side == 0 ? k0 + h : k0 - h);
      if (rc) return rc;
      double* phi = wsp<double>(pl, pl.o_z2);
      rc = apply_operator(pl, st, x, phi, PBTC_FP64, 1);
      if (!rc) rc = apply_operator(pl, st, x, y, PBTC_FP64, 0);
      if (rc) return rc;
      std::vector<double> r1, r2, r3;
      rc = pair_dots(pl, st, tq, q, phi, &r1);
      if (!rc) rc = pair_dots(pl, st, tr, lam, y, &r2);
      if (!rc) rc = pair_dots(pl, st, tr, lam, wsp<double>(pl, pl.o_b), &r3);
      if (rc) return rc;
      val[side].assign(group.size(), 0.0);
      for (size_t i = 0; i < oq.size(); ++i) val[side][oq[i]] += r1[i];
      for (size_t i = 0; i < orow.size(); ++i) val[side][orow[i]] += r3[i] - r2[i];
    }
    rc = set_kappa(k0);
    if (rc) return rc;
    for (size_t gi = 0; gi < group.size(); ++gi)
      dkap[group[gi]] = 0.5 * C * (val[0][gi] - val[1][gi]) / (2.0 * h);
  }
  // kappa = 0 (Laplace regions): the derivative kernels are d G / d kappa =
  // -1/(4 pi) and d (n . grad G) / d kappa = 0 there, so with
  // Psi_s = sum_j A_j psi_j over surface s, Lambda_rb = sum of lam over a row
  // block, E_rb = sum_i lam_i e_i (e from k_dk0_diag: the self-term remainder)
  // and Q_p the charge of region p:
  //   q^T S' x    = Q_p sum_{reaction terms of p} sigma c (-Psi_s / (4 pi))
  //   lam^T A' x  = sum_{rows of p} sum_terms -sigma c (-Psi_s / (4 pi) Lambda_rb
  //                                                    + [s = t] E_rb)
  //   lam^T B' q  = sum_{rows of p} Lambda_rb (-Q_p / (4 pi eps_p))
  bool any0 = false;
  for (int p = 0; p < pl.nreg; ++p) any0 = any0 || pl.prob.regions[p].kappa == 0.0;
  if (any0) {
    double* e = wsp<double>(pl, pl.o_z2);         // np_tot values
    double* ones = e + pl.np_tot;                  // np_tot values (o_z2 holds 2 np_tot)
    rc = launch_dk0_diag(pl, st, x, e);
    if (rc) return rc;
    hipLaunchKernelGGL(k_ones_f64, dim3(nblocks(pl.np_tot, T)), dim3(T), 0, st, ones, pl.np_tot);
    PBTC_LAUNCH_CHECK();
    std::vector<long long> tP, tL, tE;
    for (int s = 0; s < pl.nsurf; ++s) {
      const int64_t ns = pl.pan_off[s + 1] - pl.pan_off[s];
      tP.insert(tP.end(), {(long long)pl.pan_off[s], (long long)(pl.unk_off[s] + ns), (long long)ns});
    }
    for (const RowBlock& rb : pl.rows) {
      tL.insert(tL.end(), {(long long)rb.row_off, 0LL, (long long)rb.n});
      tE.insert(tE.end(), {(long long)rb.row_off, (long long)pl.pan_off[rb.t], (long long)rb.n});
    }
    std::vector<double> Psi, Lam, Ed;
    rc = pair_dots(pl, st, tP, wsp<double>(pl, pl.o_area), x, &Psi);
    if (!rc) rc = pair_dots(pl, st, tL, lam, ones, &Lam);
    if (!rc) rc = pair_dots(pl, st, tE, lam, e, &Ed);
    if (rc) return rc;
    for (int p = 0; p < pl.nreg; ++p) {
      const Region& R = pl.prob.regions[p];
      if (R.kappa != 0.0) continue;
      double Qp = 0.0;
      for (double v : pl.prob.charges[p].q) Qp += v;
      double qSx = 0.0, lAx = 0.0, lBq = 0.0;
      for (const RowBlock& rb : pl.reac_rows)
        if (rb.r == p)
          for (const RowTerm& t : rb.terms) qSx += Qp * t.sigma_c * (-Psi[pl.blocks[t.block].s] * kInv4Pi);
      for (size_t i = 0; i < pl.rows.size(); ++i) {
        const RowBlock& rb = pl.rows[i];
        if (rb.r != p) continue;
        for (const RowTerm& t : rb.terms) {
          const int s = pl.blocks[t.block].s;
          lAx += -t.sigma_c * (-Psi[s] * kInv4Pi * Lam[i] + (s == rb.t ? Ed[i] : 0.0));
        }
        lBq += Lam[i] * (-Qp * kInv4Pi / R.eps);
      }
      dkap[p] = 0.5 * C * (qSx - lAx + lBq);
    }
  }
  // restore the forward outputs of x (phi_reac on the device)
  rc = apply_operator(pl, st, x, wsp<double>(pl, pl.o_phi_reac), PBTC_FP64, 1);
  if (rc) return rc;
  PBTC_HIP(hipStreamSynchronize(st));
  if (dk)
    for (int p = 0; p < pl.nreg; ++p) dk[p] = gE * dkap[p];
  if (de)
    for (int p = 0; p < pl.nreg; ++p) de[p] = gE * deps[p];
  if (res) {
    res->energy_kJmol = pl.energy;
    res->n_iter = iters;
    res->converged = conv ? 1 : 0;
    res->final_rel_res = rel;
    res->n_matvec_fp32 = n32;
    res->n_matvec_fp64 = n64;
    res->n_refine = nref;
    prof_collect(pl);
    for (int k = 0; k < kProfKinds; ++k) {
      res->t_kernel_s[k] = pl.prof_t[k];
      res->n_kernel_launch[k] = pl.prof_n[k];
      res->kernel_flop[k] = pl.prof_flop[k];
    }
  }
  pl.adj_history = hist;
  if (!conv) {
    pl.err = "adjoint GMRES did not reach the tolerance within max_iter";
    return PBTC_ENOCONV;
  }
  return PBTC_OK;
}


}  // namespace pbtc
