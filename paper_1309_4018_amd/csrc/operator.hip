// One evaluation of the BEM operator by the treecode (sec. 2.3).
//
// The matrix-vector product is an N-body sum (Eq. nbody) whose sources are
// the Gauss points of every panel weighted by the panel unknowns and whose
// targets are the collocation points (sec. 2.3, treecode-accelerated BEM).
// For every block (target set t, source surface s) and each of its Green's
// functions G the kernels accumulate, at every target x,
//   S(x) = sum_y W_y psi_j(y) G(x, y)           (single layer, V psi)
//   D(x) = sum_y W_y phi_j(y) n_j . grad_y G(x, y)  (double layer, K phi)
// with G = 1/(4 pi R) or exp(-kappa R)/(4 pi R) (Eq. nBEM, Eq. matel):
//   prep      source records (y, W psi, W phi n) from the unknown vector
//   p2m, m2m  moments of every cell: P2M at the leaves, shifted to the
//             parents (sec. 2.3: moments formed at the twigs, then shifted
//             and added upward)
//   p2p       direct sums over the cells of a group's near list (R = 0
//             pairs -- a target on its own centroid Gauss point -- skipped)
//   m2p       Taylor coefficients by recurrence contracted with the cell
//             moments (Eq. multexp) over the group's far list
//   near      FP64-built corrections for the self and near-singular panels
//   combine   1/2 phi_t - sum_s sigma_rs (c_rs S - D) per row block
#include <algorithm>
#include <cmath>

#include "device_util.h"
#include "kernel_common.h"
#include "taylor.h"

namespace pbtc {

namespace {

// ------------------------------------------------------------------- prep
template <typename real>
__global__ void k_prep(int64_t ngp, const double* __restrict__ gx, const double* __restrict__ gy,
                       const double* __restrict__ gz, const double* __restrict__ gw,
                       const int* __restrict__ gpid, const int* __restrict__ pidx,
                       const double* __restrict__ nx, const double* __restrict__ ny,
                       const double* __restrict__ nz, const double* __restrict__ x,
                       Src<real>* __restrict__ src) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ngp) return;
  const int p = gpid[j];
  const double w = gw[j];
  const double phi = x[pidx[2 * p]], psi = x[pidx[2 * p + 1]];
  Src<real> s;
  s.x = (real)gx[j];
  s.y = (real)gy[j];
  s.z = (real)gz[j];
  s.q = (real)(w * psi);
  s.px = (real)(w * phi * nx[p]);
  s.py = (real)(w * phi * ny[p]);
  s.pz = (real)(w * phi * nz[p]);
  s.pad = (real)0;
  src[j] = s;
}

// ------------------------------------------------------------- moments
// Moments of every cell about its centre c (Eq. multexp):
//   M_SL[k] = sum q (y - c)^k,   M_DL[k] = sum_d p_d k_d (y - c)^(k - e_d).
// A span root is a cell of at most kSpanSources sources whose parent has more
// (or a tree root that small); every cell of a span root's subtree takes one
// work-group that computes its moments directly from its own (Morton-
// contiguous) sources, staged through LDS kMomChunk at a time.  The work-
// groups of one span are consecutive in a list that is dealt to the XCDs in
// contiguous runs, so that a span's sources come from HBM once and from that
// XCD's L2 for the deeper cells.  The larger (upper) cells follow level by
// level, bottom-up: each adds its children's moments shifted to its own
// centre by the multi-index binomial theorem (sec. 2.3: moments shifted to
// the parents and added),
//   (y - c_u)^k = sum_{j <= k} C(k, j) h^(k - j) (y - c_s)^j,   h = c_s - c_u,
// which holds for both moment kinds (the double layer is a linear map of the
// same monomials), so upper cells never re-read the sources.
constexpr int kMomThreads = 256;

template <typename real, int P>
__global__ __launch_bounds__(kMomThreads) void k_p2m_cell(const int4* __restrict__ chunks,
                                                          const Cell* __restrict__ cells,
                                                          const Src<real>* __restrict__ src,
                                                          real* __restrict__ mom) {
  constexpr int N = ncoef(P);
  constexpr int G = N <= kMomThreads ? kMomThreads / N : 1;  // groups of sources
  constexpr int KPT = (N + kMomThreads - 1) / kMomThreads;   // coefficients per thread
  static_assert(kMomChunk <= kMomThreads, "one source per thread while staging");
  __shared__ real pw[kMomChunk][3][P + 1];
  __shared__ real sq[kMomChunk][4];
  __shared__ real red[G][2 * N];
  const int4 ch = chunks[xcd_block(blockIdx.x, gridDim.x)];  // (cell, first source, count)
  const Cell& cl = cells[ch.x];
  const real cx = (real)cl.cx, cy = (real)cl.cy, cz = (real)cl.cz;
  const int tid = threadIdx.x;
  const int g = N <= kMomThreads ? tid / N : 0;
  int kk[KPT][3];
  bool on[KPT];
  real ms[KPT], md[KPT];
#pragma unroll
  for (int q = 0; q < KPT; ++q) {
    const int k = N <= kMomThreads ? tid - g * N : tid + q * kMomThreads;
    on[q] = N <= kMomThreads ? tid < G * N : k < N;
    mindex_inv(on[q] ? k : 0, kk[q][0], kk[q][1], kk[q][2]);
    ms[q] = md[q] = 0;
  }
  Src<real> nxt;
  if (tid < min(kMomChunk, ch.z)) nxt = src[ch.y + tid];
  for (int b0 = 0; b0 < ch.z; b0 += kMomChunk) {
    const int nj = min(kMomChunk, ch.z - b0);
    if (tid < nj) {
      const Src<real> s = nxt;
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
      sq[tid][0] = s.q;
      sq[tid][1] = s.px;
      sq[tid][2] = s.py;
      sq[tid][3] = s.pz;
    }
    __syncthreads();
    // the next batch is loaded while this one is used
    if (b0 + kMomChunk + tid < ch.z && tid < kMomChunk) nxt = src[ch.y + b0 + kMomChunk + tid];
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      if (!on[q]) continue;
      const int k1 = kk[q][0], k2 = kk[q][1], k3 = kk[q][2];
      auto term = [&](int t, real& s_acc, real& d_acc) {
        const real X = pw[t][0][k1], Y = pw[t][1][k2], Z = pw[t][2][k3];
        s_acc += sq[t][0] * X * Y * Z;
        real dl = 0;
        if (k1) dl += sq[t][1] * real(k1) * pw[t][0][k1 - 1] * Y * Z;
        if (k2) dl += sq[t][2] * real(k2) * X * pw[t][1][k2 - 1] * Z;
        if (k3) dl += sq[t][3] * real(k3) * X * Y * pw[t][2][k3 - 1];
        d_acc += dl;
      };
      // four sources per step into independent sums, so that their LDS
      // reads are in flight together
      real s4[4] = {0, 0, 0, 0}, d4[4] = {0, 0, 0, 0};
      int t = g;
      for (; t + 3 * G < nj; t += 4 * G) {
#pragma unroll
        for (int u = 0; u < 4; ++u) term(t + u * G, s4[u], d4[u]);
      }
      for (; t < nj; t += G) term(t, s4[0], d4[0]);
      ms[q] += (s4[0] + s4[1]) + (s4[2] + s4[3]);
      md[q] += (d4[0] + d4[1]) + (d4[2] + d4[3]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < KPT; ++q) {
    if (!on[q]) continue;
    const int k = N <= kMomThreads ? tid - g * N : tid + q * kMomThreads;
    red[g][k] = ms[q];
    red[g][N + k] = md[q];
  }
  __syncthreads();
  for (int k = tid; k < 2 * N; k += kMomThreads) {
    real v = 0;
#pragma unroll
    for (int gg = 0; gg < G; ++gg) v += red[gg][k];
    mom[(size_t)ch.x * 2 * N + k] = v;
  }
}

// binomial coefficients C(n, k), n, k <= kMaxP
struct Binom {
  int c[kMaxP + 1][kMaxP + 1];
  constexpr Binom() : c() {
    for (int n = 0; n <= kMaxP; ++n) {
      c[n][0] = 1;
      for (int k = 1; k <= n; ++k) c[n][k] = c[n - 1][k - 1] + (k <= n - 1 ? c[n - 1][k] : 0);
    }
  }
};
__constant__ Binom kBinom = Binom();

// Moments of the upper cells of one tree level (bottom-up, one launch per
// level): a cell's moments are the sum of its children's (span cells or upper
// cells of the level below, both final), each shifted to the cell's centre.
// The children's moments, the powers of their offsets h and the binomials are
// staged in LDS; one thread per output coefficient walks its terms
// j <= k in one flat loop (the lanes of a wave differ in k, so nested loops
// over (j1, j2, j3) would run the union of their bounds).
template <typename real, int P>
__global__ __launch_bounds__(256) void k_m2m_up(const int* __restrict__ ucells,
                                                const Cell* __restrict__ cells,
                                                real* __restrict__ mom) {
  constexpr int N = ncoef(P), N2 = 2 * N;
  __shared__ real sm[8][N2];
  __shared__ real hp[8][3][P + 1];
  __shared__ real bin[P + 1][P + 1];
  const int u = ucells[blockIdx.x];
  const Cell& cu = cells[u];
  const int nch = cu.nchild, c0 = cu.child;
  const int tid = threadIdx.x;
  for (int i = tid; i < nch * N2; i += 256) {
    const int r = i / N2, k = i - r * N2;
    sm[r][k] = mom[(size_t)(c0 + r) * N2 + k];
  }
  if (tid < 3 * nch) {
    const int r = tid / 3, d = tid - 3 * r;
    const Cell& ch = cells[c0 + r];
    const double h = d == 0 ? ch.cx - cu.cx : d == 1 ? ch.cy - cu.cy : ch.cz - cu.cz;
    real v = 1;
    for (int e = 0; e <= P; ++e) {
      hp[r][d][e] = v;
      v *= (real)h;
    }
  }
  for (int i = tid; i < (P + 1) * (P + 1); i += 256)
    bin[i / (P + 1)][i % (P + 1)] = real(kBinom.c[i / (P + 1)][i % (P + 1)]);
  __syncthreads();
  for (int k = tid; k < N2; k += 256) {
    int a, b, c;
    mindex_inv(k < N ? k : k - N, a, b, c);
    const int half = k < N ? 0 : N;
    const int nt = (a + 1) * (b + 1) * (c + 1);
    real acc = 0;
    for (int r = 0; r < nch; ++r) {
      const real* M = sm[r] + half;
      real s = 0;
      int j1 = 0, j2 = 0, j3 = 0;
      for (int t = 0; t < nt; ++t) {
        s += (bin[a][j1] * hp[r][0][a - j1]) * (bin[b][j2] * hp[r][1][b - j2]) *
             (bin[c][j3] * hp[r][2][c - j3]) * M[mindex(j1, j2, j3)];
        // next (j1, j2, j3), j3 fastest
        const bool w3 = j3 == c, w2 = w3 && j2 == b;
        j3 = w3 ? 0 : j3 + 1;
        j2 = w2 ? 0 : (w3 ? j2 + 1 : j2);
        j1 = w2 ? j1 + 1 : j1;
      }
      acc += s;
    }
    mom[(size_t)u * N2 + k] = acc;
  }
}

// ------------------------------------------------------------------- p2p
// Work is split into wavefront units: a unit is one target group (64
// targets, one per lane) and a run of its list entries.  The four waves of a
// work-group take four independent units; every index a wave loops over is
// made wave-uniform so that sources and moments come through scalar loads.
// Each unit writes its partial sums; a second kernel adds the units of an
// item in a fixed order (deterministic) and stores S and D.
constexpr int kItemThreads = 256;
constexpr int kWaves = kItemThreads / 64;

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// One (target, source) pair: single and double layer of the block's kernels.
// k0, k1: kappa of kernel slots 0 / 1; a0, a1 = exp_arg(k0), exp_arg(k1).
template <typename real, int KS>
__device__ __forceinline__ void pair(real x, real y, real z, const Src<real>& s, real k0, real k1,
                                     real a0, real a1, real (&acc)[4]) {
  const real dx = x - s.x, dy = y - s.y, dz = z - s.z;
  const real r2 = dx * dx + dy * dy + dz * dz;
  const real rinv = r2 > real(0) ? rsqrt_(r2) : real(0);
  const real pd = s.px * dx + s.py * dy + s.pz * dz;
  const real t = rinv * rinv;
  if (KS == KS_L || KS == KS_LY) {
    acc[0] += s.q * rinv;
    acc[1] += pd * (t * rinv);
  }
  // Yukawa double layer: pd e (1 + kappa r) / r^3 = pd (e / r) (1/r^2 + kappa / r)
  if (KS == KS_Y || KS == KS_LY || KS == KS_YY) {
    const real kap = KS == KS_LY ? k1 : k0;
    const real ea = KS == KS_LY ? a1 : a0;
    const real r = r2 * rinv;
    const real er = exp_scaled(ea * r) * rinv;
    const int o = KS == KS_LY ? 2 : 0;
    acc[o] += s.q * er;
    acc[o + 1] += pd * (er * (kap * rinv + t));
  }
  if (KS == KS_YY) {
    const real r = r2 * rinv;
    const real er = exp_scaled(a1 * r) * rinv;
    acc[2] += s.q * er;
    acc[3] += pd * (er * (k1 * rinv + t));
  }
}

template <int KS>
constexpr int nacc() {
  return KS == KS_L || KS == KS_Y ? 2 : 4;
}

// partial[(u * 4 + q) * 64 + lane]
template <typename real, int NQ>
__device__ __forceinline__ void unit_store(real* __restrict__ partial, int u, const real (&acc)[4]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < NQ; ++q) partial[((size_t)u * 4 + q) * 64 + lane] = acc[q];
}

template <typename real, int KS>
__global__ __launch_bounds__(kItemThreads) void k_p2p(UnitArgs a, const real* __restrict__ tx,
                                                      const real* __restrict__ ty,
                                                      const real* __restrict__ tz,
                                                      const Src<real>* __restrict__ src,
                                                      real* __restrict__ partial) {
  const int u = uni(xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6));
  if (u >= a.nunits) return;
  const int4 un = a.units[u];
  const int item = uni(un.x), e0 = uni(un.y), e1 = uni(un.z);
  const DevBlock& b = a.blocks[uni(a.item_block[item])];
  const long long g = item - b.item_off;
  const long long t0 = b.tgt_off + g * kGroup;
  const int nt = (int)min((long long)kGroup, b.ntgt - g * kGroup);
  const int lane = threadIdx.x & 63;
  const long long ti = t0 + min(lane, nt - 1);
  const real x = tx[ti], y = ty[ti], z = tz[ti];
  const real k0 = (real)b.kappa0, k1 = (real)b.kappa1;
  const real a0 = exp_arg(k0), a1 = exp_arg(k1);
  real acc[4] = {0, 0, 0, 0};
  for (int e = e0; e < e1; ++e) {
    const int c = uni(a.cells_list[e]);
    const int beg = uni(a.cells[c].begin), end = beg + uni(a.cells[c].count);
    int j = beg;
    // four sources per step: their scalar loads are issued together
    for (; j + 3 < end; j += 4) {
      const Src<real> s0 = src[j], s1 = src[j + 1], s2 = src[j + 2], s3 = src[j + 3];
      pair<real, KS>(x, y, z, s0, k0, k1, a0, a1, acc);
      pair<real, KS>(x, y, z, s1, k0, k1, a0, a1, acc);
      pair<real, KS>(x, y, z, s2, k0, k1, a0, a1, acc);
      pair<real, KS>(x, y, z, s3, k0, k1, a0, a1, acc);
    }
    for (; j < end; ++j) {
      const Src<real> s0 = src[j];
      pair<real, KS>(x, y, z, s0, k0, k1, a0, a1, acc);
    }
  }
  unit_store<real, nacc<KS>()>(partial, u, acc);
}

// ------------------------------------------------------------------- m2p
// One Green's function per launch (KIND 0 Laplace, 1 Yukawa) for the block's
// kernel slot `slot`, so that the two recurrences of a Laplace + Yukawa
// block never share a register allocation.
template <typename real, int P, int KIND>
__global__ __launch_bounds__(kItemThreads) void k_m2p(UnitArgs a, const real* __restrict__ tx,
                                                      const real* __restrict__ ty,
                                                      const real* __restrict__ tz,
                                                      const real* __restrict__ mom, int slot,
                                                      real* __restrict__ partial) {
  constexpr int N = ncoef(P);
  const int u = uni(xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6));
  if (u >= a.nunits) return;
  const int4 un = a.units[u];
  const int item = uni(un.x), e0 = uni(un.y), e1 = uni(un.z);
  const DevBlock& b = a.blocks[uni(a.item_block[item])];
  const long long g = item - b.item_off;
  const long long t0 = b.tgt_off + g * kGroup;
  const int nt = (int)min((long long)kGroup, b.ntgt - g * kGroup);
  const int lane = threadIdx.x & 63;
  const long long ti = t0 + min(lane, nt - 1);
  const real x = tx[ti], y = ty[ti], z = tz[ti];
  const real kap = (real)(slot == 0 ? b.kappa0 : b.kappa1);
  // The cell's moments go through a per-wavefront LDS slice (broadcast
  // reads), double-buffered: the next cell's moments and centre are loaded
  // into registers while the current cell is evaluated.
  constexpr int PER = (2 * N + 63) / 64;
  __shared__ real smom[kWaves][2][2 * N];
  const int wv = uni(threadIdx.x >> 6);
  real pre[PER];
  double pcx = 0, pcy = 0, pcz = 0;
  auto fetch = [&](int e) {
    const int c = uni(a.cells_list[e]);
    const Cell& cl = a.cells[c];
    pcx = cl.cx;
    pcy = cl.cy;
    pcz = cl.cz;
    const real* Mg = mom + (size_t)c * 2 * N;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int k = lane + 64 * q;
      pre[q] = k < 2 * N ? Mg[k] : real(0);
    }
  };
  real acc[4] = {0, 0, 0, 0};
  if (e0 < e1) fetch(e0);
  int buf = 0;
  for (int e = e0; e < e1; ++e) {
    real* M = smom[wv][buf];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int k = lane + 64 * q;
      if (k < 2 * N) M[k] = pre[q];
    }
    const real dx = x - (real)pcx, dy = y - (real)pcy, dz = z - (real)pcz;
    wave_sync();  // this buffer is written; the other one was last read a cell ago
    if (e + 1 < e1) fetch(e + 1);
    const real r2 = dx * dx + dy * dy + dz * dz;
    const real rinv = rsqrt_(r2);
    if (KIND == 0)
      taylor_laplace<P, real>(dx, dy, dz, rinv, M, acc[0], acc[1]);
    else
      taylor_yukawa<P, real>(dx, dy, dz, rinv, exp_neg(kap * (r2 * rinv)), kap, M, acc[0], acc[1]);
    buf ^= 1;
  }
  unit_store<real, 2>(partial, u, acc);
}

// Sum of the units of every listed item, times 1/(4 pi), into S and D of
// kernel slots first_slot.. (mode 0 store, mode 1 add).  The four waves of
// the work-group take the item's units round-robin (wave w: units w, w + 4,
// ...), so that four times as many loads are in flight; their sums are then
// added in wave order (fixed order: deterministic).
constexpr int kReduceWaves = 4;

template <typename real, int NQ>
__global__ __launch_bounds__(64 * kReduceWaves) void k_reduce(
    const int* __restrict__ list, const int* __restrict__ uptr, const int* __restrict__ item_block,
    const DevBlock* __restrict__ blocks, const int* __restrict__ tidx,
    const real* __restrict__ partial, double* __restrict__ S, double* __restrict__ D, int mode,
    int first_slot) {
  __shared__ double lds[kReduceWaves - 1][NQ][64];
  const int l = blockIdx.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  const int u0 = uptr[l], u1 = uptr[l + 1];
  int u = u0 + w;
  // two units per step per wave
  for (; u + kReduceWaves < u1; u += 2 * kReduceWaves) {
    real p[2][NQ];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        p[k][q] = partial[((size_t)(u + k * kReduceWaves) * 4 + q) * 64 + lane];
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] += (double)p[0][q] + (double)p[1][q];
  }
  if (u < u1)
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] += (double)partial[((size_t)u * 4 + q) * 64 + lane];
  if (w > 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds[w - 1][q][lane] = v[q];
  __syncthreads();
  if (w > 0) return;
  const int item = list[l];
  const DevBlock& b = blocks[item_block[item]];
  const long long g = item - b.item_off;
  const long long t0 = b.tgt_off + g * kGroup;
  const int nt = (int)min((long long)kGroup, b.ntgt - g * kGroup);
  if (lane >= nt) return;
#pragma unroll
  for (int k = 0; k < kReduceWaves - 1; ++k)
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] += lds[k][q][lane];
  const long long i = tidx[t0 + lane] - b.tgt_off;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const long long out = (first_slot + (q >> 1) == 0 ? b.out0 : b.out1) + i;
    double* dst = (q & 1) ? D : S;
    const double val = v[q] * kInv4Pi;
    if (mode == 0)
      dst[out] = val;
    else
      dst[out] += val;
  }
}

// ----------------------------------------------------------- near field
// S[out_k + i] += sum_e dV_k(e) psi(col), D[out_k + i] += sum_e dK_k(e) phi(col)
// kNearLanes consecutive lanes share a row and stride over its entries, so a
// wavefront's loads of the entry values are contiguous; a fixed butterfly adds
// the lanes' sums.
constexpr int kNearLanes = 4;

template <typename real>
__device__ __forceinline__ void load_near4(const real* __restrict__ v, real& a, real& b, real& c,
                                           real& d);
template <>
__device__ __forceinline__ void load_near4<float>(const float* __restrict__ v, float& a, float& b,
                                                  float& c, float& d) {
  const float4 q = *reinterpret_cast<const float4*>(v);
  a = q.x;
  b = q.y;
  c = q.z;
  d = q.w;
}
template <>
__device__ __forceinline__ void load_near4<double>(const double* __restrict__ v, double& a,
                                                   double& b, double& c, double& d) {
  const double2 q0 = *reinterpret_cast<const double2*>(v);
  const double2 q1 = *reinterpret_cast<const double2*>(v + 2);
  a = q0.x;
  b = q0.y;
  c = q1.x;
  d = q1.y;
}

template <typename real>
__global__ void k_near_apply(long long r0, long long r1, const int* __restrict__ row_block,
                             const DevBlock* __restrict__ blocks, const long long* __restrict__ ptr,
                             const int* __restrict__ col, const real* __restrict__ val,
                             const int* __restrict__ pidx, const double* __restrict__ x,
                             double* __restrict__ S, double* __restrict__ D) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long row = r0 + gid / kNearLanes;
  const int sub = (int)(gid % kNearLanes);
  const bool live = row < r1;
  real s0 = 0, d0 = 0, s1 = 0, d1 = 0;
  int nk = 1;
  if (live) {
    nk = blocks[row_block[row]].nk;
    const long long e1 = ptr[row + 1];
    for (long long e = ptr[row] + sub; e < e1; e += kNearLanes) {
      const int p = col[e];
      const real phi = (real)x[pidx[2 * p]], psi = (real)x[pidx[2 * p + 1]];
      real v0, v1, v2, v3;
      load_near4<real>(val + 4 * e, v0, v1, v2, v3);
      s0 += v0 * psi;
      d0 += v1 * phi;
      if (nk == 2) {
        s1 += v2 * psi;
        d1 += v3 * phi;
      }
    }
  }
#pragma unroll
  for (int o = 1; o < kNearLanes; o <<= 1) {
    s0 += __shfl_xor(s0, o, 64);
    d0 += __shfl_xor(d0, o, 64);
    s1 += __shfl_xor(s1, o, 64);
    d1 += __shfl_xor(d1, o, 64);
  }
  if (!live || sub != 0) return;
  const DevBlock& b = blocks[row_block[row]];
  const long long i = row - b.nf_row;
  S[b.out0 + i] += (double)s0;
  D[b.out0 + i] += (double)d0;
  if (nk == 2) {
    S[b.out1 + i] += (double)s1;
    D[b.out1 + i] += (double)d1;
  }
}

// ------------------------------------------------------------- combine
__global__ void k_combine(const DevRowBlock* __restrict__ rows, const DevRowTerm* __restrict__ terms,
                          const double* __restrict__ x, const double* __restrict__ S,
                          const double* __restrict__ D, double* __restrict__ y) {
  const DevRowBlock rb = rows[blockIdx.y];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rb.n) return;
  double acc = 0.0;
  for (int t = rb.term_off; t < rb.term_off + rb.nterms; ++t) {
    const DevRowTerm tm = terms[t];
    acc += tm.sigma_c * S[tm.out + i] - tm.sigma * D[tm.out + i];
  }
  y[rb.row_off + i] = rb.half * (rb.half != 0.0 ? x[rb.phi_off + i] : 0.0) + rb.sign * acc;
}

}  // namespace

// ------------------------------------------------------------ host side
template <typename real>
static int launch_moments(pbtc_plan_t& pl, hipStream_t st, real* mom, const Src<real>* src) {
  const Cell* cells = wsp<Cell>(pl, pl.o_cells);
  const int4* chunks = wsp<int4>(pl, pl.o_mchunks);
  const int* ucells = wsp<int>(pl, pl.o_mcell);
  const unsigned nch = (unsigned)pl.n_mchunks;
#define PBTC_MOM(PP)                                                                          \
  case PP:                                                                                    \
    if (nch > 0)                                                                              \
      hipLaunchKernelGGL((k_p2m_cell<real, PP>), dim3(nch), dim3(kMomThreads), 0, st, chunks, \
                         cells, src, mom);                                                    \
    for (size_t l = 0; l + 1 < pl.up_level.size(); ++l)                                       \
      if (pl.up_level[l + 1] > pl.up_level[l])                                                \
        hipLaunchKernelGGL((k_m2m_up<real, PP>), dim3(pl.up_level[l + 1] - pl.up_level[l]),   \
                           dim3(256), 0, st, ucells + pl.up_level[l], cells, mom);            \
    break;
  switch (pl.P) {
    PBTC_MOM(2)
    PBTC_MOM(4)
    PBTC_MOM(6)
    PBTC_MOM(8)
    PBTC_MOM(10)
    default:
      pl.err = "unsupported P";
      return PBTC_EINVAL;
  }
#undef PBTC_MOM
  PBTC_LAUNCH_CHECK();
  return PBTC_OK;
}

template <typename real, int KIND>
static void launch_m2p(pbtc_plan_t& pl, hipStream_t st, const UnitArgs& a, int grid, const real* tx,
                       const real* ty, const real* tz, const real* mom, int slot, real* partial) {
#define PBTC_M2P(PP)                                                                           \
  case PP:                                                                                     \
    hipLaunchKernelGGL((k_m2p<real, PP, KIND>), dim3(grid), dim3(kItemThreads), 0, st, a, tx, ty, \
                       tz, mom, slot, partial);                                                \
    break;
  switch (pl.P) {
    PBTC_M2P(2)
    PBTC_M2P(4)
    PBTC_M2P(6)
    PBTC_M2P(8)
    PBTC_M2P(10)
    default:
      break;
  }
#undef PBTC_M2P
}

// Timing of one kernel launch (kind 0 P2P, 1 Laplace M2P, 2 Yukawa M2P of
// A x; 3, 4, 5 of A^T x) with events on the launch stream; only FP32
// operator evaluations are timed.
void prof_mark(pbtc_plan_t& pl, hipStream_t st, bool on, int kind, double flop, bool begin) {
  if (!pl.prm.profile || !on) return;
  if (begin) {
    pbtc_plan_t::ProfEvent ev;
    if (!pl.prof_pool.empty()) {
      ev = pl.prof_pool.back();
      pl.prof_pool.pop_back();
    } else if (hipEventCreate(&ev.a) != hipSuccess) {
      return;  // profiling is best effort: no event, no sample
    } else if (hipEventCreate(&ev.b) != hipSuccess) {
      (void)hipEventDestroy(ev.a);
      return;
    }
    ev.kind = kind;
    ev.flop = flop;
    ev.recorded = hipEventRecord(ev.a, st) == hipSuccess;
    pl.prof.push_back(ev);
  } else if (!pl.prof.empty()) {
    pbtc_plan_t::ProfEvent& ev = pl.prof.back();
    ev.recorded = ev.recorded && hipEventRecord(ev.b, st) == hipSuccess;
  }
}

// y = A x (phase 0) or phi_reac = S x (phase 1) in precision `prec`.
// capture: the launches are being recorded into a launch graph (no timing
// events, the moment pass always on the side stream).
template <typename real>
static int apply_impl(pbtc_plan_t& pl, hipStream_t st, const double* x, double* y, int phase,
                      bool capture = false) {
  const int T = 256;
  Src<real>* src = wsp<Src<real>>(pl, sizeof(real) == 4 ? pl.o_src32 : pl.o_src64);
  real* mom = wsp<real>(pl, sizeof(real) == 4 ? pl.o_mom32 : pl.o_mom64);
  const real* tx = wsp<real>(pl, sizeof(real) == 4 ? pl.o_txf : pl.o_tx);
  const real* ty = wsp<real>(pl, sizeof(real) == 4 ? pl.o_tyf : pl.o_ty);
  const real* tz = wsp<real>(pl, sizeof(real) == 4 ? pl.o_tzf : pl.o_tz);
  hipLaunchKernelGGL(k_prep<real>, dim3(nblocks(pl.ngp, T)), dim3(T), 0, st, pl.ngp,
                     wsp<double>(pl, pl.o_gx), wsp<double>(pl, pl.o_gy), wsp<double>(pl, pl.o_gz),
                     wsp<double>(pl, pl.o_gw), wsp<int>(pl, pl.o_gpid), wsp<int>(pl, pl.o_pidx),
                     wsp<double>(pl, pl.o_nx), wsp<double>(pl, pl.o_ny), wsp<double>(pl, pl.o_nz), x,
                     src);
  PBTC_LAUNCH_CHECK();
  const bool tree = pl.prm.op == PBTC_OP_TREECODE;
  bool timed = false;
  if (sizeof(real) == 4 && phase == 0 && pl.prm.profile > 0 && !capture)
    timed = pl.prof_count++ % pl.prm.profile == 0;
  // the moment pass (latency-bound) runs on a second stream beside the
  // P2P launches (ALU-bound); M2P waits for it.  A sampled (timed)
  // evaluation runs it first instead, so that each timed launch has the GPU
  // to itself.
  const bool fork = tree && pl.n_far > 0 && !timed;
  if (fork) {
    if (!pl.side) {
      PBTC_HIP(hipStreamCreateWithFlags(&pl.side, hipStreamNonBlocking));
      PBTC_HIP(hipEventCreateWithFlags(&pl.ev_fork, hipEventDisableTiming));
      PBTC_HIP(hipEventCreateWithFlags(&pl.ev_join, hipEventDisableTiming));
    }
    PBTC_HIP(hipEventRecord(pl.ev_fork, st));
    PBTC_HIP(hipStreamWaitEvent(pl.side, pl.ev_fork, 0));
    int rc = launch_moments<real>(pl, pl.side, mom, src);
    if (rc) return rc;
    PBTC_HIP(hipEventRecord(pl.ev_join, pl.side));
  } else if (tree) {
    int rc = launch_moments<real>(pl, st, mom, src);
    if (rc) return rc;
  }
  bool joined = !fork;
  UnitArgs a;
  a.item_block = wsp<int>(pl, pl.o_items);
  a.blocks = wsp<DevBlock>(pl, pl.o_blocks);
  a.cells = wsp<Cell>(pl, pl.o_cells);
  const int* tidx = wsp<int>(pl, pl.o_tidx);
  double* S = wsp<double>(pl, pl.o_S);
  double* D = wsp<double>(pl, pl.o_D);
  real* partial = wsp<real>(pl, pl.o_partial);
  for (int ks = 0; ks < KS_COUNT; ++ks) {
    const int n = (int)pl.item_list[phase][ks].size();
    if (n == 0) continue;
    const int* list = wsp<int>(pl, pl.o_item_list[phase][ks]);
    // P2P over the near lists
    {
      const UnitSet& us = pl.units[phase][ks][0];
      a.units = wsp<int4>(pl, pl.o_units + 16 * us.off);
      a.nunits = (int)us.n;
      a.cells_list = wsp<int>(pl, pl.o_near);
      const int grid = nblocks(us.n, kWaves);
      prof_mark(pl, st, timed, 0, pl.launch_flop_p2p[phase][ks], true);
      // no units (every cell seen through its expansion): the reduction
      // below still stores the zero P2P sums
      if (grid > 0) switch (ks) {
        case KS_L:
          hipLaunchKernelGGL((k_p2p<real, KS_L>), dim3(grid), dim3(kItemThreads), 0, st, a, tx, ty, tz, src, partial);
          break;
        case KS_Y:
          hipLaunchKernelGGL((k_p2p<real, KS_Y>), dim3(grid), dim3(kItemThreads), 0, st, a, tx, ty, tz, src, partial);
          break;
        case KS_LY:
          hipLaunchKernelGGL((k_p2p<real, KS_LY>), dim3(grid), dim3(kItemThreads), 0, st, a, tx, ty, tz, src, partial);
          break;
        case KS_YY:
          hipLaunchKernelGGL((k_p2p<real, KS_YY>), dim3(grid), dim3(kItemThreads), 0, st, a, tx, ty, tz, src, partial);
          break;
      }
      prof_mark(pl, st, timed, 0, 0.0, false);
      const int* uptr = wsp<int>(pl, pl.o_uptr + 4 * us.ptr_off);
      if (ks == KS_L || ks == KS_Y)
        hipLaunchKernelGGL((k_reduce<real, 2>), dim3(n), dim3(64 * kReduceWaves), 0, st, list,
                           uptr, a.item_block, a.blocks, tidx, partial, S, D, 0, 0);
      else
        hipLaunchKernelGGL((k_reduce<real, 4>), dim3(n), dim3(64 * kReduceWaves), 0, st, list,
                           uptr, a.item_block, a.blocks, tidx, partial, S, D, 0, 0);
      PBTC_LAUNCH_CHECK();
    }
    if (tree && pl.n_far > 0) {
      const UnitSet& us = pl.units[phase][ks][1];
      if (us.n == 0) continue;
      if (!joined) {
        PBTC_HIP(hipStreamWaitEvent(st, pl.ev_join, 0));
        joined = true;
      }
      a.units = wsp<int4>(pl, pl.o_units + 16 * us.off);
      a.nunits = (int)us.n;
      a.cells_list = wsp<int>(pl, pl.o_far);
      const int grid = nblocks(us.n, kWaves);
      const int* uptr = wsp<int>(pl, pl.o_uptr + 4 * us.ptr_off);
      // kernel of slot 0 and (for two-kernel blocks) slot 1
      const int kind0 = (ks == KS_L || ks == KS_LY) ? 0 : 1;
      const bool two = ks == KS_LY || ks == KS_YY;
      for (int slot = 0; slot < (two ? 2 : 1); ++slot) {
        const int kind = slot == 0 ? kind0 : 1;
        // this kernel's share of the block's M2P operations
        const double fl = pl.launch_flop_m2p[phase][ks] * m2p_flop_one(pl.P, kind) /
                          m2p_flop_per_eval(pl.P, ks);
        prof_mark(pl, st, timed, 1 + kind, fl, true);
        if (kind == 0)
          launch_m2p<real, 0>(pl, st, a, grid, tx, ty, tz, mom, slot, partial);
        else
          launch_m2p<real, 1>(pl, st, a, grid, tx, ty, tz, mom, slot, partial);
        prof_mark(pl, st, timed, 1 + kind, 0.0, false);
        hipLaunchKernelGGL((k_reduce<real, 2>), dim3(n), dim3(64 * kReduceWaves), 0, st, list,
                           uptr, a.item_block, a.blocks, tidx, partial, S, D, 1, slot);
      }
      PBTC_LAUNCH_CHECK();
    }
  }
  if (!joined) PBTC_HIP(hipStreamWaitEvent(st, pl.ev_join, 0));  // no far field in this phase
  // near-field corrections of this phase's blocks
  const long long r0 = phase == 0 ? 0 : pl.nf_fwd_rows;
  const long long r1 = phase == 0 ? pl.nf_fwd_rows : pl.nf_rows;
  if (r1 > r0) {
    hipLaunchKernelGGL(k_near_apply<real>, dim3(nblocks((r1 - r0) * kNearLanes, T)), dim3(T), 0, st,
                       r0, r1,
                       wsp<int>(pl, pl.o_nf_rowblk), wsp<DevBlock>(pl, pl.o_blocks),
                       wsp<long long>(pl, pl.o_nf_ptr), wsp<int>(pl, pl.o_nf_col),
                       wsp<real>(pl, sizeof(real) == 4 ? pl.o_nf_v32 : pl.o_nf_v64),
                       wsp<int>(pl, pl.o_pidx), x, S, D);
    PBTC_LAUNCH_CHECK();
  }
  // combine
  const auto& rows = phase == 0 ? pl.rows : pl.reac_rows;
  if (!rows.empty()) {
    int64_t nmax = 0;
    for (const auto& r : rows) nmax = std::max(nmax, r.n);
    dim3 grid(nblocks(nmax, T), (unsigned)rows.size());
    hipLaunchKernelGGL(k_combine, grid, dim3(T), 0, st,
                       wsp<DevRowBlock>(pl, phase == 0 ? pl.o_rows : pl.o_reac_rows),
                       wsp<DevRowTerm>(pl, phase == 0 ? pl.o_terms : pl.o_reac_terms), x, S, D,
                       y);
    PBTC_LAUNCH_CHECK();
  }
  return PBTC_OK;
}

// Folds finished profiling events into the plan's totals (stream synchronised).
void prof_collect(pbtc_plan_t& pl) {
  for (auto& ev : pl.prof) {
    float ms = 0.0f;
    if (ev.recorded && hipEventElapsedTime(&ms, ev.a, ev.b) == hipSuccess) {
      pl.prof_t[ev.kind] += 1e-3 * ms;
      pl.prof_n[ev.kind] += 1;
      pl.prof_flop[ev.kind] += ev.flop;
    }
    pl.prof_pool.push_back(ev);
  }
  pl.prof.clear();
}

void release_op_graphs(pbtc_plan_t& pl) {
  for (int p = 0; p < 2; ++p)
    for (int ph = 0; ph < 2; ++ph) {
      if (pl.op_exec[p][ph]) (void)hipGraphExecDestroy(pl.op_exec[p][ph]);
      if (pl.op_graph[p][ph]) (void)hipGraphDestroy(pl.op_graph[p][ph]);
      pl.op_exec[p][ph] = nullptr;
      pl.op_graph[p][ph] = nullptr;
      pl.op_graph_ws[p][ph] = nullptr;
    }
}

// Records the kernel sequence of one operator evaluation (all blocks of all
// regions and systems, the side-stream moment pass as a parallel branch)
// into a launch graph that reads x from o_gxin and writes y to o_gyout.
// Kernel nodes only: no memset or copy node is recorded.
static int capture_operator(pbtc_plan_t& pl, int precision, int phase) {
  const int p = precision == PBTC_FP64 ? 0 : 1;
  if (pl.op_exec[p][phase]) (void)hipGraphExecDestroy(pl.op_exec[p][phase]);
  if (pl.op_graph[p][phase]) (void)hipGraphDestroy(pl.op_graph[p][phase]);
  pl.op_exec[p][phase] = nullptr;
  pl.op_graph[p][phase] = nullptr;
  if (!pl.cap_stream) PBTC_HIP(hipStreamCreateWithFlags(&pl.cap_stream, hipStreamNonBlocking));
  if (!pl.side) {
    PBTC_HIP(hipStreamCreateWithFlags(&pl.side, hipStreamNonBlocking));
    PBTC_HIP(hipEventCreateWithFlags(&pl.ev_fork, hipEventDisableTiming));
    PBTC_HIP(hipEventCreateWithFlags(&pl.ev_join, hipEventDisableTiming));
  }
  const double* x = wsp<double>(pl, pl.o_gxin);
  double* y = wsp<double>(pl, pl.o_gyout);
  PBTC_HIP(hipStreamBeginCapture(pl.cap_stream, hipStreamCaptureModeThreadLocal));
  const int rc = p == 0 ? apply_impl<double>(pl, pl.cap_stream, x, y, phase, true)
                        : apply_impl<float>(pl, pl.cap_stream, x, y, phase, true);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(pl.cap_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  PBTC_HIP(e);
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(g);
    PBTC_HIP(ei);
  }
  size_t nodes = 0;
  PBTC_HIP(hipGraphGetNodes(g, nullptr, &nodes));
  pl.op_graph[p][phase] = g;
  pl.op_exec[p][phase] = ex;
  pl.op_graph_gen[p][phase] = pl.setup_gen;
  pl.op_graph_ws[p][phase] = pl.ws;
  pl.op_kernels[p][phase] = (int)nodes;
  return PBTC_OK;
}

// y = A x (phase 0) or phi_reac = S x (phase 1).  With params.op_graph the
// evaluation is one replay of the captured launch graph (x copied into its
// input buffer first and the result out of its output buffer after, unless
// the caller passes those buffers); an evaluation sampled for kernel timing
// launches its kernels one by one.
int apply_operator(pbtc_plan_t& pl, hipStream_t st, const double* x, double* y, int precision,
                   int phase) {
  const bool fp32 = precision != PBTC_FP64;
  const bool sampled = fp32 && phase == 0 && pl.prm.profile > 0 &&
                       pl.prof_count % pl.prm.profile == 0;
  if (!pl.prm.op_graph || sampled)
    return fp32 ? apply_impl<float>(pl, st, x, y, phase) : apply_impl<double>(pl, st, x, y, phase);
  const int p = fp32 ? 1 : 0;
  if (!pl.op_exec[p][phase] || pl.op_graph_gen[p][phase] != pl.setup_gen ||
      pl.op_graph_ws[p][phase] != pl.ws) {
    const int rc = capture_operator(pl, precision, phase);
    if (rc) return rc;
  }
  double* xin = wsp<double>(pl, pl.o_gxin);
  double* yout = wsp<double>(pl, pl.o_gyout);
  const int64_t ny = phase == 0 ? pl.nunk : pl.nq;
  if (x != xin)
    PBTC_HIP(hipMemcpyAsync(xin, x, 8 * pl.nunk, hipMemcpyDeviceToDevice, st));
  PBTC_HIP(hipGraphLaunch(pl.op_exec[p][phase], st));
  if (y != yout && ny > 0)
    PBTC_HIP(hipMemcpyAsync(y, yout, 8 * ny, hipMemcpyDeviceToDevice, st));
  if (fp32 && phase == 0) {
    if (pl.prm.profile > 0) ++pl.prof_count;
    ++pl.n_graph_launch;
  }
  return PBTC_OK;
}

// Descriptor tables (blocks, rows, item lists) to the device.
int upload_descriptors(pbtc_plan_t& pl, hipStream_t st) {
  std::vector<DevBlock> db(pl.blocks.size());
  for (size_t i = 0; i < pl.blocks.size(); ++i) {
    const Block& b = pl.blocks[i];
    const TargetSet& ts = pl.tsets[b.t];
    DevBlock& d = db[i];
    d.t = b.t;
    d.s = b.s;
    d.ks = b.ks;
    d.nk = b.nk;
    d.kappa0 = b.kappa[0];
    d.kappa1 = b.kappa[1];
    d.out0 = b.out[0];
    d.out1 = b.out[1];
    d.tgt_off = ts.off;
    d.ntgt = ts.n;
    d.grp_off = ts.grp_off;
    d.gp_off = pl.gp_off[b.s];
    d.gp_n = pl.gp_off[b.s + 1] - pl.gp_off[b.s];
    d.pan_off = pl.pan_off[b.s];
    d.item_off = b.item_off;
    d.nf_row = b.nf_row;
    d.root = b.s;  // roots are cells 0 .. nsurf-1
    d.self = (ts.kind == 0 && ts.id == b.s) ? 1 : 0;
    d.tkind = ts.kind;
    d.pad = 0;
    d.aitem_off = pl.blk_aitem_off[i];
    d.gpgrp_off = pl.gpgrp_off[b.s];
    d.aout0 = pl.blk_aout0[i];
    d.aout1 = pl.blk_aout1[i];
    d.csc_off = pl.blk_csc_off[i];
    d.slot0 = (int)pl.blk_slot0[i];
    d.lslot0 = pl.blk_lslot0.empty() ? 0 : pl.blk_lslot0[i];
    // automatic: a cell goes to P2P when its sources cost less there than
    // one M2P evaluation (issue slots are about 0.7 of the flop ratio of
    // the two kernels on gfx950)
    d.direct_below = pl.prm.direct_below >= 0
                         ? pl.prm.direct_below
                         : (int)std::lround(0.7 * m2p_flop_per_eval(pl.P, b.ks) /
                                            p2p_flop_per_pair(b.ks));
    d.troot = b.t;  // the target-set trees have one root per target set, in order
  }
  PBTC_HIP(hipMemcpyAsync(wsp<DevBlock>(pl, pl.o_blocks), db.data(), sizeof(DevBlock) * db.size(),
                          hipMemcpyHostToDevice, st));
  auto rows_to_dev = [&](const std::vector<RowBlock>& rows, bool surf, size_t orow,
                         size_t oterm) -> int {
    std::vector<DevRowBlock> r(rows.size());
    std::vector<DevRowTerm> t;
    for (size_t i = 0; i < rows.size(); ++i) {
      r[i].row_off = rows[i].row_off;
      r[i].n = rows[i].n;
      r[i].phi_off = rows[i].phi_off;
      r[i].term_off = (int)t.size();
      r[i].nterms = (int)rows[i].terms.size();
      r[i].half = surf ? 0.5 : 0.0;
      r[i].sign = surf ? -1.0 : 1.0;
      for (const RowTerm& rt : rows[i].terms) {
        DevRowTerm d;
        d.out = pl.blocks[rt.block].out[rt.kidx];
        d.sigma_c = rt.sigma_c;
        d.sigma = rt.sigma;
        t.push_back(d);
      }
    }
    if (!r.empty())
      PBTC_HIP(hipMemcpyAsync(wsp<DevRowBlock>(pl, orow), r.data(), sizeof(DevRowBlock) * r.size(),
                              hipMemcpyHostToDevice, st));
    if (!t.empty())
      PBTC_HIP(hipMemcpyAsync(wsp<DevRowTerm>(pl, oterm), t.data(), sizeof(DevRowTerm) * t.size(),
                              hipMemcpyHostToDevice, st));
    PBTC_HIP(hipStreamSynchronize(st));
    return PBTC_OK;
  };
  int rc = rows_to_dev(pl.rows, true, pl.o_rows, pl.o_terms);
  if (rc) return rc;
  rc = rows_to_dev(pl.reac_rows, false, pl.o_reac_rows, pl.o_reac_terms);
  if (rc) return rc;
  PBTC_HIP(hipMemcpyAsync(wsp<int>(pl, pl.o_items), pl.item_block.data(), 4 * pl.item_block.size(),
                          hipMemcpyHostToDevice, st));
  for (int ph = 0; ph < 2; ++ph)
    for (int ks = 0; ks < KS_COUNT; ++ks)
      if (!pl.item_list[ph][ks].empty())
        PBTC_HIP(hipMemcpyAsync(wsp<int>(pl, pl.o_item_list[ph][ks]), pl.item_list[ph][ks].data(),
                                4 * pl.item_list[ph][ks].size(), hipMemcpyHostToDevice, st));
  {
    // independent systems: system of every unknown and charge, reduction chunks
    std::vector<int> cu(pl.nunk), cq(std::max<int64_t>(pl.nq, 1), 0);
    for (int s = 0; s < pl.nsurf; ++s)
      for (int64_t u = pl.unk_off[s]; u < pl.unk_off[s + 1]; ++u) cu[u] = pl.comp_of_surface[s];
    for (int r = 0; r < pl.nreg; ++r)
      for (int64_t k = pl.q_off_region[r]; k < pl.q_off_region[r + 1]; ++k) cq[k] = pl.comp_of_region[r];
    PBTC_HIP(hipMemcpyAsync(wsp<int>(pl, pl.o_comp_of_unk), cu.data(), 4 * cu.size(),
                            hipMemcpyHostToDevice, st));
    PBTC_HIP(hipMemcpyAsync(wsp<int>(pl, pl.o_comp_q), cq.data(), 4 * cq.size(), hipMemcpyHostToDevice, st));
    PBTC_HIP(hipMemcpyAsync(wsp<int4>(pl, pl.o_chunks), pl.dot_chunks.data(), 16 * pl.dot_chunks.size(),
                            hipMemcpyHostToDevice, st));
    PBTC_HIP(hipMemcpyAsync(wsp<int4>(pl, pl.o_chunks) + pl.dot_chunks.size(), pl.comp_chunk0.data(),
                            4 * pl.comp_chunk0.size(), hipMemcpyHostToDevice, st));
    PBTC_HIP(hipStreamSynchronize(st));
  }
  {
    std::vector<int> rb(pl.nf_rows);
    for (size_t bi = 0; bi < pl.blocks.size(); ++bi) {
      const Block& b = pl.blocks[bi];
      for (int64_t i = 0; i < pl.tsets[b.t].n; ++i) rb[b.nf_row + i] = (int)bi;
    }
    PBTC_HIP(hipMemcpyAsync(wsp<int>(pl, pl.o_nf_rowblk), rb.data(), 4 * rb.size(),
                            hipMemcpyHostToDevice, st));
    PBTC_HIP(hipStreamSynchronize(st));
  }
  return PBTC_OK;
}

}  // namespace pbtc
