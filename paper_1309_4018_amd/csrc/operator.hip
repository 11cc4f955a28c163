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
// The double layer is formed from three dipole-weighted moments
// W_d[j] = sum p_d (y - c)^j, |j| <= P - 1, as M_DL[k] = sum_d k_d W_d[k - e_d],
// so that a (source, coefficient) term costs one monomial product and four
// FMAs.
//
// A span root is a cell of at most kSpanSources sources whose parent has more
// (or a tree root that small).  The cells of a span root's subtree are
// formed directly from the sources, in jobs: breadth-first runs of the
// span's cells of at most kMomJob sources in all, one work-group each, which
// stages the sources of its cells in LDS once.  Neighbouring small jobs of
// consecutive spans (adjacent sources) share a work-group.
// The larger (upper) cells then add the moments of the span roots below
// them, shifted to their own centres by the multi-index binomial theorem
// (sec. 2.3: moments shifted towards the root and added),
//   (y - c_u)^k = sum_{j <= k} C(k, j) h^(k - j) (y - c_s)^j,   h = c_s - c_u,
// which holds for both moment kinds (the double layer is a linear map of the
// same monomials), so upper cells never re-read the sources.
//
// Inside a job the work is split so that waves rarely wait for each other:
// cells the host marks as shared (more than kMomShared sources, or the only
// cell of its job) are summed by all four waves, a quarter of the sources
// each, and combined after one barrier; every other cell belongs to one wave
// (round robin over the job's cells, largest first), which sums all of its
// sources and assembles the double layer with wave-level synchronisation only.
// A lane owns coefficients lane, lane + 64, ...; for a run of kMomRows staged
// sources the lanes first write each source's power table into the wave's
// LDS slice -- (y-c)_x^a (y-c)_y^b for a + b <= P, then (y-c)_z^c -- so that a
// (source, coefficient) term is two LDS reads, one product and four FMAs.
constexpr int kMomWaves = 4;
constexpr int kMomThreads = 64 * kMomWaves;
constexpr int kMomRows = 32;       // sources per fill of a wave's power table
constexpr int kSpanCellsLds = 64;  // span cells whose entries are staged in LDS

__host__ __device__ constexpr int mom_xy_terms(int P) { return (P + 1) * (P + 2) / 2; }
__host__ __device__ constexpr int mom_row(int P) { return mom_xy_terms(P) + P + 1; }

// Per-coefficient constants of the moment pass, indexed by k (lane + 64 p):
// e[k][0] = power-table offsets (x-y entry | z entry << 8) | a << 16 |
// b << 20 | c << 24 for k = (a, b, c); e[k][1] = the entries k - e_d of the
// dipole moments (10 bits each, 0 where k_d = 0).  Indices past the last
// coefficient repeat k = 0.
template <int P>
struct MomLaneTable {
  static constexpr int KP = (ncoef(P) + 63) / 64;
  int e[KP * 64][2];
  constexpr MomLaneTable() : e() {
    for (int deg = 0; deg <= P; ++deg)
      for (int a = deg; a >= 0; --a)
        for (int b = deg - a; b >= 0; --b) {
          const int c = deg - a - b;
          const int k = mindex(a, b, c);
          const int ixy = a * (P + 1) - a * (a - 1) / 2 + b, iz = mom_xy_terms(P) + c;
          e[k][0] = ixy | (iz << 8) | (a << 16) | (b << 20) | (c << 24);
          e[k][1] = (a ? mindex(a - 1, b, c) : 0) | ((b ? mindex(a, b - 1, c) : 0) << 10) |
                    ((c ? mindex(a, b, c - 1) : 0) << 20);
        }
    for (int k = ncoef(P); k < KP * 64; ++k) {
      e[k][0] = e[0][0];
      e[k][1] = e[0][1];
    }
  }
};
template <int P>
__constant__ MomLaneTable<P> kMomLanes = MomLaneTable<P>();

template <typename real>
struct alignas(4 * sizeof(real)) Wt4 {
  real v[4];  // q, p_x, p_y, p_z of a source
};

// Sums sources [lo, lo + n) of the staged span into acc (coefficient k =
// lane + 64 p, weights q, p_x, p_y, p_z) about centre c; slice is the wave's
// power-table scratch.
template <typename real, int P, int KP>
__device__ __forceinline__ void mom_accumulate(const real (*sxyz)[3], const Wt4<real>* sw, real* slice,
                                               int lo, int n, real cx, real cy, real cz,
                                               const int (&ixy)[KP], const int (&iz)[KP],
                                               real (&acc)[KP][4]) {
  constexpr int ROW = mom_row(P), TXY = mom_xy_terms(P);
  const int lane = threadIdx.x & 63;
  for (int r0 = 0; r0 < n; r0 += kMomRows) {
    const int nr = min(kMomRows, n - r0);
    if (lane < nr) {
      const int t = lo + r0 + lane;
      const real dx = sxyz[t][0] - cx, dy = sxyz[t][1] - cy, dz = sxyz[t][2] - cz;
      real px[P + 1], py[P + 1];
      px[0] = py[0] = 1;
#pragma unroll
      for (int a = 1; a <= P; ++a) {
        px[a] = px[a - 1] * dx;
        py[a] = py[a - 1] * dy;
      }
      real* row = slice + lane * ROW;
#pragma unroll
      for (int a = 0; a <= P; ++a)
#pragma unroll
        for (int b = 0; a + b <= P; ++b) row[a * (P + 1) - a * (a - 1) / 2 + b] = px[a] * py[b];
      real v = 1;
#pragma unroll
      for (int c = 0; c <= P; ++c) {
        row[TXY + c] = v;
        v *= dz;
      }
    }
    wave_sync();  // the power tables are written
#pragma unroll 4
    for (int t = 0; t < nr; ++t) {
      const Wt4<real> wt = sw[lo + r0 + t];
      const real* row = slice + t * ROW;
#pragma unroll
      for (int p = 0; p < KP; ++p) {
        const real m = row[ixy[p]] * row[iz[p]];
        // the dipole moments are needed below degree P only: a pass of
        // degree-P coefficients sums the charge term alone
        constexpr int kLow = ncoef(P - 1);
        const int nw = 64 * p >= kLow ? 1 : 4;
#pragma unroll
        for (int i = 0; i < nw; ++i) acc[p][i] += wt.v[i] * m;
      }
    }
    wave_sync();  // the rows are read before the next fill
  }
}

template <typename real, int P>
__global__ __launch_bounds__(kMomThreads) void k_mom_span(const int4* __restrict__ spans,
                                                          const int4* __restrict__ scells,
                                                          const double4* __restrict__ cent,
                                                          const Src<real>* __restrict__ src,
                                                          real* __restrict__ mom) {
  constexpr int N = ncoef(P);
  constexpr int KP = (N + 63) / 64;  // coefficients per lane
  constexpr int TXY = mom_xy_terms(P);
  constexpr int SLICE = kMomRows * mom_row(P);
  static_assert(4 * N <= SLICE, "a wave's partial moments fit its slice");
  static_assert(kSpanCell <= kSpanSources && kSpanCellsLds <= kMomThreads,
                "a span's sources and cell entries fit the staging arrays");
  __shared__ real sxyz[kSpanSources][3];
  __shared__ Wt4<real> sw[kSpanSources];
  __shared__ real slice[kMomWaves][SLICE];
  __shared__ int4 sce[kSpanCellsLds];
  __shared__ real scc[kSpanCellsLds][3];
  // job: (first entry of its cells in scells, number of cells, first
  // source, sources); XCD x runs the x-th contiguous run of the job list
  const int4 sp = spans[xcd_block(blockIdx.x, gridDim.x)];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (tid < min(sp.y, kSpanCellsLds)) {
    const double4 cc = cent[sp.x + tid];
    sce[tid] = scells[sp.x + tid];
    scc[tid][0] = (real)cc.x;
    scc[tid][1] = (real)cc.y;
    scc[tid][2] = (real)cc.z;
  }
  for (int t = tid; t < sp.w; t += kMomThreads) {
    const Src<real> s = src[sp.z + t];
    sxyz[t][0] = s.x;
    sxyz[t][1] = s.y;
    sxyz[t][2] = s.z;
    Wt4<real> wt;
    wt.v[0] = s.q;
    wt.v[1] = s.px;
    wt.v[2] = s.py;
    wt.v[3] = s.pz;
    sw[t] = wt;
  }
  // this lane's coefficients: power-table offsets, and the entries
  // k - e_d of the dipole moments that form the double layer
  int ixy[KP], iz[KP], jd[KP][3], kd[KP][3];
#pragma unroll
  for (int p = 0; p < KP; ++p) {
    const int e0 = kMomLanes<P>.e[lane + 64 * p][0], e1 = kMomLanes<P>.e[lane + 64 * p][1];
    ixy[p] = e0 & 255;
    iz[p] = (e0 >> 8) & 255;
    kd[p][0] = (e0 >> 16) & 15;
    kd[p][1] = (e0 >> 20) & 15;
    kd[p][2] = e0 >> 24;
    jd[p][0] = e1 & 1023;
    jd[p][1] = (e1 >> 10) & 1023;
    jd[p][2] = e1 >> 20;
  }
  __syncthreads();
  // entry e: (cell, first source, sources, shared flag) and its centre
  auto entry = [&](int e, int4& ce, real& cx, real& cy, real& cz) {
    if (e < kSpanCellsLds) {
      ce = sce[e];
      cx = scc[e][0];
      cy = scc[e][1];
      cz = scc[e][2];
    } else {
      ce = scells[sp.x + e];
      const double4 cc = cent[sp.x + e];
      cx = (real)cc.x;
      cy = (real)cc.y;
      cz = (real)cc.z;
    }
    ce.x = __builtin_amdgcn_readfirstlane(ce.x);  // wave-uniform loop bounds
    ce.y = __builtin_amdgcn_readfirstlane(ce.y);
    ce.z = __builtin_amdgcn_readfirstlane(ce.z);
    ce.w = __builtin_amdgcn_readfirstlane(ce.w);
  };
  real* my = slice[w];
  // shared cells (listed first): a quarter of the sources per wave
  int e = 0;
  for (; e < sp.y; ++e) {
    int4 ce;
    real cx, cy, cz;
    entry(e, ce, cx, cy, cz);
    if (!ce.w) break;
    const int q = (ce.z + kMomWaves - 1) / kMomWaves;
    const int n = max(0, min(q, ce.z - w * q));
    real acc[KP][4] = {};
    mom_accumulate<real, P, KP>(sxyz, sw, my, ce.y - sp.z + w * q, n, cx, cy, cz, ixy, iz, acc);
#pragma unroll
    for (int p = 0; p < KP; ++p) {
      const int k = lane + 64 * p;
      if (k < N)
#pragma unroll
        for (int i = 0; i < 4; ++i) my[i * N + k] = acc[p][i];
    }
    __syncthreads();  // the four partial sums are in the slices
    for (int k = tid; k < N; k += kMomThreads) {
      const int e0 = kMomLanes<P>.e[k][0], e1 = kMomLanes<P>.e[k][1];
      const int a = (e0 >> 16) & 15, b = (e0 >> 20) & 15, c = e0 >> 24;
      const int j0 = e1 & 1023, j1 = (e1 >> 10) & 1023, j2 = e1 >> 20;
      real s = 0, w0 = 0, w1 = 0, w2 = 0;
#pragma unroll
      for (int v = 0; v < kMomWaves; ++v) {
        s += slice[v][k];
        w0 += slice[v][N + j0];
        w1 += slice[v][2 * N + j1];
        w2 += slice[v][3 * N + j2];
      }
      mom[(size_t)ce.x * 2 * N + k] = s;
      mom[(size_t)ce.x * 2 * N + N + k] = real(a) * w0 + real(b) * w1 + real(c) * w2;
    }
    __syncthreads();  // the slices are read before they are refilled
  }
  // the other cells, one wave each
  for (e += w; e < sp.y; e += kMomWaves) {
    int4 ce;
    real cx, cy, cz;
    entry(e, ce, cx, cy, cz);
    real acc[KP][4] = {};
    mom_accumulate<real, P, KP>(sxyz, sw, my, ce.y - sp.z, ce.z, cx, cy, cz, ixy, iz, acc);
#pragma unroll
    for (int p = 0; p < KP; ++p) {
      const int k = lane + 64 * p;
      if (k < N)
#pragma unroll
        for (int d = 0; d < 3; ++d) my[d * N + k] = acc[p][1 + d];
    }
    wave_sync();  // the dipole moments are in the slice
#pragma unroll
    for (int p = 0; p < KP; ++p) {
      const int k = lane + 64 * p;
      if (k < N) {
        const real dl = real(kd[p][0]) * my[jd[p][0]] + real(kd[p][1]) * my[N + jd[p][1]] +
                        real(kd[p][2]) * my[2 * N + jd[p][2]];
        mom[(size_t)ce.x * 2 * N + k] = acc[p][0];
        mom[(size_t)ce.x * 2 * N + N + k] = dl;
      }
    }
    wave_sync();  // the slice is read before the next cell's power tables
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

// Moments of the upper cells: each is the sum of the moments of the span
// roots below it (a contiguous run of the depth-first span list), each
// shifted to the cell's centre.  A work-group takes one part of at most
// mom_up_batch(P) span roots of one cell.  The three-dimensional shift
// factors into one-dimensional shifts along x, then y, then z (the binomial
// sum is a product over the axes): the span roots' moments are unpacked into
// a dense (P+1)^3 array in LDS, and a thread shifts one line of it
// ("pencil": fixed indices on the other two axes, at most P+1 entries) in
// registers, with the binomials as constants.  Entries of total degree > P
// are never read or written.  A cell of one part stores its moments; the
// parts of a larger cell store partial sums that k_mom_up_sum adds in part
// order (deterministic).  Parts are listed by their first span root and
// dealt to the XCDs in contiguous runs, so a span root's moments are read
// by one XCD at every level.
template <typename real, int P>
__global__ __launch_bounds__(256) void k_mom_up_part(const int4* __restrict__ parts,
                                                     const int* __restrict__ proot,
                                                     const double* __restrict__ ph,
                                                     real* __restrict__ mom,
                                                     real* __restrict__ partial) {
  constexpr int N = ncoef(P), N2 = 2 * N, Q = P + 1;
  constexpr int R = mom_up_batch(P);
  constexpr int NPEN = Q * (Q + 1) / 2;  // pencils per kind and axis
  constexpr int OPT = (N2 + 255) / 256;  // outputs per thread
  constexpr Binom B{};
  __shared__ real D[R][2][Q][Q][Q];
  __shared__ real hp[R][3][Q];
  __shared__ int abc[N];       // a | b << 8 | c << 16 of coefficient k
  __shared__ int pen_mn[NPEN];  // m | n << 8 of pencil p
  __shared__ int root[R];
  const int part = xcd_block(blockIdx.x, gridDim.x);
  const int4 pt = parts[part];  // (upper cell, first span, end span, partial slot or -1)
  const int u = pt.x, nr = pt.z - pt.y;
  const int tid = threadIdx.x;
  for (int k = tid; k < N; k += 256) {
    int a, b, c;
    mindex_inv(k, a, b, c);
    abc[k] = a | (b << 8) | (c << 16);
  }
  if (tid < NPEN) {
    int pen = tid, m = 0;
    while (pen >= Q - m) pen -= Q - m++;
    pen_mn[tid] = m | (pen << 8);
  }
  // the part's span roots and their offsets from the cell's centre (R
  // slots per part, unused ones zero), read without waiting for pt
  if (tid < R) root[tid] = proot[(size_t)part * R + tid];
  if (tid < 3 * R) {
    const int r = tid / 3, d = tid - 3 * r;
    const double h = ph[((size_t)part * R + r) * 3 + d];
    real v = 1;
    for (int e = 0; e < Q; ++e) {
      hp[r][d][e] = v;
      v *= (real)h;
    }
  }
  __syncthreads();
  for (int i = tid; i < nr * N2; i += 256) {
    const int r = i / N2, k = i - r * N2;
    const int s = k < N ? 0 : 1;
    const int t = abc[k - s * N];
    D[r][s][t & 255][(t >> 8) & 255][t >> 16] = mom[(size_t)root[r] * N2 + k];
  }
  __syncthreads();
#pragma unroll
  for (int axis = 0; axis < 3; ++axis) {
    for (int i = tid; i < nr * 2 * NPEN; i += 256) {
      const int r = i / (2 * NPEN), rest = i - r * 2 * NPEN;
      const int s = rest / NPEN;
      const int mn = pen_mn[rest - s * NPEN];
      const int m = mn & 255, n = mn >> 8, len = Q - m - n;
      real* base;
      int stride;
      if (axis == 0) {
        base = &D[r][s][0][m][n];
        stride = Q * Q;
      } else if (axis == 1) {
        base = &D[r][s][m][0][n];
        stride = Q;
      } else {
        base = &D[r][s][m][n][0];
        stride = 1;
      }
      const real* h = hp[r][axis];
      real v[Q], hv[Q];
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        v[j] = j < len ? base[j * stride] : real(0);
        hv[j] = h[j];
      }
      // in place, highest degree first: v[a] = sum_{j <= a} C(a, j) h^(a-j) v[j]
#pragma unroll
      for (int a = Q - 1; a >= 1; --a) {
        real t = v[a];
#pragma unroll
        for (int j = 0; j < a; ++j) t += (real(B.c[a][j]) * hv[a - j]) * v[j];
        v[a] = t;
      }
#pragma unroll
      for (int j = 0; j < Q; ++j)
        if (j < len) base[j * stride] = v[j];
    }
    __syncthreads();
  }
  real* dst = pt.w < 0 ? mom + (size_t)u * N2 : partial + (size_t)pt.w * N2;
#pragma unroll
  for (int o = 0; o < OPT; ++o) {
    const int k = tid + 256 * o;
    if (k < N2) {
      const int s = k < N ? 0 : 1;
      const int t = abc[k - s * N];
      const int a = t & 255, b = (t >> 8) & 255, c = t >> 16;
      real acc = 0;
      for (int r = 0; r < nr; ++r) acc += D[r][s][a][b][c];
      dst[k] = acc;
    }
  }
}

// Moments of an upper cell of several parts: the sum of the parts' partial
// moments.  Wave w of W adds parts w, w + W, ..., then the W wave sums are
// added in wave order (deterministic).
template <typename real, int P>
constexpr int sum_waves() {
  constexpr int per = ((2 * ncoef(P) + 63) / 64) * 64 * (int)sizeof(real);
  return 16 * per <= 49152 ? 16 : 8 * per <= 49152 ? 8 : 4;
}

template <typename real, int P>
__global__ __launch_bounds__((64 * sum_waves<real, P>())) void k_mom_up_sum(
    const int4* __restrict__ sums, const real* __restrict__ partial, real* __restrict__ mom) {
  constexpr int N2 = 2 * ncoef(P);
  constexpr int OPW = (N2 + 63) / 64;  // outputs per lane
  constexpr int kSumWaves = sum_waves<real, P>();
  __shared__ real red[kSumWaves][OPW * 64];
  const int4 sm = sums[blockIdx.x];  // (upper cell, first part, parts)
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  real acc[OPW];
#pragma unroll
  for (int o = 0; o < OPW; ++o) acc[o] = 0;
  int p = w;
  for (; p + 3 * kSumWaves < sm.z; p += 4 * kSumWaves)  // four loads in flight per output
#pragma unroll
    for (int o = 0; o < OPW; ++o) {
      const int k = lane + 64 * o;
      if (k < N2) {
        const real* q = partial + (size_t)(sm.y + p) * N2 + k;
        const real v0 = q[0], v1 = q[(size_t)kSumWaves * N2], v2 = q[(size_t)2 * kSumWaves * N2],
                   v3 = q[(size_t)3 * kSumWaves * N2];
        acc[o] += (v0 + v1) + (v2 + v3);
      }
    }
  for (; p < sm.z; p += kSumWaves)
#pragma unroll
    for (int o = 0; o < OPW; ++o) {
      const int k = lane + 64 * o;
      if (k < N2) acc[o] += partial[(size_t)(sm.y + p) * N2 + k];
    }
#pragma unroll
  for (int o = 0; o < OPW; ++o) red[w][lane + 64 * o] = acc[o];
  __syncthreads();
  for (int k = threadIdx.x; k < N2; k += 64 * kSumWaves) {
    real v = 0;
#pragma unroll
    for (int ww = 0; ww < kSumWaves; ++ww) v += red[ww][k];
    mom[(size_t)sm.x * N2 + k] = v;
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

// Lanes of a wavefront: target t = lane % kGroup of the unit's group, quarter
// q = lane / kGroup.  The quarters' partial sums of a target are added
// across the wave (fixed order) and lanes 0 .. kGroup-1 store the unit's
// sums: partial[(u * 4 + i) * kGroup + t].
template <typename real, int NQ>
__device__ __forceinline__ void unit_store(real* __restrict__ partial, int u, real (&acc)[4],
                                           int off = 0) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
#pragma unroll
    for (int m = kGroup; m < 64; m <<= 1) acc[i] += __shfl_xor(acc[i], m);
  }
  if (lane < kGroup)
#pragma unroll
    for (int i = 0; i < NQ; ++i) partial[((size_t)u * 4 + off + i) * kGroup + lane] = acc[i];
}

// P2P: the sources of the unit's cells form one stream (cells in list order)
// that passes through a per-wavefront LDS slice 64 sources at a time: one
// load per lane, whatever cell the source lies in (a lane finds it by binary
// search over the prefix of the cells' counts), the next chunk loaded while
// the current one is used.  The four lanes of a target take every fourth
// staged source, so that a pair's operands are all vector registers.
template <typename real, int KS>
__global__ __launch_bounds__(kItemThreads) void k_p2p(UnitArgs a, const real* __restrict__ tx,
                                                      const real* __restrict__ ty,
                                                      const real* __restrict__ tz,
                                                      const Src<real>* __restrict__ src,
                                                      real* __restrict__ partial) {
  __shared__ Src<real> stage[kWaves][64];
  __shared__ int cbeg[kWaves][64], cpre[kWaves][64];
  const int u = uni(xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6));
  if (u >= a.nunits) return;
  const int wv = uni(threadIdx.x >> 6);
  const int4 un = a.units[u];
  const int item = uni(un.x), e0 = uni(un.y), e1 = uni(un.z);
  const DevBlock& b = a.blocks[uni(a.item_block[item])];
  const long long g = item - b.item_off;
  const long long t0 = b.tgt_off + g * kGroup;
  const int nt = (int)min((long long)kGroup, b.ntgt - g * kGroup);
  const int lane = threadIdx.x & 63, qt = lane / kGroup;
  const long long ti = t0 + min(lane % kGroup, nt - 1);
  const real x = tx[ti], y = ty[ti], z = tz[ti];
  const real k0 = (real)b.kappa0, k1 = (real)b.kappa1;
  const real a0 = exp_arg(k0), a1 = exp_arg(k1);
  real acc[4] = {0, 0, 0, 0};
  // a source record travels in seven registers (no aggregate copies)
  real cur[7] = {0, 0, 0, 0, 0, 0, 0}, nxt[7] = {0, 0, 0, 0, 0, 0, 0};
  auto load = [&](real (&v)[7], int j) {
    const Src<real>& r = src[j];
    v[0] = r.x;
    v[1] = r.y;
    v[2] = r.z;
    v[3] = r.q;
    v[4] = r.px;
    v[5] = r.py;
    v[6] = r.pz;
  };
  // source of stream position p of the current batch of cells
  int ncb = 0;
  auto source_of = [&](int p) {
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
      if (lo + step < ncb && cpre[wv][lo + step] <= p) lo += step;
    return cbeg[wv][lo] + (p - cpre[wv][lo]);
  };
  for (int eb = e0; eb < e1; eb += 64) {
    // a batch of up to 64 cells: first sources and the exclusive prefix of
    // their counts
    ncb = min(64, e1 - eb);
    int beg = 0, cnt = 0;
    if (lane < ncb) {
      const int c = a.cells_list[eb + lane];
      beg = a.cells[c].begin;
      cnt = a.cells[c].count;
    }
    int incl = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int v = __shfl_up(incl, d);
      if (lane >= d) incl += v;
    }
    const int total = __shfl(incl, 63);
    wave_sync();  // the previous batch's table is no longer read
    cbeg[wv][lane] = beg;
    cpre[wv][lane] = incl - cnt;
    wave_sync();
    if (lane < total) load(cur, source_of(lane));
    for (int p0 = 0; p0 < total; p0 += 64) {
      const int n = min(64, total - p0);
      if (p0 + 64 + lane < total) load(nxt, source_of(p0 + 64 + lane));
      if (lane < n) {
        Src<real>& d = stage[wv][lane];
        d.x = cur[0];
        d.y = cur[1];
        d.z = cur[2];
        d.q = cur[3];
        d.px = cur[4];
        d.py = cur[5];
        d.pz = cur[6];
      }
      wave_sync();
      int j = qt;
      for (; j + 3 * kQuarters < n; j += 4 * kQuarters) {
        const Src<real> s0 = stage[wv][j], s1 = stage[wv][j + kQuarters],
                        s2 = stage[wv][j + 2 * kQuarters], s3 = stage[wv][j + 3 * kQuarters];
        pair<real, KS>(x, y, z, s0, k0, k1, a0, a1, acc);
        pair<real, KS>(x, y, z, s1, k0, k1, a0, a1, acc);
        pair<real, KS>(x, y, z, s2, k0, k1, a0, a1, acc);
        pair<real, KS>(x, y, z, s3, k0, k1, a0, a1, acc);
      }
      for (; j < n; j += kQuarters) {
        const Src<real> s0 = stage[wv][j];
        pair<real, KS>(x, y, z, s0, k0, k1, a0, a1, acc);
      }
      wave_sync();  // the slice is read before the next chunk overwrites it
#pragma unroll
      for (int i = 0; i < 7; ++i) cur[i] = nxt[i];
    }
  }
  unit_store<real, nacc<KS>()>(partial, u, acc);
}

// ------------------------------------------------------------------- m2p
// Green's function KIND0 of kernel slot `slot` (0 Laplace, 1 Yukawa), and
// with KIND1 >= 0 also KIND1 of slot 1 for the same (target, cell) pairs
// (blocks of two kernels: one pass over the cells, the geometry and the
// staged moments shared).  Per step the wave evaluates four cells of the
// unit, one per quarter of its lanes: the four cells' moments pass through a
// per-wavefront LDS slice (the lanes of a quarter read the same addresses).
template <typename real, int P>
constexpr int m2p_waves() {
  constexpr int per = kQuarters * 2 * ncoef(P) * (int)sizeof(real);
  return kWaves * per <= 49152 ? kWaves : 2 * per <= 49152 ? 2 : 1;
}

template <typename real, int P, int KIND>
__device__ __forceinline__ void m2p_eval(real dx, real dy, real dz, real r2, real rinv, real kap,
                                         const real* __restrict__ M, real& s, real& d) {
  if (KIND == 0)
    taylor_laplace<P, real>(dx, dy, dz, rinv, M, s, d);
  else
    taylor_yukawa<P, real>(dx, dy, dz, rinv, exp_neg(kap * (r2 * rinv)), kap, M, s, d);
}

template <typename real, int P, int KIND0, int KIND1>
__global__ __launch_bounds__((64 * m2p_waves<real, P>())) void k_m2p(
    UnitArgs a, const real* __restrict__ tx, const real* __restrict__ ty,
    const real* __restrict__ tz, const real* __restrict__ mom, int slot,
    real* __restrict__ partial) {
  constexpr int N = ncoef(P), N2 = 2 * N;
  constexpr int W = m2p_waves<real, P>();
  constexpr int PER = (N2 + kGroup - 1) / kGroup;  // moment values per lane and step
  __shared__ real smom[W][kQuarters][N2];
  const int u = uni(xcd_block(blockIdx.x, gridDim.x) * W + (threadIdx.x >> 6));
  if (u >= a.nunits) return;
  const int wv = uni(threadIdx.x >> 6);
  const int4 un = a.units[u];
  const int item = uni(un.x), e0 = uni(un.y), e1 = uni(un.z);
  const DevBlock& b = a.blocks[uni(a.item_block[item])];
  const long long g = item - b.item_off;
  const long long t0 = b.tgt_off + g * kGroup;
  const int nt = (int)min((long long)kGroup, b.ntgt - g * kGroup);
  const int lane = threadIdx.x & 63, qt = lane / kGroup, tl = lane % kGroup;
  const long long ti = t0 + min(tl, nt - 1);
  const real x = tx[ti], y = ty[ti], z = tz[ti];
  const real kap0 = (real)(slot == 0 ? b.kappa0 : b.kappa1), kap1 = (real)b.kappa1;
  real* M = &smom[wv][0][0];
  real acc[4] = {0, 0, 0, 0};
  for (int e = e0; e < e1; e += kQuarters) {
    // the cell of this lane's quarter among the four from entry e
    const int cm = e + qt < e1 ? a.cells_list[e + qt] : -1;
    wave_sync();  // the previous step's reads of the slice are done
    real cx = 0, cy = 0, cz = 0;
    if (cm >= 0) {
      const real* Mg = mom + (size_t)cm * N2;
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        const int k = tl + kGroup * r;
        if (k < N2) M[qt * N2 + k] = Mg[k];
      }
      const Cell& cl = a.cells[cm];
      cx = (real)cl.cx;
      cy = (real)cl.cy;
      cz = (real)cl.cz;
    }
    wave_sync();  // the four cells' moments are in the slice
    if (cm >= 0) {
      const real* Mq = M + qt * N2;
      const real dx = x - cx, dy = y - cy, dz = z - cz;
      const real r2 = dx * dx + dy * dy + dz * dz;
      const real rinv = rsqrt_(r2);
      m2p_eval<real, P, KIND0>(dx, dy, dz, r2, rinv, kap0, Mq, acc[0], acc[1]);
      if (KIND1 >= 0) {
        // the second recurrence after the first, reading the moments from
        // LDS again (no interleaving, no moments held across: the registers
        // of one recurrence at a time)
        __asm__ volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        m2p_eval<real, P, (KIND1 > 0 ? 1 : 0)>(dx, dy, dz, r2, rinv, kap1, Mq, acc[2], acc[3]);
      }
    }
  }
  // one Green's function of slot 1 (the second of a pair, launched on its
  // own) fills the unit's values 2 and 3
  unit_store<real, KIND1 >= 0 ? 4 : 2>(partial, u, acc, KIND1 >= 0 ? 0 : 2 * slot);
}

// Sum of the P2P units and the M2P units of every listed item, times
// 1/(4 pi), stored into S and D of the block's kernel slots.  One wavefront
// per item: lane = target t (lane % kGroup) of quarter q (lane / kGroup);
// quarter q adds units q, q + 4, ... of each set, then the quarters' sums are
// added across the wave (fixed order: deterministic).  uptr_f = null: no
// far-field units.
constexpr int kReduceWaves = 4;

template <typename real, int NQ>
__device__ __forceinline__ void add_units(double (&v)[NQ], const real* __restrict__ partial,
                                          int u0, int u1, int t, int qt) {
  int u = u0 + qt;
  // two units per step per lane
  for (; u + kQuarters < u1; u += 2 * kQuarters) {
    real p[2][NQ];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        p[k][q] = partial[((size_t)(u + k * kQuarters) * 4 + q) * kGroup + t];
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] += (double)p[0][q] + (double)p[1][q];
  }
  if (u < u1)
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] += (double)partial[((size_t)u * 4 + q) * kGroup + t];
}

template <typename real, int NQ>
__global__ __launch_bounds__(64 * kReduceWaves) void k_reduce(
    int nlist, const int* __restrict__ list, const int* __restrict__ uptr_n,
    const real* __restrict__ partial_n, const int* __restrict__ uptr_f,
    const real* __restrict__ partial_f, const int* __restrict__ item_block,
    const DevBlock* __restrict__ blocks, const int* __restrict__ tidx, double* __restrict__ S,
    double* __restrict__ D) {
  const int l = blockIdx.x * kReduceWaves + (threadIdx.x >> 6);
  if (l >= nlist) return;
  const int lane = threadIdx.x & 63, t = lane % kGroup, qt = lane / kGroup;
  // the output rows first, so that their loads overlap those of the units
  const int item = list[l];
  const DevBlock& b = blocks[item_block[item]];
  const long long g = item - b.item_off;
  const int nt = (int)min((long long)kGroup, b.ntgt - g * kGroup);
  const long long i = lane < nt ? tidx[b.tgt_off + g * kGroup + lane] - b.tgt_off : 0;
  const long long out0 = b.out0 + i, out1 = b.out1 + i;
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  if (uptr_n) add_units<real, NQ>(v, partial_n, uptr_n[l], uptr_n[l + 1], t, qt);
  if (uptr_f) add_units<real, NQ>(v, partial_f, uptr_f[l], uptr_f[l + 1], t, qt);
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int m = kGroup; m < 64; m <<= 1) v[q] += __shfl_xor(v[q], m);
  if (lane >= nt) return;
  // S and D already hold the near-field corrections of these rows
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const long long out = (q >> 1) == 0 ? out0 : out1;
    ((q & 1) ? D : S)[out] += v[q] * kInv4Pi;
  }
}

// ----------------------------------------------------------- near field
// S[out_k + i] = sum_e dV_k(e) psi(col), D[out_k + i] = sum_e dK_k(e) phi(col)
// (every target of every block has a row, so this stores every entry that
// the reductions then add their sums to)
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
  S[b.out0 + i] = (double)s0;
  D[b.out0 + i] = (double)d0;
  if (nk == 2) {
    S[b.out1 + i] = (double)s1;
    D[b.out1 + i] = (double)d1;
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
  const int4* scells = wsp<int4>(pl, pl.o_mchunks);
  const double4* cent = wsp<double4>(pl, pl.o_mcent);
  const int4* spans = wsp<int4>(pl, pl.o_mspans);
  const int* proot = wsp<int>(pl, pl.o_mproot);
  const double* ph = wsp<double>(pl, pl.o_mph);
  const int4* parts = wsp<int4>(pl, pl.o_mparts);
  const int4* sums = wsp<int4>(pl, pl.o_musum);
  real* partial = wsp<real>(pl, pl.o_mpart);
  const unsigned nsp = (unsigned)pl.n_mspans, npt = (unsigned)pl.n_mparts,
                 nsum = (unsigned)pl.n_musum;
#define PBTC_MOM(PP)                                                                          \
  case PP:                                                                                    \
    if (nsp > 0)                                                                              \
      hipLaunchKernelGGL((k_mom_span<real, PP>), dim3(nsp), dim3(kMomThreads), 0, st, spans,  \
                         scells, cent, src, mom);                                             \
    if (npt > 0)                                                                              \
      hipLaunchKernelGGL((k_mom_up_part<real, PP>), dim3(npt), dim3(256), 0, st, parts,       \
                         proot, ph, mom, partial);                                            \
    if (nsum > 0)                                                                             \
      hipLaunchKernelGGL((k_mom_up_sum<real, PP>), dim3(nsum), dim3(64 * sum_waves<real, PP>()), \
                         0, st, sums, partial, mom);                                          \
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

template <typename real, int KIND0, int KIND1>
static void launch_m2p(pbtc_plan_t& pl, hipStream_t st, const UnitArgs& a, const real* tx,
                       const real* ty, const real* tz, const real* mom, int slot, real* partial) {
#define PBTC_M2P(PP)                                                                           \
  case PP: {                                                                                   \
    constexpr int W = m2p_waves<real, PP>();                                                   \
    hipLaunchKernelGGL((k_m2p<real, PP, KIND0, KIND1>), dim3(nblocks(a.nunits, W)),           \
                       dim3(64 * W), 0, st, a, tx, ty, tz, mom, slot, partial);                \
    break;                                                                                     \
  }
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
  // The far field (moment pass, then M2P) runs on a second stream beside
  // the P2P launches, so that each fills the other's ramps and tails; the
  // near units are reduced behind P2P, the far units once both streams are
  // done.  A sampled (timed) evaluation runs everything
  // on one stream instead, moment pass first, so that each timed launch has
  // the GPU to itself.
  const bool fork = tree && pl.n_far > 0 && !timed;
  if (fork && !pl.side) {
    PBTC_HIP(hipStreamCreateWithFlags(&pl.side, hipStreamNonBlocking));
    PBTC_HIP(hipEventCreateWithFlags(&pl.ev_fork, hipEventDisableTiming));
    PBTC_HIP(hipEventCreateWithFlags(&pl.ev_join, hipEventDisableTiming));
  }
  const hipStream_t sf = fork ? pl.side : st;  // stream of the far field
  if (fork) {
    PBTC_HIP(hipEventRecord(pl.ev_fork, st));
    PBTC_HIP(hipStreamWaitEvent(pl.side, pl.ev_fork, 0));
  }
  if (tree) {
    int rc = launch_moments<real>(pl, sf, mom, src);
    if (rc) return rc;
  }
  UnitArgs a;
  a.item_block = wsp<int>(pl, pl.o_items);
  a.blocks = wsp<DevBlock>(pl, pl.o_blocks);
  a.cells = wsp<Cell>(pl, pl.o_cells);
  const int* tidx = wsp<int>(pl, pl.o_tidx);
  double* S = wsp<double>(pl, pl.o_S);
  double* D = wsp<double>(pl, pl.o_D);
  real* partial = wsp<real>(pl, pl.o_partial);
  // P2P over the near lists of kernel set ks; each unit set writes its own
  // region of the partial sums (by the set's first unit), so that one
  // reduction adds the near and the far units
  auto p2p = [&](int ks, hipStream_t s) -> int {
    const UnitSet& un = pl.units[phase][ks][0];
    UnitArgs u = a;
    u.units = wsp<int4>(pl, pl.o_units + 16 * un.off);
    u.nunits = (int)un.n;
    u.cells_list = wsp<int>(pl, pl.o_near);
    real* part_n = partial + (size_t)un.off * 4 * kGroup;
    const int grid = nblocks(un.n, kWaves);
    prof_mark(pl, s, timed, 0, pl.launch_flop_p2p[phase][ks], true);
    // no units (every cell seen through its expansion): the reduction
    // still stores the (M2P or zero) sums
    if (grid > 0) switch (ks) {
      case KS_L:
        hipLaunchKernelGGL((k_p2p<real, KS_L>), dim3(grid), dim3(kItemThreads), 0, s, u, tx, ty, tz, src, part_n);
        break;
      case KS_Y:
        hipLaunchKernelGGL((k_p2p<real, KS_Y>), dim3(grid), dim3(kItemThreads), 0, s, u, tx, ty, tz, src, part_n);
        break;
      case KS_LY:
        hipLaunchKernelGGL((k_p2p<real, KS_LY>), dim3(grid), dim3(kItemThreads), 0, s, u, tx, ty, tz, src, part_n);
        break;
      case KS_YY:
        hipLaunchKernelGGL((k_p2p<real, KS_YY>), dim3(grid), dim3(kItemThreads), 0, s, u, tx, ty, tz, src, part_n);
        break;
    }
    prof_mark(pl, s, timed, 0, 0.0, false);
    PBTC_LAUNCH_CHECK();
    return PBTC_OK;
  };
  auto has_far = [&](int ks) { return tree && pl.n_far > 0 && pl.units[phase][ks][1].n > 0; };
  // M2P over the far lists of kernel set ks
  auto m2p = [&](int ks, hipStream_t s) -> int {
    const UnitSet& uf = pl.units[phase][ks][1];
    UnitArgs u = a;
    u.units = wsp<int4>(pl, pl.o_units + 16 * uf.off);
    u.nunits = (int)uf.n;
    u.cells_list = wsp<int>(pl, pl.o_far);
    real* part_f = partial + (size_t)uf.off * 4 * kGroup;
    if (ks == KS_L || ks == KS_Y) {
      const int kind = ks == KS_L ? 0 : 1;
      prof_mark(pl, s, timed, 1 + kind, pl.launch_flop_m2p[phase][ks], true);
      if (kind == 0)
        launch_m2p<real, 0, -1>(pl, s, u, tx, ty, tz, mom, 0, part_f);
      else
        launch_m2p<real, 1, -1>(pl, s, u, tx, ty, tz, mom, 0, part_f);
      prof_mark(pl, s, timed, 1 + kind, 0.0, false);
    } else if (sizeof(real) == 8) {
      // FP64: the two recurrences of a pair need too many registers for one
      // pass (one wave per SIMD); each kernel in a launch of its own
      if (ks == KS_LY)
        launch_m2p<real, 0, -1>(pl, s, u, tx, ty, tz, mom, 0, part_f);
      else
        launch_m2p<real, 1, -1>(pl, s, u, tx, ty, tz, mom, 0, part_f);
      launch_m2p<real, 1, -1>(pl, s, u, tx, ty, tz, mom, 1, part_f);
    } else {
      // two kernels (Laplace + Yukawa, or two Yukawa) in one pass
      prof_mark(pl, s, timed, kProfM2PPair, pl.launch_flop_m2p[phase][ks], true);
      if (ks == KS_LY)
        launch_m2p<real, 0, 1>(pl, s, u, tx, ty, tz, mom, 0, part_f);
      else
        launch_m2p<real, 1, 1>(pl, s, u, tx, ty, tz, mom, 0, part_f);
      prof_mark(pl, s, timed, kProfM2PPair, 0.0, false);
    }
    PBTC_LAUNCH_CHECK();
    return PBTC_OK;
  };
  // S and D of kernel set ks += the sums of its near units (near) or of its
  // far units (!near)
  auto reduce = [&](int ks, bool near, hipStream_t s) -> int {
    const int n = (int)pl.item_list[phase][ks].size();
    const int* list = wsp<int>(pl, pl.o_item_list[phase][ks]);
    const UnitSet& un = pl.units[phase][ks][0];
    const UnitSet& uf = pl.units[phase][ks][1];
    const int* uptr_n = near ? wsp<int>(pl, pl.o_uptr + 4 * un.ptr_off) : nullptr;
    const real* part_n = near ? partial + (size_t)un.off * 4 * kGroup : nullptr;
    const int* uptr_f = near ? nullptr : wsp<int>(pl, pl.o_uptr + 4 * uf.ptr_off);
    const real* part_f = near ? nullptr : partial + (size_t)uf.off * 4 * kGroup;
    if (ks == KS_L || ks == KS_Y)
      hipLaunchKernelGGL((k_reduce<real, 2>), dim3(nblocks(n, kReduceWaves)),
                         dim3(64 * kReduceWaves), 0, s, n, list, uptr_n, part_n, uptr_f, part_f,
                         a.item_block, a.blocks, tidx, S, D);
    else
      hipLaunchKernelGGL((k_reduce<real, 4>), dim3(nblocks(n, kReduceWaves)),
                         dim3(64 * kReduceWaves), 0, s, n, list, uptr_n, part_n, uptr_f, part_f,
                         a.item_block, a.blocks, tidx, S, D);
    PBTC_LAUNCH_CHECK();
    return PBTC_OK;
  };
  // near-field corrections of this phase's blocks: they store S and D of
  // every row, which the reductions then add to (on the main stream, beside
  // the far field)
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
  int rc = PBTC_OK;
  if (fork) {
    for (int ks = 0; ks < KS_COUNT && !rc; ++ks)
      if (!pl.item_list[phase][ks].empty() && has_far(ks)) rc = m2p(ks, pl.side);
    if (rc) return rc;
    PBTC_HIP(hipEventRecord(pl.ev_join, pl.side));
    // the near units' sums are added while the far field still runs
    for (int ks = 0; ks < KS_COUNT && !rc; ++ks)
      if (!pl.item_list[phase][ks].empty()) {
        rc = p2p(ks, st);
        if (!rc) rc = reduce(ks, true, st);
      }
    if (rc) return rc;
    PBTC_HIP(hipStreamWaitEvent(st, pl.ev_join, 0));
    for (int ks = 0; ks < KS_COUNT && !rc; ++ks)
      if (!pl.item_list[phase][ks].empty() && has_far(ks)) rc = reduce(ks, false, st);
  } else {
    for (int ks = 0; ks < KS_COUNT && !rc; ++ks) {
      if (pl.item_list[phase][ks].empty()) continue;
      rc = p2p(ks, st);
      if (!rc) rc = reduce(ks, true, st);
      if (!rc && has_far(ks)) rc = m2p(ks, st);
      if (!rc && has_far(ks)) rc = reduce(ks, false, st);
    }
  }
  if (rc) return rc;
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
    // the first evaluation after a set-up runs kernel by kernel, the second
    // captures the graph that the later ones replay: an operator used once
    // per set-up (the FP64 residual of a refined solve, the reaction
    // potential) costs no capture
    if (pl.op_direct_gen[p][phase] != pl.setup_gen) {
      pl.op_direct_gen[p][phase] = pl.setup_gen;
      return fp32 ? apply_impl<float>(pl, st, x, y, phase) : apply_impl<double>(pl, st, x, y, phase);
    }
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
