// Problem description and host-side validation (no device work).
//
// The problem statement follows sec. 2.1 (Eq. pde) and sec. 2.2 (multi-surface
// problems): dielectric regions with permittivity eps and inverse Debye
// length kappa, closed surfaces separating an inner from an outer region,
// point charges inside one region.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <unordered_map>

#include "internal.h"

namespace pbtc {

bool triangle_rule(int k, double* bary, double* w);
bool gauss_legendre(int n, double* x, double* w);

namespace {

bool finite(double v) { return std::isfinite(v); }

struct EdgeKey {
  uint64_t operator()(const std::pair<int32_t, int32_t>& e) const {
    return (uint64_t(uint32_t(e.first)) << 32) ^ uint64_t(uint32_t(e.second)) * 0x9E3779B97F4A7C15ull;
  }
};

// Uniform grid over the (y, z) projections of a surface's triangles, for
// parity counts of rays cast along +x.
struct RayGrid {
  const Surface* s = nullptr;
  double y0 = 0, z0 = 0, dy = 1, dz = 1;
  int ny = 1, nz = 1;
  std::vector<int> start, list;

  void build(const Surface& surf) {
    s = &surf;
    const int64_t np = surf.np();
    double ymin = 1e300, ymax = -1e300, zmin = 1e300, zmax = -1e300;
    for (int64_t i = 0; i < surf.nv(); ++i) {
      ymin = std::min(ymin, surf.v[3 * i + 1]);
      ymax = std::max(ymax, surf.v[3 * i + 1]);
      zmin = std::min(zmin, surf.v[3 * i + 2]);
      zmax = std::max(zmax, surf.v[3 * i + 2]);
    }
    const int n = std::max(1, (int)std::sqrt((double)np / 2.0));
    ny = nz = n;
    y0 = ymin;
    z0 = zmin;
    dy = std::max((ymax - ymin) / n, 1e-12);
    dz = std::max((zmax - zmin) / n, 1e-12);
    std::vector<int> cnt(ny * nz + 1, 0);
    auto cells = [&](int64_t t, int& a0, int& a1, int& b0, int& b1) {
      double lo_y = 1e300, hi_y = -1e300, lo_z = 1e300, hi_z = -1e300;
      for (int k = 0; k < 3; ++k) {
        const double* p = &surf.v[3 * surf.t[3 * t + k]];
        lo_y = std::min(lo_y, p[1]);
        hi_y = std::max(hi_y, p[1]);
        lo_z = std::min(lo_z, p[2]);
        hi_z = std::max(hi_z, p[2]);
      }
      a0 = std::clamp((int)std::floor((lo_y - y0) / dy), 0, ny - 1);
      a1 = std::clamp((int)std::floor((hi_y - y0) / dy), 0, ny - 1);
      b0 = std::clamp((int)std::floor((lo_z - z0) / dz), 0, nz - 1);
      b1 = std::clamp((int)std::floor((hi_z - z0) / dz), 0, nz - 1);
    };
    for (int64_t t = 0; t < np; ++t) {
      int a0, a1, b0, b1;
      cells(t, a0, a1, b0, b1);
      for (int a = a0; a <= a1; ++a)
        for (int b = b0; b <= b1; ++b) cnt[a * nz + b + 1]++;
    }
    for (int i = 0; i < ny * nz; ++i) cnt[i + 1] += cnt[i];
    start = cnt;
    list.assign(cnt[ny * nz], 0);
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t t = 0; t < np; ++t) {
      int a0, a1, b0, b1;
      cells(t, a0, a1, b0, b1);
      for (int a = a0; a <= a1; ++a)
        for (int b = b0; b <= b1; ++b) list[fill[a * nz + b]++] = (int)t;
    }
  }

  // +1 inside, 0 outside, -1 degenerate (ray grazes an edge or vertex)
  int inside(double x, double y, double z) const {
    if (y < y0 || z < z0) return 0;
    const int a = (int)std::floor((y - y0) / dy), b = (int)std::floor((z - z0) / dz);
    if (a >= ny || b >= nz) return 0;
    int crossings = 0;
    for (int i = start[a * nz + b]; i < start[a * nz + b + 1]; ++i) {
      const int t = list[i];
      const double* p0 = &s->v[3 * s->t[3 * t + 0]];
      const double* p1 = &s->v[3 * s->t[3 * t + 1]];
      const double* p2 = &s->v[3 * s->t[3 * t + 2]];
      // signed areas in the (y, z) plane
      const double e0 = (p1[1] - p0[1]) * (z - p0[2]) - (p1[2] - p0[2]) * (y - p0[1]);
      const double e1 = (p2[1] - p1[1]) * (z - p1[2]) - (p2[2] - p1[2]) * (y - p1[1]);
      const double e2 = (p0[1] - p2[1]) * (z - p2[2]) - (p0[2] - p2[2]) * (y - p2[1]);
      const double scale = 1e-12 * (std::fabs(e0) + std::fabs(e1) + std::fabs(e2) + 1e-300);
      const bool pos = e0 > scale && e1 > scale && e2 > scale;
      const bool neg = e0 < -scale && e1 < -scale && e2 < -scale;
      if (!pos && !neg) {
        const bool maybe = (e0 >= -scale && e1 >= -scale && e2 >= -scale) ||
                           (e0 <= scale && e1 <= scale && e2 <= scale);
        if (maybe) return -1;
        continue;
      }
      // x of the plane through the triangle at (y, z)
      const double w0 = e1, w1 = e2, w2 = e0, ws = w0 + w1 + w2;
      const double xt = (w0 * p0[0] + w1 * p1[0] + w2 * p2[0]) / ws;
      if (xt > x) crossings++;
    }
    return crossings & 1;
  }
};

}  // namespace

std::string validate_problem(const pbtc_problem& p, const pbtc_params& prm, int* code) {
  char buf[512];
  auto fail = [&](int c, const char* msg) {
    *code = c;
    return std::string(msg);
  };
  *code = PBTC_OK;
  // parameters
  double tb[3 * kMaxRule], tw[kMaxRule];
  if (prm.K != 1 && prm.K != 3 && prm.K != 4 && prm.K != 7)
    return fail(PBTC_EINVAL, "K must be 1, 3, 4 or 7");
  if (prm.K_fine != 7 && prm.K_fine != 19) return fail(PBTC_EINVAL, "K_fine must be 7 or 19");
  if (!triangle_rule(prm.K, tb, tw)) return fail(PBTC_EINVAL, "bad K");
  if (prm.N_k < 1 || prm.N_k > kMaxNk) return fail(PBTC_EINVAL, "N_k must be in 1..32");
  if (!(prm.thres >= 0.0) || !finite(prm.thres)) return fail(PBTC_EINVAL, "thres must be >= 0");
  if (!(prm.theta > 0.0 && prm.theta < 1.0)) return fail(PBTC_EINVAL, "theta must be in (0, 1)");
  if (prm.P != 2 && prm.P != 4 && prm.P != 6 && prm.P != 8 && prm.P != 10)
    return fail(PBTC_EINVAL, "P must be 2, 4, 6, 8 or 10");
  if (prm.ncrit < 0 || prm.ncrit == 1 || prm.ncrit > kSpanSources)
    return fail(PBTC_EINVAL, "ncrit must be 0 (auto) or in 2..256");
  if (!(prm.tol > 0.0 && prm.tol < 1.0)) return fail(PBTC_EINVAL, "tol must be in (0, 1)");
  if (prm.restart < 1 || prm.restart > 256) return fail(PBTC_EINVAL, "restart must be in 1..256");
  if (prm.max_iter < 1) return fail(PBTC_EINVAL, "max_iter must be >= 1");
  if (prm.precision < PBTC_FP64 || prm.precision > PBTC_FP32)
    return fail(PBTC_EINVAL, "unknown precision");
  if (prm.op != PBTC_OP_TREECODE && prm.op != PBTC_OP_DIRECT) return fail(PBTC_EINVAL, "unknown op");
  if (!(prm.inner_tol > 0.0 && prm.inner_tol < 1.0)) return fail(PBTC_EINVAL, "inner_tol must be in (0, 1)");
  if (prm.max_refine < 1) return fail(PBTC_EINVAL, "max_refine must be >= 1");
  if (prm.profile < 0) return fail(PBTC_EINVAL, "profile must be >= 0");
  if (prm.precond != PBTC_PREC_NONE && prm.precond != PBTC_PREC_BLOCK_DIAG)
    return fail(PBTC_EINVAL, "unknown precond");
  if (prm.op_graph != 0 && prm.op_graph != 1) return fail(PBTC_EINVAL, "op_graph must be 0 or 1");
  if (prm.unit_sources != 0 && (prm.unit_sources < 64 || prm.unit_sources > 8192))
    return fail(PBTC_EINVAL, "unit_sources must be 0 (auto) or in 64..8192");
  if (prm.unit_cells != 0 && (prm.unit_cells < 1 || prm.unit_cells > 1024))
    return fail(PBTC_EINVAL, "unit_cells must be 0 (auto) or in 1..1024");
  // regions
  const int nreg = (int)p.regions.size();
  if (nreg < 2) return fail(PBTC_EINVAL, "need at least two regions");
  for (int r = 0; r < nreg; ++r) {
    if (!(p.regions[r].eps > 0.0) || !finite(p.regions[r].eps) || !(p.regions[r].kappa >= 0.0) ||
        !finite(p.regions[r].kappa)) {
      std::snprintf(buf, sizeof buf, "region %d: eps must be > 0 and kappa >= 0, finite", r);
      return fail(PBTC_EINVAL, buf);
    }
  }
  if (p.surfaces.empty()) return fail(PBTC_EINVAL, "no surface");
  std::vector<int> bounded(nreg, 0);
  for (size_t si = 0; si < p.surfaces.size(); ++si) {
    const Surface& s = p.surfaces[si];
    bounded[s.inner]++;
    bounded[s.outer]++;
    for (double v : s.v)
      if (!finite(v)) {
        std::snprintf(buf, sizeof buf, "surface %zu: vertex coordinate not finite", si);
        return fail(PBTC_EINVAL, buf);
      }
    // closedness: every directed edge once, its reverse once
    std::unordered_map<std::pair<int32_t, int32_t>, int, EdgeKey> edges;
    edges.reserve(3 * s.np());
    double vol = 0.0;
    for (int64_t t = 0; t < s.np(); ++t) {
      const int32_t a = s.t[3 * t], b = s.t[3 * t + 1], c = s.t[3 * t + 2];
      const double* A = &s.v[3 * a];
      const double* B = &s.v[3 * b];
      const double* C = &s.v[3 * c];
      const double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
      const double e2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
      const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                           e1[0] * e2[1] - e1[1] * e2[0]};
      const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      const double l2 = std::max(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2],
                                 e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
      if (!(nn > 1e-10 * l2) || a == b || b == c || a == c) {
        std::snprintf(buf, sizeof buf, "surface %zu: degenerate triangle %lld", si, (long long)t);
        return fail(PBTC_EMESH, buf);
      }
      vol += A[0] * (B[1] * C[2] - B[2] * C[1]) - A[1] * (B[0] * C[2] - B[2] * C[0]) +
             A[2] * (B[0] * C[1] - B[1] * C[0]);
      const int32_t es[3][2] = {{a, b}, {b, c}, {c, a}};
      for (auto& e : es) {
        if (++edges[{e[0], e[1]}] > 1) {
          std::snprintf(buf, sizeof buf,
                        "surface %zu: edge (%d, %d) used twice in the same direction "
                        "(inconsistent orientation or non-manifold)",
                        si, e[0], e[1]);
          return fail(PBTC_EMESH, buf);
        }
      }
    }
    for (auto& kv : edges) {
      if (edges.find({kv.first.second, kv.first.first}) == edges.end()) {
        std::snprintf(buf, sizeof buf, "surface %zu: open at edge (%d, %d)", si, kv.first.first,
                      kv.first.second);
        return fail(PBTC_EMESH, buf);
      }
    }
    if (!(vol > 0.0)) {
      std::snprintf(buf, sizeof buf,
                    "surface %zu: triangles must be counter-clockwise seen from the outer "
                    "region (enclosed volume %.3g <= 0)",
                    si, vol / 6.0);
      return fail(PBTC_EMESH, buf);
    }
  }
  for (int r = 0; r < nreg; ++r)
    if (!bounded[r]) {
      std::snprintf(buf, sizeof buf, "region %d touches no surface", r);
      return fail(PBTC_EINVAL, buf);
    }
  // charges
  int64_t nq = 0;
  for (int r = 0; r < nreg; ++r) {
    const ChargeSet& c = p.charges[r];
    nq += c.n();
    for (double v : c.xyz)
      if (!finite(v)) return fail(PBTC_EINVAL, "charge position not finite");
    for (double v : c.q)
      if (!finite(v)) return fail(PBTC_EINVAL, "charge value not finite");
  }
  if (nq == 0) return fail(PBTC_EINVAL, "no charges");
  if (prm.validate_charges) {
    std::vector<RayGrid> grids(p.surfaces.size());
    for (size_t si = 0; si < p.surfaces.size(); ++si) grids[si].build(p.surfaces[si]);
    for (int r = 0; r < nreg; ++r) {
      const ChargeSet& c = p.charges[r];
      for (int64_t k = 0; k < c.n(); ++k) {
        for (size_t si = 0; si < p.surfaces.size(); ++si) {
          const Surface& s = p.surfaces[si];
          if (s.inner != r && s.outer != r) continue;
          double x = c.xyz[3 * k], y = c.xyz[3 * k + 1], z = c.xyz[3 * k + 2];
          int in = grids[si].inside(x, y, z);
          for (int tries = 1; in < 0 && tries < 8; ++tries) {
            // nudge the ray off an edge or vertex it grazes
            in = grids[si].inside(x, y + 1.3e-7 * tries, z - 0.7e-7 * tries);
          }
          if (in < 0) in = 0;
          if ((in == 1) != (s.inner == r)) {
            std::snprintf(buf, sizeof buf,
                          "charge %lld of region %d lies %s surface %zu, so it is not in its region",
                          (long long)k, r, in ? "inside" : "outside", si);
            return fail(PBTC_ECHARGE, buf);
          }
        }
      }
    }
  }
  return std::string();
}

}  // namespace pbtc
