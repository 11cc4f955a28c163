// Plan construction: block structure of the operator and workspace layout.
//
// Multi-surface formulation (sec. 2.2; the paper defers the derivation to
// Altman et al., this is Green's third identity written in every region):
// surface s separates its inner region I(s) from its outer region O(s) and
// carries phi_s and psi_s (d phi / dn on the inner side).  Region r is
// bounded by B(r) = {s : r in {I(s), O(s)}}, with sigma_rs = +1 if I(s) = r
// else -1 and c_rs = 1 if I(s) = r else eps_I(s) / eps_r.  The rows of
// surface t seen from region r in {I(t), O(t)} are
//   1/2 phi_t - sum_{s in B(r)} sigma_rs (c_rs V_r^{ts} psi_s - K_r^{ts} phi_s)
//     = sum_{k in r} q_k / eps_r G_r(x, x_k),
// which for one surface is Eq. matrix.  The reaction potential at a charge
// in region r is sum_{s in B(r)} sigma_rs (c_rs V_r psi_s - K_r phi_s)
// (Eq. reac_integral).
//
// A block is the interaction of one target set (a surface's collocation
// points, or the charges of a region) with the Gauss points of one source
// surface; the moments of a surface do not depend on the Green's function,
// so a block evaluates every distinct kernel (Laplace or Yukawa with a
// given kappa) that any region containing both needs, from one tree walk.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>

#include "internal.h"

namespace pbtc {

bool triangle_rule(int k, double* bary, double* w);
bool gauss_legendre(int n, double* x, double* w);
std::string validate_problem(const pbtc_problem& p, const pbtc_params& prm, int* code);

namespace {

int kernel_set(int nk, const double* kap) {
  if (nk == 1) return kap[0] == 0.0 ? KS_L : KS_Y;
  if (kap[0] == 0.0) return KS_LY;
  return KS_YY;
}

}  // namespace

void compute_layout(pbtc_plan_t& pl);

int build_plan(pbtc_plan_t& pl) {
  const pbtc_problem& P = pl.prob;
  pl.nsurf = (int)P.surfaces.size();
  pl.nreg = (int)P.regions.size();
  pl.P = pl.prm.P;
  pl.ncrit = pl.prm.ncrit > 0 ? pl.prm.ncrit : 128;
  const int nP = ncoef(pl.P);
  pl.direct_below = pl.prm.direct_below >= 0 ? pl.prm.direct_below : nP / 2;
  triangle_rule(pl.prm.K, pl.rule_b, pl.rule_w);
  triangle_rule(pl.prm.K_fine, pl.fine_b, pl.fine_w);
  gauss_legendre(pl.prm.N_k, pl.gl_x, pl.gl_w);

  // panels, vertices, Gauss points, unknowns
  pl.pan_off.assign(pl.nsurf + 1, 0);
  pl.v_off.assign(pl.nsurf + 1, 0);
  pl.gp_off.assign(pl.nsurf + 1, 0);
  pl.unk_off.assign(pl.nsurf + 1, 0);
  for (int s = 0; s < pl.nsurf; ++s) {
    pl.pan_off[s + 1] = pl.pan_off[s] + P.surfaces[s].np();
    pl.v_off[s + 1] = pl.v_off[s] + P.surfaces[s].nv();
    pl.gp_off[s + 1] = pl.gp_off[s] + P.surfaces[s].np() * pl.prm.K;
    pl.unk_off[s + 1] = pl.unk_off[s] + 2 * P.surfaces[s].np();
  }
  pl.np_tot = pl.pan_off[pl.nsurf];
  pl.nv_tot = pl.v_off[pl.nsurf];
  pl.ngp = pl.gp_off[pl.nsurf];
  pl.nunk = pl.unk_off[pl.nsurf];
  pl.q_off_region.assign(pl.nreg + 1, 0);
  for (int r = 0; r < pl.nreg; ++r) pl.q_off_region[r + 1] = pl.q_off_region[r] + P.charges[r].n();
  pl.nq = pl.q_off_region[pl.nreg];
  if (pl.ngp >= (int64_t(1) << 31) - 1 || pl.np_tot >= (int64_t(1) << 30))
    return PBTC_EINVAL;

  // target sets: surfaces, then the charge set of every region with charges
  pl.tsets.clear();
  pl.tset_of_surface.assign(pl.nsurf, -1);
  pl.tset_of_region.assign(pl.nreg, -1);
  int64_t toff = 0, goff = 0;
  for (int s = 0; s < pl.nsurf; ++s) {
    TargetSet ts;
    ts.kind = 0;
    ts.id = s;
    ts.off = toff;
    ts.n = P.surfaces[s].np();
    ts.grp_off = goff;
    ts.ngrp = (ts.n + kGroup - 1) / kGroup;
    toff += ts.n;
    goff += ts.ngrp;
    pl.tset_of_surface[s] = (int)pl.tsets.size();
    pl.tsets.push_back(ts);
  }
  for (int r = 0; r < pl.nreg; ++r) {
    if (P.charges[r].n() == 0) continue;
    TargetSet ts;
    ts.kind = 1;
    ts.id = r;
    ts.off = toff;
    ts.n = P.charges[r].n();
    ts.grp_off = goff;
    ts.ngrp = (ts.n + kGroup - 1) / kGroup;
    toff += ts.n;
    goff += ts.ngrp;
    pl.tset_of_region[r] = (int)pl.tsets.size();
    pl.tsets.push_back(ts);
  }
  pl.ntgt = toff;
  pl.ngrp = goff;

  auto inner = [&](int s) { return P.surfaces[s].inner; };
  auto outer = [&](int s) { return P.surfaces[s].outer; };
  auto bounds = [&](int r, int s) { return inner(s) == r || outer(s) == r; };
  auto sigma = [&](int r, int s) { return inner(s) == r ? 1.0 : -1.0; };
  auto ratio = [&](int r, int s) {
    return inner(s) == r ? 1.0 : P.regions[inner(s)].eps / P.regions[r].eps;
  };

  // forward blocks
  pl.blocks.clear();
  std::vector<int> fwd_block(pl.nsurf * pl.nsurf, -1);
  int64_t out = 0, items = 0;
  pl.dense_equiv = 0.0;
  for (int t = 0; t < pl.nsurf; ++t) {
    for (int s = 0; s < pl.nsurf; ++s) {
      Block b;
      b.t = pl.tset_of_surface[t];
      b.s = s;
      b.nk = 0;
      for (int r : {inner(t), outer(t)}) {
        if (!bounds(r, s)) continue;
        const double k = P.regions[r].kappa;
        bool seen = false;
        for (int i = 0; i < b.nk; ++i) seen |= (b.kappa[i] == k);
        if (!seen) b.kappa[b.nk++] = k;
      }
      if (b.nk == 0) continue;
      if (b.nk == 2 && b.kappa[1] == 0.0) std::swap(b.kappa[0], b.kappa[1]);
      b.ks = kernel_set(b.nk, b.kappa);
      for (int i = 0; i < b.nk; ++i) {
        b.out[i] = out;
        out += pl.tsets[b.t].n;
      }
      b.item_off = items;
      items += pl.tsets[b.t].ngrp;
      fwd_block[t * pl.nsurf + s] = (int)pl.blocks.size();
      pl.blocks.push_back(b);
    }
  }
  auto kidx = [&](const Block& b, double k) { return b.kappa[0] == k ? 0 : 1; };
  // rows
  pl.rows.clear();
  for (int t = 0; t < pl.nsurf; ++t) {
    const int64_t nt = P.surfaces[t].np();
    int half = 0;
    for (int r : {inner(t), outer(t)}) {
      RowBlock rb;
      rb.t = t;
      rb.r = r;
      rb.row_off = pl.unk_off[t] + half * nt;
      rb.n = nt;
      rb.phi_off = pl.unk_off[t];
      int64_t src = 0;
      for (int s = 0; s < pl.nsurf; ++s) {
        if (!bounds(r, s)) continue;
        const int bi = fwd_block[t * pl.nsurf + s];
        RowTerm term;
        term.block = bi;
        term.kidx = kidx(pl.blocks[bi], P.regions[r].kappa);
        term.sigma_c = sigma(r, s) * ratio(r, s);
        term.sigma = sigma(r, s);
        rb.terms.push_back(term);
        src += P.surfaces[s].np() * pl.prm.K;
      }
      pl.dense_equiv += double(nt) * double(src);
      pl.rows.push_back(rb);
      ++half;
    }
  }
  // reaction blocks and rows
  pl.reac_rows.clear();
  for (int r = 0; r < pl.nreg; ++r) {
    if (pl.tset_of_region[r] < 0) continue;
    RowBlock rb;
    rb.t = pl.tset_of_region[r];
    rb.r = r;
    rb.row_off = pl.q_off_region[r];
    rb.n = P.charges[r].n();
    rb.phi_off = 0;
    for (int s = 0; s < pl.nsurf; ++s) {
      if (!bounds(r, s)) continue;
      Block b;
      b.t = pl.tset_of_region[r];
      b.s = s;
      b.nk = 1;
      b.kappa[0] = P.regions[r].kappa;
      b.ks = kernel_set(1, b.kappa);
      b.reaction = true;
      b.out[0] = out;
      out += pl.tsets[b.t].n;
      b.item_off = items;
      items += pl.tsets[b.t].ngrp;
      RowTerm term;
      term.block = (int)pl.blocks.size();
      term.kidx = 0;
      term.sigma_c = sigma(r, s) * ratio(r, s);
      term.sigma = sigma(r, s);
      rb.terms.push_back(term);
      pl.blocks.push_back(b);
    }
    pl.reac_rows.push_back(rb);
  }
  pl.nout = out;
  pl.nitems = items;
  // near-field rows (one per target of every block), forward blocks first
  int64_t nfr = 0;
  pl.nf_fwd_rows = 0;
  for (Block& b : pl.blocks) {
    b.nf_row = nfr;
    nfr += pl.tsets[b.t].n;
    if (!b.reaction) pl.nf_fwd_rows = nfr;
  }
  pl.nf_rows = nfr;
  // items: (block, group) pairs, and per-kernel-set launch lists
  pl.item_block.assign(pl.nitems, 0);
  for (int ph = 0; ph < 2; ++ph)
    for (int ks = 0; ks < KS_COUNT; ++ks) pl.item_list[ph][ks].clear();
  for (size_t bi = 0; bi < pl.blocks.size(); ++bi) {
    const Block& b = pl.blocks[bi];
    for (int64_t g = 0; g < pl.tsets[b.t].ngrp; ++g) {
      pl.item_block[b.item_off + g] = (int)bi;
      pl.item_list[b.reaction ? 1 : 0][b.ks].push_back((int)(b.item_off + g));
    }
  }

  // host-side geometric bounds per surface: bounding cube, max panel length,
  // max distance from a panel centre to its vertices
  pl.cube.assign(4 * pl.nsurf, 0.0);
  pl.max_len.assign(pl.nsurf, 0.0);
  pl.max_reach.assign(pl.nsurf, 0.0);
  for (int s = 0; s < pl.nsurf; ++s) {
    const Surface& S = P.surfaces[s];
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < S.nv(); ++i)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], S.v[3 * i + d]);
        hi[d] = std::max(hi[d], S.v[3 * i + d]);
      }
    double half = 0.0;
    for (int d = 0; d < 3; ++d) {
      pl.cube[4 * s + d] = 0.5 * (lo[d] + hi[d]);
      half = std::max(half, 0.5 * (hi[d] - lo[d]));
    }
    pl.cube[4 * s + 3] = half * (1.0 + 1e-6) + 1e-9;
    for (int64_t t = 0; t < S.np(); ++t) {
      const double* a = &S.v[3 * S.t[3 * t]];
      const double* b = &S.v[3 * S.t[3 * t + 1]];
      const double* c = &S.v[3 * S.t[3 * t + 2]];
      const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
      const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
      const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                           e1[0] * e2[1] - e1[1] * e2[0]};
      const double area = 0.5 * std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      pl.max_len[s] = std::max(pl.max_len[s], std::sqrt(2.0 * area));
      double cen[3];
      for (int d = 0; d < 3; ++d) cen[d] = (a[d] + b[d] + c[d]) / 3.0;
      for (const double* v : {a, b, c}) {
        const double dd = std::sqrt((v[0] - cen[0]) * (v[0] - cen[0]) +
                                    (v[1] - cen[1]) * (v[1] - cen[1]) +
                                    (v[2] - cen[2]) * (v[2] - cen[2]));
        pl.max_reach[s] = std::max(pl.max_reach[s], dd);
      }
    }
  }

  // independent systems: connected components of regions linked by surfaces;
  // each must own a contiguous run of surfaces (else one system is used)
  {
    std::vector<int> parent(pl.nreg);
    for (int r = 0; r < pl.nreg; ++r) parent[r] = r;
    std::function<int(int)> find = [&](int r) { return parent[r] == r ? r : parent[r] = find(parent[r]); };
    for (int s = 0; s < pl.nsurf; ++s) {
      const int a = find(inner(s)), b = find(outer(s));
      if (a != b) parent[a] = b;
    }
    std::vector<int> label(pl.nreg, -1);
    pl.comp_of_surface.assign(pl.nsurf, 0);
    int nc = 0;
    for (int s = 0; s < pl.nsurf; ++s) {
      const int root = find(inner(s));
      if (label[root] < 0) label[root] = nc++;
      pl.comp_of_surface[s] = label[root];
    }
    bool contiguous = true;
    for (int s = 1; s < pl.nsurf; ++s)
      if (pl.comp_of_surface[s] < pl.comp_of_surface[s - 1] ||
          pl.comp_of_surface[s] > pl.comp_of_surface[s - 1] + 1)
        contiguous = false;
    if (!contiguous) {
      nc = 1;
      std::fill(pl.comp_of_surface.begin(), pl.comp_of_surface.end(), 0);
    }
    pl.ncomp = std::max(nc, 1);
    pl.comp_of_region.assign(pl.nreg, 0);
    for (int r = 0; r < pl.nreg; ++r)
      pl.comp_of_region[r] = contiguous && label[find(r)] >= 0 ? label[find(r)] : 0;
    pl.comp_u0.assign(pl.ncomp, 0);
    pl.comp_u1.assign(pl.ncomp, 0);
    for (int c = 0; c < pl.ncomp; ++c) {
      int64_t lo = pl.nunk, hi = 0;
      for (int s = 0; s < pl.nsurf; ++s)
        if (pl.comp_of_surface[s] == c) {
          lo = std::min(lo, pl.unk_off[s]);
          hi = std::max(hi, pl.unk_off[s + 1]);
        }
      pl.comp_u0[c] = lo;
      pl.comp_u1[c] = hi;
    }
    // Krylov reduction chunks never straddle two systems
    constexpr int64_t kChunk = kDotChunk;
    pl.dot_chunks.clear();
    pl.comp_chunk0.assign(pl.ncomp + 1, 0);
    for (int c = 0; c < pl.ncomp; ++c) {
      pl.comp_chunk0[c] = (int)pl.dot_chunks.size();
      for (int64_t a = pl.comp_u0[c]; a < pl.comp_u1[c]; a += kChunk)
        pl.dot_chunks.push_back(make_int4(c, (int)a, (int)std::min(a + kChunk, pl.comp_u1[c]), 0));
    }
    pl.comp_chunk0[pl.ncomp] = (int)pl.dot_chunks.size();
    pl.coul_host.assign(2 * (size_t)pl.nreg + 1 + (size_t)pl.ncomp, 0.0);
  }

  // transposed operator: Gauss-point groups, items, kernel slots, CSC columns
  pl.gpgrp_off.assign(pl.nsurf + 1, 0);
  for (int s = 0; s < pl.nsurf; ++s)
    pl.gpgrp_off[s + 1] = pl.gpgrp_off[s] + (pl.gp_off[s + 1] - pl.gp_off[s] + kAGroup - 1) / kAGroup;
  pl.ngpgrp = pl.gpgrp_off[pl.nsurf];
  const size_t nb = pl.blocks.size();
  pl.blk_slot0.assign(nb, 0);
  pl.blk_aout0.assign(nb, 0);
  pl.blk_aout1.assign(nb, 0);
  pl.blk_aitem_off.assign(nb, 0);
  pl.blk_csc_off.assign(nb, 0);
  pl.aitem_block.clear();
  for (int ph = 0; ph < 2; ++ph)
    for (int ks = 0; ks < KS_COUNT; ++ks) pl.aitem_list[ph][ks].clear();
  int64_t nslot = 0, aout = 0, aitems = 0, ncsc = 0;
  // transposed moments live per cell of a target-set tree, one record per
  // kernel slot of the blocks on that tree: local slot numbers per tree
  pl.blk_lslot0.assign(nb, 0);
  {
    std::vector<int> per_tree(pl.tsets.size(), 0);
    pl.adj_ms = 1;
    for (size_t bi = 0; bi < nb; ++bi) {
      const Block& b = pl.blocks[bi];
      pl.blk_lslot0[bi] = per_tree[b.t];
      per_tree[b.t] += b.nk;
      pl.adj_ms = std::max(pl.adj_ms, per_tree[b.t]);
    }
  }
  for (size_t bi = 0; bi < nb; ++bi) {
    const Block& b = pl.blocks[bi];
    const int64_t ngs = pl.gp_off[b.s + 1] - pl.gp_off[b.s];
    pl.blk_slot0[bi] = nslot;
    pl.blk_aout0[bi] = aout;
    pl.blk_aout1[bi] = aout + (b.nk == 2 ? ngs : 0);
    nslot += b.nk;
    aout += b.nk * ngs;
    pl.blk_aitem_off[bi] = aitems;
    const int64_t ng = pl.gpgrp_off[b.s + 1] - pl.gpgrp_off[b.s];
    for (int64_t g = 0; g < ng; ++g) {
      pl.aitem_block.push_back((int)bi);
      pl.aitem_list[b.reaction ? 1 : 0][b.ks].push_back((int)(aitems + g));
    }
    aitems += ng;
    pl.blk_csc_off[bi] = ncsc;
    ncsc += pl.pan_off[b.s + 1] - pl.pan_off[b.s];
  }
  pl.nitems_adj = aitems;
  pl.naout = aout;
  pl.ncsc = ncsc;
  // kernel slots: weights from the rows that use each (block, kernel)
  for (int ph = 0; ph < 2; ++ph) {
    pl.slots[ph].clear();
    pl.gather_slots[ph].clear();
    pl.gathers[ph].assign(pl.nsurf, DevGather{0, 0});
  }
  std::vector<DevSlot> all(nslot);
  for (size_t bi = 0; bi < nb; ++bi) {
    const Block& b = pl.blocks[bi];
    for (int k = 0; k < b.nk; ++k) {
      DevSlot& d = all[pl.blk_slot0[bi] + k];
      d.out = b.out[k];
      d.n = pl.tsets[b.t].n;
      d.ncontrib = 0;
      d.block = (int)bi;
      d.lam_off[0] = d.lam_off[1] = 0;
      d.cS[0] = d.cS[1] = d.cD[0] = d.cD[1] = 0.0;
    }
  }
  // forward rows: row = 1/2 phi - sum sigma (c S - D)  ->  muS += -sigma c lam, muD += sigma lam
  for (const RowBlock& rb : pl.rows)
    for (const RowTerm& t : rb.terms) {
      DevSlot& d = all[pl.blk_slot0[t.block] + t.kidx];
      d.lam_off[d.ncontrib] = rb.row_off;
      d.cS[d.ncontrib] = -t.sigma_c;
      d.cD[d.ncontrib] = t.sigma;
      ++d.ncontrib;
    }
  // reaction rows: phi_reac = sum sigma (c S - D)  ->  muS += sigma c q, muD += -sigma q
  for (const RowBlock& rb : pl.reac_rows)
    for (const RowTerm& t : rb.terms) {
      DevSlot& d = all[pl.blk_slot0[t.block] + t.kidx];
      d.lam_off[d.ncontrib] = rb.row_off;
      d.cS[d.ncontrib] = t.sigma_c;
      d.cD[d.ncontrib] = -t.sigma;
      ++d.ncontrib;
    }
  for (int ph = 0; ph < 2; ++ph) {
    for (int s = 0; s < pl.nsurf; ++s) {
      pl.gathers[ph][s].slot_off = (int)pl.gather_slots[ph].size();
      for (size_t bi = 0; bi < nb; ++bi) {
        const Block& b = pl.blocks[bi];
        if (b.s != s || (b.reaction ? 1 : 0) != ph) continue;
        for (int k = 0; k < b.nk; ++k) pl.gather_slots[ph].push_back((int)(pl.blk_slot0[bi] + k));
      }
      pl.gathers[ph][s].nslots = (int)pl.gather_slots[ph].size() - pl.gathers[ph][s].slot_off;
    }
    for (const DevSlot& d : all)
      if (pl.blocks[d.block].reaction == (ph == 1)) pl.slots[ph].push_back(d);
  }

  // bounding cubes of the target sets (Morton order of the targets)
  pl.tcube.assign(4 * pl.tsets.size(), 0.0);
  for (size_t ti = 0; ti < pl.tsets.size(); ++ti) {
    const TargetSet& ts = pl.tsets[ti];
    if (ts.kind == 0) {
      for (int d = 0; d < 4; ++d) pl.tcube[4 * ti + d] = pl.cube[4 * ts.id + d];
      continue;
    }
    const ChargeSet& c = P.charges[ts.id];
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t k = 0; k < c.n(); ++k)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], c.xyz[3 * k + d]);
        hi[d] = std::max(hi[d], c.xyz[3 * k + d]);
      }
    double half = 0.0;
    for (int d = 0; d < 3; ++d) {
      pl.tcube[4 * ti + d] = 0.5 * (lo[d] + hi[d]);
      half = std::max(half, 0.5 * (hi[d] - lo[d]));
    }
    pl.tcube[4 * ti + 3] = half * (1.0 + 1e-6) + 1e-6;
  }

  // initial capacities (grown by pbtc_setup when too small)
  if (pl.cap_cells == 0) pl.cap_cells = 8 * pl.ngp / std::max(2, pl.ncrit / 2) + 64 * pl.nsurf + 1024;
  if (pl.cap_near == 0) pl.cap_near = 48 * pl.nitems + 1024;
  if (pl.cap_far == 0)
    pl.cap_far = (pl.prm.op == PBTC_OP_DIRECT ? 1 : 160) * pl.nitems + 1024;
  if (pl.cap_units == 0) pl.cap_units = 8 * pl.nitems + 1024;
  if (pl.cap_mparts == 0) pl.cap_mparts = pl.cap_cells / 4 + 1024;
  if (pl.cap_aunits == 0) pl.cap_aunits = 8 * pl.nitems_adj + 1024;
  if (pl.cap_auptr == 0) pl.cap_auptr = 2 * pl.nitems_adj + 64;
  if (pl.cap_tcells == 0) pl.cap_tcells = pl.ntgt / 16 + 64 * (int64_t)pl.tsets.size() + 1024;
  if (pl.cap_anear == 0) pl.cap_anear = 48 * pl.nitems_adj + 1024;
  if (pl.cap_amchunks == 0)
    pl.cap_amchunks = (pl.cap_tcells + 8 * pl.ntgt / kMomSpan + 1024) * pl.adj_ms;
  if (pl.cap_ampairs == 0) pl.cap_ampairs = pl.cap_tcells * pl.adj_ms + 64;
  if (pl.cap_afar == 0) pl.cap_afar = (pl.prm.op == PBTC_OP_DIRECT ? 1 : 160) * pl.nitems_adj + 1024;
  if (pl.cap_nf == 0) {
    int64_t n = 0;
    for (const Block& b : pl.blocks) n += pl.tsets[b.t].n;
    pl.cap_nf = 24 * n + 1024;
  }
  compute_layout(pl);
  return PBTC_OK;
}

void compute_layout(pbtc_plan_t& pl) {
  Layout L;
  const int64_t nP = ncoef(pl.P);
  const int m = pl.prm.restart;
  const int64_t n = pl.nunk;
  // inputs
  pl.o_verts = L.add(8 * 3 * pl.nv_tot);
  pl.o_tris = L.add(4 * 3 * pl.np_tot);
  pl.o_pan_surf = L.add(4 * pl.np_tot);
  pl.o_qxyz = L.add(8 * 3 * std::max<int64_t>(pl.nq, 1));
  pl.o_q = L.add(8 * std::max<int64_t>(pl.nq, 1));
  pl.o_qreg = L.add(4 * std::max<int64_t>(pl.nq, 1));
  // panels
  pl.o_cx = L.add(8 * pl.np_tot);
  pl.o_cy = L.add(8 * pl.np_tot);
  pl.o_cz = L.add(8 * pl.np_tot);
  pl.o_pidx = L.add(8 * pl.np_tot);
  pl.o_pinv = L.add(8 * 4 * pl.np_tot);
  pl.o_ptab = L.add(8 * 3 * pl.nsurf);
  pl.o_flags = L.add(4 * 16);
  pl.o_qtab = L.add(8 * (2 * pl.nreg + 1));
  pl.o_nx = L.add(8 * pl.np_tot);
  pl.o_ny = L.add(8 * pl.np_tot);
  pl.o_nz = L.add(8 * pl.np_tot);
  pl.o_area = L.add(8 * pl.np_tot);
  pl.o_len = L.add(8 * pl.np_tot);
  // targets
  pl.o_tx = L.add(8 * pl.ntgt);
  pl.o_ty = L.add(8 * pl.ntgt);
  pl.o_tz = L.add(8 * pl.ntgt);
  pl.o_txf = L.add(4 * pl.ntgt);
  pl.o_tyf = L.add(4 * pl.ntgt);
  pl.o_tzf = L.add(4 * pl.ntgt);
  pl.o_tidx = L.add(4 * pl.ntgt);
  pl.o_grp = L.add(8 * 4 * pl.ngrp);
  pl.o_grp_tab = L.add(8 * 2 * pl.ngrp);
  // Gauss points (sorted) and sort scratch
  const int64_t nkey = std::max(pl.ngp, pl.ntgt);
  pl.o_gx = L.add(8 * pl.ngp);
  pl.o_gy = L.add(8 * pl.ngp);
  pl.o_gz = L.add(8 * pl.ngp);
  pl.o_gw = L.add(8 * pl.ngp);
  pl.o_gpid = L.add(4 * pl.ngp);
  pl.o_gidx = L.add(4 * pl.ngp);
  pl.o_gkey = L.add(8 * nkey);
  pl.o_gtmpk = L.add(8 * nkey);
  pl.o_gtmpv = L.add(4 * nkey);
  pl.o_keys2 = L.add(4 * nkey);
  pl.o_hist = L.add(4 * (256 * (nkey / 256 + 2) + nkey / 16 + 4096));
  pl.o_tkey = L.add(8 * pl.ntgt);
  pl.o_tkey2 = L.add(8 * pl.ntgt);
  pl.o_tval = L.add(4 * pl.ntgt);
  pl.o_tval2 = L.add(4 * pl.ntgt);
  pl.o_tkey_sorted = L.add(8 * pl.ntgt);
  pl.o_src64 = L.add(8 * 8 * pl.ngp);
  pl.o_src32 = L.add(4 * 8 * pl.ngp);
  // block outputs and descriptors
  pl.o_S = L.add(8 * pl.nout);
  pl.o_D = L.add(8 * pl.nout);
  pl.o_blocks = L.add(sizeof(DevBlock) * pl.blocks.size());
  size_t nterm = 0, nrterm = 0;
  for (auto& r : pl.rows) nterm += r.terms.size();
  for (auto& r : pl.reac_rows) nrterm += r.terms.size();
  pl.o_rows = L.add(sizeof(DevRowBlock) * pl.rows.size());
  pl.o_terms = L.add(sizeof(DevRowTerm) * std::max<size_t>(nterm, 1));
  pl.o_reac_rows = L.add(sizeof(DevRowBlock) * std::max<size_t>(pl.reac_rows.size(), 1));
  pl.o_reac_terms = L.add(sizeof(DevRowTerm) * std::max<size_t>(nrterm, 1));
  pl.o_items = L.add(4 * pl.nitems);
  for (int ph = 0; ph < 2; ++ph)
    for (int ks = 0; ks < KS_COUNT; ++ks)
      pl.o_item_list[ph][ks] = L.add(4 * std::max<size_t>(pl.item_list[ph][ks].size(), 1));
  pl.o_nf_rowblk = L.add(4 * std::max<int64_t>(pl.nf_rows, 1));
  // Krylov (FP64)
  pl.o_b = L.add(8 * n);
  pl.o_x = L.add(8 * n);
  pl.o_r = L.add(8 * n);
  pl.o_w = L.add(8 * n);
  pl.o_tmp = L.add(8 * n);
  pl.o_ptmp = L.add(8 * n);
  pl.o_lam = L.add(8 * n);
  pl.o_adj_rhs = L.add(8 * n);
  pl.o_V = L.add(8 * (size_t)(m + 1) * n);
  pl.o_H = L.add(8 * (size_t)(m + 1) * (m + 1));
  pl.o_givens = L.add(8 * 4 * (size_t)(m + 2));
  pl.o_scal = L.add(8 * 64);
  // chunk partials (m + 1 per chunk), two coefficient sets per system, the
  // norm partials of the fused second pass (16 per chunk), reduction scratch
  pl.o_red = L.add(8 * ((size_t)(m + 1) * (pl.dot_chunks.size() + 2 * (size_t)pl.ncomp) +
                         16 * pl.dot_chunks.size() + (size_t)(m + 2) * 1024));
  pl.o_phi_reac = L.add(8 * std::max<int64_t>(pl.nq, 1));
  pl.o_energy = L.add(8 * (pl.ncomp + 64));
  pl.o_coul = L.add(8 * (pl.ncomp + 1));
  pl.o_z2 = L.add(8 * std::max<int64_t>(n, pl.nq));
  pl.o_gxin = L.add(8 * n);
  pl.o_gyout = L.add(8 * std::max<int64_t>(n, pl.nq));
  pl.o_comp_of_unk = L.add(4 * n);
  pl.o_chunks = L.add(16 * std::max<size_t>(pl.dot_chunks.size(), 1) + 4 * (pl.ncomp + 1));
  pl.o_comp_q = L.add(4 * std::max<int64_t>(pl.nq, 1));
  // per system: H ((m+1)^2), Givens (4 (m+2)), scalars (16)
  pl.o_kstate = L.add(8 * (size_t)pl.ncomp * ((size_t)(m + 1) * (m + 1) + 4 * (m + 2) + 16));
  pl.o_surf_tab = L.add(8 * (9 * (pl.nsurf + 1) + pl.tsets.size() + 1 + 16));
  pl.o_dots = L.add(8 * 4096);
  pl.o_crows = L.add(sizeof(DevCoulRow) * pl.rows.size() + 4 * (pl.nreg + 1 + pl.rows.size()) + 16);
  // transposed operator
  pl.o_gpos32 = L.add(4 * 8 * pl.ngp);
  pl.o_gpos64 = L.add(8 * 8 * pl.ngp);
  pl.o_gp_pos = L.add(4 * pl.ngp);
  pl.o_gpgrp = L.add(8 * 4 * std::max<int64_t>(pl.ngpgrp, 1));
  pl.o_mu_s = L.add(8 * pl.nout);
  pl.o_mu_d = L.add(8 * pl.nout);
  pl.o_asrc32 = L.add(4 * 8 * std::max<int64_t>(pl.nf_rows, 1));
  pl.o_asrc64 = L.add(8 * 8 * std::max<int64_t>(pl.nf_rows, 1));
  pl.o_aout_s = L.add(8 * std::max<int64_t>(pl.naout, 1));
  pl.o_aout_d = L.add(8 * std::max<int64_t>(pl.naout, 1));
  pl.o_aitems = L.add(4 * std::max<int64_t>(pl.nitems_adj, 1));
  for (int ph = 0; ph < 2; ++ph) {
    for (int ks = 0; ks < KS_COUNT; ++ks)
      pl.o_aitem_list[ph][ks] = L.add(4 * std::max<size_t>(pl.aitem_list[ph][ks].size(), 1));
    pl.o_slots[ph] = L.add(sizeof(DevSlot) * std::max<size_t>(pl.slots[ph].size(), 1));
    pl.o_gather[ph] = L.add(sizeof(DevGather) * std::max<int>(pl.nsurf, 1));
    pl.o_gather_slots[ph] = L.add(4 * std::max<size_t>(pl.gather_slots[ph].size(), 1));
  }
  pl.o_csc_ptr = L.add(8 * (pl.ncsc + 1));
  {
    int64_t ns = 0;
    for (const Block& b : pl.blocks) ns += b.nk;
    pl.o_slot_block = L.add(4 * std::max<int64_t>(ns, 1));
    pl.o_slot_kidx = L.add(4 * std::max<int64_t>(ns, 1));
    for (int ph = 0; ph < 2; ++ph) {
      pl.o_adj_blist[ph] = L.add(4 * std::max<size_t>(pl.blocks.size(), 1));
      pl.o_adj_sids[ph] = L.add(4 * std::max<int64_t>(ns, 1));
      pl.o_adj_tslot[ph] = L.add(4 * std::max<int64_t>((int64_t)pl.tsets.size() * pl.adj_ms, 1));
    }
    pl.o_adj_tab = L.add(8 * 2 * (pl.nsurf + 1));
  }
  pl.o_csc_fill = L.add(8 * (pl.ncsc + 1));
  pl.o_anear_ptr = L.add(8 * (pl.nitems_adj + 1));
  pl.o_afar_ptr = L.add(8 * (pl.nitems_adj + 1));
  pl.fixed_bytes = L.total;
  // tree
  pl.o_cells = L.add(sizeof(Cell) * pl.cap_cells);
  pl.o_cnt = L.add(8 * (pl.cap_cells + 1));
  pl.o_scan = L.add(8 * (std::max<int64_t>(pl.cap_cells, pl.nitems) + 2));
  pl.o_mom64 = L.add(8 * 2 * nP * pl.cap_cells);
  pl.o_mom32 = L.add(4 * 2 * nP * pl.cap_cells);
  pl.o_mchunks = L.add(16 * pl.cap_cells);
  pl.o_mcent = L.add(32 * pl.cap_cells);
  pl.o_mspans = L.add(16 * pl.cap_cells);
  pl.o_mproot = L.add(4 * mom_up_batch(pl.P) * pl.cap_mparts);
  pl.o_mph = L.add(24 * mom_up_batch(pl.P) * pl.cap_mparts);
  pl.o_musum = L.add(16 * pl.cap_cells);
  pl.o_mparts = L.add(16 * pl.cap_mparts);
  pl.o_mpart = L.add(8 * 2 * nP * pl.cap_mparts);
  // lists
  pl.o_near_ptr = L.add(8 * (pl.nitems + 1));
  pl.o_far_ptr = L.add(8 * (pl.nitems + 1));
  pl.o_near = L.add(4 * pl.cap_near);
  pl.o_far = L.add(4 * pl.cap_far);
  // near-field correction (CSR over global targets of each block)
  int64_t nrow = 0;
  for (const Block& b : pl.blocks) nrow += pl.tsets[b.t].n;
  pl.o_nf_ptr = L.add(8 * (nrow + 1));
  pl.o_nf_col = L.add(4 * pl.cap_nf);
  pl.o_nf_v64 = L.add(8 * 4 * pl.cap_nf);
  pl.o_nf_v32 = L.add(4 * 4 * pl.cap_nf);
  pl.o_csc_ent = L.add(4 * pl.cap_nf);
  pl.o_csc_row = L.add(4 * pl.cap_nf);
  // transposed-operator trees and lists
  pl.o_tcells = L.add(sizeof(Cell) * pl.cap_tcells);
  pl.o_tcnt = L.add(8 * (pl.cap_tcells + 1));
  pl.o_amom32 = L.add(4 * (size_t)adj_mom_len(pl.P) * pl.cap_tcells * pl.adj_ms);
  pl.o_amom64 = L.add(8 * (size_t)adj_mom_len(pl.P) * pl.cap_tcells * pl.adj_ms);
  pl.o_amchunks = L.add(16 * pl.cap_amchunks);
  pl.o_ampairs = L.add(16 * pl.cap_ampairs);
  pl.o_ampart = L.add(8 * 2 * nP * pl.cap_amchunks);
  pl.o_anear = L.add(4 * pl.cap_anear);
  pl.o_units = L.add(16 * pl.cap_units);
  pl.o_uptr = L.add(4 * (2 * pl.nitems + 64));
  pl.o_aunits = L.add(16 * pl.cap_aunits);
  pl.o_auptr = L.add(4 * pl.cap_auptr);
  pl.o_partial = L.add(8 * 4 * 64 * std::max(pl.cap_units, pl.cap_aunits));
  pl.o_afar = L.add(4 * pl.cap_afar);
  pl.ws_bytes = L.total + 4096;
}

}  // namespace pbtc
