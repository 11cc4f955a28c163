// C interface of libpbtc (see include/pbtc.h for the contract).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <new>
#include <unordered_map>

#include "device_util.h"
#include "internal.h"
#include "taylor.h"

namespace pbtc {
bool triangle_rule(int k, double* bary, double* w);
bool gauss_legendre(int n, double* x, double* w);
std::string validate_problem(const pbtc_problem& p, const pbtc_params& prm, int* code);
int build_plan(pbtc_plan_t& pl);
void compute_layout(pbtc_plan_t& pl);
int device_setup(pbtc_plan_t& pl, hipStream_t st, int* need_retry);
int device_solve(pbtc_plan_t& pl, hipStream_t st, pbtc_result* res);
int update_charges(pbtc_plan_t& pl, hipStream_t st);
int device_backward(pbtc_plan_t& pl, hipStream_t st, double gE, double* dq, double* dk, double* de,
                    pbtc_result* res);
int apply_operator(pbtc_plan_t& pl, hipStream_t st, const double* x, double* y, int precision,
                   int phase);
int apply_transpose(pbtc_plan_t& pl, hipStream_t st, const double* x, double* y, int precision,
                    int phase);
int apply_precond(pbtc_plan_t& pl, hipStream_t st, const double* x, double* y, bool transpose,
                  bool accumulate);
double wall_seconds();
int device_coulomb(pbtc_plan_t& pl, hipStream_t st, double* total, double* per_system);
int device_coulomb_noalloc(pbtc_plan_t& pl, hipStream_t st, double* total, double* per_system);
void release_op_graphs(pbtc_plan_t& pl);

// The merged problem of a pbtc_solve_batch call and where each member's
// regions, systems, unknowns and charges sit in it.
struct BatchCache {
  std::vector<uint64_t> serials;  // members, in call order
  std::vector<uint64_t> charge_versions;
  pbtc_plan_t* merged = nullptr;
  std::vector<int> reg0, comp0;   // first region / system of every member (+ end)
  std::vector<int64_t> unk0, q0;  // first unknown / charge of every member (+ end)
  ~BatchCache() { delete merged; }
};
}  // namespace pbtc

using namespace pbtc;

namespace {

thread_local std::string g_err;
std::atomic<uint64_t> g_serial{1};

// Which plan last set up each workspace (a workspace holds the device state
// of one plan at a time).
std::mutex g_ws_mu;
std::unordered_map<const void*, uint64_t> g_ws_owner;

void claim_ws(const void* ws, const pbtc_plan_t* pl) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  g_ws_owner[ws] = pl->serial;
}

bool owns_ws(const void* ws, const pbtc_plan_t* pl) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  const auto it = g_ws_owner.find(ws);
  return it != g_ws_owner.end() && it->second == pl->serial;
}

void release_ws(const pbtc_plan_t* pl) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  for (auto it = g_ws_owner.begin(); it != g_ws_owner.end();)
    it = it->second == pl->serial ? g_ws_owner.erase(it) : std::next(it);
}

// True when `ws` holds this plan's set-up device state.
bool ready(const pbtc_plan_t* pl, const void* ws) {
  return pl->setup_done && pl->ws == ws && owns_ws(ws, pl);
}

int fail_global(int code, const char* msg) {
  try {
    g_err = msg;
  } catch (...) {
  }
  return code;
}

int fail_plan(pbtc_plan_t* pl, int code, const std::string& msg) {
  try {
    pl->err = msg;
  } catch (...) {
  }
  return code;
}

// Runs the body of an entry point: a C++ exception (std::bad_alloc from a
// host table, ...) becomes PBTC_EHOST with a message instead of crossing the
// C interface.  `pl` receives the message (NULL: the thread's last error).
template <typename F>
int guarded(pbtc_plan_t* pl, F&& body) noexcept {
  const char* msg = "internal error";
  try {
    return body();
  } catch (const std::bad_alloc&) {
    msg = "out of host memory";
  } catch (const std::exception& e) {
    try {
      const std::string m = std::string("internal error: ") + e.what();
      return pl ? fail_plan(pl, PBTC_EHOST, m) : fail_global(PBTC_EHOST, m.c_str());
    } catch (...) {
    }
  } catch (...) {
  }
  return pl ? fail_plan(pl, PBTC_EHOST, msg) : fail_global(PBTC_EHOST, msg);
}

bool finite_all(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

void fill_sizes(const pbtc_plan_t* pl, pbtc_result* res) {
  if (!res) return;
  res->n_p2p_pairs = pl->p2p_pairs;
  res->n_m2p_evals = pl->m2p_evals;
  res->n_dense_equiv = pl->dense_equiv;
  res->n_near_entries = (double)pl->n_nf;
  res->workspace_needed = pl->ws_bytes;
  res->tile_sources = pl->tile_sources;
  res->tile_cells = pl->tile_cells;
}

// Set-up on a workspace, growing capacity estimates as needed.
int setup_impl(pbtc_plan_t* pl, void* ws, size_t bytes, hipStream_t st, pbtc_result* res,
               bool reuse_inputs = false) {
  const bool same = pl->ws == ws && owns_ws(ws, pl);
  pl->setup_done = false;
  pl->solved = false;
  pl->dev_solved = false;
  // another plan (or another workspace) held this memory: nothing in it is ours
  if (!reuse_inputs || pl->inputs_ws != ws || !same) pl->inputs_ws = nullptr;
  if (!same) pl->adj_done = false;
  for (int attempt = 0; attempt < 4; ++attempt) {
    if (bytes < pl->ws_bytes) {
      if (res) res->workspace_needed = pl->ws_bytes;
      return fail_plan(pl, PBTC_EWORKSPACE,
                       "workspace of " + std::to_string(bytes) + " bytes is smaller than the " +
                           std::to_string(pl->ws_bytes) + " bytes this plan needs");
    }
    pl->ws = ws;
    claim_ws(ws, pl);
    const double t0 = wall_seconds();
    int retry = 0;
    const int rc = device_setup(*pl, st, &retry);
    if (rc == PBTC_EWORKSPACE && retry) {
      compute_layout(*pl);
      pl->inputs_ws = nullptr;
      pl->adj_done = false;
      continue;
    }
    if (rc) return rc;
    pl->setup_done = true;
    pl->charges_dirty = false;
    if (res) {
      res->t_setup_s = wall_seconds() - t0;
      for (int k = 0; k < 6; ++k) res->t_setup_phase_s[k] = pl->setup_phase[k];
    }
    fill_sizes(pl, res);
    return PBTC_OK;
  }
  return fail_plan(pl, PBTC_EWORKSPACE, "workspace estimate did not converge");
}

// Plan of a problem: validation, block structure, layout.
int make_plan(const pbtc_problem& p, const pbtc_params& prm, pbtc_plan_t** out) {
  *out = nullptr;
  int code = PBTC_OK;
  std::string msg = validate_problem(p, prm, &code);
  if (code) return fail_global(code, msg.c_str());
  std::unique_ptr<pbtc_plan_t> pl(new pbtc_plan_t());
  pl->serial = g_serial.fetch_add(1);
  pl->prob = p;
  pl->prm = prm;
  const int rc = build_plan(*pl);
  if (rc) return fail_global(rc, "problem too large for 32-bit indices");
  *out = pl.release();
  return PBTC_OK;
}

// Solve on a workspace: set-up when needed, charges, GMRES, energy.
int solve_impl(pbtc_plan_t* plan, void* ws, size_t bytes, hipStream_t st, bool force_setup,
               pbtc_result* res) {
  if (force_setup || !ready(plan, ws)) {
    const int rc = setup_impl(plan, ws, bytes, st, res, force_setup);
    if (rc) return rc;
  } else if (bytes < plan->ws_bytes) {
    res->workspace_needed = plan->ws_bytes;
    return fail_plan(plan, PBTC_EWORKSPACE, "workspace smaller than the plan needs");
  }
  fill_sizes(plan, res);
  if (plan->charges_dirty) {
    const int rc = update_charges(*plan, st);
    if (rc) return rc;
  }
  return device_solve(*plan, st, res);
}

bool same_params(const pbtc_params& a, const pbtc_params& b) {
  return a.K == b.K && a.K_fine == b.K_fine && a.N_k == b.N_k && a.thres == b.thres &&
         a.theta == b.theta && a.P == b.P && a.ncrit == b.ncrit &&
         a.direct_below == b.direct_below && a.tol == b.tol && a.restart == b.restart &&
         a.max_iter == b.max_iter && a.precision == b.precision && a.op == b.op &&
         a.inner_tol == b.inner_tol && a.max_refine == b.max_refine &&
         a.validate_charges == b.validate_charges && a.profile == b.profile &&
         a.precond == b.precond && a.op_graph == b.op_graph &&
         a.unit_sources == b.unit_sources && a.unit_cells == b.unit_cells;
}

// The merged plan of a batch (kept with plans[0] while the members stay the
// same), with the members' current charge values.
int batch_plan(pbtc_plan_t** plans, int n, BatchCache** out) {
  pbtc_plan_t* head = plans[0];
  BatchCache* bc = head->batch;
  bool hit = bc && (int)bc->serials.size() == n;
  for (int i = 0; hit && i < n; ++i) hit = bc->serials[i] == plans[i]->serial;
  if (!hit) {
    delete bc;
    head->batch = nullptr;
    std::unique_ptr<BatchCache> fresh(new BatchCache());
    pbtc_problem merged;
    fresh->reg0.push_back(0);
    fresh->comp0.push_back(0);
    fresh->unk0.push_back(0);
    fresh->q0.push_back(0);
    int ncomp = 0;
    for (int i = 0; i < n; ++i) {
      const pbtc_problem& P = plans[i]->prob;
      const int r0 = (int)merged.regions.size();
      for (size_t r = 0; r < P.regions.size(); ++r) {
        merged.regions.push_back(P.regions[r]);
        merged.charges.push_back(P.charges[r]);
      }
      for (const Surface& s : P.surfaces) {
        Surface c = s;
        c.inner += r0;
        c.outer += r0;
        merged.surfaces.push_back(std::move(c));
      }
      ncomp += plans[i]->ncomp;
      fresh->serials.push_back(plans[i]->serial);
      fresh->charge_versions.push_back(plans[i]->charge_version);
      fresh->reg0.push_back((int)merged.regions.size());
      fresh->comp0.push_back(ncomp);
      fresh->unk0.push_back(fresh->unk0.back() + plans[i]->nunk);
      fresh->q0.push_back(fresh->q0.back() + plans[i]->nq);
    }
    const int rc = make_plan(merged, head->prm, &fresh->merged);
    if (rc) return fail_plan(head, rc, std::string("batch: ") + g_err);
    if (fresh->merged->ncomp != ncomp)
      return fail_plan(head, PBTC_EINVAL,
                       "batch: a plan's systems are not contiguous in its surface order");
    bc = fresh.release();
    head->batch = bc;
  }
  // charge values changed since the merged plan copied them
  for (int i = 0; i < n; ++i) {
    if (bc->charge_versions[i] == plans[i]->charge_version) continue;
    const pbtc_problem& P = plans[i]->prob;
    for (size_t r = 0; r < P.regions.size(); ++r)
      bc->merged->prob.charges[bc->reg0[i] + r].q = P.charges[r].q;
    bc->merged->charges_dirty = true;
    bc->merged->solved = false;
    bc->merged->dev_solved = false;
    bc->charge_versions[i] = plans[i]->charge_version;
  }
  *out = bc;
  return PBTC_OK;
}

}  // namespace

extern "C" {

int pbtc_version(int* major, int* minor) {
  if (major) *major = PBTC_VERSION_MAJOR;
  if (minor) *minor = PBTC_VERSION_MINOR;
  return PBTC_OK;
}

int pbtc_problem_create(pbtc_problem** out) {
  return guarded(nullptr, [&] {
    if (!out) return fail_global(PBTC_EINVAL, "out is NULL");
    *out = new pbtc_problem();
    return PBTC_OK;
  });
}

void pbtc_problem_destroy(pbtc_problem* p) { delete p; }

int pbtc_add_region(pbtc_problem* p, double eps, double kappa, int* region_id) {
  return guarded(nullptr, [&] {
    if (!p) return fail_global(PBTC_EINVAL, "problem is NULL");
    if (!(eps > 0.0) || !std::isfinite(eps) || !(kappa >= 0.0) || !std::isfinite(kappa))
      return fail_global(PBTC_EINVAL, "eps must be > 0 and kappa >= 0, both finite");
    Region r;
    r.eps = eps;
    r.kappa = kappa;
    p->regions.push_back(r);
    p->charges.emplace_back();
    if (region_id) *region_id = (int)p->regions.size() - 1;
    return PBTC_OK;
  });
}

int pbtc_add_surface(pbtc_problem* p, const double* verts, int64_t nv, const int32_t* tris,
                     int64_t np, int inner_region, int outer_region, int* surface_id) {
  return guarded(nullptr, [&] {
    if (!p) return fail_global(PBTC_EINVAL, "problem is NULL");
    const int nreg = (int)p->regions.size();
    if (inner_region < 0 || inner_region >= nreg || outer_region < 0 || outer_region >= nreg)
      return fail_global(PBTC_EINVAL, "unknown region id");
    if (inner_region == outer_region)
      return fail_global(PBTC_EINVAL, "inner and outer region are equal");
    if (nv < 3 || np < 4 || !verts || !tris)
      return fail_global(PBTC_EINVAL, "a closed surface needs >= 3 vertices and >= 4 triangles");
    if (np >= (int64_t(1) << 30) || nv >= (int64_t(1) << 31))
      return fail_global(PBTC_EINVAL, "surface too large");
    for (int64_t i = 0; i < 3 * np; ++i)
      if (tris[i] < 0 || tris[i] >= nv)
        return fail_global(PBTC_EINVAL, "triangle index out of range");
    if (!finite_all(verts, 3 * nv)) return fail_global(PBTC_EINVAL, "vertex coordinate not finite");
    Surface s;
    s.v.assign(verts, verts + 3 * nv);
    s.t.assign(tris, tris + 3 * np);
    s.inner = inner_region;
    s.outer = outer_region;
    p->surfaces.push_back(std::move(s));
    if (surface_id) *surface_id = (int)p->surfaces.size() - 1;
    return PBTC_OK;
  });
}

int pbtc_set_charges(pbtc_problem* p, int region_id, const double* xyz, const double* q, int64_t nq) {
  return guarded(nullptr, [&] {
    if (!p) return fail_global(PBTC_EINVAL, "problem is NULL");
    if (region_id < 0 || region_id >= (int)p->regions.size())
      return fail_global(PBTC_EINVAL, "unknown region id");
    if (nq < 0 || (nq > 0 && (!xyz || !q))) return fail_global(PBTC_EINVAL, "bad charge arrays");
    if (!finite_all(xyz, 3 * nq) || !finite_all(q, nq))
      return fail_global(PBTC_EINVAL, "charge position or value not finite");
    ChargeSet& c = p->charges[region_id];
    c.xyz.assign(xyz, xyz + 3 * nq);
    c.q.assign(q, q + nq);
    return PBTC_OK;
  });
}

int pbtc_params_default(pbtc_params* prm) {
  if (!prm) return fail_global(PBTC_EINVAL, "params is NULL");
  prm->K = 4;
  prm->K_fine = 19;
  prm->N_k = 5;
  prm->thres = 2.0;
  prm->theta = 0.5;
  prm->P = 6;
  prm->ncrit = 0;
  prm->direct_below = -1;
  prm->tol = 1e-5;
  prm->restart = 100;
  prm->max_iter = 1000;
  prm->precision = PBTC_FP32_REFINED;
  prm->op = PBTC_OP_TREECODE;
  prm->inner_tol = 1e-6;
  prm->max_refine = 10;
  prm->validate_charges = 1;
  prm->profile = 0;
  prm->precond = PBTC_PREC_NONE;
  prm->unit_sources = 0;
  prm->unit_cells = 0;
  prm->op_graph = 1;
  return PBTC_OK;
}

int pbtc_validate(const pbtc_problem* p, const pbtc_params* prm) {
  return guarded(nullptr, [&] {
    if (!p || !prm) return fail_global(PBTC_EINVAL, "problem or params is NULL");
    int code = PBTC_OK;
    std::string msg = validate_problem(*p, *prm, &code);
    if (code) return fail_global(code, msg.c_str());
    return PBTC_OK;
  });
}

int pbtc_plan(const pbtc_problem* p, const pbtc_params* prm, pbtc_plan_t** out,
              size_t* workspace_bytes) {
  return guarded(nullptr, [&] {
    if (!p || !prm || !out) return fail_global(PBTC_EINVAL, "NULL argument");
    const int rc = make_plan(*p, *prm, out);
    if (rc) return rc;
    if (workspace_bytes) *workspace_bytes = (*out)->ws_bytes;
    return PBTC_OK;
  });
}

pbtc_plan_s::~pbtc_plan_s() {
  for (auto* v : {&prof, &prof_pool})
    for (auto& ev : *v) {
      (void)hipEventDestroy(ev.a);
      (void)hipEventDestroy(ev.b);
    }
  for (hipEvent_t e : res_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : {ev_fork, ev_join})
    if (e) (void)hipEventDestroy(e);
  release_op_graphs(*this);
  if (side) (void)hipStreamDestroy(side);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  if (res_pin) (void)hipHostFree(res_pin);
  delete batch;
}

void pbtc_plan_destroy(pbtc_plan_t* plan) {
  if (!plan) return;
  release_ws(plan);
  if (plan->batch && plan->batch->merged) release_ws(plan->batch->merged);
  delete plan;
}

int pbtc_plan_sizes(const pbtc_plan_t* plan, int64_t* n_unknowns, int64_t* n_charges,
                    int* n_surfaces, int* n_regions) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  if (n_unknowns) *n_unknowns = plan->nunk;
  if (n_charges) *n_charges = plan->nq;
  if (n_surfaces) *n_surfaces = plan->nsurf;
  if (n_regions) *n_regions = plan->nreg;
  return PBTC_OK;
}

int pbtc_setup(pbtc_plan_t* plan, void* d_workspace, size_t bytes, void* hip_stream,
               pbtc_result* res) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  return guarded(plan, [&] {
    if (!d_workspace) return fail_plan(plan, PBTC_EINVAL, "workspace is NULL");
    if (res) std::memset(res, 0, sizeof(*res));
    return setup_impl(plan, d_workspace, bytes, (hipStream_t)hip_stream, res);
  });
}

int pbtc_solve(pbtc_plan_t* plan, void* d_workspace, size_t bytes, void* hip_stream,
               int force_setup, pbtc_result* res) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  return guarded(plan, [&] {
    if (!d_workspace) return fail_plan(plan, PBTC_EINVAL, "workspace is NULL");
    pbtc_result local;
    pbtc_result* r = res ? res : &local;
    std::memset(r, 0, sizeof(*r));
    return solve_impl(plan, d_workspace, bytes, (hipStream_t)hip_stream, force_setup != 0, r);
  });
}

int pbtc_solve_batch(pbtc_plan_t** plans, int n, void* d_workspace, size_t bytes,
                     void* hip_stream, pbtc_result* res) {
  if (!plans || n < 1) return fail_global(PBTC_EINVAL, "plans is NULL or n < 1");
  for (int i = 0; i < n; ++i)
    if (!plans[i]) return fail_global(PBTC_EINVAL, "a plan is NULL");
  pbtc_plan_t* head = plans[0];
  return guarded(head, [&] {
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < i; ++j)
        if (plans[j] == plans[i]) return fail_plan(head, PBTC_EINVAL, "batch: a plan appears twice");
      if (!same_params(plans[i]->prm, head->prm))
        return fail_plan(head, PBTC_EINVAL, "batch: the plans' parameters differ");
    }
    if (res) std::memset(res, 0, sizeof(pbtc_result) * (size_t)n);
    BatchCache* bc = nullptr;
    int rc = batch_plan(plans, n, &bc);
    if (rc) return rc;
    pbtc_plan_t* m = bc->merged;
    if (bytes < m->ws_bytes) {
      if (res)
        for (int i = 0; i < n; ++i) res[i].workspace_needed = m->ws_bytes;
      return fail_plan(head, PBTC_EWORKSPACE,
                       "batch workspace of " + std::to_string(bytes) + " bytes; the batch needs " +
                           std::to_string(m->ws_bytes));
    }
    if (!d_workspace) return fail_plan(head, PBTC_EINVAL, "workspace is NULL");
    pbtc_result all;
    std::memset(&all, 0, sizeof(all));
    rc = solve_impl(m, d_workspace, bytes, (hipStream_t)hip_stream, false, &all);
    if (rc == PBTC_EWORKSPACE && res)
      for (int i = 0; i < n; ++i) res[i].workspace_needed = all.workspace_needed;
    if (rc && rc != PBTC_ENOCONV) return fail_plan(head, rc, "batch: " + m->err);
    // scatter the merged solution to the members
    for (int i = 0; i < n; ++i) {
      pbtc_plan_t* p = plans[i];
      const int64_t u0 = bc->unk0[i], u1 = bc->unk0[i + 1], q0 = bc->q0[i], q1 = bc->q0[i + 1];
      p->x_host.assign(m->x_host.begin() + u0, m->x_host.begin() + u1);
      p->phi_reac_host.assign(m->phi_reac_host.begin() + q0, m->phi_reac_host.begin() + q1);
      p->history = m->history;
      const int c0 = bc->comp0[i], c1 = bc->comp0[i + 1];
      p->comp_energy.assign(m->comp_energy.begin() + c0, m->comp_energy.begin() + c1);
      p->comp_rel.assign(m->comp_rel.begin() + c0, m->comp_rel.begin() + c1);
      p->comp_conv.assign(m->comp_conv.begin() + c0, m->comp_conv.begin() + c1);
      double e = 0.0, worst = 0.0;
      bool conv = true;
      for (int c = 0; c < c1 - c0; ++c) {
        e += p->comp_energy[c];
        worst = std::max(worst, p->comp_rel[c]);
        conv = conv && p->comp_conv[c] != 0;
      }
      p->energy = e;
      p->solved = true;
      p->dev_solved = false;  // the solution lives in the batch workspace only
      if (res) {
        res[i] = all;
        res[i].energy_kJmol = e;
        res[i].converged = conv ? 1 : 0;
        res[i].final_rel_res = worst;
      }
    }
    if (rc == PBTC_ENOCONV)
      return fail_plan(head, PBTC_ENOCONV, "batch: GMRES did not reach the tolerance within max_iter");
    return PBTC_OK;
  });
}

int pbtc_get_surface(const pbtc_plan_t* plan, int surface_id, double* phi, double* dphidn_inner) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  if (!plan->solved) return fail_global(PBTC_EINVAL, "no solution yet (call pbtc_solve)");
  if (surface_id < 0 || surface_id >= plan->nsurf) return fail_global(PBTC_EINVAL, "unknown surface");
  const int64_t o = plan->unk_off[surface_id];
  const int64_t n = plan->pan_off[surface_id + 1] - plan->pan_off[surface_id];
  if (phi) std::memcpy(phi, plan->x_host.data() + o, 8 * n);
  if (dphidn_inner) std::memcpy(dphidn_inner, plan->x_host.data() + o + n, 8 * n);
  return PBTC_OK;
}

int pbtc_get_phi_reac(const pbtc_plan_t* plan, double* phi_reac) {
  if (!plan || !phi_reac) return fail_global(PBTC_EINVAL, "NULL argument");
  if (!plan->solved) return fail_global(PBTC_EINVAL, "no solution yet (call pbtc_solve)");
  std::memcpy(phi_reac, plan->phi_reac_host.data(), 8 * plan->nq);
  return PBTC_OK;
}

int pbtc_get_history(const pbtc_plan_t* plan, double* rel_res, int cap, int* n_iter) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  const int n = (int)plan->history.size();
  if (n_iter) *n_iter = n;
  if (rel_res)
    for (int i = 0; i < n && i < cap; ++i) rel_res[i] = plan->history[i];
  return PBTC_OK;
}

int pbtc_matvec(pbtc_plan_t* plan, void* d_workspace, void* hip_stream, const double* d_x,
                double* d_y, int precision) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  return guarded(plan, [&] {
    if (!ready(plan, d_workspace))
      return fail_plan(plan, PBTC_EINVAL, "workspace not set up for this plan (call pbtc_setup)");
    if (!d_x || !d_y || d_x == d_y)
      return fail_plan(plan, PBTC_EINVAL, "x and y must be distinct device buffers");
    if (precision != PBTC_FP64 && precision != PBTC_FP32)
      return fail_plan(plan, PBTC_EINVAL, "precision must be PBTC_FP64 or PBTC_FP32");
    return apply_operator(*plan, (hipStream_t)hip_stream, d_x, d_y, precision, 0);
  });
}

int pbtc_matvec_transpose(pbtc_plan_t* plan, void* d_workspace, void* hip_stream, const double* d_x,
                          double* d_y, int precision) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  return guarded(plan, [&] {
    if (!ready(plan, d_workspace))
      return fail_plan(plan, PBTC_EINVAL, "workspace not set up for this plan (call pbtc_setup)");
    if (!d_x || !d_y || d_x == d_y)
      return fail_plan(plan, PBTC_EINVAL, "x and y must be distinct device buffers");
    if (precision != PBTC_FP64 && precision != PBTC_FP32)
      return fail_plan(plan, PBTC_EINVAL, "precision must be PBTC_FP64 or PBTC_FP32");
    return apply_transpose(*plan, (hipStream_t)hip_stream, d_x, d_y, precision, 0);
  });
}

int pbtc_precond_apply(pbtc_plan_t* plan, void* d_workspace, void* hip_stream, const double* d_x,
                       double* d_y, int transpose) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  return guarded(plan, [&] {
    if (!ready(plan, d_workspace))
      return fail_plan(plan, PBTC_EINVAL, "workspace not set up for this plan (call pbtc_setup)");
    if (!d_x || !d_y || d_x == d_y)
      return fail_plan(plan, PBTC_EINVAL, "x and y must be distinct device buffers");
    return apply_precond(*plan, (hipStream_t)hip_stream, d_x, d_y, transpose != 0, false);
  });
}

int pbtc_coulomb_energy(pbtc_plan_t* plan, void* d_workspace, void* hip_stream, double* total,
                        double* per_system) {
  if (!plan || !total) return fail_global(PBTC_EINVAL, "NULL argument");
  return guarded(plan, [&] {
    if (!ready(plan, d_workspace))
      return fail_plan(plan, PBTC_EINVAL, "workspace not set up for this plan (call pbtc_setup)");
    return device_coulomb(*plan, (hipStream_t)hip_stream, total, per_system);
  });
}

int pbtc_coulomb_energy_noalloc(pbtc_plan_t* plan, void* d_workspace, void* hip_stream,
                                double* total, double* per_system) {
  if (!plan || !total) return fail_global(PBTC_EINVAL, "NULL argument");
  return guarded(plan, [&] {
    if (!ready(plan, d_workspace))
      return fail_plan(plan, PBTC_EINVAL, "workspace not set up for this plan (call pbtc_setup)");
    return device_coulomb_noalloc(*plan, (hipStream_t)hip_stream, total, per_system);
  });
}

int pbtc_rhs(pbtc_plan_t* plan, void* d_workspace, void* hip_stream, double* d_b) {
  if (!plan || !d_b) return fail_global(PBTC_EINVAL, "NULL argument");
  return guarded(plan, [&] {
    if (!ready(plan, d_workspace))
      return fail_plan(plan, PBTC_EINVAL, "workspace not set up for this plan (call pbtc_setup)");
    if (plan->charges_dirty) {
      const int rc = update_charges(*plan, (hipStream_t)hip_stream);
      if (rc) return rc;
    }
    const hipError_t e = hipMemcpyAsync(d_b, static_cast<char*>(plan->ws) + plan->o_b,
                                        8 * plan->nunk, hipMemcpyDeviceToDevice,
                                        (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail_plan(plan, PBTC_EDEVICE, hipGetErrorString(e));
    return PBTC_OK;
  });
}

int pbtc_backward(pbtc_plan_t* plan, void* d_workspace, size_t bytes, void* hip_stream, double gE,
                  double* dE_dq, double* dE_dkappa, double* dE_deps, pbtc_result* res) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  return guarded(plan, [&] {
    if (!plan->dev_solved || !ready(plan, d_workspace) || bytes < plan->ws_bytes)
      return fail_plan(plan, PBTC_EINVAL, "call pbtc_solve on this workspace first");
    pbtc_result local;
    pbtc_result* r = res ? res : &local;
    std::memset(r, 0, sizeof(*r));
    fill_sizes(plan, r);
    return device_backward(*plan, (hipStream_t)hip_stream, gE, dE_dq, dE_dkappa, dE_deps, r);
  });
}

int pbtc_get_tree(pbtc_plan_t* plan, void* d_workspace, void* hip_stream, pbtc_tree_sizes* sizes,
                  double* cells, double* gauss_points, int64_t* surface_gp, double* targets,
                  double* groups, int64_t* items, int64_t* near_ptr, int32_t* near_cells,
                  int64_t* far_ptr, int32_t* far_cells) {
  if (!plan || !sizes) return fail_global(PBTC_EINVAL, "NULL argument");
  return guarded(plan, [&] {
    if (!ready(plan, d_workspace))
      return fail_plan(plan, PBTC_EINVAL, "workspace not set up for this plan (call pbtc_setup)");
    pbtc_plan_t& pl = *plan;
    hipStream_t st = (hipStream_t)hip_stream;
    sizes->n_cells = pl.n_cells;
    sizes->n_gauss_points = pl.ngp;
    sizes->n_targets = pl.ntgt;
    sizes->n_groups = pl.ngrp;
    sizes->n_items = pl.nitems;
    sizes->n_near = pl.n_near;
    sizes->n_far = pl.n_far;
    sizes->n_surfaces = pl.nsurf;
    sizes->ncrit = pl.ncrit;
    auto dev = [&](size_t off) { return static_cast<const char*>(pl.ws) + off; };
    auto get = [&](void* dst, size_t off, size_t bytes) -> int {
      if (bytes == 0) return PBTC_OK;
      PBTC_HIP(hipMemcpyAsync(dst, dev(off), bytes, hipMemcpyDeviceToHost, st));
      return PBTC_OK;
    };
    int rc = PBTC_OK;
    std::vector<Cell> hc;
    if (cells) {
      hc.resize(pl.n_cells);
      rc = get(hc.data(), pl.o_cells, sizeof(Cell) * pl.n_cells);
    }
    std::vector<double> x, y, z;
    if (!rc && gauss_points) {
      x.resize(pl.ngp), y.resize(pl.ngp), z.resize(pl.ngp);
      rc = get(x.data(), pl.o_gx, 8 * pl.ngp);
      if (!rc) rc = get(y.data(), pl.o_gy, 8 * pl.ngp);
      if (!rc) rc = get(z.data(), pl.o_gz, 8 * pl.ngp);
    }
    std::vector<double> tx, ty, tz;
    if (!rc && targets) {
      tx.resize(pl.ntgt), ty.resize(pl.ntgt), tz.resize(pl.ntgt);
      rc = get(tx.data(), pl.o_tx, 8 * pl.ntgt);
      if (!rc) rc = get(ty.data(), pl.o_ty, 8 * pl.ntgt);
      if (!rc) rc = get(tz.data(), pl.o_tz, 8 * pl.ntgt);
    }
    std::vector<double> gs;
    if (!rc && groups) {
      gs.resize(4 * pl.ngrp);
      rc = get(gs.data(), pl.o_grp, 32 * pl.ngrp);
    }
    std::vector<long long> np_, fp_;
    if (!rc && near_ptr) {
      np_.resize(pl.nitems + 1);
      rc = get(np_.data(), pl.o_near_ptr, 8 * (pl.nitems + 1));
    }
    if (!rc && far_ptr) {
      fp_.resize(pl.nitems + 1);
      rc = get(fp_.data(), pl.o_far_ptr, 8 * (pl.nitems + 1));
    }
    if (!rc && near_cells) rc = get(near_cells, pl.o_near, 4 * pl.n_near);
    if (!rc && far_cells) rc = get(far_cells, pl.o_far, 4 * pl.n_far);
    if (rc) return rc;
    PBTC_HIP(hipStreamSynchronize(st));
    for (int64_t c = 0; c < (int64_t)hc.size(); ++c) {
      const Cell& q = hc[c];
      double* o = cells + 9 * c;
      o[0] = q.cx, o[1] = q.cy, o[2] = q.cz, o[3] = q.h, o[4] = q.rb;
      o[5] = q.begin, o[6] = q.count, o[7] = q.nchild > 0 ? q.child : -1, o[8] = q.nchild;
    }
    for (int64_t i = 0; i < (int64_t)x.size(); ++i)
      gauss_points[3 * i] = x[i], gauss_points[3 * i + 1] = y[i], gauss_points[3 * i + 2] = z[i];
    if (surface_gp)
      for (int sf = 0; sf < pl.nsurf; ++sf)
        surface_gp[2 * sf] = pl.gp_off[sf], surface_gp[2 * sf + 1] = pl.gp_off[sf + 1];
    for (int64_t i = 0; i < (int64_t)tx.size(); ++i)
      targets[3 * i] = tx[i], targets[3 * i + 1] = ty[i], targets[3 * i + 2] = tz[i];
    if (groups)
      for (const TargetSet& ts : pl.tsets)
        for (int64_t g = 0; g < ts.ngrp; ++g) {
          double* o = groups + 6 * (ts.grp_off + g);
          const double* gsp = gs.data() + 4 * (ts.grp_off + g);
          o[0] = gsp[0], o[1] = gsp[1], o[2] = gsp[2], o[3] = gsp[3];
          o[4] = (double)(ts.off + g * kGroup);
          o[5] = (double)std::min<int64_t>(kGroup, ts.n - g * kGroup);
        }
    if (items)
      for (int64_t it = 0; it < pl.nitems; ++it) {
        const int bi = pl.item_block[it];
        const Block& b = pl.blocks[bi];
        const TargetSet& ts = pl.tsets[b.t];
        const int db = pl.prm.direct_below >= 0
                           ? pl.prm.direct_below
                           : (int)std::lround(0.7 * m2p_flop_per_eval(pl.P, b.ks) / p2p_flop_per_pair(b.ks));
        items[4 * it] = b.s;
        items[4 * it + 1] = ts.grp_off + (it - b.item_off);
        items[4 * it + 2] = db;
        items[4 * it + 3] = bi;
      }
    for (size_t i = 0; i < np_.size(); ++i) near_ptr[i] = np_[i];
    for (size_t i = 0; i < fp_.size(); ++i) far_ptr[i] = fp_[i];
    return PBTC_OK;
  });
}

int pbtc_get_systems(const pbtc_plan_t* plan, int* n_systems, double* energy_kJmol,
                     double* rel_res, int64_t* first_unknown) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  if (n_systems) *n_systems = plan->ncomp;
  if ((energy_kJmol || rel_res) && !plan->solved)
    return fail_global(PBTC_EINVAL, "no solution yet (call pbtc_solve)");
  for (int c = 0; c < plan->ncomp; ++c) {
    if (energy_kJmol) energy_kJmol[c] = plan->comp_energy[c];
    if (rel_res) rel_res[c] = c < (int)plan->comp_rel.size() ? plan->comp_rel[c] : 0.0;
    if (first_unknown) first_unknown[c] = plan->comp_u0[c];
  }
  return PBTC_OK;
}

int pbtc_set_charge_values(pbtc_plan_t* plan, const double* q) {
  if (!plan || !q) return fail_global(PBTC_EINVAL, "NULL argument");
  if (!finite_all(q, plan->nq)) return fail_plan(plan, PBTC_EINVAL, "charge value not finite");
  for (int r = 0; r < plan->nreg; ++r) {
    ChargeSet& c = plan->prob.charges[r];
    for (int64_t k = 0; k < c.n(); ++k) c.q[k] = q[plan->q_off_region[r] + k];
  }
  plan->charges_dirty = true;
  plan->solved = false;
  plan->dev_solved = false;
  ++plan->charge_version;
  return PBTC_OK;
}

int pbtc_triangle_rule(int K, double* bary, double* weights) {
  if (!bary || !weights) return fail_global(PBTC_EINVAL, "NULL argument");
  if (!triangle_rule(K, bary, weights)) return fail_global(PBTC_EINVAL, "no rule with that K");
  return PBTC_OK;
}

int pbtc_gauss_legendre(int n, double* nodes, double* weights) {
  if (!nodes || !weights) return fail_global(PBTC_EINVAL, "NULL argument");
  if (!gauss_legendre(n, nodes, weights)) return fail_global(PBTC_EINVAL, "n must be in 1..32");
  return PBTC_OK;
}

const char* pbtc_last_error(const pbtc_plan_t* plan) {
  if (plan) return plan->err.c_str();
  return g_err.c_str();
}

}  // extern "C"
