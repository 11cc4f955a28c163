// C interface of libpbtc (see include/pbtc.h for the contract).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

namespace pbtc {
bool triangle_rule(int k, double* bary, double* w);
bool gauss_legendre(int n, double* x, double* w);
std::string validate_problem(const pbtc_problem& p, const pbtc_params& prm, int* code);
int build_plan(pbtc_plan& pl);
void compute_layout(pbtc_plan& pl);
int device_setup(pbtc_plan& pl, hipStream_t st, int* need_retry);
int device_solve(pbtc_plan& pl, hipStream_t st, pbtc_result* res);
int update_charges(pbtc_plan& pl, hipStream_t st);
int device_backward(pbtc_plan& pl, hipStream_t st, double gE, double* dq, double* dk, double* de,
                    pbtc_result* res);
int apply_operator(pbtc_plan& pl, hipStream_t st, const double* x, double* y, int precision,
                   int phase);
int apply_transpose(pbtc_plan& pl, hipStream_t st, const double* x, double* y, int precision,
                    int phase);
int apply_precond(pbtc_plan& pl, hipStream_t st, const double* x, double* y, bool transpose,
                  bool accumulate);
double wall_seconds();
int device_coulomb(pbtc_plan& pl, hipStream_t st, double* total, double* per_system);
}  // namespace pbtc

using namespace pbtc;

namespace {

thread_local std::string g_err;

int fail_global(int code, const char* msg) {
  g_err = msg;
  return code;
}

int fail_plan(pbtc_plan* pl, int code, const std::string& msg) {
  pl->err = msg;
  return code;
}

bool finite_all(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

void fill_sizes(const pbtc_plan* pl, pbtc_result* res) {
  if (!res) return;
  res->n_p2p_pairs = pl->p2p_pairs;
  res->n_m2p_evals = pl->m2p_evals;
  res->n_dense_equiv = pl->dense_equiv;
  res->n_near_entries = (double)pl->n_nf;
  res->workspace_needed = pl->ws_bytes;
}

// Set-up on a workspace, growing capacity estimates as needed.
int setup_impl(pbtc_plan* pl, void* ws, size_t bytes, hipStream_t st, pbtc_result* res,
               bool reuse_inputs = false) {
  pl->setup_done = false;
  pl->solved = false;
  if (!reuse_inputs || pl->inputs_ws != ws) pl->inputs_ws = nullptr;
  for (int attempt = 0; attempt < 4; ++attempt) {
    if (bytes < pl->ws_bytes) {
      if (res) res->workspace_needed = pl->ws_bytes;
      return fail_plan(pl, PBTC_EWORKSPACE,
                       "workspace of " + std::to_string(bytes) + " bytes is smaller than the " +
                           std::to_string(pl->ws_bytes) + " bytes this plan needs");
    }
    pl->ws = ws;
    const double t0 = wall_seconds();
    int retry = 0;
    const int rc = device_setup(*pl, st, &retry);
    if (rc == PBTC_EWORKSPACE && retry) {
      compute_layout(*pl);
      pl->inputs_ws = nullptr;
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

}  // namespace

extern "C" {

int pbtc_version(int* major, int* minor) {
  if (major) *major = PBTC_VERSION_MAJOR;
  if (minor) *minor = PBTC_VERSION_MINOR;
  return PBTC_OK;
}

int pbtc_problem_create(pbtc_problem** out) {
  if (!out) return fail_global(PBTC_EINVAL, "out is NULL");
  *out = new (std::nothrow) pbtc_problem();
  if (!*out) return fail_global(PBTC_EINVAL, "out of host memory");
  return PBTC_OK;
}

void pbtc_problem_destroy(pbtc_problem* p) { delete p; }

int pbtc_add_region(pbtc_problem* p, double eps, double kappa, int* region_id) {
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
}

int pbtc_add_surface(pbtc_problem* p, const double* verts, int64_t nv, const int32_t* tris,
                     int64_t np, int inner_region, int outer_region, int* surface_id) {
  if (!p) return fail_global(PBTC_EINVAL, "problem is NULL");
  const int nreg = (int)p->regions.size();
  if (inner_region < 0 || inner_region >= nreg || outer_region < 0 || outer_region >= nreg)
    return fail_global(PBTC_EINVAL, "unknown region id");
  if (inner_region == outer_region) return fail_global(PBTC_EINVAL, "inner and outer region are equal");
  if (nv < 3 || np < 4 || !verts || !tris)
    return fail_global(PBTC_EINVAL, "a closed surface needs >= 3 vertices and >= 4 triangles");
  if (np >= (int64_t(1) << 30) || nv >= (int64_t(1) << 31)) return fail_global(PBTC_EINVAL, "surface too large");
  for (int64_t i = 0; i < 3 * np; ++i)
    if (tris[i] < 0 || tris[i] >= nv) return fail_global(PBTC_EINVAL, "triangle index out of range");
  if (!finite_all(verts, 3 * nv)) return fail_global(PBTC_EINVAL, "vertex coordinate not finite");
  Surface s;
  s.v.assign(verts, verts + 3 * nv);
  s.t.assign(tris, tris + 3 * np);
  s.inner = inner_region;
  s.outer = outer_region;
  p->surfaces.push_back(std::move(s));
  if (surface_id) *surface_id = (int)p->surfaces.size() - 1;
  return PBTC_OK;
}

int pbtc_set_charges(pbtc_problem* p, int region_id, const double* xyz, const double* q, int64_t nq) {
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
  return PBTC_OK;
}

int pbtc_validate(const pbtc_problem* p, const pbtc_params* prm) {
  if (!p || !prm) return fail_global(PBTC_EINVAL, "problem or params is NULL");
  int code = PBTC_OK;
  std::string msg = validate_problem(*p, *prm, &code);
  if (code) return fail_global(code, msg.c_str());
  return PBTC_OK;
}

int pbtc_plan_create(const pbtc_problem* p, const pbtc_params* prm, pbtc_plan** out,
                     size_t* workspace_bytes) {
  if (!p || !prm || !out) return fail_global(PBTC_EINVAL, "NULL argument");
  *out = nullptr;
  int code = PBTC_OK;
  std::string msg = validate_problem(*p, *prm, &code);
  if (code) return fail_global(code, msg.c_str());
  pbtc_plan* pl = new (std::nothrow) pbtc_plan();
  if (!pl) return fail_global(PBTC_EINVAL, "out of host memory");
  pl->prob = *p;
  pl->prm = *prm;
  const int rc = build_plan(*pl);
  if (rc) {
    delete pl;
    return fail_global(rc, "problem too large for 32-bit indices");
  }
  *out = pl;
  if (workspace_bytes) *workspace_bytes = pl->ws_bytes;
  return PBTC_OK;
}

pbtc_plan::~pbtc_plan() {
  for (auto* v : {&prof, &prof_pool})
    for (auto& ev : *v) {
      (void)hipEventDestroy(ev.a);
      (void)hipEventDestroy(ev.b);
    }
  for (hipEvent_t e : res_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : {ev_fork, ev_join})
    if (e) (void)hipEventDestroy(e);
  if (side) (void)hipStreamDestroy(side);
  if (res_pin) (void)hipHostFree(res_pin);
}

void pbtc_plan_destroy(pbtc_plan* plan) { delete plan; }

int pbtc_plan_sizes(const pbtc_plan* plan, int64_t* n_unknowns, int64_t* n_charges,
                    int* n_surfaces, int* n_regions) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  if (n_unknowns) *n_unknowns = plan->nunk;
  if (n_charges) *n_charges = plan->nq;
  if (n_surfaces) *n_surfaces = plan->nsurf;
  if (n_regions) *n_regions = plan->nreg;
  return PBTC_OK;
}

int pbtc_setup(pbtc_plan* plan, void* d_workspace, size_t bytes, void* hip_stream, pbtc_result* res) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  if (!d_workspace) return fail_plan(plan, PBTC_EINVAL, "workspace is NULL");
  if (res) std::memset(res, 0, sizeof(*res));
  return setup_impl(plan, d_workspace, bytes, (hipStream_t)hip_stream, res);
}

int pbtc_solve(pbtc_plan* plan, void* d_workspace, size_t bytes, void* hip_stream, int force_setup,
               pbtc_result* res) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  if (!d_workspace) return fail_plan(plan, PBTC_EINVAL, "workspace is NULL");
  pbtc_result local;
  if (!res) res = &local;
  std::memset(res, 0, sizeof(*res));
  hipStream_t st = (hipStream_t)hip_stream;
  if (force_setup || !plan->setup_done || plan->ws != d_workspace) {
    const int rc = setup_impl(plan, d_workspace, bytes, st, res, force_setup != 0);
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

int pbtc_get_surface(const pbtc_plan* plan, int surface_id, double* phi, double* dphidn_inner) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  if (!plan->solved) return fail_global(PBTC_EINVAL, "no solution yet (call pbtc_solve)");
  if (surface_id < 0 || surface_id >= plan->nsurf) return fail_global(PBTC_EINVAL, "unknown surface");
  const int64_t o = plan->unk_off[surface_id];
  const int64_t n = plan->pan_off[surface_id + 1] - plan->pan_off[surface_id];
  if (phi) std::memcpy(phi, plan->x_host.data() + o, 8 * n);
  if (dphidn_inner) std::memcpy(dphidn_inner, plan->x_host.data() + o + n, 8 * n);
  return PBTC_OK;
}

int pbtc_get_phi_reac(const pbtc_plan* plan, double* phi_reac) {
  if (!plan || !phi_reac) return fail_global(PBTC_EINVAL, "NULL argument");
  if (!plan->solved) return fail_global(PBTC_EINVAL, "no solution yet (call pbtc_solve)");
  std::memcpy(phi_reac, plan->phi_reac_host.data(), 8 * plan->nq);
  return PBTC_OK;
}

int pbtc_get_history(const pbtc_plan* plan, double* rel_res, int cap, int* n_iter) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  const int n = (int)plan->history.size();
  if (n_iter) *n_iter = n;
  if (rel_res)
    for (int i = 0; i < n && i < cap; ++i) rel_res[i] = plan->history[i];
  return PBTC_OK;
}

int pbtc_matvec(pbtc_plan* plan, void* d_workspace, void* hip_stream, const double* d_x, double* d_y,
                int precision) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  if (!plan->setup_done || plan->ws != d_workspace)
    return fail_plan(plan, PBTC_EINVAL, "workspace not set up (call pbtc_setup)");
  if (!d_x || !d_y || d_x == d_y) return fail_plan(plan, PBTC_EINVAL, "x and y must be distinct device buffers");
  if (precision != PBTC_FP64 && precision != PBTC_FP32)
    return fail_plan(plan, PBTC_EINVAL, "precision must be PBTC_FP64 or PBTC_FP32");
  return apply_operator(*plan, (hipStream_t)hip_stream, d_x, d_y, precision, 0);
}

int pbtc_matvec_transpose(pbtc_plan* plan, void* d_workspace, void* hip_stream, const double* d_x,
                          double* d_y, int precision) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  if (!plan->setup_done || plan->ws != d_workspace)
    return fail_plan(plan, PBTC_EINVAL, "workspace not set up (call pbtc_setup)");
  if (!d_x || !d_y || d_x == d_y) return fail_plan(plan, PBTC_EINVAL, "x and y must be distinct device buffers");
  if (precision != PBTC_FP64 && precision != PBTC_FP32)
    return fail_plan(plan, PBTC_EINVAL, "precision must be PBTC_FP64 or PBTC_FP32");
  return apply_transpose(*plan, (hipStream_t)hip_stream, d_x, d_y, precision, 0);
}

int pbtc_precond_apply(pbtc_plan* plan, void* d_workspace, void* hip_stream, const double* d_x,
                       double* d_y, int transpose) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  if (!plan->setup_done || plan->ws != d_workspace)
    return fail_plan(plan, PBTC_EINVAL, "workspace not set up (call pbtc_setup)");
  if (!d_x || !d_y || d_x == d_y) return fail_plan(plan, PBTC_EINVAL, "x and y must be distinct device buffers");
  return apply_precond(*plan, (hipStream_t)hip_stream, d_x, d_y, transpose != 0, false);
}

int pbtc_coulomb_energy(pbtc_plan* plan, void* d_workspace, void* hip_stream, double* total,
                        double* per_system) {
  if (!plan || !total) return fail_global(PBTC_EINVAL, "NULL argument");
  if (!plan->setup_done || plan->ws != d_workspace)
    return fail_plan(plan, PBTC_EINVAL, "workspace not set up (call pbtc_setup)");
  const int rc = device_coulomb(*plan, (hipStream_t)hip_stream, total, per_system);
  if (rc) return fail_plan(plan, rc, plan->err.c_str());
  return PBTC_OK;
}

int pbtc_rhs(pbtc_plan* plan, void* d_workspace, void* hip_stream, double* d_b) {
  if (!plan || !d_b) return fail_global(PBTC_EINVAL, "NULL argument");
  if (!plan->setup_done || plan->ws != d_workspace)
    return fail_plan(plan, PBTC_EINVAL, "workspace not set up (call pbtc_setup)");
  const hipError_t e = hipMemcpyAsync(d_b, static_cast<char*>(plan->ws) + plan->o_b,
                                      8 * plan->nunk, hipMemcpyDeviceToDevice,
                                      (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail_plan(plan, PBTC_EDEVICE, hipGetErrorString(e));
  return PBTC_OK;
}

int pbtc_backward(pbtc_plan* plan, void* d_workspace, size_t bytes, void* hip_stream, double gE,
                  double* dE_dq, double* dE_dkappa, double* dE_deps, pbtc_result* res) {
  if (!plan) return fail_global(PBTC_EINVAL, "plan is NULL");
  if (!plan->solved || plan->ws != d_workspace || bytes < plan->ws_bytes)
    return fail_plan(plan, PBTC_EINVAL, "call pbtc_solve on this workspace first");
  pbtc_result local;
  if (!res) res = &local;
  std::memset(res, 0, sizeof(*res));
  fill_sizes(plan, res);
  return device_backward(*plan, (hipStream_t)hip_stream, gE, dE_dq, dE_dkappa, dE_deps, res);
}

int pbtc_get_systems(const pbtc_plan* plan, int* n_systems, double* energy_kJmol,
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

int pbtc_set_charge_values(pbtc_plan* plan, const double* q) {
  if (!plan || !q) return fail_global(PBTC_EINVAL, "NULL argument");
  if (!finite_all(q, plan->nq)) return fail_plan(plan, PBTC_EINVAL, "charge value not finite");
  for (int r = 0; r < plan->nreg; ++r) {
    ChargeSet& c = plan->prob.charges[r];
    for (int64_t k = 0; k < c.n(); ++k) c.q[k] = q[plan->q_off_region[r] + k];
  }
  plan->charges_dirty = true;
  plan->solved = false;
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

const char* pbtc_last_error(const pbtc_plan* plan) {
  if (plan) return plan->err.c_str();
  return g_err.c_str();
}

}  // extern "C"
