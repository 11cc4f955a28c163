/*
 * pbtc.h -- C interface of libpbtc, a treecode-accelerated boundary-element
 * Poisson-Boltzmann solver for AMD Instinct MI355X (gfx950).
 *
 * Method: arXiv:1309.4018 (Cooper, Bardhan, Barba).  The problem statement
 * follows sec. 2.1 (Eq. pde: Poisson with point charges inside the molecule,
 * linearized Poisson-Boltzmann with inverse Debye length kappa in the
 * solvent, continuity of the potential and of eps d phi/dn on every
 * interface) and sec. 2.2 (single- and multi-surface problems: Stern layers
 * and solvent-filled cavities add surfaces).  The discrete operator is the
 * constant-element, centroid-collocation BEM of sec. 2.2 (Eqs. nBEM_disc,
 * matrix, matel), evaluated by the Cartesian-Taylor treecode of sec. 2.3
 * (Eqs. nbody, taylor, multexp, MAC) with semi-analytic self integrals and a
 * K_fine-point rule in the near-singular zone; the system is solved by GMRES
 * (sec. 2.3, one operator evaluation per iteration, tree and lists built
 * once) and the solvation energy follows Eqs. reac_integral and solv.
 *
 * Conventions
 *   Units: angstrom, elementary charge e, kJ/mol.
 *   Regions: permittivity eps > 0 and kappa >= 0 (kappa = 0: Laplace).
 *   Surfaces: closed triangulations, each separating an inner region from an
 *     outer region; triangles counter-clockwise seen from the outer region,
 *     so the normal points from the inner into the outer region.
 *   Unknowns of surface s: phi_s (potential at each panel centre) and
 *     psi_s = d phi / d n on the inner side; the outer-side derivative is
 *     (eps_inner / eps_outer) psi_s.
 *   Unknown vector layout (pbtc_matvec): for each surface in creation order,
 *     [phi_s (n_s), psi_s (n_s)], FP64.
 *
 * Ownership
 *   Host input arrays belong to the caller and are copied during the call.
 *   Output buffers are caller-allocated.  All device memory is ONE workspace
 *   that the caller allocates (any device allocation >= the size that
 *   pbtc_plan reports) and passes to every device call together with a
 *   hipStream_t (NULL = the default stream).  The library never calls
 *   hipMalloc/hipFree.  A workspace holds the device state of ONE plan (or
 *   of one batch, pbtc_solve_batch) between calls: tree, lists, near-field
 *   tables, solution.  The library remembers which plan last set a workspace
 *   up: a solve on a workspace that another plan (or batch) has used since,
 *   or on a different workspace pointer, rebuilds the state first, and the
 *   calls that need the state (pbtc_matvec, pbtc_backward, ...) return
 *   PBTC_EINVAL instead of reading another plan's data.
 *
 * Errors
 *   Every int-returning function returns PBTC_OK (0) or a negative code.
 *   pbtc_last_error(plan) returns the message of the plan's last error
 *   (pbtc_last_error(NULL): the calling thread's last error of a call that
 *   has no plan).  No C++ exception crosses this interface.
 *
 * Threading
 *   A plan or problem must not be used by two threads at once; different
 *   plans are independent.  Device work is issued on the caller's stream;
 *   calls that return host results synchronise that stream.
 */
#ifndef PBTC_H
#define PBTC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PBTC_VERSION_MAJOR 1
#define PBTC_VERSION_MINOR 0

#define PBTC_OK 0
#define PBTC_EINVAL -1     /* bad argument, NaN/Inf, unknown id, bad call order */
#define PBTC_EMESH -2      /* degenerate panel, open or mis-oriented surface */
#define PBTC_ECHARGE -3    /* a charge is not inside its region */
#define PBTC_EWORKSPACE -4 /* workspace too small; pbtc_result.workspace_needed */
#define PBTC_EDEVICE -5    /* HIP runtime error */
#define PBTC_ENOCONV -6    /* GMRES hit max_iter; outputs hold the last iterate */
#define PBTC_KERNEL_KINDS 7 /* kernel kinds timed in pbtc_result */
#define PBTC_EHOST -7      /* host-side failure: out of host memory or another
                              internal error (no exception leaves the library) */

/* Arithmetic of the operator kernels (tree passes, P2P, M2P, near field). */
#define PBTC_FP64 0         /* everything in FP64 */
#define PBTC_FP32_REFINED 1 /* FP32 operator inside FP64 iterative refinement */
#define PBTC_FP32 2         /* FP32 operator, FP64 Krylov; no refinement */

/* How the operator is evaluated. */
#define PBTC_OP_TREECODE 0 /* Taylor treecode: M2P where the MAC holds, P2P else */
#define PBTC_OP_DIRECT 1   /* every pair by the K-point rule (dense, O(N^2)) */

/* Right preconditioner of the GMRES solves.  The paper names none (sec. 2.3);
 * the block-diagonal one leaves the solution and the residual test
 * unchanged (GMRES on A M^-1, x = M^-1 y) and only reduces iterations. */
#define PBTC_PREC_NONE 0
#define PBTC_PREC_BLOCK_DIAG 1 /* per panel, the 2 x 2 block of A coupling its
                                  two rows (inner / outer region) with its own
                                  phi and psi: self terms only */

typedef struct pbtc_problem pbtc_problem;
typedef struct pbtc_plan_s pbtc_plan_t;

typedef struct {
  /* discretisation (sec. 3, parameter tables) */
  int K;         /* Gauss points per panel: 1, 3, 4 or 7 */
  int K_fine;    /* points of the near-singular rule: 7 or 19 */
  int N_k;       /* Gauss-Legendre points per sub-triangle of the self term */
  double thres;  /* near-singular zone: |x - centre_j| < thres * L_j, L = sqrt(2A) */
  /* treecode (sec. 2.3) */
  double theta;  /* MAC: accept a cell when theta * r_tb > r_b */
  int P;         /* Taylor order: 2, 4, 6, 8 or 10 */
  int ncrit;     /* split a cell holding >= ncrit sources (2..256); 0 = automatic */
  int direct_below; /* a MAC-accepted cell with fewer sources goes to P2P; -1 =
                       auto: per block, where P2P costs less than one M2P
                       evaluation of the block's kernels */
  /* solver (sec. 2.3: Krylov; tolerance from the parameter tables) */
  double tol;       /* stop at ||b - A x|| / ||b|| <= tol */
  int restart;      /* GMRES restart length m (<= 256) */
  int max_iter;     /* total GMRES iterations (all restarts, all refinements) */
  int precision;    /* PBTC_FP64, PBTC_FP32_REFINED or PBTC_FP32 */
  int op;           /* PBTC_OP_TREECODE or PBTC_OP_DIRECT */
  double inner_tol; /* FP32_REFINED: relative tolerance floor of inner solves */
  int max_refine;   /* FP32_REFINED: maximum outer refinement steps */
  int validate_charges; /* 1: check every charge lies inside its region */
  int profile;      /* n > 0: time the P2P and M2P kernel launches of every
                       n-th evaluation of the FP32 operator (A x, and A^T x
                       in pbtc_backward) with HIP events on the caller's
                       stream (pbtc_result.t_kernel_s ...); 0: off.  Other
                       evaluations run the far field (moment pass, M2P) on a
                       second stream beside the near field (near-field
                       corrections, P2P) and replay the launch graph; a
                       timed one launches kernel by kernel on one stream
                       with the moment pass first, so that each timed launch
                       has the GPU alone */
  int precond;      /* PBTC_PREC_NONE or PBTC_PREC_BLOCK_DIAG (forward and
                       adjoint solves) */
  int unit_sources; /* work tile of P2P: one wavefront takes a group of 16
                       targets (four lanes per target) and a run of its
                       near-list cells of at most this many sources (whole
                       cells; 64..8192); 0 = automatic: the largest of 2048,
                       1024, 512 that gives the launch ~1.5 rounds of waves
                       on the GPU (a short tail).  The transposed operator
                       (64 Gauss points per wavefront) uses a quarter. */
  int unit_cells;   /* work tile of M2P: a group of 16 targets and at most
                       this many of its far cells (1..1024); 0 = automatic:
                       the largest of 128, 64, 32 by the same rule (a
                       quarter for the transposed operator) */
  int op_graph;     /* 1: evaluations of A x (all surface-pair blocks of
                       all regions and systems) are replayed as ONE captured
                       HIP launch graph of its kernels, captured once per
                       set-up and precision at the second evaluation (the
                       first after a set-up launches its kernels one by one);
                       0: the kernels are always launched one by one (same
                       kernels, same results bit for bit) */
} pbtc_params;

typedef struct {
  double energy_kJmol;   /* solvation energy, Eq. solv */
  int n_iter;            /* GMRES iterations (all restarts / refinements) */
  int converged;         /* 1 if the explicit residual met tol */
  double final_rel_res;  /* explicit ||b - A x|| / ||b|| (FP64 operator) */
  int n_matvec_fp32;     /* operator evaluations in FP32 whose results were used
                            (the evaluation GMRES queues while it reads the
                            previous residual is not counted when discarded) */
  int n_matvec_fp64;     /* operator evaluations in FP64, likewise */
  int n_refine;          /* outer refinement steps (FP32_REFINED) */
  double t_setup_s;      /* device set-up: geometry, tree, lists, near field, RHS */
  double t_solve_s;      /* Krylov solve incl. refinement */
  double t_energy_s;     /* reaction potential + energy */
  double n_p2p_pairs;    /* per operator evaluation: (target, Gauss point) pairs in P2P */
  double n_m2p_evals;    /* per operator evaluation: (target, cell) Taylor evaluations */
  double n_dense_equiv;  /* per operator evaluation: sum over regions of targets x sources */
  double n_near_entries; /* near-field correction entries */
  size_t workspace_needed; /* bytes (set on PBTC_EWORKSPACE and on success) */
  /* with params.profile: summed HIP-event durations, launch counts and
   * algorithmic FP operations of the P2P and M2P kernel launches of the
   * FP32 operator (A x) during the call; M2P counts every M2P launch */
  double t_p2p_s, t_m2p_s;
  int n_p2p_launch, n_m2p_launch;
  double p2p_flop, m2p_flop;
  /* the share of the M2P launches of Yukawa-only blocks */
  double t_m2p_yuk_s;
  int n_m2p_yuk_launch;
  double m2p_yuk_flop;
  /* host wall-clock split of the last device set-up (seconds): [0] panels,
   * Gauss points and targets in Morton order, [1] octrees, [2] interaction
   * lists, [3] near-field columns, [4] work-unit and moment tables built on
   * the host while the GPU computes the near-field values, preconditioner
   * blocks and Coulomb right-hand side, [5] the rest of that GPU work */
  double t_setup_phase_s[6];
  /* kernels of one evaluation of the FP32 operator A x (the nodes of its
   * launch graph) and how many evaluations replayed the graph in the call */
  int op_kernels;
  int op_graph_launches;
  /* with params.profile, per kernel kind -- [0] P2P, [1] Laplace M2P,
   * [2] Yukawa M2P of the FP32 A x (pbtc_solve), [3] P2P, [4] Laplace M2P,
   * [5] Yukawa M2P of the FP32 A^T x (pbtc_backward), [6] M2P of the FP32
   * A x for blocks of two Green's functions (Laplace + Yukawa or two Yukawa
   * kernels evaluated in one pass over the cells) -- the summed HIP-event
   * seconds, the timed launches and their algorithmic floating-point
   * operations (FMA = 2, a transcendental = 1) */
  double t_kernel_s[PBTC_KERNEL_KINDS];
  int n_kernel_launch[PBTC_KERNEL_KINDS];
  double kernel_flop[PBTC_KERNEL_KINDS];
  /* the P2P and M2P work tiles the set-up used (params.unit_sources and
   * unit_cells, or the automatic choice) */
  int tile_sources, tile_cells;
} pbtc_result;

/* Library version; never fails. */
int pbtc_version(int* major, int* minor);

/* Problem description (host only). */
int pbtc_problem_create(pbtc_problem** out);
void pbtc_problem_destroy(pbtc_problem* p);
/* Adds a region; ids are 0, 1, 2, ... in call order.  EINVAL: eps <= 0,
 * kappa < 0 or not finite. */
int pbtc_add_region(pbtc_problem* p, double eps, double kappa, int* region_id);
/* Adds a closed surface: verts (nv x 3, row-major), tris (np x 3 vertex
 * indices, counter-clockwise seen from outer_region).  The arrays are copied.
 * EINVAL: unknown or equal region ids, sizes < 1, indices out of range. */
int pbtc_add_surface(pbtc_problem* p, const double* verts, int64_t nv, const int32_t* tris,
                     int64_t np, int inner_region, int outer_region, int* surface_id);
/* Sets (replaces) the point charges of one region: xyz (nq x 3), q (nq). */
int pbtc_set_charges(pbtc_problem* p, int region_id, const double* xyz, const double* q,
                     int64_t nq);

/* Defaults: K=4, K_fine=19, N_k=5, thres=2.0, theta=0.5, P=6, ncrit=0,
 * direct_below=-1, tol=1e-5, restart=100, max_iter=1000,
 * precision=PBTC_FP32_REFINED, op=PBTC_OP_TREECODE, inner_tol=1e-6,
 * max_refine=10, validate_charges=1, profile=0, precond=PBTC_PREC_NONE,
 * unit_sources=0, unit_cells=0, op_graph=1. */
int pbtc_params_default(pbtc_params* prm);

/* Host-side checks only (no device work): parameter ranges; every region is
 * bounded by a surface; every surface closed (each directed edge matched by
 * its reverse exactly once), non-degenerate and oriented with its normal
 * toward the outer region (positive enclosed volume for an outer region
 * that contains infinity or encloses the surface); every charge finite and
 * (if validate_charges) inside its region (ray parity against the region's
 * bounding surfaces).  Returns EINVAL, EMESH or ECHARGE with a message. */
int pbtc_validate(const pbtc_problem* p, const pbtc_params* prm);

/* Validates, fixes the block structure (which surface pairs interact in
 * which region) and returns the workspace size for pbtc_setup/pbtc_solve.
 * The size includes an estimate for the interaction lists; pbtc_setup
 * returns EWORKSPACE with the exact need if the estimate was low.  The
 * problem is copied: later changes to it do not reach the plan. */
int pbtc_plan(const pbtc_problem* p, const pbtc_params* prm, pbtc_plan_t** out,
              size_t* workspace_bytes);
void pbtc_plan_destroy(pbtc_plan_t* plan);

/* Unknowns (2 * total panels), charges, surfaces and regions of a plan. */
int pbtc_plan_sizes(const pbtc_plan_t* plan, int64_t* n_unknowns, int64_t* n_charges,
                    int* n_surfaces, int* n_regions);

/* Device set-up on the caller's workspace and stream, once per geometry
 * (sec. 2.3: the tree and interaction lists are built once and reused by
 * every iteration): copies the inputs to the device, forms panel geometry
 * and Gauss points, sorts them in Morton order, builds one octree per
 * surface, the interaction lists, the near-singular correction tables and
 * the Coulomb right-hand side.  Synchronises the stream.  res may be NULL. */
int pbtc_setup(pbtc_plan_t* plan, void* d_workspace, size_t bytes, void* hip_stream,
               pbtc_result* res);

/* Solves the BEM system by GMRES and evaluates the solvation energy.  Runs
 * pbtc_setup first when the workspace is not set up; force_setup != 0
 * rebuilds every device structure (geometry, Gauss points, tree, lists,
 * near field, right-hand side) from the inputs already in the workspace.
 * Returns ENOCONV (outputs valid) when max_iter is reached. */
int pbtc_solve(pbtc_plan_t* plan, void* d_workspace, size_t bytes, void* hip_stream,
               int force_setup, pbtc_result* res);

/* After pbtc_solve: phi (n_s) and d phi/dn on the inner side (n_s) of one
 * surface in its triangle order (host buffers). */
int pbtc_get_surface(const pbtc_plan_t* plan, int surface_id, double* phi, double* dphidn_inner);
/* Reaction potential at every charge (regions in id order, charges in the
 * order given), host buffer of n_charges. */
int pbtc_get_phi_reac(const pbtc_plan_t* plan, double* phi_reac);
/* GMRES implicit relative residual per iteration (host buffer). */
int pbtc_get_history(const pbtc_plan_t* plan, double* rel_res, int cap, int* n_iter);

/* y = A x with the plan's operator (sec. 2.2 Eq. matrix and its
 * multi-surface form), x and y DEVICE pointers to n_unknowns FP64 values,
 * evaluated in `precision` (PBTC_FP64 or PBTC_FP32) with the plan's op.
 * Requires pbtc_setup on the same workspace.  Does not synchronise. */
int pbtc_matvec(pbtc_plan_t* plan, void* d_workspace, void* hip_stream, const double* d_x,
                double* d_y, int precision);
/* y = A^T x (exact transpose of the same discrete operator).  Device
 * pointers as for pbtc_matvec. */
int pbtc_matvec_transpose(pbtc_plan_t* plan, void* d_workspace, void* hip_stream,
                          const double* d_x, double* d_y, int precision);
/* y = M^-1 x (transpose = 0) or y = M^-T x (transpose = 1) for the
 * block-diagonal preconditioner M of PBTC_PREC_BLOCK_DIAG, whatever
 * params.precond says.  For panel p of surface t with unknowns phi_p, psi_p
 * (Eq. matrix and its multi-surface form; the self integral of sec. 2.3):
 *   M_p = [[1/2, -V_I(p,p)], [1/2, (eps_I / eps_O) V_O(p,p)]],
 * rows (t, inner region I) and (t, outer region O), V_r(p,p) the singular
 * integral of G_r over p at its centre (the double layer of a flat panel at
 * its own centre is zero).  M^-1 maps a vector in row layout to the unknown
 * layout (both are the pbtc_matvec layout).  x, y: distinct DEVICE buffers of
 * n_unknowns FP64 values; requires pbtc_setup on the workspace; does not
 * synchronise.  EINVAL for NULL or aliased buffers. */
int pbtc_precond_apply(pbtc_plan_t* plan, void* d_workspace, void* hip_stream, const double* d_x,
                       double* d_y, int transpose);
/* Coulomb energy of the point charges (Eq. total_energy: the total energy
 * of a species is its solvation energy plus this term; Eq. bind_energy
 * combines three of them).  Pairs within each region, with that region's
 * permittivity: E_C = k_e sum_r sum_{i<j in r} q_i q_j / (eps_r |x_i - x_j|)
 * in kJ/mol (charges of different regions interact through the reaction
 * potential only).  FP64 on the device; *total (host) receives the sum and
 * per_system (host, n_systems values as in pbtc_get_systems, may be NULL)
 * each independent system's share.  Requires pbtc_setup on the workspace;
 * synchronises the stream.  EINVAL for NULL total or when two charges of one
 * region coincide (non-finite energy). */
int pbtc_coulomb_energy(pbtc_plan_t* plan, void* d_workspace, void* hip_stream, double* total,
                        double* per_system);
/* pbtc_coulomb_energy for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid allocation):
 * the same arguments, kernels and results, with the scratch the kernels need
 * (the Coulomb potential at every charge, the region table, the per-system
 * sums) in a fixed device array inside the library instead of the plan's
 * workspace; the plan's charges are read from d_workspace as before.
 * Limits: at most 1,048,576 charges and 2 n_regions + 1 + n_systems <= 65,536
 * (EINVAL beyond).  The array (9 MiB) is held by each GPU the library runs on
 * until the process ends and is shared by every call on that GPU: calls that
 * overlap on one GPU (different streams or threads) race.  No device or host
 * memory is allocated during the call. */
int pbtc_coulomb_energy_noalloc(pbtc_plan_t* plan, void* d_workspace, void* hip_stream,
                                double* total, double* per_system);
/* The Coulomb right-hand side b (Eq. matel Q) into a device buffer of
 * n_unknowns FP64 values. */
int pbtc_rhs(pbtc_plan_t* plan, void* d_workspace, void* hip_stream, double* d_b);

/* Gradients of the solvation energy by the adjoint method: solves
 * A^T lambda = S^T q (S: unknowns -> reaction potential at the charges)
 * with GMRES on the transposed operator, then
 *   dE/dq_k     = 1/2 C (S x + B^T lambda)_k,
 *   dE/dkappa_r = 1/2 C [q^T S'_r x - lambda^T A'_r x + lambda^T B'_r q],
 *   dE/deps_r   likewise with the eps derivatives,
 * C = 4 pi k_e.  Requires a converged pbtc_solve on the same workspace.
 * Host outputs: dE_dq (n_charges), dE_dkappa and dE_deps (n_regions); any
 * may be NULL.  The energy is scaled by gE (dL/dE of a caller's loss). */
int pbtc_backward(pbtc_plan_t* plan, void* d_workspace, size_t bytes, void* hip_stream,
                  double gE, double* dE_dq, double* dE_dkappa, double* dE_deps,
                  pbtc_result* res);

/* Independent systems.  A problem may hold several molecules whose regions
 * never meet (an uneven batch): every connected component of the region
 * graph (regions linked by surfaces) is a linear system of its own, with its
 * own Krylov space, Givens rotations and convergence test, while every
 * operator evaluation of all systems shares each kernel launch.  The
 * surfaces of one system must be added consecutively (else the whole problem
 * is solved as one system).  After pbtc_solve: n_systems, and per system
 * (host buffers of n_systems, any may be NULL) the solvation energy, the
 * explicit FP64 relative residual, and the first unknown / charge index. */
int pbtc_get_systems(const pbtc_plan_t* plan, int* n_systems, double* energy_kJmol,
                     double* rel_res, int64_t* first_unknown);

/* Solves n plans (sec. 2.1-2.2 problem statement, one per molecule) as one
 * batch on one workspace: every GMRES iteration of all their systems shares
 * each kernel launch (an uneven batch of molecules), while every system keeps
 * its own Krylov space, Givens rotations and convergence test, so the
 * results equal those of n separate pbtc_solve calls up to rounding.
 *   plans: n >= 1 distinct plans made with identical pbtc_params (EINVAL
 *     otherwise); the library merges their problems (regions, surfaces and
 *     charges in plan order) into one internal plan that it keeps with
 *     plans[0] and reuses while the same plans are passed in the same order
 *     (charge values set with pbtc_set_charge_values are carried over).
 *   d_workspace, bytes: one device workspace for the whole batch.  When it is
 *     smaller than the batch needs (bytes = 0 asks), the call returns
 *     EWORKSPACE with the size in res[0].workspace_needed and does no work.
 *   res: host array of n results: energy_kJmol, converged and final_rel_res
 *     are per plan; n_iter, matvec counts, timings and interaction counts
 *     are the batch's.
 * Afterwards pbtc_get_surface, pbtc_get_phi_reac, pbtc_get_history (the
 * batch's history: per iteration the largest implicit residual over its
 * systems) and pbtc_get_systems answer per plan.  The batch state lives in
 * the batch workspace, so pbtc_backward on a member needs pbtc_solve on
 * the member's own workspace first.  Returns ENOCONV if any system missed
 * the tolerance (every plan's outputs are still filled). */
int pbtc_solve_batch(pbtc_plan_t** plans, int n, void* d_workspace, size_t bytes,
                     void* hip_stream, pbtc_result* res);

/* Replaces the values (not the positions) of every charge of a plan, in the
 * order of pbtc_get_phi_reac (nq values, host).  The next pbtc_solve reuses
 * the device set-up and only rebuilds the right-hand side. */
int pbtc_set_charge_values(pbtc_plan_t* plan, const double* q);

/* Host-side tables used by the library (no device work), for checking:
 * barycentric points (K x 3) and weights (K) of the K-point triangle rule;
 * Gauss-Legendre nodes and weights on [-1, 1]. */
int pbtc_triangle_rule(int K, double* bary, double* weights);
int pbtc_gauss_legendre(int n, double* nodes, double* weights);

/* Sizes of the source octrees and forward interaction lists (pbtc_get_tree). */
typedef struct {
  int64_t n_cells, n_gauss_points, n_targets, n_groups, n_items, n_near, n_far;
  int n_surfaces, ncrit;
} pbtc_tree_sizes;

/* The octrees over the Gauss points and the forward interaction lists of the
 * set-up on d_workspace (sec. 2.3: cells split while they hold ncrit or more
 * points; Eq. MAC), copied to host buffers for checking; synchronises the
 * stream.  sizes is required; every buffer may be NULL (then skipped):
 *   cells        n_cells x 9 FP64: centre x, y, z, half edge, r_b (largest
 *                centre-point distance), first Gauss point, count, first
 *                child, number of children (0: a leaf); cells of all
 *                surfaces, surface s's root is cell s
 *   gauss_points n_gauss_points x 3: the Gauss points in tree order
 *   surface_gp   n_surfaces x 2 int64: each surface's range of them
 *   targets      n_targets x 3: targets (collocation points, then charges)
 *                in group order
 *   groups       n_groups x 6 FP64: bounding sphere (x, y, z, radius), first
 *                target, number of targets of every target group
 *   items        n_items x 4 int64 (one per block and target group): the
 *                source surface's root cell, the group, the block's P2P
 *                threshold (MAC-accepted cells with fewer points are P2P),
 *                the block
 *   near_ptr, far_ptr  n_items + 1 int64 offsets into near / far (int32
 *                cell ids)
 * EINVAL without a set-up of this plan on d_workspace. */
int pbtc_get_tree(pbtc_plan_t* plan, void* d_workspace, void* hip_stream, pbtc_tree_sizes* sizes,
                  double* cells, double* gauss_points, int64_t* surface_gp, double* targets,
                  double* groups, int64_t* items, int64_t* near_ptr, int32_t* near_cells,
                  int64_t* far_ptr, int32_t* far_cells);

/* Message of the last error of `plan` (or of the calling thread when plan
 * is NULL).  The pointer stays valid until the next call on that plan. */
const char* pbtc_last_error(const pbtc_plan_t* plan);

#ifdef __cplusplus
}
#endif

#endif /* PBTC_H */
