// Internal structures of libpbtc shared by the host driver and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "pbtc.h"

namespace pbtc {

constexpr double kPi = 3.14159265358979323846;
constexpr double kInv4Pi = 0.0795774715459476678844;  // 1 / (4 pi)
// k_e = e^2 N_A / (4 pi eps_0 * 1 angstrom) in kJ A / (mol e^2)
constexpr double kCoulomb = 1389.35458;

constexpr int kMaxP = 10;
// Timed kernel kinds: 0 P2P, 1 Laplace M2P, 2 Yukawa M2P of A x; 3 P2P,
// 4 Laplace M2P, 5 Yukawa M2P of A^T x; 6 M2P of two Green's functions per
// cell pass (Laplace + Yukawa or two Yukawa blocks) of A x.
constexpr int kProfKinds = 7;
constexpr int kProfM2PPair = 6;
// Targets per target group of the forward operator: the interaction lists
// are built per group (group MAC); a wavefront evaluates one group with four
// lanes per target, each lane taking a quarter of the group's sources or
// cells.  Smaller groups see more cells through their expansions (a tighter
// group sphere), so fewer source points go to P2P.
constexpr int kGroup = 16;
constexpr int kQuarters = 64 / kGroup;  // lanes per target
constexpr int kNearRun = 16;            // targets per near-field search wavefront
constexpr double kNearSplit = 4.0;       // a near-field run is walked in parts when its sphere exceeds this many reaches
// Gauss points per target group of the transposed operator (one lane each:
// with the Gauss points four to a panel, smaller groups cut few pairs)
constexpr int kAGroup = 64;
constexpr int kDotChunk = 4096;  // Krylov reduction chunk (entries of one system)
constexpr int kNearSlots = 128; // near-field columns per row kept by the single traversal
constexpr int kMaxLevels = 21;   // 63-bit Morton keys, 21 bits per axis
constexpr int kMaxNk = 32;
constexpr int kMomChunk = 128;   // sources staged at a time by the direct moment pass
constexpr int kMomSpan = 1024;   // sources per block of the transposed operator's moment pass
constexpr int kSpanSources = 256;  // largest cell whose moments one work-group forms from its sources
// non-leaf cells of at most this many sources form their moments with their
// subtree in one work-group; larger ones (and all cells above) by upward shifts
constexpr int kSpanCell = 256;
// a span cell of more sources than this (or the only cell of its span, when
// it has more than kMomSharedLone) is summed by all waves of the span's
// work-group; smaller cells by one wave each
constexpr int kMomShared = 64;
constexpr int kMomSharedLone = 16;
// sources (summed over cells) of one work-group of the span moment pass
constexpr int kMomJob = 128;

// Span roots shifted per work-group into one upper cell by the upward moment
// pass: as many as fit 48 KiB of LDS in the dense (P+1)^3 FP64 layout of
// both moment kinds (the same table serves both precisions).
__host__ __device__ constexpr int mom_up_batch(int P) {
  return 16 * 2 * (P + 1) * (P + 1) * (P + 1) * 8 <= 49152  ? 16
         : 8 * 2 * (P + 1) * (P + 1) * (P + 1) * 8 <= 49152 ? 8
         : 4 * 2 * (P + 1) * (P + 1) * (P + 1) * 8 <= 49152 ? 4
         : 2 * 2 * (P + 1) * (P + 1) * (P + 1) * 8 <= 49152 ? 2
                                                            : 1;
}
constexpr int kMaxRule = 19;

__host__ __device__ constexpr int ncoef(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

// Work tiles of P2P (sources per unit) and M2P (far cells per unit).  Left
// automatic (0), a tile is the largest of (512, 256, 128) sources or (32, 16,
// 8) cells whose units still fill every SIMD with waves for ~1.5 rounds
// (kUnitRounds x the waves the GPU holds at once), so that the launch's tail
// -- waves finishing at different times -- is short; `work(t)` returns the
// number of units a tile t gives.
constexpr double kUnitRounds = 1.5;
template <typename F>
int auto_tile(int fixed, const int (&choices)[3], double waves_resident, F work) {
  if (fixed > 0) return fixed;
  for (int t : choices)
    if (work(t) >= kUnitRounds * waves_resident) return t;
  return choices[2];
}
// values per (cell, kernel slot) of the transposed operator's moments:
// single layer to order P, the three double-layer gradient arrays to P + 1
__host__ __device__ constexpr int adj_mom_len(int p) { return ncoef(p) + 3 * ncoef(p + 1); }

// Kernel sets evaluated by one block: up to two distinct Green's functions.
enum KernelSet : int { KS_L = 0, KS_Y = 1, KS_LY = 2, KS_YY = 3, KS_COUNT = 4 };

// ---------------------------------------------------------------- host model
struct Region {
  double eps = 1.0, kappa = 0.0;
};

struct Surface {
  std::vector<double> v;    // nv x 3
  std::vector<int32_t> t;   // np x 3
  int inner = -1, outer = -1;
  int64_t nv() const { return (int64_t)v.size() / 3; }
  int64_t np() const { return (int64_t)t.size() / 3; }
};

struct ChargeSet {
  std::vector<double> xyz, q;
  int64_t n() const { return (int64_t)q.size(); }
};

}  // namespace pbtc

struct pbtc_problem {
  std::vector<pbtc::Region> regions;
  std::vector<pbtc::Surface> surfaces;
  std::vector<pbtc::ChargeSet> charges;  // one per region
};

namespace pbtc {

// A target set is either the collocation points of one surface or the
// charges of one region.
struct TargetSet {
  int kind = 0;  // 0 surface, 1 charges
  int id = 0;    // surface id or region id
  int64_t off = 0, n = 0;          // global target index range
  int64_t grp_off = 0, ngrp = 0;   // global target-group range
};

// Interaction of one target set with the Gauss points of one source surface,
// for one or two Green's functions.
struct Block {
  int t = 0, s = 0;
  int ks = KS_L;
  int nk = 1;
  double kappa[2] = {0.0, 0.0};
  int64_t out[2] = {0, 0};   // offsets of this block's S/D outputs per kernel
  bool reaction = false;     // targets are charges (evaluated after the solve)
  int64_t item_off = 0;      // first (block, group) item
  int64_t nf_row = 0;        // first near-field correction row
};

struct RowTerm {
  int block = 0, kidx = 0;
  double sigma_c = 0.0, sigma = 0.0;
};

// Rows of surface t seen from region r (or, for reaction rows, the charges
// of region r).
struct RowBlock {
  int t = 0, r = 0;
  int64_t row_off = 0, n = 0, phi_off = 0;
  std::vector<RowTerm> terms;
};

// --------------------------------------------------------- device structures
struct DevBlock {
  int t, s, ks, nk;
  double kappa0, kappa1;
  long long out0, out1;
  long long tgt_off, ntgt;   // global target range of the target set
  long long grp_off;         // first global group of the target set
  long long gp_off, gp_n;    // sorted Gauss-point segment of the source surface
  long long pan_off;         // first panel of the source surface
  long long item_off;        // first (block, group) item
  long long nf_row;          // first near-field row (one row per target)
  int root;                  // root cell of the source surface
  int self;                  // 1 if the target set is the source surface itself
  int tkind;                 // 0: surface collocation points, 1: charges
  int pad;
  // transposed evaluation: sources at the targets of t, targets at the
  // Gauss points of s
  long long aitem_off;       // first (block, Gauss-point group) item
  long long gpgrp_off;       // first Gauss-point group of surface s
  long long aout0, aout1;    // per-Gauss-point outputs of kernel slots 0 / 1
  long long csc_off;         // first transposed near-field column of this block
  int slot0;                 // kernel slot of kernel 0 (slot0 + 1 for kernel 1)
  int troot;                 // root cell of the target-set tree
  int lslot0;                // slot of kernel 0 among the slots of its target-set tree
  int direct_below;          // MAC-accepted cells with fewer sources go to P2P
};

// Weights of one (block, kernel) slot of the transposed operator:
// muS = sum_c cS[c] lam[lam_off[c] + i], muD likewise (at most two rows).
struct DevSlot {
  long long out;        // offset of mu in the S/D-shaped arrays (= block out[k])
  long long n;          // targets of the block's target set
  long long lam_off[2];
  double cS[2], cD[2];
  int ncontrib, block;
};

// Per surface: the slots (blocks x kernels) whose sources are its Gauss points.
struct DevGather {
  int slot_off, nslots;
};

struct DevRowBlock {
  long long row_off, n, phi_off;
  int term_off, nterms;
  double half;  // 1/2 for surface rows, 0 for reaction rows
  double sign;  // -1 for surface rows (1/2 phi - sum), +1 for reaction rows
};

struct DevRowTerm {
  long long out;       // offset into the S and D arrays
  double sigma_c, sigma;
};

// A forward row block as the Coulomb right-hand side and its transpose see
// it: rows [row_off, row_off + n) of surface panels pan_first.., the charges
// [q0, q0 + nq) of the row block's region, its 1/eps and kappa.
struct DevCoulRow {
  long long row_off, n, pan_first, q0, nq;
  double inv_eps, kappa;
  long long pad;
};

struct Cell {
  double cx, cy, cz;  // box centre (expansion centre y_c)
  double h;           // half edge of the box
  double rb;          // max distance from the centre to a source
  int begin, count;   // sorted Gauss-point range (global index)
  int child, nchild;  // first child cell, number of children (0: leaf)
  int level, surf;
};

// Workspace layout: byte offsets of every device array.
struct Layout {
  size_t total = 0;
  size_t add(size_t bytes) {
    size_t o = (total + 255) & ~size_t(255);
    total = o + bytes;
    return o;
  }
};

struct Timer;
struct BatchCache;  // merged plan of pbtc_solve_batch, kept by the batch's first plan

// A run of work units (one wavefront each) over the lists of one kernel set.
struct UnitSet {
  int64_t off = 0, n = 0;   // units [off, off + n) of the unit pool
  int64_t ptr_off = 0;      // per listed item: first unit (n_items + 1 entries)
};

}  // namespace pbtc

// Plan: everything the host knows about a problem plus the device layout.
struct pbtc_plan_s {
  pbtc_problem prob;
  pbtc_params prm;
  std::string err;

  // sizes
  int nsurf = 0, nreg = 0, P = 6, ncrit = 64, direct_below = 0;
  int64_t np_tot = 0, nv_tot = 0, ngp = 0, nq = 0, ntgt = 0, ngrp = 0, nunk = 0;
  std::vector<int64_t> pan_off, v_off, gp_off, unk_off, q_off_region;
  std::vector<pbtc::TargetSet> tsets;
  std::vector<int> tset_of_surface, tset_of_region;
  std::vector<pbtc::Block> blocks;
  std::vector<pbtc::RowBlock> rows, reac_rows;
  int64_t nout = 0;      // S/D values over all blocks and kernels
  int64_t nitems = 0;    // (block, group) pairs
  std::vector<double> cube;  // per surface: cx, cy, cz, half
  std::vector<double> max_len, max_reach;  // per surface: max L, max centroid-vertex distance
  double rule_b[3 * pbtc::kMaxRule], rule_w[pbtc::kMaxRule];
  double fine_b[3 * pbtc::kMaxRule], fine_w[pbtc::kMaxRule];
  double gl_x[pbtc::kMaxNk], gl_w[pbtc::kMaxNk];

  // capacities (grown after a failed set-up)
  int64_t cap_cells = 0, cap_near = 0, cap_far = 0, cap_nf = 0;

  // device offsets
  size_t o_verts, o_tris, o_pan_surf, o_qxyz, o_q, o_qreg;
  size_t o_cx, o_cy, o_cz, o_nx, o_ny, o_nz, o_area, o_len;      // panels, FP64
  size_t o_pidx;                                                 // per panel: phi, psi index (int2)
  size_t o_pinv = 0;   // per panel: inverse of the 2 x 2 diagonal block (row-major FP64)
  size_t o_ptab = 0;   // per surface: kappa_inner, kappa_outer, eps_inner / eps_outer
  size_t o_ptmp = 0;   // preconditioned Krylov vector (n FP64)
  size_t o_flags = 0;  // device status flags (16 int)
  size_t o_qtab = 0;   // per region: first charge (nreg + 1 long long), eps (nreg double)
  size_t o_coul = 0;   // Coulomb energy per system (ncomp double)
  // moment pass: span cells (cell, first source, count), spans (first span
  // cell, cells, first source, count) and their root cells, upward parts
  // (upper cell, first span, end span, sole part) and sums (upper cell,
  // first part, parts), the parts' partial moments
  size_t o_mchunks = 0, o_mcent = 0, o_mspans = 0, o_mproot = 0, o_mph = 0, o_mparts = 0,
         o_musum = 0, o_mpart = 0;
  int64_t n_mchunks = 0, n_mspans = 0, n_mparts = 0, n_musum = 0, cap_mparts = 0;
  // direct moment pass of the transposed operator: chunks (cell, first
  // source, count, slot) and (cell x local slot, first chunk, end chunk)
  // pairs, per phase in [off[ph], off[ph + 1])
  size_t o_amchunks = 0, o_ampairs = 0, o_ampart = 0;
  int64_t cap_amchunks = 0, cap_ampairs = 0;
  int64_t am_chunk_off[3] = {0, 0, 0}, am_pair_off[3] = {0, 0, 0};
  std::vector<double> ptab_host;  // host copy of the o_ptab table
  std::vector<double> qtab_host;  // host copy of the o_qtab table
  std::vector<long long> tset_off_host;  // first target of every target set, then ntgt
  // Coulomb row table: DevCoulRow per forward row block, then per region the
  // CSR (nreg + 1 int offsets, row block indices) of its row blocks
  size_t o_crows = 0;
  std::vector<char> crow_host;
  size_t o_tx, o_ty, o_tz, o_tidx;                               // sorted targets (FP64) + perm
  size_t o_txf, o_tyf, o_tzf;                                    // sorted targets FP32
  size_t o_grp;                                                  // group spheres (4 doubles)
  size_t o_gx, o_gy, o_gz, o_gw, o_gpid, o_gkey, o_gtmpk, o_gtmpv, o_gidx;  // Gauss points
  size_t o_src64, o_src32;                                       // source records per matvec
  size_t o_keys2, o_hist;                                        // sort scratch
  size_t o_cells, o_cnt, o_scan;                                 // tree
  size_t o_mom64, o_mom32;                                       // moments
  size_t o_near_ptr, o_far_ptr, o_near, o_far;                   // lists (CSR over items)
  size_t o_nf_ptr, o_nf_col, o_nf_v64, o_nf_v32;                 // near-field correction
  size_t o_S, o_D;                                               // block outputs (FP64)
  size_t o_blocks, o_rows, o_terms, o_reac_rows, o_reac_terms;   // descriptors
  size_t o_items;                                                // item -> block (int2)
  size_t o_b, o_x, o_r, o_w, o_tmp, o_V, o_H, o_givens, o_scal, o_red;  // Krylov
  size_t o_phi_reac, o_energy;
  size_t o_lam, o_adj_rhs;
  size_t fixed_bytes = 0;
  size_t ws_bytes = 0;

  // independent systems (connected components of the region graph, e.g. the
  // molecules of a batch): unknown range, charge range, Krylov chunks
  int ncomp = 1;
  std::vector<int> comp_of_surface, comp_of_region;
  std::vector<int64_t> comp_u0, comp_u1;       // unknown range per component
  std::vector<int4> dot_chunks;                 // (component, start, end, -)
  std::vector<int> comp_chunk0;                 // first chunk per component (+ end)
  std::vector<double> comp_energy;
  std::vector<int> comp_iters;
  std::vector<double> comp_rel;
  size_t o_comp_of_unk = 0, o_chunks = 0, o_comp_q = 0, o_kstate = 0;
  // device state
  void* ws = nullptr;
  void* inputs_ws = nullptr;  // workspace that already holds the uploaded inputs
  // profiling (params.profile): events around P2P (kind 0) and M2P (kind 1)
  struct ProfEvent {
    int kind = 0;
    double flop = 0.0;
    hipEvent_t a = nullptr, b = nullptr;
    bool recorded = false;  // both events recorded on the stream
  };
  std::vector<ProfEvent> prof, prof_pool;
  // per kernel kind: 0 P2P, 1 Laplace M2P, 2 Yukawa M2P of A x; 3, 4, 5 the
  // same of A^T x
  double prof_t[pbtc::kProfKinds] = {}, prof_flop[pbtc::kProfKinds] = {};
  int prof_n[pbtc::kProfKinds] = {};
  int64_t prof_count = 0;   // FP32 operator evaluations seen by the sampler
  int64_t aprof_count = 0;  // the same for the transposed operator
  double setup_phase[6] = {0, 0, 0, 0, 0, 0};  // host seconds per set-up phase
  // GMRES residual readback: pinned host slots and their events
  double* res_pin = nullptr;
  int res_pin_n = 0;
  hipEvent_t res_ev[2] = {nullptr, nullptr};
  // second stream of the operator (the moment pass runs beside P2P) and the
  // events that fork and join it (created on first use)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // launch graphs of the operator per [precision FP64 / FP32][phase]: the
  // kernel sequence captured on cap_stream with x and y in o_gxin / o_gyout,
  // valid for the set-up generation and workspace it was captured on
  hipStream_t cap_stream = nullptr;
  hipGraph_t op_graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipGraphExec_t op_exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  uint64_t op_graph_gen[2][2] = {{0, 0}, {0, 0}};
  void* op_graph_ws[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  // set-up generation of the last evaluation launched kernel by kernel
  // because its graph was stale (the next one captures)
  uint64_t op_direct_gen[2][2] = {{0, 0}, {0, 0}};
  int op_kernels[2][2] = {{0, 0}, {0, 0}};  // kernel nodes per graph
  uint64_t setup_gen = 0;                   // bumped by every device set-up
  int64_t n_graph_launch = 0;               // graph replays of the FP32 A x
  size_t o_gxin = 0, o_gyout = 0;
  ~pbtc_plan_s();
  std::vector<double> item_flop_p2p[2][pbtc::KS_COUNT], item_flop_m2p[2][pbtc::KS_COUNT];
  double launch_flop_p2p[2][pbtc::KS_COUNT] = {}, launch_flop_m2p[2][pbtc::KS_COUNT] = {};
  double alaunch_flop_p2p[2][pbtc::KS_COUNT] = {}, alaunch_flop_m2p[2][pbtc::KS_COUNT] = {};
  bool setup_done = false;
  int n_levels = 0;
  std::vector<int> level_begin;  // cell index where each level starts (+ end)
  int64_t n_cells = 0, n_near = 0, n_far = 0, n_nf = 0;
  // item ids grouped by kernel set, for forward (0) and reaction (1) blocks
  std::vector<int> item_list[2][pbtc::KS_COUNT];
  size_t o_item_list[2][pbtc::KS_COUNT];
  std::vector<int> item_block;    // item -> block
  std::vector<double> tcube;      // per target set: cx, cy, cz, half
  int64_t nf_rows = 0, nf_fwd_rows = 0;
  // transposed operator (pbtc_backward, pbtc_matvec_transpose)
  bool adj_done = false;
  int64_t ngpgrp = 0, nitems_adj = 0, naout = 0, ncsc = 0, n_tcells = 0;
  int64_t cap_tcells = 0, cap_anear = 0, cap_afar = 0, n_anear = 0, n_afar = 0;
  std::vector<int64_t> gpgrp_off;   // per surface
  std::vector<int> aitem_block;
  std::vector<int> aitem_list[2][pbtc::KS_COUNT];
  size_t o_aitem_list[2][pbtc::KS_COUNT];
  std::vector<pbtc::DevSlot> slots[2];   // phase 0: rows of A, phase 1: reaction rows
  std::vector<int> gather_slots[2];      // per phase, slots grouped by surface
  std::vector<pbtc::DevGather> gathers[2];
  std::vector<int> tlevel_begin;
  int n_tlevels = 0;
  std::vector<int64_t> blk_slot0, blk_aout0, blk_aout1, blk_aitem_off, blk_csc_off;
  std::vector<int> blk_lslot0;  // local slot of kernel 0 in its target-set tree
  int adj_ms = 1;               // largest number of slots on one target-set tree
  size_t o_tkey_sorted = 0, o_gpos32 = 0, o_gpos64 = 0, o_gp_pos = 0, o_gpgrp = 0;
  size_t o_mu_s = 0, o_mu_d = 0, o_asrc32 = 0, o_asrc64 = 0, o_aout_s = 0, o_aout_d = 0;
  size_t o_aitems = 0, o_slots[2] = {0, 0}, o_gather[2] = {0, 0}, o_gather_slots[2] = {0, 0};
  size_t o_csc_ptr = 0, o_csc_ent = 0, o_csc_fill = 0;
  size_t o_tcells = 0, o_tcnt = 0, o_amom32 = 0, o_amom64 = 0;
  size_t o_anear_ptr = 0, o_afar_ptr = 0, o_anear = 0, o_afar = 0;
  size_t o_z2 = 0, o_dots = 0, o_surf_tab = 0;
  // wavefront work units: [phase][kernel set][0 = P2P, 1 = M2P]
  pbtc::UnitSet units[2][pbtc::KS_COUNT][2];
  int64_t cap_units = 0, n_units = 0, n_uptr = 0;
  int tile_sources = 512, tile_cells = 32;  // work tiles of the last set-up
  size_t o_units = 0, o_uptr = 0, o_partial = 0;
  // transposed operator: units, slot and block tables
  pbtc::UnitSet aunits[2][pbtc::KS_COUNT][2];
  int64_t cap_aunits = 0, cap_auptr = 0;
  size_t o_aunits = 0, o_auptr = 0, o_slot_block = 0, o_slot_kidx = 0, o_adj_tab = 0;
  size_t o_adj_blist[2] = {0, 0}, o_adj_sids[2] = {0, 0}, o_csc_row = 0;
  size_t o_adj_tslot[2] = {0, 0};  // per phase: [target-set tree][local slot] -> slot or -1
  std::vector<int> adj_tslot_host[2];
  std::vector<int> adj_blist[2], adj_sids[2];
  std::vector<double> adj_history;
  size_t o_nf_rowblk = 0;                          // near-field row -> block (int)
  size_t o_grp_tab = 0;                            // group target offsets and counts
  size_t o_tkey = 0, o_tkey2 = 0, o_tval = 0, o_tval2 = 0;  // target sort buffers
  double p2p_pairs = 0, m2p_evals = 0, dense_equiv = 0;
  bool solved = false;        // host results (x_host, phi_reac_host, energy) are current
  bool dev_solved = false;    // the plan's own workspace holds the solution of its charges
  bool charges_dirty = false;
  uint64_t serial = 0;        // unique per plan (batch cache identity)
  uint64_t charge_version = 0;  // bumped by pbtc_set_charge_values
  std::vector<int> comp_conv;   // per system: converged in the last solve
  pbtc::BatchCache* batch = nullptr;  // owned; see abi.cpp
  // host table of the allocation-free Coulomb energy (region offsets, eps,
  // per-system sums), sized when the plan is made
  std::vector<double> coul_host;

  // host results
  std::vector<double> x_host, phi_reac_host, history;
  double energy = 0.0;
};
