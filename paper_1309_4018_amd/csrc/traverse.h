// Tree traversals of the treecode set-up by one wavefront per target group.
//
// Interaction lists (sec. 2.3, MAC of Eq. MAC with the group's bounding
// sphere): starting at the root, a cell that the group sees under the MAC is
// a far cell (M2P), or a near cell when it holds fewer than direct_below
// sources; a leaf that fails the MAC is a near cell (P2P); any other cell is
// opened.  The wave keeps a stack of opened cells in LDS; each step pops up to
// 8 of them and its 64 lanes test their children (8 per cell) at once, so a
// traversal costs one dependent round trip per step instead of one per cell.
// The emission order is fixed by the lane order (deterministic).
#pragma once

#include "kernel_common.h"

namespace pbtc {

constexpr int kTravWaves = 4;         // wavefronts per work-group
constexpr int kTravStack = 2048;      // opened cells per wave (LDS)

__device__ __forceinline__ uint64_t lanes_below(int lane) { return (1ull << lane) - 1ull; }

// Outcome of one traversal step for the lane's cell.
enum { TV_NONE = 0, TV_NEAR, TV_FAR, TV_OPEN };

// Lists of one item.  mode 0: counts only; mode 1: also writes near[pn + i]
// and far[pf + i] below the capacities.  stack: this wave's LDS slice.  Sets
// *overflow when the stack would overflow (the lists are then incomplete).
// Every lane returns the same counts.
__device__ inline void wave_lists(const Cell* __restrict__ cells, int root, double gx, double gy,
                                  double gz, double gr, double theta, int direct_below, int mode,
                                  long long pn, long long pf, int* __restrict__ near,
                                  int* __restrict__ far, long long cap_near, long long cap_far,
                                  int* stack, long long* nn_out, long long* nf_out,
                                  int* overflow) {
  const int lane = threadIdx.x & 63;
  long long nn = 0, nf = 0;
  int sp = 0;
  // the root is tested by lane 0 alone; afterwards children of opened cells
  bool first = true;
  while (first || sp > 0) {
    int c = -1;
    int np = 0;
    if (first) {
      c = lane == 0 ? root : -1;
    } else {
      np = min(sp, 8);
      if (sp - np + 8 * np > kTravStack) np = (kTravStack - sp) / 7;
      if (np <= 0) {
        if (lane == 0) *overflow = 1;
        break;
      }
      sp -= np;
      const int pi = lane >> 3, k = lane & 7;
      if (pi < np) {
        const int par = stack[sp + pi];
        const Cell& pc = cells[par];
        if (k < pc.nchild) c = pc.child + k;
      }
      wave_sync();  // the popped slots are read before they are reused
    }
    first = false;
    int kind = TV_NONE;
    if (c >= 0) {
      const Cell cl = cells[c];
      if (cl.count > 0) {
        const double dx = gx - cl.cx, dy = gy - cl.cy, dz = gz - cl.cz;
        const double rtb = sqrt(dx * dx + dy * dy + dz * dz) - gr;
        if (theta * rtb > cl.rb)
          kind = cl.count < direct_below ? TV_NEAR : TV_FAR;
        else
          kind = cl.nchild == 0 ? TV_NEAR : TV_OPEN;
      }
    }
    const uint64_t below = lanes_below(lane);
    const uint64_t mn = __ballot(kind == TV_NEAR);
    const uint64_t mf = __ballot(kind == TV_FAR);
    const uint64_t mo = __ballot(kind == TV_OPEN);
    if (mode == 1) {
      if (kind == TV_NEAR) {
        const long long at = nn + __popcll(mn & below);
        if (pn + at < cap_near) near[pn + at] = c;
      } else if (kind == TV_FAR) {
        const long long at = nf + __popcll(mf & below);
        if (pf + at < cap_far) far[pf + at] = c;
      }
    }
    if (kind == TV_OPEN) stack[sp + __popcll(mo & below)] = c;
    nn += __popcll(mn);
    nf += __popcll(mf);
    sp += __popcll(mo);
    wave_sync();
  }
  *nn_out = nn;
  *nf_out = nf;
}

// Leaves of the tree under `root` that may hold a source within `reach` of
// some point of the sphere (gx, gy, gz, gr): a cell is skipped when
// |centre - g| - r_b - gr > reach.  leaf(c, centre x, y, z, r_b) is called by
// the whole wave, in a fixed order, with wave-uniform arguments.
template <typename F>
__device__ inline void wave_leaves_within(const Cell* __restrict__ cells, int root, double gx,
                                          double gy, double gz, double gr, double reach,
                                          int* stack, int* overflow, F&& leaf) {
  const int lane = threadIdx.x & 63;
  int sp = 0;
  bool first = true;
  while (first || sp > 0) {
    int c = -1;
    if (first) {
      c = lane == 0 ? root : -1;
    } else {
      int np = min(sp, 8);
      if (sp - np + 8 * np > kTravStack) np = (kTravStack - sp) / 7;
      if (np <= 0) {
        if (lane == 0) *overflow = 1;
        break;
      }
      sp -= np;
      const int pi = lane >> 3, k = lane & 7;
      if (pi < np) {
        const int par = stack[sp + pi];
        const Cell& pc = cells[par];
        if (k < pc.nchild) c = pc.child + k;
      }
      wave_sync();
    }
    first = false;
    int kind = TV_NONE;
    double ccx = 0.0, ccy = 0.0, ccz = 0.0, crb = 0.0;
    if (c >= 0) {
      const Cell cl = cells[c];
      ccx = cl.cx;
      ccy = cl.cy;
      ccz = cl.cz;
      crb = cl.rb;
      if (cl.count > 0) {
        const double dx = gx - cl.cx, dy = gy - cl.cy, dz = gz - cl.cz;
        if (sqrt(dx * dx + dy * dy + dz * dz) - cl.rb - gr <= reach)
          kind = cl.nchild == 0 ? TV_NEAR : TV_OPEN;
      }
    }
    const uint64_t below = lanes_below(lane);
    const uint64_t mo = __ballot(kind == TV_OPEN);
    if (kind == TV_OPEN) stack[sp + __popcll(mo & below)] = c;
    sp += __popcll(mo);
    wave_sync();
    uint64_t ml = __ballot(kind == TV_NEAR);
    while (ml) {
      const int l = __ffsll((unsigned long long)ml) - 1;
      ml &= ml - 1;
      leaf(__builtin_amdgcn_readfirstlane(__shfl(c, l, 64)), __shfl(ccx, l, 64),
           __shfl(ccy, l, 64), __shfl(ccz, l, 64), __shfl(crb, l, 64));
    }
  }
}

}  // namespace pbtc
