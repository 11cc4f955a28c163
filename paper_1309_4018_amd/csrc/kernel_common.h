// Shared device helpers of the operator kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace pbtc {

// Arguments of the work-unit kernels (P2P and M2P, forward and transposed):
// units (item, first list entry, end entry, -), the item -> block map, the
// blocks, the cell list of this kernel kind and the cells.
struct UnitArgs {
  const int4* units;
  int nunits;
  const int* item_block;
  const DevBlock* blocks;
  const int* cells_list;
  const Cell* cells;
};

// One source record of the treecode: position, single-layer strength and
// double-layer dipole (forward operator), or position and the adjoint
// weights of up to two kernels (transposed operator).
template <typename real>
struct alignas(16) Src {
  real x, y, z, q, px, py, pz, pad;
};

template <typename real>
__device__ __forceinline__ real rsqrt_(real v);
template <>
__device__ __forceinline__ float rsqrt_(float v) {
  return __builtin_amdgcn_rsqf(v);
}
// FP64 (v > 0, finite): the hardware estimate refined by two Newton steps for
// 1/sqrt(v), y <- y + y (1 - v y^2) / 2, each of which doubles the number of
// correct bits; the result lies within two units in the last place.
template <>
__device__ __forceinline__ double rsqrt_(double v) {
  double y = __builtin_amdgcn_rsq(v);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double e = fma(-v * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// exp(-v): FP32 through the hardware exp2, FP64 through the math library
template <typename real>
__device__ __forceinline__ real exp_neg(real v);
template <>
__device__ __forceinline__ float exp_neg(float v) {
  return __builtin_amdgcn_exp2f(-1.4426950408889634f * v);
}
template <>
__device__ __forceinline__ double exp_neg(double v) {
  return exp(-v);
}

// exp(a * r) with a = exp_arg(kappa) = -kappa (FP64) or -kappa log2(e) (FP32,
// hardware exp2): one multiply per evaluation
template <typename real>
__host__ __device__ __forceinline__ real exp_arg(real kappa);
template <>
__host__ __device__ __forceinline__ float exp_arg(float kappa) {
  return -1.4426950408889634f * kappa;
}
template <>
__host__ __device__ __forceinline__ double exp_arg(double kappa) {
  return -kappa;
}
template <typename real>
__device__ __forceinline__ real exp_scaled(real a_times_r);
template <>
__device__ __forceinline__ float exp_scaled(float v) {
  return __builtin_amdgcn_exp2f(v);
}
template <>
__device__ __forceinline__ double exp_scaled(double v) {
  return exp(v);
}

// XCD-aware work-group order.  The dispatcher deals work-group b of a launch
// to XCD b % 8, and each XCD has its own L2; consecutive work units (Morton-
// ordered target groups) touch nearby sources, so each XCD is given one
// contiguous run of logical blocks instead of every eighth one.  A bijection
// of [0, nb).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / kXcds, r = nb % kXcds;
  const int x = b % kXcds, i = b / kXcds;
  return x * q + min(x, r) + i;
}

// Orders LDS accesses of the lanes of one wavefront (no work-group barrier):
// writes before the call are visible to every lane of the wave after it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace pbtc
