// Small device utilities shared by the kernels of libpbtc.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace pbtc {

template <typename T>
inline T* wsp(const pbtc_plan_t& pl, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(pl.ws) + off);
}

inline int nblocks(int64_t n, int per) { return (int)((n + per - 1) / per); }

// Exclusive prefix sum in place over data[0..n); data[n] receives the total.
// `scratch` must hold nblocks(n, 4096) + 1 values.
template <typename T>
void scan_exclusive(T* data, int64_t n, T* scratch, hipStream_t st);

// Stable LSD radix sort of 64-bit keys with 32-bit values (8 passes of 8
// bits); tmp buffers of the same length; hist holds 256 * (n / 256 + 1) ints.
void radix_sort64(uint64_t* keys, int* vals, uint64_t* tmpk, int* tmpv, int* hist, int64_t n,
                  hipStream_t st);

// The same sort of several segments at once: vals[i] must hold the element's
// position i before sorting, and seg_off (device, nseg + 1 ascending offsets
// covering [0, n)) delimits the segments; each segment ends up sorted in
// place, exactly as a separate stable sort of it would leave it.  Extra passes
// over the segment index follow the 8 key passes.
void radix_sort64_seg(uint64_t* keys, int* vals, uint64_t* tmpk, int* tmpv, int* hist, int64_t n,
                      const long long* seg_off, int nseg, hipStream_t st);

#define PBTC_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      pl.err = std::string("HIP error: ") + hipGetErrorString(e_) + " at " +  \
               __FILE__ + ":" + std::to_string(__LINE__);                     \
      return PBTC_EDEVICE;                                                    \
    }                                                                         \
  } while (0)

#define PBTC_LAUNCH_CHECK() PBTC_HIP(hipGetLastError())

}  // namespace pbtc
