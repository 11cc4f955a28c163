// Device primitives used by the one-off set-up: prefix sums and a stable
// radix sort of Morton keys.
#include "device_util.h"

namespace pbtc {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanThreads * kScanPer;

// Block-wide inclusive scan of one value per thread (1024 threads, wave64).
template <typename T>
__device__ T block_inclusive(T v, T* lds_warp) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  if (lane == 63) lds_warp[wid] = v;
  __syncthreads();
  if (wid == 0) {
    T w = lane < (kScanThreads / 64) ? lds_warp[lane] : T(0);
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      T u = __shfl_up(w, o, 64);
      if (lane >= o) w += u;
    }
    if (lane < (kScanThreads / 64)) lds_warp[lane] = w;
  }
  __syncthreads();
  if (wid > 0) v += lds_warp[wid - 1];
  return v;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const T* __restrict__ d, int64_t n,
                                                            T* __restrict__ sums) {
  __shared__ T w[16];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int64_t i = base + (int64_t)threadIdx.x * kScanPer + k;
    if (i < n) s += d[i];
  }
  s = block_inclusive(s, w);
  if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = s;
}

// Single block: exclusive scan of the tile sums, total into sums[nt].
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(T* __restrict__ sums, int64_t nt) {
  __shared__ T w[16];
  __shared__ T carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t b = 0; b < nt; b += kScanThreads) {
    const int64_t i = b + threadIdx.x;
    const T v = i < nt ? sums[i] : T(0);
    const T inc = block_inclusive(v, w);
    const T c = carry;
    if (i < nt) sums[i] = c + inc - v;
    __syncthreads();
    if (threadIdx.x == kScanThreads - 1) carry = c + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[nt] = carry;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(T* __restrict__ d, int64_t n,
                                                            const T* __restrict__ sums) {
  __shared__ T w[16];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  T v[kScanPer];
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = base + k < n ? d[base + k] : T(0);
    s += v[k];
  }
  const T inc = block_inclusive(s, w);
  T run = sums[blockIdx.x] + inc - s;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) d[base + k] = run;
    run += v[k];
  }
}

template <typename T>
__global__ void k_put_total(T* d, int64_t n, const T* sums, int64_t nt) {
  d[n] = sums[nt];
}

// ---------------------------------------------------------------- radix sort
constexpr int kSortThreads = 256;  // one element per thread per tile

// Digit of one element for the pass at bit `shift`: a byte of the key for
// shift < 64, above that a byte of the element's segment (the largest s with
// seg_off[s] <= val; the value is the element's position before sorting).
__device__ __forceinline__ int sort_digit(uint64_t key, int val, int shift,
                                          const long long* __restrict__ seg_off, int nseg) {
  if (shift < 64) return (int)((key >> shift) & 255);
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg_off[mid] <= val) lo = mid;
    else hi = mid - 1;
  }
  return (lo >> (shift - 64)) & 255;
}

__global__ __launch_bounds__(kSortThreads) void k_digit_hist(const uint64_t* __restrict__ keys,
                                                             const int* __restrict__ vals,
                                                             int64_t n, int shift, int ntiles,
                                                             const long long* __restrict__ seg_off,
                                                             int nseg, int* __restrict__ hist) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
  if (i < n) atomicAdd(&h[sort_digit(keys[i], shift < 64 ? 0 : vals[i], shift, seg_off, nseg)], 1);
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: rank of each element among equal digits of its tile, in
// tile order, from wave ballots (8 bits matched bit by bit) and per-wave
// digit counts.
__global__ __launch_bounds__(kSortThreads) void k_digit_scatter(
    const uint64_t* __restrict__ keys, const int* __restrict__ vals, int64_t n, int shift,
    int ntiles, const long long* __restrict__ seg_off, int nseg, const int* __restrict__ offs,
    uint64_t* __restrict__ okeys, int* __restrict__ ovals) {
  __shared__ int wave_cnt[kSortThreads / 64][256];
  for (int k = threadIdx.x; k < (kSortThreads / 64) * 256; k += kSortThreads)
    (&wave_cnt[0][0])[k] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
  const bool valid = i < n;
  const uint64_t key = valid ? keys[i] : 0;
  const int val = valid ? vals[i] : 0;
  const int digit = valid ? sort_digit(key, val, shift, seg_off, nseg) : 0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (digit >> b) & 1;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  const uint64_t below = peers & ((1ull << lane) - 1ull);
  const int rank = __popcll(below);
  if (valid && below == 0) wave_cnt[wid][digit] = __popcll(peers);
  __syncthreads();
  if (!valid) return;
  int before = 0;
  for (int w = 0; w < wid; ++w) before += wave_cnt[w][digit];
  const int dst = offs[(int64_t)digit * ntiles + blockIdx.x] + before + rank;
  okeys[dst] = key;
  ovals[dst] = val;
}

}  // namespace

template <typename T>
void scan_exclusive(T* data, int64_t n, T* scratch, hipStream_t st) {
  const int nt = nblocks(n, kScanTile);
  if (n <= 0) {
    hipLaunchKernelGGL(k_scan_sums<T>, dim3(1), dim3(kScanThreads), 0, st, scratch, (int64_t)0);
    hipLaunchKernelGGL(k_put_total<T>, dim3(1), dim3(1), 0, st, data, (int64_t)0, scratch,
                       (int64_t)0);
    return;
  }
  hipLaunchKernelGGL(k_tile_sums<T>, dim3(nt), dim3(kScanThreads), 0, st, data, n, scratch);
  hipLaunchKernelGGL(k_scan_sums<T>, dim3(1), dim3(kScanThreads), 0, st, scratch, (int64_t)nt);
  hipLaunchKernelGGL(k_tile_scan<T>, dim3(nt), dim3(kScanThreads), 0, st, data, n, scratch);
  hipLaunchKernelGGL(k_put_total<T>, dim3(1), dim3(1), 0, st, data, n, scratch, (int64_t)nt);
}

template void scan_exclusive<int>(int*, int64_t, int*, hipStream_t);
template void scan_exclusive<long long>(long long*, int64_t, long long*, hipStream_t);

void radix_sort64_seg(uint64_t* keys, int* vals, uint64_t* tmpk, int* tmpv, int* hist, int64_t n,
                      const long long* seg_off, int nseg, hipStream_t st) {
  if (n <= 1) return;
  int seg_bits = 0;
  while (nseg > 1 && (1ll << seg_bits) < nseg) ++seg_bits;
  const int passes = 8 + (seg_bits + 7) / 8;
  const int ntiles = nblocks(n, kSortThreads);
  const int64_t nh = 256ll * ntiles;
  int* scratch = hist + nh + 1;
  uint64_t* src_k = keys;
  int* src_v = vals;
  uint64_t* dst_k = tmpk;
  int* dst_v = tmpv;
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(k_digit_hist, dim3(ntiles), dim3(kSortThreads), 0, st, src_k, src_v, n,
                       shift, ntiles, seg_off, nseg, hist);
    scan_exclusive<int>(hist, nh, scratch, st);
    hipLaunchKernelGGL(k_digit_scatter, dim3(ntiles), dim3(kSortThreads), 0, st, src_k, src_v, n,
                       shift, ntiles, seg_off, nseg, hist, dst_k, dst_v);
    std::swap(src_k, dst_k);
    std::swap(src_v, dst_v);
  }
  if (src_k != keys) {
    (void)hipMemcpyAsync(keys, src_k, 8 * n, hipMemcpyDeviceToDevice, st);
    (void)hipMemcpyAsync(vals, src_v, 4 * n, hipMemcpyDeviceToDevice, st);
  }
}

void radix_sort64(uint64_t* keys, int* vals, uint64_t* tmpk, int* tmpv, int* hist, int64_t n,
                  hipStream_t st) {
  radix_sort64_seg(keys, vals, tmpk, tmpv, hist, n, nullptr, 1, st);
}

}  // namespace pbtc
