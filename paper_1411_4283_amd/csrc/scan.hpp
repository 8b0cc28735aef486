// Segmented exclusive prefix sum (one segment per geometry) in three passes:
// tile sums, a scan of the tile sums per segment, and the tile-local scan plus offset.
#pragma once

#include "common.hpp"

namespace cutcell {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

inline long long scan_tiles(long long len) { return (len + kScanTile - 1) / kScanTile; }

template <typename T>
__device__ __forceinline__ T block_exclusive(T v, T* sh, T& total) {
  // inclusive scan of one value per thread across the block (Hillis-Steele in LDS)
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    T add = (t >= off) ? sh[t - off] : T(0);
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  total = sh[kScanThreads - 1];
  T incl = sh[t];
  __syncthreads();
  return incl - v;
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const Tin* __restrict__ in, long long len,
                                                              long long seg_stride, Tout* __restrict__ tile_sums,
                                                              long long ntiles) {
  __shared__ Tout sh[kScanThreads];
  const long long seg = blockIdx.y;
  const long long tile = blockIdx.x;
  const Tin* src = in + seg * seg_stride;
  long long base = tile * kScanTile + (long long)threadIdx.x * kScanItems;
  Tout s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < len) s += (Tout)src[base + i];
  Tout total;
  block_exclusive<Tout>(s, sh, total);
  if (threadIdx.x == 0) tile_sums[seg * ntiles + tile] = total;
}

template <typename Tout>
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(Tout* __restrict__ tile_sums, long long ntiles,
                                                             Tout* __restrict__ seg_totals) {
  __shared__ Tout sh[kScanThreads];
  const long long seg = blockIdx.x;
  Tout* s = tile_sums + seg * ntiles;
  Tout carry = 0;
  for (long long b = 0; b < ntiles; b += kScanThreads) {
    long long i = b + threadIdx.x;
    Tout v = (i < ntiles) ? s[i] : Tout(0);
    Tout total;
    Tout ex = block_exclusive<Tout>(v, sh, total);
    if (i < ntiles) s[i] = ex + carry;
    carry += total;
  }
  if (threadIdx.x == 0 && seg_totals) seg_totals[seg] = carry;
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const Tin* __restrict__ in, long long len,
                                                              long long seg_stride, const Tout* __restrict__ tile_sums,
                                                              long long ntiles, Tout* __restrict__ out,
                                                              long long out_stride) {
  __shared__ Tout sh[kScanThreads];
  const long long seg = blockIdx.y;
  const long long tile = blockIdx.x;
  const Tin* src = in + seg * seg_stride;
  Tout* dst = out + seg * out_stride;
  long long base = tile * kScanTile + (long long)threadIdx.x * kScanItems;
  Tout v[kScanItems];
  Tout s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < len) ? (Tout)src[base + i] : Tout(0);
    s += v[i];
  }
  Tout total;
  Tout run = block_exclusive<Tout>(s, sh, total) + tile_sums[seg * ntiles + tile];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < len) dst[base + i] = run;
    run += v[i];
  }
}

// out[seg][i] = sum_{k<i} in[seg][k]; seg_totals[seg] = sum of segment (may be null).
// tmp must hold nseg * scan_tiles(len) elements of Tout.
template <typename Tin, typename Tout>
int exclusive_scan(const Tin* in, long long len, long long in_stride, int nseg, Tout* out, long long out_stride,
                   Tout* seg_totals, Tout* tmp, hipStream_t st) {
  if (len <= 0) return CUTCELL_OK;
  long long nt = scan_tiles(len);
  dim3 grid((unsigned)nt, (unsigned)nseg);
  hipLaunchKernelGGL((k_scan_tiles<Tin, Tout>), grid, dim3(kScanThreads), 0, st, in, len, in_stride, tmp, nt);
  hipLaunchKernelGGL((k_scan_sums<Tout>), dim3(nseg), dim3(kScanThreads), 0, st, tmp, nt, seg_totals);
  hipLaunchKernelGGL((k_scan_apply<Tin, Tout>), grid, dim3(kScanThreads), 0, st, in, len, in_stride, tmp, nt, out,
                     out_stride);
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

}  // namespace cutcell
