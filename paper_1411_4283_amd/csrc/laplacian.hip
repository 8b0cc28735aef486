// The operator as one sparse matrix over volumes (Sec. 2.2, eq. 'laplacian over V'):
//   L_v = vol_scale[v] * sum over v's faces f of sigma_vf s_f^T Phi = sum_k lap_v[k] Phi[k],
// lap_v the sigma-signed, volume-scaled merge of the stencil rows of v's <= 2D+1 faces.
// The apply is then one CSR gather per volume: for a regular 3D volume at path radius 3
// about 129 entries instead of the ~264 face entries it shares, and no flux array.
//
// One wave per volume merges the face rows (each sorted by column, columns distinct): an
// entry's position in the merged list is its index in its own row plus, for every other
// row, the number of that row's entries ordered before it (binary search; equal columns
// ordered by row).  Runs of equal columns are summed in that order and scaled by
// vol_scale.  A count pass and a fill pass run the same code; the result does not depend
// on the launch (no atomics).
#include <algorithm>

#include "gather.hpp"
#include "scan.hpp"
#include "solve.hpp"

namespace cutcell {

constexpr int kLapPad = 1024;   // >= (2D+1) rows of <= kMaxRows entries

template <int D, bool FILL>
__global__ __launch_bounds__(64) void k_lap_rows(long long n_vol, const int32_t* __restrict__ vol_face,
                                                 const double* __restrict__ vol_scale,
                                                 const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                 const double* __restrict__ val, int32_t* __restrict__ count,
                                                 const int64_t* __restrict__ lap_ptr, int32_t* __restrict__ lap_col,
                                                 double* __restrict__ lap_val, int32_t* too_long) {
  constexpr int S = 2 * D + 1;
  static_assert(S * kMaxRows <= kLapPad, "merge buffer too small");
  __shared__ int32_t ukey[kLapPad];
  __shared__ double uval[kLapPad];
  __shared__ int32_t skey[kLapPad];
  __shared__ double sval[kLapPad];
  const long long v = blockIdx.x;
  if (v >= n_vol) return;
  const int lane = threadIdx.x;
  int64_t start[S];
  int len[S], off[S];
  double sg[S];
  int tot = 0;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const int32_t f = vol_face[v * S + k];
    start[k] = 0;
    len[k] = 0;
    if (f >= 0) {
      start[k] = row_ptr[f];
      len[k] = (int)(row_ptr[f + 1] - start[k]);
    }
    sg[k] = (k < 2 * D && (k & 1) == 0) ? -1.0 : 1.0;   // low faces point into v
    off[k] = tot;
    tot += len[k];
  }
  if (tot > kLapPad) {   // rows not from a build (a build has at most kMaxRows per face)
    if (lane == 0) {
      if (!FILL) count[v] = 0;
      if (too_long) atomicOr(too_long, 1);
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < S; ++k)
    for (int i = lane; i < len[k]; i += 64) {
      ukey[off[k] + i] = col[start[k] + i];
      uval[off[k] + i] = sg[k] * val[start[k] + i];
    }
  __syncthreads();
  for (int idx = lane; idx < tot; idx += 64) {
    int own = 0;
#pragma unroll
    for (int k = 1; k < S; ++k)
      if (idx >= off[k]) own = k;
    const int32_t key = ukey[idx];
    int rank = idx - off[own];
#pragma unroll
    for (int l = 0; l < S; ++l) {
      if (l == own) continue;
      // entries of row l before key: columns < key, and == key from rows before `own`
      int lo = 0, hi = len[l];
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int32_t c = ukey[off[l] + mid];
        if (c < key || (l < own && c == key)) lo = mid + 1;
        else hi = mid;
      }
      rank += lo;
    }
    skey[rank] = key;
    sval[rank] = uval[idx];
  }
  __syncthreads();
  // each lane takes a contiguous chunk; a run starts where the column changes
  const int chunk = (tot + 63) / 64;
  const int b = min(lane * chunk, tot), e = min(b + chunk, tot);
  int heads = 0;
  for (int i = b; i < e; ++i) heads += (i == 0 || skey[i] != skey[i - 1]);
  int incl = heads;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if constexpr (!FILL) {
    if (lane == 63) count[v] = incl;
    return;
  } else {
    int64_t pos = lap_ptr[v] + (incl - heads);
    const double sc = vol_scale[v];
    for (int i = b; i < e; ++i) {
      if (i > 0 && skey[i] == skey[i - 1]) continue;
      double s = 0.0;
      for (int j = i; j < tot && skey[j] == skey[i]; ++j) s += sval[j];
      lap_col[pos] = skey[i];
      lap_val[pos] = sc * s;
      ++pos;
    }
  }
}

size_t laplacian_temp_bytes(long long n_vol) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const long long n = std::max<long long>(n_vol, 1);
  return al(sizeof(int32_t) * n) + al(sizeof(int64_t) * (scan_tiles(n) + 1)) + al(sizeof(int32_t));
}

int laplacian_count(int D, long long n_vol, const int64_t* row_ptr, const int32_t* col, const double* val,
                    const int32_t* vol_face, const double* vol_scale, int64_t* lap_ptr, int64_t* nnz, char* ws,
                    size_t ws_bytes, hipStream_t st) {
  if (ws_bytes < laplacian_temp_bytes(n_vol)) return fail(CUTCELL_E_WORKSPACE, "Laplacian workspace too small");
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const long long n1 = std::max<long long>(n_vol, 1);
  int32_t* cnt = (int32_t*)ws;
  int64_t* tmp = (int64_t*)(ws + al(sizeof(int32_t) * n1));
  int32_t* too_long = (int32_t*)(ws + al(sizeof(int32_t) * n1) + al(sizeof(int64_t) * (scan_tiles(n1) + 1)));
  *nnz = 0;
  if (n_vol <= 0) {
    const int64_t zero = 0;
    CC_HIP(hipMemcpyAsync(lap_ptr, &zero, sizeof(int64_t), hipMemcpyHostToDevice, st));
    CC_HIP(hipStreamSynchronize(st));
    return CUTCELL_OK;
  }
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, too_long, 1LL, 0);
  if (D == 3)
    hipLaunchKernelGGL((k_lap_rows<3, false>), dim3((unsigned)n_vol), dim3(64), 0, st, n_vol, vol_face, vol_scale,
                       row_ptr, col, val, cnt, nullptr, nullptr, nullptr, too_long);
  else
    hipLaunchKernelGGL((k_lap_rows<2, false>), dim3((unsigned)n_vol), dim3(64), 0, st, n_vol, vol_face, vol_scale,
                       row_ptr, col, val, cnt, nullptr, nullptr, nullptr, too_long);
  int rc = exclusive_scan<int32_t, int64_t>(cnt, n_vol, n_vol, 1, lap_ptr, n_vol, lap_ptr + n_vol, tmp, st);
  if (rc) return rc;
  int32_t bad = 0;
  CC_HIP(hipMemcpyAsync(nnz, lap_ptr + n_vol, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  CC_HIP(hipMemcpyAsync(&bad, too_long, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  CC_HIP(hipGetLastError());
  if (bad) return fail(CUTCELL_E_UNSUPPORTED, "a volume's face rows hold more than 1024 entries");
  return CUTCELL_OK;
}

int laplacian_fill(int D, long long n_vol, const int64_t* row_ptr, const int32_t* col, const double* val,
                   const int32_t* vol_face, const double* vol_scale, const int64_t* lap_ptr, int32_t* lap_col,
                   double* lap_val, hipStream_t st) {
  if (n_vol <= 0) return CUTCELL_OK;
  if (D == 3)
    hipLaunchKernelGGL((k_lap_rows<3, true>), dim3((unsigned)n_vol), dim3(64), 0, st, n_vol, vol_face, vol_scale,
                       row_ptr, col, val, nullptr, lap_ptr, lap_col, lap_val, nullptr);
  else
    hipLaunchKernelGGL((k_lap_rows<2, true>), dim3((unsigned)n_vol), dim3(64), 0, st, n_vol, vol_face, vol_scale,
                       row_ptr, col, val, nullptr, lap_ptr, lap_col, lap_val, nullptr);
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

// L = lap Phi: one CSR gather over the volumes (F rows per wave, U rounds of 64 entries)
int apply_laplacian(int D, long long n_vol, const int64_t* lap_ptr, const int32_t* lap_col, const double* lap_val,
                    const double* phi, double* lphi, hipStream_t st) {
  if (n_vol <= 0) return CUTCELL_OK;
  const int T = 256;
  if (D == 3) {
    constexpr int F = 4, U = 10;  // ~129 entries per regular volume (the fastest shape measured)
    const long long waves = (n_vol + F - 1) / F;
    hipLaunchKernelGGL((k_flux<F, U>), dim3((unsigned)((waves * 64 + T - 1) / T)), dim3(T), 0, st, n_vol, lap_ptr,
                       lap_col, lap_val, phi, lphi);
  } else {
    constexpr int F = 8, U = 4;   // ~25-40 entries per volume
    const long long waves = (n_vol + F - 1) / F;
    hipLaunchKernelGGL((k_flux<F, U>), dim3((unsigned)((waves * 64 + T - 1) / T)), dim3(T), 0, st, n_vol, lap_ptr,
                       lap_col, lap_val, phi, lphi);
  }
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

}  // namespace cutcell
