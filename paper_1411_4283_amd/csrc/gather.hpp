// CSR row gather out[r] = sum_{j in row r} val[j] x[col[j]]: the face fluxes of the
// operator apply, and the rows of the volume Laplacian.
#pragma once

#include "kernels.hpp"

namespace cutcell {

// One wave streams the contiguous nonzeros of F consecutive faces: in each of U rounds
// every lane loads one (col, val) pair, so a load instruction covers 64 consecutive
// entries (256 B of col, 512 B of val, non-temporal) and all of a round's loads are in
// flight before the first Phi gather.  Products are summed per face by masking against
// the faces' row bounds, then reduced across the wave in a fixed order.  Products and
// sums stay separate roundings (no contraction): the compressed apply reproduces these
// sums bit for bit.  With SKIP, the faces `skip` marks are left out: their entries are
// neither loaded nor gathered and their outputs not written.
template <int F, int U, bool SKIP>
__device__ __forceinline__ void flux_group(long long w, int lane, long long n_face, const int64_t* __restrict__ row_ptr,
                                           const int32_t* __restrict__ col, const double* __restrict__ val,
                                           const double* __restrict__ phi, double* __restrict__ flux,
                                           const uint8_t* __restrict__ skip) {
#pragma clang fp contract(off)
  const long long f0 = w * F;
  if (f0 >= n_face) return;
  bool sk[F];
  bool all = true;
#pragma unroll
  for (int i = 0; i < F; ++i) {
    sk[i] = SKIP && (f0 + i >= n_face || skip[f0 + i] != 0);
    all = all && sk[i];
  }
  if (SKIP && all) return;
  int64_t bnd[F + 1];
#pragma unroll
  for (int i = 0; i <= F; ++i) bnd[i] = row_ptr[(f0 + i < n_face) ? f0 + i : n_face];
  double s[F];
#pragma unroll
  for (int i = 0; i < F; ++i) s[i] = 0.0;
  for (int64_t e0 = bnd[0]; e0 < bnd[F]; e0 += 64 * U) {
    int32_t c[U];
    double v[U];
    int64_t e[U];
    bool live[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      e[u] = e0 + lane + 64 * u;
      bool in = e[u] < bnd[F];
#pragma unroll
      for (int i = 0; i < F; ++i) in = in && !(sk[i] && e[u] >= bnd[i] && e[u] < bnd[i + 1]);
      live[u] = in;
      c[u] = in ? __builtin_nontemporal_load(col + e[u]) : 0;
      v[u] = in ? __builtin_nontemporal_load(val + e[u]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // a lane out of the rows, or of a skipped face, reaches no written sum
      const double p = (SKIP && !live[u]) ? 0.0 : v[u] * phi[c[u]];
#pragma unroll
      for (int i = 0; i < F; ++i) s[i] += (e[u] >= bnd[i] && e[u] < bnd[i + 1]) ? p : 0.0;
    }
  }
#pragma unroll
  for (int i = 0; i < F; ++i)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s[i] += __shfl_xor(s[i], off, 64);
  if (lane < F && f0 + lane < n_face) {
    double o = s[0];
    bool k = sk[0];
#pragma unroll
    for (int i = 1; i < F; ++i)
      if (lane == i) {
        o = s[i];
        k = sk[i];
      }
    if (!k) flux[f0 + lane] = o;
  }
}

// The CSR pass as a kernel: flux_group without skips, written out (the shared template
// costs the 10-round instance 14 registers and a wave per SIMD).
template <int F, int U>
__global__ __launch_bounds__(256) void k_flux(long long n_face, const int64_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col, const double* __restrict__ val,
                                              const double* __restrict__ phi, double* __restrict__ flux) {
#pragma clang fp contract(off)
  const long long w = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const long long f0 = w * F;
  if (f0 >= n_face) return;
  int64_t bnd[F + 1];
#pragma unroll
  for (int i = 0; i <= F; ++i) bnd[i] = row_ptr[(f0 + i < n_face) ? f0 + i : n_face];
  double s[F];
#pragma unroll
  for (int i = 0; i < F; ++i) s[i] = 0.0;
  for (int64_t e0 = bnd[0]; e0 < bnd[F]; e0 += 64 * U) {
    int32_t c[U];
    double v[U];
    int64_t e[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      e[u] = e0 + lane + 64 * u;
      const bool in = e[u] < bnd[F];
      c[u] = in ? __builtin_nontemporal_load(col + e[u]) : 0;
      v[u] = in ? __builtin_nontemporal_load(val + e[u]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double p = v[u] * phi[c[u]];
#pragma unroll
      for (int i = 0; i < F; ++i) s[i] += (e[u] >= bnd[i] && e[u] < bnd[i + 1]) ? p : 0.0;
    }
  }
#pragma unroll
  for (int i = 0; i < F; ++i)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s[i] += __shfl_xor(s[i], off, 64);
  if (lane < F && f0 + lane < n_face) {
    double o = s[0];
#pragma unroll
    for (int i = 1; i < F; ++i)
      if (lane == i) o = s[i];
    flux[f0 + lane] = o;
  }
}

}  // namespace cutcell
