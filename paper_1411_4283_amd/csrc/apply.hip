// Operator apply (Sec. 2.2, eq. 'laplacian over V'; Sec. 3.3):
//   flux_f = s_f^T Phi                        (CSR gather, HBM bound)
//   L_v    = 1/(kappa_v h^D) sum_f sigma flux_f (gather over the volume's <= 2D+1 faces)
// Both passes are gathers, so every output is written once and the result is
// deterministic (no atomics).
#include "kernels.hpp"

namespace cutcell {

// One wave streams the contiguous nonzeros of F consecutive faces: in each of U rounds
// every lane loads one (col, val) pair, so a load instruction covers 64 consecutive
// entries (256 B of col, 512 B of val, non-temporal) and all of a round's loads are in
// flight before the first Phi gather.  Products are summed per face by masking against
// the faces' row bounds, then reduced across the wave in a fixed order.
template <int F, int U>
__global__ __launch_bounds__(256) void k_flux(long long n_face, const int64_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col, const double* __restrict__ val,
                                              const double* __restrict__ phi, double* __restrict__ flux) {
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

template <int D>
__global__ __launch_bounds__(256) void k_divergence(long long n_vol, const int32_t* __restrict__ vol_face,
                                                    const double* __restrict__ vol_scale,
                                                    const double* __restrict__ flux, double* __restrict__ lphi) {
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= n_vol) return;
  constexpr int S = 2 * D + 1;
  const int32_t* vf = vol_face + v * S;
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int32_t lo = vf[2 * d], hi = vf[2 * d + 1];
    if (lo >= 0) s -= flux[lo];   // the low face's normal +e_d points into v
    if (hi >= 0) s += flux[hi];
  }
  const int32_t e = vf[2 * D];
  if (e >= 0) s += flux[e];       // the EB normal points out of the fluid
  lphi[v] = vol_scale[v] * s;
}

int apply_operator(int D, long long n_face, long long n_vol, const int64_t* row_ptr, const int32_t* col,
                   const double* val, const int32_t* vol_face, const double* vol_scale, const double* phi,
                   double* lphi, double* flux, double* flux_tmp, hipStream_t st) {
  (void)flux_tmp;
  if (n_face > 0) {
    // faces per wave and rounds: about 88 rows per face in 3D order 4, 20-35 in 2D
    const int T = 256;
    if (D == 3) {
      constexpr int F = 4, U = 6;
      const long long waves = (n_face + F - 1) / F;
      hipLaunchKernelGGL((k_flux<F, U>), dim3((unsigned)((waves * 64 + T - 1) / T)), dim3(T), 0, st, n_face, row_ptr,
                         col, val, phi, flux);
    } else {
      constexpr int F = 8, U = 4;
      const long long waves = (n_face + F - 1) / F;
      hipLaunchKernelGGL((k_flux<F, U>), dim3((unsigned)((waves * 64 + T - 1) / T)), dim3(T), 0, st, n_face, row_ptr,
                         col, val, phi, flux);
    }
  }
  if (n_vol > 0) {
    if (D == 3)
      hipLaunchKernelGGL(k_divergence<3>, dim3((unsigned)((n_vol + 255) / 256)), dim3(256), 0, st, n_vol, vol_face,
                         vol_scale, flux, lphi);
    else
      hipLaunchKernelGGL(k_divergence<2>, dim3((unsigned)((n_vol + 255) / 256)), dim3(256), 0, st, n_vol, vol_face,
                         vol_scale, flux, lphi);
  }
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

}  // namespace cutcell
