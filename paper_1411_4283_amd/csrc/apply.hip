// Operator apply (Sec. 2.2, eq. 'laplacian over V'; Sec. 3.3):
//   flux_f = s_f^T Phi                        (CSR gather, HBM bound)
//   L_v    = 1/(kappa_v h^D) sum_f sigma flux_f (gather over the volume's <= 2D+1 faces)
// Both passes are gathers, so every output is written once and the result is
// deterministic (no atomics).
#include "kernels.hpp"

namespace cutcell {

// SW lanes per CSR row; a 64-lane wave handles 64/SW rows.  Loads of col/val stream
// once (non-temporal), Phi is re-read through the caches.
template <int SW>
__global__ __launch_bounds__(256) void k_flux(long long n_face, const int64_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col, const double* __restrict__ val,
                                              const double* __restrict__ phi, double* __restrict__ flux) {
  const long long gt = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long f = gt / SW;
  const int sl = threadIdx.x % SW;
  double s = 0.0;
  if (f < n_face) {
    const int64_t a = row_ptr[f], b = row_ptr[f + 1];
    for (int64_t j = a + sl; j < b; j += SW) {
      const int32_t c = __builtin_nontemporal_load(col + j);
      const double v = __builtin_nontemporal_load(val + j);
      s = fma(v, phi[c], s);
    }
  }
#pragma unroll
  for (int off = SW / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, SW);
  if (f < n_face && sl == 0) flux[f] = s;
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
    const int T = 256;
    if (D == 3) {
      constexpr int SW = 32;
      hipLaunchKernelGGL((k_flux<SW>), dim3((unsigned)((n_face * SW + T - 1) / T)), dim3(T), 0, st, n_face, row_ptr, col,
                         val, phi, flux);
    } else {
      constexpr int SW = 16;
      hipLaunchKernelGGL((k_flux<SW>), dim3((unsigned)((n_face * SW + T - 1) / T)), dim3(T), 0, st, n_face, row_ptr, col,
                         val, phi, flux);
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
