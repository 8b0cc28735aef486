// Operator apply (Sec. 2.2, eq. 'laplacian over V'; Sec. 3.3):
//   flux_f = s_f^T Phi                        (CSR gather, HBM bound)
//   L_v    = 1/(kappa_v h^D) sum_f sigma flux_f (gather over the volume's <= 2D+1 faces)
// Both passes are gathers, so every output is written once and the result is
// deterministic (no atomics).
#include "gather.hpp"

namespace cutcell {

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

int flux_faces(int D, long long n_face, const int64_t* row_ptr, const int32_t* col, const double* val,
               const double* phi, double* flux, hipStream_t st) {
  if (n_face <= 0) return CUTCELL_OK;
  // faces per wave and rounds: about 88 rows per face in 3D order 4, 20-35 in 2D
  const int T = 256;
  if (D == 3) {
    constexpr int F = kFluxFaces3, U = kFluxRounds3;
    const long long waves = (n_face + F - 1) / F;
    hipLaunchKernelGGL((k_flux<F, U>), dim3((unsigned)((waves * 64 + T - 1) / T)), dim3(T), 0, st, n_face, row_ptr,
                       col, val, phi, flux);
  } else {
    constexpr int F = kFluxFaces2, U = kFluxRounds2;
    const long long waves = (n_face + F - 1) / F;
    hipLaunchKernelGGL((k_flux<F, U>), dim3((unsigned)((waves * 64 + T - 1) / T)), dim3(T), 0, st, n_face, row_ptr,
                       col, val, phi, flux);
  }
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

int divergence(int D, long long n_vol, const int32_t* vol_face, const double* vol_scale, const double* flux,
               double* lphi, hipStream_t st) {
  if (n_vol <= 0) return CUTCELL_OK;
  if (D == 3)
    hipLaunchKernelGGL(k_divergence<3>, dim3((unsigned)((n_vol + 255) / 256)), dim3(256), 0, st, n_vol, vol_face,
                       vol_scale, flux, lphi);
  else
    hipLaunchKernelGGL(k_divergence<2>, dim3((unsigned)((n_vol + 255) / 256)), dim3(256), 0, st, n_vol, vol_face,
                       vol_scale, flux, lphi);
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

int apply_operator(int D, long long n_face, long long n_vol, const int64_t* row_ptr, const int32_t* col,
                   const double* val, const int32_t* vol_face, const double* vol_scale, const double* phi,
                   double* lphi, double* flux, double* flux_tmp, hipStream_t st) {
  (void)flux_tmp;
  int rc = flux_faces(D, n_face, row_ptr, col, val, phi, flux, st);
  if (rc) return rc;
  return divergence(D, n_vol, vol_face, vol_scale, flux, lphi, st);
}

}  // namespace cutcell
