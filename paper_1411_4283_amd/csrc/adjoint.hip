// Adjoints of the operator apply and of the stencils (derivatives of Sec. 2.2 and
// Sec. 2.2.1).  Every output is produced by exactly one thread group in a fixed order, so
// repeated calls give identical bits (no floating-point atomics):
//   * the transpose (CSC) of the stencils is a stable radix sort of the CSR positions by
//     column, so each Phi entry lists its nonzeros in ascending CSR position;
//   * the apply adjoint scatters each volume's cotangent onto its at most 2D+1 faces in two
//     passes (a face is the high face of at most one volume and the low face of at most
//     one), then gathers Phi-bar through the transpose;
//   * the moment gradients of the rows are summed per Phi entry through the transpose.
#include <algorithm>
#include <string>

#include <hipcub/hipcub.hpp>

#include "kernels.hpp"
#include "rows.hpp"

namespace cutcell {

static inline unsigned nblocks(long long n, int t) { return (unsigned)((n + t - 1) / t); }

// ---- transpose -------------------------------------------------------------------------
__global__ void k_iota(int32_t* p, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

// col_ptr from the sorted columns: entry k starts at the first position whose key is >= k
__global__ void k_col_ptr(long long nnz, long long n_phi, const int32_t* __restrict__ keys,
                          int64_t* __restrict__ col_ptr) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i > nnz) return;
  const long long prev = (i == 0) ? -1 : keys[i - 1];
  const long long cur = (i == nnz) ? n_phi : keys[i];
  for (long long k = prev + 1; k <= cur; ++k) col_ptr[k] = i;
}

// face of each listed CSR position (binary search in row_ptr)
__global__ void k_nz_face(long long nnz, long long n_face, const int64_t* __restrict__ row_ptr,
                          const int32_t* __restrict__ nz, int32_t* __restrict__ nz_face) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const int64_t j = nz[i];
  long long lo = 0, hi = n_face;   // row_ptr[lo] <= j < row_ptr[hi]
  while (hi - lo > 1) {
    const long long mid = (lo + hi) >> 1;
    if (row_ptr[mid] <= j) lo = mid;
    else hi = mid;
  }
  nz_face[i] = (int32_t)lo;
}

static int key_bits(long long n_phi) {
  int b = 1;
  while ((1LL << b) < n_phi) ++b;
  return b;
}

size_t transpose_temp_bytes(long long nnz, long long n_phi) {
  size_t temp = 0;
  if (nnz > 0)
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, temp, (const int32_t*)nullptr, (int32_t*)nullptr,
                                             (const int32_t*)nullptr, (int32_t*)nullptr, (int)nnz, 0,
                                             key_bits(n_phi), (hipStream_t)0);
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  return al(temp) + 2 * al(sizeof(int32_t) * (size_t)std::max<long long>(nnz, 1));
}

int build_transpose(long long n_face, long long n_phi, long long nnz, const int64_t* row_ptr, const int32_t* col,
                    int64_t* col_ptr, int32_t* nz, int32_t* nz_face, char* ws, size_t ws_bytes, hipStream_t st) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  size_t temp = 0;
  if (nnz > 0)
    CC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, temp, (const int32_t*)nullptr, (int32_t*)nullptr,
                                              (const int32_t*)nullptr, (int32_t*)nullptr, (int)nnz, 0,
                                              key_bits(n_phi), st));
  const size_t need = al(temp) + 2 * al(sizeof(int32_t) * (size_t)std::max<long long>(nnz, 1));
  if (!ws || ws_bytes < need) return fail(CUTCELL_E_WORKSPACE, "transpose workspace too small: need " + std::to_string(need));
  int32_t* keys_out = (int32_t*)(ws + al(temp));
  int32_t* vals_in = (int32_t*)(ws + al(temp) + al(sizeof(int32_t) * (size_t)std::max<long long>(nnz, 1)));
  if (nnz > 0) {
    hipLaunchKernelGGL(k_iota, dim3(nblocks(nnz, 256)), dim3(256), 0, st, vals_in, nnz);
    CC_HIP(hipcub::DeviceRadixSort::SortPairs(ws, temp, col, keys_out, vals_in, nz, (int)nnz, 0, key_bits(n_phi), st));
    hipLaunchKernelGGL(k_nz_face, dim3(nblocks(nnz, 256)), dim3(256), 0, st, nnz, n_face, row_ptr, nz, nz_face);
  }
  hipLaunchKernelGGL(k_col_ptr, dim3(nblocks(nnz + 1, 256)), dim3(256), 0, st, nnz, n_phi, keys_out, col_ptr);
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

// ---- apply adjoint ------------------------------------------------------------------------
// dl/dflux_f = sum over the volumes v of f of sigma_vf * scale_v * lbar_v.  Pass 0 adds the
// volumes for which f is the high or the EB face (sigma = +1), pass 1 the volumes for which
// f is the low face (sigma = -1).
template <int D, int PASS>
__global__ __launch_bounds__(256) void k_face_cotangent(long long n_vol, const int32_t* __restrict__ vol_face,
                                                        const double* __restrict__ vol_scale,
                                                        const double* __restrict__ lbar, double* __restrict__ fbar) {
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= n_vol) return;
  constexpr int S = 2 * D + 1;
  const int32_t* vf = vol_face + v * S;
  const double c = vol_scale[v] * lbar[v];
  if (PASS == 0) {
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (vf[2 * d + 1] >= 0) fbar[vf[2 * d + 1]] += c;
    if (vf[2 * D] >= 0) fbar[vf[2 * D]] += c;
  } else {
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (vf[2 * d] >= 0) fbar[vf[2 * d]] -= c;
  }
}

// Phi-bar_k = sum over the nonzeros j of column k of val[j] * fbar[face(j)]
template <int SW>
__global__ __launch_bounds__(256) void k_phi_bar(long long n_phi, const int64_t* __restrict__ col_ptr,
                                                 const int32_t* __restrict__ nz, const int32_t* __restrict__ nz_face,
                                                 const double* __restrict__ val, const double* __restrict__ fbar,
                                                 double* __restrict__ phi_bar) {
  const long long gt = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long k = gt / SW;
  const int sl = threadIdx.x % SW;
  double s = 0.0;
  if (k < n_phi) {
    const int64_t a = col_ptr[k], b = col_ptr[k + 1];
    for (int64_t i = a + sl; i < b; i += SW) s = fma(val[nz[i]], fbar[nz_face[i]], s);
  }
#pragma unroll
  for (int off = SW / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, SW);
  if (k < n_phi && sl == 0) phi_bar[k] = s;
}

// val-bar_j = fbar[f] * Phi[col[j]] over the rows of face f
template <int SW>
__global__ __launch_bounds__(256) void k_val_bar(long long n_face, const int64_t* __restrict__ row_ptr,
                                                 const int32_t* __restrict__ col, const double* __restrict__ fbar,
                                                 const double* __restrict__ phi, double* __restrict__ val_bar) {
  const long long gt = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long f = gt / SW;
  const int sl = threadIdx.x % SW;
  if (f >= n_face) return;
  const double c = fbar[f];
  const int64_t a = row_ptr[f], b = row_ptr[f + 1];
  for (int64_t j = a + sl; j < b; j += SW) val_bar[j] = c * phi[col[j]];
}

// scale-bar_v = lbar_v * sum over v's faces of sigma * flux (L_v = scale_v times that sum)
template <int D>
__global__ __launch_bounds__(256) void k_scale_bar(long long n_vol, const int32_t* __restrict__ vol_face,
                                                   const double* __restrict__ flux, const double* __restrict__ lbar,
                                                   double* __restrict__ scale_bar) {
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= n_vol) return;
  constexpr int S = 2 * D + 1;
  const int32_t* vf = vol_face + v * S;
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int32_t lo = vf[2 * d], hi = vf[2 * d + 1];
    if (lo >= 0) s -= flux[lo];
    if (hi >= 0) s += flux[hi];
  }
  const int32_t e = vf[2 * D];
  if (e >= 0) s += flux[e];
  scale_bar[v] = lbar[v] * s;
}

template <int D>
static void apply_adjoint_t(long long n_face, long long n_vol, long long n_phi, const int64_t* row_ptr,
                            const int32_t* col, const double* val, const int32_t* vol_face, const double* vol_scale,
                            const Transpose& tr, const double* phi, const double* flux, const double* lbar,
                            double* phi_bar, double* val_bar, double* scale_bar, double* fbar, hipStream_t st) {
  constexpr int SW = (D == 3) ? 32 : 16;
  if (n_face > 0) hipLaunchKernelGGL(k_fill_f64, dim3(nblocks(n_face, 256)), dim3(256), 0, st, fbar, n_face, 0.0);
  if (n_vol > 0) {
    hipLaunchKernelGGL((k_face_cotangent<D, 0>), dim3(nblocks(n_vol, 256)), dim3(256), 0, st, n_vol, vol_face, vol_scale,
                       lbar, fbar);
    hipLaunchKernelGGL((k_face_cotangent<D, 1>), dim3(nblocks(n_vol, 256)), dim3(256), 0, st, n_vol, vol_face, vol_scale,
                       lbar, fbar);
    if (scale_bar)
      hipLaunchKernelGGL(k_scale_bar<D>, dim3(nblocks(n_vol, 256)), dim3(256), 0, st, n_vol, vol_face, flux, lbar,
                         scale_bar);
  }
  if (n_phi > 0)
    hipLaunchKernelGGL(k_phi_bar<SW>, dim3(nblocks(n_phi * SW, 256)), dim3(256), 0, st, n_phi, tr.col_ptr, tr.nz,
                       tr.nz_face, val, fbar, phi_bar);
  if (val_bar && n_face > 0)
    hipLaunchKernelGGL(k_val_bar<SW>, dim3(nblocks(n_face * SW, 256)), dim3(256), 0, st, n_face, row_ptr, col, fbar, phi,
                       val_bar);
}

int apply_adjoint(int D, long long n_face, long long n_vol, long long n_phi, const int64_t* row_ptr,
                  const int32_t* col, const double* val, const int32_t* vol_face, const double* vol_scale,
                  const Transpose& tr, const double* phi, const double* flux, const double* lbar, double* phi_bar,
                  double* val_bar, double* scale_bar, double* fbar, hipStream_t st) {
  if (D == 3)
    apply_adjoint_t<3>(n_face, n_vol, n_phi, row_ptr, col, val, vol_face, vol_scale, tr, phi, flux, lbar, phi_bar,
                       val_bar, scale_bar, fbar, st);
  else
    apply_adjoint_t<2>(n_face, n_vol, n_phi, row_ptr, col, val, vol_face, vol_scale, tr, phi, flux, lbar, phi_bar,
                       val_bar, scale_bar, fbar, st);
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

// ---- moment gradients of the rows -----------------------------------------------------------
// For Phi entry k with stored moments m (about its own centre) and each nonzero j of its
// column, in face f with x0:  Abar_j = (W r)_j y_f - (W z)_j w_f,  delta_j = x_k/h - x0/h,
//   g = sum_j S(delta_j)^T Abar_j,   dl/dm = g / m_0 - e_0 (g . m) / m_0^2
// (A~_j = S(delta_j) m / m_0, and the sum of Abar_j . A~_j over j is g . m / m_0).
// Volumes add the gradient through their EB face's centroid (owner_grad) and through
// 1/(kappa h^D) in the apply (scale_bar).  One wave per Phi entry, a lane per nonzero; the
// 64 lane sums are added in lane order.

template <int D, int Q>
__global__ __launch_bounds__(64) void k_moment_reduce(ReduceArgs R) {
  constexpr int M = Dims<D, Q>::M, Mf = Dims<D, Q>::Mf;
  __shared__ double part[64][M + 1];
  __shared__ double tot[M + 1];
  const long long k = blockIdx.x;
  if (k >= R.n_phi) return;
  const int lane = threadIdx.x;
  int lo = 0, hi = R.G;           // offs[lo] <= k < offs[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (R.offs[mid] <= k) lo = mid;
    else hi = mid;
  }
  const int gi = lo;
  const GeomPtrs gp = R.geoms[gi];
  const int64_t loc = k - R.offs[gi];
  const int64_t n_vol = R.counts[4 * gi + 0], n_eb = R.counts[4 * gi + 1];
  const int32_t* vol_cell = R.vol_cell_ws + (long long)gi * R.g.ncell;
  const RowSource rs =
      row_source<D, Q>(R.g, gp, loc, n_vol, n_eb, vol_cell, R.box_lf_ws + (long long)gi * R.g.nboxslot);
  double g[M];
  static_for<0, M>([&](auto I) { g[I] = 0.0; });
  const int64_t a = R.tr.col_ptr[k], b = R.tr.col_ptr[k + 1];
  for (int64_t i = a + lane; i < b; i += 64) {
    const int64_t j = R.tr.nz[i];
    const int32_t f = R.tr.nz_face[i];
    const double wr = R.nz_rz[2 * j], wz = R.nz_rz[2 * j + 1];
    const double* yw = R.face_yw + (long long)f * 2 * M;
    double ab[M];
    static_for<0, M>([&](auto I) { ab[I] = wr * yw[I] - wz * yw[M + I]; });
    double dl[3] = {0, 0, 0};
    for (int ax = 0; ax < D; ++ax) dl[ax] = rs.ctr[ax] - R.face_x0[(long long)f * 4 + ax];
    recentre_T<D, Q>(ab, dl);
    static_for<0, M>([&](auto I) { g[I] += ab[I]; });
  }
  static_for<0, M>([&](auto I) { part[lane][I] = g[I]; });
  __syncthreads();
  double m[M];
  load_row_moments<D, Q>(rs, m);
  if (lane < M) {
    double s = 0.0;
    for (int l = 0; l < 64; ++l) s += part[l][lane];
    tot[lane] = s;
  }
  __syncthreads();
  double gm = 0.0;
  static_for<0, M>([&](auto I) { gm = fma(tot[I], m[I], gm); });
  if (lane >= M) return;
  const double m0 = m[0];
  double out = tot[lane] / m0;
  if (lane == 0) out -= gm / (m0 * m0);
  const GradPtrs gr = R.grads[gi];
  if (rs.dd < 0 && loc < n_vol) {
    const long long vg = R.offs[(R.G + 1) + gi] + loc;          // global volume index
    if (lane == 0 && R.scale_bar) out -= R.scale_bar[vg] * R.vol_scale[vg] / m0;   // d(1/(kappa h^D))/d kappa
    const int32_t fe = R.vol_face[vg * (2 * D + 1) + 2 * D];
    if (fe >= 0 && lane <= D) out += R.owner_grad[(long long)fe * 4 + lane];
    gr.vol_mom[(long long)rs.cell * M + lane] = out;
  } else if (rs.dd < 0) {
    gr.eb_mom[(loc - n_vol) * M + lane] = out;
  } else {
    // box face: only the transverse moments are stored; the face kernel has already
    // written their flux-vector part
    const int sl = face_slot<D, Q>(lane, rs.dd);
    if (sl >= 0) gr.face_mom[rs.dd][rs.loc * Mf + sl] += out;
  }
}

int reduce_moments(const cutcell_opts& o, const ReduceArgs& R, hipStream_t st) {
  if (R.n_phi <= 0) return CUTCELL_OK;
  const dim3 grid((unsigned)R.n_phi), block(64);
  if (o.dim == 2 && o.order == 2) hipLaunchKernelGGL((k_moment_reduce<2, 2>), grid, block, 0, st, R);
  else if (o.dim == 2 && o.order == 4) hipLaunchKernelGGL((k_moment_reduce<2, 4>), grid, block, 0, st, R);
  else if (o.dim == 3 && o.order == 2) hipLaunchKernelGGL((k_moment_reduce<3, 2>), grid, block, 0, st, R);
  else if (o.dim == 3 && o.order == 4) hipLaunchKernelGGL((k_moment_reduce<3, 4>), grid, block, 0, st, R);
  else return fail(CUTCELL_E_UNSUPPORTED, "order/dimension");
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

}  // namespace cutcell
