// Discrete Poisson solve with the flux-divergence operator (Sec. 3.2: L(Phi) = f for the
// volume values of Phi, the boundary rows of Phi holding Dirichlet data).
//
// L is affine in the volume values x:  L([x | bc]) = A x + L([0 | bc]).  Restarted GMRES(m)
// solves A x = f - L([0 | bc]) with right Jacobi preconditioning (A D^-1 y = b, x = D^-1 y,
// D = diag A).  Every vector operation is a kernel here; the host keeps only the small
// Hessenberg matrix and its Givens rotations.  Orthogonalisation is classical Gram-Schmidt
// done twice (CGS2): one batched inner-product kernel and one batched update per pass.
// All reductions sum per-block partials in a fixed order, so a solve is deterministic.
#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "solve.hpp"

namespace cutcell {

constexpr int kDotBlock = 256;
constexpr int kDotBlocks = 512;      // fixed number of partial sums per inner product

static inline unsigned nb(long long n, int t) { return (unsigned)((n + t - 1) / t); }

// Phi index of every volume: geometry g's volumes sit at phi_off[g] + (v - vol_off[g])
__global__ void k_vol_phi(long long n_vol, int G, const int64_t* __restrict__ phi_off,
                          const int64_t* __restrict__ vol_off, int32_t* __restrict__ vol_phi) {
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= n_vol) return;
  int lo = 0, hi = G;                // vol_off[lo] <= v < vol_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (vol_off[mid] <= v) lo = mid;
    else hi = mid;
  }
  vol_phi[v] = (int32_t)(phi_off[lo] + (v - vol_off[lo]));
}

__global__ void k_scatter(long long n, const int32_t* __restrict__ idx, const double* __restrict__ x,
                          double* __restrict__ phi) {
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v < n) phi[idx[v]] = x[v];
}

__global__ void k_copy(long long n, const double* __restrict__ a, double* __restrict__ b) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// out = alpha * a + beta * b (out may alias a or b)
__global__ void k_axpby(long long n, double alpha, const double* a, double beta, const double* b, double* out) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) out[i] = alpha * a[i] + beta * b[i];
}

__global__ void k_mul(long long n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] * b[i];
}

// D^-1: A_vv = vol_scale[v] * sum over v's faces of sigma * (the face's coefficient on v)
template <int D>
__global__ void k_jacobi(long long n_vol, const int32_t* __restrict__ vol_face, const double* __restrict__ vol_scale,
                         const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                         const double* __restrict__ val, const int32_t* __restrict__ vol_phi,
                         double* __restrict__ dinv) {
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= n_vol) return;
  constexpr int S = 2 * D + 1;
  const int32_t me = vol_phi[v];
  double s = 0.0;
  for (int k = 0; k < S; ++k) {
    const int32_t f = vol_face[v * S + k];
    if (f < 0) continue;
    const double sigma = (k < 2 * D && (k & 1) == 0) ? -1.0 : 1.0;   // low faces point into v
    int64_t lo = row_ptr[f], hi = row_ptr[f + 1];                       // col ascending: search
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (col[mid] < me) lo = mid + 1;
      else hi = mid;
    }
    if (lo < row_ptr[f + 1] && col[lo] == me) s += sigma * val[lo];
  }
  const double a = vol_scale[v] * s;
  dinv[v] = (a != 0.0 && isfinite(a)) ? 1.0 / a : 1.0;
}

// partial[i][b] = block b's share of V_i . w for i < k, and of w . w as entry k when
// `self` (V row-major [k][n]).  Eight products per pass over w; each is summed per thread
// in a fixed order, across the wave by butterfly shuffles, then over the block's waves.
constexpr int kChunk = 8;
__global__ __launch_bounds__(kDotBlock) void k_mdot(long long n, int k, int self, const double* __restrict__ V,
                                                     const double* __restrict__ w, double* __restrict__ partial) {
  __shared__ double red[kDotBlock / 64][kChunk];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int kk = k + (self ? 1 : 0);
  for (int i0 = 0; i0 < kk; i0 += kChunk) {
    double acc[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) acc[u] = 0.0;
    for (long long t = blockIdx.x * (long long)kDotBlock + threadIdx.x; t < n; t += (long long)kDotBlocks * kDotBlock) {
      const double wt = w[t];
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        const int i = i0 + u;
        if (i < k) acc[u] = fma(V[(long long)i * n + t], wt, acc[u]);
        else if (i == k && self) acc[u] = fma(wt, wt, acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc[u] += __shfl_xor(acc[u], off, 64);
    if (lane == 0)
#pragma unroll
      for (int u = 0; u < kChunk; ++u) red[wv][u] = acc[u];
    __syncthreads();
    if ((int)threadIdx.x < kChunk) {
      double sum = 0.0;
      for (int q = 0; q < kDotBlock / 64; ++q) sum += red[q][threadIdx.x];
      const int i = i0 + threadIdx.x;
      if (i < kk) partial[(long long)i * kDotBlocks + blockIdx.x] = sum;
    }
    __syncthreads();
  }
}

// out[i] = sum of partial[i][0..kDotBlocks) in a fixed order (one block per i)
__global__ __launch_bounds__(kDotBlock) void k_mdot_final(const double* __restrict__ partial, double* __restrict__ out) {
  __shared__ double red[kDotBlock];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < kDotBlocks; b += kDotBlock) s += partial[(long long)i * kDotBlocks + b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = kDotBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// After the second Gram-Schmidt pass: d holds its coefficients c[0..k) and, in d[k], the
// squared norm of the vector it started from, so the new norm is sqrt(d[k] - |c|^2) (c is
// at rounding level after the first pass).  hn[0] = norm, hn[1] = 1/norm (0 if the norm
// vanishes: a lucky breakdown).
__global__ void k_norm_after(const double* __restrict__ d, int k, double* __restrict__ hn) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double c2 = 0.0;
  for (int i = 0; i < k; ++i) c2 = fma(d[i], d[i], c2);
  const double q = d[k] - c2;
  const double r = q > 0.0 ? sqrt(q) : 0.0;
  hn[0] = r;
  hn[1] = r > 0.0 ? 1.0 / r : 0.0;
}

// out = s[1] * w (s on the device)
__global__ void k_scale_dev(long long n, const double* __restrict__ w, const double* __restrict__ sc,
                            double* __restrict__ out) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t < n) out[t] = w[t] * sc[1];
}

// w -= sum_{i<k} c[i] V_i
__global__ void k_maxpy(long long n, int k, const double* __restrict__ c, const double* __restrict__ V,
                        double* __restrict__ w) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  double s = w[t];
  for (int i = 0; i < k; ++i) s = fma(-c[i], V[i * n + t], s);
  w[t] = s;
}

static inline size_t coef_words(int m) { return (size_t)(m + 1) + (m + 2) + 2; }   // pass 1 | pass 2 | norm

size_t solve_workspace_bytes(long long n_vol, long long n_phi, long long n_face, int m) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t nv = std::max<long long>(n_vol, 1);
  return al(sizeof(double) * n_phi) * 2 + al(sizeof(double) * std::max<long long>(n_face, 1)) +
         al(sizeof(double) * nv) * 5 + al(sizeof(int32_t) * nv) + al(sizeof(double) * nv * (m + 1)) +
         al(sizeof(double) * kDotBlocks * (m + 2)) + al(sizeof(double) * coef_words(m)) + al(sizeof(double) * (m + 1));
}

int solve_poisson(const SolveOp& op, int G, const int64_t* phi_off, const int64_t* vol_off, const double* phi_bc,
                  const double* f, double* x, int m, int max_iters, double rtol, char* ws, size_t ws_bytes,
                  int* iters_out, double* relres_out) {
  const long long n = op.n_vol;
  if (ws_bytes < solve_workspace_bytes(n, op.n_phi, op.n_face, m))
    return fail(CUTCELL_E_WORKSPACE, "solve workspace too small");
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  size_t off = 0;
  auto take = [&](size_t bytes) { char* p = ws + off; off += al(bytes); return p; };
  const size_t nv = std::max<long long>(n, 1);
  double* phi = (double*)take(sizeof(double) * op.n_phi);     // [x | bc]
  double* phi0 = (double*)take(sizeof(double) * op.n_phi);    // [v | 0]
  double* flux = (double*)take(sizeof(double) * std::max<long long>(op.n_face, 1));
  double* b = (double*)take(sizeof(double) * nv);
  double* w = (double*)take(sizeof(double) * nv);
  double* z = (double*)take(sizeof(double) * nv);
  double* dinv = (double*)take(sizeof(double) * nv);
  double* tmp = (double*)take(sizeof(double) * nv);
  int32_t* vphi = (int32_t*)take(sizeof(int32_t) * nv);
  double* V = (double*)take(sizeof(double) * nv * (m + 1));
  double* partial = (double*)take(sizeof(double) * kDotBlocks * (m + 2));
  double* cbuf = (double*)take(sizeof(double) * coef_words(m));   // pass-1 | pass-2 coefficients | norm
  double* coef = (double*)take(sizeof(double) * (m + 1));
  double* c1 = cbuf;
  double* c2 = cbuf + (m + 1);
  double* hnb = cbuf + (m + 1) + (m + 2);
  std::vector<double> hc(coef_words(m));
  hipStream_t st = op.st;
  const int T = 256;
  const unsigned gv = nb(n, T);

  auto apply = [&](const double* p, double* out) {
    if (op.lap_ptr) return apply_laplacian(op.D, n, op.lap_ptr, op.lap_col, op.lap_val, p, out, st);
    return apply_operator(op.D, op.n_face, n, op.row_ptr, op.col, op.val, op.vol_face, op.vol_scale, p, out, flux,
                          nullptr, st);
  };
  // A v = L([v | 0])
  auto matvec = [&](const double* v, double* out) {
    hipLaunchKernelGGL(k_scatter, dim3(gv), dim3(T), 0, st, n, vphi, v, phi0);
    return apply(phi0, out);
  };
  // V^T y (k vectors) and, with self, y.y as entry k, into out on the device
  auto mdot = [&](int k, int self, const double* y, double* out) {
    hipLaunchKernelGGL(k_mdot, dim3(kDotBlocks), dim3(kDotBlock), 0, st, n, k, self, V, y, partial);
    hipLaunchKernelGGL(k_mdot_final, dim3(k + self), dim3(kDotBlock), 0, st, partial, out);
  };
  // ||y||^2 read back to the host
  auto norm2 = [&](const double* y, double* out) {
    mdot(0, 1, y, hnb);
    CC_HIP(hipMemcpyAsync(out, hnb, sizeof(double), hipMemcpyDeviceToHost, st));
    CC_HIP(hipStreamSynchronize(st));
    return (int)CUTCELL_OK;
  };

  hipLaunchKernelGGL(k_vol_phi, dim3(gv), dim3(T), 0, st, n, G, phi_off, vol_off, vphi);
  hipLaunchKernelGGL(k_copy, dim3(nb(op.n_phi, T)), dim3(T), 0, st, op.n_phi, phi_bc, phi);
  hipLaunchKernelGGL(k_fill_f64, dim3(nb(op.n_phi, T)), dim3(T), 0, st, phi0, op.n_phi, 0.0);
  hipLaunchKernelGGL(k_fill_f64, dim3(gv), dim3(T), 0, st, z, n, 0.0);
  // b = f - L([0 | bc])
  hipLaunchKernelGGL(k_scatter, dim3(gv), dim3(T), 0, st, n, vphi, z, phi);
  int rc = apply(phi, tmp);
  if (rc) return rc;
  hipLaunchKernelGGL(k_axpby, dim3(gv), dim3(T), 0, st, n, 1.0, f, -1.0, tmp, b);
  if (op.D == 3)
    hipLaunchKernelGGL(k_jacobi<3>, dim3(gv), dim3(T), 0, st, n, op.vol_face, op.vol_scale, op.row_ptr, op.col,
                       op.val, vphi, dinv);
  else
    hipLaunchKernelGGL(k_jacobi<2>, dim3(gv), dim3(T), 0, st, n, op.vol_face, op.vol_scale, op.row_ptr, op.col,
                       op.val, vphi, dinv);
  double nb2 = 0.0;
  rc = norm2(b, &nb2);
  if (rc) return rc;
  const double bnorm = std::sqrt(nb2);
  if (!std::isfinite(bnorm)) return fail(CUTCELL_E_INVALID_ARG, "non-finite right-hand side or boundary data");
  if (bnorm == 0.0) {               // the solution is x = 0
    hipLaunchKernelGGL(k_fill_f64, dim3(gv), dim3(T), 0, st, x, n, 0.0);
    CC_HIP(hipStreamSynchronize(st));
    if (iters_out) *iters_out = 0;
    if (relres_out) *relres_out = 0.0;
    return CUTCELL_OK;
  }
  int it = 0;
  double res = bnorm;
  std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  for (;;) {
    // r = b - A x; the exit test always uses this true residual
    rc = matvec(x, tmp);
    if (rc) return rc;
    hipLaunchKernelGGL(k_axpby, dim3(gv), dim3(T), 0, st, n, 1.0, b, -1.0, tmp, V);
    double r2 = 0.0;
    rc = norm2(V, &r2);
    if (rc) return rc;
    const double beta = std::sqrt(r2);
    res = beta;
    if (!(beta > rtol * bnorm) || it >= max_iters) break;
    hipLaunchKernelGGL(k_axpby, dim3(gv), dim3(T), 0, st, n, 1.0 / beta, V, 0.0, V, V);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int j = 0;
    for (; j < m && it < max_iters; ++j, ++it) {
      double* vj = V + (long long)j * n;
      double* vn = V + (long long)(j + 1) * n;
      hipLaunchKernelGGL(k_mul, dim3(gv), dim3(T), 0, st, n, dinv, vj, z);     // z = D^-1 v_j
      rc = matvec(z, w);
      if (rc) return rc;
      // classical Gram-Schmidt twice; the coefficients stay on the device, the new
      // vector's norm comes from the second pass, and the host reads all of them once
      mdot(j + 1, 0, w, c1);
      hipLaunchKernelGGL(k_maxpy, dim3(gv), dim3(T), 0, st, n, j + 1, c1, V, w);
      mdot(j + 1, 1, w, c2);
      hipLaunchKernelGGL(k_maxpy, dim3(gv), dim3(T), 0, st, n, j + 1, c2, V, w);
      hipLaunchKernelGGL(k_norm_after, dim3(1), dim3(1), 0, st, c2, j + 1, hnb);
      hipLaunchKernelGGL(k_scale_dev, dim3(gv), dim3(T), 0, st, n, w, hnb, vn);
      CC_HIP(hipMemcpyAsync(hc.data(), cbuf, sizeof(double) * coef_words(m), hipMemcpyDeviceToHost, st));
      CC_HIP(hipStreamSynchronize(st));
      std::vector<double> h(j + 1);
      for (int i = 0; i <= j; ++i) h[i] = hc[i] + hc[(m + 1) + i];
      const double hn = hc[(m + 1) + (m + 2)];
      // Givens rotations on column j of H
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
      }
      const double r = std::hypot(h[j], hn);
      cs[j] = r > 0.0 ? h[j] / r : 1.0;
      sn[j] = r > 0.0 ? hn / r : 0.0;
      h[j] = r;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      for (int i = 0; i <= j; ++i) H[i * m + j] = h[i];
      res = std::fabs(g[j + 1]);
      if (res <= rtol * bnorm || hn == 0.0) {
        ++j;
        ++it;
        break;
      }
    }
    // y = H^-1 g (upper triangular j x j); x += D^-1 V y
    for (int i = j - 1; i >= 0; --i) {
      double s = g[i];
      for (int k = i + 1; k < j; ++k) s -= H[i * m + k] * y[k];
      y[i] = s / H[i * m + i];
    }
    std::vector<double> ny(j);
    for (int i = 0; i < j; ++i) ny[i] = -y[i];
    CC_HIP(hipMemcpyAsync(coef, ny.data(), sizeof(double) * j, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_fill_f64, dim3(gv), dim3(T), 0, st, tmp, n, 0.0);
    hipLaunchKernelGGL(k_maxpy, dim3(gv), dim3(T), 0, st, n, j, coef, V, tmp);   // tmp = V y
    hipLaunchKernelGGL(k_mul, dim3(gv), dim3(T), 0, st, n, dinv, tmp, tmp);
    hipLaunchKernelGGL(k_axpby, dim3(gv), dim3(T), 0, st, n, 1.0, x, 1.0, tmp, x);
    CC_HIP(hipStreamSynchronize(st));
  }
  CC_HIP(hipGetLastError());
  if (iters_out) *iters_out = it;
  if (relres_out) *relres_out = res / bnorm;
  if (!std::isfinite(res)) return fail(CUTCELL_E_BREAKDOWN, "GMRES produced a non-finite residual");
  return res <= rtol * bnorm ? CUTCELL_OK : CUTCELL_W_NOT_CONVERGED;
}

// ---------------------------------------------------------------------------------------
// Extreme eigenvalues of the volume operator A (L restricted to the volume values, the
// boundary entries of Phi zero) from Arnoldi's method on the GPU (the spectra of
// Sec. 3.4 / 3.5, at any size).

// Eigenvalues of an n x n upper Hessenberg matrix (row-major, leading dimension ld) by
// shifted QR iterations in complex arithmetic: Givens rotations reduce the active block
// minus mu I to triangular form R, the block becomes R Q + mu I, mu is the eigenvalue of
// its trailing 2 x 2 part nearer the last diagonal entry (Wilkinson's shift, perturbed
// every 11th step), and the block deflates from the bottom once a subdiagonal entry is
// below the rounding level of its diagonal neighbours.  Host code.  Returns 0, or -1 if an
// eigenvalue needs more than 200 steps.
int hessenberg_eigs(int n, const double* H, int ld, double* re, double* im) {
  using cd = std::complex<double>;
  std::vector<cd> a((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) a[(size_t)i * n + j] = (j >= i - 1) ? cd(H[(size_t)i * ld + j], 0.0) : cd(0.0, 0.0);
  auto A = [&](int i, int j) -> cd& { return a[(size_t)i * n + j]; };
  const double eps = 2.220446049250313e-16;
  int hi = n - 1, steps = 0;
  while (hi >= 0) {
    int lo = hi;
    while (lo > 0 && std::abs(A(lo, lo - 1)) > eps * (std::abs(A(lo, lo)) + std::abs(A(lo - 1, lo - 1)))) --lo;
    if (lo > 0) A(lo, lo - 1) = 0.0;
    if (lo == hi) {
      re[hi] = A(hi, hi).real();
      im[hi] = A(hi, hi).imag();
      --hi;
      steps = 0;
      continue;
    }
    if (++steps > 200) return -1;
    const cd a11 = A(hi - 1, hi - 1), a12 = A(hi - 1, hi), a21 = A(hi, hi - 1), a22 = A(hi, hi);
    const cd half = 0.5 * (a11 + a22);
    const cd disc = std::sqrt(0.25 * (a11 - a22) * (a11 - a22) + a12 * a21);
    const cd m1 = half + disc, m2 = half - disc;
    cd mu = (std::abs(m1 - a22) < std::abs(m2 - a22)) ? m1 : m2;
    if (steps % 11 == 10) mu = a22 + std::abs(a21);
    for (int k = lo; k <= hi; ++k) A(k, k) -= mu;
    std::vector<cd> cs(hi - lo), sn(hi - lo);
    for (int k = lo; k < hi; ++k) {            // R = Q^H (H - mu I)
      const cd x = A(k, k), y = A(k + 1, k);
      const double r = std::hypot(std::abs(x), std::abs(y));
      const cd c = r > 0.0 ? x / r : cd(1.0, 0.0), s = r > 0.0 ? y / r : cd(0.0, 0.0);
      cs[k - lo] = c;
      sn[k - lo] = s;
      for (int j = k; j <= hi; ++j) {
        const cd u = A(k, j), v = A(k + 1, j);
        A(k, j) = std::conj(c) * u + std::conj(s) * v;
        A(k + 1, j) = -s * u + c * v;
      }
    }
    for (int k = lo; k < hi; ++k) {            // R Q
      const cd c = cs[k - lo], s = sn[k - lo];
      for (int i = lo; i <= std::min(k + 1, hi); ++i) {
        const cd u = A(i, k), v = A(i, k + 1);
        A(i, k) = c * u + s * v;
        A(i, k + 1) = -std::conj(s) * u + std::conj(c) * v;
      }
    }
    for (int k = lo; k <= hi; ++k) A(k, k) += mu;
  }
  return 0;
}

// Relative residuals of Ritz pairs: for (theta, y) with H y = theta y (y of unit norm), the
// Arnoldi relation gives |A V y - theta V y| = |h_{k+1,k}| |y_k|; res = that / |theta|.
// y from three steps of inverse iteration with H - theta I (complex Gaussian elimination
// with partial pivoting; theta nudged by 1e-13 relative so the matrix stays invertible).
// Host code; k at most 256 (else res = -1).
void ritz_residuals(int k, const double* H, int ld, double hlast, const double* re, const double* im, double* res) {
  using cd = std::complex<double>;
  if (k > 256) {
    for (int t = 0; t < k; ++t) res[t] = -1.0;
    return;
  }
  std::vector<cd> M((size_t)k * k), y(k), b(k);
  for (int t = 0; t < k; ++t) {
    const cd th(re[t], im[t]);
    const cd sh = th + cd(std::abs(th) * 1e-13 + 1e-300, 0.0);
    for (int i = 0; i < k; ++i) y[i] = 1.0 / std::sqrt((double)k);
    for (int iter = 0; iter < 3; ++iter) {
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j)
          M[(size_t)i * k + j] = (j >= i - 1 ? cd(H[(size_t)i * ld + j], 0.0) : cd(0.0, 0.0)) - (i == j ? sh : cd(0.0));
      b = y;
      for (int c = 0; c < k; ++c) {
        int pr = c;
        for (int r = c + 1; r < k; ++r)
          if (std::abs(M[(size_t)r * k + c]) > std::abs(M[(size_t)pr * k + c])) pr = r;
        if (pr != c) {
          for (int j = c; j < k; ++j) std::swap(M[(size_t)c * k + j], M[(size_t)pr * k + j]);
          std::swap(b[c], b[pr]);
        }
        const cd piv = M[(size_t)c * k + c];
        if (std::abs(piv) == 0.0) continue;
        for (int r = c + 1; r < k; ++r) {
          const cd fct = M[(size_t)r * k + c] / piv;
          if (fct == cd(0.0)) continue;
          for (int j = c; j < k; ++j) M[(size_t)r * k + j] -= fct * M[(size_t)c * k + j];
          b[r] -= fct * b[c];
        }
      }
      for (int i = k - 1; i >= 0; --i) {
        cd acc = b[i];
        for (int j = i + 1; j < k; ++j) acc -= M[(size_t)i * k + j] * y[j];
        const cd piv = M[(size_t)i * k + i];
        y[i] = std::abs(piv) > 0.0 ? acc / piv : cd(0.0);
      }
      double nrm = 0.0;
      for (int i = 0; i < k; ++i) nrm += std::norm(y[i]);
      nrm = std::sqrt(nrm);
      if (!(nrm > 0.0) || !std::isfinite(nrm)) break;
      for (int i = 0; i < k; ++i) y[i] /= nrm;
    }
    res[t] = std::abs(hlast) * std::abs(y[k - 1]) / std::max(std::abs(th), 1e-300);
  }
}

// start vector: a fixed pseudo-random vector (splitmix64 of the index) in [-1, 1)
__global__ void k_start_vector(long long n, double* __restrict__ v) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned long long z = (unsigned long long)i + 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  z ^= z >> 31;
  v[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

size_t ritz_workspace_bytes(long long n_vol, long long n_phi, long long n_face, int k, int inner_m) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t nv = std::max<long long>(n_vol, 1);
  return al(sizeof(double) * n_phi) * 2 + al(sizeof(double) * std::max<long long>(n_face, 1)) +
         al(sizeof(double) * nv) + al(sizeof(int32_t) * nv) + al(sizeof(double) * nv * (k + 1)) +
         al(sizeof(double) * kDotBlocks * (k + 2)) + al(sizeof(double) * coef_words(k)) +
         (inner_m > 0 ? solve_workspace_bytes(n_vol, n_phi, n_face, inner_m) : 0);
}

int ritz_values(const SolveOp& op, int G, const int64_t* phi_off, const int64_t* vol_off, int mode, int k,
                double inner_rtol, int inner_m, int inner_max, double* ritz_re, double* ritz_im, double* ritz_res,
                double* hess, int* n_out, char* ws, size_t ws_bytes) {
  const long long n = op.n_vol;
  if (ws_bytes < ritz_workspace_bytes(n, op.n_phi, op.n_face, k, mode == 1 ? inner_m : 0))
    return fail(CUTCELL_E_WORKSPACE, "Ritz workspace too small");
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  size_t off = 0;
  auto take = [&](size_t bytes) { char* p = ws + off; off += al(bytes); return p; };
  const size_t nv = std::max<long long>(n, 1);
  double* zero_bc = (double*)take(sizeof(double) * op.n_phi);   // Phi = 0 (the inner solves' data)
  double* phi0 = (double*)take(sizeof(double) * op.n_phi);      // [v | 0]
  double* flux = (double*)take(sizeof(double) * std::max<long long>(op.n_face, 1));
  double* w = (double*)take(sizeof(double) * nv);
  int32_t* vphi = (int32_t*)take(sizeof(int32_t) * nv);
  double* V = (double*)take(sizeof(double) * nv * (k + 1));
  double* partial = (double*)take(sizeof(double) * kDotBlocks * (k + 2));
  double* cbuf = (double*)take(sizeof(double) * coef_words(k));
  char* inner_ws = ws + off;
  double* c1 = cbuf;
  double* c2 = cbuf + (k + 1);
  double* hnb = cbuf + (k + 1) + (k + 2);
  std::vector<double> hc(coef_words(k));
  hipStream_t st = op.st;
  const int T = 256;
  const unsigned gv = nb(n, T);
  auto mdot = [&](int kk, int self, const double* y, double* out) {
    hipLaunchKernelGGL(k_mdot, dim3(kDotBlocks), dim3(kDotBlock), 0, st, n, kk, self, V, y, partial);
    hipLaunchKernelGGL(k_mdot_final, dim3(kk + self), dim3(kDotBlock), 0, st, partial, out);
  };
  hipLaunchKernelGGL(k_vol_phi, dim3(gv), dim3(T), 0, st, n, G, phi_off, vol_off, vphi);
  hipLaunchKernelGGL(k_fill_f64, dim3(nb(op.n_phi, T)), dim3(T), 0, st, phi0, op.n_phi, 0.0);
  hipLaunchKernelGGL(k_fill_f64, dim3(nb(op.n_phi, T)), dim3(T), 0, st, zero_bc, op.n_phi, 0.0);
  hipLaunchKernelGGL(k_start_vector, dim3(gv), dim3(T), 0, st, n, V);
  double n2 = 0.0;
  mdot(0, 1, V, hnb);
  CC_HIP(hipMemcpyAsync(&n2, hnb, sizeof(double), hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  hipLaunchKernelGGL(k_axpby, dim3(gv), dim3(T), 0, st, n, 1.0 / std::sqrt(n2), V, 0.0, V, V);
  std::vector<double> Hm((size_t)(k + 1) * k, 0.0);
  int kk = k, inner_fail = 0;
  for (int j = 0; j < k; ++j) {
    double* vj = V + (long long)j * n;
    double* vn = V + (long long)(j + 1) * n;
    if (mode == 0) {
      hipLaunchKernelGGL(k_scatter, dim3(gv), dim3(T), 0, st, n, vphi, vj, phi0);
      int rc = op.lap_ptr ? apply_laplacian(op.D, n, op.lap_ptr, op.lap_col, op.lap_val, phi0, w, st)
                          : apply_operator(op.D, op.n_face, n, op.row_ptr, op.col, op.val, op.vol_face,
                                           op.vol_scale, phi0, w, flux, nullptr, st);
      if (rc) return rc;
    } else {
      hipLaunchKernelGGL(k_fill_f64, dim3(gv), dim3(T), 0, st, w, n, 0.0);
      int it = 0;
      double rr = 0.0;
      const int rc = solve_poisson(op, G, phi_off, vol_off, zero_bc, vj, w, inner_m, inner_max, inner_rtol, inner_ws,
                                   solve_workspace_bytes(n, op.n_phi, op.n_face, inner_m), &it, &rr);
      if (rc == CUTCELL_W_NOT_CONVERGED) inner_fail = 1;
      else if (rc) return rc;
    }
    mdot(j + 1, 0, w, c1);
    hipLaunchKernelGGL(k_maxpy, dim3(gv), dim3(T), 0, st, n, j + 1, c1, V, w);
    mdot(j + 1, 1, w, c2);
    hipLaunchKernelGGL(k_maxpy, dim3(gv), dim3(T), 0, st, n, j + 1, c2, V, w);
    hipLaunchKernelGGL(k_norm_after, dim3(1), dim3(1), 0, st, c2, j + 1, hnb);
    hipLaunchKernelGGL(k_scale_dev, dim3(gv), dim3(T), 0, st, n, w, hnb, vn);
    CC_HIP(hipMemcpyAsync(hc.data(), cbuf, sizeof(double) * coef_words(k), hipMemcpyDeviceToHost, st));
    CC_HIP(hipStreamSynchronize(st));
    for (int i = 0; i <= j; ++i) Hm[(size_t)i * k + j] = hc[i] + hc[(k + 1) + i];
    const double hn = hc[(k + 1) + (k + 2)];
    Hm[(size_t)(j + 1) * k + j] = hn;
    if (!(hn > 0.0)) {       // invariant subspace: its eigenvalues are exact
      kk = j + 1;
      break;
    }
  }
  CC_HIP(hipGetLastError());
  if (hess)
    for (size_t i = 0; i < Hm.size(); ++i) hess[i] = Hm[i];
  if (hessenberg_eigs(kk, Hm.data(), k, ritz_re, ritz_im)) return fail(CUTCELL_E_BREAKDOWN, "Hessenberg QR did not converge");
  if (ritz_res) ritz_residuals(kk, Hm.data(), k, kk < k ? 0.0 : Hm[(size_t)kk * k + (kk - 1)], ritz_re, ritz_im, ritz_res);
  if (mode == 1)                // eigenvalues of A^-1: invert
    for (int i = 0; i < kk; ++i) {
      const double a = ritz_re[i], b = ritz_im[i], d = a * a + b * b;
      ritz_re[i] = d > 0.0 ? a / d : 0.0;
      ritz_im[i] = d > 0.0 ? -b / d : 0.0;
    }
  *n_out = kk;
  return inner_fail ? CUTCELL_W_NOT_CONVERGED : CUTCELL_OK;
}

}  // namespace cutcell
