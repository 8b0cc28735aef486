// Householder QR path of the per-face stencils (Sec. 2.2.1, eq. 'stencil equation
// solution'; rows, centring and weights of Sec. 2.4), for the faces the Gram path cannot
// resolve to the stencil tolerance: an equilibrated pivot ratio below kRouteTol, or a
// refinement that has not settled (k_stencil routes them here), and every face when the
// caller asks for this factorisation.
//
// One wavefront owns one face, B lives in shared memory:
//   1. rows in double-double: the offsets (x_i - x0)/h (exact half-integers for grid and
//      box faces; for an EB face x0 = cell centre + first moments / zeroth moment), the
//      binomial re-centring and the division by the zeroth moment carry ~106 bits, so B
//      = W A~ and F~ are known to far below FP64 rounding; the weights stay FP64 (an
//      error in W moves the stencil by about as much, whatever the conditioning);
//   2. columns scaled by powers of two to unit 2-norm (exact);
//   3. Householder QR of the FP64 part of B in place (LAPACK conventions): at step k the
//      dot products of the pivot column with every trailing column are split over the
//      wave, a group of lanes per column, and the update runs on the same layout;
//   4. the minimum-norm solution of B^T z = F~ by Bjorck's refinement of the augmented
//      system [I B; B^T 0]: the residuals r1 = B y - z and r2 = F~ - B^T z in
//      double-double from the stored B, the corrections from the FP64 factors
//      (g = Q^T r1, a = R^-T r2, dy = R^-1 (a - g1), dz = Q [a; g2]), repeated until the
//      correction no longer changes z (at most kQrRefine times).  With residuals this
//      accurate the iteration converges to z rounded to FP64 as long as cond(B) eps < 1.
//   5. val = h^(D-2) W z; status RANK_DEFICIENT when min|R_kk| <= kQrRankTol max|R_kk|.
#pragma once

#include "stencil_impl.hpp"

namespace cutcell {

constexpr double kQrRankTol = 1e-12;
constexpr int kQrRefine = 6;

// ---- wave reductions (butterfly: every lane ends with the same, fixed-order result) -------
__device__ __forceinline__ double wave_sum_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

template <int D, int Q>
struct QrSmem {
  static constexpr int M = Dims<D, Q>::M, MS = Dims<D, Q>::MS, M1 = Dims<D, Q>::M1;
  double Bq[kMaxRows * MS];   // Householder factors: R on and above the diagonal, v below
  double Bh[kMaxRows * MS];   // B = W A~ (columns scaled), high parts
  double Bl[kMaxRows * MS];   //                             low parts
  double part[64];            // partial dot products of one step
  double wv[M];               // dot products of the pivot column with the trailing columns
  double tau[M];
  double colsc[M];            // column scales (powers of two)
  double zs[kMaxRows];        // z, for B^T z
  double nuh[D][M1];          // EB normal moments about x0, high and low parts
  double nul[D][M1];
};

// Face of global index F (as face_info, for a face given by index).
__device__ __forceinline__ FaceInfo face_info_of(const StencilArgs& A, int32_t F) {
  FaceInfo fi;
  fi.F = F;
  const int32_t code = A.fcode[F];
  fi.gi = code >> 4;
  fi.kind = (code >> 2) & 3;
  fi.dn = code & 3;
  fi.ref = A.fref[F];
  fi.n_vol = A.counts[4 * fi.gi + 0];
  fi.n_eb = A.counts[4 * fi.gi + 1];
  fi.phi0 = A.offs[fi.gi];
  fi.rp = A.row_ptr[F];
  fi.N = (int)(A.row_ptr[F + 1] - fi.rp);
  return fi;
}

// t <- H_k t, t in the row layout (lane r holds rows r, r + 64)
template <int D, int Q>
__device__ __forceinline__ void apply_reflector(const QrSmem<D, Q>& sm, int k, int N, int lane, double* t) {
  constexpr int MS = Dims<D, Q>::MS;
  double part = 0.0;
  static_for<0, 2>([&](auto R) {
    const int r = lane + 64 * R;
    if (r >= k && r < N) part = fma(r == k ? 1.0 : sm.Bq[r * MS + k], t[R], part);
  });
  const double td = sm.tau[k] * wave_sum_f64(part);
  static_for<0, 2>([&](auto R) {
    const int r = lane + 64 * R;
    if (r >= k && r < N) t[R] = fma(-td, r == k ? 1.0 : sm.Bq[r * MS + k], t[R]);
  });
}

// x (lane p < M) <- R^-T x  (forward substitution; R^T is lower triangular)
template <int D, int Q>
__device__ __forceinline__ double solve_rt(const QrSmem<D, Q>& sm, int lane, double x) {
  constexpr int M = Dims<D, Q>::M, MS = Dims<D, Q>::MS;
  for (int k = 0; k < M; ++k) {
    const double ak = readlane_f64(x, k) / sm.Bq[k * MS + k];
    if (lane == k) x = ak;
    else if (lane > k && lane < M) x = fma(-sm.Bq[k * MS + lane], ak, x);
  }
  return x;
}

// x (lane p < M) <- R^-1 x  (back substitution)
template <int D, int Q>
__device__ __forceinline__ double solve_r(const QrSmem<D, Q>& sm, int lane, double x) {
  constexpr int M = Dims<D, Q>::M, MS = Dims<D, Q>::MS;
  for (int k = M - 1; k >= 0; --k) {
    const double yk = readlane_f64(x, k) / sm.Bq[k * MS + k];
    if (lane == k) x = yk;
    else if (lane < k) x = fma(-sm.Bq[lane * MS + k], yk, x);
  }
  return x;
}

template <int D, int Q, bool NEU>
__device__ void qr_face(const StencilArgs& A, int32_t F, QrSmem<D, Q>& sm, int lane, double* __restrict__ val,
                        int8_t* __restrict__ status, int32_t* flagged) {
  using DM = Dims<D, Q>;
  constexpr int M = DM::M, MS = DM::MS, M1 = DM::M1;
  FaceInfo fi = face_info_of(A, F);
  const GeomPtrs gp = A.geoms[fi.gi];
  face_x0<D, Q>(A.g, gp, fi);
  dd x0[3];
  face_x0_dd<D, Q>(A.g, gp, fi, x0);
  const int N = fi.N;
  const int32_t* vol_cell = A.vol_cell_ws + (long long)fi.gi * A.g.ncell;
  const int32_t* box_lf = A.box_lf_ws + (long long)fi.gi * A.g.nboxslot;

  // ---- rows and flux vector in double-double --------------------------------------------
  bool finite = true;
  double wreg[2] = {0.0, 0.0};
  static_for<0, 2>([&](auto R) {
    const int r = lane + 64 * R;
    if (r < N) {
      const RowSource rs = row_source<D, Q>(A.g, gp, (int64_t)A.col[fi.rp + r] - fi.phi0, fi.n_vol, fi.n_eb,
                                            vol_cell, box_lf);
      dd m[M];
      double w;
      finite = dd_row<D, Q, NEU>(gp, rs, x0, A.wpow, m, w) && finite;
      wreg[R] = w;
      static_for<0, M>([&](auto I) {
        sm.Bh[r * MS + I] = m[I].hi;
        sm.Bl[r * MS + I] = m[I].lo;
      });
    }
  });
  dd fv = dd_from(0.0);
  if (fi.kind == 0) {
    const double* fm = A.geoms[fi.gi].face_mom[fi.dn] + (fi.ref - A.g.foff[fi.dn]) * DM::Mf;
    if (lane < M) {
      constexpr auto& T = kMono<D, Q>;
      const int dn = fi.dn;
      const int e0 = T.e[lane][0], e1 = T.e[lane][1], e2 = T.e[lane][2];
      const int pd = (dn == 0) ? e0 : (dn == 1 ? e1 : e2);
      if (pd == 1) {
        int s;
        if (D == 2) s = mono_index<1>(dn == 0 ? e1 : e0, 0, 0);
        else if (dn == 0) s = mono_index<2>(e1, e2, 0);
        else if (dn == 1) s = mono_index<2>(e0, e2, 0);
        else s = mono_index<2>(e0, e1, 0);
        fv = dd_from(fm[s]);
      }
    }
  } else {
    if (lane < D) {
      dd nu[M1];
      const double* src = gp.eb_nmom + ((long long)fi.ref * D + lane) * M1;
      static_for<0, M1>([&](auto I) { nu[I] = dd_from(src[I]); });
      const int32_t c = fi.owner_cell;
      const int cown[3] = {(int)(c % A.g.n[0]), (int)((c / A.g.n[0]) % A.g.n[1]),
                           (int)(c / ((long long)A.g.n[0] * A.g.n[1]))};
      dd dl[3];
      for (int ax = 0; ax < 3; ++ax) dl[ax] = dd_from(0.0);
      for (int ax = 0; ax < D; ++ax) dl[ax] = dd_sub(dd_from(cown[ax] + 0.5), x0[ax]);   // (c - x0)/h
      recentre_dd<D, Q - 1>(nu, dl);
      static_for<0, M1>([&](auto I) {
        sm.nuh[lane][I] = nu[I].hi;
        sm.nul[lane][I] = nu[I].lo;
      });
    }
    __syncthreads();
    if (lane < M) {
      constexpr auto& T = kMono<D, Q>;
      for (int ax = 0; ax < D; ++ax) {
        int e[3] = {T.e[lane][0], T.e[lane][1], T.e[lane][2]};
        const int p = e[ax];
        if (p > 0) {
          e[ax] -= 1;
          const int j = mono_index<D>(e[0], e[1], e[2]);
          fv = dd_add(fv, dd_mul_d(dd{sm.nuh[ax][j], sm.nul[ax][j]}, (double)p));
        }
      }
    }
  }
  finite = __all(finite) && __all(dd_isfinite(fv));
  __syncthreads();

  // ---- column scales: powers of two bringing every column to 2-norm in [1, 2) -------------
  bool zero_col = false;
  if (lane < M) {
    double c2 = 0.0;
    for (int r = 0; r < N; ++r) c2 = fma(sm.Bh[r * MS + lane], sm.Bh[r * MS + lane], c2);
    zero_col = !(c2 > 0.0);
    sm.colsc[lane] = (c2 > 0.0 && isfinite(c2)) ? ldexp(1.0, -ilogb(sqrt(c2))) : 1.0;
  }
  zero_col = __any(zero_col);
  __syncthreads();
  if (lane < M) {
    const double s = sm.colsc[lane];
    fv.hi *= s;
    fv.lo *= s;
  }
  static_for<0, 2>([&](auto R) {
    const int r = lane + 64 * R;
    if (r < N) {
      static_for<0, M>([&](auto I) {
        const double s = sm.colsc[I];
        const double h = sm.Bh[r * MS + I] * s;
        sm.Bh[r * MS + I] = h;
        sm.Bl[r * MS + I] *= s;
        sm.Bq[r * MS + I] = h;
      });
    }
  });
  __syncthreads();

  int st = CUTCELL_STATUS_OK;
  if (!finite) st = CUTCELL_STATUS_NONFINITE;
  else if (zero_col) st = CUTCELL_STATUS_RANK_DEFICIENT;

  // ---- Householder QR of the FP64 part, in place ------------------------------------------
  double rmax = 0.0, rmin = 1e300;
  if (st == CUTCELL_STATUS_OK) {
    for (int k = 0; k < M; ++k) {
      const int m = M - k;                      // columns k..M-1
      const int G = (64 / m > 0) ? 64 / m : 1;  // lanes per column
      const int jj = lane / G, g = lane - jj * G;
      const bool act = jj < m;
      const int j = k + jj;
      double part = 0.0;
      if (act)
        for (int r = k + 1 + g; r < N; r += G) part = fma(sm.Bq[r * MS + k], sm.Bq[r * MS + j], part);
      sm.part[lane] = part;
      __syncthreads();
      if (act && g == 0) {
        double s = 0.0;
        for (int q = 0; q < G; ++q) s += sm.part[lane + q];
        sm.wv[j] = s;
      }
      __syncthreads();
      const double alpha = sm.Bq[k * MS + k];
      const double sigma2 = sm.wv[k];
      double beta = alpha, tau = 0.0, inv = 0.0;
      if (sigma2 != 0.0) {
        beta = -copysign(sqrt(fma(alpha, alpha, sigma2)), alpha);
        tau = (beta - alpha) / beta;
        inv = 1.0 / (alpha - beta);
      }
      if (act) {
        // v^T C_j = C_kj + inv * (x below k)^T C_j;  C_rj -= tau v_r (v^T C_j)
        const double tsj = (j > k) ? tau * fma(sm.wv[j], inv, sm.Bq[k * MS + j]) : 0.0;
        for (int r = k + g; r < N; r += G) {
          const double vr = (r == k) ? 1.0 : sm.Bq[r * MS + k] * inv;
          if (j > k) sm.Bq[r * MS + j] = fma(-tsj, vr, sm.Bq[r * MS + j]);
          else sm.Bq[r * MS + k] = (r == k) ? beta : vr;
        }
      }
      if (lane == 0) sm.tau[k] = tau;
      rmax = fmax(rmax, fabs(beta));
      rmin = fmin(rmin, fabs(beta));
      __syncthreads();
    }
    if (!(rmin > kQrRankTol * rmax)) st = CUTCELL_STATUS_RANK_DEFICIENT;
  }

  // ---- minimum-norm solution by refinement of the augmented system -------------------------
  double zr[2] = {0.0, 0.0};
  double yl = 0.0;   // lane p: y_p
  if (st == CUTCELL_STATUS_OK) {
    for (int it = 0; it < kQrRefine; ++it) {
      // r1 = B y - z (rows) and r2 = F~ - B^T z (columns), in double-double
      double r1[2] = {0.0, 0.0};
      static_for<0, 2>([&](auto R) {
        const int r = lane + 64 * R;
        dd acc = dd_from(-zr[R]);
        static_for<0, M>([&](auto P) {
          const double yp = readlane_f64(yl, P);
          if (r < N) acc = dd_add(acc, dd_mul_d(dd{sm.Bh[r * MS + P], sm.Bl[r * MS + P]}, yp));
        });
        r1[R] = (r < N) ? acc.hi : 0.0;
        if (r < N) sm.zs[r] = zr[R];
      });
      __syncthreads();
      double r2 = 0.0;
      if (lane < M) {
        dd acc = fv;
        for (int r = 0; r < N; ++r)
          acc = dd_sub(acc, dd_mul_d(dd{sm.Bh[r * MS + lane], sm.Bl[r * MS + lane]}, sm.zs[r]));
        r2 = acc.hi;
      }
      __syncthreads();
      // g = Q^T r1;  a = R^-T r2;  dy = R^-1 (a - g1);  dz = Q [a; g2]
      double gr[2] = {r1[0], r1[1]};
      for (int k = 0; k < M; ++k) apply_reflector<D, Q>(sm, k, N, lane, gr);
      const double a = (lane < M) ? solve_rt<D, Q>(sm, lane, r2) : 0.0;
      const double c = solve_r<D, Q>(sm, lane, (lane < M) ? a - gr[0] : 0.0);
      double tz[2] = {(lane < M) ? a : gr[0], gr[1]};
      for (int k = M - 1; k >= 0; --k) apply_reflector<D, Q>(sm, k, N, lane, tz);
      double dmax = 0.0, zmax = 0.0;
      static_for<0, 2>([&](auto R) {
        const int r = lane + 64 * R;
        if (r < N) {
          zr[R] += tz[R];
          dmax = fmax(dmax, fabs(tz[R]));
          zmax = fmax(zmax, fabs(zr[R]));
        }
      });
      if (lane < M) yl += c;
      dmax = wave_max_f64(dmax);
      zmax = wave_max_f64(zmax);
      if (!(dmax > 0x1p-52 * zmax)) break;
    }
  }

  static_for<0, 2>([&](auto R) {
    const int r = lane + 64 * R;
    if (r < N) {
      double v = (st == CUTCELL_STATUS_OK) ? A.hscale * wreg[R] * zr[R] : 0.0;
      if constexpr (NEU) {
        const int64_t k = (int64_t)A.col[fi.rp + r] - fi.phi0;
        if (k >= fi.n_vol && k < fi.n_vol + fi.n_eb) v *= A.h;
      }
      val[fi.rp + r] = v;
    }
  });
  if (lane == 0) {
    status[fi.F] = (int8_t)st;
    if (st != CUTCELL_STATUS_OK) atomicAdd(flagged, 1);
  }
}

// The faces list[0 .. n) (n from the device when count_dev is given), each by one
// workgroup of one wave in turn; the grid walks the list.
template <int D, int Q, bool NEU>
__global__ __launch_bounds__(64) void k_stencil_qr(StencilArgs A, const int32_t* __restrict__ list,
                                                  const int32_t* __restrict__ count_dev, long long count_host,
                                                  double* __restrict__ val, int8_t* __restrict__ status,
                                                  int32_t* flagged) {
  __shared__ QrSmem<D, Q> sm;
  const long long n = count_dev ? (long long)*count_dev : count_host;
  for (long long t = blockIdx.x; t < n; t += gridDim.x) {
    qr_face<D, Q, NEU>(A, list[t], sm, threadIdx.x, val, status, flagged);
    __syncthreads();   // the next face reuses the shared memory
  }
}

}  // namespace cutcell
