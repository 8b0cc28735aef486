// Householder QR path of the per-face stencils (Sec. 2.2.1, eq. 'stencil equation
// solution'; rows, centring and weights of Sec. 2.4), for the faces the Gram path cannot
// resolve to the stencil tolerance: an equilibrated pivot ratio below kRouteTol, or a
// refinement that has not settled (k_stencil routes them here), and every face when the
// caller asks for this factorisation.
//
// One wavefront owns one face; the factors live in shared memory, the exact B in a slot of
// the workspace:
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
//   5. val = h^(D-2) W z; status RANK_DEFICIENT when min|R_kk| <= kRankTol max|R_kk|.
#pragma once

#include "stencil_impl.hpp"

namespace cutcell {

constexpr int kQrRefine = 6;

// ---- wave reductions --------------------------------------------------------------------
// Within each row of 16 lanes by DPP moves (quad swaps, then the 8- and 16-lane mirrors),
// which leave every lane of the row with the same partial result; then the four row
// results in lane order.  Every lane returns the same value, in a fixed order.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum_f64(double v) {
  v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);   // row_half_mirror
  v += dpp_f64<0x140>(v);   // row_mirror
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}
__device__ __forceinline__ double wave_max_f64(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)), fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

template <int D, int Q>
struct QrSmem {
  static constexpr int M = Dims<D, Q>::M, MS = Dims<D, Q>::MS, M1 = Dims<D, Q>::M1;
  double Bq[kMaxRows * MS];   // Householder factors: R on and above the diagonal, v below
  double part[64];            // partial dot products of one step
  double wv[M];               // dot products of the pivot column with the trailing columns
  double tau[M];
  double rdiag[M];            // 1 / R_kk
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
    const double ak = readlane_f64(x, k) * sm.rdiag[k];
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
    const double yk = readlane_f64(x, k) * sm.rdiag[k];
    if (lane == k) x = yk;
    else if (lane < k) x = fma(-sm.Bq[lane * MS + k], yk, x);
  }
  return x;
}

template <int D, int Q, bool NEU>
__device__ void qr_face(const StencilArgs& A, int32_t F, QrSmem<D, Q>& sm, double* __restrict__ Bh,
                        double* __restrict__ Bl, int lane, double* __restrict__ val, int8_t* __restrict__ status,
                        int32_t* flagged) {
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
        Bh[r * MS + I] = m[I].hi;
        Bl[r * MS + I] = m[I].lo;
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
    for (int r = 0; r < N; ++r) c2 = fma(Bh[r * MS + lane], Bh[r * MS + lane], c2);
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
        const double h = Bh[r * MS + I] * s;
        Bh[r * MS + I] = h;
        Bl[r * MS + I] *= s;
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
      double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;   // four chains keep loads in flight
      if (act) {
        int r = k + 1 + g;
        for (; r + 3 * G < N; r += 4 * G) {
          p0 = fma(sm.Bq[r * MS + k], sm.Bq[r * MS + j], p0);
          p1 = fma(sm.Bq[(r + G) * MS + k], sm.Bq[(r + G) * MS + j], p1);
          p2 = fma(sm.Bq[(r + 2 * G) * MS + k], sm.Bq[(r + 2 * G) * MS + j], p2);
          p3 = fma(sm.Bq[(r + 3 * G) * MS + k], sm.Bq[(r + 3 * G) * MS + j], p3);
        }
        for (; r < N; r += G) p0 = fma(sm.Bq[r * MS + k], sm.Bq[r * MS + j], p0);
      }
      sm.part[lane] = (p0 + p1) + (p2 + p3);
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
        int r = k + g;
        for (; r + 3 * G < N; r += 4 * G) {   // four rows: every load before any store
          double x[4], c[4];
          static_for<0, 4>([&](auto U) {
            x[U] = sm.Bq[(r + U * G) * MS + k];
            c[U] = sm.Bq[(r + U * G) * MS + j];
          });
          static_for<0, 4>([&](auto U) {
            const int rr = r + U * G;
            const double vr = (rr == k) ? 1.0 : x[U] * inv;
            if (j > k) sm.Bq[rr * MS + j] = fma(-tsj, vr, c[U]);
            else sm.Bq[rr * MS + k] = (rr == k) ? beta : vr;
          });
        }
        for (; r < N; r += G) {
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
    if (!(rmin > kRankTol * rmax)) st = CUTCELL_STATUS_RANK_DEFICIENT;
    if (lane < M) sm.rdiag[lane] = 1.0 / sm.Bq[lane * MS + lane];
    __syncthreads();
  }

  // ---- minimum-norm solution by refinement of the augmented system -------------------------
  double zr[2] = {0.0, 0.0};
  double yl = 0.0;   // lane p: y_p
  if (st == CUTCELL_STATUS_OK) {
    for (int it = 0; it < kQrRefine; ++it) {
      // r1 = B y - z (rows) and r2 = F~ - B^T z (columns), with B = Bh + Bl: the Bh terms in
      // compensated arithmetic (Dot2, two chains), the Bl terms (below 2^-53 of them) plainly
      double r1[2] = {0.0, 0.0};
      static_for<0, 2>([&](auto R) {
        const int r = lane + 64 * R;
        Dot2 d0{-zr[R], 0.0}, d1{0.0, 0.0};
        double lo = 0.0;
        static_for<0, M>([&](auto P) {
          const double yp = readlane_f64(yl, P);
          if (r < N) {
            if constexpr (P % 2 == 0) dot2_add(d0, Bh[r * MS + P], yp);
            else dot2_add(d1, Bh[r * MS + P], yp);
            lo = fma(Bl[r * MS + P], yp, lo);
          }
        });
        r1[R] = (r < N) ? dot2_merge(d0, Dot2{d1.s, d1.c + lo}) : 0.0;
        if (r < N) sm.zs[r] = zr[R];
      });
      __syncthreads();
      double r2 = 0.0;
      if (lane < M) {
        Dot2 d0{fv.hi, fv.lo}, d1{0.0, 0.0};
        double lo = 0.0;
        int r = 0;
        for (; r + 1 < N; r += 2) {
          dot2_add(d0, -Bh[r * MS + lane], sm.zs[r]);
          dot2_add(d1, -Bh[(r + 1) * MS + lane], sm.zs[r + 1]);
          lo = fma(-Bl[r * MS + lane], sm.zs[r], lo);
          lo = fma(-Bl[(r + 1) * MS + lane], sm.zs[r + 1], lo);
        }
        if (r < N) {
          dot2_add(d0, -Bh[r * MS + lane], sm.zs[r]);
          lo = fma(-Bl[r * MS + lane], sm.zs[r], lo);
        }
        r2 = dot2_merge(d0, Dot2{d1.s, d1.c + lo});
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
// workgroup of one wave in turn; the grid (at most kQrSlots workgroups) walks the list.
// Workgroup b keeps the exact B of its face (high and low parts, read only by the
// refinement residuals) in slot b of bslots, kMaxRows * MS doubles each; shared memory
// holds the factors, so that four faces fit on a CU.
template <int D, int Q, bool NEU>
__global__ __launch_bounds__(64) void k_stencil_qr(StencilArgs A, const int32_t* __restrict__ list,
                                                  const int32_t* __restrict__ count_dev, long long count_host,
                                                  double* __restrict__ bslots, double* __restrict__ val,
                                                  int8_t* __restrict__ status, int32_t* flagged) {
  constexpr int MS = Dims<D, Q>::MS;
  __shared__ QrSmem<D, Q> sm;
  double* Bh = bslots + (long long)blockIdx.x * 2 * kMaxRows * MS;
  double* Bl = Bh + kMaxRows * MS;
  const long long n = count_dev ? (long long)*count_dev : count_host;
  for (long long t = blockIdx.x; t < n; t += gridDim.x) {
    qr_face<D, Q, NEU>(A, list[t], sm, Bh, Bl, threadIdx.x, val, status, flagged);
    __syncthreads();   // the next face reuses the shared memory and the slot
  }
}

}  // namespace cutcell
