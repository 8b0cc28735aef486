// Per-face weighted least-squares flux stencils (Sec. 2.2.1, eq. 'stencil equation
// solution'; neighbours, centring and weights of Sec. 2.4).
//
// The stencil s~ = W (A~^T W)^+ F~ is W z with z the minimum-norm solution of
// B^T z = F~, B = W A~ (N x M, N >= M, full column rank): z = B (B^T B)^-1 F~.  One
// wavefront owns one face:
//   1. rows: each lane builds its row(s) of B in registers -- the row's moments,
//      re-centred to x0 by the binomial theorem, divided by the zeroth moment and
//      scaled by the weight -- and stores them in LDS; a row whose zeroth moment is
//      below kSmallCell is formed in double-double and rounded (the moments of a small
//      cut cell about its centre nearly cancel when shifted to x0);
//   2. G = B^T B on the FP64 matrix cores (v_mfma_f64_16x16x4f64, 16 x 16 tiles, rows
//      of B as the contraction index); lane i collects row i from the tiles with
//      ds_bpermute (no shared-memory copy of G);
//   3. G is equilibrated to unit diagonal and inverted by symmetric Gauss-Jordan sweeps,
//      lane i holding row i in registers; the sweep pivots are the Cholesky pivots;
//   4. z from the semi-normal equations z = B G^-1 F~ followed by one step of refinement
//      with the residual F~ - B^T z computed from B itself in compensated arithmetic
//      (twice the working precision), which leaves the error of rounding B to FP64, a few
//      1e-17 cond(B), where the initial error is ~cond(B)^2 eps;
//   5. val = h^(D-2) W z.
// Under Neumann EB conditions (a separate kernel instance) the EB rows are the
// normal-derivative rows of eq. 'Neu moment eq for cp' and their values carry h^(D-1);
// the EB faces themselves have a one-entry stencil (their area) and are written by
// k_insufficient, the kernel of faces with fewer rows than monomials.
// Status: fewer rows than monomials or a non-finite entry flag the face.  A face is left to
// the Householder QR path (stencil_qr.hpp), which also decides rank deficiency, when
//   * its condition bound sqrt(||G^||_inf ||G^^-1||_F) (>= cond_2 of the equilibrated B,
//     and within 1.35x of it on the workloads) exceeds kCondRoute: with the rows of small
//     cells formed in double-double (below) the stencil is good to about 1.5e-16 cond,
//     which must stay below the 1e-11 it is held to;
//   * its smallest pivot square root is at most kRouteTol times the largest; or
//   * its refinement step moved the stencil by more than kSettleTol of its size (the error
//     left after the step is about the square of that fraction).
#pragma once

#include <algorithm>

#include "kernels.hpp"
#include "rows.hpp"
#include "rows_dd.hpp"

namespace cutcell {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr double kRouteTol = 1e-4;
constexpr double kRankTol = 1e-12;       // rank deficiency: min |R_kk| <= kRankTol max |R_kk|
constexpr double kCondRoute = 3e4;
constexpr double kSmallCell = 1e-3;      // rows (and EB flux vectors) of smaller cells in double-double
constexpr double kSettleTol = 1e-6;
// Faces whose bound on cond(G^) stays below this (cond(B) below about 3e3) refine in
// plain FP64.  Past it, z = B y and the residuals are summed in compensated arithmetic and
// z is kept as a double-double: the rounding of an FP64 product B y leaves in z a part
// outside the range of B, which the residual cannot see and refinement cannot remove,
// of relative size up to about cond(B) eps (4e-12 at cond(B) = 3e4, the routing bound).
constexpr double kDot2Cond = 1e7;
constexpr int kRefine = 1;
constexpr int kRefineBackward = 2;   // refinement steps of the adjoint's least-squares solve
constexpr int kStatusRoute = 100;        // internal: the face goes to the QR path

// Compensated dot product (Ogita, Rump and Oishi, SIAM J. Sci. Comput. 26(6), 2005,
// algorithm Dot2): s + c holds the running sum as if it were carried in twice the working
// precision.  The product's rounding error comes from the FMA, the sum's from TwoSum.
struct Dot2 {
  double s, c;
};
__device__ __forceinline__ void dot2_add(Dot2& a, double x, double y) {
#pragma clang fp contract(off)
  const double p = x * y;
  const double e = __builtin_fma(x, y, -p);
  const double s = a.s + p;
  const double bb = s - a.s;
  const double q = (a.s - (s - bb)) + (p - bb);
  a.s = s;
  a.c += q + e;
}
// a + b as an unevaluated sum s + c
__device__ __forceinline__ Dot2 dot2_join(Dot2 a, Dot2 b) {
#pragma clang fp contract(off)
  const double s = a.s + b.s;
  const double bb = s - a.s;
  const double q = (a.s - (s - bb)) + (b.s - bb);
  return Dot2{s, (a.c + b.c) + q};
}
__device__ __forceinline__ double dot2_merge(Dot2 a, Dot2 b) {
#pragma clang fp contract(off)
  const double s = a.s + b.s;
  const double bb = s - a.s;
  const double q = (a.s - (s - bb)) + (b.s - bb);
  return s + ((a.c + b.c) + q);
}

// 1/d from v_rcp_f64 and two Newton steps (each squares the relative error)
__device__ __forceinline__ double recip_f64(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}


// One row of B = W A~ about x0 (in units of h: x0h = x0 / h) from the row's stored
// moments m (overwritten) and centre; returns its weight in w, and false if the row
// holds a non-finite value.
template <int D, int Q>
__device__ __forceinline__ bool finish_row(const double* ctr, const double* x0h, double* m, double& w, double wpow) {
  constexpr int M = Dims<D, Q>::M;
  double delta[3] = {0, 0, 0};
  double d2 = 0;
  for (int ax = 0; ax < D; ++ax) {
    delta[ax] = ctr[ax] - x0h[ax];
    d2 += delta[ax] * delta[ax];
  }
  w = row_weight(d2, wpow);
  const double mu0 = m[0];
  recentre<D, Q>(m, delta);
  const double sc = w / mu0;
  bool finite = isfinite(sc);
  static_for<0, M>([&](auto I) {
    m[I] *= sc;
    finite = finite && isfinite(m[I]);
  });
  return finite;
}

// Neumann row of EB face e about x0 (eq. 'Neu moment eq for cp'): the flux of each
// monomial xi^p through the face, sum_d p_d nu_d^(p - e_d)(x0), over the face area m^0,
// times the row's weight.  The normal moments are stored about the cut cell's centre
// `ctr` and re-centred to x0 like the other rows.  Returns false on a non-finite value.
template <int D, int Q>
__device__ __forceinline__ bool neumann_row(const GeomPtrs& gp, int32_t e, const double* ctr, const double* x0h,
                                            double* m, double& w, double wpow) {
  constexpr int M = Dims<D, Q>::M, M1 = Dims<D, Q>::M1;
  double delta[3] = {0, 0, 0};
  double d2 = 0;
  for (int ax = 0; ax < D; ++ax) {
    delta[ax] = ctr[ax] - x0h[ax];
    d2 += delta[ax] * delta[ax];
  }
  w = row_weight(d2, wpow);
  const double sc = w / gp.eb_mom[(long long)e * M];
  static_for<0, M>([&](auto I) { m[I] = 0.0; });
  static_for<0, D>([&](auto AX) {
    double nu[M1];
    const double* src = gp.eb_nmom + ((long long)e * D + AX) * M1;
    static_for<0, M1>([&](auto I) { nu[I] = src[I]; });
    recentre<D, Q - 1>(nu, delta);
    static_for<0, M>([&](auto I) {
      constexpr int pd = kMono<D, Q>.e[I][AX];
      if constexpr (pd > 0) {
        constexpr int j = mono_index<D>(kMono<D, Q>.e[I][0] - (AX == 0), kMono<D, Q>.e[I][1] - (AX == 1),
                                        kMono<D, Q>.e[I][2] - (AX == 2));
        m[I] = fma((double)pd, nu[j], m[I]);
      }
    });
  });
  bool finite = isfinite(sc);
  static_for<0, M>([&](auto I) {
    m[I] *= sc;
    finite = finite && isfinite(m[I]);
  });
  return finite;
}

// Columns of G beyond the full 16-wide tiles (at most 4, done on the vector ALUs).
template <int D, int Q>
struct GramSplit {
  static constexpr int M = Dims<D, Q>::M, MT = Dims<D, Q>::MT;
  static constexpr int MTF = (MT > 1 && M - 16 * (MT - 1) <= 4) ? MT - 1 : MT;   // tiles per side
  static constexpr int MV = M - 16 * MTF > 0 ? M - 16 * MTF : 0;                // trailing columns
};

// Shared memory of one face (one wave) in the forward kernel: B, and one buffer that holds
// in turn the EB normal moments, the trailing Gram columns and z.  Everything else a lane
// needs (W of its rows, its F~ entry, z of its rows) stays in registers.  On MI355X a
// wave of this kernel is latency-bound, so the bytes per wave set how many waves share a
// CU: 39.6 KB with a Gram buffer and W, F~ in shared memory, 27.7 KB like this (3D
// order 4, 96 rows).
template <int D, int Q, int NPAD>
struct LeanSmem {
  static constexpr bool kFull = false;
  static constexpr int M = Dims<D, Q>::M, MS = Dims<D, Q>::MS, M1 = Dims<D, Q>::M1;
  static constexpr int MV = GramSplit<D, Q>::MV;
  double Bs[NPAD * MS];      // rows of B = W A~
  union {
    struct {
      double zs[NPAD];                 // z = B y (refinement; the pivot row of the sweep)
      double zl[NPAD];                 // its low part where z is a double-double
    };
    double nus[D][M1];                 // EB normal moments about x0 (flux vector)
    double tt[M * (MV > 0 ? MV : 1)];  // trailing Gram columns (transposition)
  };
};

// Shared memory of one face in the adjoint kernel, which reads W, z, y and the normal
// moments again after the forward solve.
template <int D, int Q, int NPAD>
struct FaceSmem {
  static constexpr bool kFull = true;
  static constexpr int M = Dims<D, Q>::M, MS = Dims<D, Q>::MS, M1 = Dims<D, Q>::M1;
  static constexpr int MV = GramSplit<D, Q>::MV;
  double Bs[NPAD * MS];      // rows of B = W A~
  double tt[M * (MV > 0 ? MV : 1)];
  double gsum[M + 1];        // per-component sums of the adjoint
  double ys[M + 1];          // y = G^-1 F~
  double zs[NPAD];           // z = B y
  double zl[NPAD];           // its low part where z is a double-double
  double wls[NPAD];          // W
  double nus[D][M1];         // EB normal moments about x0
};

// 64-bit ds_bpermute: the value of v in lane src_lane
__device__ __forceinline__ double bpermute_f64(double v, int src_lane) {
  const int lo = __builtin_amdgcn_ds_bpermute(src_lane * 4, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src_lane * 4, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Everything about the face that the row and flux computations need.
struct FaceInfo {
  int32_t F;
  int gi, kind, dn;
  int32_t ref;
  int64_t n_vol, n_eb, phi0, rp;
  int N;
  double x0h[3];             // x0 / h
  double off[3];             // EB faces: centroid offset from the cut cell's centre (/h)
  int32_t owner_cell;        // EB faces: the cut cell
};

// x0 of the face (in units of h): the face centre, or for an EB face the centroid of its
// cut volume (whose offset from the cell centre is kept in fi.off).  Loads only.
template <int D, int Q>
__device__ __forceinline__ void face_x0(const GridDims& g, const GeomPtrs& gp, FaceInfo& fi) {
  constexpr int M = Dims<D, Q>::M;
  const int dn = fi.dn;
  for (int ax = 0; ax < 3; ++ax) { fi.x0h[ax] = 0.0; fi.off[ax] = 0.0; }
  fi.owner_cell = -1;
  if (fi.kind == 0) {
    const long long loc = fi.ref - g.foff[dn];
    const int m0 = g.n[0] + (dn == 0), m1 = g.n[1] + (dn == 1);
    const int j[3] = {(int)(loc % m0), (int)((loc / m0) % m1), (int)(loc / ((long long)m0 * m1))};
    for (int ax = 0; ax < D; ++ax) fi.x0h[ax] = (ax == dn) ? (double)j[ax] : j[ax] + 0.5;
    return;
  }
  const int32_t c = gp.eb_cell[fi.ref];
  fi.owner_cell = c;
  const int cown[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long long)g.n[0] * g.n[1]))};
  const double* vm = gp.vol_mom + (long long)c * M;
  const double k0 = vm[0];
  for (int ax = 0; ax < D; ++ax) {
    fi.off[ax] = vm[1 + ax] / k0;          // first moments: degree-1 monomials e_1..e_D
    fi.x0h[ax] = cown[ax] + 0.5 + fi.off[ax];
  }
}

// x0 / h in double-double: exact for grid and box faces; for an EB face the cut cell's
// centre plus its first moments over its zeroth moment (face_x0 must have run).
template <int D, int Q>
__device__ __forceinline__ void face_x0_dd(const GridDims& g, const GeomPtrs& gp, const FaceInfo& fi, dd* x0) {
  constexpr int M = Dims<D, Q>::M;
  for (int ax = 0; ax < 3; ++ax) x0[ax] = dd_from(fi.x0h[ax]);
  if (fi.kind == 0) return;
  const int32_t c = fi.owner_cell;
  const int cown[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long long)g.n[0] * g.n[1]))};
  const double* vm = gp.vol_mom + (long long)c * M;
  const dd k0 = dd_from(vm[0]);
  for (int ax = 0; ax < D; ++ax) x0[ax] = dd_add(dd_from(cown[ax] + 0.5), dd_div(dd_from(vm[1 + ax]), k0));
}

// Entry `lane` of the flux vector F~ (0 for lanes >= M) and, for EB faces, the normal
// moments re-centred to x0 (sm.nus, lanes 0..D-1 one component each).  Ends with a barrier.
template <int D, int Q, class SM>
__device__ __forceinline__ double face_flux(const GridDims& g, const GeomPtrs& gp, const FaceInfo& fi, SM& sm,
                                            int lane, const dd* x0dd) {
  constexpr int M = Dims<D, Q>::M, Mf = Dims<D, Q>::Mf, M1 = Dims<D, Q>::M1;
  const int dn = fi.dn;
  double fv = 0.0;
  if (fi.kind == 0) {
    // F~_p = face moment of p - e_d when p_d = 1 (reference normal +e_d)
    const double* fm = gp.face_mom[dn] + (fi.ref - g.foff[dn]) * Mf;
    if (lane < M) {
      constexpr auto& T = kMono<D, Q>;
      const int e0 = T.e[lane][0], e1 = T.e[lane][1], e2 = T.e[lane][2];
      const int pd = (dn == 0) ? e0 : (dn == 1 ? e1 : e2);
      if (pd == 1) {
        int s;
        if (D == 2) s = mono_index<1>(dn == 0 ? e1 : e0, 0, 0);
        else if (dn == 0) s = mono_index<2>(e1, e2, 0);
        else if (dn == 1) s = mono_index<2>(e0, e2, 0);
        else s = mono_index<2>(e0, e1, 0);
        fv = fm[s];
      }
    }
    __syncthreads();
    return fv;
  }
  const bool small = gp.vol_mom[(long long)fi.owner_cell * M] < kSmallCell;
  if (lane < D && !small) {
    double nu[M1];
    const double* src = gp.eb_nmom + ((long long)fi.ref * D + lane) * M1;
    static_for<0, M1>([&](auto I) { nu[I] = src[I]; });
    double dl[3] = {-fi.off[0], -fi.off[1], -fi.off[2]};   // (c - x0)/h
    recentre<D, Q - 1>(nu, dl);
    static_for<0, M1>([&](auto I) { sm.nus[lane][I] = nu[I]; });
  } else if (lane < D) {   // a small cut cell: the shift to its centroid in double-double
    dd nu[M1];
    const double* src = gp.eb_nmom + ((long long)fi.ref * D + lane) * M1;
    static_for<0, M1>([&](auto I) { nu[I] = dd_from(src[I]); });
    const int32_t c = fi.owner_cell;
    const int cown[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long long)g.n[0] * g.n[1]))};
    dd dl[3] = {dd_from(0.0), dd_from(0.0), dd_from(0.0)};
    for (int ax = 0; ax < D; ++ax) dl[ax] = dd_sub(dd_from(cown[ax] + 0.5), x0dd[ax]);   // (c - x0)/h
    recentre_dd<D, Q - 1>(nu, dl);
    static_for<0, M1>([&](auto I) { sm.nus[lane][I] = nu[I].hi + nu[I].lo; });
  }
  __syncthreads();
  if (lane < M) {
    constexpr auto& T = kMono<D, Q>;
    for (int ax = 0; ax < D; ++ax) {
      int e[3] = {T.e[lane][0], T.e[lane][1], T.e[lane][2]};
      const int p = e[ax];
      if (p > 0) {
        e[ax] -= 1;
        fv += p * sm.nus[ax][mono_index<D>(e[0], e[1], e[2])];
      }
    }
  }
  __syncthreads();
  return fv;
}

// Rows, Gram matrix, inverse and the refined semi-normal solve of one face.  Leaves B in
// shared memory, -G^^-1 (row `lane`) in a[], the column equilibration in sdiag, and W and
// z of rows lane, lane + 64, ... in wreg[], zreg[]; the adjoint's layout (SM::kFull) also
// keeps W, z and y in shared memory.  Returns the face status, or kStatusRoute.
template <int D, int Q, int NPAD, bool NEU, class SM>
__device__ __forceinline__ int face_forward(const GridDims& g, const GeomPtrs& gp, const FaceInfo& fi,
                                            const int32_t* __restrict__ vol_cell, const int32_t* __restrict__ box_lf,
                                            const int32_t* __restrict__ col, SM& sm, int lane, double* a,
                                            double& sdiag, double* wreg, double* zreg, double wpow,
                                            bool* rank_low = nullptr) {
  using DM = Dims<D, Q>;
  constexpr int M = DM::M, MS = DM::MS;
  static_assert(M < NPAD, "the sweep's pivot buffer (zs) needs a slot past M");
  double* Bs = sm.Bs;
  const int N = fi.N;

  // ---- rows of B ----------------------------------------------------------------------
  // Lane r builds rows r, r + 64, ...: every row's index chain (col -> cell -> moments) is
  // issued before the first row is finished, so the dependent loads of all rows overlap.
  constexpr int NR = (NPAD + 63) / 64;
  bool finite = true;
  dd x0dd[3];
  face_x0_dd<D, Q>(g, gp, fi, x0dd);
  RowSource rsrc[NR];
  static_for<0, NR>([&](auto R) {
    const int r = lane + 64 * R;
    if (r < N) rsrc[R] = row_source<D, Q>(g, gp, (int64_t)col[fi.rp + r] - fi.phi0, fi.n_vol, fi.n_eb, vol_cell,
                                          box_lf);
  });
  static_for<0, NR>([&](auto R) {
    const int r = lane + 64 * R;
    wreg[R] = 0.0;
    if (r < NPAD) {
      double m[M];
      double wr = 0.0;
      if (r < N) {
        const bool neu_row = NEU && rsrc[R].eb >= 0;
        const double m0 = neu_row ? gp.eb_mom[(long long)rsrc[R].eb * M] : rsrc[R].src[0];
        if (!(m0 >= kSmallCell)) {   // a small cell (or a non-finite moment): double-double
          dd md[M];
          finite = dd_row<D, Q, NEU>(gp, rsrc[R], x0dd, wpow, md, wr) && finite;
          static_for<0, M>([&](auto I) { m[I] = md[I].hi; });
        } else if (neu_row) {
          finite = neumann_row<D, Q>(gp, rsrc[R].eb, rsrc[R].ctr, fi.x0h, m, wr, wpow) && finite;
        } else {
          load_row_moments<D, Q>(rsrc[R], m);
          finite = finish_row<D, Q>(rsrc[R].ctr, fi.x0h, m, wr, wpow) && finite;
        }
      } else {
        static_for<0, M>([&](auto I) { m[I] = 0.0; });
      }
      static_for<0, M>([&](auto I) { Bs[r * MS + I] = m[I]; });
      wreg[R] = wr;
      if constexpr (SM::kFull) sm.wls[r] = wr;
    }
  });
  const double fv = face_flux<D, Q>(g, gp, fi, sm, lane, x0dd);   // barrier: B complete
  const bool allfinite = __all(finite) && __all(isfinite(fv));

  // ---- G = B^T B: full 16-column tiles on the matrix cores --------------------------------
  // (v_mfma_f64_16x16x4f64, rows of B as the contraction index; every tile, the lower
  // ones too, so each lane can fetch its row below).  A narrow trailing block (at most 4
  // columns, e.g. 3 of M = 35) is done on the vector ALUs instead: as a 16-wide tile it
  // would be mostly padding, and FP64 MFMA has no more throughput than FP64 FMA on this
  // chip.
  constexpr int MTF = GramSplit<D, Q>::MTF, MV = GramSplit<D, Q>::MV;
  dbl4 acc[MTF][MTF];
#pragma unroll
  for (int i = 0; i < MTF; ++i)
#pragma unroll
    for (int j = 0; j < MTF; ++j) acc[i][j] = dbl4{0, 0, 0, 0};
  const int lr = lane >> 4, lc = lane & 15;
#pragma unroll
  for (int k0 = 0; k0 < NPAD; k0 += 4) {
    double x[MTF];
#pragma unroll
    for (int i = 0; i < MTF; ++i) {
      const int cidx = 16 * i + lc;
      x[i] = (cidx < M) ? Bs[(k0 + lr) * MS + cidx] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < MTF; ++i)
#pragma unroll
      for (int j = 0; j < MTF; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[i], x[j], acc[i][j], 0, 0, 0);
  }
  double gt[MV > 0 ? MV : 1];   // lane l: G[l][16 MTF + c] for the trailing columns c
  if constexpr (MV > 0) {
    static_for<0, MV>([&](auto C) { gt[C] = 0.0; });
    if (lane < M) {
      double g0[MV], g1[MV];
      static_for<0, MV>([&](auto C) { g0[C] = 0.0; g1[C] = 0.0; });
      for (int k = 0; k < NPAD; k += 2) {
        const double b0 = Bs[k * MS + lane], b1 = Bs[(k + 1) * MS + lane];
        static_for<0, MV>([&](auto C) {
          g0[C] = fma(b0, Bs[k * MS + 16 * MTF + C], g0[C]);
          g1[C] = fma(b1, Bs[(k + 1) * MS + 16 * MTF + C], g1[C]);
        });
      }
      static_for<0, MV>([&](auto C) { gt[C] = g0[C] + g1[C]; });
    }
  }
  // Row `lane` of G into a[].  Tile (i, j) register q of lane 16 r' + c' holds
  // G[16i + r' + 4q][16j + c'] (the output layout of v_mfma_f64_16x16x4f64), so lane l
  // reading lane 16 r' + l % 16 gets G[16i + r' + 4q][l] = G[l][16i + r' + 4q] from tile
  // (i, l / 16): a fixed register for every lane, as ds_bpermute needs.
  const int band = lane >> 4;
  static_for<0, MTF>([&](auto I) {
    static_for<0, 4>([&](auto RR) {
      static_for<0, 4>([&](auto QQ) {
        constexpr int c = 16 * I + RR + 4 * QQ;
        if constexpr (c < M) {
          const int src = 16 * RR + lc;
          double v = bpermute_f64(acc[I][0][(int)QQ], src);
          static_for<1, MTF>([&](auto J) {
            const double vj = bpermute_f64(acc[I][J][(int)QQ], src);
            v = (band == J) ? vj : v;
          });
          a[c] = v;
        }
      });
    });
  });
  if constexpr (MV > 0) {
    static_for<0, MV>([&](auto C) { a[16 * MTF + C] = gt[C]; });
    // rows beyond the tiles: G[l][c] = G[c][l], entry l - 16 MTF of gt in lane c
    if (lane < M) static_for<0, MV>([&](auto C) { sm.tt[lane * MV + C] = gt[C]; });
    __syncthreads();
    if (lane >= 16 * MTF && lane < M) {
      const int cc = lane - 16 * MTF;
      static_for<0, 16 * MTF>([&](auto C) { a[C] = sm.tt[C * MV + cc]; });
    }
    __syncthreads();
  }

  // ---- equilibrate to unit diagonal and invert: lane i holds row i ----------------------------
  // Symmetric Gauss-Jordan sweeps over the pivots k = 0..M-1 turn G^ into -G^-1 in place;
  // the pivot of step k is the k-th Schur complement pivot (L_kk^2 of the Cholesky factor),
  // which gives the rank and routing tests.  Values that every lane needs from one lane
  // (the pivot rows, E, the right-hand sides) go through a shared-memory slot per lane and
  // come back as broadcast loads, in place of v_readlane through scalar registers.
  const bool act = lane < M;
  double* piv = sm.zs;   // free between the flux vector and the refinement
  const int pslot = lane < M ? lane : M;   // lanes past M write an unused slot (M < NPAD)
  double gdiag = 1.0;
  static_for<0, M>([&](auto C) { gdiag = (lane == C) ? a[C] : gdiag; });
  sdiag = act ? 1.0 / sqrt(gdiag) : 1.0;
  piv[pslot] = sdiag;
  static_for<0, M>([&](auto J) { a[J] = act ? a[J] * sdiag * piv[J] : 0.0; });
  double gnorm = 0.0;   // ||G^||_inf: largest absolute row sum of the equilibrated Gram matrix
  static_for<0, M>([&](auto J) { gnorm += fabs(a[J]); });
  double pmax = 0.0, pmin = 1e300;   // extreme pivots L_kk^2 (the tests square their bounds)
  // Step k:  a_ij -= (a_ik / d) a_kj  (i, j != k);  a_ik /= d;  a_kj /= d;  a_kk = -1/d.
  // Each lane scales its multiplier once (u = a_ik / d; on lane k, 1 - 1/d turns the
  // pivot row into a_kj / d), so every entry is one FMA.  The sweep keeps the matrix
  // symmetric (up to rounding), so the pivot row is the pivot column: every lane stores
  // its entry of column k in shared memory (one store) and all lanes read the row back
  // with broadcast loads, eight entries at a time before their FMAs.
  static_for<0, M>([&](auto K) {
    constexpr int k = K;
    piv[pslot] = a[k];
    const double d = piv[k];
    const double dp = d > 0.0 ? d : 0.0;
    pmax = fmax(pmax, dp);
    pmin = fmin(pmin, dp);
    const double rd = recip_f64(d);
    const double u = (lane == k) ? 1.0 - rd : a[k] * rd;
    static_for<0, (M + 7) / 8>([&](auto G) {
      double pr[8];
      static_for<0, 8>([&](auto I) {
        constexpr int j = 8 * G + I;
        if constexpr (j < M && j != k) pr[I] = piv[j];
      });
      static_for<0, 8>([&](auto I) {
        constexpr int j = 8 * G + I;
        if constexpr (j < M && j != k) a[j] = fma(-u, pr[I], a[j]);
      });
    });
    a[k] = (lane == k) ? -rd : u;
  });
  const bool pivots_ok = (pmin > kRouteTol * kRouteTol * pmax) && (pmax > 0.0);
  double inv2 = 0.0;    // ||G^^-1||_F^2, from the rows of the inverse
  static_for<0, M>([&](auto J) { inv2 = fma(a[J], a[J], inv2); });
  for (int o = 32; o > 0; o >>= 1) {
    gnorm = fmax(gnorm, __shfl_xor(gnorm, o));
    inv2 += __shfl_xor(inv2, o);
  }
  const double cbound = gnorm * sqrt(inv2);   // wave-uniform
  const bool cond_ok = cbound <= kCondRoute * kCondRoute;
  const bool dot2 = !(cbound <= kDot2Cond);

  // ---- semi-normal solve with one refinement step (compensated past kDot2Cond) ---------
  // y = G^-1 rhs with G^ = E G E (E = diag(sdiag)):  y = E (-a) (E rhs).  Lane p holds
  // component p of F~, rhs and y; lane r holds z of its rows r, r + 64 (past kDot2Cond
  // as zreg + zlo).
  double rhs = fv * sdiag;
  double ysum = 0.0;
  double dlast = 0.0;   // largest change of W z in the refinement step
  double zlo[NR];
  static_for<0, NR>([&](auto R) {
    zreg[R] = 0.0;
    zlo[R] = 0.0;
  });
  for (int it = 0; it <= kRefine; ++it) {
    double tq[4] = {0.0, 0.0, 0.0, 0.0};
    piv[pslot] = rhs;
    static_for<0, M>([&](auto J) { tq[J % 4] = fma(-a[J], piv[J], tq[J % 4]); });
    const double t = (tq[0] + tq[1]) + (tq[2] + tq[3]);
    const double dy = act ? t * sdiag : 0.0;
    ysum += dy;
    piv[pslot] = dy;
    // z += B dy
    static_for<0, NR>([&](auto R) {
      const int r = lane + 64 * R;
      if (r < NPAD) {
        double inc;
        if (dot2) {
          Dot2 d0{0.0, 0.0}, d1{0.0, 0.0};
          static_for<0, M>([&](auto J) {
            if constexpr (J % 2 == 0) dot2_add(d0, Bs[r * MS + J], piv[J]);
            else dot2_add(d1, Bs[r * MS + J], piv[J]);
          });
          const Dot2 d = dot2_join(d0, d1);
          dd zs2 = dd_add(dd{zreg[R], zlo[R]}, dd{d.s, d.c});
          zreg[R] = zs2.hi;
          zlo[R] = zs2.lo;
          inc = d.s + d.c;
        } else {
          double sq4[4] = {0.0, 0.0, 0.0, 0.0};
          static_for<0, M>([&](auto J) { sq4[J % 4] = fma(Bs[r * MS + J], piv[J], sq4[J % 4]); });
          inc = (sq4[0] + sq4[1]) + (sq4[2] + sq4[3]);
          zreg[R] += inc;
        }
        if (it == kRefine) dlast = fmax(dlast, fabs(wreg[R] * inc));
      }
    });
    if (it == kRefine) break;
    // residual of B^T z = F~ (two interleaved sums, compensated past kDot2Cond, where the
    // low part of z enters the compensation); z goes through LDS, B^T is read by columns
    static_for<0, NR>([&](auto R) {
      const int r = lane + 64 * R;
      if (r < NPAD) {
        sm.zs[r] = zreg[R];
        sm.zl[r] = zlo[R];
      }
    });
    __syncthreads();
    double res = 0.0;
    if (act && dot2) {
      Dot2 d0{fv, 0.0}, d1{0.0, 0.0};
      double lo = 0.0;
#pragma unroll 4
      for (int r = 0; r < NPAD; r += 2) {
        dot2_add(d0, -Bs[(r + 0) * MS + lane], sm.zs[r + 0]);
        dot2_add(d1, -Bs[(r + 1) * MS + lane], sm.zs[r + 1]);
        lo = fma(-Bs[(r + 0) * MS + lane], sm.zl[r + 0], lo);
        lo = fma(-Bs[(r + 1) * MS + lane], sm.zl[r + 1], lo);
      }
      d1.c += lo;
      res = dot2_merge(d0, d1);
    } else if (act) {
      double p0 = fv, p1 = 0.0;
#pragma unroll 4
      for (int r = 0; r < NPAD; r += 2) {
        p0 = fma(-Bs[(r + 0) * MS + lane], sm.zs[r + 0], p0);
        p1 = fma(-Bs[(r + 1) * MS + lane], sm.zs[r + 1], p1);
      }
      res = p0 + p1;
    }
    rhs = res * sdiag;
    __syncthreads();
  }
  if (dot2) static_for<0, NR>([&](auto R) { zreg[R] += zlo[R]; });
  if constexpr (SM::kFull) {
    static_for<0, NR>([&](auto R) {
      const int r = lane + 64 * R;
      if (r < NPAD) sm.zs[r] = zreg[R];
    });
    if (act) sm.ys[lane] = ysum;
    __syncthreads();
  }
  // has the refinement settled?  The step's change of the stencil W z against its size
  double smax = 0.0;
  static_for<0, NR>([&](auto R) { smax = fmax(smax, fabs(wreg[R] * zreg[R])); });
  for (int o = 32; o > 0; o >>= 1) {
    dlast = fmax(dlast, __shfl_xor(dlast, o));
    smax = fmax(smax, __shfl_xor(smax, o));
  }
  const bool settled = dlast <= kSettleTol * smax;
  if (rank_low) *rank_low = !((pmin > kRankTol * kRankTol * pmax) && (pmax > 0.0));
  if (!allfinite) return CUTCELL_STATUS_NONFINITE;
  if (!pivots_ok || !cond_ok || !settled) return kStatusRoute;
  return CUTCELL_STATUS_OK;
}

struct StencilArgs {
  GridDims g;
  int G;
  double hscale;
  const int32_t* perm;
  long long nbin;
  const int32_t* fcode;
  const int32_t* fref;
  const GeomPtrs* geoms;
  const int64_t* counts;
  const int64_t* offs;
  const int32_t* vol_cell_ws;
  const int32_t* box_lf_ws;
  const int64_t* row_ptr;
  const int32_t* col;
  // schedule: workgroup b runs on XCD b % xcd (the dispatcher deals workgroups out to the
  // XCDs in turn) and walks that XCD's contiguous chunk of the bin with stride per_xcd
  int xcd;
  int per_xcd;
  double h;            // grid spacing (Neumann rows carry one more power of h)
  double wpow;         // weight exponent p of W = (2 |delta|)^-p
  int32_t* qr_list;    // faces left to the Householder QR path, and their count
  int32_t* qr_count;
  int route;           // 1: such faces go to the QR path; 0: the Gram path keeps every face
};

// Faces of a bin taken by workgroup blockIdx.x in turn (-1 when done).  With xcd = 1 and a
// grid of nbin workgroups this is one face per workgroup in bin order.
struct FaceWalk {
  long long chunk, k, base;
  int step;
  __device__ FaceWalk(const StencilArgs& A) {
    const int b = blockIdx.x;
    chunk = (A.nbin + A.xcd - 1) / A.xcd;
    base = (long long)(b % A.xcd) * chunk;
    k = b / A.xcd;
    step = A.per_xcd;
  }
  __device__ long long next() {
    if (k >= chunk) return -1;
    const long long t = base + k;
    k += step;
    return t;
  }
};

__device__ __forceinline__ FaceInfo face_info(const StencilArgs& A, long long t) {
  FaceInfo fi;
  fi.F = A.perm[t];
  const int32_t code = A.fcode[fi.F];
  fi.gi = code >> 4;
  fi.kind = (code >> 2) & 3;
  fi.dn = code & 3;
  fi.ref = A.fref[fi.F];
  fi.n_vol = A.counts[4 * fi.gi + 0];
  fi.n_eb = A.counts[4 * fi.gi + 1];
  fi.phi0 = A.offs[fi.gi];
  fi.rp = A.row_ptr[fi.F];
  fi.N = (int)(A.row_ptr[fi.F + 1] - fi.rp);
  return fi;
}

// One face per workgroup (WALK = false: face t of the bin, t from the XCD mapping), or a
// persistent workgroup that walks its chunk (WALK = true).  Two instances because the
// loop costs the single-face kernel registers.
template <int D, int Q, int NPAD, bool NEU>
__device__ __forceinline__ void stencil_face(const StencilArgs& A, long long t, LeanSmem<D, Q, NPAD>& sm, int lane,
                                             double* __restrict__ val, int8_t* __restrict__ status, int32_t* flagged) {
  constexpr int M = Dims<D, Q>::M, NR = (NPAD + 63) / 64;
  FaceInfo fi = face_info(A, t);
  const GeomPtrs gp = A.geoms[fi.gi];
  face_x0<D, Q>(A.g, gp, fi);
  double a[M], wreg[NR], zreg[NR];
  double sdiag;
  bool rank_low = false;
  int st = face_forward<D, Q, NPAD, NEU>(A.g, gp, fi, A.vol_cell_ws + (long long)fi.gi * A.g.ncell,
                                         A.box_lf_ws + (long long)fi.gi * A.g.nboxslot, A.col, sm, lane, a, sdiag,
                                         wreg, zreg, A.wpow, &rank_low);
  if (st == kStatusRoute) {
    if (A.route) {   // the QR path writes this face's values and status
      if (lane == 0) A.qr_list[atomicAdd(A.qr_count, 1)] = fi.F;
      return;
    }
    st = rank_low ? CUTCELL_STATUS_RANK_DEFICIENT : CUTCELL_STATUS_OK;
  }
  static_for<0, NR>([&](auto R) {
    const int r = lane + 64 * R;
    if (r < fi.N) {
      double v = (st == CUTCELL_STATUS_OK) ? A.hscale * wreg[R] * zreg[R] : 0.0;
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

// (two waves per SIMD: the register budget of 256 includes the matrix-core accumulators)
template <int D, int Q, int NPAD, bool WALK, bool NEU = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_stencil(StencilArgs A, double* __restrict__ val, int8_t* __restrict__ status,
                                               int32_t* flagged) {
  __shared__ LeanSmem<D, Q, NPAD> sm;
  const int lane = threadIdx.x;
  FaceWalk walk(A);
  if constexpr (!WALK) {
    const long long t = walk.next();
    if (t >= 0 && t < A.nbin) stencil_face<D, Q, NPAD, NEU>(A, t, sm, lane, val, status, flagged);
  } else {
    for (long long t = walk.next(); t >= 0 && t < A.nbin; t = walk.next()) {
      stencil_face<D, Q, NPAD, NEU>(A, t, sm, lane, val, status, flagged);
      __syncthreads();   // the next face reuses the shared memory
    }
  }
}

// ---------------------------------------------------------------------------------------
// Adjoint of the stencil of one face (the derivative of the solution of Sec. 2.2.1).
// With s~ = W z, z = B y, y = G^-1 F~, G = B^T B and a given s~bar:
//   zbar = W s~bar,  Wbar_i = s~bar_i z_i (through s~ = W z),
//   w = G^-1 B^T zbar (a least-squares solve, refined like the forward), r = zbar - B w,
//   Bbar = r y^T - z w^T,  Fbar = w,  Abar = W Bbar,  Wbar_i += Bbar_i . A~_i.
// Bbar_i . B_i = r_i z_i - z_i (B w)_i needs no pass over the row.  The rows' moments
// get S(delta_i)^T Abar_i / mu0 - e_0 (Abar_i . A~_i) / mu0; that sum over the faces a
// row appears in is formed per Phi entry by k_moment_reduce from what this kernel keeps:
// y and w of the face, x0, and (W r, W z) per row.  For an EB face x0 is the centroid of
// the cut volume, so every row's delta and weight and the re-centred normal moments also
// depend on that volume's moments 0..D; their gradient goes to owner_grad.

template <int D, int Q, int NPAD>
__global__ __launch_bounds__(64) void k_stencil_backward(StencilArgs A, BackwardArgs B) {
  using DM = Dims<D, Q>;
  constexpr int M = DM::M, MS = DM::MS, Mf = DM::Mf, M1 = DM::M1;
  __shared__ FaceSmem<D, Q, NPAD> sm;
  __shared__ double zbar[NPAD];   // W s~bar, then the residual r = zbar - B w
  __shared__ double bw[NPAD];     // B w
  __shared__ double wv[M + 1];    // w
  __shared__ double gdx[64][3];   // per-lane sums of dl/dx0 over the rows
  const long long t = blockIdx.x;
  if (t >= A.nbin) return;
  const int lane = threadIdx.x;
  FaceInfo fi = face_info(A, t);
  const GeomPtrs gp = A.geoms[fi.gi];
  face_x0<D, Q>(A.g, gp, fi);
  double a[M];
  double sdiag;
  const int32_t* vol_cell = A.vol_cell_ws + (long long)fi.gi * A.g.ncell;
  const int32_t* box_lf = A.box_lf_ws + (long long)fi.gi * A.g.nboxslot;
  const bool act = lane < M;
  const int N = fi.N;
  double* yw = B.face_yw + (long long)fi.F * 2 * M;
  double* og = B.owner_grad + (long long)fi.F * 4;
  if (lane < 4) B.face_x0[(long long)fi.F * 4 + lane] = (lane < 3) ? fi.x0h[lane] : 0.0;
  // a face whose stencil gets no cotangent contributes nothing: skip its solve
  bool any = false;
  for (int r = lane; r < N; r += 64) any = any || (B.val_bar[fi.rp + r] != 0.0);
  if (!__any(any)) {
    for (int r = lane; r < N; r += 64) {
      B.nz_rz[2 * (fi.rp + r)] = 0.0;
      B.nz_rz[2 * (fi.rp + r) + 1] = 0.0;
      if (B.weight_bar) B.weight_bar[fi.rp + r] = 0.0;
    }
    if (act) { yw[lane] = 0.0; yw[M + lane] = 0.0; }
    if (lane < 4) og[lane] = 0.0;
    return;
  }
  double wreg[(NPAD + 63) / 64], zreg[(NPAD + 63) / 64];
  const int st = face_forward<D, Q, NPAD, false>(A.g, gp, fi, vol_cell, box_lf, A.col, sm, lane, a, sdiag, wreg, zreg,
                                                 A.wpow);
  const double* Bs = sm.Bs;
  // a flagged face has s = 0 whatever its inputs: no gradient (the forward status decides
  // for the faces the forward build solved by Householder QR)
  if (st == CUTCELL_STATUS_NONFINITE || B.fwd_status[fi.F] != CUTCELL_STATUS_OK) {
    for (int r = lane; r < N; r += 64) {
      B.nz_rz[2 * (fi.rp + r)] = 0.0;
      B.nz_rz[2 * (fi.rp + r) + 1] = 0.0;
      if (B.weight_bar) B.weight_bar[fi.rp + r] = 0.0;
    }
    if (act) { yw[lane] = 0.0; yw[M + lane] = 0.0; }
    if (lane < 4) og[lane] = 0.0;
    return;
  }
  // s~bar = h^(D-2) val_bar;  zbar = W s~bar;  the direct part of Wbar in gdx-free regs
  for (int r = lane; r < NPAD; r += 64) {
    const double sb = (r < N) ? A.hscale * B.val_bar[fi.rp + r] : 0.0;
    zbar[r] = sm.wls[r] * sb;
  }
  __syncthreads();
  // w = G^-1 B^T zbar, refined:  w += G^-1 B^T (zbar - B w); lane p holds w_p
  constexpr int NR = (NPAD + 63) / 64;
  double wl = 0.0;
  for (int it = 0; it <= kRefineBackward; ++it) {
    double res = 0.0;
    if (act) {
      double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
      for (int r = 0; r < NPAD; r += 4) {
        double e0 = zbar[r + 0], e1 = zbar[r + 1], e2 = zbar[r + 2], e3 = zbar[r + 3];
        if (it > 0) { e0 -= bw[r + 0]; e1 -= bw[r + 1]; e2 -= bw[r + 2]; e3 -= bw[r + 3]; }
        r0 = fma(Bs[(r + 0) * MS + lane], e0, r0);
        r1 = fma(Bs[(r + 1) * MS + lane], e1, r1);
        r2 = fma(Bs[(r + 2) * MS + lane], e2, r2);
        r3 = fma(Bs[(r + 3) * MS + lane], e3, r3);
      }
      res = (r0 + r1) + (r2 + r3);
    }
    const double rhs = res * sdiag;
    double tq[4] = {0.0, 0.0, 0.0, 0.0};
    static_for<0, M>([&](auto J) { tq[J % 4] = fma(-a[J], readlane_f64(rhs, J), tq[J % 4]); });
    if (act) wl += ((tq[0] + tq[1]) + (tq[2] + tq[3])) * sdiag;
    __syncthreads();
    static_for<0, NR>([&](auto R) {
      const int r = lane + 64 * R;
      if (r < NPAD) {
        double s = 0.0;
        static_for<0, M>([&](auto J) { s = fma(Bs[r * MS + J], readlane_f64(wl, J), s); });
        bw[r] = s;
      }
    });
    __syncthreads();
  }
  if (act) wv[lane] = wl;
  __syncthreads();
  if (act) {
    yw[lane] = sm.ys[lane];
    yw[M + lane] = wl;
  }
  // per row: r = zbar - B w;  Wbar;  (W r, W z) for the moment reduction;  EB x0 terms
  double gx[3] = {0, 0, 0};
  for (int r = lane; r < N; r += 64) {
    const double W = sm.wls[r], zz = sm.zs[r];
    const double rr = zbar[r] - bw[r];
    const double sb = A.hscale * B.val_bar[fi.rp + r];
    const double bdot = zz * (rr - bw[r]);            // Bbar_i . B_i
    const double wtot = sb * zz + bdot / W;           // dl/dW_i
    if (B.weight_bar) B.weight_bar[fi.rp + r] = wtot;
    B.nz_rz[2 * (fi.rp + r)] = W * rr;
    B.nz_rz[2 * (fi.rp + r) + 1] = W * zz;
    if (fi.kind == 1) {
      // delta_i = x_i/h - x0h: d B_ip / d delta_d = p_d B_i,p-e_d (weight fixed), and
      // dW/d delta_d = -p W delta_d / |delta|^2 outside half a cell (W = (2|delta|)^-p)
      const RowSource rs = row_source<D, Q>(A.g, gp, (int64_t)A.col[fi.rp + r] - fi.phi0, fi.n_vol, fi.n_eb,
                                            vol_cell, box_lf);
      double dl[3] = {0, 0, 0}, d2 = 0.0;
      for (int ax = 0; ax < D; ++ax) {
        dl[ax] = rs.ctr[ax] - fi.x0h[ax];
        d2 += dl[ax] * dl[ax];
      }
      double gd[3] = {0, 0, 0};
      static_for<0, M>([&](auto P) {
        constexpr int p = P;
        const double bb = rr * sm.ys[p] - zz * wv[p];   // Bbar_ip
        static_for<0, D>([&](auto AX) {
          constexpr int ax = AX;
          constexpr int pd = kMono<D, Q>.e[p][ax];
          if constexpr (pd > 0) {
            constexpr int q = mono_index<D>(kMono<D, Q>.e[p][0] - (ax == 0), kMono<D, Q>.e[p][1] - (ax == 1),
                                            kMono<D, Q>.e[p][2] - (ax == 2));
            gd[ax] = fma(bb * pd, Bs[r * MS + q], gd[ax]);
          }
        });
      });
      if (sqrt(d2) >= 0.5)
        for (int ax = 0; ax < D; ++ax) gd[ax] += wtot * (-A.wpow * W * dl[ax] / d2);
      for (int ax = 0; ax < D; ++ax) gx[ax] -= gd[ax];   // d delta / d x0h = -1
    }
  }
  // flux-vector gradient Fbar = w
  if (fi.kind == 0) {
    if (lane < 4) og[lane] = 0.0;
    if (act) {
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
        B.grads[fi.gi].face_mom[dn][(fi.ref - A.g.foff[dn]) * Mf + s] = wv[lane];
      }
    }
    return;
  }
  // EB face: F~_p = sum_d p_d nu'_{d, p - e_d} with nu' the normal moments re-centred by
  // delta0 = (c - x0)/h:  nu'bar_{d,q} = (q_d + 1) w_{q + e_d},  nubar = S(delta0)^T nu'bar,
  // and d nu'_{d,q} / d delta0_k = q_k nu'_{d, q - e_k}
  for (int ax = 0; ax < 3; ++ax) gdx[lane][ax] = gx[ax];
  __syncthreads();
  if (lane < D) {
    double nb[M1];
    double g0[3] = {0, 0, 0};
    static_for<0, M1>([&](auto I) {
      constexpr int i = I;
      constexpr int q0 = kMono<D, Q - 1>.e[i][0], q1 = kMono<D, Q - 1>.e[i][1], q2 = kMono<D, Q - 1>.e[i][2];
      const int qd = (lane == 0) ? q0 : (lane == 1 ? q1 : q2);
      const int up = mono_index<D>(q0 + (lane == 0), q1 + (lane == 1), q2 + (lane == 2));
      nb[i] = (qd + 1) * wv[up];
    });
    static_for<0, M1>([&](auto I) {
      constexpr int i = I;
      static_for<0, D>([&](auto K) {
        constexpr int k = K;
        constexpr int qk = kMono<D, Q - 1>.e[i][k];
        if constexpr (qk > 0) {
          constexpr int src = mono_index<D>(kMono<D, Q - 1>.e[i][0] - (k == 0), kMono<D, Q - 1>.e[i][1] - (k == 1),
                                            kMono<D, Q - 1>.e[i][2] - (k == 2));
          g0[k] = fma(nb[i] * qk, sm.nus[lane][src], g0[k]);
        }
      });
    });
    double d0[3] = {-fi.off[0], -fi.off[1], -fi.off[2]};
    recentre_T<D, Q - 1>(nb, d0);
    double* dst = B.grads[fi.gi].eb_nmom + ((long long)fi.ref * D + lane) * M1;
    static_for<0, M1>([&](auto I) { dst[I] = nb[I]; });
    for (int k = 0; k < 3; ++k) sm.gsum[lane * 3 + k] = g0[k];   // dl/d delta0 from component `lane`
  }
  __syncthreads();
  if (lane == 0) {
    // dl/dx0h = sum over rows (gdx) - dl/d delta0;  x0h_d = centre_d + m^{e_d} / m^0
    double gxh[3] = {0, 0, 0};
    for (int l = 0; l < 64; ++l)
      for (int ax = 0; ax < D; ++ax) gxh[ax] += gdx[l][ax];
    for (int c = 0; c < D; ++c)
      for (int k = 0; k < D; ++k) gxh[k] -= sm.gsum[c * 3 + k];
    const double* vm = gp.vol_mom + (long long)fi.owner_cell * M;
    const double m0 = vm[0];
    double g0 = 0.0;
    for (int ax = 0; ax < D; ++ax) {
      og[1 + ax] = gxh[ax] / m0;
      g0 -= gxh[ax] * vm[1 + ax] / (m0 * m0);
    }
    og[0] = g0;
    for (int ax = D; ax < 3; ++ax) og[1 + ax] = 0.0;
  }
}

// ---------------------------------------------------------------------------------------
// Launches

inline StencilArgs stencil_args(const Work& w, double hscale, const int32_t* perm, long long nbin,
                               const int64_t* row_ptr, const int32_t* col) {
  StencilArgs A;
  A.xcd = 1;
  A.per_xcd = 1;
  A.g = w.dims;
  A.G = w.G;
  A.hscale = hscale;
  A.perm = perm;
  A.nbin = nbin;
  A.fcode = w.fcode;
  A.fref = w.fref;
  A.geoms = w.geoms;
  A.counts = w.counts;
  A.offs = w.offs;
  A.vol_cell_ws = w.vol_cell;
  A.box_lf_ws = w.box_lf;
  A.row_ptr = row_ptr;
  A.col = col;
  A.h = 0.0;
  A.wpow = 5.0;
  A.qr_list = w.qr_list;
  A.qr_count = w.qr_count;
  A.route = 1;
  return A;
}

// Launch shape of one bin: xcd = 1 or the number of XCDs whose chunks the bin is split
// into; per_xcd = 0 for one workgroup per face, else the persistent workgroups per chunk;
// split: which kernel widths take the bin's parts 0 and 1 (its faces with at most
// NPAD - 8 and NPAD - 4 rows) where narrower instances are compiled -- 0: part 0 at
// NPAD - 8 and part 1 at NPAD - 4; 1: none, the whole bin at NPAD rows; 2: part 0 at
// NPAD - 8 only; 3: parts 0 and 1 at NPAD - 4.
struct BinSchedule {
  int xcd = 1;
  int per_xcd = 0;
  int split = 0;
  bool route = true;   // faces the Gram path cannot resolve go to the QR path
};

template <int D, int Q, int NPAD, bool FWD_ONLY = false>
static void launch_bin(const Work& w, double hscale, const int32_t* perm, long long nbin, const int64_t* row_ptr,
                       const int32_t* col, double* val, int8_t* status, hipStream_t st, const BackwardArgs* bw,
                       BinSchedule sc, bool neu, double h, double wpow) {
  if (nbin <= 0) return;
  StencilArgs A = stencil_args(w, hscale, perm, nbin, row_ptr, col);
  A.wpow = wpow;
  if constexpr (!FWD_ONLY) {
    if (bw) {
      hipLaunchKernelGGL((k_stencil_backward<D, Q, NPAD>), dim3((unsigned)nbin), dim3(64), 0, st, A, *bw);
      return;
    }
  }
  const int X = sc.xcd > 1 ? sc.xcd : 1;
  const long long chunk = (nbin + X - 1) / X;
  const long long per = sc.per_xcd > 0 ? std::min<long long>(sc.per_xcd, chunk) : chunk;
  A.xcd = X;
  A.per_xcd = (int)per;
  A.route = sc.route ? 1 : 0;
  if (neu) {   // one workgroup per face (no persistent instance of the Neumann kernel)
    A.per_xcd = (int)chunk;
    A.h = h;
    hipLaunchKernelGGL((k_stencil<D, Q, NPAD, false, true>), dim3((unsigned)(X * chunk)), dim3(64), 0, st, A, val,
                       status, w.flagged);
    return;
  }
  if (per < chunk)
    hipLaunchKernelGGL((k_stencil<D, Q, NPAD, true>), dim3((unsigned)(X * per)), dim3(64), 0, st, A, val, status,
                       w.flagged);
  else
    hipLaunchKernelGGL((k_stencil<D, Q, NPAD, false>), dim3((unsigned)(X * per)), dim3(64), 0, st, A, val, status,
                       w.flagged);
}

// Waves of the forward kernel that one 80 KB shared-memory pool (two SIMDs) holds: measured
// on MI355X, residency follows two such pools per CU rather than the 160 KB total.  At most
// 4 (2 per SIMD at the kernel's register count).
template <int D, int Q, int NPAD>
constexpr int pool_waves() {
  constexpr int n = 81920 / (int)sizeof(LeanSmem<D, Q, NPAD>);
  return n < 4 ? n : 4;
}

// A narrower kernel instance of P rows pays for a part of a bin of NPAD rows when it fits
// more waves per pool (3D order 4: 88 and 92 rows for the 96-row bin, whose regular faces
// have 88 rows; no other bin of the orders and dimensions built).
template <int D, int Q, int P, int NPAD>
constexpr bool narrower_pays() {
  if constexpr (P < Dims<D, Q>::M) return false;
  else return pool_waves<D, Q, P>() > pool_waves<D, Q, NPAD>();
}

// One row bin: its part 0 (n0 faces, at most NPAD - 8 rows) and part 1 (n1 faces, at most
// NPAD - 4 rows) come first in its order; each runs on the narrowest instance that pays,
// the rest on the NPAD-row instance.  The adjoint runs the whole bin at NPAD rows.
template <int D, int Q, int NPAD>
void launch_row_bin(const Work& w, double hscale, const int32_t* perm, long long nbin, long long n0, long long n1,
                    const int64_t* row_ptr, const int32_t* col, double* val, int8_t* status, hipStream_t st,
                    const BackwardArgs* bw, BinSchedule sc, bool neu, double h, double wpow) {
  constexpr int P0 = NPAD - kBinRows / 2, P1 = NPAD - kBinRows / 4;
  long long done = 0;
  if (!bw) {
    if constexpr (narrower_pays<D, Q, P0, NPAD>()) {
      if (sc.split == 0 || sc.split == 2) {
        launch_bin<D, Q, P0, true>(w, hscale, perm, n0, row_ptr, col, val, status, st, bw, sc, neu, h, wpow);
        done = n0;
      }
    }
    if constexpr (narrower_pays<D, Q, P1, NPAD>()) {
      if (sc.split == 0 || sc.split == 3) {
        launch_bin<D, Q, P1, true>(w, hscale, perm + done, n0 + n1 - done, row_ptr, col, val, status, st, bw, sc,
                                   neu, h, wpow);
        done = n0 + n1;
      }
    }
  }
  launch_bin<D, Q, NPAD>(w, hscale, perm + done, nbin - done, row_ptr, col, val, status, st, bw, sc, neu, h, wpow);
}

// Narrower instances compiled for the bin of NPAD rows: bit 0 for NPAD - 8, bit 1 for NPAD - 4.
template <int D, int Q, int NPAD>
constexpr int narrow_mask() {
  return (narrower_pays<D, Q, NPAD - kBinRows / 2, NPAD>() ? 1 : 0) |
         (narrower_pays<D, Q, NPAD - kBinRows / 4, NPAD>() ? 2 : 0);
}

// the same for dimension, order and bin b known at run time (the split modes to tune)
inline int narrow_mask_of(int D, int Q, int b) {
  auto pick = [&](auto DD, auto QQ) {
    constexpr int Dc = decltype(DD)::value, Qc = decltype(QQ)::value;
    switch (b) {
      case 1: return narrow_mask<Dc, Qc, 32>();
      case 2: return narrow_mask<Dc, Qc, 48>();
      case 3: return narrow_mask<Dc, Qc, 64>();
      case 4: return narrow_mask<Dc, Qc, 80>();
      case 5: return narrow_mask<Dc, Qc, 96>();
      case 6: return narrow_mask<Dc, Qc, 112>();
      case 7: return narrow_mask<Dc, Qc, 128>();
      default: return 0;
    }
  };
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  using I4 = std::integral_constant<int, 4>;
  if (D == 2) return Q == 2 ? pick(I2{}, I2{}) : pick(I2{}, I4{});
  return Q == 2 ? pick(I3{}, I2{}) : pick(I3{}, I4{});
}

// Explicit instantiations: each (dimension, order, bin) lives in one stencil_d*q*.hip file,
// so the library's kernels compile in parallel (the 3D order-4 bins over three files).
#define CC_ROW_BIN(DD, QQ, P, EXT) \
  EXT template void launch_row_bin<DD, QQ, P>(const Work&, double, const int32_t*, long long, long long, long long, \
                                              const int64_t*, const int32_t*, double*, int8_t*, hipStream_t, \
                                              const BackwardArgs*, BinSchedule, bool, double, double);
#define CC_ROW_BINS_ALL(DD, QQ, EXT) \
  CC_ROW_BIN(DD, QQ, 16, EXT) CC_ROW_BIN(DD, QQ, 32, EXT) CC_ROW_BIN(DD, QQ, 48, EXT) CC_ROW_BIN(DD, QQ, 64, EXT) \
  CC_ROW_BIN(DD, QQ, 80, EXT) CC_ROW_BIN(DD, QQ, 96, EXT) CC_ROW_BIN(DD, QQ, 112, EXT) CC_ROW_BIN(DD, QQ, 128, EXT)
CC_ROW_BINS_ALL(2, 2, extern) CC_ROW_BINS_ALL(2, 4, extern) CC_ROW_BINS_ALL(3, 2, extern)
CC_ROW_BIN(3, 4, 48, extern) CC_ROW_BIN(3, 4, 64, extern) CC_ROW_BIN(3, 4, 80, extern)
CC_ROW_BIN(3, 4, 96, extern) CC_ROW_BIN(3, 4, 112, extern) CC_ROW_BIN(3, 4, 128, extern)

// The row bins of one (dimension, order): one launch per bin (two for a split bin).
template <int D, int Q>
int dispatch_row_bins(const Work& w, double hscale, const int32_t* bin_count, const int64_t* row_ptr,
                      const int32_t* col, double* val, int8_t* status, hipStream_t st, const BackwardArgs* bw,
                      const BinSchedule* sched, int only_bin, bool neu, double h, double wpow) {
  constexpr int M = binom(Q + D, D);
  long long start = 0;
  for (int b = 0; b < kMaxBins; ++b) {
    const long long nb = bin_count[b];
    const int32_t* p = w.perm + start;
    start += nb;
    if (nb == 0 || (only_bin >= 0 && b != only_bin)) continue;
    const int npad = kBinRows * (b + 1);
    if (npad < M) return fail(CUTCELL_E_INVALID_ARG, "internal: face with N >= M in a bin narrower than M");
    const long long n0 = bin_count[kPartWords + b], n1 = bin_count[kPartWords + kMaxBins + b];
    switch (npad) {
#define CC_BIN(P) \
  case P: \
    if constexpr (M <= P) \
      launch_row_bin<D, Q, P>(w, hscale, p, nb, n0, n1, row_ptr, col, val, status, st, bw, sched[b], neu, h, \
                              wpow); \
    break;
      CC_BIN(16) CC_BIN(32) CC_BIN(48) CC_BIN(64) CC_BIN(80) CC_BIN(96) CC_BIN(112) CC_BIN(128)
#undef CC_BIN
    }
  }
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

#define CC_DISPATCH(DD, QQ, EXT) \
  EXT template int dispatch_row_bins<DD, QQ>(const Work&, double, const int32_t*, const int64_t*, const int32_t*, \
                                             double*, int8_t*, hipStream_t, const BackwardArgs*, const BinSchedule*, \
                                             int, bool, double, double);
CC_DISPATCH(2, 2, extern) CC_DISPATCH(2, 4, extern) CC_DISPATCH(3, 2, extern) CC_DISPATCH(3, 4, extern)

}  // namespace cutcell
