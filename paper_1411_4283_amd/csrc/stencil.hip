// Per-face weighted least-squares flux stencils (Sec. 2.2.1, eq. 'stencil equation
// solution'; neighbours, centring and weights of Sec. 2.4).
//
// The stencil s~ = W (A~^T W)^+ F~ is W z with z the minimum-norm solution of
// B^T z = F~, B = W A~ (N x M, N >= M, full column rank): z = B (B^T B)^-1 F~.  One
// wavefront owns one face:
//   1. rows: each lane builds its row(s) of B in registers -- the row's moments,
//      re-centred to x0 by the binomial theorem, divided by the zeroth moment and
//      scaled by the weight -- and stores them in LDS;
//   2. G = B^T B on the FP64 matrix cores (v_mfma_f64_16x16x4f64, 16 x 16 tiles of the
//      upper triangle, rows of B as the contraction index);
//   3. G is equilibrated to unit diagonal and inverted by symmetric Gauss-Jordan sweeps,
//      lane i holding row i in registers; the sweep pivots are the Cholesky pivots;
//   4. z from the semi-normal equations z = B G^-1 F~ followed by two steps of
//      refinement with the residual F~ - B^T z computed from B itself, which brings the
//      error down to that of a backward-stable solve (cond(B) * eps);
//   5. val = h^(D-2) W z.
// Status: fewer rows than monomials, a pivot square root below 1e-7 times the largest after
// equilibration (numerically rank deficient), or a non-finite entry flag the face.
#include "kernels.hpp"
#include "rows.hpp"

namespace cutcell {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr double kRankTol = 1e-7;
constexpr int kRefine = 2;

// One row of B = W A~ about x0 (in units of h: x0h = x0 / h), with its weight.
// Returns false if the row holds a non-finite value.
template <int D, int Q>
__device__ __forceinline__ bool build_row(const GridDims& g, const GeomPtrs& gp, int64_t phi_local, int64_t n_vol,
                                          int64_t n_eb, const int32_t* vol_cell, const int32_t* box_lf,
                                          const double* x0h, double* m, double& w) {
  constexpr int M = Dims<D, Q>::M;
  const RowSource rs = row_source<D, Q>(g, gp, phi_local, n_vol, n_eb, vol_cell, box_lf);
  load_row_moments<D, Q>(rs, m);
  double delta[3] = {0, 0, 0};
  double d2 = 0;
  for (int ax = 0; ax < D; ++ax) {
    delta[ax] = rs.ctr[ax] - x0h[ax];
    d2 += delta[ax] * delta[ax];
  }
  w = row_weight(d2);
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

// Shared memory of one face (one wave).
template <int D, int Q, int NPAD>
struct FaceSmem {
  static constexpr int M = Dims<D, Q>::M, MS = Dims<D, Q>::MS, M1 = Dims<D, Q>::M1;
  double Bs[NPAD * MS];      // rows of B = W A~
  double Ls[M * MS];         // Gram matrix, then the pivot rows of the inversion
  double vec[2][M + 1];      // F~ and a broadcast vector
  double ys[M + 1];          // y = G^-1 F~
  double zs[NPAD];           // z = B y
  double wls[NPAD];          // W
  double nus[D][M1];         // EB normal moments about x0
};

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

// x0, the flux vector F~ (in sm.vec[0]) and, for EB faces, the re-centred normal moments
template <int D, int Q, int NPAD>
__device__ __forceinline__ void face_setup(const GridDims& g, const GeomPtrs& gp, FaceInfo& fi,
                                           FaceSmem<D, Q, NPAD>& sm, int lane) {
  constexpr int M = Dims<D, Q>::M, Mf = Dims<D, Q>::Mf, M1 = Dims<D, Q>::M1;
  const int dn = fi.dn;
  for (int ax = 0; ax < 3; ++ax) { fi.x0h[ax] = 0.0; fi.off[ax] = 0.0; }
  fi.owner_cell = -1;
  if (fi.kind == 0) {
    const long long loc = fi.ref - g.foff[dn];
    const int m0 = g.n[0] + (dn == 0), m1 = g.n[1] + (dn == 1);
    const int j[3] = {(int)(loc % m0), (int)((loc / m0) % m1), (int)(loc / ((long long)m0 * m1))};
    for (int ax = 0; ax < D; ++ax) fi.x0h[ax] = (ax == dn) ? (double)j[ax] : j[ax] + 0.5;
    // F~_p = face moment of p - e_d when p_d = 1 (reference normal +e_d)
    const double* fm = gp.face_mom[dn] + loc * Mf;
    if (lane < M) {
      double fv = 0.0;
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
      sm.vec[0][lane] = fv;
    }
    __syncthreads();
    return;
  }
  // EB face: x0 = centroid of the cut volume; the normal moments (about the cell centre)
  // are re-centred to x0 by lanes 0..D-1, one component each
  const int32_t c = gp.eb_cell[fi.ref];
  fi.owner_cell = c;
  const int cown[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long long)g.n[0] * g.n[1]))};
  const double* vm = gp.vol_mom + (long long)c * M;
  const double k0 = vm[0];
  for (int ax = 0; ax < D; ++ax) {
    fi.off[ax] = vm[1 + ax] / k0;          // first moments: degree-1 monomials e_1..e_D
    fi.x0h[ax] = cown[ax] + 0.5 + fi.off[ax];
  }
  if (lane < D) {
    double nu[M1];
    const double* src = gp.eb_nmom + ((long long)fi.ref * D + lane) * M1;
    static_for<0, M1>([&](auto I) { nu[I] = src[I]; });
    double dl[3] = {-fi.off[0], -fi.off[1], -fi.off[2]};   // (c - x0)/h
    recentre<D, Q - 1>(nu, dl);
    static_for<0, M1>([&](auto I) { sm.nus[lane][I] = nu[I]; });
  }
  __syncthreads();
  if (lane < M) {
    constexpr auto& T = kMono<D, Q>;
    double fv = 0.0;
    for (int ax = 0; ax < D; ++ax) {
      int e[3] = {T.e[lane][0], T.e[lane][1], T.e[lane][2]};
      const int p = e[ax];
      if (p > 0) {
        e[ax] -= 1;
        fv += p * sm.nus[ax][mono_index<D>(e[0], e[1], e[2])];
      }
    }
    sm.vec[0][lane] = fv;
  }
  __syncthreads();
}

// Rows, Gram matrix, inverse and the refined semi-normal solve of one face.  Leaves B, W,
// z and y in shared memory and -G^^-1 (row `lane`) in a[], the column
// equilibration in sdiag.  Returns the face status.
template <int D, int Q, int NPAD>
__device__ __forceinline__ int face_forward(const GridDims& g, const GeomPtrs& gp, const FaceInfo& fi,
                                            const int32_t* __restrict__ vol_cell, const int32_t* __restrict__ box_lf,
                                            const int32_t* __restrict__ col, FaceSmem<D, Q, NPAD>& sm, int lane,
                                            double* a, double& sdiag) {
  using DM = Dims<D, Q>;
  constexpr int M = DM::M, MT = DM::MT, MS = DM::MS;
  double* Bs = sm.Bs;
  double* Ls = sm.Ls;
  const int N = fi.N;

  // ---- rows of B ----------------------------------------------------------------------
  bool finite = true;
#pragma unroll 1
  for (int r = lane; r < NPAD; r += 64) {
    double m[M];
    double wr = 0.0;
    if (r < N) {
      const int64_t loc = (int64_t)col[fi.rp + r] - fi.phi0;
      finite = build_row<D, Q>(g, gp, loc, fi.n_vol, fi.n_eb, vol_cell, box_lf, fi.x0h, m, wr) && finite;
    } else {
      static_for<0, M>([&](auto I) { m[I] = 0.0; });
    }
    static_for<0, M>([&](auto I) { Bs[r * MS + I] = m[I]; });
    sm.wls[r] = wr;
    sm.zs[r] = 0.0;
  }
  __syncthreads();
  const bool allfinite = __all(finite) && __all(lane >= M || isfinite(sm.vec[0][lane < M ? lane : 0]));

  // ---- G = B^T B on the matrix cores ----------------------------------------------------
  dbl4 acc[MT][MT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < MT; ++j) acc[i][j] = dbl4{0, 0, 0, 0};
  const int lr = lane >> 4, lc = lane & 15;
#pragma unroll
  for (int k0 = 0; k0 < NPAD; k0 += 4) {
    double x[MT];
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      const int cidx = 16 * i + lc;
      x[i] = (cidx < M) ? Bs[(k0 + lr) * MS + cidx] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = i; j < MT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[i], x[j], acc[i][j], 0, 0, 0);
  }
  // tile (i, j), register q holds G[16i + lane/16 + 4q][16j + lane%16] (the output layout
  // of v_mfma_f64_16x16x4f64); each entry of the symmetric matrix is written once
  // (r <= c) together with its mirror
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = i; j < MT; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * i + lr + 4 * q, c = 16 * j + lc;
        if (r < M && c < M && r <= c) {
          Ls[r * MS + c] = acc[i][j][q];
          Ls[c * MS + r] = acc[i][j][q];
        }
      }
  __syncthreads();

  // ---- equilibrate to unit diagonal and invert: lane i holds row i ----------------------------
  // Symmetric Gauss-Jordan sweeps over the pivots k = 0..M-1 turn G^ into -G^-1 in place;
  // the pivot of step k is the k-th Schur complement pivot (L_kk^2 of the Cholesky factor),
  // which gives the rank test.  Lane k's row is the pivot row (= column, by symmetry); the
  // other lanes read it with v_readlane, so a sweep step touches neither LDS nor a barrier.
  const bool act = lane < M;
  const int li = act ? lane : 0;         // clamped index for inactive lanes' LDS reads
  sdiag = act ? 1.0 / sqrt(Ls[li * MS + li]) : 1.0;
  static_for<0, M>([&](auto J) { a[J] = act ? Ls[li * MS + J] * sdiag * readlane_f64(sdiag, J) : 0.0; });
  double pmax = 0.0, pmin = 1e300;
  static_for<0, M>([&](auto K) {
    constexpr int k = K;
    const double d = readlane_f64(a[k], k);
    const double sq = sqrt(d > 0.0 ? d : 0.0);
    pmax = fmax(pmax, sq);
    pmin = fmin(pmin, sq);
    const double rd = 1.0 / d;
    const double u = (lane == k) ? d - 1.0 : a[k];      // a_ik (before this step)
    static_for<0, M>([&](auto J) {
      constexpr int j = J;
      const double wj = (j == k) ? 1.0 - rd : readlane_f64(a[j], k) * rd;
      a[j] = fma(-u, wj, a[j]);
    });
    if (lane == k) a[k] = -rd;
  });
  const bool rankok = (pmin > kRankTol * pmax) && (pmax > 0.0);
  int st = CUTCELL_STATUS_OK;
  if (!allfinite) st = CUTCELL_STATUS_NONFINITE;
  else if (!rankok) st = CUTCELL_STATUS_RANK_DEFICIENT;

  // ---- semi-normal solve with refinement ----------------------------------------------------
  // y = G^-1 rhs with G^ = E G E (E = diag(sdiag)):  y = E (-a) (E rhs).  Lane p holds
  // component p of F~, rhs and y; lane r holds z of its rows r, r + 64.
  constexpr int NR = (NPAD + 63) / 64;
  const double fv = act ? sm.vec[0][lane] : 0.0;
  double rhs = fv * sdiag;
  double ysum = 0.0;
  double zr[NR];
  static_for<0, NR>([&](auto R) { zr[R] = 0.0; });
  for (int it = 0; it <= kRefine; ++it) {
    double t = 0.0;
    static_for<0, M>([&](auto J) { t = fma(-a[J], readlane_f64(rhs, J), t); });
    const double dy = act ? t * sdiag : 0.0;
    ysum += dy;
    // z += B dy
    static_for<0, NR>([&](auto R) {
      const int r = lane + 64 * R;
      if (r < NPAD) {
        double s0 = 0.0, s1 = 0.0;
        static_for<0, M>([&](auto J) {
          if constexpr (J % 2 == 0) s0 = fma(Bs[r * MS + J], readlane_f64(dy, J), s0);
          else s1 = fma(Bs[r * MS + J], readlane_f64(dy, J), s1);
        });
        zr[R] += s0 + s1;
      }
    });
    if (it == kRefine) break;
    // residual of B^T z = F~, equilibrated; z goes through LDS, B^T is read by columns
    static_for<0, NR>([&](auto R) {
      const int r = lane + 64 * R;
      if (r < NPAD) sm.zs[r] = zr[R];
    });
    __syncthreads();
    double res = 0.0;
    if (act) {
      double r0 = fv, r1 = 0.0, r2 = 0.0, r3 = 0.0;
#pragma unroll 4
      for (int r = 0; r < NPAD; r += 4) {
        r0 = fma(-Bs[(r + 0) * MS + lane], sm.zs[r + 0], r0);
        r1 = fma(-Bs[(r + 1) * MS + lane], sm.zs[r + 1], r1);
        r2 = fma(-Bs[(r + 2) * MS + lane], sm.zs[r + 2], r2);
        r3 = fma(-Bs[(r + 3) * MS + lane], sm.zs[r + 3], r3);
      }
      res = (r0 + r1) + (r2 + r3);
    }
    rhs = res * sdiag;
    __syncthreads();
  }
  static_for<0, NR>([&](auto R) {
    const int r = lane + 64 * R;
    if (r < NPAD) sm.zs[r] = zr[R];
  });
  if (act) sm.ys[lane] = ysum;
  __syncthreads();
  return st;
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

template <int D, int Q, int NPAD>
__global__ __launch_bounds__(64) void k_stencil(StencilArgs A, double* __restrict__ val, int8_t* __restrict__ status,
                                               int32_t* flagged) {
  constexpr int M = Dims<D, Q>::M;
  __shared__ FaceSmem<D, Q, NPAD> sm;
  const long long t = blockIdx.x;
  if (t >= A.nbin) return;
  const int lane = threadIdx.x;
  FaceInfo fi = face_info(A, t);
  const GeomPtrs gp = A.geoms[fi.gi];
  face_setup<D, Q, NPAD>(A.g, gp, fi, sm, lane);
  double a[M];
  double sdiag;
  const int st = face_forward<D, Q, NPAD>(A.g, gp, fi, A.vol_cell_ws + (long long)fi.gi * A.g.ncell,
                                          A.box_lf_ws + (long long)fi.gi * A.g.nboxslot, A.col, sm, lane, a, sdiag);
  for (int r = lane; r < fi.N; r += 64)
    val[fi.rp + r] = (st == CUTCELL_STATUS_OK) ? A.hscale * sm.wls[r] * sm.zs[r] : 0.0;
  if (lane == 0) {
    status[fi.F] = (int8_t)st;
    if (st != CUTCELL_STATUS_OK) atomicAdd(flagged, 1);
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
  face_setup<D, Q, NPAD>(A.g, gp, fi, sm, lane);
  double a[M];
  double sdiag;
  const int32_t* vol_cell = A.vol_cell_ws + (long long)fi.gi * A.g.ncell;
  const int32_t* box_lf = A.box_lf_ws + (long long)fi.gi * A.g.nboxslot;
  const int st = face_forward<D, Q, NPAD>(A.g, gp, fi, vol_cell, box_lf, A.col, sm, lane, a, sdiag);
  const bool act = lane < M;
  const double* Bs = sm.Bs;
  const int N = fi.N;
  double* yw = B.face_yw + (long long)fi.F * 2 * M;
  double* og = B.owner_grad + (long long)fi.F * 4;
  if (lane < 4) B.face_x0[(long long)fi.F * 4 + lane] = (lane < 3) ? fi.x0h[lane] : 0.0;
  if (st != CUTCELL_STATUS_OK) {   // a flagged face has s = 0 whatever its inputs: no gradient
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
  for (int it = 0; it <= kRefine; ++it) {
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
    double t = 0.0;
    static_for<0, M>([&](auto J) { t = fma(-a[J], readlane_f64(rhs, J), t); });
    if (act) wl += t * sdiag;
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
      // dW/d delta_d = -5 W delta_d / |delta|^2 outside half a cell
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
        for (int ax = 0; ax < D; ++ax) gd[ax] += wtot * (-5.0 * W * dl[ax] / d2);
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
    for (int k = 0; k < 3; ++k) sm.vec[1][lane * 3 + k] = g0[k];   // dl/d delta0 from component `lane`
  }
  __syncthreads();
  if (lane == 0) {
    // dl/dx0h = sum over rows (gdx) - dl/d delta0;  x0h_d = centre_d + m^{e_d} / m^0
    double gxh[3] = {0, 0, 0};
    for (int l = 0; l < 64; ++l)
      for (int ax = 0; ax < D; ++ax) gxh[ax] += gdx[l][ax];
    for (int c = 0; c < D; ++c)
      for (int k = 0; k < D; ++k) gxh[k] -= sm.vec[1][c * 3 + k];
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

// faces with fewer rows than monomials: zero stencil, status INSUFFICIENT_ROWS
__global__ void k_insufficient(const int32_t* __restrict__ perm, long long n, const int64_t* __restrict__ row_ptr,
                               double* val, int8_t* status, int32_t* flagged) {
  long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int32_t F = perm[t];
  for (int64_t j = row_ptr[F]; j < row_ptr[F + 1]; ++j) val[j] = 0.0;
  status[F] = CUTCELL_STATUS_INSUFFICIENT_ROWS;
  atomicAdd(flagged, 1);
}

static StencilArgs stencil_args(const Work& w, double hscale, const int32_t* perm, long long nbin,
                                const int64_t* row_ptr, const int32_t* col) {
  StencilArgs A;
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
  return A;
}

// faces with fewer rows than monomials carry no gradient
__global__ void k_insufficient_backward(const int32_t* __restrict__ perm, long long n,
                                        const int64_t* __restrict__ row_ptr, int M, BackwardArgs B) {
  long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int32_t F = perm[t];
  for (int64_t j = row_ptr[F]; j < row_ptr[F + 1]; ++j) {
    B.nz_rz[2 * j] = 0.0;
    B.nz_rz[2 * j + 1] = 0.0;
    if (B.weight_bar) B.weight_bar[j] = 0.0;
  }
  for (int p = 0; p < 2 * M; ++p) B.face_yw[(long long)F * 2 * M + p] = 0.0;
  for (int k = 0; k < 4; ++k) {
    B.owner_grad[(long long)F * 4 + k] = 0.0;
    B.face_x0[(long long)F * 4 + k] = 0.0;
  }
}

template <int D, int Q, int NPAD>
static void launch_bin(const Work& w, double hscale, const int32_t* perm, long long nbin, const int64_t* row_ptr,
                       const int32_t* col, double* val, int8_t* status, hipStream_t st, const BackwardArgs* bw) {
  if (nbin <= 0) return;
  const StencilArgs A = stencil_args(w, hscale, perm, nbin, row_ptr, col);
  if (bw)
    hipLaunchKernelGGL((k_stencil_backward<D, Q, NPAD>), dim3((unsigned)nbin), dim3(64), 0, st, A, *bw);
  else
    hipLaunchKernelGGL((k_stencil<D, Q, NPAD>), dim3((unsigned)nbin), dim3(64), 0, st, A, val, status, w.flagged);
}

template <int D, int Q>
static int dispatch_bins(const Work& w, double hscale, const int32_t* bin_count, const int64_t* row_ptr,
                         const int32_t* col, double* val, int8_t* status, hipStream_t st, const BackwardArgs* bw) {
  constexpr int M = binom(Q + D, D);
  long long start = 0;
  for (int b = 0; b < kMaxBins; ++b) {
    const long long nb = bin_count[b];
    const int32_t* p = w.perm + start;
    start += nb;
    if (nb == 0) continue;
    const int npad = kBinRows * (b + 1);
    if (npad < M) return fail(CUTCELL_E_INVALID_ARG, "internal: face with N >= M in a bin narrower than M");
    switch (npad) {
      case 16: if constexpr (M <= 16) launch_bin<D, Q, 16>(w, hscale, p, nb, row_ptr, col, val, status, st, bw); break;
      case 32: if constexpr (M <= 32) launch_bin<D, Q, 32>(w, hscale, p, nb, row_ptr, col, val, status, st, bw); break;
      case 48: launch_bin<D, Q, 48>(w, hscale, p, nb, row_ptr, col, val, status, st, bw); break;
      case 64: launch_bin<D, Q, 64>(w, hscale, p, nb, row_ptr, col, val, status, st, bw); break;
      case 80: launch_bin<D, Q, 80>(w, hscale, p, nb, row_ptr, col, val, status, st, bw); break;
      case 96: launch_bin<D, Q, 96>(w, hscale, p, nb, row_ptr, col, val, status, st, bw); break;
      case 112: launch_bin<D, Q, 112>(w, hscale, p, nb, row_ptr, col, val, status, st, bw); break;
      case 128: launch_bin<D, Q, 128>(w, hscale, p, nb, row_ptr, col, val, status, st, bw); break;
    }
  }
  const long long ninsuf = bin_count[kMaxBins];
  if (ninsuf > 0 && bw)
    hipLaunchKernelGGL(k_insufficient_backward, dim3((unsigned)((ninsuf + 255) / 256)), dim3(256), 0, st,
                       w.perm + start, ninsuf, row_ptr, (int)M, *bw);
  else if (ninsuf > 0)
    hipLaunchKernelGGL(k_insufficient, dim3((unsigned)((ninsuf + 255) / 256)), dim3(256), 0, st, w.perm + start,
                       ninsuf, row_ptr, val, status, w.flagged);
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

static int run_bins(const Work& w, const cutcell_opts& o, const int32_t* bin_count, const int64_t* row_ptr,
                    const int32_t* col, double* val, int8_t* status, hipStream_t st, const BackwardArgs* bw) {
  double hscale = 1.0;
  for (int d = 0; d < o.dim - 2; ++d) hscale *= o.h;   // h^(D-2)
  if (o.dim == 2 && o.order == 2) return dispatch_bins<2, 2>(w, hscale, bin_count, row_ptr, col, val, status, st, bw);
  if (o.dim == 2 && o.order == 4) return dispatch_bins<2, 4>(w, hscale, bin_count, row_ptr, col, val, status, st, bw);
  if (o.dim == 3 && o.order == 2) return dispatch_bins<3, 2>(w, hscale, bin_count, row_ptr, col, val, status, st, bw);
  if (o.dim == 3 && o.order == 4) return dispatch_bins<3, 4>(w, hscale, bin_count, row_ptr, col, val, status, st, bw);
  return fail(CUTCELL_E_UNSUPPORTED, "order/dimension");
}

int solve_stencils(const Work& w, const cutcell_opts& o, const int32_t* bin_count, long long n_face,
                   const int64_t* row_ptr, const int32_t* col, double* val, int8_t* status, hipStream_t st) {
  (void)n_face;
  return run_bins(w, o, bin_count, row_ptr, col, val, status, st, nullptr);
}

int backward_stencils(const Work& w, const cutcell_opts& o, const int32_t* bin_count, const int64_t* row_ptr,
                      const int32_t* col, const BackwardArgs& bw, hipStream_t st) {
  return run_bins(w, o, bin_count, row_ptr, col, nullptr, nullptr, st, &bw);
}

}  // namespace cutcell
