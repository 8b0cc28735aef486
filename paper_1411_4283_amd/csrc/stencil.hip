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

namespace cutcell {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr double kRankTol = 1e-7;
constexpr int kRefine = 2;

template <int D, int Q>
struct Dims {
  static constexpr int M = binom(Q + D, D);
  static constexpr int Mf = binom(Q + D - 1, D - 1);
  static constexpr int M1 = binom(Q - 1 + D, D);
  static constexpr int MT = (M + 15) / 16;   // 16-wide tiles covering M columns
  static constexpr int MS = M | 1;           // odd LDS row stride (fewer bank conflicts)
};

// transverse face-monomial index of the D-variate monomial idx when its exponent in the
// face direction dd is 0, else -1
template <int D, int Q>
__host__ __device__ constexpr int face_slot(int idx, int dd) {
  const auto& T = kMono<D, Q>;
  const int a = T.e[idx][0], b = T.e[idx][1], c = T.e[idx][2];
  if (D == 2) {
    if (dd == 0) return a == 0 ? mono_index<1>(b, 0, 0) : -1;
    return b == 0 ? mono_index<1>(a, 0, 0) : -1;
  }
  if (dd == 0) return a == 0 ? mono_index<2>(b, c, 0) : -1;
  if (dd == 1) return b == 0 ? mono_index<2>(a, c, 0) : -1;
  return c == 0 ? mono_index<2>(a, b, 0) : -1;
}

// One row of A~ about x0 (in units of h: x0h = x0 / h), with its weight and centre.
// Returns false if the row holds a non-finite value.
template <int D, int Q>
__device__ __forceinline__ bool build_row(const GridDims& g, const GeomPtrs& gp, int64_t phi_local, int64_t n_vol,
                                          int64_t n_eb, const int32_t* vol_cell, const int32_t* box_lf,
                                          const double* x0h, double* m, double& w) {
  constexpr int M = Dims<D, Q>::M, Mf = Dims<D, Q>::Mf;
  double ctr[3] = {0, 0, 0};   // row centre / h
  if (phi_local < n_vol + n_eb) {
    int32_t c;
    const double* src;
    if (phi_local < n_vol) {
      c = vol_cell[phi_local];
      src = gp.vol_mom + (long long)c * M;
    } else {
      const int64_t e = phi_local - n_vol;
      c = gp.eb_cell[e];
      src = gp.eb_mom + e * M;
    }
    const int ci[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long long)g.n[0] * g.n[1]))};
    for (int ax = 0; ax < D; ++ax) ctr[ax] = ci[ax] + 0.5;
    static_for<0, M>([&](auto I) { m[I] = src[I]; });
  } else {
    const int32_t lf = box_lf[phi_local - n_vol - n_eb];
    const int dd = (lf >= g.foff[1]) + (lf >= g.foff[2]);
    const long long loc = lf - g.foff[dd];
    const int m0 = g.n[0] + (dd == 0), m1 = g.n[1] + (dd == 1);
    const int j[3] = {(int)(loc % m0), (int)((loc / m0) % m1), (int)(loc / ((long long)m0 * m1))};
    for (int ax = 0; ax < D; ++ax) ctr[ax] = (ax == dd) ? (double)j[ax] : j[ax] + 0.5;
    const double* src = gp.face_mom[dd] + loc * Mf;
    auto embed = [&](auto DD) {
      static_for<0, M>([&](auto I) {
        constexpr int sl = face_slot<D, Q>(I, DD);
        if constexpr (sl >= 0) m[I] = src[sl];
        else m[I] = 0.0;
      });
    };
    if (dd == 0) embed(std::integral_constant<int, 0>{});
    else if (dd == 1) embed(std::integral_constant<int, 1>{});
    else if constexpr (D == 3) embed(std::integral_constant<int, 2>{});
  }
  double delta[3] = {0, 0, 0};
  double d2 = 0;
  for (int ax = 0; ax < D; ++ax) {
    delta[ax] = ctr[ax] - x0h[ax];
    d2 += delta[ax] * delta[ax];
  }
  const double dist = sqrt(d2);
  if (dist < 0.5) {
    w = 1.0;
  } else {
    const double t = 2.0 * dist;
    const double t2 = t * t;
    w = 1.0 / (t2 * t2 * t);
  }
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

template <int D, int Q, int NPAD>
__global__ __launch_bounds__(64) void k_stencil(GridDims g, int G, double hscale, const int32_t* __restrict__ perm,
                                               long long nbin, const int32_t* __restrict__ fcode,
                                               const int32_t* __restrict__ fref, const GeomPtrs* __restrict__ geoms,
                                               const int64_t* __restrict__ counts, const int64_t* __restrict__ offs,
                                               const int32_t* __restrict__ vol_cell_ws,
                                               const int32_t* __restrict__ box_lf_ws, const int64_t* __restrict__ row_ptr,
                                               const int32_t* __restrict__ col, double* __restrict__ val,
                                               int8_t* __restrict__ status, int32_t* flagged) {
  using DM = Dims<D, Q>;
  constexpr int M = DM::M, Mf = DM::Mf, M1 = DM::M1, MT = DM::MT, MS = DM::MS;
  __shared__ double Bs[NPAD * MS];
  __shared__ double Ls[M * MS];
  __shared__ double vec[2][M + 1];
  __shared__ double zs[NPAD];
  __shared__ double wls[NPAD];
  __shared__ double nus[D][M1];

  const long long t = blockIdx.x;
  if (t >= nbin) return;
  const int lane = threadIdx.x;
  const int32_t F = perm[t];
  const int32_t code = fcode[F];
  const int gi = code >> 4, kind = (code >> 2) & 3, dn = code & 3;
  const int32_t ref = fref[F];
  const GeomPtrs gp = geoms[gi];
  const int64_t n_vol = counts[4 * gi + 0], n_eb = counts[4 * gi + 1];
  const int64_t phi0 = offs[gi];
  const int32_t* vol_cell = vol_cell_ws + (long long)gi * g.ncell;
  const int32_t* box_lf = box_lf_ws + (long long)gi * g.nboxslot;
  const int64_t rp = row_ptr[F];
  const int N = (int)(row_ptr[F + 1] - rp);

  // ---- x0 (in units of h) and the flux vector F~ ------------------------------------
  double x0h[3] = {0, 0, 0};
  int cown[3] = {0, 0, 0};
  if (kind == 0) {
    const long long loc = ref - g.foff[dn];
    const int m0 = g.n[0] + (dn == 0), m1 = g.n[1] + (dn == 1);
    const int j[3] = {(int)(loc % m0), (int)((loc / m0) % m1), (int)(loc / ((long long)m0 * m1))};
    for (int ax = 0; ax < D; ++ax) x0h[ax] = (ax == dn) ? (double)j[ax] : j[ax] + 0.5;
    // F~_p = face moment of p - e_d when p_d = 1 (reference normal +e_d)
    const double* fm = gp.face_mom[dn] + loc * Mf;
    if (lane < M) {
      double fv = 0.0;
      constexpr auto& T = kMono<D, Q>;
      // lanes index the monomial table at run time (constant-memory loads)
      int e0 = T.e[lane][0], e1 = T.e[lane][1], e2 = T.e[lane][2];
      int pd = (dn == 0) ? e0 : (dn == 1 ? e1 : e2);
      if (pd == 1) {
        int s;
        if (D == 2) s = mono_index<1>(dn == 0 ? e1 : e0, 0, 0);
        else if (dn == 0) s = mono_index<2>(e1, e2, 0);
        else if (dn == 1) s = mono_index<2>(e0, e2, 0);
        else s = mono_index<2>(e0, e1, 0);
        fv = fm[s];
      }
      vec[0][lane] = fv;
    }
  } else {
    // EB face: x0 = centroid of the cut volume; the normal moments (about the cell
    // centre) are re-centred to x0 by lanes 0..D-1, one component each
    const int32_t c = gp.eb_cell[ref];
    cown[0] = (int)(c % g.n[0]);
    cown[1] = (int)((c / g.n[0]) % g.n[1]);
    cown[2] = (int)(c / ((long long)g.n[0] * g.n[1]));
    const double* vm = gp.vol_mom + (long long)c * M;
    const double k0 = vm[0];
    double off[3] = {0, 0, 0};
    for (int ax = 0; ax < D; ++ax) {
      off[ax] = vm[1 + ax] / k0;          // first moments: degree-1 monomials e_1..e_D
      x0h[ax] = cown[ax] + 0.5 + off[ax];
    }
    if (lane < D) {
      double nu[M1];
      const double* src = gp.eb_nmom + ((long long)ref * D + lane) * M1;
      static_for<0, M1>([&](auto I) { nu[I] = src[I]; });
      double dl[3] = {-off[0], -off[1], -off[2]};   // (c - x0)/h
      recentre<D, Q - 1>(nu, dl);
      static_for<0, M1>([&](auto I) { nus[lane][I] = nu[I]; });
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
          fv += p * nus[ax][mono_index<D>(e[0], e[1], e[2])];
        }
      }
      vec[0][lane] = fv;
    }
  }

  // ---- rows of B ----------------------------------------------------------------------
  bool finite = true;
#pragma unroll 1
  for (int r = lane; r < NPAD; r += 64) {
    double m[M];
    double wr = 0.0;
    if (r < N) {
      const int64_t loc = (int64_t)col[rp + r] - phi0;
      finite = build_row<D, Q>(g, gp, loc, n_vol, n_eb, vol_cell, box_lf, x0h, m, wr) && finite;
    } else {
      static_for<0, M>([&](auto I) { m[I] = 0.0; });
    }
    static_for<0, M>([&](auto I) { Bs[r * MS + I] = m[I]; });
    wls[r] = wr;
    zs[r] = 0.0;
  }
  __syncthreads();
  const bool allfinite = __all(finite) && __all(lane >= M || isfinite(vec[0][lane < M ? lane : 0]));

  // ---- G = B^T B on the matrix cores ----------------------------------------------------
  dbl4 acc[MT][MT];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < MT; ++b) acc[a][b] = dbl4{0, 0, 0, 0};
  const int lr = lane >> 4, lc = lane & 15;
#pragma unroll 2
  for (int k0 = 0; k0 < NPAD; k0 += 4) {
    double x[MT];
#pragma unroll
    for (int a = 0; a < MT; ++a) {
      const int cidx = 16 * a + lc;
      x[a] = (cidx < M) ? Bs[(k0 + lr) * MS + cidx] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int b = a; b < MT; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[a], x[b], acc[a][b], 0, 0, 0);
  }
  // tile (a, b), register q holds G[16a + lane/16 + 4q][16b + lane%16] (the output layout
  // of v_mfma_f64_16x16x4f64); each entry of the symmetric matrix is written once
  // (i <= j) together with its mirror
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = a; b < MT; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 16 * a + lr + 4 * q, j = 16 * b + lc;
        if (i < M && j < M && i <= j) {
          Ls[i * MS + j] = acc[a][b][q];
          Ls[j * MS + i] = acc[a][b][q];
        }
      }
  __syncthreads();

  // ---- equilibrate to unit diagonal and invert: lane i holds row i ----------------------------
  // Symmetric Gauss-Jordan sweeps over the pivots k = 0..M-1 turn G^ into -G^-1 in place;
  // the pivot of step k is the k-th Schur complement pivot (L_kk^2 of the Cholesky factor),
  // which gives the rank test.  The pivot row (= column, by symmetry) goes through LDS.
  const bool act = lane < M;
  const int li = act ? lane : 0;         // clamped index for inactive lanes' LDS reads
  const double sdiag = act ? 1.0 / sqrt(Ls[li * MS + li]) : 1.0;
  if (act) vec[1][lane] = sdiag;
  __syncthreads();
  double a[M];
  static_for<0, M>([&](auto J) { a[J] = act ? Ls[li * MS + J] * sdiag * vec[1][J] : 0.0; });
  __syncthreads();
  double* prow = Ls;                     // the factored matrix is no longer needed in LDS
  double pmax = 0.0, pmin = 1e300;
  static_for<0, M>([&](auto K) {
    constexpr int k = K;
    if (lane == k) static_for<0, M>([&](auto J) { prow[J] = a[J]; });
    __syncthreads();
    const double d = prow[k];
    const double sq = sqrt(d > 0.0 ? d : 0.0);
    pmax = fmax(pmax, sq);
    pmin = fmin(pmin, sq);
    const double rd = 1.0 / d;
    const double u = (lane == k) ? d - 1.0 : prow[li];   // a_ik = a_ki
    static_for<0, M>([&](auto J) {
      constexpr int j = J;
      const double wj = (j == k) ? 1.0 - rd : prow[j] * rd;
      a[j] = fma(-u, wj, a[j]);
    });
    if (lane == k) a[k] = -rd;
    __syncthreads();
  });
  const bool rankok = (pmin > kRankTol * pmax) && (pmax > 0.0);
  int st = CUTCELL_STATUS_OK;
  if (!allfinite) st = CUTCELL_STATUS_NONFINITE;
  else if (!rankok) st = CUTCELL_STATUS_RANK_DEFICIENT;

  // ---- semi-normal solve with refinement ----------------------------------------------------
  // y = G^-1 rhs with G^ = E G E (E = diag(sdiag)):  y = E (-a) (E rhs)
  if (act) vec[1][lane] = vec[0][lane] * sdiag;      // E F~
  __syncthreads();
  for (int it = 0; it <= kRefine; ++it) {
    double y = 0.0;
    static_for<0, M>([&](auto J) { y = fma(-a[J], vec[1][J], y); });
    __syncthreads();
    if (act) vec[1][lane] = y * sdiag;
    __syncthreads();
    // z += B y
#pragma unroll 1
    for (int r = lane; r < NPAD; r += 64) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < M; ++j) s = fma(Bs[r * MS + j], vec[1][j], s);
      zs[r] += s;
    }
    __syncthreads();
    if (it == kRefine) break;
    // residual of B^T z = F~, equilibrated
    double res = 0.0;
    if (act) {
      res = vec[0][lane];
      for (int r = 0; r < N; ++r) res = fma(-Bs[r * MS + lane], zs[r], res);
    }
    __syncthreads();
    if (act) vec[1][lane] = res * sdiag;
    __syncthreads();
  }

  // ---- outputs ---------------------------------------------------------------------------
  for (int r = lane; r < N; r += 64) val[rp + r] = (st == CUTCELL_STATUS_OK) ? hscale * wls[r] * zs[r] : 0.0;
  if (lane == 0) {
    status[F] = (int8_t)st;
    if (st != CUTCELL_STATUS_OK) atomicAdd(flagged, 1);
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

template <int D, int Q, int NPAD>
static void launch_bin(const Work& w, double hscale, const int32_t* perm, long long nbin, const int64_t* row_ptr,
                       const int32_t* col, double* val, int8_t* status, hipStream_t st) {
  if (nbin <= 0) return;
  hipLaunchKernelGGL((k_stencil<D, Q, NPAD>), dim3((unsigned)nbin), dim3(64), 0, st, w.dims, w.G, hscale, perm, nbin,
                     w.fcode, w.fref, w.geoms, w.counts, w.offs, w.vol_cell, w.box_lf, row_ptr, col, val, status,
                     w.flagged);
}

template <int D, int Q>
static int dispatch_bins(const Work& w, double hscale, const int32_t* bin_count, const int64_t* row_ptr,
                         const int32_t* col, double* val, int8_t* status, hipStream_t st) {
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
      case 16: if constexpr (M <= 16) launch_bin<D, Q, 16>(w, hscale, p, nb, row_ptr, col, val, status, st); break;
      case 32: if constexpr (M <= 32) launch_bin<D, Q, 32>(w, hscale, p, nb, row_ptr, col, val, status, st); break;
      case 48: launch_bin<D, Q, 48>(w, hscale, p, nb, row_ptr, col, val, status, st); break;
      case 64: launch_bin<D, Q, 64>(w, hscale, p, nb, row_ptr, col, val, status, st); break;
      case 80: launch_bin<D, Q, 80>(w, hscale, p, nb, row_ptr, col, val, status, st); break;
      case 96: launch_bin<D, Q, 96>(w, hscale, p, nb, row_ptr, col, val, status, st); break;
      case 112: launch_bin<D, Q, 112>(w, hscale, p, nb, row_ptr, col, val, status, st); break;
      case 128: launch_bin<D, Q, 128>(w, hscale, p, nb, row_ptr, col, val, status, st); break;
    }
  }
  const long long ninsuf = bin_count[kMaxBins];
  if (ninsuf > 0)
    hipLaunchKernelGGL(k_insufficient, dim3((unsigned)((ninsuf + 255) / 256)), dim3(256), 0, st, w.perm + start,
                       ninsuf, row_ptr, val, status, w.flagged);
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

int solve_stencils(const Work& w, const cutcell_opts& o, const int32_t* bin_count, long long n_face,
                   const int64_t* row_ptr, const int32_t* col, double* val, int8_t* status, hipStream_t st) {
  (void)n_face;
  double hscale = 1.0;
  for (int d = 0; d < o.dim - 2; ++d) hscale *= o.h;   // h^(D-2)
  if (o.dim == 2 && o.order == 2) return dispatch_bins<2, 2>(w, hscale, bin_count, row_ptr, col, val, status, st);
  if (o.dim == 2 && o.order == 4) return dispatch_bins<2, 4>(w, hscale, bin_count, row_ptr, col, val, status, st);
  if (o.dim == 3 && o.order == 2) return dispatch_bins<3, 2>(w, hscale, bin_count, row_ptr, col, val, status, st);
  if (o.dim == 3 && o.order == 4) return dispatch_bins<3, 4>(w, hscale, bin_count, row_ptr, col, val, status, st);
  return fail(CUTCELL_E_UNSUPPORTED, "order/dimension");
}

}  // namespace cutcell
