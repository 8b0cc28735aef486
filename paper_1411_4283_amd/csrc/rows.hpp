// Rows of the per-face systems: where each Phi entry's moments and centre live, and the
// weights of Sec. 2.4.  Shared by the stencil solves and their adjoint.
#pragma once

#include "kernels.hpp"

namespace cutcell {

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

// Centre (in units of h) of the cell or face of Phi entry `phi_local` of one geometry and
// a pointer to its stored moments; for box faces also the face direction (else -1) and
// lattice offset.
struct RowSource {
  double ctr[3];
  const double* src;
  int dd;           // box faces: direction of the face; -1 for volumes and EB faces
  long long loc;    // box faces: index in the direction's lattice
  int32_t cell;     // volumes and EB faces: the cell
  int32_t eb;       // EB faces: the EB index; -1 otherwise
};

template <int D, int Q>
__device__ __forceinline__ RowSource row_source(const GridDims& g, const GeomPtrs& gp, int64_t phi_local,
                                                int64_t n_vol, int64_t n_eb, const int32_t* vol_cell,
                                                const int32_t* box_lf) {
  constexpr int M = Dims<D, Q>::M, Mf = Dims<D, Q>::Mf;
  RowSource rs;
  rs.ctr[0] = rs.ctr[1] = rs.ctr[2] = 0.0;
  if (phi_local < n_vol + n_eb) {
    int32_t c;
    if (phi_local < n_vol) {
      c = vol_cell[phi_local];
      rs.src = gp.vol_mom + (long long)c * M;
      rs.eb = -1;
    } else {
      const int64_t e = phi_local - n_vol;
      c = gp.eb_cell[e];
      rs.src = gp.eb_mom + e * M;
      rs.eb = (int32_t)e;
    }
    const int ci[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long long)g.n[0] * g.n[1]))};
    for (int ax = 0; ax < D; ++ax) rs.ctr[ax] = ci[ax] + 0.5;
    rs.dd = -1;
    rs.loc = -1;
    rs.cell = c;
  } else {
    const int32_t lf = box_lf[phi_local - n_vol - n_eb];
    const int dd = (lf >= g.foff[1]) + (lf >= g.foff[2]);
    const long long loc = lf - g.foff[dd];
    const int m0 = g.n[0] + (dd == 0), m1 = g.n[1] + (dd == 1);
    const int j[3] = {(int)(loc % m0), (int)((loc / m0) % m1), (int)(loc / ((long long)m0 * m1))};
    for (int ax = 0; ax < D; ++ax) rs.ctr[ax] = (ax == dd) ? (double)j[ax] : j[ax] + 0.5;
    rs.src = gp.face_mom[dd] + loc * Mf;
    rs.dd = dd;
    rs.loc = loc;
    rs.cell = -1;
    rs.eb = -1;
  }
  return rs;
}

// the row's stored moments as an M-vector (box faces: the transverse face moments, zero
// where the exponent in the face direction is positive)
template <int D, int Q>
__device__ __forceinline__ void load_row_moments(const RowSource& rs, double* m) {
  constexpr int M = Dims<D, Q>::M;
  if (rs.dd < 0) {
    static_for<0, M>([&](auto I) { m[I] = rs.src[I]; });
    return;
  }
  auto embed = [&](auto DD) {
    static_for<0, M>([&](auto I) {
      constexpr int sl = face_slot<D, Q>(I, DD);
      if constexpr (sl >= 0) m[I] = rs.src[sl];
      else m[I] = 0.0;
    });
  };
  if (rs.dd == 0) embed(std::integral_constant<int, 0>{});
  else if (rs.dd == 1) embed(std::integral_constant<int, 1>{});
  else if constexpr (D == 3) embed(std::integral_constant<int, 2>{});
}

// Weight of a row at offset delta = (x_i - x0)/h (Sec. 2.4): 1 inside half a cell, else
// (2 |delta|)^-p, p = 5 in the paper (wpow; other exponents for weight studies).
__device__ __forceinline__ double row_weight(double d2, double wpow) {
  const double dist = sqrt(d2);
  if (dist < 0.5) return 1.0;
  const double t = 2.0 * dist;
  if (wpow == 5.0) {
    const double t2 = t * t;
    return 1.0 / (t2 * t2 * t);
  }
  return pow(t, -wpow);
}

}  // namespace cutcell
