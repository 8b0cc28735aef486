// Rows of the per-face systems in double-double arithmetic (dd.hpp): the binomial
// re-centring of a row's moments to x0 and the division by the zeroth moment carry ~106
// bits.  For the rows of small cut cells the moments about the cell centre nearly cancel
// when shifted to x0 (a sliver at a cell's edge, next to the face), and FP64 would lose
// digits there; the Gram path takes these rows from here, the QR path all of its rows.
#pragma once

#include "dd.hpp"
#include "rows.hpp"

namespace cutcell {

// ---- double-double re-centring (the binomial theorem one direction at a time) -----------
template <int D, int Q, int DIR>
__device__ __forceinline__ void shift_dir_dd(dd* m, dd delta) {
  constexpr int M = kNMono<D, Q>;
  dd pw[Q + 1];
  pw[0] = dd_from(1.0);
  static_for<1, Q + 1>([&](auto K) { pw[K] = dd_mul(pw[K - 1], delta); });
  static_for_down<0, M>([&](auto IDX) {
    constexpr int idx = IDX;
    constexpr int pd = kMono<D, Q>.e[idx][DIR];
    dd acc = m[idx];
    static_for<0, (pd > 0 ? pd : 0)>([&](auto C) {
      constexpr int c = C;
      constexpr int a = (DIR == 0) ? c : kMono<D, Q>.e[idx][0];
      constexpr int b = (DIR == 1) ? c : kMono<D, Q>.e[idx][1];
      constexpr int cc = (DIR == 2) ? c : kMono<D, Q>.e[idx][2];
      constexpr int src = mono_index<D>(a, b, cc);
      constexpr double coef = (double)binom(pd, c);
      acc = dd_add(acc, dd_mul(dd_mul_d(pw[pd - c], coef), m[src]));
    });
    m[idx] = acc;
  });
}

template <int D, int Q>
__device__ __forceinline__ void recentre_dd(dd* m, const dd* delta) {
  shift_dir_dd<D, Q, 0>(m, delta[0]);
  if constexpr (D >= 2) shift_dir_dd<D, Q, 1>(m, delta[1]);
  if constexpr (D >= 3) shift_dir_dd<D, Q, 2>(m, delta[2]);
}

// One row of B = W A~ in double-double (as finish_row / neumann_row); W in FP64.
template <int D, int Q, bool NEU>
__device__ __forceinline__ bool dd_row(const GeomPtrs& gp, const RowSource& rs, const dd* x0, double wpow, dd* m,
                                       double& w) {
  constexpr int M = Dims<D, Q>::M, M1 = Dims<D, Q>::M1;
  dd delta[3];
  double d2 = 0.0;
  for (int ax = 0; ax < 3; ++ax) delta[ax] = dd_from(0.0);
  for (int ax = 0; ax < D; ++ax) {
    delta[ax] = dd_sub(dd_from(rs.ctr[ax]), x0[ax]);
    d2 += delta[ax].hi * delta[ax].hi;
  }
  w = row_weight(d2, wpow);
  double m0;
  if (NEU && rs.eb >= 0) {
    m0 = gp.eb_mom[(long long)rs.eb * M];
    static_for<0, M>([&](auto I) { m[I] = dd_from(0.0); });
    static_for<0, D>([&](auto AX) {
      dd nu[M1];
      const double* src = gp.eb_nmom + ((long long)rs.eb * D + AX) * M1;
      static_for<0, M1>([&](auto I) { nu[I] = dd_from(src[I]); });
      recentre_dd<D, Q - 1>(nu, delta);
      static_for<0, M>([&](auto I) {
        constexpr int pd = kMono<D, Q>.e[I][AX];
        if constexpr (pd > 0) {
          constexpr int j = mono_index<D>(kMono<D, Q>.e[I][0] - (AX == 0), kMono<D, Q>.e[I][1] - (AX == 1),
                                          kMono<D, Q>.e[I][2] - (AX == 2));
          m[I] = dd_add(m[I], dd_mul_d(nu[j], (double)pd));
        }
      });
    });
  } else {
    double raw[M];
    load_row_moments<D, Q>(rs, raw);
    m0 = raw[0];
    static_for<0, M>([&](auto I) { m[I] = dd_from(raw[I]); });
    recentre_dd<D, Q>(m, delta);
  }
  const dd sc = dd_div(dd_from(w), dd_from(m0));
  bool finite = dd_isfinite(sc);
  static_for<0, M>([&](auto I) {
    m[I] = dd_mul(m[I], sc);
    finite = finite && dd_isfinite(m[I]);
  });
  return finite;
}

}  // namespace cutcell
