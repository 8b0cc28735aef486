// Internal definitions shared by the library's HIP sources (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <type_traits>

#include "../../include/cutcell.h"

namespace cutcell {

// ---- errors -----------------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
#define CC_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::cutcell::fail(CUTCELL_E_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

// ---- compile-time monomial tables ---------------------------------------------------
constexpr int binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  int r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Graded order: degree ascending; inside a degree p_1 descending, then p_2 descending.
template <int D, int Q>
struct Mono {
  static constexpr int M = binom(Q + D, D);
  int e[M][3];
  constexpr Mono() : e{} {
    int n = 0;
    for (int g = 0; g <= Q; ++g) {
      if (D == 1) {
        e[n][0] = g; e[n][1] = 0; e[n][2] = 0; ++n;
      } else if (D == 2) {
        for (int a = g; a >= 0; --a) { e[n][0] = a; e[n][1] = g - a; e[n][2] = 0; ++n; }
      } else {
        for (int a = g; a >= 0; --a)
          for (int b = g - a; b >= 0; --b) { e[n][0] = a; e[n][1] = b; e[n][2] = g - a - b; ++n; }
      }
    }
  }
};

// position of the multi-index (a, b, c) in the graded order of D variables
template <int D>
__host__ __device__ constexpr int mono_index(int a, int b, int c) {
  if (D == 1) return a;
  if (D == 2) {
    int g = a + b;
    return g * (g + 1) / 2 + (g - a);
  }
  int g = a + b + c;
  return g * (g + 1) * (g + 2) / 6 + (g - a) * (g - a + 1) / 2 + (g - a - b);
}

template <int D, int Q>
inline constexpr Mono<D, Q> kMono{};

template <int D, int Q>
inline constexpr int kNMono = binom(Q + D, D);

// ---- compile-time loops ------------------------------------------------------------------
// Register arrays stay in registers only if every index is a constant when the compiler
// first sees the code; static_for hands the body a compile-time index.
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for_down(F&& f) {   // I = N-1, ..., 0
  if constexpr (N > 0) {
    f(std::integral_constant<int, N - 1>{});
    static_for_down<I, N - 1>(f);
  }
}

// ---- binomial re-centring of moments in registers -------------------------------------
// m holds moments about c in graded order; on return, moments about x0, where
// delta = (c - x0)/h:  m^p(x0) = sum_{q<=p} C(p,q) delta^(p-q) m^q(c), applied one
// direction at a time (the multi-index binomial theorem factorises over directions).
// Higher degrees are updated first, so within a line of fixed other exponents the
// entries with smaller p_DIR are still the unshifted ones when they are read.
template <int D, int Q, int DIR>
__device__ __forceinline__ void shift_dir(double* m, double delta) {
  constexpr int M = kNMono<D, Q>;
  double pw[Q + 1];
  pw[0] = 1.0;
  static_for<1, Q + 1>([&](auto K) { pw[K] = pw[K - 1] * delta; });
  static_for_down<0, M>([&](auto IDX) {
    constexpr int idx = IDX;
    constexpr int pd = kMono<D, Q>.e[idx][DIR];
    double acc = m[idx];
    static_for<0, (pd > 0 ? pd : 0)>([&](auto C) {
      constexpr int c = C;
      constexpr int a = (DIR == 0) ? c : kMono<D, Q>.e[idx][0];
      constexpr int b = (DIR == 1) ? c : kMono<D, Q>.e[idx][1];
      constexpr int cc = (DIR == 2) ? c : kMono<D, Q>.e[idx][2];
      constexpr int src = mono_index<D>(a, b, cc);
      constexpr double coef = (double)binom(pd, c);
      acc = __builtin_fma(coef * pw[pd - c], m[src], acc);
    });
    m[idx] = acc;
  });
}

template <int D, int Q>
__device__ __forceinline__ void recentre(double* m, const double* delta) {
  shift_dir<D, Q, 0>(m, delta[0]);
  if constexpr (D >= 2) shift_dir<D, Q, 1>(m, delta[1]);
  if constexpr (D >= 3) shift_dir<D, Q, 2>(m, delta[2]);
}

// Transpose of the re-centring: a^T S(delta) = (S(delta)^T a)^T, used by the adjoint.
// (S^T a)_q = sum_{p >= q} C(p,q) delta^(p-q) a_p, one direction at a time; lower degrees
// first, so the entries with a larger exponent in the line are still unchanged when read.
template <int D, int Q, int DIR>
__device__ __forceinline__ void shift_dir_T(double* a, double delta) {
  constexpr int M = kNMono<D, Q>;
  double pw[Q + 1];
  pw[0] = 1.0;
  static_for<1, Q + 1>([&](auto K) { pw[K] = pw[K - 1] * delta; });
  static_for<0, M>([&](auto IDX) {
    constexpr int idx = IDX;
    constexpr int qd = kMono<D, Q>.e[idx][DIR];
    constexpr int deg = kMono<D, Q>.e[idx][0] + kMono<D, Q>.e[idx][1] + kMono<D, Q>.e[idx][2];
    double acc = a[idx];
    static_for<1, Q - deg + 1>([&](auto T) {        // c = qd + t, t >= 1
      constexpr int t = T;
      constexpr int c = qd + t;
      constexpr int ea = (DIR == 0) ? c : kMono<D, Q>.e[idx][0];
      constexpr int eb = (DIR == 1) ? c : kMono<D, Q>.e[idx][1];
      constexpr int ec = (DIR == 2) ? c : kMono<D, Q>.e[idx][2];
      constexpr int src = mono_index<D>(ea, eb, ec);
      constexpr double coef = (double)binom(c, qd);
      acc = __builtin_fma(coef * pw[t], a[src], acc);
    });
    a[idx] = acc;
  });
}

template <int D, int Q>
__device__ __forceinline__ void recentre_T(double* a, const double* delta) {
  if constexpr (D >= 3) shift_dir_T<D, Q, 2>(a, delta[2]);
  if constexpr (D >= 2) shift_dir_T<D, Q, 1>(a, delta[1]);
  shift_dir_T<D, Q, 0>(a, delta[0]);
}

// ---- grid geometry -------------------------------------------------------------------
struct GridDims {
  int D;
  int n[3];
  long long ncell;
  long long nface[3];   // lattice faces per direction
  long long foff[4];    // offsets of the directions in the concatenated face lattice
  long long NF;         // total lattice faces
  long long nboxslot;   // cells adjacent to the box boundary, counted per (d, side)
  long long boxoff[7];  // offsets of the (d, side) slabs in the box slot space
};

inline GridDims make_dims(const cutcell_opts& o) {
  GridDims g{};
  g.D = o.dim;
  for (int d = 0; d < 3; ++d) g.n[d] = (d < o.dim) ? o.n[d] : 1;
  g.ncell = (long long)g.n[0] * g.n[1] * g.n[2];
  g.foff[0] = 0;
  for (int d = 0; d < 3; ++d) {
    long long m = 1;
    for (int e = 0; e < 3; ++e) m *= (e == d && d < o.dim) ? g.n[e] + 1 : g.n[e];
    g.nface[d] = (d < o.dim) ? m : 0;
    g.foff[d + 1] = g.foff[d] + g.nface[d];
  }
  g.NF = g.foff[3];
  g.boxoff[0] = 0;
  for (int s = 0; s < 6; ++s) {
    int d = s / 2;
    long long m = (d < o.dim) ? g.ncell / g.n[d] : 0;
    g.boxoff[s + 1] = g.boxoff[s] + m;
  }
  g.nboxslot = g.boxoff[6];
  return g;
}

// device copy of the per-geometry input pointers
struct GeomPtrs {
  const double* vol_mom;
  const double* face_mom[3];
  const int32_t* eb_cell;
  const double* eb_mom;
  const double* eb_nmom;
  int32_t n_eb;
};

// ---- wave helpers ----------------------------------------------------------------------
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ unsigned long long lanes_below(int lane) {
  return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

}  // namespace cutcell
