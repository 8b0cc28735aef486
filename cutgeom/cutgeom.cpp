// Cut-cell geometry for level-set domains: the input generator of the flux-stencil
// library's tests and benchmark. It is not part of the stencil method; it supplies the
// volume, face and embedded-boundary (EB) moments that the method consumes, plus exact
// integrals of analytic test fields.
//
// Quadrature over {psi > 0} inside a box and over {psi = 0} inside a box uses the
// dimension-by-dimension height-function recursion of R. I. Saye, "High-order
// quadrature methods for implicitly defined surfaces and volumes in hyperrectangles",
// SIAM J. Sci. Comput. 37(2), 2015: pick a height direction in which psi is monotone,
// restrict psi to the two box faces normal to it, integrate recursively over the
// lower-dimensional box split at the zero sets of those restrictions, and integrate
// along the height direction between the roots with Gauss-Legendre.
//
// Moments are scaled as the library's header states: coordinates (x - c)/h about the
// Cartesian cell (or face) centre c, integrals divided by h^D (volumes) or h^(D-1)
// (faces, EB), so the zeroth volume moment is the volume fraction kappa and the zeroth
// face moment the area fraction alpha.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <vector>

namespace {

enum Kind { BALL = 0, HALFSPACE = 1, STAR2 = 2, SH3 = 3 };

struct Shape {
  int kind = 0, dim = 2;
  double fsign = 1.0;           // fluid is {fsign * phi0 > 0}
  double c[3] = {0, 0, 0};      // centre (ball, star, SH body)
  double r = 0, amp = 0;        // radius; star amplitude
  int k = 0;                    // star petals
  double nrm[3] = {0, 0, 0}, off = 0;   // half-space phi0 = n.x - off
  double sh[16] = {0};          // SH body: R(u) = r + sum sh[j] Y_j(u)
  double H = 0;                 // bound on the Hessian norm of phi0
  bool radial = false;          // star-shaped about c: phi0 < 0 iff rho < R(u)
  double Rmin = 0, Rmax = 0;
};

// ---- real spherical harmonics, l <= 3, orthonormal, order (l, m = -l..l) -------
void sh_eval(const double* u, double* Y, double (*dY)[3]) {
  const double x = u[0], y = u[1], z = u[2];
  const double c0 = 0.28209479177387814, c1 = 0.4886025119029199;
  const double c2a = 1.0925484305920792, c20 = 0.31539156525252005, c22 = 0.5462742152960396;
  const double c33 = 0.5900435899266435, c32 = 2.890611442640554, c31 = 0.4570457994644658;
  const double c30 = 0.3731763325901154, c32b = 1.445305721320277;
  double v[16] = {
      c0,
      c1 * y, c1 * z, c1 * x,
      c2a * x * y, c2a * y * z, c20 * (3 * z * z - 1), c2a * x * z, c22 * (x * x - y * y),
      c33 * y * (3 * x * x - y * y), c32 * x * y * z, c31 * y * (5 * z * z - 1),
      c30 * (5 * z * z * z - 3 * z), c31 * x * (5 * z * z - 1), c32b * z * (x * x - y * y),
      c33 * x * (x * x - 3 * y * y)};
  for (int j = 0; j < 16; ++j) Y[j] = v[j];
  if (!dY) return;
  double g[16][3] = {
      {0, 0, 0},
      {0, c1, 0}, {0, 0, c1}, {c1, 0, 0},
      {c2a * y, c2a * x, 0}, {0, c2a * z, c2a * y}, {0, 0, c20 * 6 * z}, {c2a * z, 0, c2a * x},
      {c22 * 2 * x, -c22 * 2 * y, 0},
      {c33 * 6 * x * y, c33 * (3 * x * x - 3 * y * y), 0},
      {c32 * y * z, c32 * x * z, c32 * x * y},
      {0, c31 * (5 * z * z - 1), c31 * 10 * y * z},
      {0, 0, c30 * (15 * z * z - 3)},
      {c31 * (5 * z * z - 1), 0, c31 * 10 * x * z},
      {c32b * 2 * x * z, -c32b * 2 * y * z, c32b * (x * x - y * y)},
      {c33 * (3 * x * x - 3 * y * y), -c33 * 6 * x * y, 0}};
  for (int j = 0; j < 16; ++j)
    for (int d = 0; d < 3; ++d) dY[j][d] = g[j][d];
}

// phi0 and its gradient (before the fluid sign)
double phi0(const Shape& S, const double* x, double* g) {
  const int D = S.dim;
  switch (S.kind) {
    case BALL: {
      double s = 0;
      for (int d = 0; d < D; ++d) {
        double t = x[d] - S.c[d];
        s += t * t;
        if (g) g[d] = t / S.r;
      }
      return (s - S.r * S.r) / (2 * S.r);
    }
    case HALFSPACE: {
      double s = -S.off;
      for (int d = 0; d < D; ++d) {
        s += S.nrm[d] * x[d];
        if (g) g[d] = S.nrm[d];
      }
      return s;
    }
    case STAR2: {
      double dx = x[0] - S.c[0], dy = x[1] - S.c[1];
      double rho = std::sqrt(dx * dx + dy * dy);
      double th = std::atan2(dy, dx);
      double R = S.r + S.amp * std::cos(S.k * th);
      if (g) {
        double Rp = -S.amp * S.k * std::sin(S.k * th);
        double r2 = rho * rho;
        // grad theta = (-dy, dx)/rho^2
        g[0] = dx / rho + Rp * dy / r2;
        g[1] = dy / rho - Rp * dx / r2;
      }
      return rho - R;
    }
    case SH3: {
      double v[3] = {x[0] - S.c[0], x[1] - S.c[1], x[2] - S.c[2]};
      double rho = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      double u[3] = {v[0] / rho, v[1] / rho, v[2] / rho};
      double Y[16], dY[16][3];
      sh_eval(u, Y, g ? dY : nullptr);
      double R = S.r;
      double gp[3] = {0, 0, 0};
      for (int j = 0; j < 16; ++j) {
        R += S.sh[j] * Y[j];
        if (g)
          for (int d = 0; d < 3; ++d) gp[d] += S.sh[j] * dY[j][d];
      }
      if (g) {
        double ug = u[0] * gp[0] + u[1] * gp[1] + u[2] * gp[2];
        for (int d = 0; d < 3; ++d) g[d] = u[d] - (gp[d] - ug * u[d]) / rho;
      }
      return rho - R;
    }
  }
  return 0;
}

inline double psi(const Shape& S, const double* x, double* g) {
  double v = phi0(S, x, g);
  if (g)
    for (int d = 0; d < S.dim; ++d) g[d] *= S.fsign;
  return S.fsign * v;
}

// Zeros of psi count as fluid everywhere (root detection, segment signs, surface
// points): next to a tangency psi rounds to exactly 0 over a small interval, and one
// tie rule keeps volumes and surfaces of neighbouring cells consistent.
inline bool fluid(double v) { return v >= 0; }
inline bool changes(double fa, double fb) { return fluid(fa) != fluid(fb); }

// Bounds of psi over the box [lo, hi] (degenerate coordinates allowed).
void psi_bounds(const Shape& S, const double* lo, const double* hi, double& vmin, double& vmax) {
  const int D = S.dim;
  if (S.radial) {
    double dmin2 = 0, dmax2 = 0;
    for (int d = 0; d < D; ++d) {
      double a = lo[d] - S.c[d], b = hi[d] - S.c[d];
      double n = (a > 0) ? a : ((b < 0) ? -b : 0.0);
      double f = std::max(std::fabs(a), std::fabs(b));
      dmin2 += n * n;
      dmax2 += f * f;
    }
    if (std::sqrt(dmax2) < S.Rmin) {  // entirely inside the body: phi0 < 0
      vmin = vmax = -S.fsign;
      return;
    }
    if (std::sqrt(dmin2) > S.Rmax) {
      vmin = vmax = S.fsign;
      return;
    }
  }
  double m[3] = {0, 0, 0}, rr[3] = {0, 0, 0}, g[3] = {0, 0, 0};
  for (int d = 0; d < D; ++d) {
    m[d] = 0.5 * (lo[d] + hi[d]);
    rr[d] = 0.5 * (hi[d] - lo[d]);
  }
  double v = psi(S, m, g);
  double del = 0, r2 = 0;
  for (int d = 0; d < D; ++d) {
    del += std::fabs(g[d]) * rr[d];
    r2 += rr[d] * rr[d];
  }
  del += 0.5 * S.H * r2;
  vmin = v - del;
  vmax = v + del;
}

// Bounds of d psi / d x_k over the box.
void dpsi_bounds(const Shape& S, const double* lo, const double* hi, int k, double& gmin, double& gmax) {
  const int D = S.dim;
  double m[3] = {0, 0, 0}, g[3] = {0, 0, 0}, r2 = 0;
  for (int d = 0; d < D; ++d) {
    m[d] = 0.5 * (lo[d] + hi[d]);
    double t = 0.5 * (hi[d] - lo[d]);
    r2 += t * t;
  }
  psi(S, m, g);
  double del = S.H * std::sqrt(r2);
  gmin = g[k] - del;
  gmax = g[k] + del;
}

// ---- Gauss-Legendre on [-1, 1] ---------------------------------------------------
struct Gauss {
  std::vector<double> x, w;
  explicit Gauss(int q) : x(q), w(q) {
    for (int i = 0; i < q; ++i) {
      double t = std::cos(M_PI * (i + 0.75) / (q + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p0 = 1, p1 = t;
        for (int n = 2; n <= q; ++n) {
          double p2 = ((2 * n - 1) * t * p1 - (n - 1) * p0) / n;
          p0 = p1;
          p1 = p2;
        }
        double dp = q * (t * p1 - p0) / (t * t - 1);
        double dt = p1 / dp;
        t -= dt;
        if (std::fabs(dt) < 1e-16) {
          // final derivative at converged t
          p0 = 1; p1 = t;
          for (int n = 2; n <= q; ++n) {
            double p2 = ((2 * n - 1) * t * p1 - (n - 1) * p0) / n;
            p0 = p1;
            p1 = p2;
          }
          dp = q * (t * p1 - p0) / (t * t - 1);
          w[i] = 2.0 / ((1 - t * t) * dp * dp);
          break;
        }
      }
      x[i] = t;
    }
  }
};

// ---- quadrature recursion ------------------------------------------------------
struct Fn {           // psi with the coordinates in `mask` fixed to `val`
  unsigned mask = 0;
  double val[3] = {0, 0, 0};
  int sign = 0;       // +1: require psi > 0, -1: psi < 0, 0: no constraint (splitting only)
};

using Emit = std::function<void(double*, double)>;  // point (free coords set), weight

struct Ctx {
  const Shape* S;
  const Gauss* G;
  int maxdepth = 36;
  int err = 0;
};

inline void fill(const Fn& f, const double* x, double* y, int D) {
  for (int d = 0; d < D; ++d) y[d] = ((f.mask >> d) & 1u) ? f.val[d] : x[d];
}

inline void fbox(const Fn& f, const double* lo, const double* hi, double* blo, double* bhi, int D) {
  for (int d = 0; d < D; ++d) {
    if ((f.mask >> d) & 1u) blo[d] = bhi[d] = f.val[d];
    else { blo[d] = lo[d]; bhi[d] = hi[d]; }
  }
}

// psi along x_k with the other coordinates from y; value and derivative
inline double line_eval(const Shape& S, double* y, int k, double t, double* dv) {
  double g[3];
  y[k] = t;
  double v = psi(S, y, g);
  if (dv) *dv = g[k];
  return v;
}

// root of a sign-changing monotone bracket [a, b] (safeguarded Newton)
double bracket_root(const Shape& S, double* y, int k, double a, double b, double fa, double fb) {
  if (fa == 0) return a;
  if (fb == 0 && !fluid(fa)) return b;
  double t = a - fa * (b - a) / (fb - fa);
  if (!(t > a && t < b)) t = 0.5 * (a + b);
  for (int it = 0; it < 200; ++it) {
    double df;
    double ft = line_eval(S, y, k, t, &df);
    if (fluid(ft) == fluid(fa)) { a = t; fa = ft; } else { b = t; fb = ft; }
    double tn = (df != 0) ? t - ft / df : 0.5 * (a + b);
    if (!(tn > a && tn < b)) tn = 0.5 * (a + b);
    if (std::fabs(tn - t) <= 2e-16 * std::max(1.0, std::fabs(t)) || (b - a) <= 4e-16 * std::max(1.0, std::fabs(t)))
      return tn;
    t = tn;
  }
  return t;
}

// all roots of psi along x_k in (a, b); subdivides until monotone
void all_roots(const Shape& S, double* y, int k, double a, double b, int depth, std::vector<double>& out) {
  double m = 0.5 * (a + b), hw = 0.5 * (b - a);
  double dm;
  double fm = line_eval(S, y, k, m, &dm);
  if (std::fabs(fm) > std::fabs(dm) * hw + 0.5 * S.H * hw * hw) return;  // no root possible
  bool mono = std::fabs(dm) > S.H * hw;
  if (mono || depth > 48) {
    double fa = line_eval(S, y, k, a, nullptr), fb = line_eval(S, y, k, b, nullptr);
    if (changes(fa, fb)) out.push_back(bracket_root(S, y, k, a, b, fa, fb));
    return;
  }
  all_roots(S, y, k, a, m, depth + 1, out);
  all_roots(S, y, k, m, b, depth + 1, out);
}

void tensor(const Ctx& C, unsigned freem, const double* lo, const double* hi, double* x, double w, int d0,
            const Emit& emit) {
  const int D = C.S->dim;
  int d = d0;
  while (d < D && !((freem >> d) & 1u)) ++d;
  if (d >= D) { emit(x, w); return; }
  const Gauss& G = *C.G;
  double a = lo[d], b = hi[d], hw = 0.5 * (b - a), mid = 0.5 * (a + b);
  for (size_t i = 0; i < G.x.size(); ++i) {
    x[d] = mid + hw * G.x[i];
    tensor(C, freem, lo, hi, x, w * hw * G.w[i], d + 1, emit);
  }
}

// Integrate along x_k over [a, b] at the point x, keeping the pieces where every
// constrained function has its sign; emits Gauss points.
void line_pieces(const Ctx& C, const std::vector<Fn>& fns, double* x, int k, double a, double b, double w,
                 bool monotone, const Emit& emit) {
  const Shape& S = *C.S;
  const int D = S.dim;
  double roots[64];
  int nr = 0;
  std::vector<double> tmp;
  for (const Fn& f : fns) {
    double y[3];
    fill(f, x, y, D);
    if (monotone) {
      double fa = line_eval(S, y, k, a, nullptr), fb = line_eval(S, y, k, b, nullptr);
      if (changes(fa, fb)) {
        if (nr < 64) roots[nr++] = bracket_root(S, y, k, a, b, fa, fb);
      }
    } else {
      tmp.clear();
      all_roots(S, y, k, a, b, 0, tmp);
      for (double t : tmp)
        if (nr < 64) roots[nr++] = t;
    }
  }
  std::sort(roots, roots + nr);
  double pts[66];
  int np = 0;
  pts[np++] = a;
  for (int i = 0; i < nr; ++i)
    if (roots[i] > a && roots[i] < b) pts[np++] = roots[i];
  pts[np++] = b;
  const Gauss& G = *C.G;
  for (int s = 0; s + 1 < np; ++s) {
    double lo = pts[s], hi = pts[s + 1];
    if (!(hi > lo)) continue;
    double mid = 0.5 * (lo + hi), hw = 0.5 * (hi - lo);
    bool ok = true;
    for (const Fn& f : fns) {
      if (f.sign == 0) continue;
      double y[3];
      fill(f, x, y, D);
      y[k] = mid;
      double v = psi(S, y, nullptr);
      if ((f.sign > 0 && !fluid(v)) || (f.sign < 0 && fluid(v))) { ok = false; break; }
    }
    if (!ok) continue;
    for (size_t i = 0; i < G.x.size(); ++i) {
      x[k] = mid + hw * G.x[i];
      emit(x, w * hw * G.w[i]);
    }
  }
}

void quad(Ctx& C, unsigned freem, const double* lo, const double* hi, const std::vector<Fn>& fns_in, int depth,
          const Emit& emit) {
  const Shape& S = *C.S;
  const int D = S.dim;
  std::vector<Fn> fns;
  for (const Fn& f : fns_in) {
    double blo[3], bhi[3], vmin, vmax;
    fbox(f, lo, hi, blo, bhi, D);
    psi_bounds(S, blo, bhi, vmin, vmax);
    if (vmin > 0) { if (f.sign < 0) return; continue; }
    if (vmax < 0) { if (f.sign > 0) return; continue; }
    fns.push_back(f);
  }
  double x[3] = {0, 0, 0};
  for (int d = 0; d < D; ++d) x[d] = 0.5 * (lo[d] + hi[d]);
  if (fns.empty()) { tensor(C, freem, lo, hi, x, 1.0, 0, emit); return; }
  int nfree = __builtin_popcount(freem);
  if (nfree == 1) {
    int k = __builtin_ctz(freem);
    line_pieces(C, fns, x, k, lo[k], hi[k], 1.0, false, emit);
    return;
  }
  // height direction: largest gradient component of the first function at the centre
  double y[3] = {0, 0, 0}, g[3] = {0, 0, 0};
  fill(fns[0], x, y, D);
  psi(S, y, g);
  int k = -1;
  double best = -1;
  for (int d = 0; d < D; ++d)
    if (((freem >> d) & 1u) && std::fabs(g[d]) > best) { best = std::fabs(g[d]); k = d; }
  bool mono = true;
  for (const Fn& f : fns) {
    double blo[3], bhi[3], gmin, gmax;
    fbox(f, lo, hi, blo, bhi, D);
    dpsi_bounds(S, blo, bhi, k, gmin, gmax);
    if (!(gmin > 0 || gmax < 0)) { mono = false; break; }
  }
  if (!mono) {
    if (depth >= C.maxdepth) {
      // No monotone direction even in a box 2^-maxdepth of the cell: psi has a
      // critical point on its zero set here (a tangency).  Fall back to Gauss points
      // that each satisfy the sign conditions; the box's measure is negligible.
      tensor(C, freem, lo, hi, x, 1.0, 0, [&](double* xp, double w) {
        for (const Fn& f : fns) {
          if (f.sign == 0) continue;
          double y[3];
          fill(f, xp, y, D);
          double v = psi(S, y, nullptr);
          if ((f.sign > 0 && !fluid(v)) || (f.sign < 0 && fluid(v))) return;
        }
        emit(xp, w);
      });
      return;
    }
    int sd = -1;
    double w = -1;
    for (int d = 0; d < D; ++d)
      if (((freem >> d) & 1u) && hi[d] - lo[d] > w) { w = hi[d] - lo[d]; sd = d; }
    double mid = 0.5 * (lo[sd] + hi[sd]);
    double lo2[3], hi2[3];
    std::memcpy(lo2, lo, sizeof lo2);
    std::memcpy(hi2, hi, sizeof hi2);
    hi2[sd] = mid;
    quad(C, freem, lo2, hi2, fns, depth + 1, emit);
    std::memcpy(hi2, hi, sizeof hi2);
    lo2[sd] = mid;
    quad(C, freem, lo2, hi2, fns, depth + 1, emit);
    return;
  }
  std::vector<Fn> child;
  for (const Fn& f : fns) {
    Fn a = f;
    a.mask |= 1u << k;
    a.sign = 0;
    a.val[k] = lo[k];
    child.push_back(a);
    a.val[k] = hi[k];
    child.push_back(a);
  }
  const double a = lo[k], b = hi[k];
  quad(C, freem & ~(1u << k), lo, hi, child, depth, [&](double* xp, double w) {
    line_pieces(C, fns, xp, k, a, b, w, true, emit);
  });
}

// Surface {psi = 0} inside the box; emits point, weight (area element) and the unit
// normal pointing out of the fluid region {psi > 0}.
using EmitS = std::function<void(double*, double, const double*)>;

void surf(Ctx& C, const double* lo, const double* hi, int depth, const EmitS& emit) {
  const Shape& S = *C.S;
  const int D = S.dim;
  double vmin, vmax;
  psi_bounds(S, lo, hi, vmin, vmax);
  if (vmin > 0 || vmax < 0) return;
  double x[3] = {0, 0, 0}, g[3];
  for (int d = 0; d < D; ++d) x[d] = 0.5 * (lo[d] + hi[d]);
  psi(S, x, g);
  int k = 0;
  for (int d = 1; d < D; ++d)
    if (std::fabs(g[d]) > std::fabs(g[k])) k = d;
  double gmin, gmax;
  dpsi_bounds(S, lo, hi, k, gmin, gmax);
  if (!(gmin > 0 || gmax < 0)) {
    if (depth >= C.maxdepth) return;   // tangency: the surface inside this tiny box is dropped
    int sd = 0;
    for (int d = 1; d < D; ++d)
      if (hi[d] - lo[d] > hi[sd] - lo[sd]) sd = d;
    double mid = 0.5 * (lo[sd] + hi[sd]);
    double lo2[3], hi2[3];
    std::memcpy(lo2, lo, sizeof lo2);
    std::memcpy(hi2, hi, sizeof hi2);
    hi2[sd] = mid;
    surf(C, lo2, hi2, depth + 1, emit);
    std::memcpy(hi2, hi, sizeof hi2);
    lo2[sd] = mid;
    surf(C, lo2, hi2, depth + 1, emit);
    return;
  }
  std::vector<Fn> child(2);
  child[0].mask = child[1].mask = 1u << k;
  child[0].val[k] = lo[k];
  child[1].val[k] = hi[k];
  unsigned freem = ((1u << D) - 1u) & ~(1u << k);
  const double a = lo[k], b = hi[k];
  quad(C, freem, lo, hi, child, depth, [&](double* xp, double w) {
    double y[3];
    for (int d = 0; d < D; ++d) y[d] = xp[d];
    double fa = line_eval(S, y, k, a, nullptr), fb = line_eval(S, y, k, b, nullptr);
    if (!changes(fa, fb)) return;
    double t = bracket_root(S, y, k, a, b, fa, fb);
    y[k] = t;
    double gg[3], gn = 0;
    psi(S, y, gg);
    for (int d = 0; d < D; ++d) gn += gg[d] * gg[d];
    gn = std::sqrt(gn);
    double n[3] = {0, 0, 0};
    for (int d = 0; d < D; ++d) n[d] = -gg[d] / gn;
    emit(y, w * gn / std::fabs(gg[k]), n);
  });
}

// ---- monomials ------------------------------------------------------------------
// Graded order: total degree ascending; within a degree, p_1 descending, then p_2
// descending, ... (the last exponent varies fastest).
int monomials(int D, int Q, int (*out)[3]) {
  int n = 0;
  for (int g = 0; g <= Q; ++g) {
    if (D == 1) { out[n][0] = g; out[n][1] = out[n][2] = 0; ++n; continue; }
    for (int a = g; a >= 0; --a) {
      if (D == 2) { out[n][0] = a; out[n][1] = g - a; out[n][2] = 0; ++n; continue; }
      for (int b = g - a; b >= 0; --b) {
        out[n][0] = a; out[n][1] = b; out[n][2] = g - a - b; ++n;
      }
    }
  }
  return n;
}

struct Grid {
  int D, n[3];
  double h;
  long ncell() const { return (long)n[0] * n[1] * (D == 3 ? n[2] : 1); }
  long nface(int d) const {
    long m = 1;
    for (int e = 0; e < D; ++e) m *= (e == d) ? n[e] + 1 : n[e];
    return m;
  }
};

bool init_shape(Shape& S, int kind, int dim, const double* p, int np) {
  S = Shape();
  S.kind = kind;
  S.dim = dim;
  switch (kind) {
    case BALL:
      if (np < 5) return false;
      for (int d = 0; d < 3; ++d) S.c[d] = p[d];
      S.r = p[3];
      S.fsign = p[4];
      S.H = 1.0 / S.r;
      S.radial = true;
      S.Rmin = S.Rmax = S.r;
      return true;
    case HALFSPACE: {
      if (np < 5) return false;
      double nn = 0;
      for (int d = 0; d < dim; ++d) nn += p[d] * p[d];
      nn = std::sqrt(nn);
      for (int d = 0; d < 3; ++d) S.nrm[d] = (d < dim) ? p[d] / nn : 0;
      S.off = p[3] / nn;
      S.fsign = p[4];
      S.H = 0;
      return true;
    }
    case STAR2:
      if (np < 6 || dim != 2) return false;
      S.c[0] = p[0]; S.c[1] = p[1];
      S.r = p[2]; S.amp = p[3]; S.k = (int)p[4];
      S.fsign = p[5];
      S.radial = true;
      S.Rmin = S.r - std::fabs(S.amp);
      S.Rmax = S.r + std::fabs(S.amp);
      break;
    case SH3:
      if (np < 21 || dim != 3) return false;
      for (int d = 0; d < 3; ++d) S.c[d] = p[d];
      S.r = p[3];
      for (int j = 0; j < 16; ++j) S.sh[j] = p[4 + j];
      S.fsign = p[20];
      S.radial = true;
      break;
    default:
      return false;
  }
  // star-shaped bodies: radial bounds by sampling R on the unit sphere, Hessian bound
  // by finite differences of the analytic gradient in the shell around the surface.
  uint64_t st = 0x9E3779B97F4A7C15ull;
  auto rnd = [&]() {
    st ^= st << 13; st ^= st >> 7; st ^= st << 17;
    return (st >> 11) * (1.0 / 9007199254740992.0);
  };
  if (kind == SH3) {
    double mn = 1e300, mx = -1e300;
    for (int i = 0; i < 400; ++i)
      for (int j = 0; j < 800; ++j) {
        double th = M_PI * (i + 0.5) / 400, ph = 2 * M_PI * j / 800;
        double u[3] = {std::sin(th) * std::cos(ph), std::sin(th) * std::sin(ph), std::cos(th)};
        double Y[16];
        sh_eval(u, Y, nullptr);
        double R = S.r;
        for (int q = 0; q < 16; ++q) R += S.sh[q] * Y[q];
        mn = std::min(mn, R);
        mx = std::max(mx, R);
      }
    double marg = 0.05 * (mx - mn) + 1e-3;
    S.Rmin = mn - marg;
    S.Rmax = mx + marg;
  }
  double Hm = 0;
  const double e = 1e-6;
  for (int i = 0; i < 40000; ++i) {
    double x[3] = {S.c[0], S.c[1], S.c[2]};
    double u[3] = {0, 0, 0}, un = 0;
    do {
      un = 0;
      for (int d = 0; d < dim; ++d) { u[d] = 2 * rnd() - 1; un += u[d] * u[d]; }
    } while (un < 1e-4 || un > 1);
    un = std::sqrt(un);
    double rho = 0.5 * S.Rmin + rnd() * (1.5 * S.Rmax - 0.5 * S.Rmin);
    for (int d = 0; d < dim; ++d) x[d] += rho * u[d] / un;
    double fro = 0;
    for (int a = 0; a < dim; ++a) {
      double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]}, gp[3], gm[3];
      xp[a] += e;
      xm[a] -= e;
      phi0(S, xp, gp);
      phi0(S, xm, gm);
      for (int b = 0; b < dim; ++b) {
        double hab = (gp[b] - gm[b]) / (2 * e);
        fro += hab * hab;
      }
    }
    Hm = std::max(Hm, std::sqrt(fro));
  }
  S.H = 2.0 * Hm + 1.0;
  return true;
}

inline long cell_index(const Grid& g, const int* i) {
  return i[0] + (long)g.n[0] * (i[1] + (long)g.n[1] * (g.D == 3 ? i[2] : 0));
}

// per-candidate work: volume + EB quadrature of one cell
struct CellOut {
  double area;
};

void full_face_moments(int D, int Q, double* out) {
  // exact moments of [-1/2, 1/2]^(D-1) over transverse monomials
  int mono[64][3];
  int nm = monomials(D - 1, Q, mono);
  for (int j = 0; j < nm; ++j) {
    double v = 1;
    for (int t = 0; t < D - 1; ++t) {
      int p = mono[j][t];
      v *= (p % 2) ? 0.0 : std::pow(0.5, p) / (p + 1);
    }
    out[j] = v;
  }
}

void full_cell_moments(int D, int Q, double* out) {
  int mono[128][3];
  int nm = monomials(D, Q, mono);
  for (int j = 0; j < nm; ++j) {
    double v = 1;
    for (int t = 0; t < D; ++t) {
      int p = mono[j][t];
      v *= (p % 2) ? 0.0 : std::pow(0.5, p) / (p + 1);
    }
    out[j] = v;
  }
}

// ---- analytic test fields ----------------------------------------------------------
// kind 0: sum of sine products  phi(x) = sum_t a_t prod_d sin(w_td x_d + p_td)
//         (params: amp[T], om[T][3], ph[T][3])
// kind 1: polynomial            phi(x) = sum_t a_t prod_d (x_d - x_ref_d)^e_td
//         (params: amp[T], exponents as doubles in om[T][3], x_ref in ph[0..2])
struct Field {
  int kind = 0, T = 0, D = 2;
  const double* amp = nullptr;
  const double* om = nullptr;
  const double* ph = nullptr;
  double val(const double* x) const {
    double s = 0;
    for (int t = 0; t < T; ++t) {
      double p = amp[t];
      for (int d = 0; d < D; ++d) p *= f1(t, d, x[d], 0);
      s += p;
    }
    return s;
  }
  void grad(const double* x, double* g) const {
    for (int d = 0; d < D; ++d) g[d] = 0;
    for (int t = 0; t < T; ++t)
      for (int d = 0; d < D; ++d) {
        double p = amp[t] * f1(t, d, x[d], 1);
        for (int e = 0; e < D; ++e)
          if (e != d) p *= f1(t, e, x[e], 0);
        g[d] += p;
      }
  }
  double lap(const double* x) const {
    double s = 0;
    for (int t = 0; t < T; ++t)
      for (int d = 0; d < D; ++d) {
        double p = amp[t] * f1(t, d, x[d], 2);
        for (int e = 0; e < D; ++e)
          if (e != d) p *= f1(t, e, x[e], 0);
        s += p;
      }
    return s;
  }
  // k-th derivative of the 1D factor of term t in direction d
  double f1(int t, int d, double x, int k) const {
    if (kind == 0) {
      double w = om[3 * t + d], u = w * x + ph[3 * t + d];
      if (k == 0) return std::sin(u);
      if (k == 1) return w * std::cos(u);
      return -w * w * std::sin(u);
    }
    int e = (int)om[3 * t + d];
    double u = x - ph[d];
    if (k > e) return 0.0;
    double c = 1;
    for (int j = 0; j < k; ++j) c *= (e - j);
    double p = 1;
    for (int j = 0; j < e - k; ++j) p *= u;
    return c * p;
  }
};

}  // namespace

extern "C" {

// Classify cells: 0 covered, 1 full, 2 candidate (the surface may cross it).
// Returns the number of candidates, or -1 on bad arguments.
long cg_classify(int kind, int dim, const double* params, int nparams, const int* n, double h,
                 int8_t* state) {
  Shape S;
  if (!init_shape(S, kind, dim, params, nparams)) return -1;
  Grid g{dim, {n[0], n[1], dim == 3 ? n[2] : 1}, h};
  long nc = g.ncell(), cnt = 0;
#pragma omp parallel for reduction(+ : cnt) schedule(static)
  for (long c = 0; c < nc; ++c) {
    int i[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long)g.n[0] * g.n[1]))};
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) { lo[d] = i[d] * h; hi[d] = (i[d] + 1) * h; }
    double vmin, vmax;
    psi_bounds(S, lo, hi, vmin, vmax);
    int8_t s = 2;
    if (vmin > 0) s = 1;
    else if (vmax < 0) s = 0;
    state[c] = s;
    cnt += (s == 2);
  }
  return cnt;
}

// Geometry and moments. `state` comes from cg_classify and is updated in place
// (candidates become 0 covered, 1 full or 2 cut). `cand` lists the candidate cells
// (ascending). Outputs:
//   vol_mom[ncell*M]            scaled volume moments about cell centres (dense)
//   face_mom_d[nface_d*Mf]      scaled grid-face moments about face centres (dense)
//   eb_mom[ncand*M], eb_nmom[ncand*D*M1], eb_area[ncand]   per candidate
// Returns the number of quadrature failures (0 on success) or -1 on bad arguments.
long cg_geometry(int kind, int dim, const double* params, int nparams, const int* n, double h, int Q,
                 int qorder, int8_t* state, const int64_t* cand, long ncand, double* vol_mom,
                 double* face_mom0, double* face_mom1, double* face_mom2, double* eb_mom, double* eb_nmom,
                 double* eb_area) {
  Shape S;
  if (!init_shape(S, kind, dim, params, nparams)) return -1;
  if (Q < 1 || Q > 6 || qorder < 2 || qorder > 40) return -1;
  Grid g{dim, {n[0], n[1], dim == 3 ? n[2] : 1}, h};
  const int D = dim;
  int mono[128][3], monof[64][3], mono1[128][3];
  const int M = monomials(D, Q, mono);
  const int Mf = monomials(D - 1, Q, monof);
  const int M1 = monomials(D, Q - 1, mono1);
  Gauss G(qorder);
  double fullc[128], fullf[64];
  full_cell_moments(D, Q, fullc);
  full_face_moments(D, Q, fullf);
  const long nc = g.ncell();
  const double hD = std::pow(h, D), hD1 = std::pow(h, D - 1);
  long nerr = 0;

  // dense volume moments for non-candidates
#pragma omp parallel for schedule(static)
  for (long c = 0; c < nc; ++c) {
    double* o = vol_mom + c * M;
    if (state[c] == 1) std::memcpy(o, fullc, sizeof(double) * M);
    else std::memset(o, 0, sizeof(double) * M);
  }

#pragma omp parallel for schedule(dynamic, 4) reduction(+ : nerr)
  for (long j = 0; j < ncand; ++j) {
    const long c = cand[j];
    int i[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long)g.n[0] * g.n[1]))};
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, ctr[3] = {0, 0, 0};
    for (int d = 0; d < D; ++d) {
      lo[d] = i[d] * h;
      hi[d] = (i[d] + 1) * h;
      ctr[d] = (i[d] + 0.5) * h;
    }
    Ctx C{&S, &G};
    double vm[128] = {0};
    std::vector<Fn> fns(1);
    fns[0].sign = 1;
    quad(C, (1u << D) - 1u, lo, hi, fns, 0, [&](double* x, double w) {
      double xi[3][8];
      for (int d = 0; d < D; ++d) {
        double t = (x[d] - ctr[d]) / h;
        xi[d][0] = 1;
        for (int p = 1; p <= Q; ++p) xi[d][p] = xi[d][p - 1] * t;
      }
      for (int m = 0; m < M; ++m) {
        double v = w;
        for (int d = 0; d < D; ++d) v *= xi[d][mono[m][d]];
        vm[m] += v;
      }
    });
    double em[128] = {0}, enm[3 * 128] = {0}, area = 0;
    surf(C, lo, hi, 0, [&](double* x, double w, const double* nv) {
      double xi[3][8];
      for (int d = 0; d < D; ++d) {
        double t = (x[d] - ctr[d]) / h;
        xi[d][0] = 1;
        for (int p = 1; p <= Q; ++p) xi[d][p] = xi[d][p - 1] * t;
      }
      area += w;
      for (int m = 0; m < M; ++m) {
        double v = w;
        for (int d = 0; d < D; ++d) v *= xi[d][mono[m][d]];
        em[m] += v;
      }
      for (int m = 0; m < M1; ++m) {
        double v = w;
        for (int d = 0; d < D; ++d) v *= xi[d][mono1[m][d]];
        for (int d = 0; d < D; ++d) enm[d * M1 + m] += v * nv[d];
      }
    });
    nerr += C.err;
    double kappa = vm[0] / hD;
    double a = area / hD1;
    double* o = vol_mom + c * M;
    if (a <= 1e-14 || kappa <= 1e-14) {
      // no embedded boundary worth keeping (or a negligible sliver of fluid):
      // snap to a full or a covered cell with exact moments
      if (kappa > 0.5) { std::memcpy(o, fullc, sizeof(double) * M); state[c] = 1; }
      else { std::memset(o, 0, sizeof(double) * M); state[c] = 0; }
      eb_area[j] = 0;
      std::memset(eb_mom + j * M, 0, sizeof(double) * M);
      std::memset(eb_nmom + j * D * M1, 0, sizeof(double) * D * M1);
      continue;
    }
    for (int m = 0; m < M; ++m) o[m] = vm[m] / hD;
    state[c] = 2;
    eb_area[j] = a;
    for (int m = 0; m < M; ++m) eb_mom[j * M + m] = em[m] / hD1;
    for (int m = 0; m < D * M1; ++m) eb_nmom[j * D * M1 + m] = enm[m] / hD1;
  }

  // faces
  double* fm[3] = {face_mom0, face_mom1, face_mom2};
  for (int d = 0; d < D; ++d) {
    long nf = g.nface(d);
    int m[3] = {g.n[0], g.n[1], g.n[2]};
    m[d] += 1;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nerr)
    for (long f = 0; f < nf; ++f) {
      int jv[3] = {(int)(f % m[0]), (int)((f / m[0]) % m[1]), (int)(f / ((long)m[0] * m[1]))};
      if (D == 2) jv[2] = 0;
      // adjacent cells: low (jv - e_d) and high (jv)
      int st[2] = {-1, -1};
      for (int s = 0; s < 2; ++s) {
        int ii[3] = {jv[0], jv[1], jv[2]};
        ii[d] -= (s == 0) ? 1 : 0;
        if (ii[d] < 0 || ii[d] >= g.n[d]) continue;
        st[s] = state[cell_index(g, ii)];
      }
      double* o = fm[d] + f * Mf;
      bool anycov = (st[0] == 0 || st[1] == 0);
      bool anycut = (st[0] == 2 || st[1] == 2);
      if (anycov) { std::memset(o, 0, sizeof(double) * Mf); continue; }
      if (!anycut) { std::memcpy(o, fullf, sizeof(double) * Mf); continue; }
      double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, ctr[3] = {0, 0, 0};
      for (int e = 0; e < D; ++e) {
        if (e == d) { lo[e] = hi[e] = ctr[e] = jv[e] * h; }
        else { lo[e] = jv[e] * h; hi[e] = (jv[e] + 1) * h; ctr[e] = (jv[e] + 0.5) * h; }
      }
      Ctx C{&S, &G};
      std::vector<Fn> fns(1);
      fns[0].sign = 1;
      fns[0].mask = 1u << d;
      fns[0].val[d] = jv[d] * h;
      double acc[64] = {0};
      quad(C, ((1u << D) - 1u) & ~(1u << d), lo, hi, fns, 0, [&](double* x, double w) {
        double xi[3][8];
        int t = 0;
        double pw[2][8];
        for (int e = 0; e < D; ++e) {
          if (e == d) continue;
          double u = (x[e] - ctr[e]) / h;
          pw[t][0] = 1;
          for (int p = 1; p <= Q; ++p) pw[t][p] = pw[t][p - 1] * u;
          ++t;
        }
        (void)xi;
        for (int mm = 0; mm < Mf; ++mm) {
          double v = w;
          for (int e = 0; e < D - 1; ++e) v *= pw[e][monof[mm][e]];
          acc[mm] += v;
        }
      });
      nerr += C.err;
      double alpha = acc[0] / hD1;
      if (alpha <= 1e-14) { std::memset(o, 0, sizeof(double) * Mf); continue; }
      for (int mm = 0; mm < Mf; ++mm) o[mm] = acc[mm] / hD1;
    }
  }
  return nerr;
}

// Exact integrals of an analytic field (see Field) over the geometry from cg_geometry
// (same state/cand). Unscaled (physical) integrals:
//   vol_int[ncell] = int_V phi, vol_lap[ncell] = int_V lap(phi)
//   face_int_d[nface_d] = int_A phi, face_flux_d[nface_d] = int_A d phi / d x_d
//   eb_int[ncand] = int_EB phi, eb_flux[ncand] = int_EB grad(phi).n  (n out of the fluid)
long cg_integrate(int kind, int dim, const double* params, int nparams, const int* n, double h, int qorder,
                  const int8_t* state, const int64_t* cand, long ncand, int field_kind, int T, const double* amp,
                  const double* om, const double* ph, double* vol_int, double* vol_lap, double* face_int0,
                  double* face_int1, double* face_int2, double* face_flux0, double* face_flux1,
                  double* face_flux2, double* eb_int, double* eb_flux) {
  Shape S;
  if (!init_shape(S, kind, dim, params, nparams)) return -1;
  Grid g{dim, {n[0], n[1], dim == 3 ? n[2] : 1}, h};
  const int D = dim;
  Gauss G(qorder);
  Field P;
  P.kind = field_kind; P.T = T; P.D = D; P.amp = amp; P.om = om; P.ph = ph;
  const long nc = g.ncell();
  long nerr = 0;
  std::vector<long> cpos(nc, -1);
  for (long j = 0; j < ncand; ++j) cpos[cand[j]] = j;

#pragma omp parallel for schedule(dynamic, 16) reduction(+ : nerr)
  for (long c = 0; c < nc; ++c) {
    vol_int[c] = 0;
    vol_lap[c] = 0;
    if (state[c] == 0) continue;
    int i[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long)g.n[0] * g.n[1]))};
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < D; ++d) { lo[d] = i[d] * h; hi[d] = (i[d] + 1) * h; }
    Ctx C{&S, &G};
    double si = 0, sl = 0;
    auto acc = [&](double* x, double w) { si += w * P.val(x); sl += w * P.lap(x); };
    if (state[c] == 1) {
      double x[3] = {0, 0, 0};
      tensor(C, (1u << D) - 1u, lo, hi, x, 1.0, 0, acc);
    } else {
      std::vector<Fn> fns(1);
      fns[0].sign = 1;
      quad(C, (1u << D) - 1u, lo, hi, fns, 0, acc);
      long j = cpos[c];
      if (j >= 0) {
        double ei = 0, ef = 0;
        surf(C, lo, hi, 0, [&](double* x, double w, const double* nv) {
          double gg[3];
          P.grad(x, gg);
          ei += w * P.val(x);
          double gn = 0;
          for (int d = 0; d < D; ++d) gn += gg[d] * nv[d];
          ef += w * gn;
        });
        eb_int[j] = ei;
        eb_flux[j] = ef;
      }
    }
    nerr += C.err;
    vol_int[c] = si;
    vol_lap[c] = sl;
  }
  double* fi[3] = {face_int0, face_int1, face_int2};
  double* ff[3] = {face_flux0, face_flux1, face_flux2};
  for (int d = 0; d < D; ++d) {
    long nf = g.nface(d);
    int m[3] = {g.n[0], g.n[1], g.n[2]};
    m[d] += 1;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nerr)
    for (long f = 0; f < nf; ++f) {
      int jv[3] = {(int)(f % m[0]), (int)((f / m[0]) % m[1]), (int)(f / ((long)m[0] * m[1]))};
      if (D == 2) jv[2] = 0;
      int st[2] = {-1, -1};
      for (int s = 0; s < 2; ++s) {
        int ii[3] = {jv[0], jv[1], jv[2]};
        ii[d] -= (s == 0) ? 1 : 0;
        if (ii[d] < 0 || ii[d] >= g.n[d]) continue;
        st[s] = state[cell_index(g, ii)];
      }
      fi[d][f] = 0;
      ff[d][f] = 0;
      if (st[0] == 0 || st[1] == 0) continue;
      bool anycut = (st[0] == 2 || st[1] == 2);
      double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
      for (int e = 0; e < D; ++e) {
        if (e == d) lo[e] = hi[e] = jv[e] * h;
        else { lo[e] = jv[e] * h; hi[e] = (jv[e] + 1) * h; }
      }
      Ctx C{&S, &G};
      double si = 0, sf = 0;
      auto acc = [&](double* x, double w) {
        x[d] = jv[d] * h;
        double gg[3];
        P.grad(x, gg);
        si += w * P.val(x);
        sf += w * gg[d];
      };
      unsigned freem = ((1u << D) - 1u) & ~(1u << d);
      if (!anycut) {
        double x[3] = {0, 0, 0};
        tensor(C, freem, lo, hi, x, 1.0, 0, acc);
      } else {
        std::vector<Fn> fns(1);
        fns[0].sign = 1;
        fns[0].mask = 1u << d;
        fns[0].val[d] = jv[d] * h;
        quad(C, freem, lo, hi, fns, 0, acc);
      }
      nerr += C.err;
      fi[d][f] = si;
      ff[d][f] = sf;
    }
  }
  return nerr;
}

// psi at points (for tests): fluid is psi > 0
int cg_psi(int kind, int dim, const double* params, int nparams, long npts, const double* x, double* out) {
  Shape S;
  if (!init_shape(S, kind, dim, params, nparams)) return -1;
  for (long i = 0; i < npts; ++i) out[i] = psi(S, x + 3 * i, nullptr);
  return 0;
}

}  // extern "C"
