// lskum_ref.cpp -- FP64 CPU oracle for the LSKUM residual sweep.
//
// TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked
// against.  Only the test suite, the smoke check and the benchmark's CPU
// baseline may load it.  It shares no code with the GPU library.
//
// Plain loops over points in index order, one point at a time, evaluated in
// the order the formulas are written (the library is built with
// -ffp-contract=off, no -ffast-math).  The per-point formulas are templates
// over the scalar type, so that the same text is also evaluated with a
// reverse-mode scalar (the adjoints) and an operation-counting one (the
// algorithmic operation count of the flux residual).
//
// Method (arXiv 2403.13287, "Theory of Meshfree LSKUM"):
//   * q-variables: eq. (13);
//   * least-squares derivatives: eq. (9)/(15) with the modified differences
//     of eq. (14) ("inner iterations", solved here by Jacobi sweeps that
//     start from the first-order least-squares solution);
//   * semi-discrete upwind scheme: eq. (10) with split-flux derivatives by
//     eq. (11) on the half-plane stencils N^{+-} (text after eq. (12)), the
//     differences taken between split fluxes of the modified q-variables;
//   * kinetic split fluxes: half-range moments of the Maxwellian of eq. (2)
//     under the CIR splitting of eq. (3);
//   * state update: eq. (16) is the forward-Euler building block of each
//     stage of the four-stage SSP Runge-Kutta scheme used here.
// Points the paper leaves open (limiter, boundary conditions, local time
// step, frame at walls, residue definition, force coefficients) follow the
// readings recorded with the design notes; each is restated at its function.
//
// The forward point loops carry OpenMP work-sharing pragmas: every point is
// computed independently into its own output slots, so a build with -fopenmp
// gives the same results bit for bit on all host cores (the CPU-throughput
// comparison).  The parity build ignores them and runs single-threaded.  The
// reverse-mode and operation-counting routines always run single-threaded
// (their tape and tally are process globals).

#include "lskum_ref.h"

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <limits>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Reverse-mode scalar for the adjoint routines.
//
// Every operation on a tape variable appends a node holding the indices of
// its (at most two) operands and the partial derivatives with respect to
// them; constants (index -1) are not recorded.  Values are computed with the
// same double operations as the plain routines, so a taped evaluation
// reproduces their results exactly.  Branches (limiter, max/min, split
// stencil membership) follow the values, so the derivative is that of the
// active branch.

namespace ad {

struct Tape {
  std::vector<int32_t> a, b;
  std::vector<double> ga, gb, adj;
  void clear() {
    a.clear();
    b.clear();
    ga.clear();
    gb.clear();
    adj.clear();
  }
  int32_t push(int32_t ia, double da, int32_t ib, double db) {
    a.push_back(ia);
    ga.push_back(da);
    b.push_back(ib);
    gb.push_back(db);
    return (int32_t)a.size() - 1;
  }
  // adjoints of every node given seeds already placed in adj
  void reverse() {
    for (int32_t k = (int32_t)a.size() - 1; k >= 0; --k) {
      const double g = adj[(size_t)k];
      if (g == 0.0) continue;
      if (a[(size_t)k] >= 0) adj[(size_t)a[(size_t)k]] += ga[(size_t)k] * g;
      if (b[(size_t)k] >= 0) adj[(size_t)b[(size_t)k]] += gb[(size_t)k] * g;
    }
  }
};

Tape *tape = nullptr;  // used by single-threaded routines only

struct Var {
  double v;
  int32_t i;
  Var() : v(0.0), i(-1) {}
  Var(double x) : v(x), i(-1) {}  // NOLINT: constants convert implicitly
  Var(double x, int32_t idx) : v(x), i(idx) {}
};

inline Var input(double x) { return Var(x, tape->push(-1, 0.0, -1, 0.0)); }
inline Var make(double v, int32_t ia, double da, int32_t ib, double db) {
  if (ia < 0 && ib < 0) return Var(v);
  return Var(v, tape->push(ia, da, ib, db));
}
inline Var operator+(Var x, Var y) { return make(x.v + y.v, x.i, 1.0, y.i, 1.0); }
inline Var operator-(Var x, Var y) { return make(x.v - y.v, x.i, 1.0, y.i, -1.0); }
inline Var operator*(Var x, Var y) { return make(x.v * y.v, x.i, y.v, y.i, x.v); }
inline Var operator/(Var x, Var y) {
  const double v = x.v / y.v;
  return make(v, x.i, 1.0 / y.v, y.i, -v / y.v);
}
inline Var operator-(Var x) { return make(-x.v, x.i, -1.0, -1, 0.0); }
inline Var &operator+=(Var &x, Var y) { return x = x + y; }
inline bool operator<(Var x, Var y) { return x.v < y.v; }
inline bool operator>(Var x, Var y) { return x.v > y.v; }
inline Var exp(Var x) {
  const double e = std::exp(x.v);
  return make(e, x.i, e, -1, 0.0);
}
inline Var log(Var x) { return make(std::log(x.v), x.i, 1.0 / x.v, -1, 0.0); }
inline Var sqrt(Var x) {
  const double r = std::sqrt(x.v);
  return make(r, x.i, 0.5 / r, -1, 0.0);
}
inline Var erf(Var x) {
  return make(std::erf(x.v), x.i, 2.0 / std::sqrt(kPi) * std::exp(-x.v * x.v), -1, 0.0);
}
inline Var cos(Var x) { return make(std::cos(x.v), x.i, -std::sin(x.v), -1, 0.0); }
inline Var sin(Var x) { return make(std::sin(x.v), x.i, std::cos(x.v), -1, 0.0); }
inline double val(Var x) { return x.v; }

}  // namespace ad

// ---------------------------------------------------------------------------
// Operation-counting scalar: evaluates the same template text in double and
// tallies each floating-point operation on state-dependent values (sums and
// differences, products, quotients, and calls of sqrt, exp, log, erf).
// Negation is free; comparisons are not arithmetic.  Operations on plain
// doubles (the geometry of an edge) are not seen.
namespace cnt {

struct Tally {
  double add = 0, mul = 0, div = 0, sqrt = 0, exp = 0, log = 0, erf = 0;
};
Tally *tally = nullptr;  // used by single-threaded routines only

struct Num {
  double v;
  Num() : v(0.0) {}
  Num(double x) : v(x) {}  // NOLINT: constants convert implicitly
};
inline Num operator+(Num x, Num y) { tally->add += 1; return Num(x.v + y.v); }
inline Num operator-(Num x, Num y) { tally->add += 1; return Num(x.v - y.v); }
inline Num operator*(Num x, Num y) { tally->mul += 1; return Num(x.v * y.v); }
inline Num operator/(Num x, Num y) { tally->div += 1; return Num(x.v / y.v); }
inline Num operator-(Num x) { return Num(-x.v); }
inline Num &operator+=(Num &x, Num y) { return x = x + y; }
inline bool operator<(Num x, Num y) { return x.v < y.v; }
inline bool operator>(Num x, Num y) { return x.v > y.v; }
inline Num sqrt(Num x) { tally->sqrt += 1; return Num(std::sqrt(x.v)); }
inline Num exp(Num x) { tally->exp += 1; return Num(std::exp(x.v)); }
inline Num log(Num x) { tally->log += 1; return Num(std::log(x.v)); }
inline Num erf(Num x) { tally->erf += 1; return Num(std::erf(x.v)); }
inline Num fabs(Num x) { return Num(std::fabs(x.v)); }
inline double val(Num x) { return x.v; }

}  // namespace cnt

inline double val(double x) { return x; }

// ---------------------------------------------------------------------------
// Point-level formulas

// Free stream, non-dimensionalised by the free-stream density and sound
// speed: rho = 1, p = 1/gamma (so a = 1), velocity = M (cos a, sin a).
template <class T>
void free_stream_prim_t(double gamma, T mach, T aoa, T w[4]) {
  using std::cos;
  using std::sin;
  w[0] = T(1.0);
  w[1] = mach * cos(aoa);
  w[2] = mach * sin(aoa);
  w[3] = T(1.0 / gamma);
}

void free_stream_prim(const lskum_ref_params &P, double w[4]) {
  free_stream_prim_t<double>(P.gamma, P.mach, P.aoa_rad, w);
}

// U = (rho, rho u, rho v, E), E = p/(gamma-1) + rho (u^2 + v^2)/2  (eq. (1))
template <class T>
void cons_from_prim(double g, const T w[4], T U[4]) {
  U[0] = w[0];
  U[1] = w[0] * w[1];
  U[2] = w[0] * w[2];
  U[3] = w[3] / (g - 1.0) + 0.5 * w[0] * (w[1] * w[1] + w[2] * w[2]);
}

template <class T>
void prim_from_cons(double g, const T U[4], T w[4]) {
  using std::fabs;
  T rho = U[0];
  T u = U[1] / rho;
  T v = U[2] / rho;
  w[0] = rho;
  w[1] = u;
  w[2] = v;
  w[3] = (g - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v));
}

// eq. (13): q = (ln rho + ln(beta)/(gamma-1) - beta (u^2+v^2), 2 beta u,
//               2 beta v, -2 beta),  beta = rho / (2 p)
template <class T>
void q_from_prim(double g, const T w[4], T q[4]) {
  using std::log;
  T beta = 0.5 * w[0] / w[3];
  q[0] = log(w[0]) + log(beta) / (g - 1.0) - beta * (w[1] * w[1] + w[2] * w[2]);
  q[1] = 2.0 * beta * w[1];
  q[2] = 2.0 * beta * w[2];
  q[3] = -2.0 * beta;
}

// Inverse of eq. (13): beta = -q4/2, u = q2/(2 beta), v = q3/(2 beta),
// rho = exp(q1 + beta (u^2+v^2) - ln(beta)/(gamma-1)), p = rho/(2 beta).
template <class T>
void prim_from_q(double g, const T q[4], T w[4]) {
  using std::exp;
  using std::log;
  T beta = -0.5 * q[3];
  T u = q[1] / (2.0 * beta);
  T v = q[2] / (2.0 * beta);
  T rho = exp(q[0] + beta * (u * u + v * v) - log(beta) / (g - 1.0));
  w[0] = rho;
  w[1] = u;
  w[2] = v;
  w[3] = rho / (2.0 * beta);
}

// Kinetic split flux G^{sign} along direction `dir` (0: s, 1: n) of the
// local state w = (rho, u_s, u_n, p): the half-range (sign * v_dir > 0)
// moments of v_dir * Psi * F with F the Maxwellian of eq. (2) carrying
// 1/(gamma-1) - 1 internal degrees of freedom.  With beta = rho/(2p),
// S = u_dir sqrt(beta), A = (1 + sign erf S)/2, B = exp(-S^2)/(2 sqrt(pi beta)):
//   mass          rho (u_dir A + sign B)
//   dir-momentum  (p + rho u_dir^2) A + sign rho u_dir B
//   other mom.    rho u_other (u_dir A + sign B)
//   energy        (E + p) u_dir A + sign (E + p/2) B
template <class T>
void split_flux(double g, int dir, int sign, const T w[4], T G[4]) {
  using std::erf;
  using std::exp;
  using std::sqrt;
  const double sg = sign > 0 ? 1.0 : -1.0;
  T rho = w[0], us = w[1], un = w[2], p = w[3];
  T ud = dir == 0 ? us : un;
  T uo = dir == 0 ? un : us;
  T beta = 0.5 * rho / p;
  T S = ud * sqrt(beta);
  T A = 0.5 * (1.0 + sg * erf(S));
  T B = exp(-(S * S)) / (2.0 * sqrt(kPi * beta));
  T F = ud * A + sg * B;
  T E = p / (g - 1.0) + 0.5 * rho * (us * us + un * un);
  G[0] = rho * F;
  T Gd = (p + rho * ud * ud) * A + sg * rho * ud * B;
  T Go = rho * uo * F;
  G[dir == 0 ? 1 : 2] = Gd;
  G[dir == 0 ? 2 : 1] = Go;
  G[3] = (E + p) * ud * A + sg * (E + 0.5 * p) * B;
}

// Venkatakrishnan limiter factor for an increment `delta` at a point whose
// stencil bounds relative to its own value are dmax >= 0 >= dmin:
//   D = dmax (delta > 0) or dmin (delta < 0),
//   phi = min(1, (D^2 + eps2 + 2 delta D) / (D^2 + 2 delta^2 + delta D + eps2)),
//   phi = 1 when delta == 0.
template <class T>
T venkat_phi(T delta, T dmax, T dmin, T eps2) {
  T D;
  if (delta > 0.0) {
    D = dmax;
  } else if (delta < 0.0) {
    D = dmin;
  } else {
    return T(1.0);
  }
  T num = D * D + eps2 + 2.0 * delta * D;
  T den = D * D + 2.0 * delta * delta + delta * D + eps2;
  T phi = num / den;
  if (phi < 1.0) return phi;
  return T(1.0);
}

// Min-max limiter factor: the increment is scaled so that the reconstructed
// value stays within the stencil bounds, phi = min(1, D/delta) with D the
// room on delta's side (dmax for delta > 0, dmin for delta < 0); phi = 1 for
// delta = 0.
template <class T>
T minmax_phi(T delta, T dmax, T dmin) {
  T D;
  if (delta > 0.0) {
    D = dmax;
  } else if (delta < 0.0) {
    D = dmin;
  } else {
    return T(1.0);
  }
  T phi = D / delta;
  if (phi < 1.0) return phi;
  return T(1.0);
}

bool finite_positive(double v) { return std::isfinite(v) && v > 0.0; }

// ---------------------------------------------------------------------------
// Cloud access helpers

struct Row {
  const int32_t *ids;
  int32_t count;
};

Row row(const lskum_ref_cloud &c, int32_t i) {
  return Row{c.col + c.row_ptr[i], c.nbr_count[i]};
}

inline double fld(const double *f, int32_t comp, int32_t n, int32_t i) {
  return f[(size_t)comp * (size_t)n + (size_t)i];
}
inline double &fld(double *f, int32_t comp, int32_t n, int32_t i) {
  return f[(size_t)comp * (size_t)n + (size_t)i];
}

// Pairwise (recursive halving) summation, fixed order.
template <class T>
T pairwise_sum(const T *v, size_t n) {
  if (n == 0) return T(0.0);
  if (n <= 8) {
    T s = T(0.0);
    for (size_t k = 0; k < n; ++k) s += v[k];
    return s;
  }
  size_t h = n / 2;
  return pairwise_sum(v, h) + pairwise_sum(v + h, n - h);
}

// ---------------------------------------------------------------------------
// Per-point formulas of the sweeps.  A point function reads the data of its
// stencil through an accessor: st.own(f, m) for the point itself and
// st.nbr(k, f, m) for its k-th real neighbour, field f = 0 (q, m < 4),
// 1 (dq, m < 8) or 2 (qlim, m < 8).  The plain sweeps pass array accessors;
// the adjoint routines pass accessors that return tape variables.

enum Field { kQ = 0, kG = 1, kL = 2 };

struct ArraySt {
  const double *f[3];
  int32_t n, i;
  const int32_t *ids;
  double own(int fld_, int m) const { return f[fld_][(size_t)m * n + i]; }
  double nbr(int k, int fld_, int m) const { return f[fld_][(size_t)m * n + ids[k]]; }
};

const int kWidth[3] = {4, 8, 8};

// eq. (13) at one point; flags a non-physical state.
template <class T>
unsigned q_point(double g, const T U[4], T q[4]) {
  T w[4];
  prim_from_cons(g, U, w);
  const unsigned flags =
      (!finite_positive(val(w[0])) || !finite_positive(val(w[3]))) ? LSKUM_REF_NONPHYSICAL : 0u;
  q_from_prim(g, w, q);
  return flags;
}

// First-order least squares (eq. (9) with the plain differences
// dq_i = q_i - q_0) over the full stencil, and the stencil bounds
// max/min of q over {P0} U N(P0) (the first point reaching the bound wins).
template <class T, class St>
void deriv_first_point(const lskum_ref_cloud &c, int32_t i, const St &st, T dq[8], T qlim[8]) {
  Row r = row(c, i);
  double sxx = 0.0, sxy = 0.0, syy = 0.0;
  T sxq[4] = {T(0.0), T(0.0), T(0.0), T(0.0)}, syq[4] = {T(0.0), T(0.0), T(0.0), T(0.0)};
  T qmax[4], qmin[4];
  for (int m = 0; m < 4; ++m) qmax[m] = qmin[m] = st.own(kQ, m);
  for (int32_t k = 0; k < r.count; ++k) {
    int32_t j = r.ids[k];
    double dx = c.x[j] - c.x[i];
    double dy = c.y[j] - c.y[i];
    sxx += dx * dx;
    sxy += dx * dy;
    syy += dy * dy;
    for (int m = 0; m < 4; ++m) {
      T qj = st.nbr(k, kQ, m);
      T d = qj - st.own(kQ, m);
      sxq[m] += dx * d;
      syq[m] += dy * d;
      if (qj > qmax[m]) qmax[m] = qj;
      if (qj < qmin[m]) qmin[m] = qj;
    }
  }
  double det = sxx * syy - sxy * sxy;
  for (int m = 0; m < 4; ++m) {
    dq[m] = (syy * sxq[m] - sxy * syq[m]) / det;
    dq[4 + m] = (sxx * syq[m] - sxy * sxq[m]) / det;
    qlim[m] = qmax[m];
    qlim[4 + m] = qmin[m];
  }
}

// One inner iteration (eq. (14)-(15)) at one point: the modified
// differences use the previous iterate of the derivatives (field kG) at
// both ends of each edge,
//   dq~_i = [q_i - (dx q_x,i + dy q_y,i)/2] - [q_0 - (dx q_x,0 + dy q_y,0)/2].
template <class T, class St>
void deriv_inner_point(const lskum_ref_cloud &c, int32_t i, const St &st, T dq[8]) {
  Row r = row(c, i);
  double sxx = 0.0, sxy = 0.0, syy = 0.0;
  T sxq[4] = {T(0.0), T(0.0), T(0.0), T(0.0)}, syq[4] = {T(0.0), T(0.0), T(0.0), T(0.0)};
  for (int32_t k = 0; k < r.count; ++k) {
    int32_t j = r.ids[k];
    double dx = c.x[j] - c.x[i];
    double dy = c.y[j] - c.y[i];
    sxx += dx * dx;
    sxy += dx * dy;
    syy += dy * dy;
    for (int m = 0; m < 4; ++m) {
      T qt_j = st.nbr(k, kQ, m) - 0.5 * (dx * st.nbr(k, kG, m) + dy * st.nbr(k, kG, 4 + m));
      T qt_0 = st.own(kQ, m) - 0.5 * (dx * st.own(kG, m) + dy * st.own(kG, 4 + m));
      T d = qt_j - qt_0;
      sxq[m] += dx * d;
      syq[m] += dy * d;
    }
  }
  double det = sxx * syy - sxy * sxy;
  for (int m = 0; m < 4; ++m) {
    dq[m] = (syy * sxq[m] - sxy * syq[m]) / det;
    dq[4 + m] = (sxx * syq[m] - sxy * sxq[m]) / det;
  }
}

// Flux residual at one point (see lskum_ref_flux_residual).
template <class T, class St>
unsigned flux_point(const lskum_ref_cloud &c, const lskum_ref_params &P, int32_t i, const St &st,
                    T R[4]) {
  const double g = P.gamma;
  unsigned flags = 0;
  const int kind = c.kind[i];
  if (kind == 2) {
    for (int m = 0; m < 4; ++m) R[m] = T(0.0);
    return 0;
  }
  const double nx = c.nx[i], ny = c.ny[i];
  const double tx = ny, ty = -nx;
  // split order: 0 = s+, 1 = s-, 2 = n+, 3 = n-
  double sss[4] = {0, 0, 0, 0}, ssn[4] = {0, 0, 0, 0}, snn[4] = {0, 0, 0, 0};
  T as[4][4], an[4][4];
  for (int sp = 0; sp < 4; ++sp)
    for (int m = 0; m < 4; ++m) as[sp][m] = an[sp][m] = T(0.0);
  int cnt[4] = {0, 0, 0, 0};
  Row r = row(c, i);
  for (int32_t k = 0; k < r.count; ++k) {
    int32_t j = r.ids[k];
    double dx = c.x[j] - c.x[i];
    double dy = c.y[j] - c.y[i];
    double ds = dx * tx + dy * ty;
    double dn = dx * nx + dy * ny;
    double dist = std::sqrt(dx * dx + dy * dy);
    double kd = P.venkat_k * dist;
    double eps2 = kd * kd * kd;
    T qt_j[4], qt_0[4];
    for (int m = 0; m < 4; ++m) {
      T qj = st.nbr(k, kQ, m), q0 = st.own(kQ, m);
      if (P.options & LSKUM_REF_FIRST_ORDER) {  // first-order scheme: q itself
        qt_j[m] = qj;
        qt_0[m] = q0;
        continue;
      }
      T del_j = -0.5 * (dx * st.nbr(k, kG, m) + dy * st.nbr(k, kG, 4 + m));
      T del_0 = -0.5 * (dx * st.own(kG, m) + dy * st.own(kG, 4 + m));
      T phi_j, phi_0;
      if (P.options & LSKUM_REF_MINMAX) {
        phi_j = minmax_phi(del_j, st.nbr(k, kL, m) - qj, st.nbr(k, kL, 4 + m) - qj);
        phi_0 = minmax_phi(del_0, st.own(kL, m) - q0, st.own(kL, 4 + m) - q0);
      } else {
        phi_j = venkat_phi(del_j, st.nbr(k, kL, m) - qj, st.nbr(k, kL, 4 + m) - qj, T(eps2));
        phi_0 = venkat_phi(del_0, st.own(kL, m) - q0, st.own(kL, 4 + m) - q0, T(eps2));
      }
      qt_j[m] = qj + phi_j * del_j;
      qt_0[m] = q0 + phi_0 * del_0;
    }
    T wj[4], w0[4];
    prim_from_q(g, qt_j, wj);
    prim_from_q(g, qt_0, w0);
    if (!(qt_j[3] < 0.0) || !(qt_0[3] < 0.0) || !finite_positive(val(wj[0])) ||
        !finite_positive(val(w0[0])) || !finite_positive(val(wj[3])) ||
        !finite_positive(val(w0[3])))
      flags |= LSKUM_REF_NONPHYSICAL;
    // velocities in P0's frame
    T lj[4] = {wj[0], wj[1] * tx + wj[2] * ty, wj[1] * nx + wj[2] * ny, wj[3]};
    T l0[4] = {w0[0], w0[1] * tx + w0[2] * ty, w0[1] * nx + w0[2] * ny, w0[3]};
    int sel[2] = {-1, -1};
    if (ds < 0.0) sel[0] = 0;
    if (ds > 0.0) sel[0] = 1;
    if (dn < 0.0 && kind == 0) sel[1] = 2;
    if (dn > 0.0) sel[1] = 3;
    for (int h = 0; h < 2; ++h) {
      int sp = sel[h];
      if (sp < 0) continue;
      int dir = sp < 2 ? 0 : 1;
      int sign = (sp == 0 || sp == 2) ? 1 : -1;
      T Gj[4], G0[4];
      split_flux(g, dir, sign, lj, Gj);
      split_flux(g, dir, sign, l0, G0);
      sss[sp] += ds * ds;
      ssn[sp] += ds * dn;
      snn[sp] += dn * dn;
      cnt[sp] += 1;
      for (int m = 0; m < 4; ++m) {
        T dG = Gj[m] - G0[m];
        as[sp][m] += ds * dG;
        an[sp][m] += dn * dG;
      }
    }
  }
  T Rf[4] = {T(0.0), T(0.0), T(0.0), T(0.0)};
  for (int sp = 0; sp < 4; ++sp) {
    if (sp == 2 && kind != 0) continue;
    double det = sss[sp] * snn[sp] - ssn[sp] * ssn[sp];
    if (cnt[sp] < 2 || !(det > 1e-12 * sss[sp] * snn[sp])) {
      flags |= LSKUM_REF_DEGENERATE;
      continue;
    }
    for (int m = 0; m < 4; ++m) {
      T d;
      if (sp < 2)
        d = (snn[sp] * as[sp][m] - ssn[sp] * an[sp][m]) / det;
      else
        d = (sss[sp] * an[sp][m] - ssn[sp] * as[sp][m]) / det;
      Rf[m] += d;
    }
  }
  R[0] = Rf[0];
  R[1] = Rf[1] * tx + Rf[2] * nx;
  R[2] = Rf[1] * ty + Rf[2] * ny;
  R[3] = Rf[3];
  return flags;
}


// ---------------------------------------------------------------------------
// Adjoint helpers: a stencil accessor whose values are tape inputs.  One
// point function is evaluated on a fresh tape, its outputs are seeded with
// their cotangents, the tape is swept backwards, and the adjoints of the
// inputs are added to the cotangent arrays of the points they came from.

struct TapeSt {
  static int off(int f, int m) { return f == kQ ? m : (f == kG ? 4 + m : 12 + m); }
  int32_t n, i;
  Row r;
  unsigned mask;  // bit f: field f is read by the point function
  std::vector<ad::Var> v;  // (count + 1) slots x 20 values: own, then neighbours
  TapeSt(const double *const f[3], int32_t n_, int32_t i_, Row r_, unsigned mask_)
      : n(n_), i(i_), r(r_), mask(mask_), v((size_t)(r_.count + 1) * 20) {
    for (int32_t s = 0; s <= r.count; ++s) {
      const int32_t pnt = s == 0 ? i : r.ids[s - 1];
      for (int fl = 0; fl < 3; ++fl) {
        if (!(mask & (1u << fl))) continue;
        for (int m = 0; m < kWidth[fl]; ++m)
          v[(size_t)s * 20 + off(fl, m)] = ad::input(f[fl][(size_t)m * n + pnt]);
      }
    }
  }
  ad::Var own(int fl, int m) const { return v[(size_t)off(fl, m)]; }
  ad::Var nbr(int k, int fl, int m) const { return v[(size_t)(k + 1) * 20 + off(fl, m)]; }
  void scatter(double *const bar[3]) const {
    for (int32_t s = 0; s <= r.count; ++s) {
      const int32_t pnt = s == 0 ? i : r.ids[s - 1];
      for (int fl = 0; fl < 3; ++fl) {
        if (!(mask & (1u << fl)) || !bar[fl]) continue;
        for (int m = 0; m < kWidth[fl]; ++m)
          bar[fl][(size_t)m * n + pnt] += ad::tape->adj[(size_t)v[(size_t)s * 20 + off(fl, m)].i];
      }
    }
  }
};

// Start a tape sweep: zero adjoints, then seed.
void seed_begin() { ad::tape->adj.assign(ad::tape->a.size(), 0.0); }
void seed(const ad::Var &x, double s) {
  if (x.i >= 0) ad::tape->adj[(size_t)x.i] += s;
}
double adjoint(const ad::Var &x) { return x.i >= 0 ? ad::tape->adj[(size_t)x.i] : 0.0; }

// Lift and drag from the wall polygon W_0..W_{m-1} (counter-clockwise):
// edge e = (W_j, W_j+1) has outward normal-length vector (dy_e, -dx_e) and
// pressure p_e = (p_j + p_j+1)/2; Cp_e = (p_e - p_inf)/(rho_inf M^2 / 2);
// (Cx, Cy) = -sum_e Cp_e nu_e (chord 1); Cl = Cy cos a - Cx sin a,
// Cd = Cx cos a + Cy sin a.  Uw(j, k) returns component k of U at point j.
template <class T, class UW>
void force_t(const lskum_ref_cloud &c, double gamma, T mach, T aoa, const UW &Uw, T clcd[2]) {
  using std::cos;
  using std::sin;
  const int32_t m = c.n_wall;
  const double pinf = 1.0 / gamma;
  T qinf = 0.5 * 1.0 * mach * mach;
  std::vector<T> fx((size_t)m), fy((size_t)m);
  for (int32_t e = 0; e < m; ++e) {
    int32_t a = c.wall_loop[e], b = c.wall_loop[(e + 1) % m];
    T Ua[4], Ub[4], wa[4], wb[4];
    for (int k = 0; k < 4; ++k) {
      Ua[k] = Uw(a, k);
      Ub[k] = Uw(b, k);
    }
    prim_from_cons(gamma, Ua, wa);
    prim_from_cons(gamma, Ub, wb);
    T pe = 0.5 * (wa[3] + wb[3]);
    T cp = (pe - pinf) / qinf;
    double ex = c.x[b] - c.x[a];
    double ey = c.y[b] - c.y[a];
    fx[(size_t)e] = -cp * ey;
    fy[(size_t)e] = cp * ex;
  }
  T Cx = pairwise_sum(fx.data(), fx.size());
  T Cy = pairwise_sum(fy.data(), fy.size());
  T ca = cos(aoa), sa = sin(aoa);
  clcd[0] = Cy * ca - Cx * sa;
  clcd[1] = Cx * ca + Cy * sa;
}

}  // namespace

// ---------------------------------------------------------------------------
// Exported point-level formulas

extern "C" {

int lskum_ref_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void lskum_ref_free_stream(const lskum_ref_params *p, double U[4]) {
  double w[4];
  free_stream_prim(*p, w);
  cons_from_prim(p->gamma, w, U);
}

void lskum_ref_q_from_prim(double gamma, const double prim[4], double q[4]) {
  q_from_prim(gamma, prim, q);
}

void lskum_ref_prim_from_q(double gamma, const double q[4], double prim[4]) {
  prim_from_q(gamma, q, prim);
}

void lskum_ref_cons_from_prim(double gamma, const double prim[4], double U[4]) {
  cons_from_prim(gamma, prim, U);
}

void lskum_ref_prim_from_cons(double gamma, const double U[4], double prim[4]) {
  prim_from_cons(gamma, U, prim);
}

void lskum_ref_split_flux(double gamma, int dir, int sign, const double w[4], double G[4]) {
  split_flux(gamma, dir, sign, w, G);
}

double lskum_ref_venkat_phi(double delta, double dmax, double dmin, double eps2) {
  return venkat_phi(delta, dmax, dmin, eps2);
}

double lskum_ref_minmax_phi(double delta, double dmax, double dmin) {
  return minmax_phi(delta, dmax, dmin);
}

// ---------------------------------------------------------------------------
// Sweeps

// Initial state: free stream everywhere, then the wall tangency projection
// (otherwise the residual of the first iteration is identically zero).
void lskum_ref_init_state(const lskum_ref_cloud *c, const lskum_ref_params *p, double *U) {
  double Uinf[4];
  lskum_ref_free_stream(p, Uinf);
  const int32_t n = c->n;
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    for (int m = 0; m < 4; ++m) fld(U, m, n, i) = Uinf[m];
    if (c->kind[i] == 1) {
      double mn = fld(U, 1, n, i) * c->nx[i] + fld(U, 2, n, i) * c->ny[i];
      fld(U, 1, n, i) = fld(U, 1, n, i) - mn * c->nx[i];
      fld(U, 2, n, i) = fld(U, 2, n, i) - mn * c->ny[i];
    }
  }
}

// eq. (13) at every point.
unsigned lskum_ref_q_vars(const lskum_ref_cloud *c, const lskum_ref_params *p, const double *U,
                          double *q) {
  unsigned flags = 0;
  const int32_t n = c->n;
#pragma omp parallel for schedule(static) reduction(|: flags)
  for (int32_t i = 0; i < n; ++i) {
    double Ui[4], qi[4];
    for (int m = 0; m < 4; ++m) Ui[m] = fld(U, m, n, i);
    flags |= q_point(p->gamma, Ui, qi);
    for (int m = 0; m < 4; ++m) fld(q, m, n, i) = qi[m];
  }
  return flags;
}

void lskum_ref_q_derivs_first(const lskum_ref_cloud *c, const double *q, double *dq,
                              double *qlim) {
  const int32_t n = c->n;
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    ArraySt st{{q, nullptr, nullptr}, n, i, c->col + c->row_ptr[i]};
    double d[8], l[8];
    deriv_first_point(*c, i, st, d, l);
    for (int m = 0; m < 8; ++m) {
      fld(dq, m, n, i) = d[m];
      fld(qlim, m, n, i) = l[m];
    }
  }
}

void lskum_ref_q_derivs_inner(const lskum_ref_cloud *c, const double *q, const double *dq_prev,
                              double *dq_next) {
  const int32_t n = c->n;
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    ArraySt st{{q, dq_prev, nullptr}, n, i, c->col + c->row_ptr[i]};
    double d[8];
    deriv_inner_point(*c, i, st, d);
    for (int m = 0; m < 8; ++m) fld(dq_next, m, n, i) = d[m];
  }
}

void lskum_ref_q_derivs(const lskum_ref_cloud *c, const lskum_ref_params *p, const double *q,
                        double *dq, double *qlim) {
  lskum_ref_q_derivs_first(c, q, dq, qlim);
  if (p->n_inner <= 0) return;
  std::vector<double> tmp((size_t)8 * (size_t)c->n);
  for (int32_t it = 0; it < p->n_inner; ++it) {
    lskum_ref_q_derivs_inner(c, q, dq, tmp.data());
    for (size_t k = 0; k < tmp.size(); ++k) dq[k] = tmp[k];
  }
}

// Flux residual at every non-outer point: the sum of the split-flux
// derivatives of eq. (10), each from eq. (11) on its half-plane stencil, in
// the point's own (s, n) frame with t = (n_y, -n_x):
//   N_s^+ = {ds < 0}, N_s^- = {ds > 0}, N_n^+ = {dn < 0}, N_n^- = {dn > 0}
// (strict, so neighbours on the splitting line are in neither half).  The
// flux differences are dG_i = G(q~_i) - G(q~_0) with the modified q of
// eq. (14), each increment limited by the Venkatakrishnan factor with
// eps^2 = (K |d_i|)^3 and the stencil bounds of its own end point.
// Interior points use all four splits (with the interior frame t = (1,0),
// n = (0,1) this is exactly the x/y scheme of eq. (10)); wall points, whose
// normal points into the fluid, use G_s^+, G_s^- and G_n^-.  Outer points
// are Dirichlet and get R = 0.  Momentum is rotated back to x/y.
unsigned lskum_ref_flux_residual(const lskum_ref_cloud *c, const lskum_ref_params *p,
                                 const double *q, const double *dq, const double *qlim,
                                 double *R) {
  const int32_t n = c->n;
  unsigned flags = 0;
#pragma omp parallel for schedule(static) reduction(|: flags)
  for (int32_t i = 0; i < n; ++i) {
    ArraySt st{{q, dq, qlim}, n, i, c->col + c->row_ptr[i]};
    double Ri[4];
    flags |= flux_point(*c, *p, i, st, Ri);
    for (int m = 0; m < 4; ++m) fld(R, m, n, i) = Ri[m];
  }
  return flags;
}

// Operation counts of the flux residual over the whole cloud, evaluated with
// the counting scalar on the given fields: counts = {add/sub, mul, div,
// sqrt, exp, log, erf} summed over all points.
unsigned lskum_ref_flux_op_counts(const lskum_ref_cloud *c, const lskum_ref_params *p,
                                  const double *q, const double *dq, const double *qlim,
                                  double counts[7]) {
  struct CountSt {
    ArraySt a;
    cnt::Num own(int f, int m) const { return cnt::Num(a.own(f, m)); }
    cnt::Num nbr(int k, int f, int m) const { return cnt::Num(a.nbr(k, f, m)); }
  };
  cnt::Tally t;
  cnt::tally = &t;
  const int32_t n = c->n;
  unsigned flags = 0;
  for (int32_t i = 0; i < n; ++i) {
    CountSt st{ArraySt{{q, dq, qlim}, n, i, c->col + c->row_ptr[i]}};
    cnt::Num Ri[4];
    flags |= flux_point(*c, *p, i, st, Ri);
  }
  cnt::tally = nullptr;
  const double v[7] = {t.add, t.mul, t.div, t.sqrt, t.exp, t.log, t.erf};
  for (int k = 0; k < 7; ++k) counts[k] = v[k];
  return flags;
}

// Local time step: dt_0 = CFL * min over the real neighbours i of
// |d_i| / (|u_i| + 3 sqrt(p_i / rho_i)).
void lskum_ref_local_dt(const lskum_ref_cloud *c, const lskum_ref_params *p, const double *U,
                        double *dt) {
  const int32_t n = c->n;
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    Row r = row(*c, i);
    double best = std::numeric_limits<double>::infinity();
    for (int32_t k = 0; k < r.count; ++k) {
      int32_t j = r.ids[k];
      double dx = c->x[j] - c->x[i];
      double dy = c->y[j] - c->y[i];
      double dist = std::sqrt(dx * dx + dy * dy);
      double Uj[4], w[4];
      for (int m = 0; m < 4; ++m) Uj[m] = fld(U, m, n, j);
      prim_from_cons(p->gamma, Uj, w);
      double speed = std::sqrt(w[1] * w[1] + w[2] * w[2]) + 3.0 * std::sqrt(w[3] / w[0]);
      double d = dist / speed;
      if (d < best) best = d;
    }
    dt[i] = p->cfl * best;
  }
}

// One stage of the four-stage, third-order SSP Runge-Kutta scheme with the
// local time step and L(U) = -R(U); each stage is the forward-Euler update of
// eq. (16) followed by a convex blend:
//   U1 = Un + dt/2 L(Un),  U2 = U1 + dt/2 L(U1),
//   U3 = 2/3 Un + 1/3 (U2 + dt/2 L(U2)),  U4 = U3 + dt/2 L(U3).
// Then: wall points drop the normal momentum (m <- m - (m.n) n); outer
// points are reset to the free stream.
void lskum_ref_rk_stage(const lskum_ref_cloud *c, const lskum_ref_params *p, int stage,
                        const double *Un, const double *R, const double *dt, double *U) {
  const int32_t n = c->n;
  double Uinf[4];
  lskum_ref_free_stream(p, Uinf);
  const double a = stage == 2 ? 2.0 / 3.0 : 0.0;
  const double b = stage == 2 ? 1.0 / 3.0 : 1.0;
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    if (c->kind[i] == 2) {
      for (int m = 0; m < 4; ++m) fld(U, m, n, i) = Uinf[m];
      continue;
    }
    for (int m = 0; m < 4; ++m) {
      double euler = fld(U, m, n, i) - 0.5 * dt[i] * fld(R, m, n, i);
      fld(U, m, n, i) = stage == 2 ? a * fld(Un, m, n, i) + b * euler : euler;
    }
    if (c->kind[i] == 1) {
      double mn = fld(U, 1, n, i) * c->nx[i] + fld(U, 2, n, i) * c->ny[i];
      fld(U, 1, n, i) = fld(U, 1, n, i) - mn * c->nx[i];
      fld(U, 2, n, i) = fld(U, 2, n, i) - mn * c->ny[i];
    }
  }
}

// One stage of the classical fourth-order Runge-Kutta scheme with the same
// local time step and L(U) = -R(U) (k_s = L of stage s's input):
//   U1 = Un + dt/2 k_0,  U2 = Un + dt/2 k_1,  U3 = Un + dt k_2,
//   U4 = Un + dt/6 (k_0 + 2 k_1 + 2 k_2 + k_3).
// Rs holds R(U0) .. R(U_stage) as consecutive [4][n] fields.  The boundary
// conditions follow every stage as in lskum_ref_rk_stage.
void lskum_ref_rk4_stage(const lskum_ref_cloud *c, const lskum_ref_params *p, int stage,
                         const double *Un, const double *Rs, const double *dt, double *U) {
  const int32_t n = c->n;
  const size_t F = 4 * (size_t)n;
  double Uinf[4];
  lskum_ref_free_stream(p, Uinf);
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    if (c->kind[i] == 2) {
      for (int m = 0; m < 4; ++m) fld(U, m, n, i) = Uinf[m];
      continue;
    }
    for (int m = 0; m < 4; ++m) {
      auto k = [&](int s) { return -fld(Rs + (size_t)s * F, m, n, i); };
      double v;
      if (stage < 2)
        v = fld(Un, m, n, i) + 0.5 * dt[i] * k(stage);
      else if (stage == 2)
        v = fld(Un, m, n, i) + dt[i] * k(2);
      else
        v = fld(Un, m, n, i) + dt[i] / 6.0 * (k(0) + 2.0 * k(1) + 2.0 * k(2) + k(3));
      fld(U, m, n, i) = v;
    }
    if (c->kind[i] == 1) {
      double mn = fld(U, 1, n, i) * c->nx[i] + fld(U, 2, n, i) * c->ny[i];
      fld(U, 1, n, i) = fld(U, 1, n, i) - mn * c->nx[i];
      fld(U, 2, n, i) = fld(U, 2, n, i) - mn * c->ny[i];
    }
  }
}

// L2 norm of the density residual over interior and wall points.
double lskum_ref_residual_norm(const lskum_ref_cloud *c, const double *R) {
  std::vector<double> v;
  v.reserve((size_t)c->n);
  for (int32_t i = 0; i < c->n; ++i)
    if (c->kind[i] != 2) v.push_back(R[i] * R[i]);
  return std::sqrt(pairwise_sum(v.data(), v.size()));
}

// Lift and drag coefficients of the wall polygon (see force_t).
void lskum_ref_force_coeffs(const lskum_ref_cloud *c, const lskum_ref_params *p,
                            const double *U, double clcd[2]) {
  const int32_t n = c->n;
  auto Uw = [&](int32_t j, int k) { return fld(U, k, n, j); };
  force_t<double>(*c, p->gamma, p->mach, p->aoa_rad, Uw, clcd);
}

unsigned lskum_ref_iterate(const lskum_ref_cloud *c, const lskum_ref_params *p, int32_t iters,
                           double *U, double *hist) {
  const size_t n = (size_t)c->n;
  // Rs keeps the residual of every stage (the classical RK4 update needs all four)
  std::vector<double> Un(4 * n), q(4 * n), dq(8 * n), qlim(8 * n), Rs(16 * n), dt(n);
  const bool rk4 = (p->options & LSKUM_REF_RK4) != 0;
  unsigned flags = 0;
  for (int32_t it = 0; it < iters; ++it) {
    lskum_ref_local_dt(c, p, U, dt.data());
    for (size_t k = 0; k < 4 * n; ++k) Un[k] = U[k];
    for (int s = 0; s < 4; ++s) {
      double *R = Rs.data() + (size_t)s * 4 * n;
      flags |= lskum_ref_q_vars(c, p, U, q.data());
      lskum_ref_q_derivs(c, p, q.data(), dq.data(), qlim.data());
      flags |= lskum_ref_flux_residual(c, p, q.data(), dq.data(), qlim.data(), R);
      if (s == 0 && hist) hist[it] = lskum_ref_residual_norm(c, R);
      if (rk4)
        lskum_ref_rk4_stage(c, p, s, Un.data(), Rs.data(), dt.data(), U);
      else
        lskum_ref_rk_stage(c, p, s, Un.data(), R, dt.data(), U);
    }
  }
  return flags;
}

// ---------------------------------------------------------------------------
// Adjoints (reverse mode through the same point formulas, differentiating
// the branch each limiter, max/min and stencil test takes).

// Cotangent of the residual map (U_int, theta) -> R, where the rows of the
// outer points are the free stream U_inf(theta), theta = (M, alpha):
//   Ubar     = (dR/dU)^T Rbar at interior and wall rows, 0 at outer rows;
//   thetabar = sum over outer rows j of (dR/dU_j)^T Rbar . dU_inf/dtheta.
// The derivative recomputes q and every derivative iterate, then runs the
// passes backwards: flux, inner sweeps n_inner..1, first-order pass
// (derivatives and stencil bounds), q-variables.
unsigned lskum_ref_residual_vjp(const lskum_ref_cloud *c, const lskum_ref_params *p,
                                const double *U, const double *Rbar, double *Ubar,
                                double thetabar[2]) {
  const int32_t n = c->n;
  const size_t N = (size_t)n;
  const int K = p->n_inner > 0 ? p->n_inner : 0;
  unsigned flags = 0;
  std::vector<double> q(4 * N), qlim(8 * N);
  std::vector<std::vector<double>> dq((size_t)K + 1, std::vector<double>(8 * N));
  flags |= lskum_ref_q_vars(c, p, U, q.data());
  lskum_ref_q_derivs_first(c, q.data(), dq[0].data(), qlim.data());
  for (int k = 1; k <= K; ++k)
    lskum_ref_q_derivs_inner(c, q.data(), dq[(size_t)k - 1].data(), dq[(size_t)k].data());

  ad::Tape tp;
  ad::tape = &tp;
  std::vector<double> qbar(4 * N, 0.0), gbar(8 * N, 0.0), lbar(8 * N, 0.0), gprev(8 * N);

  // flux residual
  for (int32_t i = 0; i < n; ++i) {
    if (c->kind[i] == 2) continue;
    tp.clear();
    const double *f[3] = {q.data(), dq[(size_t)K].data(), qlim.data()};
    TapeSt st(f, n, i, row(*c, i), 7u);
    ad::Var R[4];
    flags |= flux_point(*c, *p, i, st, R);
    seed_begin();
    for (int m = 0; m < 4; ++m) seed(R[m], fld(Rbar, m, n, i));
    tp.reverse();
    double *bar[3] = {qbar.data(), gbar.data(), lbar.data()};
    st.scatter(bar);
  }
  // inner sweeps, last first
  for (int k = K; k >= 1; --k) {
    std::fill(gprev.begin(), gprev.end(), 0.0);
    for (int32_t i = 0; i < n; ++i) {
      tp.clear();
      const double *f[3] = {q.data(), dq[(size_t)k - 1].data(), nullptr};
      TapeSt st(f, n, i, row(*c, i), 3u);
      ad::Var d[8];
      deriv_inner_point(*c, i, st, d);
      seed_begin();
      for (int m = 0; m < 8; ++m) seed(d[m], fld(gbar.data(), m, n, i));
      tp.reverse();
      double *bar[3] = {qbar.data(), gprev.data(), nullptr};
      st.scatter(bar);
    }
    gbar.swap(gprev);
  }
  // first-order derivatives and stencil bounds
  for (int32_t i = 0; i < n; ++i) {
    tp.clear();
    const double *f[3] = {q.data(), nullptr, nullptr};
    TapeSt st(f, n, i, row(*c, i), 1u);
    ad::Var d[8], l[8];
    deriv_first_point(*c, i, st, d, l);
    seed_begin();
    for (int m = 0; m < 8; ++m) {
      seed(d[m], fld(gbar.data(), m, n, i));
      seed(l[m], fld(lbar.data(), m, n, i));
    }
    tp.reverse();
    double *bar[3] = {qbar.data(), nullptr, nullptr};
    st.scatter(bar);
  }
  // q-variables; outer rows go to theta
  double ubar_outer[4] = {0.0, 0.0, 0.0, 0.0};
  for (int32_t i = 0; i < n; ++i) {
    tp.clear();
    ad::Var Ui[4], qi[4];
    for (int m = 0; m < 4; ++m) Ui[m] = ad::input(fld(U, m, n, i));
    q_point(p->gamma, Ui, qi);
    seed_begin();
    for (int m = 0; m < 4; ++m) seed(qi[m], fld(qbar.data(), m, n, i));
    tp.reverse();
    for (int m = 0; m < 4; ++m) {
      const double g = adjoint(Ui[m]);
      if (c->kind[i] == 2) {
        ubar_outer[m] += g;
        fld(Ubar, m, n, i) = 0.0;
      } else {
        fld(Ubar, m, n, i) = g;
      }
    }
  }
  tp.clear();
  ad::Var mach = ad::input(p->mach), aoa = ad::input(p->aoa_rad), w[4], Uinf[4];
  free_stream_prim_t(p->gamma, mach, aoa, w);
  cons_from_prim(p->gamma, w, Uinf);
  seed_begin();
  for (int m = 0; m < 4; ++m) seed(Uinf[m], ubar_outer[m]);
  tp.reverse();
  thetabar[0] = adjoint(mach);
  thetabar[1] = adjoint(aoa);
  ad::tape = nullptr;
  return flags;
}

// Cotangent of (Cl, Cd) with weights Jbar = (Jbar_l, Jbar_d):
//   Ubar = (d(Jbar.C)/dU)^T (non-zero at wall points only),
//   thetabar = d(Jbar.C)/d(M, alpha) at fixed U.
void lskum_ref_force_coeffs_vjp(const lskum_ref_cloud *c, const lskum_ref_params *p,
                                const double *U, const double Jbar[2], double *Ubar,
                                double thetabar[2]) {
  const int32_t n = c->n;
  ad::Tape tp;
  ad::tape = &tp;
  std::vector<ad::Var> Uv(4 * (size_t)n);
  for (int32_t e = 0; e < c->n_wall; ++e) {
    const int32_t j = c->wall_loop[e];
    for (int k = 0; k < 4; ++k) Uv[(size_t)k * n + j] = ad::input(fld(U, k, n, j));
  }
  ad::Var mach = ad::input(p->mach), aoa = ad::input(p->aoa_rad), C[2];
  auto Uw = [&](int32_t j, int k) { return Uv[(size_t)k * n + j]; };
  force_t<ad::Var>(*c, p->gamma, mach, aoa, Uw, C);
  seed_begin();
  seed(C[0], Jbar[0]);
  seed(C[1], Jbar[1]);
  tp.reverse();
  for (size_t k = 0; k < 4 * (size_t)n; ++k) Ubar[k] = adjoint(Uv[k]);
  thetabar[0] = adjoint(mach);
  thetabar[1] = adjoint(aoa);
  ad::tape = nullptr;
}

}  // extern "C"
