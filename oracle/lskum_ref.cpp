// lskum_ref.cpp -- FP64 CPU oracle for the LSKUM residual sweep.
//
// TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked
// against.  Only the test suite, the smoke check and the benchmark's CPU
// baseline may load it.  It shares no code with the GPU library.
//
// Plain loops over points in index order, one point at a time, evaluated in
// the order the formulas are written (the library is built with
// -ffp-contract=off, no -ffast-math).  The per-point formulas are templates
// over the scalar type so that the same text can later be evaluated with an
// operation-counting or a reverse-mode scalar.
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

#include "lskum_ref.h"

#include <cmath>
#include <cstddef>
#include <limits>
#include <vector>

namespace {

const double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Point-level formulas

// Free stream, non-dimensionalised by the free-stream density and sound
// speed: rho = 1, p = 1/gamma (so a = 1), velocity = M (cos a, sin a).
void free_stream_prim(const lskum_ref_params &P, double w[4]) {
  w[0] = 1.0;
  w[1] = P.mach * std::cos(P.aoa_rad);
  w[2] = P.mach * std::sin(P.aoa_rad);
  w[3] = 1.0 / P.gamma;
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
double pairwise_sum(const double *v, size_t n) {
  if (n == 0) return 0.0;
  if (n <= 8) {
    double s = 0.0;
    for (size_t k = 0; k < n; ++k) s += v[k];
    return s;
  }
  size_t h = n / 2;
  return pairwise_sum(v, h) + pairwise_sum(v + h, n - h);
}

}  // namespace

// ---------------------------------------------------------------------------
// Exported point-level formulas

extern "C" {

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

// ---------------------------------------------------------------------------
// Sweeps

// Initial state: free stream everywhere, then the wall tangency projection
// (otherwise the residual of the first iteration is identically zero).
void lskum_ref_init_state(const lskum_ref_cloud *c, const lskum_ref_params *p, double *U) {
  double Uinf[4];
  lskum_ref_free_stream(p, Uinf);
  const int32_t n = c->n;
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
  for (int32_t i = 0; i < n; ++i) {
    double Ui[4], w[4], qi[4];
    for (int m = 0; m < 4; ++m) Ui[m] = fld(U, m, n, i);
    prim_from_cons(p->gamma, Ui, w);
    if (!finite_positive(w[0]) || !finite_positive(w[3])) flags |= LSKUM_REF_NONPHYSICAL;
    q_from_prim(p->gamma, w, qi);
    for (int m = 0; m < 4; ++m) fld(q, m, n, i) = qi[m];
  }
  return flags;
}

// First-order least squares (eq. (9) with the plain differences
// dq_i = q_i - q_0) over the full stencil, and the stencil bounds
// max/min of q over {P0} U N(P0).
void lskum_ref_q_derivs_first(const lskum_ref_cloud *c, const double *q, double *dq,
                              double *qlim) {
  const int32_t n = c->n;
  for (int32_t i = 0; i < n; ++i) {
    Row r = row(*c, i);
    double sxx = 0.0, sxy = 0.0, syy = 0.0;
    double sxq[4] = {0, 0, 0, 0}, syq[4] = {0, 0, 0, 0};
    double qmax[4], qmin[4];
    for (int m = 0; m < 4; ++m) qmax[m] = qmin[m] = fld(q, m, n, i);
    for (int32_t k = 0; k < r.count; ++k) {
      int32_t j = r.ids[k];
      double dx = c->x[j] - c->x[i];
      double dy = c->y[j] - c->y[i];
      sxx += dx * dx;
      sxy += dx * dy;
      syy += dy * dy;
      for (int m = 0; m < 4; ++m) {
        double qj = fld(q, m, n, j);
        double d = qj - fld(q, m, n, i);
        sxq[m] += dx * d;
        syq[m] += dy * d;
        if (qj > qmax[m]) qmax[m] = qj;
        if (qj < qmin[m]) qmin[m] = qj;
      }
    }
    double det = sxx * syy - sxy * sxy;
    for (int m = 0; m < 4; ++m) {
      fld(dq, m, n, i) = (syy * sxq[m] - sxy * syq[m]) / det;
      fld(dq, 4 + m, n, i) = (sxx * syq[m] - sxy * sxq[m]) / det;
      fld(qlim, m, n, i) = qmax[m];
      fld(qlim, 4 + m, n, i) = qmin[m];
    }
  }
}

// One inner iteration (eq. (14)-(15)): the modified differences use the
// previous iterate of the derivatives at both ends of each edge,
//   dq~_i = [q_i - (dx q_x,i + dy q_y,i)/2] - [q_0 - (dx q_x,0 + dy q_y,0)/2],
// and the same least-squares solve gives the next iterate (Jacobi: every
// point reads only the previous iterate).
void lskum_ref_q_derivs_inner(const lskum_ref_cloud *c, const double *q, const double *dq_prev,
                              double *dq_next) {
  const int32_t n = c->n;
  for (int32_t i = 0; i < n; ++i) {
    Row r = row(*c, i);
    double sxx = 0.0, sxy = 0.0, syy = 0.0;
    double sxq[4] = {0, 0, 0, 0}, syq[4] = {0, 0, 0, 0};
    for (int32_t k = 0; k < r.count; ++k) {
      int32_t j = r.ids[k];
      double dx = c->x[j] - c->x[i];
      double dy = c->y[j] - c->y[i];
      sxx += dx * dx;
      sxy += dx * dy;
      syy += dy * dy;
      for (int m = 0; m < 4; ++m) {
        double qt_j = fld(q, m, n, j) -
                      0.5 * (dx * fld(dq_prev, m, n, j) + dy * fld(dq_prev, 4 + m, n, j));
        double qt_0 = fld(q, m, n, i) -
                      0.5 * (dx * fld(dq_prev, m, n, i) + dy * fld(dq_prev, 4 + m, n, i));
        double d = qt_j - qt_0;
        sxq[m] += dx * d;
        syq[m] += dy * d;
      }
    }
    double det = sxx * syy - sxy * sxy;
    for (int m = 0; m < 4; ++m) {
      fld(dq_next, m, n, i) = (syy * sxq[m] - sxy * syq[m]) / det;
      fld(dq_next, 4 + m, n, i) = (sxx * syq[m] - sxy * sxq[m]) / det;
    }
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
  const double g = p->gamma;
  unsigned flags = 0;
  for (int32_t i = 0; i < n; ++i) {
    const int kind = c->kind[i];
    if (kind == 2) {
      for (int m = 0; m < 4; ++m) fld(R, m, n, i) = 0.0;
      continue;
    }
    const double nx = c->nx[i], ny = c->ny[i];
    const double tx = ny, ty = -nx;
    // split order: 0 = s+, 1 = s-, 2 = n+, 3 = n-
    double sss[4] = {0, 0, 0, 0}, ssn[4] = {0, 0, 0, 0}, snn[4] = {0, 0, 0, 0};
    double as[4][4] = {{0}}, an[4][4] = {{0}};
    int cnt[4] = {0, 0, 0, 0};
    Row r = row(*c, i);
    for (int32_t k = 0; k < r.count; ++k) {
      int32_t j = r.ids[k];
      double dx = c->x[j] - c->x[i];
      double dy = c->y[j] - c->y[i];
      double ds = dx * tx + dy * ty;
      double dn = dx * nx + dy * ny;
      double dist = std::sqrt(dx * dx + dy * dy);
      double kd = p->venkat_k * dist;
      double eps2 = kd * kd * kd;
      double qt_j[4], qt_0[4];
      for (int m = 0; m < 4; ++m) {
        double qj = fld(q, m, n, j), q0 = fld(q, m, n, i);
        double del_j = -0.5 * (dx * fld(dq, m, n, j) + dy * fld(dq, 4 + m, n, j));
        double del_0 = -0.5 * (dx * fld(dq, m, n, i) + dy * fld(dq, 4 + m, n, i));
        double phi_j = venkat_phi(del_j, fld(qlim, m, n, j) - qj, fld(qlim, 4 + m, n, j) - qj,
                                  eps2);
        double phi_0 = venkat_phi(del_0, fld(qlim, m, n, i) - q0, fld(qlim, 4 + m, n, i) - q0,
                                  eps2);
        qt_j[m] = qj + phi_j * del_j;
        qt_0[m] = q0 + phi_0 * del_0;
      }
      double wj[4], w0[4];
      prim_from_q(g, qt_j, wj);
      prim_from_q(g, qt_0, w0);
      if (!(qt_j[3] < 0.0) || !(qt_0[3] < 0.0) || !finite_positive(wj[0]) ||
          !finite_positive(w0[0]) || !finite_positive(wj[3]) || !finite_positive(w0[3]))
        flags |= LSKUM_REF_NONPHYSICAL;
      // velocities in P0's frame
      double lj[4] = {wj[0], wj[1] * tx + wj[2] * ty, wj[1] * nx + wj[2] * ny, wj[3]};
      double l0[4] = {w0[0], w0[1] * tx + w0[2] * ty, w0[1] * nx + w0[2] * ny, w0[3]};
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
        double Gj[4], G0[4];
        split_flux(g, dir, sign, lj, Gj);
        split_flux(g, dir, sign, l0, G0);
        sss[sp] += ds * ds;
        ssn[sp] += ds * dn;
        snn[sp] += dn * dn;
        cnt[sp] += 1;
        for (int m = 0; m < 4; ++m) {
          double dG = Gj[m] - G0[m];
          as[sp][m] += ds * dG;
          an[sp][m] += dn * dG;
        }
      }
    }
    double Rf[4] = {0, 0, 0, 0};
    for (int sp = 0; sp < 4; ++sp) {
      if (sp == 2 && kind != 0) continue;
      double det = sss[sp] * snn[sp] - ssn[sp] * ssn[sp];
      if (cnt[sp] < 2 || !(det > 1e-12 * sss[sp] * snn[sp])) {
        flags |= LSKUM_REF_DEGENERATE;
        continue;
      }
      for (int m = 0; m < 4; ++m) {
        double d;
        if (sp < 2)
          d = (snn[sp] * as[sp][m] - ssn[sp] * an[sp][m]) / det;
        else
          d = (sss[sp] * an[sp][m] - ssn[sp] * as[sp][m]) / det;
        Rf[m] += d;
      }
    }
    fld(R, 0, n, i) = Rf[0];
    fld(R, 1, n, i) = Rf[1] * tx + Rf[2] * nx;
    fld(R, 2, n, i) = Rf[1] * ty + Rf[2] * ny;
    fld(R, 3, n, i) = Rf[3];
  }
  return flags;
}

// Local time step: dt_0 = CFL * min over the real neighbours i of
// |d_i| / (|u_i| + 3 sqrt(p_i / rho_i)).
void lskum_ref_local_dt(const lskum_ref_cloud *c, const lskum_ref_params *p, const double *U,
                        double *dt) {
  const int32_t n = c->n;
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

// L2 norm of the density residual over interior and wall points.
double lskum_ref_residual_norm(const lskum_ref_cloud *c, const double *R) {
  std::vector<double> v;
  v.reserve((size_t)c->n);
  for (int32_t i = 0; i < c->n; ++i)
    if (c->kind[i] != 2) v.push_back(R[i] * R[i]);
  return std::sqrt(pairwise_sum(v.data(), v.size()));
}

// Lift and drag from the wall polygon W_0..W_{m-1} (counter-clockwise):
// edge e = (W_j, W_j+1) has outward normal-length vector (dy_e, -dx_e) and
// pressure p_e = (p_j + p_j+1)/2; Cp_e = (p_e - p_inf)/(rho_inf M^2 / 2);
// (Cx, Cy) = -sum_e Cp_e nu_e (chord 1); Cl = Cy cos a - Cx sin a,
// Cd = Cx cos a + Cy sin a.
void lskum_ref_force_coeffs(const lskum_ref_cloud *c, const lskum_ref_params *p,
                            const double *U, double clcd[2]) {
  const int32_t n = c->n, m = c->n_wall;
  const double pinf = 1.0 / p->gamma;
  const double qinf = 0.5 * 1.0 * p->mach * p->mach;
  std::vector<double> fx((size_t)m), fy((size_t)m);
  for (int32_t e = 0; e < m; ++e) {
    int32_t a = c->wall_loop[e], b = c->wall_loop[(e + 1) % m];
    double Ua[4], Ub[4], wa[4], wb[4];
    for (int k = 0; k < 4; ++k) {
      Ua[k] = fld(U, k, n, a);
      Ub[k] = fld(U, k, n, b);
    }
    prim_from_cons(p->gamma, Ua, wa);
    prim_from_cons(p->gamma, Ub, wb);
    double pe = 0.5 * (wa[3] + wb[3]);
    double cp = (pe - pinf) / qinf;
    double ex = c->x[b] - c->x[a];
    double ey = c->y[b] - c->y[a];
    fx[(size_t)e] = -cp * ey;
    fy[(size_t)e] = cp * ex;
  }
  double Cx = pairwise_sum(fx.data(), fx.size());
  double Cy = pairwise_sum(fy.data(), fy.size());
  double ca = std::cos(p->aoa_rad), sa = std::sin(p->aoa_rad);
  clcd[0] = Cy * ca - Cx * sa;
  clcd[1] = Cx * ca + Cy * sa;
}

unsigned lskum_ref_iterate(const lskum_ref_cloud *c, const lskum_ref_params *p, int32_t iters,
                           double *U, double *hist) {
  const size_t n = (size_t)c->n;
  std::vector<double> Un(4 * n), q(4 * n), dq(8 * n), qlim(8 * n), R(4 * n), dt(n);
  unsigned flags = 0;
  for (int32_t it = 0; it < iters; ++it) {
    lskum_ref_local_dt(c, p, U, dt.data());
    for (size_t k = 0; k < 4 * n; ++k) Un[k] = U[k];
    for (int s = 0; s < 4; ++s) {
      flags |= lskum_ref_q_vars(c, p, U, q.data());
      lskum_ref_q_derivs(c, p, q.data(), dq.data(), qlim.data());
      flags |= lskum_ref_flux_residual(c, p, q.data(), dq.data(), qlim.data(), R.data());
      if (s == 0 && hist) hist[it] = lskum_ref_residual_norm(c, R.data());
      lskum_ref_rk_stage(c, p, s, Un.data(), R.data(), dt.data(), U);
    }
  }
  return flags;
}

}  // extern "C"
