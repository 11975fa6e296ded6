/* lskum_ref.h -- FP64 CPU oracle for the LSKUM residual sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the GPU library is checked against.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header or table with the GPU library.
 *
 * Every pointer is a HOST pointer.  Arrays are structure-of-arrays,
 * component-major: a field with c components over n points is stored as
 * f[c*n + i].  All floating point is IEEE binary64, evaluated in source
 * order (built with -ffp-contract=off), with glibc's exp/log/erf/sqrt.
 *
 * Field layouts:
 *   U    [4][n]  conserved (rho, rho*u, rho*v, E)
 *   q    [4][n]  q-variables, eq. (13)
 *   dq   [8][n]  rows 0..3: dq_m/dx, rows 4..7: dq_m/dy
 *   qlim [8][n]  rows 0..3: max of q_m over {i} U N(i), rows 4..7: min
 *   R    [4][n]  flux residual (sum of split-flux derivatives), x/y momentum
 *   dt   [n]     local time step
 */
#ifndef LSKUM_REF_H
#define LSKUM_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n;               /* number of points */
  const double *x, *y;     /* [n] coordinates */
  const double *nx, *ny;   /* [n] unit normal; tangent t = (ny, -nx) */
  const int8_t *kind;      /* [n] 0 interior, 1 wall, 2 outer */
  const int64_t *row_ptr;  /* [n+1] */
  const int32_t *col;      /* neighbour ids; row i starts at row_ptr[i] */
  const int32_t *nbr_count;/* [n] real neighbours of row i */
  const int32_t *wall_loop;/* [n_wall] wall ids, counter-clockwise */
  int32_t n_wall;
} lskum_ref_cloud;

typedef struct {
  double gamma;    /* ratio of specific heats */
  double mach;     /* free-stream Mach number */
  double aoa_rad;  /* angle of attack, radians */
  double cfl;      /* CFL number of the local time step */
  double venkat_k; /* limiter constant K: eps^2 = (K |d|)^3 */
  int32_t n_inner; /* corrective (inner) LS sweeps after the first-order one */
  int32_t options; /* scheme variant bits (0: the default scheme) */
} lskum_ref_params;

/* options bits */
#define LSKUM_REF_FIRST_ORDER 1u /* split fluxes of q itself (no reconstruction) */
#define LSKUM_REF_MINMAX      2u /* min-max limiter instead of Venkatakrishnan */
#define LSKUM_REF_RK4         4u /* classical four-stage Runge-Kutta time stepping */

/* status bits returned by the sweep routines */
#define LSKUM_REF_NONPHYSICAL 1u  /* rho, p or beta <= 0, or non-finite */
#define LSKUM_REF_DEGENERATE  2u  /* a used half-plane stencil is singular */

/* threads the forward sweeps use: omp_get_max_threads() in the OpenMP
 * build, 1 in the parity build */
int lskum_ref_threads(void);

/* point-level formulas (exported for the pinning tests) */
void lskum_ref_free_stream(const lskum_ref_params *p, double U[4]);
void lskum_ref_q_from_prim(double gamma, const double prim[4], double q[4]);
void lskum_ref_prim_from_q(double gamma, const double q[4], double prim[4]);
void lskum_ref_cons_from_prim(double gamma, const double prim[4], double U[4]);
void lskum_ref_prim_from_cons(double gamma, const double U[4], double prim[4]);
/* split flux in a local frame: w = (rho, u_s, u_n, p); dir 0 = s, 1 = n;
 * sign +1 or -1.  Output ordered (mass, s-momentum, n-momentum, energy). */
void lskum_ref_split_flux(double gamma, int dir, int sign, const double w[4], double G[4]);
/* limiter factor phi for increment delta with bounds dmax >= 0 >= dmin */
double lskum_ref_venkat_phi(double delta, double dmax, double dmin, double eps2);
/* min-max limiter factor: min(1, D/delta), D the bound on delta's side */
double lskum_ref_minmax_phi(double delta, double dmax, double dmin);

/* sweep routines (one call = one pass over all points) */
void lskum_ref_init_state(const lskum_ref_cloud *c, const lskum_ref_params *p, double *U);
unsigned lskum_ref_q_vars(const lskum_ref_cloud *c, const lskum_ref_params *p,
                          const double *U, double *q);
void lskum_ref_q_derivs_first(const lskum_ref_cloud *c, const double *q, double *dq,
                              double *qlim);
void lskum_ref_q_derivs_inner(const lskum_ref_cloud *c, const double *q,
                              const double *dq_prev, double *dq_next);
/* first-order pass followed by n_inner Jacobi sweeps */
void lskum_ref_q_derivs(const lskum_ref_cloud *c, const lskum_ref_params *p,
                        const double *q, double *dq, double *qlim);
unsigned lskum_ref_flux_residual(const lskum_ref_cloud *c, const lskum_ref_params *p,
                                 const double *q, const double *dq, const double *qlim,
                                 double *R);
void lskum_ref_local_dt(const lskum_ref_cloud *c, const lskum_ref_params *p,
                        const double *U, double *dt);
void lskum_ref_rk_stage(const lskum_ref_cloud *c, const lskum_ref_params *p, int stage,
                        const double *Un, const double *R, const double *dt, double *U);
/* classical RK4 stage: Rs holds the residuals of stages 0..stage as
 * consecutive [4][n] fields; U receives stage `stage`'s output */
void lskum_ref_rk4_stage(const lskum_ref_cloud *c, const lskum_ref_params *p, int stage,
                         const double *Un, const double *Rs, const double *dt, double *U);
double lskum_ref_residual_norm(const lskum_ref_cloud *c, const double *R);
void lskum_ref_force_coeffs(const lskum_ref_cloud *c, const lskum_ref_params *p,
                            const double *U, double clcd[2]);

/* operation counts of lskum_ref_flux_residual on these fields, summed over
 * the cloud: counts[7] = {add/sub, mul, div, sqrt, exp, log, erf} on
 * state-dependent values (edge geometry in plain doubles is not counted) */
unsigned lskum_ref_flux_op_counts(const lskum_ref_cloud *c, const lskum_ref_params *p,
                                  const double *q, const double *dq, const double *qlim,
                                  double counts[7]);

/* whole iterations: U is advanced in place; hist[k] receives the residual
 * norm of iteration k (first stage).  Returns the OR of all status bits. */
unsigned lskum_ref_iterate(const lskum_ref_cloud *c, const lskum_ref_params *p,
                           int32_t iters, double *U, double *hist);

/* adjoints (reverse mode through the same formulas, active branches).
 * residual_vjp: the residual as a function of the interior and wall rows of
 * U and of theta = (M, alpha [rad]), the outer rows being U_inf(theta):
 *   Ubar [4][n] = (dR/dU)^T Rbar, zero at outer rows;
 *   thetabar[2] = sum_outer (dR/dU_j)^T Rbar . dU_inf/dtheta.
 * force_coeffs_vjp: Jbar = weights of (Cl, Cd); Ubar [4][n] (wall rows
 * only non-zero) and thetabar[2] = partial derivatives at fixed U. */
unsigned lskum_ref_residual_vjp(const lskum_ref_cloud *c, const lskum_ref_params *p,
                                const double *U, const double *Rbar, double *Ubar,
                                double thetabar[2]);
void lskum_ref_force_coeffs_vjp(const lskum_ref_cloud *c, const lskum_ref_params *p,
                                const double *U, const double Jbar[2], double *Ubar,
                                double thetabar[2]);

#ifdef __cplusplus
}
#endif
#endif
