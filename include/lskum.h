/* lskum.h -- C ABI of the MI355X (gfx950) LSKUM residual sweep library.
 *
 * Least-squares kinetic upwind method (LSKUM) for the 2D Euler equations on
 * a point cloud, arXiv 2403.13287 ("Theory of Meshfree LSKUM"): q-variables
 * (eq. (13)), least-squares q-derivatives with inner iterations (eq. (14),
 * (15)), limited reconstruction of the modified q-variables, kinetic split
 * fluxes on half-plane stencils (eq. (10)-(12)), the flux residual, the
 * local time step and a four-stage Runge-Kutta state update built from the
 * forward-Euler update of eq. (16).
 *
 * Conventions
 * -----------
 * - Every field array passed to a sweep call is a DEVICE pointer (for
 *   example torch.cuda tensor storage) in point-major layout: a field with
 *   c components over n points is f[i*c + m] (one contiguous record per
 *   point, so a neighbour's values come in one cache line).  FP64
 *   throughout.  4-component fields must be 32-byte aligned, 8-component
 *   fields 64-byte aligned (LSKUM_ERR_INVALID_ARG otherwise).
 *     U    [n][4]  conserved (rho, rho u, rho v, E)
 *     q    [n][4]  q-variables of eq. (13)
 *     dq   [n][8]  0..3 dq_m/dx, 4..7 dq_m/dy
 *     qlim [n][8]  0..3 max of q_m over {i} U N(i), 4..7 min
 *     R    [n][4]  flux residual, dU/dt = -R (x/y momentum)
 *     dt   [n]     local time step
 * - The caller owns every field buffer; the library never frees caller
 *   memory.  The plan owns the device copies of the geometry and the
 *   connectivity and the tables built from them (allocated in
 *   lskum_plan_create, on a tile-size change, or by the first VJP call) and
 *   frees them all in lskum_plan_destroy.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Sweep calls are asynchronous on that stream; they return LSKUM_OK once
 *   the work is enqueued, or a negative status for invalid arguments or a
 *   failed launch.  Non-physical states met inside kernels are recorded in a
 *   device status word and reported by lskum_status().
 * - Calls on one plan must not run concurrently on different streams: they
 *   share the plan's status word and reduction scratch.
 * - No C++ exception crosses this interface.
 */
#ifndef LSKUM_H
#define LSKUM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LSKUM_OK = 0,
  LSKUM_ERR_INVALID_ARG = -1, /* null pointer, bad size or stage index   */
  LSKUM_ERR_BAD_CLOUD = -2,   /* connectivity fails validation           */
  LSKUM_ERR_HIP = -3,         /* a HIP runtime call or launch failed     */
  LSKUM_ERR_NONPHYSICAL = -4, /* rho, p or beta <= 0 or non-finite met   */
  LSKUM_ERR_NO_MEMORY = -5,   /* device allocation failed                */
  LSKUM_ERR_DEGENERATE = -6,  /* a used half-plane stencil is singular   */
  LSKUM_ERR_SCRATCH_LIMIT = -7 /* cloud larger than a static scratch     */
} lskum_status_t;

/* Point cloud, HOST pointers, read only inside lskum_plan_create. */
typedef struct {
  int32_t n;                 /* number of points, >= 1                          */
  int32_t k_pad;             /* padded row width (columns stored per row)       */
  const double *x, *y;       /* [n] coordinates                                 */
  const double *nx, *ny;     /* [n] unit normal; tangent t = (ny, -nx).  Wall:  */
                             /*     into the fluid; outer: outward; interior:   */
                             /*     the frame of the split stencils             */
  const int8_t *kind;        /* [n] 0 interior, 1 wall, 2 outer (Dirichlet)     */
  const int64_t *row_ptr;    /* [n+1] row i = col[row_ptr[i] .. row_ptr[i+1])   */
  const int32_t *col;        /* neighbour ids, ascending distance, padded       */
  const int32_t *nbr_count;  /* [n] real neighbours in row i (first entries)    */
  const int32_t *wall_loop;  /* [n_wall] wall ids, counter-clockwise            */
  int32_t n_wall;
} lskum_cloud;

/* Flow and scheme settings. */
typedef struct {
  double gamma;     /* ratio of specific heats (1.4)                            */
  double mach;      /* free-stream Mach number; free stream is rho = 1,         */
                    /* p = 1/gamma, velocity = M (cos aoa, sin aoa)             */
  double aoa_rad;   /* angle of attack                                          */
  double cfl;       /* CFL number of the local time step                        */
  double venkat_k;  /* limiter constant K, eps^2 = (K |d_i|)^3                  */
  int32_t n_inner;  /* Jacobi inner sweeps after the first-order LS solve, >= 0 */
  int32_t options;  /* scheme variant bits, 0 = the default scheme (below)      */
} lskum_params;

/* options bits.  LSKUM_FIRST_ORDER: the split fluxes of q itself (no
 * reconstruction; the paper's first-order scheme before the defect
 * correction of eq. (14)), so the flux reads no derivatives and
 * lskum_iterate skips the derivative passes.  LSKUM_MINMAX: the min-max
 * limiter phi = min(1, D/delta) (reconstructed values stay within the
 * stencil bounds) instead of Venkatakrishnan's.  The adjoint entry points
 * support the default residual only (LSKUM_ERR_INVALID_ARG for either bit). */
#define LSKUM_FIRST_ORDER 1
#define LSKUM_MINMAX 2
/* LSKUM_RK4: lskum_iterate advances each iteration with the classical
 * fourth-order Runge-Kutta scheme (lskum_rk4_stage) in place of the SSP
 * Runge-Kutta (4,3) stages; the residual and its adjoints are unchanged. */
#define LSKUM_RK4 4

/* Launch tuning of a plan: the block size (= points per LDS tile of the
 * gather kernels), whether the blocks of the flux kernel and of the
 * per-point kernels are relabelled so that each of the 8 XCDs walks one
 * contiguous range of points (its L2 then holds that range's neighbours;
 * the derivative passes and the local time step always do), and the flux
 * kernel's block size (= points whose records it stages in LDS).  Results
 * do not depend on the tuning. */
typedef struct {
  int32_t block;          /* 128, 256 or 512 (0: 512)                         */
  int32_t xcd_contiguous; /* 0 (default): round-robin over the XCDs;     */
                          /* 1: each XCD walks one contiguous range       */
  int32_t flux_block;     /* 64, 128 or 256 (0: 64)                           */
} lskum_tuning;

typedef struct lskum_plan_s *lskum_plan;
typedef struct lskum_graph_s *lskum_graph;

/* Build a plan on the current HIP device: validates the cloud (ids in
 * range, no self links among the real neighbours, counts within the row,
 * k_pad equal to every row's length) and uploads coordinates, normals,
 * kinds and a column-major copy of the connectivity.  Returns
 * LSKUM_ERR_BAD_CLOUD on a validation failure, LSKUM_ERR_NO_MEMORY or
 * LSKUM_ERR_HIP on device failures; *out is NULL unless LSKUM_OK. */
int lskum_plan_create(lskum_plan *out, const lskum_cloud *cloud, const lskum_params *params,
                      void *stream);

/* Batched plan over n_clouds independent clouds (uneven sizes, each with its
 * own Mach number and angle of attack in params[c]; gamma, cfl, venkat_k and
 * n_inner must be equal across clouds, and all clouds share k_pad).  The
 * clouds are concatenated in the given order: cloud c occupies points
 * lskum_plan_offset(plan, c) .. lskum_plan_offset(plan, c+1)-1 of every field,
 * so all sweep calls below advance every cloud at once; the reductions
 * (residual norm, force coefficients) are per cloud.  tuning may be NULL.
 * A plan from lskum_plan_create is a batch of one cloud.  Errors as for
 * lskum_plan_create, plus LSKUM_ERR_INVALID_ARG for differing shared
 * settings or k_pad. */
int lskum_batch_plan_create(lskum_plan *out, int32_t n_clouds, const lskum_cloud *clouds,
                            const lskum_params *params, const lskum_tuning *tuning,
                            void *stream);
int lskum_plan_destroy(lskum_plan plan);
/* Replace the flow/scheme settings of an existing plan (same clouds);
 * params points to one struct per cloud. */
int lskum_plan_set_params(lskum_plan plan, const lskum_params *params);
int lskum_plan_set_tuning(lskum_plan plan, const lskum_tuning *tuning);
int32_t lskum_plan_n(lskum_plan plan);                       /* total points     */
int32_t lskum_plan_clouds(lskum_plan plan);                  /* number of clouds */
int32_t lskum_plan_offset(lskum_plan plan, int32_t cloud);   /* first point; cloud = n_clouds gives n */

/* Free stream with the wall tangency projection applied at wall points. */
int lskum_init_state(lskum_plan plan, double *U, void *stream);

/* eq. (13): q-variables from the conserved state at every point. */
int lskum_q_vars(lskum_plan plan, const double *U, double *q, void *stream);

/* Least-squares q-derivatives (eq. (9) with dq_i = q_i - q_0, then
 * params.n_inner Jacobi sweeps of eq. (14)-(15)) and the stencil bounds
 * qlim.  `work` is an [n][16] scratch buffer (64-byte aligned; unused when
 * n_inner is 0); the final iterate is in dq.  dq, qlim and work must not
 * share a byte with each other or with q (LSKUM_ERR_INVALID_ARG). */
int lskum_q_derivs(lskum_plan plan, const double *q, double *dq, double *qlim, double *work,
                   void *stream);

/* lskum_q_derivs without the `work` argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the inner sweeps' [n][16] scratch is a
 * static device array of the library (128 MiB, held on every GPU the
 * library runs on until the process ends), so the call allocates nothing.
 * dq and qlim equal those of lskum_q_derivs bit for bit.  Plans of more
 * than 1048576 points with n_inner > 0 get LSKUM_ERR_SCRATCH_LIMIT; other
 * errors as lskum_q_derivs, and LSKUM_ERR_HIP if the scratch's device
 * address could not be resolved when the plan was created.  Every call on
 * one GPU uses that GPU's one array: calls that overlap in time on one GPU
 * (other streams, other plans, other host threads) race and give wrong
 * results; calls ordered on one stream are safe. */
int lskum_q_derivs_static(lskum_plan plan, const double *q, double *dq, double *qlim,
                          void *stream);

/* Flux residual: the sum of the split-flux derivatives of eq. (10), each
 * from eq. (11) on its half-plane stencil of the point's (s, n) frame, with
 * differences of split fluxes of the limited modified q-variables of
 * eq. (14).  Interior points use G_s+-, G_n+-; wall points G_s+-, G_n-;
 * outer points get R = 0.  R must not share a byte with q, dq or qlim,
 * which other points read as neighbours (LSKUM_ERR_INVALID_ARG). */
int lskum_flux_residual(lskum_plan plan, const double *q, const double *dq, const double *qlim,
                        double *R, void *stream);

/* lskum_flux_residual, then, in the same launch, stage `stage` (0..3) of the
 * SSP Runge-Kutta (4,3) scheme on U (as lskum_rk_stage, from that residual)
 * and the q-variables of eq. (13) of the updated state into q_next (as
 * lskum_q_vars): the stage update and eq. (13) need only the point's own
 * values, so they run as the flux kernel's epilogue instead of two more
 * passes over memory.  R, U, q_next and Un equal those of the three
 * separate calls bit for bit.  Un, U, R and q_next are [n][4] (32-byte
 * aligned), dt is [n]; all device memory owned by the caller.  U holds the
 * previous stage on entry and the new one on return; q_next receives the q
 * of the next stage; Un as in lskum_rk_stage (stage 0 writes it).  The
 * written buffers R, U, q_next and Un must not share a byte with each
 * other or with q, dq, qlim (which other points still read as neighbours)
 * or dt (a point stores R before it reads its own U, Un and dt).  Non-physical new states set the status word as lskum_q_vars
 * does.  The stage is always SSP: the plan's LSKUM_RK4 bit is not read
 * here.  Returns LSKUM_ERR_INVALID_ARG for a null or misaligned pointer,
 * stage outside 0..3 or overlapping buffers as above. */
int lskum_flux_residual_stage(lskum_plan plan, int stage, const double *q, const double *dq,
                              const double *qlim, double *Un, const double *dt, double *R,
                              double *U, double *q_next, void *stream);

/* Local time step: dt_i = CFL * min_j |d_ij| / (|u_j| + 3 sqrt(p_j/rho_j)). */
int lskum_local_dt(lskum_plan plan, const double *U, double *dt, void *stream);

/* Stage `stage` (0..3) of the SSP Runge-Kutta (4,3) scheme with L = -R:
 * U <- a Un + b (U - dt/2 R), (a, b) = (0, 1) except stage 2: (2/3, 1/3);
 * then wall points drop normal momentum and outer points are reset to the
 * free stream.  U holds the previous stage on entry.  Un is the step's
 * starting state: stage 0, whose incoming U is that state, stores it in Un
 * for the later stages (so no copy is needed between steps).  U and Un
 * must not share a byte with each other, R or dt (LSKUM_ERR_INVALID_ARG). */
int lskum_rk_stage(lskum_plan plan, int stage, double *Un, const double *R,
                   const double *dt, double *U, void *stream);

/* Stage `stage` (0..3) of the classical fourth-order Runge-Kutta scheme
 * with L = -R and the same local time step: stages 0..2 write
 * U = Un - c dt R with c = 1/2, 1/2, 1 and the last writes
 * U = Un - dt/6 (R0 + 2 R1 + 2 R2 + R3), where R_s is the residual of stage
 * s's input.  acc ([n][4], caller-owned, 32-byte aligned) carries
 * R0 + 2 R1 + 2 R2 between the calls of one step: stage 0 overwrites it,
 * stages 1 and 2 update it, stage 3 only reads it.  Boundary conditions as
 * in lskum_rk_stage; Un as there (stage 0 stores its incoming U in it).  U,
 * Un and acc must not share a byte with each other, R or dt
 * (LSKUM_ERR_INVALID_ARG). */
int lskum_rk4_stage(lskum_plan plan, int stage, double *Un, const double *R,
                    const double *dt, double *acc, double *U, void *stream);

/* Deterministic L2 norm of the density residual over interior and wall
 * points, per cloud: out[c] (device, n_clouds doubles). */
int lskum_residual_norm(lskum_plan plan, const double *R, double *out, void *stream);

/* Lift and drag coefficients from each cloud's wall polygon (trapezoidal
 * pressure per edge, chord 1): clcd[2c], clcd[2c+1] (device). */
int lskum_force_coeffs(lskum_plan plan, const double *U, double *clcd, void *stream);

/* Bytes of device workspace lskum_iterate needs for this plan. */
size_t lskum_workspace_bytes(lskum_plan plan);

/* Advance U by `iters` iterations (each: local time step from U^n, then four
 * stages of q_vars -> q_derivs -> flux_residual -> rk_stage, the SSP stages
 * as lskum_flux_residual_stage).
 * hist[k*n_clouds + c] (device, may be NULL) receives the residual norm of
 * iteration k's first stage for cloud c.  `ws` is a device buffer of
 * lskum_workspace_bytes(plan) bytes, 256-byte aligned. */
int lskum_iterate(lskum_plan plan, int32_t iters, double *U, double *hist, void *ws,
                  void *stream);

/* Batched run: lskum_iterate over every cloud of a (batch) plan, with the
 * residual history cloud-major: hist[c*iters + k] (device, may be NULL) is
 * the residual norm of cloud c at iteration k's first stage.  U is the
 * concatenated state [n][4]; ws as for lskum_iterate.  Each cloud's history
 * and state equal those of the same cloud in a plan of its own.
 * LSKUM_ERR_INVALID_ARG also when hist overlaps U or ws. */
int lskum_batch_run(lskum_plan plan, int32_t iters, double *U, double *hist, void *ws,
                    void *stream);

/* Capture `iters` iterations of lskum_iterate on U into a HIP graph (one
 * launch replays them all).  Each replay appends the residual norms of its
 * iterations to hist as rows [row][n_clouds], row counted on the device
 * from 0 (reset here) up to hist_rows-1 (later rows are dropped); hist may
 * be NULL.  U, hist and ws stay bound to the graph.  One graph per plan at
 * a time: replays share the plan's row counter. */
int lskum_graph_create(lskum_graph *out, lskum_plan plan, int32_t iters, double *U, double *hist,
                       int32_t hist_rows, void *ws, void *stream);
int lskum_graph_launch(lskum_graph graph, void *stream);
int lskum_graph_destroy(lskum_graph graph);

/* Dirichlet rows: writes each cloud's free stream (from its current params)
 * at the outer points of U; other rows are left as they are. */
int lskum_set_far_field(lskum_plan plan, double *U, void *stream);

/* ---------------------------------------------------------------------
 * Adjoints (vector-Jacobian products), reverse mode through the formulas
 * of lskum_q_vars, lskum_q_derivs and lskum_flux_residual (eq. (9)-(15) and
 * the split fluxes of eq. (2)-(3)), differentiating the branch the forward
 * takes at each limiter, stencil max/min (the first slot attaining it, the
 * point itself first) and half-plane membership test.
 *
 * theta = (M, alpha [rad]) per cloud.  The residual is taken as a function
 * of the interior and wall rows of U and of theta, the outer rows being the
 * free stream U_inf(theta) of eq. (1) with rho = 1, p = 1/gamma.
 * ------------------------------------------------------------------- */

/* Bytes of device workspace lskum_flux_residual_vjp needs:
 * (49 + 8 n_inner) doubles per point (each field rounded up to 256 bytes)
 * for q, every derivative iterate, the bounds, the slots attaining them and
 * the cotangents.  Nothing is stored per edge: each edge's reverse is
 * recomputed where its cotangent is consumed. */
size_t lskum_vjp_workspace_bytes(lskum_plan plan);

/* Ubar = (dR/dU)^T Rbar at interior and wall rows, 0 at outer rows;
 * thetabar[2c], thetabar[2c+1] = the Mach and alpha cotangents of cloud c,
 * i.e. sum over its outer rows j of (dR/dU_j)^T Rbar . dU_inf/dtheta.
 * U, Rbar, Ubar: device [n][4] (Rbar is ignored at outer rows); thetabar:
 * device [n_clouds][2]; ws: device, lskum_vjp_workspace_bytes(plan) bytes,
 * 256-byte aligned.  q and the derivatives are recomputed from U.  The
 * first call on a plan also builds the plan's transposed connectivity and
 * its LDS tile tables (rebuilt when the tile size changes; synchronous;
 * LSKUM_ERR_INVALID_ARG beyond 2^25 - 1 points or 64 slots per row). */
int lskum_flux_residual_vjp(lskum_plan plan, const double *U, const double *Rbar, double *Ubar,
                            double *thetabar, void *ws, void *stream);

/* Cotangent of the force coefficients: with Jbar[2c], Jbar[2c+1] the
 * weights of (Cl, Cd) of cloud c (device), writes Ubar = d(Jbar . C)/dU
 * (device [n][4], non-zero at wall points only) and thetabar[2c..2c+1] =
 * d(Jbar . C)/d(M, alpha) at fixed U (device). */
int lskum_force_coeffs_vjp(lskum_plan plan, const double *U, const double *Jbar, double *Ubar,
                           double *thetabar, void *stream);

/* Steady adjoint.  At a steady state U of the projected system (outer rows
 * Dirichlet, wall rows with zero normal momentum), the total derivative of
 * an output J(U, theta) is dJ/dtheta = dJ/dtheta|_U - thetabar(Lambda),
 * where thetabar(Lambda) is the theta cotangent of lskum_flux_residual_vjp
 * with Rbar = Lambda and Lambda solves Pi (dR/dU)^T Lambda = Pi g,
 * g = (dJ/dU)^T, Pi clearing outer rows and the normal momentum of wall
 * rows.  lskum_adjoint_iterate runs `iters` pseudo-time steps
 *   Lambda <- Pi (Lambda - dt/2 ((dR/dU)^T Lambda - g)),
 * dt the local time step of U (lskum_local_dt); the iteration matrix is
 * similar to the transpose of the linearised forward iteration's, so it
 * converges where the forward does.  Lambda (device [n][4]) is read as the
 * initial iterate and overwritten; hist[k*n_clouds + c] (device, may be
 * NULL) receives the L2 norm over cloud c of Pi((dR/dU)^T Lambda - g)
 * before step k.  g: device [n][4].  ws: device,
 * lskum_adjoint_workspace_bytes(plan) bytes, 256-byte aligned.  q and the
 * derivative iterates of U are computed once per call. */
size_t lskum_adjoint_workspace_bytes(lskum_plan plan);
int lskum_adjoint_iterate(lskum_plan plan, const double *U, const double *g, double *Lambda,
                          int32_t iters, double *hist, void *ws, void *stream);

/* The total derivative of J = sum_c Jbar[2c] Cl_c + Jbar[2c+1] Cd_c with
 * respect to theta_c = (M, alpha [rad]) at the steady state U, from the
 * adjoint Lambda of lskum_adjoint_iterate:
 *   total[2c..2c+1] = dJ/dtheta_c|_U - thetabar_c(Lambda),
 * the first term the partial of lskum_force_coeffs_vjp, the second the theta
 * cotangent of lskum_flux_residual_vjp with Rbar = Lambda.  partial (may be
 * NULL) receives the first term.  U, Lambda: device [n][4]; Jbar, total,
 * partial: device [n_clouds][2]; ws: device, lskum_adjoint_workspace_bytes
 * bytes, 256-byte aligned.  LSKUM_ERR_INVALID_ARG for null or misaligned
 * pointers or when total or partial overlaps another argument. */
int lskum_adjoint_total(lskum_plan plan, const double *U, const double *Lambda,
                        const double *Jbar, double *total, double *partial, void *ws,
                        void *stream);

/* Synchronises `stream`, then returns LSKUM_ERR_NONPHYSICAL or
 * LSKUM_ERR_DEGENERATE if a kernel has recorded one since the last clear,
 * else LSKUM_OK (or LSKUM_ERR_HIP). */
int lskum_status(lskum_plan plan, void *stream);
int lskum_clear_status(lskum_plan plan, void *stream);

const char *lskum_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* LSKUM_H */
