/*
 * ocp_admm.h -- C ABI of the batched SQP-ADMM optimal-control QP solver for
 * AMD Instinct MI355X (gfx950).
 *
 * Problem class (Sec. "Contribution", box OCP; Appendix "Optimal Control
 * Problem"): stages t = 0..N with states x_t (nx), controls u_t (nu),
 *   min  sum_t l_t + slack penalty
 *   s.t. x_0 = x_init,  f_t(x_t,u_t,x_{t+1},u_{t+1}) = 0,  g_lo <= g_t + xi_t <= g_hi.
 * Each SQP step convexifies it into the stage-wise QP of Sec. "QP
 * Approximation of OCP" / Appendix "QP Approximation":
 *   min 1/2 x'Px + q'x + slack penalty   s.t.  Cx = c,  lo <= Gx + xi <= hi
 * with P block-tridiagonal (D_t, E_t), C block-bidiagonal (A_init = [I 0],
 * [A_t^- A_t^+]) and G block-diagonal (G_t).  The QP is solved by the ADMM
 * scheme of Algorithm 3 with a block-tridiagonal Cholesky of the Schur
 * matrix S = P + sigma I + C'rho_f C + G'rho_g G (Appendix "ADMM"), and
 * differentiated by the active-set implicit VJP of Algorithm 2.
 *
 * Conventions
 *  - Stage-concatenated batches: instance b owns stages stage_off[b] ..
 *    stage_off[b+1]-1 (N_b + 1 of them); S = total stage count.  Horizons
 *    may differ per instance (ragged batches).
 *  - Every array argument is a DEVICE pointer owned by the caller, in
 *    row-major order, FP64 unless stated otherwise.  Settings structs are
 *    host memory.  The library owns only its workspace, allocated by
 *    ocp_create and freed by ocp_destroy; ocp_set_* / ocp_solve /
 *    ocp_adjoint allocate nothing.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *    asynchronous on that stream; one handle must not be used from two
 *    streams at once.
 *  - Errors are reported only through the return code (nothing aborts or
 *    throws).  Numerical trouble of one instance is reported per instance in
 *    ocp_solution.status, never as a call failure.
 */
#ifndef OCP_ADMM_H
#define OCP_ADMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ocp_handle_s* ocp_handle;

typedef enum {
  OCP_OK = 0,
  OCP_E_ARG = 1,         /* null pointer / invalid value */
  OCP_E_SHAPE = 2,       /* sizes inconsistent or not compiled in (see ocp_supported) */
  OCP_E_HIP = 3,         /* a HIP runtime call failed */
  OCP_E_NOMEM = 4,       /* workspace allocation failed */
  OCP_E_ORDER = 5,       /* call order violated (e.g. solve before set, adjoint before solve) */
  OCP_E_UNSUPPORTED = 6, /* feature not available for this model / row kind */
  OCP_E_SCRATCH = 7      /* problem larger than the no-allocation scratch (ocp_solve_noalloc) */
} ocp_status;

/* models */
enum { OCP_MODEL_QP = 0, OCP_MODEL_LTI = 1, OCP_MODEL_BICYCLE = 2 };
/* arithmetic of the ADMM iterations; the factorisation is always FP64 */
enum { OCP_PREC_FP64 = 0, OCP_PREC_MIXED = 1 };
/* inequality-row kinds: hard, L2-penalised slack (Sec. "Slack update"),
 * L1-penalised slack */
enum { OCP_ROW_HARD = 0, OCP_ROW_L2 = 1, OCP_ROW_L1 = 2 };
/* bicycle discretisation (zero-order hold on u): implicit midpoint
 * x_t + dt fc((x_t + x_{t+1})/2, u_t) - x_{t+1}, or the trapezoidal rule of
 * Remark A1, x_t + dt/2 (fc(x_t, u_t) + fc(x_{t+1}, u_t)) - x_{t+1} */
enum { OCP_INTEG_MIDPOINT = 0, OCP_INTEG_TRAPEZOID = 1 };
/* per-instance status; OCP_INFEASIBLE: at a convergence check the change of
 * the multipliers since the previous check certifies that {Cx = c, lo <= Gx
 * <= hi} is empty (Farkas: ||A'dy||_inf <= eps_pinf ||dy||_inf and
 * c'dy_f + hi'max(dy_g,0) + lo'min(dy_g,0) < -eps_pinf ||dy||_inf, the ADMM
 * infeasibility test of Banjac, Goulart, Stellato and Boyd), evaluated in
 * the original variables; problems with soft rows are never declared
 * infeasible */
enum { OCP_SOLVED = 0, OCP_MAX_ITER = 1, OCP_NON_FINITE = 2, OCP_FACTOR_BREAKDOWN = 3, OCP_INFEASIBLE = 4 };
/* per-instance adjoint status (ocp_qp_grads.adj_status): the relative FP64
 * residual ||r - K eta||_inf / ||dL/dx||_inf of the active-set KKT system after
 * the refinement sweeps is at most adj_tol (OK) or above it (RESIDUAL: the
 * sweeps did not converge, e.g. nearly dependent active rows), the result is
 * not finite, or the factorisation of the regularised Schur matrix broke down */
enum { OCP_ADJ_OK = 0, OCP_ADJ_RESIDUAL = 1, OCP_ADJ_NON_FINITE = 2, OCP_ADJ_BREAKDOWN = 3 };

typedef struct {
  int32_t batch;          /* B >= 1 */
  int32_t nx, nu, ng;     /* state, control and inequality-row counts per stage */
  int32_t model;          /* OCP_MODEL_* */
  int32_t precision;      /* OCP_PREC_* */
  int32_t time_invariant; /* OCP_MODEL_QP only: blocks given once per instance (see ocp_qp) */
} ocp_dims;

/* Solver settings (host struct).  Defaults (ocp_default_settings) are the
 * paper's: sigma = 1e-6, rho_bar_0 = 0.1, rho_f = 1e3 rho_bar, rho_g = rho_bar,
 * rho_bar in [1e-6, 1e6], adaptation every 25 iterations when the change
 * exceeds 5x (Sec. "Solving QP via ADMM", step-size selection), Armijo
 * eta = 0.4 (Appendix "Line search"), at most 1000 ADMM iterations. */
typedef struct {
  double sigma, rho0, rho_f_scale, rho_min, rho_max, k_ratio;
  double alpha;            /* over-relaxation in (0,2); default 1.6 */
  double eps_abs, eps_rel; /* ADMM stopping test, evaluated in FP64 */
  double eps_c;            /* SQP stopping tolerance (eq. sqp_stop) */
  double armijo_eta;
  double eps_active;       /* active-set tolerance scale for the adjoint */
  double adj_sigma, adj_rho; /* regularisation of the adjoint refinement */
  double adj_tol;          /* relative KKT residual after the sweeps accepted as refined
                              (adj_status OK); default 1e-10 */
  double eps_pinf;         /* infeasibility-certificate tolerance (OCP_INFEASIBLE); 0 = no test;
                              default 1e-4 */
  int32_t max_admm;        /* ADMM iterations per QP */
  int32_t k_rho;           /* rho adaptation interval (0 = never) */
  int32_t k_check;         /* convergence test interval (0 = run exactly max_admm) */
  int32_t adapt_rho;       /* 0/1 */
  int32_t warm_start;      /* 1: start from the handle's current state and rho */
  int32_t max_sqp;         /* SQP iterations (bicycle model) */
  int32_t fixed_sqp;       /* 1: run exactly max_sqp iterations */
  int32_t refine_sweeps;   /* adjoint iterative-refinement sweeps, at most (default 8; an instance
                              stops earlier once its relative residual is below adj_tol / 100) */
  int32_t adj_mode;        /* bicycle model: what ocp_adjoint differentiates (OCP_ADJ_LAST_QP,
                              OCP_ADJ_SQP_GN, OCP_ADJ_SQP_EXACT); ignored for linear models */
} ocp_settings;

/* ocp_settings.adj_mode.  LAST_QP: the last SQP iteration's QP at its own
 * ADMM solution.  SQP_GN / SQP_EXACT: the SQP solution itself -- the KKT
 * conditions of the OCP at the handle's SQP iterate (the last solve's, or one
 * restored by ocp_set_iterate), i.e. the QP convexified there with the Hessian
 * of the cost alone (Gauss-Newton, the paper's approximate second-order
 * option) or of the Lagrangian, grad^2 l + sum_t y_f,t' grad^2 f_t (exact; the
 * dynamics curvature fills D_t and the cross-stage blocks E_t). */
enum { OCP_ADJ_LAST_QP = 0, OCP_ADJ_SQP_GN = 1, OCP_ADJ_SQP_EXACT = 2 };

/* Linear time-invariant model (OCP_MODEL_LTI): x_{t+1} = A x_t + B u_t,
 * cost 1/2(x'Qx + u'Ru) for t < N and 1/2(x'Q_f x + u'Ru) at t = N, bounds
 * lo <= G (x_t,u_t) <= hi at every stage.  Shapes:
 * A [B,nx,nx], Bm [B,nx,nu], Qd [B,nx], Rd [B,nu], Qfd [B,nx] (diagonals),
 * G [ng, nx+nu] (shared by all instances and stages), lo, hi [B,ng], x0 [B,nx]. */
typedef struct {
  const double *A, *Bm, *Qd, *Rd, *Qfd, *G, *lo, *hi, *x0;
} ocp_lti;

/* General stage-wise QP (OCP_MODEL_QP).  n = nx + nu.
 * time_invariant = 0: D [S,n,n], E [S,n,n] (E_t = block (t+1,t); slot N of
 *   each instance unused), q [S,n], Am, Ap [S,nx,n], b [S,nx] (slot N
 *   unused), G [S,ng,n], lo, hi [S,ng].
 * time_invariant = 1: D [2B,n,n] (interior, terminal), E [B,n,n],
 *   Am, Ap [B,nx,n], b [B,nx], G [B,ng,n], lo, hi [B,ng]; q stays [S,n].
 * E, q and b may be NULL (zero).  x_init [B,nx].  soft [ng] (uint8 row
 * kinds, DEVICE pointer) may be NULL (all rows hard).
 * gamma2: L2 slack weight (gamma/2 ||xi||^2); gamma1: L1 slack weight. */
typedef struct {
  const double *D, *E, *q, *Am, *Ap, *b, *G, *lo, *hi, *x_init;
  const uint8_t* soft;
  double gamma2, gamma1;
} ocp_qp;

/* Kinematic bicycle (OCP_MODEL_BICYCLE, nx = 4, nu = 2, ng = 3): state
 * (px, py, yaw, v), control (a, delta); implicit-midpoint dynamics
 * x_{t+1} = x_t + dt fc((x_t + x_{t+1})/2, u_t); tracking cost
 * 1/2 (x_t - r_t)'Q(x_t - r_t) + 1/2 u_t'R u_t (Q_f at t = N); rows
 * a in [-a_bound, a_bound], delta in [-steer_bound, steer_bound] (hard) and
 * the lateral offset n_t'(p_t - p_ref,t) in [-lat_bound, lat_bound] (L1 slack,
 * weight gamma1).  ref [S,4], normal [S,2], x0 [B,4] device; scalars host.
 * Racing features (Sec. "Hardware Deployment: Autonomous Racing"): the
 * control-rate cost of eq. cost, 1/2 (u_t - u_{t+1})'diag(Wd)(u_t - u_{t+1})
 * for t < N (Wd = 0: none; it couples neighbouring stages through E_t), and
 * the fixed first control (x_0, u_0) = (x_init, u_init): u_init [B,2]
 * (device, may be NULL: u_0 free) makes the two control rows of stage 0
 * equalities, and the SQP starts from u_0 = u_init. */
typedef struct {
  const double *ref, *normal, *x0;
  double dt, wheelbase, a_bound, steer_bound, lat_bound, gamma1;
  double Qd[4], Rd[2], Qfd[4];
  int32_t integrator; /* OCP_INTEG_MIDPOINT or OCP_INTEG_TRAPEZOID */
  double Wd[2];
  const double* u_init;
} ocp_bicycle;

/* Solution buffers (device, FP64, caller-owned).  Any pointer may be NULL
 * to skip that output.  x [S,n]; xi, z_g, y_g [S,ng]; y_f [S,nx] where the
 * slot of stage 0 holds the initial-state multipliers and the slot of stage
 * t+1 the multipliers of dynamics row t; per instance [B]: status,
 * admm_iters (last QP), sqp_iters, n_factor, r_prim, r_dual (FP64
 * residuals of eq. admm:residuals), rho (final rho_bar); sqp_kkt [B,3] =
 * (stationarity, equality, inequality) of eq. sqp_stop (bicycle only). */
typedef struct {
  double *x, *xi, *z_g, *y_f, *y_g;
  int32_t *status, *admm_iters, *sqp_iters, *n_factor;
  double *r_prim, *r_dual, *rho, *sqp_kkt;
} ocp_solution;

/* Gradients of a loss w.r.t. the QP data at the last solution (device, FP64,
 * caller-owned, NULL to skip): d_q [S,n], d_Ddiag [S,n] (diagonal of D_t),
 * d_x_init [B,nx], d_lo, d_hi [S,ng], eta_x [S,n], active [S,ng] (int8:
 * -1 lower, +1 upper, 0 inactive), d_gamma2 [B] (w.r.t. the L2 slack
 * weight: sum over the active L2-slack rows of xi_i (G eta_x)_i, Sec.
 * "Backward pass" with slack variables; 0 without such rows);
 * eta_f [S,nx] (adjoint of the equality multipliers, in the slot convention
 * of ocp_solution.y_f: dL/dc = eta_f) and eta_g [S,ng] (of the inequality
 * multipliers, 0 on inactive rows); per instance [B]: adj_resid (relative
 * FP64 KKT residual after the sweeps) and adj_status (OCP_ADJ_*).  When the
 * active rows are linearly dependent the multiplier part is the one the
 * refinement reaches from zero, the minimum-norm solution. */
typedef struct {
  double *d_q, *d_Ddiag, *d_x_init, *d_lo, *d_hi, *eta_x;
  int8_t* active;
  double* d_gamma2;
  double *eta_f, *eta_g, *adj_resid;
  int32_t* adj_status;
  double *eta_xi, *d_gamma1; /* [S,ng], [B]: see ocp_adjoint */
} ocp_qp_grads;

/* Fill `s` with the defaults listed above.  Never fails. */
void ocp_default_settings(ocp_settings* s);

/* Static string for a status code. */
const char* ocp_status_string(ocp_status st);

/* 1 if kernels are compiled for (nx, nu, ng), else 0. */
int32_t ocp_supported(int32_t nx, int32_t nu, int32_t ng);

/* Workspace bytes ocp_create would allocate for these dims and horizons
 * (horizons: HOST array of B horizons N_b >= 1). */
ocp_status ocp_workspace_bytes(const ocp_dims* dims, const int32_t* horizons, size_t* bytes);

/* Allocate a solver for `dims` and the B horizons (HOST array).  On success
 * *out receives the handle.  Errors: OCP_E_ARG, OCP_E_SHAPE, OCP_E_NOMEM,
 * OCP_E_HIP. */
ocp_status ocp_create(const ocp_dims* dims, const int32_t* horizons, ocp_handle* out);

/* Free the workspace; NULL is accepted. */
ocp_status ocp_destroy(ocp_handle h);

/* Load problem data (copied into the workspace on `stream`; the caller may
 * free its buffers once the stream has passed this call).  The setter must
 * match dims.model. */
ocp_status ocp_set_lti(ocp_handle h, const ocp_lti* p, void* stream);
ocp_status ocp_set_qp(ocp_handle h, const ocp_qp* p, void* stream);
ocp_status ocp_set_bicycle(ocp_handle h, const ocp_bicycle* p, void* stream);

/* Solve all instances.  LTI / QP models: one ADMM solve (Algorithm 3).
 * Bicycle: max_sqp SQP iterations (Algorithm 1), each linearising at the
 * current iterate, solving the QP by ADMM warm-started from it and taking
 * the line-search step (Appendix "Line search").  Writes `out` (may be
 * NULL to keep the state only in the workspace). */
ocp_status ocp_solve(ocp_handle h, const ocp_settings* s, const ocp_solution* out, void* stream);

/* Copy the handle's current solution (last ocp_solve) into `out` without
 * solving again.  Errors: OCP_E_ORDER before a solve. */
ocp_status ocp_get_solution(ocp_handle h, const ocp_solution* out, void* stream);

/* Implicit-differentiation VJP at the last solution (Algorithm 2, eq.
 * bwd:noslack_kkt_matrix / loss_gradient): identify the active set, factor
 * the regularised active-set Schur matrix in FP64, refine against the exact
 * KKT system and map eta to QP-data gradients.  dL_dx [S,n] device; dL_dxi
 * [S,ng] device, the loss gradient w.r.t. the slacks, may be NULL (zero).
 * Slack rows (eq. bwd:slack_adjoint): active L2-slack rows follow the reduced
 * system of eq. bwd:slack_reduced_system -- their penalty gamma2 G_i'G_i
 * joins H, the right-hand side gets -G_i' dL/dxi_i, their eta_y = dL/dxi_i +
 * gamma2 G_i eta_x and eta_xi = -G_i eta_x (eq. bwd:slack:eta_xi_yg); L1 rows
 * with a nonzero slack carry the fixed multiplier -gamma1 sign(xi) and leave
 * the active set, their slack xi = bound - G_i x contributes -G_i' dL/dxi_i
 * to the right-hand side and dL/dxi_i to that bound (d_lo when xi > 0, d_hi
 * when xi < 0), eta_xi = -G_i eta_x, and d_gamma1 [B] = sum over them of
 * sign(xi_i) (G eta_x)_i; eta_xi is 0 on the other rows.
 * Bicycle model: the VJP is that of the last SQP iteration's QP at that QP's
 * own ADMM solution (x, y_g, xi before the line-search step), which is the
 * returned iterate once the SQP has converged with unit steps; d_Ddiag uses
 * that QP solution.  Per-instance adj_status / adj_resid report whether the
 * refinement reached settings.adj_tol.  Errors: OCP_E_ORDER before a solve,
 * OCP_E_ARG (null pointers, non-positive adj_sigma / adj_rho / eps_active /
 * adj_tol, refine_sweeps < 1). */
ocp_status ocp_adjoint(ocp_handle h, const ocp_settings* s, const double* dL_dx, const double* dL_dxi,
                       const ocp_qp_grads* out, void* stream);

/* Checkpoint restore for the SQP layer (bicycle model): load an SQP iterate
 * -- x [S,n], xi [S,ng], y_f [S,nx] (slot convention of ocp_solution.y_f), y_g
 * [S,ng], DEVICE, FP64, as ocp_solve returned it -- into the handle, so that
 * ocp_adjoint with adj_mode SQP_GN / SQP_EXACT differentiates at it even after
 * the handle solved other problems (the problem data must be those of that
 * solve: call ocp_set_bicycle again first if they changed).  Only the iterate
 * is kept between a forward and its backward; the factorisation is redone
 * there.  Errors: OCP_E_ARG (null pointers), OCP_E_UNSUPPORTED (other
 * models), OCP_E_ORDER (no problem data). */
ocp_status ocp_set_iterate(ocp_handle h, const double* x, const double* xi, const double* y_f, const double* y_g,
                           void* stream);

/* Kernel timing (observability).  Classes of the library's launches: */
enum {
  OCP_K_FACTOR = 0,  /* block-tridiagonal Cholesky (Appendix "ADMM", Schur complement) */
  OCP_K_ITER = 1,    /* ADMM iterations between stopping tests (Algorithm 3) */
  OCP_K_CHECK = 2,   /* FP64 residuals, stopping test, rho candidate (eq. admm:residuals, rho:update) */
  OCP_K_ADJOINT = 3, /* implicit-differentiation VJP (Algorithm 2) */
  OCP_K_SQP = 4,     /* bicycle linearisation and line search (Algorithm 1) */
  OCP_K_OTHER = 5,   /* per-solve initialisation */
  OCP_K_SOLVE = 6,   /* persistent ADMM solve: factorisation, iterations, checks and rho
                        adaptation of every instance in one launch (Algorithm 3) */
  OCP_K_COUNT = 7
};
/* Accumulated GPU time (HIP events on the caller's stream, bracketing each
 * launch) and launch counts per class since the last read. */
typedef struct {
  double ms[OCP_K_COUNT];
  int64_t launches[OCP_K_COUNT];
} ocp_kernel_times;

/* Turn timing on (enable != 0) or off for later calls on this handle.  While
 * on, every launch of ocp_solve / ocp_adjoint records one event pair (events
 * are created on first use and kept until ocp_destroy).  Errors: OCP_E_ARG. */
ocp_status ocp_profile(ocp_handle h, int32_t enable);

/* Wait for the recorded events, return the per-class totals in `out` (HOST
 * struct) and reset them.  Errors: OCP_E_ARG, OCP_E_HIP. */
ocp_status ocp_profile_read(ocp_handle h, ocp_kernel_times* out);

/* Graph capture of a whole step (batching and scheduling: the launch sequence
 * of one solve, and optionally the adjoint after it, recorded once and
 * replayed without per-launch host work).  Records, on `stream` (not NULL),
 * exactly the launches ocp_solve(h, s, out, stream) and -- when dL_dx and
 * grads are both given -- ocp_adjoint(h, s, dL_dx, dL_dxi, grads, stream) would issue
 * now, into a HIP graph owned by the handle (replacing any earlier one).
 * Nothing runs during capture.  The graph keeps the given device pointers:
 * the caller keeps `out`, `dL_dx` and the `grads` buffers alive and in place
 * while it replays.  Host-side decisions are frozen at capture time (for the
 * bicycle model: a cold SQP start unless warm_start was set and a solve had
 * run).  Kernel timing is suspended while capturing.  Errors: OCP_E_ARG
 * (null handle / settings / stream, dL_dx without grads or vice versa),
 * OCP_E_ORDER (no problem data), OCP_E_HIP. */
ocp_status ocp_graph_capture(ocp_handle h, const ocp_settings* s, const ocp_solution* out, const double* dL_dx,
                             const double* dL_dxi, const ocp_qp_grads* grads, void* stream);

/* Replay the captured graph on `stream`.  Errors: OCP_E_ARG, OCP_E_ORDER
 * (nothing captured), OCP_E_HIP. */
ocp_status ocp_graph_launch(ocp_handle h, void* stream);

/* Launch shape (batching and scheduling).  The substitutions of S x = eta
 * (Sec. "Primal update") run as one serial chain over the horizon
 * (interleaved iteration) for short horizons and, for horizons
 * N >= seg_min_n, segmented: the horizon is cut into four segments whose
 * chains run side by side from a zero start and are joined through the
 * segments' transfer blocks, formed after each factorisation.  The same
 * switch selects the chunked block Cholesky (Appendix "ADMM", Schur
 * complement) for the solve's and the adjoint's factorisations: five chunks,
 * three of them first reduced to their map from the entering Schur state
 * (Woodbury identity), so that every chunk is factored from its true entering
 * state in two passes whose serial depth is two fifths of the horizon.  Both
 * launch shapes solve the same system with the same blocks; results agree up
 * to rounding.  The default switch is N >= 128.
 *
 * ocp_set_segmented: set the switch for later solves on this handle (values
 * below 15 are raised to 15: segments of at least four stages; INT32_MAX
 * keeps every instance interleaved).  Drops a captured graph.  Errors:
 * OCP_E_ARG (null handle). */
ocp_status ocp_set_segmented(ocp_handle h, int32_t seg_min_n);

/* Multi-wavefront instances (Sec. "Scalability to longer planning
 * horizons"): an instance with horizon N >= mw_min_n is solved by one
 * workgroup of W wavefronts (W = 8 for stage width n <= 8, else 4) instead
 * of one wavefront.  Its chunked factorisation runs 4 W + 1 chunks and its
 * segmented substitutions 4 W segments, one per 16-lane row of the
 * workgroup, so their serial depth is about 2 / (4 W) of the horizon; the
 * FP64 convergence checks spread the stages over the same rows, and
 * wavefront 0 keeps the schedule (stopping and rho decisions) described at
 * ocp_solve.  Results agree with the one-wavefront shapes up to
 * rounding.  Default 255 (horizons of 256 stages and more); 0 turns it off.
 * Drops a captured graph.  Errors: OCP_E_ARG (null handle, or 0 < mw_min_n
 * < 16 W - 1: segments of fewer than four stages), OCP_E_HIP. */
ocp_status ocp_set_multiwave(ocp_handle h, int32_t mw_min_n);

/* Primal-update solver of the ADMM iterations (the PCG backends of the
 * paper's table of QP solver backends, the hybrid of its discussion section:
 * PCG forward, direct backward).  OCP_LINSOLVE_DIRECT (default): the
 * block-tridiagonal Cholesky of S and its two substitution chains.
 * OCP_LINSOLVE_PCG: S x~ = eta (eq. admm:schur) by block-Jacobi
 * preconditioned conjugate gradients from the current primal iterate x,
 * stopping before an iteration when ||r||_2 <= tol ||eta||_2 or after
 * max_iter iterations; the "factorisation" after a rho change forms the
 * diagonal blocks of S, their inverses and the coupling blocks instead (no
 * recursion), and every pass is stage-parallel (one wavefront per instance;
 * no segmented, chunked or multi-wavefront shapes).  Inexact solves slow
 * ADMM's convergence; the stopping test is unchanged.  The adjoint always
 * uses the direct solver.  The first switch to PCG allocates five stage
 * vectors (and, for FP64 iterations, one block per stage) on the handle.
 * Drops a captured graph.  Errors: OCP_E_ARG (null handle, unknown mode,
 * max_iter < 1, tol negative or not finite), OCP_E_NOMEM, OCP_E_HIP. */
enum { OCP_LINSOLVE_DIRECT = 0, OCP_LINSOLVE_PCG = 1 };
ocp_status ocp_set_linsolve(ocp_handle h, int32_t mode, int32_t max_iter, double tol);

/* Problem rescaling (Remark 4: states and controls normalised inside the
 * solver, transparently to the caller).  Per instance b: variable factors
 * d [B,n] (x_t = d * xh_t at every stage), inequality-row factors e_g [B,ng]
 * and a cost factor c [B] (DEVICE pointers, FP64, all > 0 and finite).  The
 * next ocp_set_lti / ocp_set_qp loads the rescaled QP
 *   D_t, E_t -> c diag(d) D_t diag(d), c diag(d) E_t diag(d);  q_t -> c d * q_t;
 *   Am_t, Ap_t -> diag(1/d_x) Am_t diag(d), diag(1/d_x) Ap_t diag(d);
 *   b_t -> b_t / d_x;  x_init -> x_init / d_x;
 *   G_t -> diag(e_g) G_t diag(d);  lo, hi -> e_g * lo, e_g * hi
 * (A_init = [I 0], A+ = [-I 0] and unit selection rows keep their form when
 * e_g = 1/d_j on a row selecting variable j; power-of-two factors make the
 * transform exact).  ADMM (Algorithm 3) iterates on it and adapts the step
 * size (eq. rho:update) from its residuals; the stopping test, the reported
 * residuals, the returned solution (x = d xh, z_g = zh/e_g, xi = xih/e_g,
 * y_f = yh_f/(c d_x), y_g = e_g yh_g/c) and the adjoint's inputs and outputs
 * are in the original variables.  d = NULL removes the rescaling.  Either way
 * the loaded data and solution are invalidated (call ocp_set_* again) and a
 * captured graph is dropped.  Models OCP_MODEL_LTI and OCP_MODEL_QP with hard
 * rows only.  Synchronises `stream` (to check the factors).  Errors:
 * OCP_E_ARG (null handle, missing e_g / c, a factor not positive and finite),
 * OCP_E_UNSUPPORTED (bicycle model; ocp_set_qp returns it for soft rows),
 * OCP_E_HIP. */
ocp_status ocp_set_scaling(ocp_handle h, const double* d, const double* e_g, const double* c, void* stream);

/* Box normalisation (Remark 4) derived on the device from every problem
 * loaded afterwards, per instance, in powers of two (the transform is exact):
 * a variable j bounded by a hard selection row of G (read at stage 0) gets
 * d_j = 2^rint(p log2 h_j), h_j the half width of its bounds, others 1;
 * e_g = 1/d_j on selection rows, 2^-rint(log2 max_j |G_rj d_j|) on other hard
 * rows; c = 2^-rint(log2 m), m the largest diagonal entry of diag(d) D_t
 * diag(d) over the instance's stages.  Then as ocp_set_scaling.  p = 0.6 is
 * the default the benchmark uses (FP32 iterations converge on the random-LTI
 * workload as often as unscaled FP64 ones).  ocp_set_scaling(h, NULL, ...)
 * removes it.  Errors: OCP_E_ARG (null handle, p negative or not finite),
 * OCP_E_UNSUPPORTED (bicycle model). */
ocp_status ocp_set_scaling_box(ocp_handle h, double p);

/* Launch shape of a batch's tail: from ADMM iteration `iteration` on, every
 * instance still running (N >= 15) takes the segmented substitutions
 * described at ocp_set_segmented, whatever its horizon.  While the batch is
 * full the interleaved sweeps read each chain block once, which is what the
 * memory system favours; once few instances remain, each is bound by the
 * serial depth of its chains, which the segments shorten.  INT32_MAX (the
 * default) keeps the switch off.  Drops a captured graph.  Errors: OCP_E_ARG
 * (null handle, negative iteration). */
ocp_status ocp_set_segmented_after(ocp_handle h, int32_t iteration);

/* Continuation of a batch's tail on two-wavefront workgroups (Sec.
 * "Scalability to longer planning horizons"; FP32 iterations): from ADMM
 * iteration `iteration` on, every instance solved on one wavefront that is
 * still running (horizon N >= 31, direct primal updates) continues on a
 * workgroup of two wavefronts.  The one-wavefront launch stops such an
 * instance at that iteration with its iterate, rho, factorisation count and
 * check state in device memory; a second launch on the same stream resumes
 * it with 8 substitution segments (4 per wavefront) and, after a later rho
 * change, the 9-chunk factorisation described at ocp_set_multiwave.  The
 * schedule of checks and rho decisions is the same, so results agree with
 * the one-wavefront solve up to rounding.  While the batch is full, one
 * wavefront per instance keeps the memory system busiest; once few instances
 * remain, each is bound by its own instruction stream, which two wavefronts
 * split.  0 (the default) turns it off.  Drops a captured graph.  Errors:
 * OCP_E_ARG (null handle, negative iteration), OCP_E_UNSUPPORTED (iteration
 * > 0 on an FP64 handle), OCP_E_NOMEM (the continuation's buffers, allocated
 * when first enabled: 8 B + 30 n^2 * 8 B per instance, plus 4 bytes),
 * OCP_E_HIP. */
ocp_status ocp_set_tail_workgroup(ocp_handle h, int32_t iteration);

/* Autotuner over the launch shape: times `reps` cold-start ocp_solve calls
 * with settings `s` on the handle's own batch for each candidate triple
 * (segmented from horizon, every running instance segmented from iteration,
 * continuation on two-wavefront workgroups from iteration): (15, never, 0),
 * (128, never, 0), (never, never, 0), (128, 150, 0), (128, 300, 0),
 * (128, 500, 0), and with FP32 iterations also (128, never, 200),
 * (128, never, 300), (128, 150, 200) -- see ocp_set_segmented,
 * ocp_set_segmented_after and ocp_set_tail_workgroup -- on `stream` (one
 * warm-up solve each; synchronises the stream), keeps the fastest for later
 * solves and returns it in *seg_min_n, *seg_after and *tail_after (HOST
 * int32; any may be NULL; never = INT32_MAX, 0 = no continuation).  The
 * solution state afterwards is that of the last timed solve: solve again
 * before reading results.  Kernel timing is suspended while it runs.
 * Errors: OCP_E_ARG (null handle / settings, reps < 1, invalid settings),
 * OCP_E_ORDER (no problem data), OCP_E_NOMEM (the continuation's buffers),
 * OCP_E_HIP. */
ocp_status ocp_autotune(ocp_handle h, const ocp_settings* s, int32_t reps, void* stream, int32_t* seg_min_n,
                        int32_t* seg_after, int32_t* tail_after);

/* Bytes of device memory the library holds on every GPU it runs on, for the
 * life of the process, as the workspace of ocp_solve_noalloc. */
#define OCP_NOALLOC_SCRATCH_BYTES (64u << 20)

/* One solve that allocates nothing, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same work as ocp_create + ocp_set_lti / ocp_set_qp /
 * ocp_set_bicycle + ocp_solve (cold start) on `stream`, with the workspace
 * taken from a file-scope device array of OCP_NOALLOC_SCRATCH_BYTES instead of
 * allocated.  `problem` points to the ocp_lti, ocp_qp or ocp_bicycle struct
 * that dims->model selects; horizons is a HOST array of B horizons; the
 * caller owns `problem`'s and `out`'s device buffers as for ocp_solve.
 * Every call on a GPU shares that GPU's scratch and overwrites what the
 * previous call left there: calls that overlap on one GPU (different
 * streams or threads) race, and nothing of a call survives the next one (no
 * ocp_get_solution / ocp_adjoint afterwards; use a handle for those).  The
 * call synchronises `stream` once (after laying out the stages).  Every
 * instance runs on one wavefront and the bicycle line search in one pass per
 * instance, so for horizons from 255 stages on (which a handle gives a
 * multi-wavefront workgroup) and past 511 (whose line search a handle splits
 * into chunks) results agree with the handle path's up to rounding; below
 * both, bit for bit.  Errors:
 * those of ocp_create / ocp_set_* / ocp_solve, and OCP_E_SCRATCH when the
 * workspace ocp_workspace_bytes reports plus the horizons exceeds
 * OCP_NOALLOC_SCRATCH_BYTES. */
ocp_status ocp_solve_noalloc(const ocp_dims* dims, const int32_t* horizons, const void* problem,
                             const ocp_settings* s, const ocp_solution* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* OCP_ADMM_H */
