/*
 * gpf.h — C ABI of the MI355X (gfx950) grid potential-flow library.
 *
 * Method: Beckers & Eldredge, "Planar potential flow on Cartesian grids"
 * (arXiv 2102.11910).  One solve computes, on an unbounded Cartesian grid,
 *
 *   w  = R_v Gamma                         regularization of point vortices
 *                                          with the M4' kernel (Sec. 2.1,
 *                                          eq. vortexregularization)
 *   s* = -L^-1 w                           lattice Green's function
 *                                          convolution (Sec. 2.1, eq. poisson)
 *   f, s0, Gamma_j                         bound vortex sheet and constraint
 *                                          forces from the Schur complement
 *                                          S = -E_s L^-1 R_s (Sec. 2.2-2.4,
 *                                          eqs. basicblock, circsystem,
 *                                          kuttasystem, kuttasystem2/3)
 *   s  = -L^-1 (w + R_s f + sum Gamma_j d_j)   final streamfunction
 *   (u, v) at the vortices                 centred differences of s averaged
 *                                          to nodes, then E_v = R_v^T (Sec. 2.1)
 *
 * Conventions
 *   Grid: n x n nodes, node (i, j) at (x0 + i dx, y0 + j dx); fields are
 *   row-major [j][i] (i fastest).  n must be a power of two, 16 <= n <= 2048.
 *   The lattice Green's function G has the gauge G(0,0) = 0.
 *   s is the streamfunction WITHOUT the uniform-flow part
 *   s_inf = U_inf y - V_inf x, unless the plan has GPF_PSI_TOTAL.
 *   Every vortex stencil (plus one node for velocities) and every surface
 *   stencil must lie inside the window: (x - x0)/dx in [2, n-3) for vortices
 *   and new vortices, in [1, n-2) for surface points.
 *
 * Memory and ownership
 *   d_* = device pointer (HIP), h_* = host pointer.  The caller owns every
 *   input/output buffer; the library never frees them and keeps no pointer
 *   to them after a call returns.  The library owns its handles and their
 *   device workspaces.  Destroy bodies before their plan, plans before the
 *   context.
 *
 * Asynchrony
 *   Solves enqueue all device work on the caller's HIP stream and return;
 *   buffers must stay valid until that stream has completed.  A plan's
 *   workspace serves one stream at a time: concurrent solves on one plan
 *   race, unless the plan has GPF_PLAN_MULTISTREAM.
 *
 * Errors
 *   Every call returns a gpf_status.  Synchronous errors (bad arguments,
 *   unsupported sizes, allocation failure, singular body) return at once and
 *   set a thread-local message readable with gpf_last_error().
 *   Data-dependent errors found on the device (a stencil leaving the window,
 *   a singular m x m edge system) are OR-ed into the caller's device status
 *   word as GPF_DEV_* bits; gpf_sync() turns them into a gpf_status.
 */
#ifndef GPF_H
#define GPF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GPF_OK = 0,
  GPF_E_INVALID = -1,      /* null/ill-formed argument, non-finite scalar      */
  GPF_E_OUT_OF_GRID = -2,  /* a stencil leaves the grid window                 */
  GPF_E_SINGULAR = -3,     /* singular Schur complement or edge system         */
  GPF_E_NOMEM = -4,        /* device or host allocation failed                 */
  GPF_E_DEVICE = -5,       /* HIP runtime error                                */
  GPF_E_UNSUPPORTED = -6,  /* size or mode not supported                       */
  GPF_E_BUSY = -7          /* serving queue full: retry later                  */
} gpf_status;

/* bits of the device status word */
#define GPF_DEV_OUT_OF_GRID 1u
#define GPF_DEV_SINGULAR    2u

/* plan flags */
#define GPF_FP32        0u   /* default: FP32 fields, FP64 Schur and constraints */
#define GPF_FP64        1u   /* every field and convolution in FP64               */
#define GPF_CONV1_FP64  2u   /* FP32 plan, but the first convolution (whose
                                surface values feed the ill-conditioned Schur
                                solve) in FP64, for every body               */
#define GPF_POLICY_AUTO 4u   /* FP32 plan; first convolution in FP64 only for
                                bodies whose measured noise amplification
                                exceeds GPF_AMP_THRESHOLD                    */
#define GPF_AMP_THRESHOLD 500.0
#define GPF_PLAN_MULTISTREAM 16u /* gpf_solve keeps one workspace (and
                                descriptor ring) per HIP stream, so solves on
                                different streams may share the plan; the
                                building blocks, time stepping and kernel
                                timing still serve one stream at a time    */
#define GPF_PSI_TOTAL   8u   /* store the total streamfunction psi = s + s_inf
                                (s_inf = U_inf y - V_inf x, Sec. 2.1) instead
                                of s; velocities are then differenced from
                                psi and U_inf is not added again.  With FP32
                                fields psi is rounded at the magnitude of
                                U_inf y, which costs velocity accuracy
                                (about ulp(|psi|)/dx); off by default       */

typedef enum {
  GPF_NOBODY = 0,          /* no surface: s = -L^-1 R_v Gamma                  */
  GPF_CIRCULATION = 1,     /* prescribed bound circulation gamma_b (eq. circsystem) */
  GPF_KUTTA_STEADY = 2,    /* Kutta condition at the body's first edge, bound
                              circulation free (eq. kuttasystem)               */
  GPF_KUTTA_SHED = 3,      /* Kutta condition at the body's m edges, each with a
                              new vortex, total circulation zero (eqs.
                              kuttasystem2, kuttasystem3); with the edge
                              bounds fmin/fmax, the generalized edge
                              conditions (eq. twovortex-gen)                   */
  GPF_PARTS = 4            /* a body of several parts (gpf_body_set_parts),
                              each with its own uniform value s0_j and its own
                              constraint from in->parts (Sec. 2.7, eq.
                              kuttasystem4)                                    */
} gpf_mode;

#define GPF_MAX_EDGES 8
#define GPF_MAX_PARTS 8

/* One part of a several-part body (mode GPF_PARTS). */
typedef struct {
  int mode;                /* GPF_CIRCULATION, GPF_KUTTA_STEADY (at the part's
                              first edge) or GPF_KUTTA_SHED (a new vortex at
                              each of the part's edges, Kelvin's theorem for
                              the part)                                        */
  double gamma_b;          /* GPF_CIRCULATION: the part's bound circulation    */
  double gamma_w;          /* GPF_KUTTA_SHED: circulation of the vortices this
                              part released before                             */
  double ub, vb, omega;    /* rigid motion of the part (eqs. velsurf, sfsurf)  */
} gpf_part;

typedef struct gpf_ctx gpf_ctx;
typedef struct gpf_plan gpf_plan;
typedef struct gpf_body gpf_body;
typedef struct gpf_batch gpf_batch;
typedef struct gpf_rk2 gpf_rk2;
typedef struct gpf_shed gpf_shed;

typedef struct {
  int n;                   /* nodes per direction (power of two, 16..2048)      */
  double dx;               /* cell size                                         */
  double x0, y0;           /* position of node (0, 0)                           */
} gpf_grid;

typedef struct {
  int nv;                              /* number of vortices (>= 0)            */
  const double *d_xv, *d_yv, *d_gv;    /* vortex x, y, strength Gamma_q         */
  double u_inf, v_inf;                 /* uniform flow (Sec. 2.1, s_inf)        */
  double ub, vb, omega;                /* rigid body velocity and rotation
                                          rate (eqs. velsurf, sfsurf)          */
  int mode;                            /* gpf_mode                              */
  double gamma_b;                      /* GPF_CIRCULATION: bound circulation    */
  int m;                               /* GPF_KUTTA_SHED: number of new vortices,
                                          equal to the body's edge count        */
  double h_xnew[GPF_MAX_EDGES];        /* GPF_KUTTA_SHED: new vortex positions, */
  double h_ynew[GPF_MAX_EDGES];        /*   one per edge, in edge order         */
  double gamma_w;                      /* GPF_KUTTA_SHED: circulation of the
                                          existing vortices; NaN = sum of d_gv  */
  double fmin[GPF_MAX_EDGES];          /* GPF_KUTTA_SHED: generalized edge      */
  double fmax[GPF_MAX_EDGES];          /*   conditions (Sec. 2.5): bounds on the
                                          non-singular sheet f~ at each edge, in
                                          edge order.  An edge where the sheet
                                          the body would carry with nothing shed
                                          (Kelvin-consistent intermediate, f~* -
                                          (fhat0.f~* + Gamma_w)/Gamma0) lies in
                                          [fmin, fmax] sheds nothing (its new
                                          vortex gets strength 0); otherwise
                                          f~_k is held at the bound it violates.  fmin = fmax = 0 (a zeroed
                                          struct) is the Kutta condition; +-inf
                                          leaves an edge free.  For a flat plate
                                          of chord c, bounds on the suction
                                          parameter map as f~ = -2 pi c sigma /
                                          Gamma0.  fmin > fmax or NaN:
                                          GPF_E_INVALID.                        */
  int nparts;                          /* GPF_PARTS: the body's part count;
                                          then ub, vb, omega, gamma_b and
                                          gamma_w above are unused, and m,
                                          h_xnew/h_ynew and fmin/fmax list the
                                          edges of the GPF_KUTTA_SHED parts in
                                          the body's edge order               */
  gpf_part parts[GPF_MAX_PARTS];       /* GPF_PARTS: one entry per part        */
} gpf_inputs;

typedef struct {
  void *d_psi;             /* n*n field s, float for FP32 plans, double for
                              GPF_FP64 plans (required)                        */
  double *d_u, *d_v;       /* nv velocities at the vortices, including the
                              uniform flow (nullable)                          */
  double *d_f;             /* ns bound sheet strength f (nullable)            */
  double *d_ftilde;        /* ns non-singular part f / f0 (nullable)          */
  double *d_scalars;       /* 4 + GPF_MAX_EDGES + 2 GPF_MAX_PARTS doubles
                              (nullable):
                              [0] circulation of the vortices sum Gamma_q,
                              [1] total circulation of the final source,
                              [2] s0 (of part 0 with GPF_PARTS),
                              [3] bound circulation <1, f> (all parts),
                              [4..11] strengths of the new vortices,
                              [12..19] GPF_PARTS: s0_j of each part,
                              [20..27] GPF_PARTS: bound circulation of each
                              part                                            */
  unsigned int *d_status;  /* device status word, OR-ed with GPF_DEV_* bits
                              (required; the caller clears it)                */
  double *d_impulse;       /* 3 doubles (nullable): linear impulse P_x, P_y
                              and angular impulse Pi_O about the origin of
                              the fluid (eqs. linimpxd, linimpyd, angimpd):
                              every vortex (new ones included) and the body's
                              sheet plus its motion term, the surface
                              velocity taken relative to the fluid at
                              infinity.  Force and moment on a single body
                              are -rho d(P, Pi_O)/dt (eq. FMimp).  With a
                              body it needs d_f.  With zero total
                              circulation it does not depend on the origin. */
} gpf_outputs;

/* Context bound to one HIP device. */
gpf_status gpf_ctx_create(int device, gpf_ctx **out);
void gpf_ctx_destroy(gpf_ctx *ctx);

/* Plan for one grid: lattice Green's function table and its spectrum
 * (Sec. 2.1, L^-1 by the lattice Green's function), twiddles and
 * workspaces.  The spectrum of the zero-padded (2n)^2 kernel is real; it is
 * stored as (n+1)^2 values with the scale -dx^2/(2n)^2 and a gauge shift of
 * its mean folded in.  Blocking (host work: table quadrature and FP64 FFT). */
gpf_status gpf_plan_create(gpf_ctx *ctx, const gpf_grid *grid, unsigned flags,
                           gpf_plan **out);
void gpf_plan_destroy(gpf_plan *plan);

/* Body: ns surface points (host arrays, FP64), segment lengths ds
 * (Sec. 2.2.1), and nedge edge indices (for the Kutta modes, Sec. 2.4).
 * Builds S = -E_s L^-1 R_s exactly in FP64 from the LGF table on the
 * device, inverts it in FP64 with partial pivoting, and forms
 * f0 = S^-1 1 (eq. f0), Gamma0 = <1, f0> (eq. circ0) and fhat0.
 * Returns GPF_E_SINGULAR for a singular S or Gamma0 == 0,
 * GPF_E_OUT_OF_GRID if a surface stencil leaves the window.  Blocking. */
gpf_status gpf_body_create(gpf_plan *plan, int ns, const double *h_xs,
                           const double *h_ys, const double *h_ds, int nedge,
                           const int *h_edges, gpf_body **out);
void gpf_body_destroy(gpf_body *body);

/* Per-body constants: Gamma0, the measured noise amplification of S^-1
 * (relative L2 change of S^-1 r per relative change of r, for the
 * highest-frequency perturbation of the unit-freestream rhs r = -y_s), and
 * whether the first convolution runs in FP64 for this body (0/1). */
gpf_status gpf_body_info(const gpf_body *body, double *gamma0, double *amp,
                         int *conv1_fp64);

/* Copy the body's f0 = S^-1 1 (ns doubles) to host memory.  Blocking. */
gpf_status gpf_body_f0(const gpf_body *body, double *h_f0);

/* Unit surface normals (ns doubles each, host).  closed = 1: the points
 * enclose a region and the normals point into the fluid; they enter the
 * impulse's body-motion term and the body's area and centroid (appendix on
 * discrete surfaces).  closed = 0: a body of zero thickness (a plate); the
 * normals only orient its two sides for the pressure (+ side = the side
 * the normal points to) and the motion term and area are zero, its two
 * faces cancelling.  A body without normals counts as of zero thickness
 * and has no pressure.  Also builds the pressure operator
 * Q = -(C_s L^-1 C_s^T)^+ C_s L^-1 R_s (Sec. 2.6.1; a closed surface's
 * uniform direction removed, dS-weighted mean of dphi zero) when every
 * point lies two nodes inside the window and ns <= 4096.  Non-finite
 * values: GPF_E_INVALID.  Blocking. */
gpf_status gpf_body_set_normals(gpf_body *body, const double *h_nx, const double *h_ny, int closed);

/* Pressure of a solved problem (Sec. 2.6.1).  d_psi and d_f are the
 * solve's field and sheet (same plan, body, inputs `in`: uniform flow,
 * body or part motion).  Writes on the device:
 *   d_dphi (ns): the potential jump across the surface, dphi = Q f;
 *   d_dp (ns): the pressure jump p+ - p- from the surface Bernoulli
 *     equation (eq. surfbernoulli), d(dphi)/dt = (dphi - d_dphi_prev)/dt
 *     when d_dphi_prev (the previous time level's d_dphi) is given, else 0;
 *   d_p (n*n, nullable): the grid pressure on the cell centres
 *     (x0 + (i+1/2) dx, y0 + (j+1/2) dx) at [j*n + i], i, j < n-1 (eq.
 *     pgrid; last row and column zero), up to a uniform value;
 *   d_pside (2 ns, nullable, needs d_p): p+ then p- on the two sides,
 *     E_c p +- dp/2.
 * rho is the fluid density.  Asynchronous on hip_stream; the body needs
 * normals (GPF_E_INVALID) and its pressure operator (GPF_E_UNSUPPORTED). */
gpf_status gpf_pressure(gpf_plan *plan, const gpf_body *body, const gpf_inputs *in,
                        const void *d_psi, const double *d_f, const double *d_dphi_prev,
                        double dt, double rho, double *d_dphi, double *d_dp, double *d_p,
                        double *d_pside, void *hip_stream);

/* Split the body's points into nparts parts (2..GPF_MAX_PARTS; h_part[p]
 * is the part of point p, every part non-empty) for mode GPF_PARTS: the
 * parts share one Schur complement (they see each other) and each has its
 * own uniform value and constraint (Sec. 2.7).  Computes per part
 * S^-1 1_j, S^-T (dS o 1_j) and the circulations of the former.  Edges
 * belong to the part of their point.  Blocking. */
gpf_status gpf_body_set_parts(gpf_body *body, int nparts, const int *h_part);

/* Enclosed area V = (<x_s, n_x> + <y_s, n_y>)/2 and centroid
 * X_c = <x_s^2 + y_s^2, n_x>/(2V), Y_c likewise with n_y (eq. centroid).
 * Without normals: area 0 and the arc-length centroid of the points. */
gpf_status gpf_body_geometry(const gpf_body *body, double *area, double *xc, double *yc);

/* Added-mass tensor (Sec. 2.6.3), 3x3 row-major into h_m: rows are unit
 * x translation, unit y translation and unit rotation about the origin,
 * columns the force x, force y and moment about the centroid coefficients:
 * rho (P_x, P_y, Pi_O - (X_c P_y - Y_c P_x)) of the sheet
 * f = S^-1 P^Gamma s_b of that motion (no Kutta condition) with its motion
 * term.  The rotation row and column follow the paper's formula, which
 * keeps the rigid surface velocity in the motion term (a circle gives
 * -pi a^4 rho there).  Blocking. */
gpf_status gpf_body_added_mass(const gpf_body *body, double rho, double *h_m);

/* One full solve (Sec. 2.2-2.4): R_v, L^-1, E_s, Schur and constraint
 * solve, R_s, L^-1, E_v.  body may be NULL only with GPF_NOBODY.
 * Asynchronous on hip_stream (NULL = default stream). */
gpf_status gpf_solve(gpf_plan *plan, const gpf_body *body,
                     const gpf_inputs *in, const gpf_outputs *out,
                     void *hip_stream);

/* ---- batches of independent problems ------------------------------------ */

/* Workspaces for up to max_problems problems solved together. */
gpf_status gpf_batch_create(gpf_ctx *ctx, int max_problems, gpf_batch **out);
void gpf_batch_destroy(gpf_batch *batch);

/* Run a batch over `lanes` (1..4) internal streams: the caller's stream is
 * forked to them with an event before the solve and joined after it, so
 * that the latency-bound kernels of one part overlap the bandwidth-bound
 * passes of another.  A batch of several configuration groups (grid sizes,
 * precisions) puts whole groups on the lanes, the costliest first on the
 * least loaded lane (cost ~ problems x n^2), so that small grids run beside
 * large ones; a batch of one group deals its members out over the lanes.
 * Results are unchanged; lanes = 1 (the default) runs everything on the
 * caller's stream.  The fork and join are events, so a captured graph
 * records them. */
gpf_status gpf_batch_set_lanes(gpf_batch *batch, int lanes);

/* The batch's current lane count (1 after create, then as set by
 * gpf_batch_set_lanes or chosen by gpf_autotune_batched); 0 for NULL. */
int gpf_batch_get_lanes(const gpf_batch *batch);

/* merge = 1 (the default) lets gpf_solve_batched run a batch of several
 * grid sizes merged (see below), with the problems whose first convolution
 * is FP64 solved (velocities included) on a side stream of the batch, and
 * the FP32 ones of the largest grid size and of the other sizes on the
 * caller's stream and a second side stream (forked from and joined to the
 * caller's stream with events); 2 runs merged batches on the caller's
 * stream alone (the same
 * kernels, none concurrent: what per-kernel timing measures); 0 makes it
 * run such a batch group by group on its lanes, the path the merged one is
 * compared with.  Results are the same bits for every value.  GPF_E_INVALID
 * for a value outside 0..2. */
gpf_status gpf_batch_set_merge(gpf_batch *batch, int merge);

/* Solve nprob independent problems (each as in gpf_solve; bodies may be
 * NULL or hold NULL for GPF_NOBODY problems).  A batch whose problems have
 * one-part bodies and FP32 fields on grids of n = 64 .. 2048 (any mix of
 * sizes, and of FP32 and FP64 first convolutions) runs merged: every stage
 * of the solve is one launch per precision of the first convolution over all
 * grid sizes, and the FP32 transform passes take their blocks from one work
 * list ordered by decreasing grid size (the largest transforms start first,
 * the small ones fill in behind them).  Otherwise problems are grouped by
 * grid size and precision and each group runs as one launch sequence whose
 * kernels cover all of its problems (one grid dimension indexes the
 * problem), on the batch's lanes.  Either way small problems share launches
 * instead of paying one launch each.
 * Problem i uses workspace i of the batch; plans and bodies may repeat.
 * Every problem needs its own output buffers and status word (a status word
 * may be shared).  Asynchronous on hip_stream; the batch serves one stream
 * at a time.  No step adds with floating-point atomics: every call gives
 * the same bits, and results equal those of solving each problem alone up
 * to rounding (merged launches shape the transforms differently). */
gpf_status gpf_solve_batched(gpf_batch *batch, int nprob, gpf_plan *const *plans,
                             const gpf_body *const *bodies, const gpf_inputs *inputs,
                             const gpf_outputs *outputs, void *hip_stream);

/* ---- serving ----------------------------------------------------------- */

/* A request server for independent solves (many callers, mixed grid sizes).
 * The server owns one resident plan per grid (gpf_server_plan), three sets
 * of max_slots problem workspaces, each with its own non-blocking HIP
 * stream, and a worker thread.  The worker takes queued requests in arrival
 * order, up to max_slots at a time, and solves them as one batch
 * (gpf_solve_batched, merged on that stream alone: merge mode 2) on a free
 * set's stream, so up to three batches run on
 * the device at once; completion is observed with an event per batch.
 * Admission: a request is refused with GPF_E_NOMEM when the server's
 * resident plans plus the three workspace sets at the largest grid seen
 * would exceed hbm_budget_bytes (bodies belong to the caller and are not
 * counted), and with GPF_E_BUSY when 64 * max_slots requests are already
 * waiting.  plan_flags (GPF_FP32, GPF_POLICY_AUTO, ...) apply to every
 * server plan.  max_slots in [1, 256]. */
typedef struct gpf_server gpf_server;
gpf_status gpf_server_create(gpf_ctx *ctx, size_t hbm_budget_bytes, int max_slots,
                             unsigned plan_flags, gpf_server **out);

/* The server's resident plan for *grid (created on first use; owned by the
 * server, valid until gpf_server_destroy).  Bodies for requests on this
 * grid are created on it with gpf_body_create. */
gpf_status gpf_server_plan(gpf_server *srv, const gpf_grid *grid, gpf_plan **out);

/* Queue one solve (as gpf_solve) on the server plan of *grid; body may be
 * NULL for GPF_NOBODY and must otherwise have been created on that plan.
 * The inputs and outputs structs are copied; the device buffers they name
 * must hold their final contents when the request is submitted (the
 * server's streams do not wait for other streams: synchronize the stream
 * that wrote or cleared them), stay valid and untouched until the request
 * is done, and no two requests in flight may share an output field.
 * Data-dependent errors go to
 * the request's d_status as with gpf_solve.  *request_id identifies the
 * request for gpf_server_poll / gpf_server_wait. */
gpf_status gpf_server_submit(gpf_server *srv, const gpf_grid *grid, const gpf_body *body,
                             const gpf_inputs *in, const gpf_outputs *out,
                             unsigned long long *request_id);

/* *done = 1 once the request's outputs are complete; then *latency_s is the
 * time from submission to the observed completion (host clock) and the
 * return value is the request's launch status (GPF_OK or the error that
 * prevented it).  An unknown or already collected id gives GPF_E_INVALID.
 * A done request is forgotten after it has been reported. */
gpf_status gpf_server_poll(gpf_server *srv, unsigned long long request_id, int *done,
                           double *latency_s);

/* Block until the request is done; as gpf_server_poll otherwise. */
gpf_status gpf_server_wait(gpf_server *srv, unsigned long long request_id, double *latency_s);

/* Finish every queued request, then free the server and its plans. */
void gpf_server_destroy(gpf_server *srv);

/* Batches dispatched so far and the most that were in flight on the device
 * at once (at most three); either pointer may be null. */
gpf_status gpf_server_stats(gpf_server *srv, unsigned long long *batches, int *max_inflight);

/* ---- time stepping ------------------------------------------------------ */

/* Vortex advection by the explicit midpoint rule (the paper advances the
 * vortices with forward Euler or RK4, Sec. 2.4 and 2.6; the midpoint rule
 * uses the same velocity evaluation):
 *     u1 = u(x);  x* = x + dt/2 u1;  u2 = u(x*);  x <- x + dt u2,
 * where every velocity evaluation is a full solve as in gpf_solve with the
 * settings of `in` (mode, uniform flow, body motion, gamma_b; the shedding
 * mode is not supported: new vortices need a release rule).  d_x, d_y (nv
 * doubles, device) are the vortex positions, updated in place by each step;
 * in->d_gv holds the strengths; in->d_xv, in->d_yv are ignored.  With
 * use_graph = 1 one step is captured once into a HIP graph (two solves and
 * two position updates) and every step replays it; the descriptor slots of
 * the plan that the capture took stay reserved until gpf_rk2_destroy, which
 * releases them (a failed capture releases them at once).  The object owns its workspace, so
 * other calls on the same plan (which may grow the plan's workspace) leave
 * the captured step valid, and the field, velocity, sheet and status buffers
 * of the last stage (gpf_rk2_fields). */
gpf_status gpf_rk2_create(gpf_plan *plan, const gpf_body *body, const gpf_inputs *in,
                          double *d_x, double *d_y, double dt, int use_graph,
                          gpf_rk2 **out);

/* Enqueue nsteps steps on hip_stream (asynchronous). */
gpf_status gpf_rk2_run(gpf_rk2 *rk, int nsteps, void *hip_stream);

/* Device buffers of the last stage: field s (n*n, plan field type),
 * velocities u, v at the midpoint positions, sheet strength f (ns, NULL
 * without a body), scalar block (as in gpf_outputs) and status word. */
gpf_status gpf_rk2_fields(const gpf_rk2 *rk, const void **d_psi, const double **d_u,
                          const double **d_v, const double **d_f,
                          const double **d_scalars, unsigned int **d_status);
/* Waits for the replays enqueued by the last gpf_rk2_run (replays enqueued
 * earlier on other streams must be complete), then frees the object and
 * returns its descriptor slots to the plan.  Destroy before the plan. */
void gpf_rk2_destroy(gpf_rk2 *rk);

/* Vortex shedding with forward Euler steps (Sec. 2.4.2: new vortices go one
 * third of the way from the edge to the last vortex released there, and the
 * vortices move with forward Euler; Sec. 2.5 for edge bounds).  Each step:
 *   1. places one new vortex per body edge k_j, at e + (z_last - e)/3, e the
 *      edge point and z_last the current position of the last vortex edge j
 *      released with nonzero strength, or at e + (h_first[2j], h_first[2j+1])
 *      before edge j has released one;
 *   2. appends the new vortices with strength zero (so the velocity is
 *      evaluated at them too) and solves in the shedding mode of `in`, edge
 *      bounds included, which gives their strengths Gamma_j (zero at an edge
 *      inside its bounds);
 *   3. stores Gamma_j and advances every vortex: x <- x + dt u(x).
 * in->mode must be GPF_KUTTA_SHED with in->m equal to the body's edge
 * count; in->h_xnew/h_ynew and in->gamma_w are ignored (Gamma_w is the sum
 * of the strengths).  Several bodies (Sec. 2.7): in->mode GPF_PARTS on a
 * body split by gpf_body_set_parts, with in->m equal to the edge count of
 * the parts in GPF_KUTTA_SHED mode; every such edge sheds (body edge order,
 * which h_first follows too), parts[j].gamma_w is the circulation part j
 * has released before the first step, and each step adds the strengths of
 * its edges' new vortices to it (kept on the device), so that each shedding
 * part keeps its bound circulation equal to minus what it has released.
 * The body stays in place: ub, vb, omega (and every part's) must be zero
 * (GPF_E_UNSUPPORTED otherwise; a translating body is the same flow as a
 * body at rest in the opposite uniform flow).  d_x, d_y, d_g are device arrays of `capacity`
 * doubles owned by the caller: the first in->nv hold the initial vortices
 * (in->d_xv/d_yv/d_gv are ignored), every step appends m vortices and
 * moves them all in place.  `out` names caller-owned buffers as for
 * gpf_solve, overwritten by every step: d_u and d_v (capacity doubles; the
 * velocities before the position update), d_scalars and d_status are
 * required, d_f and d_ftilde optional.  d_impulse, if set, is a history:
 * step k since creation writes its impulse (after the solve, new vortices
 * included, before the positions move) to d_impulse[3k..3k+2], so it must
 * hold 3 (capacity - in->nv) / m doubles; it needs d_f.  h_first holds 2m doubles (host).
 * gpf_shed_run returns GPF_E_INVALID, enqueueing nothing, when the steps
 * would exceed the capacity.  A vortex that leaves the window sets
 * GPF_DEV_OUT_OF_GRID in the status word, and the results from then on
 * are not valid. */
gpf_status gpf_shed_create(gpf_plan *plan, const gpf_body *body, const gpf_inputs *in,
                           const gpf_outputs *out, double *d_x, double *d_y, double *d_g,
                           int capacity, double dt, const double *h_first, gpf_shed **sh);

/* Enqueue nsteps steps on hip_stream (asynchronous). */
gpf_status gpf_shed_run(gpf_shed *sh, int nsteps, void *hip_stream);

/* Number of vortices after the enqueued steps (-1 for a NULL object). */
int gpf_shed_count(const gpf_shed *sh);
void gpf_shed_destroy(gpf_shed *sh);

/* ---- building blocks (asynchronous on hip_stream) ---------------------- */

/* w = R_v Gamma (eq. vortexregularization): d_w is n*n of the plan's field
 * type; accumulate = 0 overwrites, 1 adds.  Out-of-window vortices are
 * skipped and flagged in d_status. */
gpf_status gpf_regularize_vortices(gpf_plan *plan, int nv, const double *d_xv,
                                   const double *d_yv, const double *d_gv,
                                   void *d_w, int accumulate,
                                   unsigned int *d_status, void *hip_stream);

/* s = -L^-1 w by the zero-padded LGF convolution (Sec. 2.1).  d_w, d_s are
 * n*n of the plan's field type (may alias).  gamma_src must equal
 * dx^2 * sum(w) (the source circulation): the spectrum is gauge-shifted and
 * the exact shift -c * gamma_src is restored in the epilogue. */
gpf_status gpf_convolve(gpf_plan *plan, const void *d_w, void *d_s,
                        double gamma_src, void *hip_stream);

/* gpf_convolve for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and result as gpf_convolve; calls no hipMalloc,
 * hipFree or other allocating routine and enqueues no host-to-device copy.
 * The (n+1) x n complex intermediate and the launch descriptor live in a
 * fixed device array of 32.8 MiB per device (held until the process ends),
 * whose address is taken when a context is created on the device.  Limit:
 * FP32 plans up to n = 2048, FP64 plans up to n = 1024; larger grids return
 * GPF_E_UNSUPPORTED.  Every call on one device shares that array, so calls
 * that overlap on one device (two streams, two threads) race: serialize
 * them.  d_w and d_s belong to the caller (n*n of the plan's field type, may
 * alias); nothing of the array needs to be cleared between calls. */
gpf_status gpf_convolve_noalloc(gpf_plan *plan, const void *d_w, void *d_s,
                                double gamma_src, void *hip_stream);

/* r = E_s s at the body's surface points (Sec. 2.2.1); d_r: ns doubles. */
gpf_status gpf_interpolate_surface(const gpf_body *body, const void *d_s,
                                   double *d_r, void *hip_stream);

/* (u, v) = E_v of the node velocities of s, plus (u_inf, v_inf) (Sec. 2.1). */
gpf_status gpf_vortex_velocity(gpf_plan *plan, const void *d_s, int nv,
                               const double *d_xv, const double *d_yv,
                               double u_inf, double v_inf, double *d_u,
                               double *d_v, unsigned int *d_status,
                               void *hip_stream);

/* ---- the Schur complement built from batched right-hand sides ----------- */

/* The Schur complement S = -E_s L^-1 R_s (Sec. 2.2.2, eq. basicblock) built
 * column by column: the unit sheets e_q pass through the regularization
 * R_s, the convolution and the interpolation E_s, `batch` columns per
 * batched launch sequence, with FP32 (fp64 = 0) or FP64 fields; the first
 * convolution's row band and the plan's schedules apply.  The result is
 * compared with the body's exact S (built from the LGF table in FP64, as
 * gpf_body_create does): *h_rel_s = ||S_conv - S||_F / ||S||_F, and
 * *h_rel_f = relL2 of S_conv^-1 r against S^-1 r for r = -y_s (the sheet of
 * a unit uniform flow, S_conv inverted in FP64); *h_ms = the time of the
 * column build (ms).  All three nullable; *h_rel_f is infinite when S_conv
 * is singular.  A diagnostic of the build: the body keeps its exact S.
 * Blocks until done; allocates about batch (4 n^2 sizeof(T)) bytes plus
 * 3 ns^2 doubles; batch in [1, 1024], GPF_E_NOMEM beyond 16 GiB. */
gpf_status gpf_body_schur_by_convolution(gpf_body *body, int fp64, int batch, double *h_rel_s,
                                         double *h_rel_f, double *h_ms);

/* ---- convolution schedules and the autotuner --------------------------- */

/* How the three passes of the convolution (Sec. 2.1, the zero-padded LGF
 * convolution) map onto workgroups and XCDs.  Every schedule performs the
 * same transforms; they differ in speed only, and in the last bits of FP64
 * column results (the two column kernels form their twiddles differently).
 *   rows:  row passes; 0 by rule (wide workgroups when a launch gives two or
 *          more per CU), 1 narrow (2-8 sequences), 2 wide (128-byte runs of
 *          the k-major intermediate);
 *   order: row-pass XCD order; 0 by rule (dispatch order where a workgroup's
 *          runs fill whole 128-byte lines, else consecutive row blocks per
 *          XCD), 1 dispatch order, 2 consecutive row blocks per XCD;
 *   cols:  FP64 column pass for n >= 512; 0 or 2 split exchange (real and
 *          imaginary parts through LDS in turn), 1 complex exchange. */
typedef struct {
  int rows, order, cols;
} gpf_schedule;

/* Schedules live in the context, keyed by grid size n, precision (fp64 =
 * 1: the FP64 transforms, 0: FP32) and batch-size class of nb (1, 2-7, 8-31,
 * 32 and more).  Solves, batched solves and the building blocks on that
 * context use the entry of their group (the first convolution of a body
 * under the precision policy uses its FP64 entry).  gpf_schedule_set stores
 * *s (NULL: drop the entry, back to the rules); values outside the ranges
 * above give GPF_E_INVALID.  gpf_schedule_get writes the entry in force
 * (zeros where there is none). */
gpf_status gpf_schedule_set(gpf_ctx *ctx, int n, int fp64, int nb, const gpf_schedule *s);
gpf_status gpf_schedule_get(gpf_ctx *ctx, int n, int fp64, int nb, gpf_schedule *s);

/* Autotuner: times the rules and every schedule (rows 1-2 x order 1-2 x,
 * for FP64 from n = 512, cols 1-2) on nb convolutions of the plan's grid in the given
 * precision (synthetic zero sources; the time does not depend on the values),
 * stores the fastest in the context as by gpf_schedule_set, and returns it
 * in *chosen and its mean time per batched convolution (microseconds) in
 * *us (both nullable).  cache_path (nullable) names a text file of earlier
 * results, one per line "arch n fp64 class rows order cols us": a matching
 * line (same device architecture, n, precision and class) is used without
 * timing; a new result is appended.  Blocks until the timing is done;
 * allocates about 4 nb n^2 sizeof(T) bytes of device memory while it runs
 * (T: float or double).  nb must be in [1, 1024]; GPF_E_NOMEM beyond
 * 16 GiB. */
gpf_status gpf_autotune(gpf_plan *plan, int fp64, int nb, const char *cache_path,
                        gpf_schedule *chosen, double *us);

/* Autotuner on a real workload: first the batch's lane count (1..4, as by
 * gpf_batch_set_lanes), then, for every schedule entry the batch's groups
 * use (per grid size and precision; a body's first convolution under the
 * precision policy uses the FP64 entry, its second the field precision),
 * the rules and every explicit shape in turn, each choice timing the whole
 * batched solve (gpf_solve_batched with these arguments, which it runs
 * about seven times per trial on hip_stream, overwriting the outputs; a
 * lane count above one first runs it 400 times, since new streams run a
 * workload's first few hundred solves slower) and keeping the fastest (the lane count in the batch, the schedules in the
 * context).  Entries are tuned one after another, the others staying at
 * their current values.  Blocks until done; the outputs then hold the
 * result of the last solve. */
gpf_status gpf_autotune_batched(gpf_batch *batch, int nprob, gpf_plan *const *plans,
                                const gpf_body *const *bodies, const gpf_inputs *inputs,
                                const gpf_outputs *outputs, void *hip_stream);

/* ---- kernel timing ----------------------------------------------------- */

/* Kernel classes timed by HIP events recorded on the launch stream. */
#define GPF_TK_SCATTER    0   /* vortex regularization R_v                       */
#define GPF_TK_ROWS_FWD   1   /* convolution pass 1 (FP32)                       */
#define GPF_TK_COLS       2   /* convolution pass 2 (FP32)                       */
#define GPF_TK_ROWS_INV   3   /* convolution pass 3 (FP32)                       */
#define GPF_TK_ROWS_FWD64 4   /* convolution pass 1 (FP64)                       */
#define GPF_TK_COLS64     5   /* convolution pass 2 (FP64)                       */
#define GPF_TK_ROWS_INV64 6   /* convolution pass 3 (FP64)                       */
#define GPF_TK_SURFACE    7   /* E_s, Schur apply, constraints, R_s              */
#define GPF_TK_VELOCITY   8   /* velocity interpolation E_v                      */
#define GPF_TK_COUNT      9

/* Enable (1) or disable (0) per-kernel event timing for calls on this plan
 * from the calling thread; enabling clears the totals.  Timing adds one
 * event pair per timed launch; it must be off during graph capture. */
gpf_status gpf_timing_enable(gpf_plan *plan, int enable);

/* Wait for the recorded events and return the number of timed launches of
 * kernel class `kind` and their summed duration in milliseconds. */
gpf_status gpf_timing_read(gpf_plan *plan, int kind, long long *count,
                           double *total_ms);

/* ---- host utilities ---------------------------------------------------- */

/* FP64 inverse of a dense n x n matrix on the device, the operation the
 * library applies to the Schur complement S of a body (Sec. 2.2.2, App. A):
 * d_a and d_ainv are row-major device arrays of n*n doubles (d_a is read
 * only; they must not overlap), on ctx's device, queued on hip_stream (null:
 * the default stream), which the call waits for before it returns.  Gauss-
 * Jordan elimination with partial pivoting (largest |entry| of the column,
 * lowest row on ties); n <= 2048 in 16-column panels whose updates run on
 * FP64 matrix cores, larger n column by column.  *min_pivot_rel (may be
 * null) receives min |pivot| / max |a_ij|: values near 1e-14 or below mean
 * a numerically singular matrix, whose inverse is not meaningful.
 * GPF_E_INVALID for n outside [1, 8192] or null arrays. */
gpf_status gpf_invert_fp64(gpf_ctx *ctx, int n, const double *d_a, double *d_ainv,
                           void *hip_stream, double *min_pivot_rel);

/* Lattice Green's function table T[a*(nmax+1)+b] = G(a, b), 0 <= a,b <= nmax,
 * G(0,0) = 0 (host computation, no device needed). */
gpf_status gpf_lgf_table(int nmax, double *h_table);

/* Wait for hip_stream, read the status word, clear it, and map its bits to
 * a gpf_status (GPF_E_OUT_OF_GRID before GPF_E_SINGULAR). */
gpf_status gpf_sync(void *hip_stream, unsigned int *d_status);

/* Thread-local message of the last failing call on this thread. */
const char *gpf_last_error(void);

/* Library version string. */
const char *gpf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GPF_H */
