/*
 * gpmg -- MI355X (gfx950) monolithic multigrid for the ghost-point level-set Navier-Stokes method of
 * A. Coco, "A multigrid ghost-point level-set method for incompressible Navier-Stokes equations on moving
 * domains with curved boundaries" (arXiv:1911.00994).
 *
 * C ABI.  Every entry point takes plain pointers and sizes; no C++ or torch types cross this boundary.
 *
 * Problem solved (Sect. 2, eq. (spaceprobaug); Sect. 3, Alg. LS; Sect. 4, eq. (eq:LS)): on D = (-1,1)^2
 * with a body R = {phi > 0} and fluid Omega = D \ R, find (u, v, p, xi) with
 *     u - alpha lap u + grad p = f      (internal points of the two staggered velocity grids)
 *     div u - xi = g                    (internal cell centres)
 *     sum over internal p of p = 0      (mean-pressure row, eq. (eq:midpoint), scaled by 1/count)
 * and one boundary row per ghost point (biquadratic Dirichlet rows eq. (BCu) for u and v, normal-derivative
 * rows of the same interpolant for p), Dirichlet rows for the normal velocity on the box walls, and
 * second-order ghost rows for the tangential velocity on the box walls.  A Crank-Nicolson step (Sect. 2,
 * eqs. (NSCN1), (extrUdU), (NSitconv)) assembles f from the previous state and calls the solver; the
 * pressure unknown is dt * p (the paper's rescaling after eq. (spaceprob)).
 *
 * Grid layout (all arrays of this ABI): N cells per side (a power of two, >= 16), h = 2/N, W = N + 2.
 * Each grid array has W*W doubles, entry [(j+1)*W + (i+1)] for i, j in [-1, N]:
 *     u(i,j) at (-1 + i h,       -1 + (j+1/2) h)     vertical faces   (i = 0 and N are the box walls)
 *     v(i,j) at (-1 + (i+1/2) h, -1 + j h)           horizontal faces (j = 0 and N are the box walls)
 *     p(i,j) at (-1 + (i+1/2) h, -1 + (j+1/2) h)     cell centres
 * Entries that carry no equation are ignored on input and returned as stored.  The level set is sampled
 * on the half-step lattice: phi[ky*(2N+1) + kx] at (-1 + kx h/2, -1 + ky h/2), kx, ky in [0, 2N], positive
 * inside the body (Sect. 3.1).
 *
 * Ownership: the context owns every device buffer it uses.  Input pointers are borrowed for the duration of
 * the call and copied (host pointers, or device pointers when on_device != 0, which must belong to the
 * context's device).  Output pointers are caller-allocated host buffers unless stated otherwise.  All GPU
 * work is ordered on the stream given to gp_setup_grid; calls that return data to the host synchronise it.
 * A context is not thread-safe; use one context per stream.
 *
 * Errors: every call returns a gp_status; 0 is success.  On error the context stays usable unless stated.
 */
#ifndef GPMG_H
#define GPMG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gp_ctx gp_ctx;
typedef int gp_status;

enum {
  GP_OK = 0,
  GP_EINVAL = -1,    /* bad argument (N not a power of two or < 16, NULL pointer, bad option) */
  GP_ENOMEM = -2,    /* device or host allocation failed */
  GP_EHIP = -3,      /* HIP runtime error (gp_last_hip_error gives the text) */
  GP_EGEOM = -4,     /* geometry rejected: body touches the box walls, a finest-level ghost has no usable
                        row, or an internal cell has no internal face */
  GP_ENOCONV = -5,   /* max_cycles reached before the tolerance; the iterate is kept, stats are filled */
  GP_EDIVERGED = -6, /* NaN/Inf or residual growth beyond 1e6 times the initial one */
  GP_ESCRATCH = -7   /* gp_solve_noalloc: the problem's workspace exceeds the library's static scratch array */
};

enum { GP_FP64 = 0, GP_MIXED = 1 };

/* point classes returned by gp_get_classes */
enum { GP_INACTIVE = 0, GP_INTERNAL = 1, GP_GHOST = 2, GP_WALL_DIRICHLET = 3, GP_WALL_GHOST = 4, GP_EXTENSION = 5,
       GP_GHOST_EXTRAP = 7 };

/* Solver parameters.  Defaults (gp_default_params): V(2,2) cycles (nu1 = nu2 = 2, gamma = 1; the paper's
 * W cycle is gamma = 2, Sect. 4.3), lambda_ghost = 2 ghost sweeps per box sweep (Alg. relax), coarsest grid
 * 8 x 8 cells solved exactly (Sect. 4.3), Alg. 1 march limit 8 steps and bisection accuracy 0.01 h (Sect. 3.3),
 * fictitious time steps 0.9 (Dirichlet) and 0.9 h (normal derivative) (Sect. 4.1.2), extension band of 4
 * grid steps, minimum ghost-row diagonal cg_min = 0.1 on the coarse levels (below it a coarse ghost takes an
 * extrapolation row; the finest level keeps every defined eq. (BCu) row), optionally bnd_sweeps extra box sweeps
 * after each relaxation step (default 0; same colour order, each followed by lambda_ghost ghost sweeps) over the
 * cells within bnd_radius = 2 cells of a cell touching the body, coupled ghost boxes (ghost_boxes = 1: after the
 * box sweep, each cell whose internal unknowns appear in a body ghost row is relaxed together with those ghosts, on
 * the ghost_box_levels = 1 finest levels), and krylov = 8 (the solves use the cycle as the preconditioner of a
 * GCR iteration restarted after 8 directions; 0 runs the multigrid iteration of Sect. 4 on its own).  The last five fields
 * choose how the same computation is laid out on the device (results agree to rounding): fuse_small_levels = 1
 * runs the cycle of the levels with N <= 32 in one workgroup with their data in LDS, band_split_min = 3000: a
 * boundary band with at least that many cells, and the coupled boxes of a level with a colour of at least that many
 * slots, are relaxed with device-wide launches instead of one workgroup,
 * band_sector_min = 1500: a band with at least that many cells is relaxed by angular sectors, one workgroup each
 * (where the band lies far enough from its centre; otherwise as above),
 * graph_iterations = 0; 1 captures the launches of one solver iteration (cycle, mean projection, residual
 * norm) into a HIP graph at the start of each gp_solve / gp_cn_step solve and replays it every iteration
 * (gp_probe_start turns it off while its events are live), queue_ahead = 1: in FP64 solves without graphs the
 * first box sweep of the next cycle is queued before the host has read the residual norm of the current one,
 * and its workgroups return at once when that norm ends the solve (so the device does not wait for the host
 * between cycles; the iterates are the same). */
typedef struct {
  int nu1, nu2, gamma, lambda_ghost, coarsest_n, march_max, ext_radius;
  double dtau_dir, dtau_neu_over_h, bisect_eps_over_h, cg_min;
  int mixed_inner_cycles; /* FP32 cycles per FP64 refinement step in GP_MIXED solves */
  int bnd_sweeps, bnd_radius;
  int fuse_small_levels, band_split_min, graph_iterations, band_sector_min, queue_ahead;
  int ghost_boxes; /* 1: coupled ghost boxes in every relaxation step (see above); 0: plain boxes only */
  int krylov;      /* m > 0: gp_solve and gp_adjoint_solve accelerate the cycle by GCR restarted after m directions
                      (see gp_solve); 0: the cycle on its own */
  int ghost_box_levels; /* the coupled ghost boxes run on this many finest levels (default 1) */
} gp_params;

/* rigid motion: the body frame point of x at time t is R(-omega t) (x - X0 - U t); the boundary velocity at a
 * boundary point B is U + omega e_z x (B - X0 - U t) */
typedef struct {
  double X0x, X0y, Ux, Uy, omega;
} gp_rigid;

/* analytic body shapes (phi > 0 inside): kind 0: R - r; 1: R^2 - r^2; 2: 1 - (x'^2/A^2 + y'^2/B^2);
 * 3: 1 - sqrt(x'^2/A^2 + y'^2/B^2) with (x', y') rotated by p[2]; 4: A + B cos(m (theta - theta0)) - r
 * with p = {A, B, theta0, m}; 5: no body.  p = {R or A, B, angle, m}. */
typedef struct {
  int kind;
  double p[4];
} gp_shape;

typedef struct {
  int cycles;      /* multigrid cycles (inner FP32 cycles for GP_MIXED) */
  int outer;       /* FP64 refinement steps (GP_MIXED), Picard iterations (gp_cn_step) */
  double res0;     /* initial max-norm residual of the FP64 system */
  double res;      /* final max-norm residual */
  double rho;      /* last residual ratio */
  double seconds;  /* wall time of the call (host clock, includes the final synchronisation) */
  double bytes_alg; /* algorithmic HBM bytes of the call's iterations: per cycle, the compulsory traffic of each
                       level's sweeps (65 B per cell and relaxation step in FP64, 33 in FP32 storage), residual with
                       restriction and prolongation (53 B, 27), weighted by (gamma / 4)^level; per GCR iteration
                       (3 k + 12) vector passes of 8 (3 W^2 + 1) B for the k-th direction; per convergence test
                       41 B per cell */
} gp_stats;

void gp_default_params(gp_params *prm);

/* Create a context for an N x N cell grid and Reynolds number Re (used by gp_cn_step): the staggered MAC grid of
 * Sect. 3.2 on D = (-1, 1)^2 and the multigrid hierarchy of Sect. 4 (levels N, N/2, ... down to the coarsest grid of
 * Sect. 4.3, coarsest_n cells per side), with every device buffer of every level allocated here.  prm may be NULL
 * (defaults).  hip_stream is the hipStream_t all work of the context goes to; NULL makes the context create
 * its own (blocking, default priority, so it orders with the null stream; destroyed by gp_destroy).  *out is
 * NULL on error. */
gp_status gp_setup_grid(gp_ctx **out, int N, double Re, const gp_params *prm, void *hip_stream);
/* Release every device and host resource of the context (resource management; no passage of the paper). */
void gp_destroy(gp_ctx *ctx);
/* Number of grid levels of the hierarchy (Sect. 4.3: from the finest grid to the coarsest, solved exactly). */
int gp_num_levels(const gp_ctx *ctx);
const char *gp_strerror(gp_status st);
const char *gp_last_hip_error(const gp_ctx *ctx);

/* Geometry at time t (Sect. 3.1 - 3.4): classification of every grid point of every level, ghost closure,
 * Alg. 1 boundary points and ghost rows, extension points, and the exact factorisation of the coarsest
 * system.  Default boundary data are set: rigid-body velocity at B for velocity ghosts, zero normal pressure
 * derivative, wall velocities from gp_set_walls.  gp_set_levelset takes sampled phi ((2N+1)^2 doubles);
 * gp_set_levelset_analytic samples a built-in shape on the device.  motion may be NULL (body at rest). */
gp_status gp_set_levelset(gp_ctx *ctx, const double *phi_half, int on_device, double t, const gp_rigid *motion);
gp_status gp_set_levelset_analytic(gp_ctx *ctx, const gp_shape *shape, double t, const gp_rigid *motion);

/* Start building, in the background, the geometry gp_set_levelset_analytic(ctx, shape, t, motion) would build
 * (a moving body's next step is known in advance).  The build runs on a host thread and on streams of a second,
 * internal context (created at the first call: a second copy of the context's buffers), so it overlaps whatever
 * the caller runs meanwhile, and it touches neither the context's vectors nor its current geometry.  The next
 * gp_set_levelset_analytic with the same shape, t and motion (bitwise) takes the prepared geometry instead of
 * building: it waits for the build, exchanges the two geometries and sets the default boundary data.  Any other
 * geometry call, and gp_destroy, waits for the build and discards it.  Errors of the background build are not
 * reported here: gp_set_levelset_analytic then builds as usual and reports them. */
gp_status gp_prepare_levelset_analytic(gp_ctx *ctx, const gp_shape *shape, double t, const gp_rigid *motion);

/* Level-set reinitialisation (Sect. 3.1, eq. (sdf)): phi ((2N+1)^2 doubles on the context's half-step lattice,
 * host or device per on_device) is replaced in place by iters explicit pseudo-time steps of size cfl * (h/2)
 * (0 < cfl <= 0.5) towards the signed distance with the same zero set, positive inside the body: first-order
 * Godunov upwind steps, and next to the interface the distance estimate (h/2) phi / |Delta phi| of the input held
 * fixed (the interface does not move).  After iters steps the values within about iters * cfl * h/2 of the
 * interface are converged.  Use it before gp_set_levelset for a level set that is no longer a distance function
 * (a deforming body).  The first call allocates four lattice-sized buffers on the device.  GP_EINVAL for a NULL
 * phi, iters < 0 or cfl outside (0, 0.5]. */
gp_status gp_reinit_levelset(gp_ctx *ctx, double *phi, int on_device, int iters, double cfl);

/* wall velocities: {bottom u, bottom v, right u, right v, top u, top v, left u, left v} (host array of 8) */
gp_status gp_set_walls(gp_ctx *ctx, const double *walls8);

/* boundary point B and unit normal n (pointing into the body) of every boundary row of the finest level:
 * host arrays of 3*W*W*2 doubles each (grid-major, then point, then x/y); NaN where a point has no row. Wall
 * Dirichlet points report the node itself. */
gp_status gp_get_boundary_geometry(gp_ctx *ctx, double *B, double *nB);

/* boundary data as full grid arrays (W*W each, any may be NULL): the entries at ghost, wall-ghost and
 * wall-Dirichlet points are used (velocity value at B; for pressure ghosts the normal derivative of dt*p). */
gp_status gp_set_boundary_values(gp_ctx *ctx, const double *bu, const double *bv, const double *bp, int on_device);

/* linear-system interface (one solve of eq. (spaceprobaug) at the current geometry) */
gp_status gp_set_alpha(gp_ctx *ctx, double alpha);
gp_status gp_set_rhs(gp_ctx *ctx, const double *fu, const double *fv, const double *g, int on_device);
gp_status gp_set_x(gp_ctx *ctx, const double *u, const double *v, const double *p, double xi, int on_device);
gp_status gp_get_x(gp_ctx *ctx, double *u, double *v, double *p, double *xi, int on_device);
/* one multigrid cycle on the finest level followed by the mean-pressure projection; *res_inf receives the
 * max-norm residual afterwards (may be NULL) */
gp_status gp_mg_vcycle(gp_ctx *ctx, int precision, double *res_inf);
/* Solve the system of the current geometry, alpha and right-hand side (Sect. 4) from the current x until
 * ||r||_inf <= tol * max(1, ||b||_inf) (over all rows as written) or max_cycles cycles.  krylov = 0: the multigrid
 * iteration x <- x + B'(b - M x) of Sect. 4 (B' one cycle and the mean-pressure projection).  krylov = m > 0: the
 * same B' preconditions a generalized conjugate residual iteration (GCR) restarted after m directions (each
 * iteration one cycle, one product with M and the orthogonalisation; the residual is updated recursively and
 * confirmed by the true residual at convergence and at each restart).  GP_MIXED runs the cycle in FP32 storage
 * (the FP64 iteration around it).  st->cycles counts cycles (GCR iterations).  GP_ENOCONV if max_cycles is
 * reached (x keeps the last iterate), GP_EDIVERGED on NaN or growth beyond 1e6 times the initial residual. */
gp_status gp_solve(gp_ctx *ctx, int precision, double tol, int max_cycles, gp_stats *st);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): gp_solve in FP64 (same iteration, same results) without any device allocation.  gp_solve
 * allocates the GCR workspace ((3 + 2 krylov) vectors of 3 W^2 + 1 doubles) at its first call; this entry point
 * takes it from a static device array of 64 MiB that every GPU the library runs on holds until the process ends
 * (its address is looked up once per device at gp_setup_grid).  Limit: the workspace must fit 64 MiB, which holds
 * N <= 256 with the default krylov = 8 (N = 512 with krylov <= 3); larger problems return GP_ESCRATCH (the text
 * via gp_last_hip_error) without touching the context.  krylov = 0 needs no workspace (any N).  The context itself
 * (geometry, hierarchy) is allocated by gp_setup_grid and the geometry calls, so call this after them.  Calls on
 * one GPU share the array: calls that overlap in time on the same GPU (from several threads or streams) race and
 * must be serialised by the caller.  Graph replay (graph_iterations) is not used by this call. */
gp_status gp_solve_noalloc(gp_ctx *ctx, double tol, int max_cycles, gp_stats *st);
/* residual of every row (host array of 3*W*W + 1 doubles, the last entry is the mean-pressure row; may be
 * NULL) and its max norm */
gp_status gp_residual(gp_ctx *ctx, double *r, double *res_inf);

/* time stepping: gp_set_state sets (u, v, dt*p, xi) at t^0 in the current geometry; gp_cn_step advances one
 * step of size dt into the geometry set last (set it for t^{n+1} before the call).  fu, fv: forcing at
 * t^{n+1/2} (u- and v-grid arrays); g: continuity right-hand side at t^{n+1} (may be NULL for 0).  The first
 * two steps use the fixed-point iteration of eq. (NSitconv) until the test eq. (iterativeNS) passes with
 * picard_eps (or picard_max iterations), later steps the extrapolation eq. (extrUdU). */
gp_status gp_set_state(gp_ctx *ctx, const double *u, const double *v, const double *p, double xi, int on_device);
gp_status gp_cn_step(gp_ctx *ctx, double dt, const double *fu, const double *fv, const double *g, int on_device,
                     int precision, double tol, int max_cycles, double picard_eps, int picard_max, gp_stats *st);

/* inspection (tests): classes of one level (host array 3*W_l*W_l bytes); per-point ghost rows of one level
 * (host arrays, 3*W_l*W_l points): B, nB, theta (2 each), weights (9), column indices (9, global index
 * g*W_l*W_l + point), dtau, row kind (1 boundary condition, 2 extrapolation, 0 identity, -1 no row);
 * extension rows (3 sources and 3 weights per point, -1 / NaN where none) */
gp_status gp_get_classes(gp_ctx *ctx, int level, unsigned char *cls);
gp_status gp_get_ghost_rows(gp_ctx *ctx, int level, double *B, double *nB, double *theta, double *w9, int *col9,
                            double *dtau, int *kind);
gp_status gp_get_ext_rows(gp_ctx *ctx, int level, int *src3, double *w3);
/* inspection (tests): the boundary band of one level as the current geometry laid it out (Sect. 4.1, the extra
 * band relaxation): out[0] band cells, out[1] body ghost rows, out[2] angular sectors the band is relaxed over
 * (0: not in sectors), out[3] 1 when the band fits the one-workgroup LDS kernel.  out is a host array of 4 ints.
 * GP_EINVAL for a NULL argument, a level out of range or no geometry yet. */
gp_status gp_get_band_layout(gp_ctx *ctx, int level, int *out);
/* inspection (tests): the coupled ghost boxes of one level (see gp_params.ghost_boxes) in the order a relaxation
 * step visits them (colour (i + 2j) mod 5, then cell index).  counts (host int[2]) receives the number of boxes and
 * of slots (box unknowns, summed over the boxes); each other argument may be NULL: cell[boxes] the cell j*N + i,
 * off[boxes + 1] each box's first slot, idx[slots] the unknown of each slot (global index g*W*W + point: the
 * internal W, E, S, N face and pressure of the cell, then the box's ghosts in increasing order), wr[slots] 1 where
 * the box writes that value (a ghost held by several boxes of one colour is written by the first), colour_off[6]
 * the first box of each colour.  GP_EINVAL for a NULL counts, a level out of range or no geometry yet. */
gp_status gp_get_coupled_boxes(gp_ctx *ctx, int level, int *counts, int *cell, int *off, int *idx, unsigned char *wr,
                               int *colour_off);
/* relaxation steps (Alg. relax with nu = steps) on one level in FP64, on that level's current x and b */
gp_status gp_relax(gp_ctx *ctx, int level, int steps);

/* measurement: average device time in microseconds of one launch of a kernel of the FP64 cycle, recorded
 * with HIP events on the context's stream around reps repetitions on the given level's current data (the data
 * are relaxed further by the box kernel; nothing else changes).  which: 0 = box relaxation (one colour per
 * launch), 1 = residual of the internal rows, 2 = restriction, 3 = prolongation, 4 = ghost sweeps, 5 = box
 * relaxation, all five colours in one launch (tiles in LDS; GP_EINVAL where the level does not use it). */
gp_status gp_time_kernel(gp_ctx *ctx, int which, int level, int reps, double *avg_us);

/* measurement inside a run: gp_probe_start creates 2*max_launches HIP events (1 <= max_launches <= 65536) and
 * from then on the FP64 cycle launches every every-th finest-level five-colour box sweep (the first, then every
 * every-th after it; 1 <= every <= 64) with a pair of them that take the start and end times of that dispatch on
 * the context's stream (hipExtLaunchKernel), up to max_launches launches (later launches are not recorded).  A
 * recorded launch leaves the device idle for several microseconds around it, so every > 1 samples a run with
 * less of that cost; every prime to the four finest sweeps of a V(2,2) cycle samples all four of them in turn.
 * gp_probe_stop waits for the last
 * recorded event, writes the average device time of the recorded launches in microseconds (0 if none) and
 * their number, and destroys the events.  A second gp_probe_start discards the pairs of the first.  GP_EHIP
 * if the events fail. */
gp_status gp_probe_start(gp_ctx *ctx, int max_launches, int every);
gp_status gp_probe_stop(gp_ctx *ctx, double *avg_us, int *launches);

/* ---- transposed system (the adjoint of the augmented system of Sect. 3.3, eq. (spaceprobaug)) ----
 * Vectors are full unknown vectors of the finest level, n = 3*W*W + 1 doubles: the u, v and p grids (W*W each,
 * same layout as gp_set_x) and then xi, or, for right-hand sides, the rows of the same points and then the
 * mean-pressure row.  Host arrays when on_device = 0, device arrays on the context's device otherwise; the
 * caller owns them, the library copies in and out.  The matrix is the one of the current geometry and alpha.
 *
 * gp_apply_mt: y = M^T lam.
 * gp_adjoint_solve: solves M^T lam = g by lam <- lam + B'^T (g - M^T lam), where B'^T is the exact transpose of
 *   one FP64 cycle (the transposed cycle: every step of the cycle transposed, in reverse order), until
 *   ||g - M^T lam||_inf <= tol * max(1, ||g||_inf) or max_cycles (GP_ENOCONV, lam still written).  Entries of g
 *   at points that are not unknowns (extension and inactive points) are ignored.
 * gp_apply_cycle, gp_apply_cycle_t (test hooks for the transposition): x = B' b, one FP64 cycle from x = 0 with
 *   the mean-row shift (this overwrites the context's current x and b), and bbar = B'^T xbar. */
gp_status gp_apply_mt(gp_ctx *ctx, const double *lam, double *y, int on_device);
gp_status gp_adjoint_solve(gp_ctx *ctx, const double *g, double *lam, int on_device, double tol, int max_cycles,
                           gp_stats *st);
gp_status gp_apply_cycle(gp_ctx *ctx, const double *b, double *x, int on_device);
gp_status gp_apply_cycle_t(gp_ctx *ctx, const double *xbar, double *bbar, int on_device);

/* ---- reverse mode of a run of Crank-Nicolson steps (gradients of a function J of the final velocity) ----
 * gp_tape_forward runs nsteps FP64 steps of size dt from the current state (gp_set_state, geometry at t0 set),
 * the geometry of step n being the analytic shape at t0 + (n+1) dt under motion, with constant forcing fu, fv
 * (W*W grid arrays, NULL = 0) and the continuity right-hand side 0.  The body rows take the rigid boundary
 * velocity of motion plus ub_offset (host [2], NULL = 0): the body path is that of motion alone, so ub_offset is a
 * boundary-velocity parameter with the geometry held fixed.  The state before every checkpoint_every-th step is
 * kept on the device (about 11 W*W doubles each) and the context is left at the end of the run.
 * gp_tape_backward takes seed = dJ/du, dJ/dv at the end of the run (W*W grid arrays) and returns dJ/dfu, dJ/dfv
 * (W*W), dJ/d(ub_offset) (host [2]) and dJ/du, dJ/dv of the initial state (W*W; any output may be NULL).  It
 * replays each segment from its checkpoint and runs the adjoint of every step backwards: the transposed
 * convection Jacobian, extension fill and solve (gp_adjoint_solve with tol, max_cycles), and for the first two
 * steps the adjoint of the converged fixed-point iteration.  Arrays are host or device per on_device (dJdU always
 * host).  Errors: GP_EINVAL without a preceding gp_tape_forward on this context. */
gp_status gp_tape_forward(gp_ctx *ctx, const gp_shape *shape, const gp_rigid *motion, double t0, double dt, int nsteps,
                          const double *fu, const double *fv, int on_device, const double *ub_offset, double tol,
                          int max_cycles, double picard_eps, int picard_max, int checkpoint_every, gp_stats *st);
gp_status gp_tape_backward(gp_ctx *ctx, const double *seed_u, const double *seed_v, int on_device, double tol,
                           int max_cycles, double *dJdfu, double *dJdfv, double *dJdU, double *dJdu0, double *dJdv0,
                           gp_stats *st);

/* The part of dJ/dU that comes through the body path, for the last gp_tape_backward on this context.  The motion's
 * U moves the body, X(t) = X0 + U t, and with it the boundary points, the eq. (BCu) rows (Sect. 3.3) and the
 * boundary data u_b = U + omega x (B - X) of every step's geometry; with the discrete decisions of each geometry
 * held fixed (classes, ghost points, upwind stencils, the number of Alg. 1 march steps and its bisection branches)
 * these are smooth in X, and the reverse pass adds, per step n, t_{n+1} times the sum over the finest body ghost
 * rows of lam_G d(b_G - M_G x^{n+1})/dX.  The total dJ/dU of the motion's velocity is dJdU (gp_tape_backward: the
 * direct dependence of u_b on U, as for the offset) plus dJdU_path (host [2]).  *unmatched (may be NULL) counts
 * rows whose recorded Alg. 1 path did not reproduce the stored boundary point (0 when the derivative is complete).
 * Errors: GP_EINVAL without a taped run. */
gp_status gp_tape_path_gradient(gp_ctx *ctx, double *dJdU_path, int *unmatched);

#ifdef __cplusplus
}
#endif
#endif /* GPMG_H */
