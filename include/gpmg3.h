/*
 * gpmg3 -- the three-dimensional form of the solver of gpmg.h (MI355X, gfx950): the space problem of one
 * Crank-Nicolson step, eq. (spaceprobaug), on a 3-D staggered grid around a body given by a level set, carried to
 * three dimensions as the paper's outlook states it (Sect. 3, opening paragraph; Sect. 6): the ghost-point rows of
 * Sect. 3.3 with triquadratic interpolation on the 27-point upwind stencil (value for u, v, w; normal derivative
 * for p), a 7-unknown box per cell in the relaxation of Sect. 4.1 (colour (i + 2j + 3k) mod 7, no two boxes of one
 * colour reading each other's unknowns), fictitious-time ghost sweeps, the average-divergence unknown xi and the
 * mean-pressure row, and the multigrid of Sect. 4 (staggered restriction and trilinear prolongation, exact
 * coarsest solve), accelerated by GCR as in gpmg.h.
 *
 * Problem: on D = (-1,1)^3 with a body {phi > 0}, find (u, v, w, p, xi) with
 *     u - alpha lap u + grad p = f   (internal points of the three face grids)
 *     div u - xi = g                 (internal cell centres)
 *     (1/M_p) sum of the internal p = 0
 * ghost rows eq. (BCu) (triquadratic) at the body, Dirichlet rows for the normal velocity on the box walls and
 * ghost rows (3/8, 3/4, -1/8) for the tangential velocities beyond them.
 *
 * Layout: N cells per side (a power of two, >= 8), h = 2/N, W = N + 2.  Four grids of W^3 doubles (g = 0 u on
 * x-faces, 1 v on y-faces, 2 w on z-faces, 3 p at cell centres), point (i, j, k) in [-1, N]^3 of grid g at
 * g W^3 + ((k + 1) W + (j + 1)) W + (i + 1), located at x = -1 + (i + o_x) h with o = (0, 1/2, 1/2) for u,
 * (1/2, 0, 1/2) for v, (1/2, 1/2, 0) for w and (1/2, 1/2, 1/2) for p; the full unknown vector is the four grids and
 * then xi (4 W^3 + 1 doubles).  The level set lives on the half-step lattice ((2N + 1)^3 doubles,
 * [(kz (2N + 1) + ky)(2N + 1) + kx] at (-1 + kx h/2, -1 + ky h/2, -1 + kz h/2), positive inside the body).
 *
 * Ownership, streams and errors as in gpmg.h (statuses GP_*).  Host arrays unless on_device is set.
 */
#ifndef GPMG3_H
#define GPMG3_H

#include "gpmg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gp3_ctx gp3_ctx;

/* Defaults (gp3_default_params): V(2,2) cycles, lambda = 2 ghost sweeps, coarsest grid 4^3 cells solved exactly,
 * Alg. 1 march limit 8 and bisection to 0.01 h, fictitious time steps 0.9 (value rows) and 0.6 h (normal-derivative
 * rows: the 2-D value 0.9 h breaks the stability bound dtau c_G < 2 of eq. (ghostrelax) in 3-D, where c_G reaches
 * 2.6/h), cg_min = 0.1 on the coarse levels, krylov = 8 (GCR around the cycle; 0: the plain multigrid iteration). */
typedef struct {
  int nu1, nu2, gamma, lambda_ghost, coarsest_n, march_max, krylov;
  double dtau_dir, dtau_neu_over_h, bisect_eps_over_h, cg_min;
} gp3_params;

void gp3_default_params(gp3_params *prm);
/* the grid hierarchy of Sect. 4 for an N^3 cell grid (every buffer of every level allocated here) */
gp_status gp3_setup_grid(gp3_ctx **out, int N, const gp3_params *prm, void *hip_stream);
/* release every resource of the context (resource management) */
void gp3_destroy(gp3_ctx *ctx);
int gp3_num_levels(const gp3_ctx *ctx);
const char *gp3_last_hip_error(const gp3_ctx *ctx);

/* Geometry (Sect. 3.1 - 3.3 in 3-D) of every level: classification (internal iff phi < 0), ghost closure under the
 * 27-point stencils, Alg. 1 boundary points and the triquadratic rows (extrapolation rows where a row is undefined;
 * on the coarse levels also below cg_min), the wall rows; then the coarsest inverse (when alpha is set).
 * gp3_set_levelset_analytic samples on the device: kind 0 sphere R - |x - c|, kind 1 ellipsoid
 * 1 - sqrt(sum ((x - c)_d / A_d)^2), p = {R or A_x, A_y, A_z, c_x, c_y, c_z}.  GP_EGEOM if a finest ghost has no
 * usable row or an internal cell has no internal face. */
gp_status gp3_set_levelset(gp3_ctx *ctx, const double *phi, int on_device);
gp_status gp3_set_levelset_analytic(gp3_ctx *ctx, int kind, const double *p6);
/* alpha = dt / (2 Re) of eq. (spaceprobaug); refactors the coarsest system */
gp_status gp3_set_alpha(gp3_ctx *ctx, double alpha);
/* right-hand sides of the internal rows (W^3 each, any NULL = 0) and boundary data (values at B for u, v, w ghosts
 * and wall points, the normal derivative of p at B for pressure ghosts), full grid arrays */
gp_status gp3_set_rhs(gp3_ctx *ctx, const double *fu, const double *fv, const double *fw, const double *g, int on_device);
gp_status gp3_set_boundary_values(gp3_ctx *ctx, const double *bu, const double *bv, const double *bw, const double *bp,
                                  int on_device);
/* the full unknown vector (4 W^3 + 1 doubles) */
gp_status gp3_set_x(gp3_ctx *ctx, const double *x, int on_device);
gp_status gp3_get_x(gp3_ctx *ctx, double *x, int on_device);
/* inspection: classes (4 W_l^3 bytes) and per-point ghost rows of a level (B and theta 3 each, 27 weights, 27
 * columns, dtau per point; NaN / -1 where a point has no row) */
gp_status gp3_get_classes(gp3_ctx *ctx, int level, unsigned char *cls);
gp_status gp3_get_ghost_rows(gp3_ctx *ctx, int level, double *B, double *theta, double *w27, int *c27, double *dtau);
/* relaxation steps (box sweep in colour order, ghost sweeps, xi) on the finest level, from the current x as it is
 * (wall Dirichlet values included) */
gp_status gp3_relax(gp3_ctx *ctx, int steps);
/* one cycle from the current x and the mean projection; *res_inf the max-norm residual afterwards (may be NULL) */
gp_status gp3_cycle(gp3_ctx *ctx, double *res_inf);
/* solve to ||r||_inf <= tol max(1, ||b||_inf) (GCR with krylov > 0, as gp_solve); GP_ENOCONV / GP_EDIVERGED */
gp_status gp3_solve(gp3_ctx *ctx, double tol, int max_cycles, gp_stats *st);
/* residual of every row (4 W^3 + 1 doubles, the mean row last; may be NULL) and its max norm */
gp_status gp3_residual(gp3_ctx *ctx, double *r, double *res_inf);

#ifdef __cplusplus
}
#endif
#endif /* GPMG3_H */
