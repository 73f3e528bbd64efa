/*
 * gpmg oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the discrete problem and of the
 * multigrid iteration of Coco, "A multigrid ghost-point level-set method for
 * incompressible Navier-Stokes equations on moving domains with curved
 * boundaries" (arXiv:1911.00994).  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library; the product path (the
 * HIP library under paper_1911_00994_amd/csrc) shares no code with it.
 *
 * Everything is written from the paper:
 *   - time discretisation: Sect. 2, eqs. (NSCN1), (extrUdU), (NSitconv), (iterativeNS)
 *   - augmented space problem: eq. (spaceprobaug)
 *   - MAC central differences: Sect. 3.2; mid-point mean row eq. (eq:midpoint)
 *   - ghost points: Sect. 3.3, Alg. 1 (GtoB), eq. (BCu), Remark on delta
 *   - linear system: Alg. LS, eq. (eq:LS)
 *   - multigrid: Sect. 4 -- box relaxation (Sect. 4.1.1), fictitious-time ghost
 *     relaxation eqs. (fictBC),(ghostrelax), Alg. relax, restriction eqs.
 *     (restop),(restop5), bilinear interpolation (Sect. 4.3), cycles (Sect. 4.3)
 *   - moving domains: Sect. 3.4
 *   - level-set reinitialisation: Sect. 3.1, eq. (sdf) (or_reinit)
 * Readings of points the paper leaves open are listed in the design notes and
 * repeated at the place they are used.
 *
 * The system matrix is assembled literally as a CSR matrix (one row per grid
 * point of the three staggered grids plus the row of the extra scalar), and the
 * smoother takes its box blocks out of those rows and solves them with a generic
 * dense elimination.  Nothing here is tuned.
 *
 * Parity status: every function is pinned by the non-GPU tests (closed forms,
 * direct solves, manufactured solutions) except where noted "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* status codes (same numeric meaning as the public header of the library) */
#define OK 0
#define E_INVAL (-1)
#define E_NOMEM (-2)
#define E_GEOM (-4)
#define E_NOCONV (-5)
#define E_DIVERGED (-6)

/* point classes */
/* GHOSTX: ghost point whose boundary-condition row is not usable (see build_level_geometry); its row is a
 * quadratic extrapolation from the fluid side instead */
enum { C_INACTIVE = 0, C_INT = 1, C_GHOST = 2, C_WALLD = 3, C_WALLG = 4, C_EXT = 5, C_BODY = 6, C_GHOSTX = 7 };

#define MAXLEV 16

typedef struct {
  int N, W, n; /* cells per side, W = N+2, unknowns 3*W*W + 1 */
  double h;
  int lstride; /* level lattice step measured in fine lattice steps */
  unsigned char *cls; /* 3*W*W */
  /* ghost rows (classes GHOST and WALLG), one per point, canonical (grid, index) order */
  int ng;
  int *g_pt;      /* global unknown index of the ghost point */
  int *g_col;     /* 9 per row: global unknown indices */
  double *g_w;    /* 9 per row */
  double *g_dtau; /* per row */
  int *g_valid;   /* per row */
  double *g_B;    /* 2 per row: boundary point */
  double *g_nB;   /* 2 per row: unit normal at B (grid walls: outward wall normal) */
  double *g_theta;/* 2 per row */
  int *row_of;    /* 3*W*W -> ghost row id or -1 */
  /* extension points */
  int ne;
  int *e_pt, *e_src; /* e_src: 3 per point, -1 if no source found */
  double *e_w;
  int n_ext_fail;
  unsigned char *valued; /* 3*W*W: point carries a value (internal, ghost, wall, extension with sources) */
  int Mp; /* number of internal pressure points */
  double a, d; /* alpha/h^2 and 1 + 4a */
  /* CSR matrix of the level */
  int nnz;
  int *rp, *ci;
  double *va;
  /* vectors */
  double *x, *b, *r;
  /* coupled ghost boxes (see coupled_boxes): per box the cell, the unknowns (box unknowns first, then the
   * coupled ghosts) and which of them the box writes; boxes ordered by colour, then cell index */
  int nxb;
  int xb_coff[6];
  int *xb_cell, *xb_off, *xb_nbox, *xb_idx, *xb_of_cell;
  unsigned char *xb_wr;
  /* dense LU (coarsest level only) */
  double *lu;
  int *piv;
  int lu_ok;
} OLevel;

typedef struct {
  int N, L;
  OLevel lev[MAXLEV];
  double Re, alpha;
  /* parameters */
  int nu1, nu2, gamma, lambda, coarsest_n, march_max, nbis, ext_radius, colour_perm_seed, bnd_sweeps, bnd_radius;
  int ghost_boxes, lex_order, krylov, ghost_box_levels;
  double dtau_dir, dtau_neu_over_h, eps_over_h, cg_min;
  /* geometry / boundary data */
  double *phi; /* (2N+1)^2 fine half lattice */
  int have_geom;
  double motion[6]; /* X0x, X0y, Ux, Uy, omega, unused */
  double walls[8];  /* bottom u,v  right u,v  top u,v  left u,v */
  double t_geom;
  /* time stepping state (finest level layout, 3 grids of W*W) */
  int nstep;
  double *cu[3], *cv[3]; /* convection histories c^n, c^{n-1}, c^{n-2} (NaN where not computable) */
  double *lapu, *lapv;   /* Laplacian of the current state (NaN where not computable) */
  double *fbase;         /* scratch: u^n + alpha*lap u^n + dt f for u and v grids (2*W*W) */
  /* statistics */
  int last_cycles;
  double picard_res;
  double res_hist[1024];
} OSolver;

/* ------------------------------------------------------------------------- */
/* small helpers                                                             */
/* ------------------------------------------------------------------------- */

static int IX(int W, int i, int j) { return (j + 1) * W + (i + 1); }
static double sgn1(double z) { return z >= 0.0 ? 1.0 : -1.0; } /* SIGN(0) = 1 (Sect. 3.3) */

static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s); }
static void assemble_all(OSolver *S);

/* lattice sample of the level's half-step lattice (spacing h/2, 2N+1 points per axis) */
static double phi_lat(const OSolver *S, const OLevel *L, int kx, int ky) {
  int Lf = 2 * S->N + 1;
  return S->phi[(size_t)(ky * L->lstride) * Lf + (size_t)(kx * L->lstride)];
}

/* bilinear interpolant of phi on the 2x2 lattice cell containing (x,y) (Sect. 3.3):
 * value and gradient.  Cells are half-open; indices are clamped to the lattice. */
static void bilin(const OSolver *S, const OLevel *L, double x, double y, double *val, double *gx, double *gy) {
  double hl = 0.5 * L->h;
  int nl = 2 * L->N + 1;
  double fx = (x + 1.0) / hl, fy = (y + 1.0) / hl;
  int kx = (int)floor(fx), ky = (int)floor(fy);
  if (kx < 0) kx = 0;
  if (kx > nl - 2) kx = nl - 2;
  if (ky < 0) ky = 0;
  if (ky > nl - 2) ky = nl - 2;
  double tx = fx - kx, ty = fy - ky;
  double p00 = phi_lat(S, L, kx, ky), p10 = phi_lat(S, L, kx + 1, ky);
  double p01 = phi_lat(S, L, kx, ky + 1), p11 = phi_lat(S, L, kx + 1, ky + 1);
  if (val) *val = (1 - tx) * (1 - ty) * p00 + tx * (1 - ty) * p10 + (1 - tx) * ty * p01 + tx * ty * p11;
  if (gx) *gx = ((1 - ty) * (p10 - p00) + ty * (p11 - p01)) / hl;
  if (gy) *gy = ((1 - tx) * (p01 - p00) + tx * (p11 - p10)) / hl;
}

static void unit_normal(const OSolver *S, const OLevel *L, double x, double y, double *nx, double *ny) {
  double gx, gy;
  bilin(S, L, x, y, NULL, &gx, &gy);
  double m = sqrt(gx * gx + gy * gy);
  if (m > 0) {
    *nx = gx / m;
    *ny = gy / m;
  } else {
    *nx = 0;
    *ny = 0;
  }
}

/* coordinates and half-lattice index of the node (g,i,j) of a level */
static void node_xy(const OLevel *L, int g, int i, int j, double *x, double *y) {
  double h = L->h;
  if (g == 0) {
    *x = -1.0 + i * h;
    *y = -1.0 + (j + 0.5) * h;
  } else if (g == 1) {
    *x = -1.0 + (i + 0.5) * h;
    *y = -1.0 + j * h;
  } else {
    *x = -1.0 + (i + 0.5) * h;
    *y = -1.0 + (j + 0.5) * h;
  }
}
static void node_lat(int g, int i, int j, int *kx, int *ky) {
  if (g == 0) {
    *kx = 2 * i;
    *ky = 2 * j + 1;
  } else if (g == 1) {
    *kx = 2 * i + 1;
    *ky = 2 * j;
  } else {
    *kx = 2 * i + 1;
    *ky = 2 * j + 1;
  }
}

static int in_arr(const OLevel *L, int i, int j) { return i >= -1 && i <= L->N && j >= -1 && j <= L->N; }
static int gidx(const OLevel *L, int g, int i, int j) { return g * L->W * L->W + IX(L->W, i, j); }
static unsigned char cls_at(const OLevel *L, int g, int i, int j) {
  if (!in_arr(L, i, j)) return C_INACTIVE;
  return L->cls[gidx(L, g, i, j)];
}
static int valued_class(int c) { return c == C_INT || c == C_GHOST || c == C_WALLD || c == C_WALLG || c == C_GHOSTX; }
static int ghost_row_class(int c) { return c == C_GHOST || c == C_WALLG || c == C_GHOSTX; }

/* Lagrange basis of the three-point stencil at offsets 0, 1, 2 (eq. BCu) and its derivative */
static void Tq(double t, double T[3]) {
  T[0] = (1 - t) * (2 - t) / 2;
  T[1] = t * (2 - t);
  T[2] = t * (t - 1) / 2;
}
static void dTq(double t, double D[3]) {
  D[0] = t - 1.5;
  D[1] = 2 - 2 * t;
  D[2] = t - 0.5;
}

/* exported for the closed-form tests */
void or_st9_dirichlet(double thx, double thy, double *w9) {
  double Tx[3], Ty[3];
  Tq(thx, Tx);
  Tq(thy, Ty);
  for (int ky = 0; ky < 3; ky++)
    for (int kx = 0; kx < 3; kx++) w9[ky * 3 + kx] = Tx[kx] * Ty[ky];
}
void or_st9_neumann(double thx, double thy, double sx, double sy, double nx, double ny, double h, double *w9) {
  /* normal derivative of the biquadratic interpolant at B: theta = s (x_G - x)/h, so d/dx = -(s/h) d/dtheta */
  double Tx[3], Ty[3], Dx[3], Dy[3];
  Tq(thx, Tx);
  Tq(thy, Ty);
  dTq(thx, Dx);
  dTq(thy, Dy);
  for (int ky = 0; ky < 3; ky++)
    for (int kx = 0; kx < 3; kx++)
      w9[ky * 3 + kx] = -(nx * sx * Dx[kx] * Ty[ky] + ny * sy * Tx[kx] * Dy[ky]) / h;
}

/* ------------------------------------------------------------------------- */
/* level set (Sect. 3.1, eq. (eq:domains), rigid motion of Sect. 5)          */
/* ------------------------------------------------------------------------- */
/* shape kinds: 0 circle R - r, 1 circle R^2 - r^2, 2 ellipse 1 - (x'^2/A^2 + y'^2/B^2),
 * 3 ellipse 1 - sqrt(x'^2/A^2 + y'^2/B^2), 4 petals A + B cos(m (theta - theta0)) - r,
 * 5 no body (phi = -1).  sp = {A (or R), B, rotation angle or theta0, m}.
 * motion = {X0x, X0y, Ux, Uy, omega}: body frame point = R(-omega t)(x - X0 - U t). */
static double shape_phi(int kind, const double *sp, double xb, double yb) {
  if (kind == 0) return sp[0] - sqrt(xb * xb + yb * yb);
  if (kind == 1) return sp[0] * sp[0] - (xb * xb + yb * yb);
  if (kind == 2 || kind == 3) {
    double c = cos(sp[2]), s = sin(sp[2]);
    double xr = c * xb - s * yb, yr = s * xb + c * yb;
    double q = xr * xr / (sp[0] * sp[0]) + yr * yr / (sp[1] * sp[1]);
    return kind == 2 ? 1.0 - q : 1.0 - sqrt(q);
  }
  if (kind == 4) {
    double r = sqrt(xb * xb + yb * yb);
    if (r == 0.0) return sp[0] + sp[1];
    double th = atan2(yb, xb);
    return sp[0] + sp[1] * cos(sp[3] * (th - sp[2])) - r;
  }
  return -1.0;
}

int or_levelset_analytic(int kind, const double *sp, const double *motion, double t, int N, double *phi) {
  if (N < 2) return E_INVAL;
  int nl = 2 * N + 1;
  double hl = 1.0 / N; /* h/2 with h = 2/N */
  double X = motion[0] + motion[2] * t, Y = motion[1] + motion[3] * t, ang = motion[4] * t;
  double c = cos(ang), s = sin(ang);
  for (int ky = 0; ky < nl; ky++)
    for (int kx = 0; kx < nl; kx++) {
      double x = -1.0 + kx * hl - X, y = -1.0 + ky * hl - Y;
      /* rotate by -omega t */
      double xb = c * x + s * y, yb = -s * x + c * y;
      phi[(size_t)ky * nl + kx] = shape_phi(kind, sp, xb, yb);
    }
  return OK;
}

/* ------------------------------------------------------------------------- */
/* solver object                                                             */
/* ------------------------------------------------------------------------- */

static void free_level(OLevel *L) {
  free(L->cls);
  free(L->g_pt);
  free(L->g_col);
  free(L->g_w);
  free(L->g_dtau);
  free(L->g_valid);
  free(L->g_B);
  free(L->g_nB);
  free(L->g_theta);
  free(L->row_of);
  free(L->e_pt);
  free(L->e_src);
  free(L->e_w);
  free(L->valued);
  free(L->rp);
  free(L->ci);
  free(L->va);
  free(L->x);
  free(L->b);
  free(L->r);
  free(L->lu);
  free(L->piv);
  free(L->xb_cell);
  free(L->xb_off);
  free(L->xb_nbox);
  free(L->xb_idx);
  free(L->xb_wr);
  free(L->xb_of_cell);
  memset(L, 0, sizeof(*L));
}

/* iparams: nu1 nu2 gamma lambda coarsest_n march_max ext_radius colour_perm_seed bnd_sweeps bnd_radius
 *          ghost_boxes lex_order krylov ghost_box_levels
 * dparams: dtau_dir dtau_neu_over_h eps_over_h cg_min (coarse levels) */
void *or_create(int N, double Re, const int *ip, const double *dp) {
  if (N < 8 || (N & (N - 1))) return NULL;
  OSolver *S = (OSolver *)xcalloc(1, sizeof(OSolver));
  S->N = N;
  S->Re = Re;
  S->nu1 = ip[0];
  S->nu2 = ip[1];
  S->gamma = ip[2];
  S->lambda = ip[3];
  S->coarsest_n = ip[4];
  S->march_max = ip[5];
  S->ext_radius = ip[6];
  S->colour_perm_seed = ip[7];
  S->bnd_sweeps = ip[8];
  S->bnd_radius = ip[9];
  S->ghost_boxes = ip[10];
  S->lex_order = ip[11];
  S->krylov = ip[12];
  S->ghost_box_levels = ip[13];

  S->dtau_dir = dp[0];
  S->dtau_neu_over_h = dp[1];
  S->eps_over_h = dp[2];
  S->cg_min = dp[3];
  /* number of bisections: ceil(log2(dist(H,K)/eps)) with dist = h/2 (Alg. 1) */
  S->nbis = (int)ceil(log2(0.5 / S->eps_over_h) - 1e-12);
  if (S->coarsest_n < 4 || S->coarsest_n > N) {
    free(S);
    return NULL;
  }
  int L = 0;
  for (int n = N; n >= S->coarsest_n; n /= 2) {
    OLevel *lv = &S->lev[L];
    lv->N = n;
    lv->W = n + 2;
    lv->n = 3 * lv->W * lv->W + 1;
    lv->h = 2.0 / n;
    lv->lstride = N / n;
    lv->cls = (unsigned char *)xcalloc(3 * lv->W * lv->W, 1);
    lv->row_of = (int *)xcalloc(3 * lv->W * lv->W, sizeof(int));
    lv->valued = (unsigned char *)xcalloc(3 * lv->W * lv->W, 1);
    for (int q = 0; q < 3 * lv->W * lv->W; q++) lv->row_of[q] = -1;
    lv->x = (double *)xcalloc(lv->n, sizeof(double));
    lv->b = (double *)xcalloc(lv->n, sizeof(double));
    lv->r = (double *)xcalloc(lv->n, sizeof(double));
    L++;
    if (n == S->coarsest_n) break;
  }
  S->L = L;
  S->phi = (double *)xcalloc((size_t)(2 * N + 1) * (2 * N + 1), sizeof(double));
  int W = N + 2;
  for (int k = 0; k < 3; k++) {
    S->cu[k] = (double *)xcalloc(W * W, sizeof(double));
    S->cv[k] = (double *)xcalloc(W * W, sizeof(double));
  }
  S->lapu = (double *)xcalloc(W * W, sizeof(double));
  S->lapv = (double *)xcalloc(W * W, sizeof(double));
  S->fbase = (double *)xcalloc(2 * W * W, sizeof(double));
  S->alpha = 0.0;
  return S;
}

void or_destroy(void *h) {
  OSolver *S = (OSolver *)h;
  if (!S) return;
  for (int l = 0; l < S->L; l++) free_level(&S->lev[l]);
  free(S->phi);
  for (int k = 0; k < 3; k++) {
    free(S->cu[k]);
    free(S->cv[k]);
  }
  free(S->lapu);
  free(S->lapv);
  free(S->fbase);
  free(S);
}

int or_num_levels(void *h) { return ((OSolver *)h)->L; }

/* threads the library runs its parallel loops on (1 unless built with OpenMP) */
#ifdef _OPENMP
#include <omp.h>
int or_threads(void) { return omp_get_max_threads(); }
#else
int or_threads(void) { return 1; }
#endif

/* the coupled-box table of a level: counts, then (cell, slot offsets, number of box unknowns, unknown
 * indices, write flags, colour offsets) in the order the relaxation visits the boxes */
int or_coupled_box_count(void *h, int l, int *nbox, int *nslot) {
  OSolver *S = (OSolver *)h;
  if (l < 0 || l >= S->L) return E_INVAL;
  *nbox = S->lev[l].nxb;
  *nslot = S->lev[l].nxb ? S->lev[l].xb_off[S->lev[l].nxb] : 0;
  return OK;
}
int or_get_coupled_boxes(void *h, int l, int *cell, int *off, int *nbox, int *idx, unsigned char *wr, int *coff) {
  OSolver *S = (OSolver *)h;
  if (l < 0 || l >= S->L) return E_INVAL;
  OLevel *L = &S->lev[l];
  int ns = L->nxb ? L->xb_off[L->nxb] : 0;
  memcpy(cell, L->xb_cell, sizeof(int) * L->nxb);
  memcpy(off, L->xb_off, sizeof(int) * (L->nxb + 1));
  memcpy(nbox, L->xb_nbox, sizeof(int) * L->nxb);
  memcpy(idx, L->xb_idx, sizeof(int) * ns);
  memcpy(wr, L->xb_wr, ns);
  memcpy(coff, L->xb_coff, sizeof(int) * 6);
  return OK;
}
int or_level_n(void *h, int l) { return ((OSolver *)h)->lev[l].N; }

/* ------------------------------------------------------------------------- */
/* geometry: classification, ghost closure, Alg. 1, ghost rows, extension     */
/* ------------------------------------------------------------------------- */

/* Alg. 1 in two parts.  (i) From an external point, step by h/2 against the bilinear normal until the
 * interpolated level set is no longer positive: the last two points bracket the boundary.  Returns the
 * number of steps taken, or -1 if the bracket is not found within march_max steps. */
static int march_to_fluid(const OSolver *S, const OLevel *L, const double g[2], double phig, double out[2],
                          double in[2], double *phi_in) {
  double p[2] = {g[0], g[1]}, ph = phig;
  out[0] = g[0];
  out[1] = g[1];
  int steps = 0;
  for (; ph > 0; steps++) {
    if (steps == S->march_max) return -1;
    double n[2];
    out[0] = p[0];
    out[1] = p[1];
    unit_normal(S, L, p[0], p[1], &n[0], &n[1]);
    p[0] -= 0.5 * L->h * n[0];
    p[1] -= 0.5 * L->h * n[1];
    bilin(S, L, p[0], p[1], &ph, NULL, NULL);
  }
  in[0] = p[0];
  in[1] = p[1];
  *phi_in = ph;
  return steps;
}

/* (ii) Bisection of a bracketing segment for the zero of the interpolated level set: a fixed number of
 * halvings, each keeping the half whose ends still differ in sign (tested against the inner end); the
 * result is the last midpoint. */
static void bisect_segment(const OSolver *S, const OLevel *L, double in[2], double phi_in, double out[2], int iters,
                           double res[2]) {
  double mid[2] = {in[0], in[1]};
  for (int k = 0; k < iters; k++) {
    mid[0] = 0.5 * (in[0] + out[0]);
    mid[1] = 0.5 * (in[1] + out[1]);
    double pm;
    bilin(S, L, mid[0], mid[1], &pm, NULL, NULL);
    double *keep = (pm * phi_in < 0) ? out : in;
    keep[0] = mid[0];
    keep[1] = mid[1];
    if (keep == in) phi_in = pm;
  }
  res[0] = mid[0];
  res[1] = mid[1];
}

/* boundary point B of an external point G (Alg. 1).  A point on the boundary itself, or a march that lands
 * exactly on it, is its own boundary point.  Returns 1 on success. */
static int alg1(const OSolver *S, const OLevel *L, double xg, double yg, double phig, double *Bx, double *By) {
  double g[2] = {xg, yg}, out[2], in[2], phi_in = phig, B[2];
  int steps = march_to_fluid(S, L, g, phig, out, in, &phi_in);
  if (steps < 0) return 0;
  if (steps == 0 || phi_in == 0.0) {
    *Bx = steps == 0 ? xg : in[0];
    *By = steps == 0 ? yg : in[1];
    return 1;
  }
  bisect_segment(S, L, in, phi_in, out, S->nbis, B);
  *Bx = B[0];
  *By = B[1];
  return 1;
}

/* the upwind nine-point stencil of a point: sign of the bilinear normal at the point */
static void st9_signs(const OSolver *S, const OLevel *L, int g, int i, int j, double *sx, double *sy) {
  double x, y, nx, ny;
  node_xy(L, g, i, j, &x, &y);
  unit_normal(S, L, x, y, &nx, &ny);
  *sx = sgn1(nx);
  *sy = sgn1(ny);
}

static void mark_if_body(OLevel *L, int g, int i, int j, int *changed) {
  if (!in_arr(L, i, j)) return;
  int k = gidx(L, g, i, j);
  if (L->cls[k] == C_BODY) {
    L->cls[k] = C_GHOST;
    if (changed) *changed = 1;
  }
}

/* quadratic extrapolation sources for a point (g,i,j): along the grid axis closest to the bilinear normal
 * (the other axis as a second choice), towards the fluid, the first three consecutive points that are
 * internal or carry a boundary-condition ghost row; weights of the Lagrange extrapolation to offset 0
 * from offsets k0, k0+1, k0+2.  Returns 1 if found. */
static int extrap_sources(const OSolver *S, const OLevel *L, int g, int i, int j, int src[3], double w[3]) {
  double x, y, nx, ny;
  node_xy(L, g, i, j, &x, &y);
  unit_normal(S, L, x, y, &nx, &ny);
  int axes[2] = {fabs(nx) >= fabs(ny) ? 0 : 1, fabs(nx) >= fabs(ny) ? 1 : 0};
  for (int ai = 0; ai < 2; ai++) {
    int ax = axes[ai];
    int s = (int)sgn1(ax == 0 ? nx : ny);
    int di = ax == 0 ? -s : 0, dj = ax == 1 ? -s : 0;
    int k0 = 0;
    for (int q = 1; q <= 4; q++) {
      unsigned char c = cls_at(L, g, i + q * di, j + q * dj);
      if (c == C_INT || c == C_GHOST) {
        k0 = q;
        break;
      }
    }
    if (!k0) continue;
    int good = 1;
    for (int q = 0; q < 3; q++) {
      unsigned char c = cls_at(L, g, i + (k0 + q) * di, j + (k0 + q) * dj);
      if (!(c == C_INT || c == C_GHOST)) good = 0;
    }
    if (!good) continue;
    double kk = k0;
    w[0] = (kk + 1) * (kk + 2) / 2;
    w[1] = -kk * (kk + 2);
    w[2] = kk * (kk + 1) / 2;
    for (int q = 0; q < 3; q++) src[q] = gidx(L, g, i + (k0 + q) * di, j + (k0 + q) * dj);
    return 1;
  }
  return 0;
}


/* ------------------------------------------------------------------------- */
/* coupled ghost boxes                                                        */
/* ------------------------------------------------------------------------- */
/* The box of a cell (Sect. 4.1.1) holds its pressure and its four faces.  A ghost whose eq. (BCu) row (or
 * pressure normal-derivative row) has a weight on one of those internal unknowns ties the box to the
 * boundary condition: where that weight dominates the ghost's own diagonal, the ghost value is fixed by the
 * internal equations and the internal value by the ghost's row, and neither the box nor the fictitious-time
 * step of eq. (ghostrelax) alone can resolve the pair.  A coupled box therefore solves the cell's internal
 * unknowns together with every such ghost, from all their rows (a collective relaxation in the sense of
 * Sect. 4.1.1 extended across the boundary).  The table lists, per box, the box unknowns (west, east,
 * south, north face, pressure; internal ones only), then the coupled ghosts in increasing point order. */
static int cmp_long(const void *a, const void *b) {
  long x = *(const long *)a, y = *(const long *)b;
  return x < y ? -1 : x > y;
}
static int box_unknowns(const OLevel *L, int i, int j, int *U) {
  int cand[5] = {gidx(L, 0, i, j), gidx(L, 0, i + 1, j), gidx(L, 1, i, j), gidx(L, 1, i, j + 1), gidx(L, 2, i, j)};
  int m = 0;
  for (int q = 0; q < 5; q++)
    if (L->cls[cand[q]] == C_INT) U[m++] = cand[q];
  return m;
}
static void build_coupled_boxes(OLevel *L) {
  int N = L->N, W = L->W, WW = W * W;
  long P = 3L * WW;
  free(L->xb_cell);
  free(L->xb_off);
  free(L->xb_nbox);
  free(L->xb_idx);
  free(L->xb_wr);
  free(L->xb_of_cell);
  /* (cell, ghost) pairs: a ghost row's internal column belongs to the boxes of the cells it borders */
  long cap = 18L * (L->ng + 1), np = 0;
  long *pr = (long *)xcalloc(cap, sizeof(long));
  for (int r = 0; r < L->ng; r++) {
    int G = L->g_pt[r];
    if (L->cls[G] != C_GHOST) continue;
    for (int q = 0; q < 9; q++) {
      int c = L->g_col[9 * r + q];
      if (L->g_w[9 * r + q] == 0.0 || L->cls[c] != C_INT) continue;
      int g = c / WW, loc = c % WW, j = loc / W - 1, i = loc % W - 1;
      int cells[2][2], nc = 0;
      if (g == 0) {
        cells[0][0] = i - 1, cells[0][1] = j;
        cells[1][0] = i, cells[1][1] = j;
        nc = 2;
      } else if (g == 1) {
        cells[0][0] = i, cells[0][1] = j - 1;
        cells[1][0] = i, cells[1][1] = j;
        nc = 2;
      } else {
        cells[0][0] = i, cells[0][1] = j;
        nc = 1;
      }
      for (int z = 0; z < nc; z++) {
        int ci = cells[z][0], cj = cells[z][1];
        if (ci < 0 || cj < 0 || ci >= N || cj >= N) continue;
        int col = (ci + 2 * cj) % 5;
        /* key: colour, cell, ghost -- the order in which the boxes are visited */
        pr[np++] = ((long)col * N * N + (long)cj * N + ci) * P + G;
      }
    }
  }
  qsort(pr, np, sizeof(long), cmp_long);
  long nu = 0;
  for (long q = 0; q < np; q++)
    if (q == 0 || pr[q] != pr[q - 1]) pr[nu++] = pr[q];
  /* boxes */
  int nb = 0;
  for (long q = 0; q < nu; q++)
    if (q == 0 || pr[q] / P != pr[q - 1] / P) nb++;
  L->xb_cell = (int *)xcalloc(nb, sizeof(int));
  L->xb_off = (int *)xcalloc(nb + 1, sizeof(int));
  L->xb_nbox = (int *)xcalloc(nb, sizeof(int));
  L->xb_idx = (int *)xcalloc(nu + 5L * nb, sizeof(int));
  L->xb_wr = (unsigned char *)xcalloc(nu + 5L * nb, 1);
  int *seen = (int *)xcalloc(P, sizeof(int)); /* colour + 1 of the last box that writes the point */
  int b = 0, o = 0;
  for (int c = 0; c <= 5; c++) L->xb_coff[c] = 0;
  for (long q = 0; q < nu;) {
    long key = pr[q] / P;
    int col = (int)(key / ((long)N * N)), cell = (int)(key % ((long)N * N));
    int i = cell % N, j = cell / N;
    int U[5], m0 = box_unknowns(L, i, j, U);
    long q2 = q;
    while (q2 < nu && pr[q2] / P == key) q2++;
    if (m0 > 0) {
      L->xb_cell[b] = cell;
      L->xb_off[b] = o;
      L->xb_nbox[b] = m0;
      for (int a = 0; a < m0; a++) {
        L->xb_idx[o] = U[a];
        L->xb_wr[o++] = 1;
      }
      for (long z = q; z < q2; z++) {
        int G = (int)(pr[z] % P);
        L->xb_idx[o] = G;
        /* within one colour a ghost is written by the first box that holds it */
        L->xb_wr[o++] = (unsigned char)(seen[G] != col + 1);
        seen[G] = col + 1;
      }
      L->xb_coff[col + 1] = ++b;
    }
    q = q2;
  }
  for (int c = 1; c <= 5; c++)
    if (L->xb_coff[c] < L->xb_coff[c - 1]) L->xb_coff[c] = L->xb_coff[c - 1];
  L->xb_off[b] = o;
  L->nxb = b;
  L->xb_of_cell = (int *)xcalloc((size_t)N * N, sizeof(int));
  for (int q = 0; q < N * N; q++) L->xb_of_cell[q] = -1;
  for (int q = 0; q < b; q++) L->xb_of_cell[L->xb_cell[q]] = q;
  free(seen);
  free(pr);
}

static int build_level_geometry(OSolver *S, int l) {
  OLevel *L = &S->lev[l];
  int N = L->N, W = L->W;
  int wall_bad = 0;
  /* 1. classification per grid (Alg. LS: internal iff phi(P) < 0; each grid separately) */
  for (int g = 0; g < 3; g++)
    for (int j = -1; j <= N; j++)
      for (int i = -1; i <= N; i++) {
        unsigned char c = C_INACTIVE;
        int kx, ky;
        node_lat(g, i, j, &kx, &ky);
        if (g == 0) {
          if ((i == 0 || i == N) && j >= 0 && j <= N - 1)
            c = C_WALLD;
          else if ((j == -1 || j == N) && i >= 1 && i <= N - 1)
            c = C_WALLG;
          else if (i >= 1 && i <= N - 1 && j >= 0 && j <= N - 1)
            c = phi_lat(S, L, kx, ky) < 0 ? C_INT : C_BODY;
        } else if (g == 1) {
          if ((j == 0 || j == N) && i >= 0 && i <= N - 1)
            c = C_WALLD;
          else if ((i == -1 || i == N) && j >= 1 && j <= N - 1)
            c = C_WALLG;
          else if (i >= 0 && i <= N - 1 && j >= 1 && j <= N - 1)
            c = phi_lat(S, L, kx, ky) < 0 ? C_INT : C_BODY;
        } else {
          if (i >= 0 && i <= N - 1 && j >= 0 && j <= N - 1) c = phi_lat(S, L, kx, ky) < 0 ? C_INT : C_BODY;
        }
        if (l == 0 && c == C_WALLD && phi_lat(S, L, kx, ky) >= 0) wall_bad = 1; /* body touches the box */
        L->cls[gidx(L, g, i, j)] = c;
      }
  /* 2. ghost seeds: external points used by internal equations (Sect. 3.2, 3.3) */
  for (int j = 0; j <= N - 1; j++)
    for (int i = 0; i <= N; i++) {
      if (cls_at(L, 0, i, j) == C_INT) {
        mark_if_body(L, 0, i - 1, j, NULL);
        mark_if_body(L, 0, i + 1, j, NULL);
        mark_if_body(L, 0, i, j - 1, NULL);
        mark_if_body(L, 0, i, j + 1, NULL);
        mark_if_body(L, 2, i - 1, j, NULL);
        mark_if_body(L, 2, i, j, NULL);
      }
    }
  for (int j = 0; j <= N; j++)
    for (int i = 0; i <= N - 1; i++) {
      if (cls_at(L, 1, i, j) == C_INT) {
        mark_if_body(L, 1, i - 1, j, NULL);
        mark_if_body(L, 1, i + 1, j, NULL);
        mark_if_body(L, 1, i, j - 1, NULL);
        mark_if_body(L, 1, i, j + 1, NULL);
        mark_if_body(L, 2, i, j - 1, NULL);
        mark_if_body(L, 2, i, j, NULL);
      }
    }
  for (int j = 0; j <= N - 1; j++)
    for (int i = 0; i <= N - 1; i++) {
      if (cls_at(L, 2, i, j) == C_INT) {
        mark_if_body(L, 0, i, j, NULL);
        mark_if_body(L, 0, i + 1, j, NULL);
        mark_if_body(L, 1, i, j, NULL);
        mark_if_body(L, 1, i, j + 1, NULL);
      }
    }
  /* 3. closure: external points inside the nine-point stencil of a ghost are ghosts too */
  int changed = 1;
  while (changed) {
    changed = 0;
    for (int g = 0; g < 3; g++)
      for (int j = -1; j <= N; j++)
        for (int i = -1; i <= N; i++) {
          if (cls_at(L, g, i, j) != C_GHOST) continue;
          double sx, sy;
          st9_signs(S, L, g, i, j, &sx, &sy);
          for (int ky = 0; ky < 3; ky++)
            for (int kx = 0; kx < 3; kx++) mark_if_body(L, g, i - (int)sx * kx, j - (int)sy * ky, &changed);
        }
  }
  /* 4. extension points: external, not ghost, within ext_radius index steps of an internal point */
  int R = S->ext_radius;
  for (int g = 0; g < 3; g++)
    for (int j = -1; j <= N; j++)
      for (int i = -1; i <= N; i++) {
        if (cls_at(L, g, i, j) != C_BODY) continue;
        int near = 0;
        for (int dj = -R; dj <= R && !near; dj++)
          for (int di = -R; di <= R && !near; di++)
            if (cls_at(L, g, i + di, j + dj) == C_INT) near = 1;
        L->cls[gidx(L, g, i, j)] = near ? C_EXT : C_BODY;
      }
  for (int k = 0; k < 3 * W * W; k++)
    if (L->cls[k] == C_BODY) L->cls[k] = C_INACTIVE;
  /* 5. ghost rows in canonical (grid, index) order */
  free(L->g_pt);
  free(L->g_col);
  free(L->g_w);
  free(L->g_dtau);
  free(L->g_valid);
  free(L->g_B);
  free(L->g_nB);
  free(L->g_theta);
  int ng = 0;
  for (int k = 0; k < 3 * W * W; k++)
    if (L->cls[k] == C_GHOST || L->cls[k] == C_WALLG) ng++;
  L->ng = ng;
  L->g_pt = (int *)xcalloc(ng, sizeof(int));
  L->g_col = (int *)xcalloc(9 * ng, sizeof(int));
  L->g_w = (double *)xcalloc(9 * ng, sizeof(double));
  L->g_dtau = (double *)xcalloc(ng, sizeof(double));
  L->g_valid = (int *)xcalloc(ng, sizeof(int));
  L->g_B = (double *)xcalloc(2 * ng, sizeof(double));
  L->g_nB = (double *)xcalloc(2 * ng, sizeof(double));
  L->g_theta = (double *)xcalloc(2 * ng, sizeof(double));
  for (int k = 0; k < 3 * W * W; k++) L->row_of[k] = -1;
  int r = 0;
  int finest_bad = 0;
  for (int g = 0; g < 3; g++)
    for (int j = -1; j <= N; j++)
      for (int i = -1; i <= N; i++) {
        int k = gidx(L, g, i, j);
        unsigned char c = L->cls[k];
        if (c != C_GHOST && c != C_WALLG) continue;
        L->g_pt[r] = k;
        L->row_of[k] = r;
        int *col = &L->g_col[9 * r];
        double *w = &L->g_w[9 * r];
        for (int q = 0; q < 9; q++) {
          col[q] = k;
          w[q] = 0;
        }
        double xg, yg;
        node_xy(L, g, i, j, &xg, &yg);
        if (c == C_WALLG) {
          /* outer-wall tangential velocity: eq. (BCu) with the exact wall geometry,
           * theta_normal = 1/2, theta_tangential = 0 -> (3/8, 3/4, -1/8) */
          int di = 0, dj = 0;
          double Bx = xg, By = yg, nx = 0, ny = 0;
          if (g == 0) {
            dj = (j == -1) ? 1 : -1;
            By = (j == -1) ? -1.0 : 1.0;
            ny = (j == -1) ? -1.0 : 1.0;
          } else {
            di = (i == -1) ? 1 : -1;
            Bx = (i == -1) ? -1.0 : 1.0;
            nx = (i == -1) ? -1.0 : 1.0;
          }
          double T[3];
          Tq(0.5, T);
          for (int q = 0; q < 3; q++) {
            col[q] = gidx(L, g, i + q * di, j + q * dj);
            w[q] = T[q];
          }
          L->g_dtau[r] = S->dtau_dir;
          L->g_valid[r] = 1;
          for (int q = 1; q < 3; q++)
            if (L->cls[col[q]] != C_INT) L->g_valid[r] = 0;
          L->g_B[2 * r] = Bx;
          L->g_B[2 * r + 1] = By;
          L->g_nB[2 * r] = nx;
          L->g_nB[2 * r + 1] = ny;
          L->g_theta[2 * r] = (g == 0) ? 0.0 : 0.5;
          L->g_theta[2 * r + 1] = (g == 0) ? 0.5 : 0.0;
        } else {
          int kx, ky;
          node_lat(g, i, j, &kx, &ky);
          double phig = phi_lat(S, L, kx, ky);
          double sx, sy, Bx = xg, By = yg;
          st9_signs(S, L, g, i, j, &sx, &sy);
          int ok = alg1(S, L, xg, yg, phig, &Bx, &By);
          /* theta measured from G towards the fluid (the reading that makes the
           * stencil nodes 0,1,2 bracket B; see the design notes) */
          double thx = sx * (xg - Bx) / L->h, thy = sy * (yg - By) / L->h;
          double nbx, nby;
          unit_normal(S, L, Bx, By, &nbx, &nby);
          for (int ky2 = 0; ky2 < 3; ky2++)
            for (int kx2 = 0; kx2 < 3; kx2++) {
              int ii = i - (int)sx * kx2, jj = j - (int)sy * ky2;
              if (!in_arr(L, ii, jj)) {
                ok = 0;
                continue;
              }
              col[ky2 * 3 + kx2] = gidx(L, g, ii, jj);
              if (!valued_class(L->cls[col[ky2 * 3 + kx2]])) ok = 0;
            }
          if (g < 2) {
            or_st9_dirichlet(thx, thy, w);
            L->g_dtau[r] = S->dtau_dir;
          } else {
            or_st9_neumann(thx, thy, sx, sy, nbx, nby, L->h, w);
            L->g_dtau[r] = S->dtau_neu_over_h * L->h;
          }
          if (!(thx > -0.5 && thx < 1.0 && thy > -0.5 && thy < 1.0)) ok = 0;
          /* the diagonal of the row (weight of G itself, times h for the normal-derivative rows) must be
           * positive on the finest level, where the rows define the discrete problem.  The coarse levels
           * only carry the correction equations, and there a row whose diagonal is below cg_min is
           * replaced as well: a ghost barely determined by its own row slows the coarse relaxation */
          if (!((g < 2 ? w[0] : w[0] * L->h) > (l == 0 ? 0.0 : S->cg_min))) ok = 0;
          L->g_valid[r] = ok;
          L->g_B[2 * r] = Bx;
          L->g_B[2 * r + 1] = By;
          L->g_nB[2 * r] = nbx;
          L->g_nB[2 * r + 1] = nby;
          L->g_theta[2 * r] = thx;
          L->g_theta[2 * r + 1] = thy;
        }
        if (!L->g_valid[r]) L->cls[k] = C_GHOSTX;
        r++;
      }
  /* 5b. ghost points whose boundary-condition row is unusable (march failure, stencil out of the grid,
   * theta outside (-1/2, 1) or a non-positive diagonal) take a quadratic extrapolation row
   * x_G - sum w_q x_q = 0; if no sources exist the row is the identity x_G = 0 (coarse levels) or
   * the geometry is rejected (finest level) */
  for (int r2 = 0; r2 < ng; r2++) {
    int k = L->g_pt[r2];
    if (L->cls[k] != C_GHOSTX) continue;
    int *col = &L->g_col[9 * r2];
    double *w = &L->g_w[9 * r2];
    for (int q = 0; q < 9; q++) {
      col[q] = k;
      w[q] = 0;
    }
    w[0] = 1.0;
    L->g_dtau[r2] = 1.0;
    int g = k / (W * W), loc = k % (W * W), jj = loc / W - 1, ii = loc % W - 1;
    int src[3];
    double ew[3];
    if (extrap_sources(S, L, g, ii, jj, src, ew)) {
      for (int q = 0; q < 3; q++) {
        col[1 + q] = src[q];
        w[1 + q] = -ew[q];
      }
      L->g_valid[r2] = 2;
    } else {
      L->g_valid[r2] = 0;
      if (l == 0) finest_bad++;
    }
  }
  /* 6. extension sources: quadratic extrapolation along the grid axis closest to the normal,
   * from the first three internal/ghost points met towards the fluid */
  free(L->e_pt);
  free(L->e_src);
  free(L->e_w);
  int ne = 0;
  for (int k = 0; k < 3 * W * W; k++)
    if (L->cls[k] == C_EXT) ne++;
  L->ne = ne;
  L->e_pt = (int *)xcalloc(ne, sizeof(int));
  L->e_src = (int *)xcalloc(3 * ne, sizeof(int));
  L->e_w = (double *)xcalloc(3 * ne, sizeof(double));
  L->n_ext_fail = 0;
  int e = 0;
  for (int g = 0; g < 3; g++)
    for (int j = -1; j <= N; j++)
      for (int i = -1; i <= N; i++) {
        int k = gidx(L, g, i, j);
        if (L->cls[k] != C_EXT) continue;
        L->e_pt[e] = k;
        int found = extrap_sources(S, L, g, i, j, &L->e_src[3 * e], &L->e_w[3 * e]);
        if (!found) {
          /* no sources: the point carries no value */
          for (int q = 0; q < 3; q++) {
            L->e_src[3 * e + q] = -1;
            L->e_w[3 * e + q] = 0;
          }
          L->n_ext_fail++;
          L->cls[k] = C_INACTIVE;
        }
        e++;
      }
  for (int k = 0; k < 3 * W * W; k++) L->valued[k] = (unsigned char)(valued_class(L->cls[k]) || L->cls[k] == C_EXT);
  /* 7. internal pressure count for the mean row (eq. eq:midpoint) */
  L->Mp = 0;
  for (int k = 2 * W * W; k < 3 * W * W; k++)
    if (L->cls[k] == C_INT) L->Mp++;
  int empty_box = 0;
  /* every internal cell must have at least one internal face (else its box is empty of velocity) */
  for (int j = 0; j < N; j++)
    for (int i = 0; i < N; i++)
      if (cls_at(L, 2, i, j) == C_INT) {
        int nf = (cls_at(L, 0, i, j) == C_INT) + (cls_at(L, 0, i + 1, j) == C_INT) + (cls_at(L, 1, i, j) == C_INT) +
                 (cls_at(L, 1, i, j + 1) == C_INT);
        if (nf == 0 && l == 0) empty_box = 1;
      }
  build_coupled_boxes(L);
  if (L->Mp == 0 || wall_bad || finest_bad || empty_box) return E_GEOM;
  return OK;
}

/* boundary data of the finest level: rigid body velocity at B for velocity ghosts, zero normal
 * pressure derivative for pressure ghosts, wall velocities on the box */
static void default_boundary_values(OSolver *S) {
  OLevel *L = &S->lev[0];
  int N = L->N, W = L->W;
  double t = S->t_geom;
  double X = S->motion[0] + S->motion[2] * t, Y = S->motion[1] + S->motion[3] * t, om = S->motion[4];
  for (int r = 0; r < L->ng; r++) {
    int k = L->g_pt[r];
    int g = k / (W * W);
    double val = 0;
    if (L->cls[k] == C_GHOST) {
      double Bx = L->g_B[2 * r], By = L->g_B[2 * r + 1];
      if (g == 0) val = S->motion[2] - om * (By - Y);
      if (g == 1) val = S->motion[3] + om * (Bx - X);
    } else if (L->cls[k] == C_WALLG) { /* wall ghost: tangential wall velocity */
      int loc = k - g * W * W, jj = loc / W - 1, ii = loc % W - 1;
      if (g == 0) val = (jj == -1) ? S->walls[0] : S->walls[4];
      if (g == 1) val = (ii == -1) ? S->walls[7] : S->walls[3];
    }
    L->b[k] = val;
  }
  for (int g = 0; g < 2; g++)
    for (int j = -1; j <= N; j++)
      for (int i = -1; i <= N; i++) {
        int k = gidx(L, g, i, j);
        if (L->cls[k] != C_WALLD) continue;
        double val;
        if (g == 0)
          val = (i == 0) ? S->walls[6] : S->walls[2];
        else
          val = (j == 0) ? S->walls[1] : S->walls[5];
        L->b[k] = val;
        L->x[k] = val;
      }
}

static void invalidate_lu(OSolver *S) {
  for (int l = 0; l < S->L; l++) S->lev[l].lu_ok = 0;
}

int or_set_levelset(void *h, const double *phi, double t, const double *motion) {
  OSolver *S = (OSolver *)h;
  memcpy(S->phi, phi, sizeof(double) * (size_t)(2 * S->N + 1) * (2 * S->N + 1));
  if (motion)
    memcpy(S->motion, motion, 5 * sizeof(double));
  else
    memset(S->motion, 0, sizeof(S->motion));
  S->t_geom = t;
  int st = OK;
  for (int l = 0; l < S->L; l++) {
    int s = build_level_geometry(S, l);
    if (s != OK && st == OK) st = s;
  }
  if (st != OK) {
    S->have_geom = 0;
    return st;
  }
  S->have_geom = 1;
  /* points that carry no equation get a zero right-hand side */
  OLevel *L = &S->lev[0];
  for (int k = 0; k < 3 * L->W * L->W; k++)
    if (L->cls[k] == C_INACTIVE || L->cls[k] == C_EXT) L->b[k] = 0;
  default_boundary_values(S);
  if (S->alpha >= 0) assemble_all(S);
  invalidate_lu(S);
  return OK;
}

void or_set_walls(void *h, const double *w) {
  OSolver *S = (OSolver *)h;
  memcpy(S->walls, w, 8 * sizeof(double));
  if (S->have_geom) default_boundary_values(S);
}

/* boundary values as full grid arrays; entries at GHOST, WALLG and WALLD points are used */
void or_set_boundary_values(void *h, const double *bu, const double *bv, const double *bp) {
  OSolver *S = (OSolver *)h;
  OLevel *L = &S->lev[0];
  int WW = L->W * L->W;
  const double *src[3] = {bu, bv, bp};
  for (int g = 0; g < 3; g++) {
    if (!src[g]) continue;
    for (int q = 0; q < WW; q++) {
      unsigned char c = L->cls[g * WW + q];
      if (c == C_GHOST || c == C_WALLG || c == C_WALLD) {
        L->b[g * WW + q] = src[g][q];
        if (c == C_WALLD) L->x[g * WW + q] = src[g][q];
      }
    }
  }
}

int or_get_classes(void *h, int l, unsigned char *out) {
  OSolver *S = (OSolver *)h;
  if (l < 0 || l >= S->L) return E_INVAL;
  OLevel *L = &S->lev[l];
  memcpy(out, L->cls, 3 * L->W * L->W);
  return OK;
}

/* per-point dump of ghost rows: for each point of the 3 grids, B (2), nB (2), theta (2),
 * weights (9), column indices (9), dtau, valid; NaN / -1 at points without a ghost row */
int or_get_ghost_rows(void *h, int l, double *B, double *nB, double *th, double *w9, int *c9, double *dtau, int *valid) {
  OSolver *S = (OSolver *)h;
  if (l < 0 || l >= S->L) return E_INVAL;
  OLevel *L = &S->lev[l];
  int P = 3 * L->W * L->W;
  for (int k = 0; k < P; k++) {
    int r = L->row_of[k];
    for (int q = 0; q < 2; q++) {
      B[2 * k + q] = r >= 0 ? L->g_B[2 * r + q] : NAN;
      nB[2 * k + q] = r >= 0 ? L->g_nB[2 * r + q] : NAN;
      th[2 * k + q] = r >= 0 ? L->g_theta[2 * r + q] : NAN;
    }
    for (int q = 0; q < 9; q++) {
      w9[9 * k + q] = r >= 0 ? L->g_w[9 * r + q] : NAN;
      c9[9 * k + q] = r >= 0 ? L->g_col[9 * r + q] : -1;
    }
    dtau[k] = r >= 0 ? L->g_dtau[r] : NAN;
    valid[k] = r >= 0 ? L->g_valid[r] : -1;
  }
  return OK;
}

int or_get_ext_rows(void *h, int l, int *src3, double *w3, int *fail_count) {
  OSolver *S = (OSolver *)h;
  if (l < 0 || l >= S->L) return E_INVAL;
  OLevel *L = &S->lev[l];
  int P = 3 * L->W * L->W;
  for (int k = 0; k < 3 * P; k++) {
    src3[k] = -1;
    w3[k] = NAN;
  }
  for (int e = 0; e < L->ne; e++) {
    int k = L->e_pt[e];
    for (int q = 0; q < 3; q++) {
      src3[3 * k + q] = L->e_src[3 * e + q];
      w3[3 * k + q] = L->e_w[3 * e + q];
    }
  }
  *fail_count = L->n_ext_fail;
  return OK;
}

/* ------------------------------------------------------------------------- */
/* system assembly (Alg. LS, eq. eq:LS) as CSR                                */
/* ------------------------------------------------------------------------- */

static void set_level_coeffs(OSolver *S) {
  for (int l = 0; l < S->L; l++) {
    OLevel *L = &S->lev[l];
    L->a = S->alpha / (L->h * L->h);
    L->d = 1.0 + 4.0 * L->a;
  }
}

static void assemble(OSolver *S, int l) {
  OLevel *L = &S->lev[l];
  int W = L->W, WW = W * W, N = L->N;
  double h = L->h, a = L->a, d = L->d;
  int n = L->n;
  int cap = 10 * n + L->Mp + 16;
  free(L->rp);
  free(L->ci);
  free(L->va);
  L->rp = (int *)xcalloc(n + 1, sizeof(int));
  L->ci = (int *)xcalloc(cap, sizeof(int));
  L->va = (double *)xcalloc(cap, sizeof(double));
  int nz = 0;
  int xi = 3 * WW;
#define PUT(c, v)        \
  do {                   \
    L->ci[nz] = (c);     \
    L->va[nz] = (v);     \
    nz++;                \
  } while (0)
  for (int row = 0; row < n; row++) {
    L->rp[row] = nz;
    if (row == xi) { /* mean-pressure row: (1/Mp) sum over internal p = 0 */
      for (int k = 2 * WW; k < 3 * WW; k++)
        if (L->cls[k] == C_INT) PUT(k, 1.0 / L->Mp);
      continue;
    }
    int g = row / WW, loc = row % WW, j = loc / W - 1, i = loc % W - 1;
    unsigned char c = L->cls[row];
    if (c == C_INT) {
      if (g == 0) { /* u - alpha lap u + dp/dx = f^u on the horizontally staggered grid */
        PUT(row, d);
        PUT(gidx(L, 0, i - 1, j), -a);
        PUT(gidx(L, 0, i + 1, j), -a);
        PUT(gidx(L, 0, i, j - 1), -a);
        PUT(gidx(L, 0, i, j + 1), -a);
        PUT(gidx(L, 2, i, j), 1.0 / h);
        PUT(gidx(L, 2, i - 1, j), -1.0 / h);
      } else if (g == 1) {
        PUT(row, d);
        PUT(gidx(L, 1, i - 1, j), -a);
        PUT(gidx(L, 1, i + 1, j), -a);
        PUT(gidx(L, 1, i, j - 1), -a);
        PUT(gidx(L, 1, i, j + 1), -a);
        PUT(gidx(L, 2, i, j), 1.0 / h);
        PUT(gidx(L, 2, i, j - 1), -1.0 / h);
      } else { /* div u - xi = g on the central grid */
        PUT(gidx(L, 0, i + 1, j), 1.0 / h);
        PUT(gidx(L, 0, i, j), -1.0 / h);
        PUT(gidx(L, 1, i, j + 1), 1.0 / h);
        PUT(gidx(L, 1, i, j), -1.0 / h);
        PUT(xi, -1.0);
      }
    } else if (ghost_row_class(c)) {
      int r = L->row_of[row];
      for (int q = 0; q < 9; q++)
        if (L->g_w[9 * r + q] != 0.0) PUT(L->g_col[9 * r + q], L->g_w[9 * r + q]);
    } else {
      PUT(row, 1.0); /* wall Dirichlet, extension and inactive points: identity rows */
    }
    (void)N;
  }
  L->rp[n] = nz;
  L->nnz = nz;
#undef PUT
}

static void assemble_all(OSolver *S) {
  set_level_coeffs(S);
  for (int l = 0; l < S->L; l++) assemble(S, l);
}

int or_set_alpha(void *h, double alpha) {
  OSolver *S = (OSolver *)h;
  S->alpha = alpha;
  if (!S->have_geom) return E_INVAL;
  assemble_all(S);
  invalidate_lu(S);
  return OK;
}

int or_get_csr_size(void *h, int l, int *n, int *nnz) {
  OSolver *S = (OSolver *)h;
  if (l < 0 || l >= S->L) return E_INVAL;
  *n = S->lev[l].n;
  *nnz = S->lev[l].nnz;
  return OK;
}
int or_get_csr(void *h, int l, int *rp, int *ci, double *va, double *b) {
  OSolver *S = (OSolver *)h;
  OLevel *L = &S->lev[l];
  memcpy(rp, L->rp, sizeof(int) * (L->n + 1));
  memcpy(ci, L->ci, sizeof(int) * L->nnz);
  memcpy(va, L->va, sizeof(double) * L->nnz);
  if (b) memcpy(b, L->b, sizeof(double) * L->n);
  return OK;
}

/* ------------------------------------------------------------------------- */
/* linear algebra helpers                                                     */
/* ------------------------------------------------------------------------- */

static double row_dot(const OLevel *L, int row, const double *x) {
  double s = 0;
  for (int q = L->rp[row]; q < L->rp[row + 1]; q++) s += L->va[q] * x[L->ci[q]];
  return s;
}
static double row_coef(const OLevel *L, int row, int col) {
  for (int q = L->rp[row]; q < L->rp[row + 1]; q++)
    if (L->ci[q] == col) return L->va[q];
  return 0.0;
}

/* dense solve with partial pivoting (small blocks); returns 0 if singular */
static int dense_solve(int n, double *A, double *b) {
  for (int k = 0; k < n; k++) {
    int p = k;
    for (int i = k + 1; i < n; i++)
      if (fabs(A[i * n + k]) > fabs(A[p * n + k])) p = i;
    if (A[p * n + k] == 0.0) return 0;
    if (p != k) {
      for (int c = 0; c < n; c++) {
        double t = A[k * n + c];
        A[k * n + c] = A[p * n + c];
        A[p * n + c] = t;
      }
      double t = b[k];
      b[k] = b[p];
      b[p] = t;
    }
    for (int i = k + 1; i < n; i++) {
      double m = A[i * n + k] / A[k * n + k];
      for (int c = k; c < n; c++) A[i * n + c] -= m * A[k * n + c];
      b[i] -= m * b[k];
    }
  }
  for (int k = n - 1; k >= 0; k--) {
    double s = b[k];
    for (int c = k + 1; c < n; c++) s -= A[k * n + c] * b[c];
    b[k] = s / A[k * n + k];
  }
  return 1;
}

/* dense LU of the whole coarsest-level matrix (the exact "standard solver" of Sect. 4.3) */
static int coarse_factor(OLevel *L) {
  int n = L->n;
  free(L->lu);
  free(L->piv);
  L->lu = (double *)xcalloc((size_t)n * n, sizeof(double));
  L->piv = (int *)xcalloc(n, sizeof(int));
  double *A = L->lu;
  for (int r = 0; r < n; r++)
    for (int q = L->rp[r]; q < L->rp[r + 1]; q++) A[(size_t)r * n + L->ci[q]] += L->va[q];
  for (int k = 0; k < n; k++) {
    int p = k;
    for (int i = k + 1; i < n; i++)
      if (fabs(A[(size_t)i * n + k]) > fabs(A[(size_t)p * n + k])) p = i;
    L->piv[k] = p;
    if (A[(size_t)p * n + k] == 0.0) return 0;
    if (p != k)
      for (int c = 0; c < n; c++) {
        double t = A[(size_t)k * n + c];
        A[(size_t)k * n + c] = A[(size_t)p * n + c];
        A[(size_t)p * n + c] = t;
      }
    for (int i = k + 1; i < n; i++) {
      double m = A[(size_t)i * n + k] / A[(size_t)k * n + k];
      A[(size_t)i * n + k] = m;
      if (m != 0.0)
        for (int c = k + 1; c < n; c++) A[(size_t)i * n + c] -= m * A[(size_t)k * n + c];
    }
  }
  L->lu_ok = 1;
  return 1;
}
static void coarse_solve(OLevel *L, const double *b, double *x) {
  int n = L->n;
  const double *A = L->lu;
  for (int i = 0; i < n; i++) x[i] = b[i];
  for (int k = 0; k < n; k++) {
    int p = L->piv[k];
    if (p != k) {
      double t = x[k];
      x[k] = x[p];
      x[p] = t;
    }
  }
  for (int i = 0; i < n; i++) {
    double s = x[i];
    for (int c = 0; c < i; c++) s -= A[(size_t)i * n + c] * x[c];
    x[i] = s;
  }
  for (int i = n - 1; i >= 0; i--) {
    double s = x[i];
    for (int c = i + 1; c < n; c++) s -= A[(size_t)i * n + c] * x[c];
    x[i] = s / A[(size_t)i * n + i];
  }
}

/* ------------------------------------------------------------------------- */
/* multigrid components (Sect. 4)                                             */
/* ------------------------------------------------------------------------- */

/* box relaxation of the cell (i,j) (Sect. 4.1.1): the internal unknowns among p_ij and its four
 * faces are solved together from their own rows, everything else held at its current value */
static void box_relax(OLevel *L, int i, int j) {
  int cand[5] = {gidx(L, 0, i, j), gidx(L, 0, i + 1, j), gidx(L, 1, i, j), gidx(L, 1, i, j + 1), gidx(L, 2, i, j)};
  int U[5], m = 0;
  for (int q = 0; q < 5; q++)
    if (L->cls[cand[q]] == C_INT) U[m++] = cand[q];
  if (!m) return;
  double A[25], rhs[5];
  for (int a = 0; a < m; a++) {
    double s = L->b[U[a]] - row_dot(L, U[a], L->x);
    for (int c = 0; c < m; c++) {
      A[a * m + c] = row_coef(L, U[a], U[c]);
      s += A[a * m + c] * L->x[U[c]];
    }
    rhs[a] = s;
  }
  if (!dense_solve(m, A, rhs)) return;
  for (int a = 0; a < m; a++) L->x[U[a]] = rhs[a];
}

/* cells touching the body: one of the five box unknowns is neither internal nor a wall point */
static int cut_cell(const OLevel *L, int i, int j) {
  int cand[5] = {gidx(L, 0, i, j), gidx(L, 0, i + 1, j), gidx(L, 1, i, j), gidx(L, 1, i, j + 1), gidx(L, 2, i, j)};
  for (int q = 0; q < 5; q++) {
    unsigned char c = L->cls[cand[q]];
    if (c != C_INT && c != C_WALLD) return 1;
  }
  return 0;
}
static int in_band(const OLevel *L, int i, int j, int R) {
  for (int dj = -R; dj <= R; dj++)
    for (int di = -R; di <= R; di++) {
      int a = i + di, b = j + dj;
      if (a < 0 || b < 0 || a >= L->N || b >= L->N) continue;
      if (cut_cell(L, a, b)) return 1;
    }
  return 0;
}
static void ghost_sweeps(OSolver *S, OLevel *L) {
  double *nv = (double *)calloc(L->ng ? L->ng : 1, sizeof(double));
  for (int it = 0; it < S->lambda; it++) {
#pragma omp parallel for schedule(static)
    for (int r = 0; r < L->ng; r++) {
      int k = L->g_pt[r];
      nv[r] = L->x[k] + L->g_dtau[r] * (L->b[k] - row_dot(L, k, L->x));
    }
    for (int r = 0; r < L->ng; r++) L->x[L->g_pt[r]] = nv[r];
  }
  free(nv);
}

static uint64_t lcg_next(uint64_t *s) {
  *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
  return *s >> 33;
}

/* solve one coupled box from the values xs: rows and columns are the box's unknowns; every other value is
 * held at xs.  Returns 0 (and leaves sol untouched) if the block is singular. */
static int coupled_solve(const OLevel *L, int bx, const double *xs, double *sol) {
  int o = L->xb_off[bx], m = L->xb_off[bx + 1] - o;
  const int *U = &L->xb_idx[o];
  double *A = (double *)xcalloc((size_t)m * m, sizeof(double)), *rhs = (double *)xcalloc(m, sizeof(double));
  for (int a = 0; a < m; a++) {
    double t = L->b[U[a]] - row_dot(L, U[a], xs);
    for (int c = 0; c < m; c++) {
      A[a * m + c] = row_coef(L, U[a], U[c]);
      t += A[a * m + c] * xs[U[c]];
    }
    rhs[a] = t;
  }
  int ok = dense_solve(m, A, rhs);
  if (ok)
    for (int a = 0; a < m; a++) sol[a] = rhs[a];
  free(A);
  free(rhs);
  return ok;
}

/* the coupled boxes of a level, colour by colour: every box of a colour is solved from the values at the
 * start of that colour's pass (the boxes of one colour share no box unknown, but a ghost row of one box
 * may read another's unknowns); then each box writes its box unknowns and the ghosts it owns */
static void coupled_boxes(OLevel *L) {
  double *xs = (double *)xcalloc(L->n, sizeof(double));
  double *sol = (double *)xcalloc(L->xb_off[L->nxb] + 1, sizeof(double));
  int *ok = (int *)xcalloc(L->nxb + 1, sizeof(int));
  for (int c = 0; c < 5; c++) {
    int lo = L->xb_coff[c], hi = L->xb_coff[c + 1];
    if (hi == lo) continue;
    memcpy(xs, L->x, sizeof(double) * L->n);
#pragma omp parallel for schedule(dynamic, 16)
    for (int bx = lo; bx < hi; bx++) ok[bx] = coupled_solve(L, bx, xs, &sol[L->xb_off[bx]]);
    for (int bx = lo; bx < hi; bx++) {
      if (!ok[bx]) continue;
      for (int q = L->xb_off[bx]; q < L->xb_off[bx + 1]; q++)
        if (L->xb_wr[q]) L->x[L->xb_idx[q]] = sol[q];
    }
  }
  free(xs);
  free(sol);
  free(ok);
}


/* one relaxation step (Alg. relax with nu = 1).
 * Default order: box sweep in the colour order (i + 2j) mod 5 = 0..4, then the coupled boxes colour by
 * colour (ghost_boxes, on the ghost_box_levels finest levels), then lambda simultaneous ghost sweeps
 * (eq. ghostrelax).
 * Lexicographic order (the paper's GS-LEX): one pass over the cells row by row, each cell relaxed by its
 * coupled box if it has one (ghost_boxes) and by its plain box otherwise, each box seeing every earlier
 * update; then the ghost sweeps.
 * Optionally bnd_sweeps extra box sweeps restricted to the cells within bnd_radius cells of a cell touching
 * the body, each followed by lambda ghost sweeps (not part of the paper's Alg. relax; off by default).
 * Finally the average-divergence unknown xi is set so that the continuity residuals sum to zero. */
static void relax_step(OSolver *S, int l) {
  OLevel *L = &S->lev[l];
  int N = L->N, WW = L->W * L->W;
  if (S->lex_order) {
    double *sol = (double *)xcalloc(L->xb_off[L->nxb] + 1, sizeof(double));
    for (int j = 0; j < N; j++)
      for (int i = 0; i < N; i++) {
        int bx = (S->ghost_boxes && l < S->ghost_box_levels) ? L->xb_of_cell[j * N + i] : -1;
        if (bx < 0) {
          box_relax(L, i, j);
          continue;
        }
        if (coupled_solve(L, bx, L->x, sol))
          for (int q = L->xb_off[bx], a = 0; q < L->xb_off[bx + 1]; q++, a++) L->x[L->xb_idx[q]] = sol[a];
      }
    free(sol);
  } else {
    for (int col = 0; col < 5; col++) {
      if (S->colour_perm_seed == 0) {
        /* the boxes of one colour are independent (none reads what another writes), so the rows of cells may
         * run on several threads (built with OpenMP only for the CPU timing) with identical results */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < N; j++)
          for (int i = 0; i < N; i++)
            if ((i + 2 * j) % 5 == col) box_relax(L, i, j);
      } else { /* same colour, random order: must give an identical result */
        int cnt = 0;
        for (int j = 0; j < N; j++)
          for (int i = 0; i < N; i++)
            if ((i + 2 * j) % 5 == col) cnt++;
        int *list = (int *)xcalloc(cnt, sizeof(int));
        int c2 = 0;
        for (int j = 0; j < N; j++)
          for (int i = 0; i < N; i++)
            if ((i + 2 * j) % 5 == col) list[c2++] = j * N + i;
        uint64_t st = (uint64_t)S->colour_perm_seed * 7919u + (uint64_t)col;
        for (int q = cnt - 1; q > 0; q--) {
          int z = (int)(lcg_next(&st) % (uint64_t)(q + 1));
          int t = list[q];
          list[q] = list[z];
          list[z] = t;
        }
        for (int q = 0; q < cnt; q++) box_relax(L, list[q] % N, list[q] / N);
        free(list);
      }
    }
    if (S->ghost_boxes && l < S->ghost_box_levels) coupled_boxes(L);
  }
  ghost_sweeps(S, L);
  for (int q = 0; q < S->bnd_sweeps; q++) {
    for (int col = 0; col < 5; col++)
      for (int j = 0; j < N; j++)
        for (int i = 0; i < N; i++)
          if ((i + 2 * j) % 5 == col && in_band(L, i, j, S->bnd_radius)) box_relax(L, i, j);
    ghost_sweeps(S, L);
  }
  /* xi <- xi - mean(continuity residual) */
  double s = 0;
  for (int k = 2 * WW; k < 3 * WW; k++)
    if (L->cls[k] == C_INT) s += L->b[k] - row_dot(L, k, L->x);
  L->x[3 * WW] -= s / L->Mp;
}

int or_relax(void *h, int l, int steps) {
  OSolver *S = (OSolver *)h;
  if (l < 0 || l >= S->L) return E_INVAL;
  for (int q = 0; q < steps; q++) relax_step(S, l);
  return OK;
}

/* residual r = b - M x; rows without an equation get 0 */
static void residual(OLevel *L) {
#pragma omp parallel for schedule(static)
  for (int k = 0; k < L->n; k++) {
    unsigned char c = (k < 3 * L->W * L->W) ? L->cls[k] : C_INT;
    if (c == C_INT || ghost_row_class(c) || c == C_WALLD)
      L->r[k] = L->b[k] - row_dot(L, k, L->x);
    else
      L->r[k] = 0.0;
  }
}
static double norm_inf(const double *v, int n) {
  double m = 0;
  for (int k = 0; k < n; k++) {
    double a = fabs(v[k]);
    if (a > m || a != a) m = a;
  }
  return m;
}

/* boundary-aware restriction (eqs. restop, restop5): a coarse point of some class takes the standard
 * full weighting when all stencil points exist and have the same class, otherwise the plain average
 * over the stencil points of its class (0 if none) */
static void restrict_res(OSolver *S, int l) {
  OLevel *F = &S->lev[l], *C = &S->lev[l + 1];
  int WWc = C->W * C->W;
  for (int k = 0; k < C->n; k++) C->b[k] = 0;
  for (int g = 0; g < 3; g++)
#pragma omp parallel for schedule(static)
    for (int jc = -1; jc <= C->N; jc++)
      for (int ic = -1; ic <= C->N; ic++) {
        int kc = gidx(C, g, ic, jc);
        unsigned char cc = C->cls[kc];
        if (!(cc == C_INT || cc == C_GHOST || cc == C_WALLG)) continue;
        if (cc != C_INT && !C->g_valid[C->row_of[kc]]) continue;
        int fi[6], fj[6];
        double fw[6];
        int m = 0;
        if (g == 0) {
          for (int dy = 0; dy < 2; dy++)
            for (int dx = -1; dx <= 1; dx++) {
              fi[m] = 2 * ic + dx;
              fj[m] = 2 * jc + dy;
              fw[m] = (dx == 0 ? 2.0 : 1.0) / 8.0;
              m++;
            }
        } else if (g == 1) {
          for (int dy = -1; dy <= 1; dy++)
            for (int dx = 0; dx < 2; dx++) {
              fi[m] = 2 * ic + dx;
              fj[m] = 2 * jc + dy;
              fw[m] = (dy == 0 ? 2.0 : 1.0) / 8.0;
              m++;
            }
        } else {
          for (int dy = 0; dy < 2; dy++)
            for (int dx = 0; dx < 2; dx++) {
              fi[m] = 2 * ic + dx;
              fj[m] = 2 * jc + dy;
              fw[m] = 0.25;
              m++;
            }
        }
        int all = 1, cnt = 0;
        double sw = 0, sa = 0;
        for (int q = 0; q < m; q++) {
          if (!in_arr(F, fi[q], fj[q])) {
            all = 0;
            continue;
          }
          int kf = gidx(F, g, fi[q], fj[q]);
          if (F->cls[kf] == cc) {
            cnt++;
            sw += fw[q] * F->r[kf];
            sa += F->r[kf];
          } else
            all = 0;
        }
        C->b[kc] = all ? sw : (cnt ? sa / cnt : 0.0);
      }
  C->b[3 * WWc] = 0.0; /* coarse mean row */
}

static void ext_fill(OLevel *L, double *x) {
  for (int e = 0; e < L->ne; e++) {
    double v = 0;
    for (int q = 0; q < 3; q++)
      if (L->e_src[3 * e + q] >= 0) v += L->e_w[3 * e + q] * x[L->e_src[3 * e + q]];
    x[L->e_pt[e]] = v;
  }
}

/* bilinear prolongation of the coarse correction to the fine internal, ghost and wall-ghost points,
 * followed by x <- x + e (Sect. 4.3); coarse pressure outside the box is mirrored */
static void prolong_correct(OSolver *S, int l) {
  OLevel *F = &S->lev[l], *C = &S->lev[l + 1];
  int Nc = C->N;
  for (int g = 0; g < 3; g++)
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= F->N; j++)
      for (int i = -1; i <= F->N; i++) {
        int kf = gidx(F, g, i, j);
        unsigned char c = F->cls[kf];
        if (!(c == C_INT || ghost_row_class(c))) continue;
        int xi_[2], yi_[2];
        double xw[2], yw[2];
        int nx, ny;
        /* along a direction where the grid sits on cell faces (x for u, y for v) the fine index 2m
         * coincides with coarse m (weight 1) and odd indices take 1/2, 1/2; along a cell-centred
         * direction the fine index 2c lies at 1/4 of the way from coarse c to c-1 (3/4, 1/4) and 2c+1
         * at 1/4 of the way from c to c+1 */
        if (g == 0) {
          if ((i & 1) == 0) {
            xi_[0] = i / 2;
            xw[0] = 1;
            nx = 1;
          } else {
            xi_[0] = (i - 1) / 2;
            xi_[1] = (i + 1) / 2;
            xw[0] = xw[1] = 0.5;
            nx = 2;
          }
        } else {
          if ((i & 1) == 0) {
            xi_[0] = i / 2;
            xi_[1] = i / 2 - 1;
          } else {
            xi_[0] = (i - 1) / 2;
            xi_[1] = (i - 1) / 2 + 1;
          }
          xw[0] = 0.75;
          xw[1] = 0.25;
          nx = 2;
        }
        if (g == 1) {
          if ((j & 1) == 0) {
            yi_[0] = j / 2;
            yw[0] = 1;
            ny = 1;
          } else {
            yi_[0] = (j - 1) / 2;
            yi_[1] = (j + 1) / 2;
            yw[0] = yw[1] = 0.5;
            ny = 2;
          }
        } else {
          if ((j & 1) == 0) {
            yi_[0] = j / 2;
            yi_[1] = j / 2 - 1;
          } else {
            yi_[0] = (j - 1) / 2;
            yi_[1] = (j - 1) / 2 + 1;
          }
          yw[0] = 0.75;
          yw[1] = 0.25;
          ny = 2;
        }
        double e = 0;
        for (int a = 0; a < ny; a++)
          for (int b2 = 0; b2 < nx; b2++) {
            int ic = xi_[b2], jc = yi_[a];
            if (g == 2) { /* mirror outside the box */
              if (ic < 0) ic = 0;
              if (ic > Nc - 1) ic = Nc - 1;
              if (jc < 0) jc = 0;
              if (jc > Nc - 1) jc = Nc - 1;
            }
            if (!in_arr(C, ic, jc)) continue;
            e += xw[b2] * yw[a] * C->x[gidx(C, g, ic, jc)];
          }
        F->x[kf] += e;
      }
  F->x[3 * F->W * F->W] += C->x[3 * C->W * C->W];
}

static int ensure_coarse_lu(OSolver *S) {
  OLevel *C = &S->lev[S->L - 1];
  if (C->lu_ok) return 1;
  return coarse_factor(C);
}

static void mg_cycle(OSolver *S, int l) {
  OLevel *L = &S->lev[l];
  if (l == S->L - 1) {
    coarse_solve(L, L->b, L->x);
    return;
  }
  for (int q = 0; q < S->nu1; q++) relax_step(S, l);
  residual(L);
  restrict_res(S, l);
  OLevel *C = &S->lev[l + 1];
  memset(C->x, 0, sizeof(double) * C->n);
  int reps = (l + 1 == S->L - 1) ? 1 : S->gamma;
  for (int q = 0; q < reps; q++) mg_cycle(S, l + 1);
  ext_fill(C, C->x);
  prolong_correct(S, l);
  for (int q = 0; q < S->nu2; q++) relax_step(S, l);
}

/* finest level: p <- p - mean over internal points (row eq:midpoint); every other equation sees
 * only pressure differences, so the shift changes no other residual */
static void mean_project(OSolver *S) {
  OLevel *L = &S->lev[0];
  int WW = L->W * L->W;
  double s = 0;
  for (int k = 2 * WW; k < 3 * WW; k++)
    if (L->cls[k] == C_INT) s += L->x[k];
  double m = s / L->Mp;
  for (int k = 2 * WW; k < 3 * WW; k++)
    if (L->cls[k] == C_INT || L->cls[k] == C_GHOST || L->cls[k] == C_GHOSTX) L->x[k] -= m;
}

static double res_norm_finest(OSolver *S) {
  OLevel *L = &S->lev[0];
  residual(L);
  return norm_inf(L->r, L->n);
}

/* wall Dirichlet rows are identity rows u = u_b: solved exactly before iterating */
static void set_wall_dirichlet(OSolver *S) {
  OLevel *L = &S->lev[0];
  for (int k = 0; k < 3 * L->W * L->W; k++)
    if (L->cls[k] == C_WALLD) L->x[k] = L->b[k];
}

int or_cycle(void *h, double *res_inf) {
  OSolver *S = (OSolver *)h;
  if (!S->have_geom) return E_INVAL;
  if (!ensure_coarse_lu(S)) return E_GEOM;
  set_wall_dirichlet(S);
  mg_cycle(S, 0);
  mean_project(S);
  double r = res_norm_finest(S);
  if (res_inf) *res_inf = r;
  return (r != r) ? E_DIVERGED : OK;
}

/* y = M x over the rows that carry an equation (internal, ghost, wall and mean rows); 0 elsewhere */
static void matvec(OLevel *L, const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int k = 0; k < L->n; k++) {
    unsigned char c = (k < 3 * L->W * L->W) ? L->cls[k] : C_INT;
    y[k] = (c == C_INT || ghost_row_class(c) || c == C_WALLD) ? row_dot(L, k, x) : 0.0;
  }
}
static double dot(const double *a, const double *b, int n) {
  double s = 0;
  for (int k = 0; k < n; k++) s += a[k] * b[k];
  return s;
}

/* the cycle as a linear operator on a residual vector: one cycle from zero with right-hand side r, the mean
 * projection, then the pressure unknowns shifted by the mean-row entry of r (the cycle itself solves the other
 * rows and leaves the mean at zero; a constant pressure shift changes no other row).  z = 0 where no equation. */
static void precondition(OSolver *S, const double *r, double *z) {
  OLevel *L = &S->lev[0];
  int WW = L->W * L->W;
  double *sb = L->b, *sx = L->x;
  L->b = (double *)r;
  L->x = z;
  for (int k = 0; k < L->n; k++) z[k] = 0.0;
  set_wall_dirichlet(S);
  mg_cycle(S, 0);
  mean_project(S);
  for (int k = 2 * WW; k < 3 * WW; k++)
    if (L->cls[k] == C_INT || L->cls[k] == C_GHOST || L->cls[k] == C_GHOSTX) z[k] += r[3 * WW];
  for (int k = 0; k < 3 * WW; k++) {
    unsigned char c = L->cls[k];
    if (!(c == C_INT || ghost_row_class(c) || c == C_WALLD)) z[k] = 0.0;
  }
  L->b = sb;
  L->x = sx;
}

/* Solve M x = b to ||r||_inf <= tol max(1, ||b||_inf).
 * krylov = 0: repeated cycles x <- x + B'(b - M x) (the multigrid iteration of Sect. 4 on its own).
 * krylov = m > 0: the same cycle B' as the preconditioner of a generalized conjugate residual iteration (GCR,
 * restarted after m directions): z = B' r, q = M z, q and z orthogonalised against the stored q's (classical
 * Gram-Schmidt, one pass), normalised, x += (r.q) z, r -= (r.q) q.  The residual is updated recursively; when
 * it meets the tolerance the true residual is formed and the iteration restarts from it if it does not.
 * stats: cycles, res0, res, rho (last residual ratio). */
int or_solve(void *h, double tol, int max_cycles, double *stats) {
  OSolver *S = (OSolver *)h;
  if (!S->have_geom) return E_INVAL;
  if (!ensure_coarse_lu(S)) return E_GEOM;
  OLevel *L = &S->lev[0];
  set_wall_dirichlet(S);
  double r0 = res_norm_finest(S);
  double bn = norm_inf(L->b, L->n);
  double thr = tol * (bn > 1 ? bn : 1);
  double r = r0, rprev = r0;
  int c = 0;
  double rho = 0;
  int status = r0 == r0 ? OK : E_DIVERGED; /* NaN in the data */
  if (status != OK) max_cycles = 0;
  S->res_hist[0] = r0;
  if (S->krylov <= 0) {
    while (r > thr && c < max_cycles) {
      mg_cycle(S, 0);
      mean_project(S);
      rprev = r;
      r = res_norm_finest(S);
      c++;
      if (c < 1024) S->res_hist[c] = r;
      rho = r / rprev;
      if (r != r || r > 1e6 * (r0 > 1 ? r0 : 1)) {
        status = E_DIVERGED;
        break;
      }
    }
  } else {
    int n = L->n, m = S->krylov;
    double *rv = (double *)xcalloc(n, sizeof(double)), *zv = (double *)xcalloc(n, sizeof(double));
    double *qv = (double *)xcalloc(n, sizeof(double));
    double *Q = (double *)xcalloc((size_t)m * n, sizeof(double)), *Z = (double *)xcalloc((size_t)m * n, sizeof(double));
    double *beta = (double *)xcalloc(m, sizeof(double));
    memcpy(rv, L->r, sizeof(double) * n); /* true residual from res_norm_finest */
    int k = 0;
    while (r > thr && c < max_cycles) {
      precondition(S, rv, zv);
      matvec(L, zv, qv);
      for (int i = 0; i < k; i++) beta[i] = dot(&Q[(size_t)i * n], qv, n);
      for (int i = 0; i < k; i++)
        for (int e = 0; e < n; e++) {
          qv[e] -= beta[i] * Q[(size_t)i * n + e];
          zv[e] -= beta[i] * Z[(size_t)i * n + e];
        }
      double nu = sqrt(dot(qv, qv, n));
      c++;
      if (!(nu > 0)) { /* no new direction: the residual is already in the span (or the cycle broke down) */
        status = (nu == nu) ? E_NOCONV : E_DIVERGED;
        break;
      }
      for (int e = 0; e < n; e++) {
        qv[e] /= nu;
        zv[e] /= nu;
      }
      double a = dot(rv, qv, n);
      for (int e = 0; e < n; e++) {
        L->x[e] += a * zv[e];
        rv[e] -= a * qv[e];
      }
      memcpy(&Q[(size_t)k * n], qv, sizeof(double) * n);
      memcpy(&Z[(size_t)k * n], zv, sizeof(double) * n);
      k++;
      rprev = r;
      r = norm_inf(rv, n);
      if (r <= thr || k == m) { /* confirm with the true residual, or restart from it */
        r = res_norm_finest(S);
        memcpy(rv, L->r, sizeof(double) * n);
        k = 0;
      }
      if (c < 1024) S->res_hist[c] = r;
      rho = r / rprev;
      if (r != r || r > 1e6 * (r0 > 1 ? r0 : 1)) {
        status = E_DIVERGED;
        break;
      }
    }
    free(rv);
    free(zv);
    free(qv);
    free(Q);
    free(Z);
    free(beta);
  }
  S->last_cycles = c;
  if (stats) {
    stats[0] = c;
    stats[1] = r0;
    stats[2] = r;
    stats[3] = rho;
  }
  if (status != OK) return status;
  return r <= thr ? OK : E_NOCONV;
}

int or_res_history(void *h, double *out, int n) {
  OSolver *S = (OSolver *)h;
  int m = S->last_cycles + 1;
  if (m > n) m = n;
  if (m > 1024) m = 1024;
  memcpy(out, S->res_hist, m * sizeof(double));
  return m;
}

/* ------------------------------------------------------------------------- */
/* state / rhs access (finest level, three W x W grids + xi)                  */
/* ------------------------------------------------------------------------- */

void or_set_rhs(void *h, const double *fu, const double *fv, const double *g) {
  OSolver *S = (OSolver *)h;
  OLevel *L = &S->lev[0];
  int WW = L->W * L->W;
  const double *src[3] = {fu, fv, g};
  for (int gg = 0; gg < 3; gg++)
    for (int q = 0; q < WW; q++)
      if (L->cls[gg * WW + q] == C_INT) L->b[gg * WW + q] = src[gg] ? src[gg][q] : 0.0;
  L->b[3 * WW] = 0.0;
}

void or_set_x(void *h, const double *u, const double *v, const double *p, double xi) {
  OSolver *S = (OSolver *)h;
  OLevel *L = &S->lev[0];
  int WW = L->W * L->W;
  memcpy(L->x, u, WW * sizeof(double));
  memcpy(L->x + WW, v, WW * sizeof(double));
  memcpy(L->x + 2 * WW, p, WW * sizeof(double));
  L->x[3 * WW] = xi;
}
void or_get_x(void *h, double *u, double *v, double *p, double *xi) {
  OSolver *S = (OSolver *)h;
  OLevel *L = &S->lev[0];
  int WW = L->W * L->W;
  memcpy(u, L->x, WW * sizeof(double));
  memcpy(v, L->x + WW, WW * sizeof(double));
  memcpy(p, L->x + 2 * WW, WW * sizeof(double));
  *xi = L->x[3 * WW];
}
void or_get_b(void *h, double *b) {
  OSolver *S = (OSolver *)h;
  memcpy(b, S->lev[0].b, S->lev[0].n * sizeof(double));
}
int or_residual(void *h, double *r, double *res_inf) {
  OSolver *S = (OSolver *)h;
  OLevel *L = &S->lev[0];
  residual(L);
  if (r) memcpy(r, L->r, L->n * sizeof(double));
  if (res_inf) *res_inf = norm_inf(L->r, L->n);
  return OK;
}
void or_ext_fill_finest(void *h) {
  OSolver *S = (OSolver *)h;
  ext_fill(&S->lev[0], S->lev[0].x);
}
int or_ext_fail_count(void *h, int l) { return ((OSolver *)h)->lev[l].n_ext_fail; }

/* ------------------------------------------------------------------------- */
/* Crank-Nicolson step (Sect. 2, Sect. 3.4)                                   */
/* ------------------------------------------------------------------------- */

static int valued_pt(const OLevel *L, int g, int i, int j) {
  if (!in_arr(L, i, j)) return 0;
  return L->valued[gidx(L, g, i, j)];
}

/* convective term u.grad u with the central differences of Sect. 3.2, cross velocity averaged from the
 * four surrounding nodes of the other grid; Laplacian by the five-point formula.  NaN where a stencil
 * point carries no value in the current geometry. */
static void convection_and_laplacian(OSolver *S, double *cu, double *cv, double *lu, double *lv) {
  OLevel *L = &S->lev[0];
  int N = L->N, W = L->W, WW = W * W;
  double h = L->h;
  const double *u = L->x, *v = L->x + WW;
  unsigned char *val = (unsigned char *)xcalloc(3 * WW, 1);
  for (int g = 0; g < 2; g++)
    for (int j = -1; j <= N; j++)
      for (int i = -1; i <= N; i++) val[gidx(L, g, i, j)] = (unsigned char)valued_pt(L, g, i, j);
#define VU(i, j) (in_arr(L, i, j) && val[gidx(L, 0, i, j)])
#define VV(i, j) (in_arr(L, i, j) && val[gidx(L, 1, i, j)])
#define U(i, j) u[IX(W, i, j)]
#define V(i, j) v[IX(W, i, j)]
  for (int j = -1; j <= N; j++)
    for (int i = -1; i <= N; i++) {
      int k = IX(W, i, j);
      cu[k] = NAN;
      lu[k] = NAN;
      cv[k] = NAN;
      lv[k] = NAN;
      if (VU(i, j) && VU(i - 1, j) && VU(i + 1, j) && VU(i, j - 1) && VU(i, j + 1)) {
        lu[k] = (U(i - 1, j) + U(i + 1, j) + U(i, j - 1) + U(i, j + 1) - 4 * U(i, j)) / (h * h);
        if (VV(i - 1, j) && VV(i, j) && VV(i - 1, j + 1) && VV(i, j + 1)) {
          double vb = 0.25 * (V(i - 1, j) + V(i, j) + V(i - 1, j + 1) + V(i, j + 1));
          cu[k] = U(i, j) * (U(i + 1, j) - U(i - 1, j)) / (2 * h) + vb * (U(i, j + 1) - U(i, j - 1)) / (2 * h);
        }
      }
      if (VV(i, j) && VV(i - 1, j) && VV(i + 1, j) && VV(i, j - 1) && VV(i, j + 1)) {
        lv[k] = (V(i - 1, j) + V(i + 1, j) + V(i, j - 1) + V(i, j + 1) - 4 * V(i, j)) / (h * h);
        if (VU(i, j - 1) && VU(i + 1, j - 1) && VU(i, j) && VU(i + 1, j)) {
          double ub = 0.25 * (U(i, j - 1) + U(i + 1, j - 1) + U(i, j) + U(i + 1, j));
          cv[k] = ub * (V(i + 1, j) - V(i - 1, j)) / (2 * h) + V(i, j) * (V(i, j + 1) - V(i, j - 1)) / (2 * h);
        }
      }
    }
#undef VU
#undef VV
#undef U
#undef V
  free(val);
}

/* set the state at t^0 in the current geometry; computes c^0 and lap u^0 */
int or_set_state(void *h, const double *u, const double *v, const double *p, double xi) {
  OSolver *S = (OSolver *)h;
  if (!S->have_geom) return E_INVAL;
  or_set_x(h, u, v, p, xi);
  int WW = S->lev[0].W * S->lev[0].W;
  convection_and_laplacian(S, S->cu[0], S->cv[0], S->lapu, S->lapv);
  for (int q = 0; q < WW; q++) {
    S->cu[1][q] = S->cu[2][q] = NAN;
    S->cv[1][q] = S->cv[2][q] = NAN;
  }
  S->nstep = 0;
  return OK;
}

/* test hook: replace the convection histories c^n, c^{n-1}, c^{n-2} (u and v grids, finest layout) and the
 * step counter, so that the next step's treatment of the convection can be checked in closed form */
void or_set_conv_history(void *h, const double *cu0, const double *cv0, const double *cu1, const double *cv1,
                         const double *cu2, const double *cv2, int nstep) {
  OSolver *S = (OSolver *)h;
  int WW = S->lev[0].W * S->lev[0].W;
  const double *src[6] = {cu0, cv0, cu1, cv1, cu2, cv2};
  for (int k = 0; k < 3; k++) {
    memcpy(S->cu[k], src[2 * k], WW * sizeof(double));
    memcpy(S->cv[k], src[2 * k + 1], WW * sizeof(double));
  }
  S->nstep = nstep;
}

/* stats: [0] cycles total, [1] picard iterations, [2] final residual, [3] last rho */
int or_cn_step(void *h, double dt, const double *fu, const double *fv, const double *g, double tol, int max_cycles,
               double picard_eps, int picard_max, double *stats) {
  OSolver *S = (OSolver *)h;
  if (!S->have_geom) return E_INVAL;
  OLevel *L = &S->lev[0];
  int W = L->W, WW = W * W;
  double alpha = dt / (2.0 * S->Re);
  S->alpha = alpha;
  assemble_all(S);
  invalidate_lu(S);
  /* explicit part on the internal points of the new domain: u^n + alpha lap u^n + dt f^{n+1/2} */
  double *fb = S->fbase;
  const double *lap[2] = {S->lapu, S->lapv};
  const double *ff[2] = {fu, fv};
  int bad = 0;
  for (int gg = 0; gg < 2; gg++)
    for (int q = 0; q < WW; q++) {
      int k = gg * WW + q;
      fb[k] = 0;
      if (L->cls[k] != C_INT) continue;
      fb[k] = L->x[k] + alpha * lap[gg][q] + dt * (ff[gg] ? ff[gg][q] : 0.0);
      if (fb[k] != fb[k]) bad = 1;
    }
  if (bad) return E_GEOM;
  for (int q = 0; q < WW; q++)
    if (L->cls[2 * WW + q] == C_INT) L->b[2 * WW + q] = g ? g[q] : 0.0;
  L->b[3 * WW] = 0.0;
  double st[4] = {0, 0, 0, 0};
  int total_cycles = 0, status = OK, picard_its = 0;
  S->picard_res = 0;
  if (S->nstep >= 2) {
    /* convection extrapolated from the three previous levels (eq. extrUdU) */
    for (int gg = 0; gg < 2; gg++) {
      double **c = gg == 0 ? S->cu : S->cv;
      for (int q = 0; q < WW; q++) {
        int k = gg * WW + q;
        if (L->cls[k] != C_INT) continue;
        double C = c[0][q] + 0.5 * c[1][q] - 0.5 * c[2][q];
        if (C != C) return E_GEOM;
        L->b[k] = fb[k] - dt * C;
      }
    }
    status = or_solve(h, tol, max_cycles, st);
    total_cycles = (int)st[0];
  } else {
    /* mid-point convection with the fixed-point iteration of eq. (NSitconv); first iterate u^n */
    double *cnu = (double *)xcalloc(WW, sizeof(double)), *cnv = (double *)xcalloc(WW, sizeof(double));
    double *tlu = (double *)xcalloc(WW, sizeof(double)), *tlv = (double *)xcalloc(WW, sizeof(double));
    memcpy(cnu, S->cu[0], WW * sizeof(double));
    memcpy(cnv, S->cv[0], WW * sizeof(double));
    for (int gg = 0; gg < 2; gg++) { /* k = 0: c(u^{n+1,0}) = c(u^n) */
      const double *cn = gg == 0 ? cnu : cnv;
      for (int q = 0; q < WW; q++) {
        int k = gg * WW + q;
        if (L->cls[k] != C_INT) continue;
        if (cn[q] != cn[q]) {
          free(cnu);
          free(cnv);
          free(tlu);
          free(tlv);
          return E_GEOM;
        }
        L->b[k] = fb[k] - dt * cn[q];
      }
    }
    double fbn = 0;
    for (int k = 0; k < 2 * WW; k++)
      if (L->cls[k] == C_INT && fabs(fb[k]) > fbn) fbn = fabs(fb[k]);
    for (;;) {
      status = or_solve(h, tol, max_cycles, st);
      total_cycles += (int)st[0];
      picard_its++;
      if (status != OK && status != E_NOCONV) break;
      ext_fill(L, L->x);
      double *tmpcu = (double *)xcalloc(WW, sizeof(double)), *tmpcv = (double *)xcalloc(WW, sizeof(double));
      convection_and_laplacian(S, tmpcu, tmpcv, tlu, tlv);
      /* test of eq. (iterativeNS): momentum residual with the convection of the new iterate */
      double rn = 0;
      for (int gg = 0; gg < 2; gg++) {
        const double *cn = gg == 0 ? cnu : cnv, *ck = gg == 0 ? tmpcu : tmpcv;
        for (int q = 0; q < WW; q++) {
          int k = gg * WW + q;
          if (L->cls[k] != C_INT) continue;
          double C = 0.5 * (cn[q] + ck[q]);
          double rr = fb[k] - dt * C - row_dot(L, k, L->x);
          if (fabs(rr) > rn || rr != rr) rn = fabs(rr);
          L->b[k] = fb[k] - dt * C;
        }
      }
      free(tmpcu);
      free(tmpcv);
      double thr = picard_eps * (fbn > 1 ? fbn : 1);
      S->picard_res = rn;
      if (rn < thr || picard_its >= picard_max) break;
    }
    free(cnu);
    free(cnv);
    free(tlu);
    free(tlv);
  }
  /* finish the step: extension values, new convection / Laplacian, history shift */
  ext_fill(L, L->x);
  double *old2u = S->cu[2], *old2v = S->cv[2];
  S->cu[2] = S->cu[1];
  S->cv[2] = S->cv[1];
  S->cu[1] = S->cu[0];
  S->cv[1] = S->cv[0];
  S->cu[0] = old2u;
  S->cv[0] = old2v;
  convection_and_laplacian(S, S->cu[0], S->cv[0], S->lapu, S->lapv);
  S->nstep++;
  if (stats) {
    stats[0] = total_cycles;
    stats[1] = picard_its;
    stats[2] = st[2];
    stats[3] = st[3];
    stats[4] = S->picard_res;
  }
  return status;
}

/* ------------------------------------------------------------------------- */
/* hooks for the closed-form tests of the transfer operators                  */
/* ------------------------------------------------------------------------- */
/* restrict a fine-level residual vector (length of level l) to level l+1 */
int or_test_restrict(void *h, int l, const double *r_fine, double *b_coarse) {
  OSolver *S = (OSolver *)h;
  if (l < 0 || l + 1 >= S->L) return E_INVAL;
  OLevel *F = &S->lev[l], *C = &S->lev[l + 1];
  memcpy(F->r, r_fine, F->n * sizeof(double));
  restrict_res(S, l);
  memcpy(b_coarse, C->b, C->n * sizeof(double));
  return OK;
}
/* prolongate a coarse vector (level l+1) and add it to a fine vector (level l) */
int or_test_prolong(void *h, int l, const double *e_coarse, double *x_fine) {
  OSolver *S = (OSolver *)h;
  if (l < 0 || l + 1 >= S->L) return E_INVAL;
  OLevel *F = &S->lev[l], *C = &S->lev[l + 1];
  double *sx = (double *)xcalloc(F->n, sizeof(double)), *sc = (double *)xcalloc(C->n, sizeof(double));
  memcpy(sx, F->x, F->n * sizeof(double));
  memcpy(sc, C->x, C->n * sizeof(double));
  memcpy(F->x, x_fine, F->n * sizeof(double));
  memcpy(C->x, e_coarse, C->n * sizeof(double));
  prolong_correct(S, l);
  memcpy(x_fine, F->x, F->n * sizeof(double));
  memcpy(F->x, sx, F->n * sizeof(double));
  memcpy(C->x, sc, C->n * sizeof(double));
  free(sx);
  free(sc);
  return OK;
}

/* ------------------------------------------------------------------------- */
/* level-set reinitialisation, Sect. 3.1 eq. (sdf)                            */
/* ------------------------------------------------------------------------- */
/* Steady state of d(phi_d)/d(mu) = sgn(phi) (1 - |grad phi_d|), phi_d = phi at mu = 0, on an n x n lattice of
 * spacing dx (entry [ky * n + kx]).  The paper fixes the equation, not its discretisation; this reading:
 *   - explicit Euler steps in the fictitious time mu with dmu = cfl * dx, iters steps;
 *   - |grad phi_d| by the Godunov upwind approximation of first order: with the one-sided differences
 *     a = (phi_i - phi_{i-1})/dx, b = (phi_{i+1} - phi_i)/dx (c, d likewise in y), where sgn(phi) > 0 the
 *     x part is max(max(a, 0)^2, min(b, 0)^2), where sgn(phi) < 0 it is max(min(a, 0)^2, max(b, 0)^2);
 *     outside the lattice the nearest lattice value is repeated (zero one-sided difference);
 *   - at the points next to the interface (phi changes sign towards a lattice neighbour, or phi = 0) the
 *     distance estimate D = dx phi / |Delta phi| of the initial data replaces the upwind step, so that the
 *     interface stays where phi puts it: phi_d <- phi_d - (dmu / dx) (sgn(phi) |phi_d| - D), with |Delta phi|
 *     the length of the vector of the largest of the central and the two one-sided differences per axis
 *     (bounded below by 1e-300);
 *   - sgn(0) = 0 (a point on the interface does not move).
 * Pins: a linear level set of any slope becomes the exact signed distance; on a circle the result approaches
 * R - r at first order and the zero set does not move. */
static double rs_max3(double a, double b, double c) {
  double m = a > b ? a : b;
  return m > c ? m : c;
}
int or_reinit(const double *phi0, int n, double dx, int iters, double cfl, double *out) {
  if (n < 2 || !(dx > 0) || iters < 0 || !(cfl > 0)) return E_INVAL;
  size_t nn = (size_t)n * n;
  double *cur = (double *)xcalloc(nn, sizeof(double)), *nxt = (double *)xcalloc(nn, sizeof(double));
  double *Dest = (double *)xcalloc(nn, sizeof(double));
  signed char *sg = (signed char *)xcalloc(nn, 1);
  unsigned char *near = (unsigned char *)xcalloc(nn, 1);
#define P0(i, j) phi0[(size_t)(j) * n + (i)]
  for (int j = 0; j < n; j++)
    for (int i = 0; i < n; i++) {
      size_t k = (size_t)j * n + i;
      double p = P0(i, j);
      sg[k] = p > 0 ? 1 : (p < 0 ? -1 : 0);
      int im = i > 0 ? i - 1 : i, ip = i < n - 1 ? i + 1 : i, jm = j > 0 ? j - 1 : j, jp = j < n - 1 ? j + 1 : j;
      int cross = p == 0.0 || p * P0(im, j) < 0 || p * P0(ip, j) < 0 || p * P0(i, jm) < 0 || p * P0(i, jp) < 0;
      near[k] = (unsigned char)cross;
      if (cross) {
        double ex = rs_max3(fabs(P0(ip, j) - P0(im, j)) / 2, fabs(P0(ip, j) - p), fabs(p - P0(im, j)));
        double ey = rs_max3(fabs(P0(i, jp) - P0(i, jm)) / 2, fabs(P0(i, jp) - p), fabs(p - P0(i, jm)));
        double len = sqrt(ex * ex + ey * ey);
        if (len < 1e-300) len = 1e-300;
        Dest[k] = dx * p / len;
      }
      cur[k] = p;
    }
#undef P0
  const double dmu = cfl * dx;
  for (int it = 0; it < iters; it++) {
    for (int j = 0; j < n; j++)
      for (int i = 0; i < n; i++) {
        size_t k = (size_t)j * n + i;
        double p = cur[k];
        if (sg[k] == 0) {
          nxt[k] = p;
          continue;
        }
        if (near[k]) {
          nxt[k] = p - (dmu / dx) * (sg[k] * fabs(p) - Dest[k]);
          continue;
        }
        int im = i > 0 ? i - 1 : i, ip = i < n - 1 ? i + 1 : i, jm = j > 0 ? j - 1 : j, jp = j < n - 1 ? j + 1 : j;
        double a = (p - cur[(size_t)j * n + im]) / dx, b = (cur[(size_t)j * n + ip] - p) / dx;
        double c = (p - cur[(size_t)jm * n + i]) / dx, d = (cur[(size_t)jp * n + i] - p) / dx;
        double gx, gy;
        if (sg[k] > 0) {
          double a1 = a > 0 ? a : 0, b1 = b < 0 ? b : 0, c1 = c > 0 ? c : 0, d1 = d < 0 ? d : 0;
          gx = a1 * a1 > b1 * b1 ? a1 * a1 : b1 * b1;
          gy = c1 * c1 > d1 * d1 ? c1 * c1 : d1 * d1;
        } else {
          double a1 = a < 0 ? a : 0, b1 = b > 0 ? b : 0, c1 = c < 0 ? c : 0, d1 = d > 0 ? d : 0;
          gx = a1 * a1 > b1 * b1 ? a1 * a1 : b1 * b1;
          gy = c1 * c1 > d1 * d1 ? c1 * c1 : d1 * d1;
        }
        nxt[k] = p - dmu * sg[k] * (sqrt(gx + gy) - 1.0);
      }
    double *t = cur;
    cur = nxt;
    nxt = t;
  }
  memcpy(out, cur, nn * sizeof(double));
  free(cur);
  free(nxt);
  free(Dest);
  free(sg);
  free(near);
  return OK;
}
