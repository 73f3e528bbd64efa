/*
 * gpmg 3-D oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the three-dimensional extension of the method of Coco,
 * "A multigrid ghost-point level-set method for incompressible Navier-Stokes equations on moving domains with
 * curved boundaries" (arXiv:1911.00994): the space problem of one Crank-Nicolson step, eq. (spaceprobaug), on a
 * 3-D staggered grid around a body given by a level set, with the ghost-point boundary rows of Sect. 3.3 carried
 * to three dimensions as the paper's outlook states it (Sect. 3, opening paragraph; Sect. 6): triquadratic
 * interpolation on the 27-point upwind stencil, a 7-unknown box per cell in the relaxation of Sect. 4.1, and the
 * multigrid of Sect. 4.  Only the test suite may load this library; the HIP path shares no code with it.
 *
 * Grid: D = (-1, 1)^3, N cells per side, h = 2/N, W = N + 2; four staggered grids (g = 0 u on x-faces, 1 v on
 * y-faces, 2 w on z-faces, 3 p at cell centres), each W^3 points (i, j, k) in [-1, N]^3 at
 * x = -1 + (i + o_x) h with o = (0, 1/2, 1/2) for u, (1/2, 0, 1/2) for v, (1/2, 1/2, 0) for w, (1/2, 1/2, 1/2) for p.
 * Unknown vector: the four grids, then xi (4 W^3 + 1 entries); point (g, i, j, k) at
 * g W^3 + ((k + 1) W + (j + 1)) W + (i + 1).  The level set is sampled on the half-step lattice of the finest
 * grid ((2N + 1)^3 points, spacing h/2, positive inside the body); level l uses every 2^l-th lattice point.
 *
 * Rows (the 3-D restatement of Alg. LS):
 *   internal u: (1 + 6a) u - a (sum of the 6 neighbours) + (p_E - p_W)/h = f,  a = alpha/h^2 (v, w alike);
 *   internal p: (u_E - u_W + v_N - v_S + w_T - w_B)/h - xi = g;
 *   mean row: (1/M_p) sum of the internal p = 0;
 *   body ghosts: eq. (BCu) with the triquadratic interpolant (Dirichlet, u v w) and its normal derivative (p);
 *   walls: normal velocity Dirichlet rows; tangential velocity ghost rows (3/8, 3/4, -1/8) of the wall geometry.
 * Readings carried over from the 2-D oracle (listed in the design notes): theta towards the fluid, paper rows on
 * the finest level where defined, extrapolation rows otherwise, coarse rows below cg_min replaced, colour order
 * of the boxes, lambda Jacobi ghost sweeps, xi and mean-pressure relaxation.  Readings new in 3-D: the colour of
 * cell (i, j, k) is (i + 2j + 3k) mod 7 (no two boxes of one colour read each other's unknowns, checked by
 * enumeration in the tests), and the prolongation renormalises the trilinear weights over the coarse points that
 * carry a value (no extension points in 3-D).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OK 0
#define E_INVAL (-1)
#define E_GEOM (-4)
#define E_NOCONV (-5)
#define E_DIVERGED (-6)

enum { C_INACTIVE = 0, C_INT = 1, C_GHOST = 2, C_WALLD = 3, C_WALLG = 4, C_BODY = 6, C_GHOSTX = 7 };

static void *xcalloc(size_t n, size_t s) {
  void *p = calloc(n ? n : 1, s ? s : 1);
  if (!p) {
    fprintf(stderr, "oracle3: out of memory\n");
    abort();
  }
  return p;
}

typedef struct {
  int N, W, lstride;
  double h;
  long W3, n; /* points per grid, unknowns (4 W^3 + 1) */
  unsigned char *cls;
  double *x, *b, *r;
  /* ghost rows, per point: row index (-1 none); rows: point, 27 columns and weights, dtau, boundary point, theta */
  int *rowof;
  int ng;
  int *g_pt, *g_col;
  double *g_w, *g_dtau, *g_B, *g_th;
  int Mp;
  /* coarsest: dense LU of the whole system */
  int nc;
  int *c_map; /* unknown -> dense index (-1 none) */
  double *c_LU;
  int *c_piv;
} L3;

typedef struct {
  int N, L;
  int nu1, nu2, gamma, lam, coarsest_n, march_max, krylov;
  double dtau_dir, dtau_neu_over_h, eps_over_h, cg_min, alpha;
  int nbis;
  double *phi; /* (2N + 1)^3 */
  int have_geom;
  L3 lev[12];
  double hist[512];
  int nhist;
} S3;

/* ------------------------------------------------------------------------- */
/* indexing                                                                   */
/* ------------------------------------------------------------------------- */
static long gi3(const L3 *L, int g, int i, int j, int k) {
  return g * L->W3 + ((long)(k + 1) * L->W + (j + 1)) * L->W + (i + 1);
}
static int in3(const L3 *L, int i, int j, int k) {
  return i >= -1 && i <= L->N && j >= -1 && j <= L->N && k >= -1 && k <= L->N;
}
static void unpack(const L3 *L, long p, int *g, int *i, int *j, int *k) {
  *g = (int)(p / L->W3);
  long q = p - *g * L->W3;
  *k = (int)(q / ((long)L->W * L->W)) - 1;
  q -= (long)(*k + 1) * L->W * L->W;
  *j = (int)(q / L->W) - 1;
  *i = (int)(q - (long)(*j + 1) * L->W) - 1;
}
static const double OFS[4][3] = {{0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}, {0.5, 0.5, 0.5}};
static void node_xyz(const L3 *L, int g, int i, int j, int k, double X[3]) {
  X[0] = -1.0 + (i + OFS[g][0]) * L->h;
  X[1] = -1.0 + (j + OFS[g][1]) * L->h;
  X[2] = -1.0 + (k + OFS[g][2]) * L->h;
}
static int valued(int c) { return c == C_INT || c == C_GHOST || c == C_GHOSTX || c == C_WALLD || c == C_WALLG; }
static int rowed(int c) { return c == C_GHOST || c == C_GHOSTX || c == C_WALLG; }

/* ------------------------------------------------------------------------- */
/* level set: lattice samples and the trilinear interpolant (Sect. 3.1)       */
/* ------------------------------------------------------------------------- */
static double lat(const S3 *S, const L3 *L, int a, int b, int c) {
  long n = 2L * S->N + 1, s = L->lstride;
  return S->phi[((long)c * s * n + (long)b * s) * n + (long)a * s];
}
/* value and gradient of the trilinear interpolant on the lattice cell holding X (half-open, clamped) */
static void trilin(const S3 *S, const L3 *L, const double X[3], double *val, double g[3]) {
  double hl = 0.5 * L->h;
  int nl = 2 * L->N + 1, c[3];
  double t[3];
  for (int d = 0; d < 3; d++) {
    double f = (X[d] + 1.0) / hl;
    c[d] = (int)floor(f);
    if (c[d] < 0) c[d] = 0;
    if (c[d] > nl - 2) c[d] = nl - 2;
    t[d] = f - c[d];
  }
  double v[2][2][2];
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++)
      for (int e = 0; e < 2; e++) v[e][b][a] = lat(S, L, c[0] + a, c[1] + b, c[2] + e);
  double s = 0, gx = 0, gy = 0, gz = 0;
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++)
      for (int e = 0; e < 2; e++) {
        double wx = a ? t[0] : 1 - t[0], wy = b ? t[1] : 1 - t[1], wz = e ? t[2] : 1 - t[2];
        double dx = a ? 1 : -1, dy = b ? 1 : -1, dz = e ? 1 : -1;
        s += wx * wy * wz * v[e][b][a];
        gx += dx * wy * wz * v[e][b][a];
        gy += wx * dy * wz * v[e][b][a];
        gz += wx * wy * dz * v[e][b][a];
      }
  if (val) *val = s;
  if (g) {
    g[0] = gx / hl;
    g[1] = gy / hl;
    g[2] = gz / hl;
  }
}
static void normal3(const S3 *S, const L3 *L, const double X[3], double n[3]) {
  double g[3];
  trilin(S, L, X, NULL, g);
  double m = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  for (int d = 0; d < 3; d++) n[d] = m > 0 ? g[d] / m : 0.0;
}

/* Alg. 1 (3-D): march from G against the normal in steps of h/2 until the interpolant is not positive, then a
 * fixed number of bisections of the last step; the boundary point is the last midpoint.  Returns 0 on failure. */
static int boundary_point3(const S3 *S, const L3 *L, const double G[3], double phig, double B[3]) {
  double H[3] = {G[0], G[1], G[2]}, K[3] = {G[0], G[1], G[2]}, ph = phig;
  int it = 0;
  while (ph > 0) {
    if (it == S->march_max) return 0;
    double n[3];
    for (int d = 0; d < 3; d++) K[d] = H[d];
    normal3(S, L, H, n);
    for (int d = 0; d < 3; d++) H[d] -= 0.5 * L->h * n[d];
    trilin(S, L, H, &ph, NULL);
    it++;
  }
  if (it == 0 || ph == 0.0) {
    for (int d = 0; d < 3; d++) B[d] = H[d];
    return 1;
  }
  double M[3] = {H[0], H[1], H[2]};
  for (int q = 0; q < S->nbis; q++) {
    for (int d = 0; d < 3; d++) M[d] = 0.5 * (H[d] + K[d]);
    double pm;
    trilin(S, L, M, &pm, NULL);
    if (pm * ph < 0) {
      for (int d = 0; d < 3; d++) K[d] = M[d];
    } else {
      for (int d = 0; d < 3; d++) H[d] = M[d];
      ph = pm;
    }
  }
  for (int d = 0; d < 3; d++) B[d] = M[d];
  return 1;
}

/* three-point Lagrange basis at offsets 0, 1, 2 and its derivative */
static void T3(double t, double T[3]) {
  T[0] = (1 - t) * (2 - t) / 2;
  T[1] = t * (2 - t);
  T[2] = t * (t - 1) / 2;
}
static void D3(double t, double D[3]) {
  D[0] = t - 1.5;
  D[1] = 2 - 2 * t;
  D[2] = t - 0.5;
}
/* weights of the 27-point rows, index (c * 3 + b) * 3 + a for the stencil point G - (a s_x, b s_y, c s_z) h:
 * Dirichlet (triquadratic value at B), Neumann (n . grad of it at B; theta = s (x_G - x)/h, so d/dx = -(s/h) d/dtheta) */
void o3_st27_dirichlet(const double th[3], double *w) {
  double Tx[3], Ty[3], Tz[3];
  T3(th[0], Tx);
  T3(th[1], Ty);
  T3(th[2], Tz);
  for (int c = 0; c < 3; c++)
    for (int b = 0; b < 3; b++)
      for (int a = 0; a < 3; a++) w[(c * 3 + b) * 3 + a] = Tx[a] * Ty[b] * Tz[c];
}
void o3_st27_neumann(const double th[3], const double s[3], const double n[3], double h, double *w) {
  double T[3][3], D[3][3];
  for (int d = 0; d < 3; d++) {
    T3(th[d], T[d]);
    D3(th[d], D[d]);
  }
  for (int c = 0; c < 3; c++)
    for (int b = 0; b < 3; b++)
      for (int a = 0; a < 3; a++)
        w[(c * 3 + b) * 3 + a] = -(n[0] * s[0] * D[0][a] * T[1][b] * T[2][c] + n[1] * s[1] * T[0][a] * D[1][b] * T[2][c] +
                                   n[2] * s[2] * T[0][a] * T[1][b] * D[2][c]) / h;
}

/* ------------------------------------------------------------------------- */
/* geometry of one level                                                      */
/* ------------------------------------------------------------------------- */
static void free_level(L3 *L) {
  free(L->cls);
  free(L->x);
  free(L->b);
  free(L->r);
  free(L->rowof);
  free(L->g_pt);
  free(L->g_col);
  free(L->g_w);
  free(L->g_dtau);
  free(L->g_B);
  free(L->g_th);
  free(L->c_map);
  free(L->c_LU);
  free(L->c_piv);
  memset(L, 0, sizeof(*L));
}

/* points an internal row of (g, i, j, k) reads (up to 7; returns the count) */
static int int_row_cols(const L3 *L, int g, int i, int j, int k, long *cols) {
  int m = 0;
  if (g < 3) {
    static const int d6[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    cols[m++] = gi3(L, g, i, j, k);
    for (int q = 0; q < 6; q++) cols[m++] = gi3(L, g, i + d6[q][0], j + d6[q][1], k + d6[q][2]);
    cols[m++] = gi3(L, 3, i, j, k);
    cols[m++] = gi3(L, 3, i - (g == 0), j - (g == 1), k - (g == 2));
  } else {
    cols[m++] = gi3(L, 0, i, j, k);
    cols[m++] = gi3(L, 0, i + 1, j, k);
    cols[m++] = gi3(L, 1, i, j, k);
    cols[m++] = gi3(L, 1, i, j + 1, k);
    cols[m++] = gi3(L, 2, i, j, k);
    cols[m++] = gi3(L, 2, i, j, k + 1);
  }
  return m;
}

/* the 27-point upwind stencil of a ghost: signs of the normal at G, columns; 0 if it leaves the array */
static int st27(const S3 *S, const L3 *L, int g, int i, int j, int k, double s[3], long *col) {
  double X[3], n[3];
  node_xyz(L, g, i, j, k, X);
  normal3(S, L, X, n);
  for (int d = 0; d < 3; d++) s[d] = n[d] >= 0 ? 1.0 : -1.0;
  int ok = 1;
  for (int c = 0; c < 3; c++)
    for (int b = 0; b < 3; b++)
      for (int a = 0; a < 3; a++) {
        int ii = i - (int)s[0] * a, jj = j - (int)s[1] * b, kk = k - (int)s[2] * c;
        if (!in3(L, ii, jj, kk)) {
          ok = 0;
          col[(c * 3 + b) * 3 + a] = gi3(L, g, i, j, k);
        } else {
          col[(c * 3 + b) * 3 + a] = gi3(L, g, ii, jj, kk);
        }
      }
  return ok;
}

/* quadratic extrapolation row along the grid axis closest to the normal: x_G - sum w_q x_q = 0 from the first
 * three consecutive valued non-extrapolated points towards the fluid.  Returns 1 if found. */
static int extrap_row(const S3 *S, const L3 *L, int g, int i, int j, int k, long *col, double *w) {
  double X[3], n[3];
  node_xyz(L, g, i, j, k, X);
  normal3(S, L, X, n);
  int order[3] = {0, 1, 2};
  for (int a = 0; a < 3; a++)
    for (int b = a + 1; b < 3; b++)
      if (fabs(n[order[b]]) > fabs(n[order[a]])) {
        int t = order[a];
        order[a] = order[b];
        order[b] = t;
      }
  for (int q = 0; q < 3; q++) {
    int ax = order[q], sg = n[ax] >= 0 ? 1 : -1;
    int di[3] = {0, 0, 0};
    di[ax] = -sg;
    for (int k0 = 1; k0 <= 4; k0++) {
      int okk = 1;
      long c3[3];
      for (int m = 0; m < 3; m++) {
        int ii = i + di[0] * (k0 + m), jj = j + di[1] * (k0 + m), kk = k + di[2] * (k0 + m);
        if (!in3(L, ii, jj, kk)) {
          okk = 0;
          break;
        }
        long p = gi3(L, g, ii, jj, kk);
        int c = L->cls[p];
        if (!(c == C_INT || c == C_GHOST || c == C_WALLD)) {
          okk = 0;
          break;
        }
        c3[m] = p;
      }
      if (!okk) continue;
      /* Lagrange extrapolation to offset 0 from offsets k0, k0 + 1, k0 + 2 */
      double t0 = k0, t1 = k0 + 1, t2 = k0 + 2;
      w[0] = (0 - t1) * (0 - t2) / ((t0 - t1) * (t0 - t2));
      w[1] = (0 - t0) * (0 - t2) / ((t1 - t0) * (t1 - t2));
      w[2] = (0 - t0) * (0 - t1) / ((t2 - t0) * (t2 - t1));
      for (int m = 0; m < 3; m++) col[m] = c3[m];
      return 1;
    }
  }
  return 0;
}

static int build_level(S3 *S, int l) {
  L3 *L = &S->lev[l];
  const int N = L->N;
  const long P = 4 * L->W3;
  unsigned char *cls = L->cls;
  memset(cls, C_INACTIVE, P);
  /* 1. classification: walls, internal (phi < 0) and body points */
  for (int g = 0; g < 4; g++)
    for (int k = -1; k <= N; k++)
      for (int j = -1; j <= N; j++)
        for (int i = -1; i <= N; i++) {
          int I[3] = {i, j, k};
          long p = gi3(L, g, i, j, k);
          int out = 0, ring = 0, normal_wall = 0;
          for (int d = 0; d < 3; d++) {
            int lo = (g < 3 && d == g) ? 0 : 0, hi = (g < 3 && d == g) ? N : N - 1;
            (void)lo;
            if (I[d] < 0 || I[d] > hi) {
              out++;
              ring = d;
            }
            if (g < 3 && d == g && (I[d] == 0 || I[d] == N)) normal_wall = 1;
          }
          if (g == 3) {
            if (out) continue;
          } else {
            if (out >= 2) continue;
            if (out == 1) {
              /* tangential ghost beyond a wall (the wall normal is the axis that left the box) */
              int inward_ok = 1;
              for (int d = 0; d < 3; d++)
                if (d != ring && (I[d] < 0 || I[d] > ((d == g) ? N : N - 1))) inward_ok = 0;
              if (inward_ok && ring != g) cls[p] = C_WALLG;
              continue;
            }
            if (normal_wall) {
              cls[p] = C_WALLD;
              continue;
            }
          }
          int a = 2 * i + (g == 0 ? 0 : 1), b = 2 * j + (g == 1 ? 0 : 1), c = 2 * k + (g == 2 ? 0 : 1);
          cls[p] = lat(S, L, a, b, c) < 0 ? C_INT : C_BODY;
        }
  /* 2. ghosts: body points read by internal rows, closed under the 27-point stencils of ghosts */
  long cols[9];
  for (long p = 0; p < P; p++) {
    if (cls[p] != C_INT) continue;
    int g, i, j, k;
    unpack(L, p, &g, &i, &j, &k);
    int m = int_row_cols(L, g, i, j, k, cols);
    for (int q = 0; q < m; q++)
      if (cls[cols[q]] == C_BODY) cls[cols[q]] = C_GHOST;
  }
  for (int changed = 1; changed;) {
    changed = 0;
    for (long p = 0; p < P; p++) {
      if (cls[p] != C_GHOST) continue;
      int g, i, j, k;
      unpack(L, p, &g, &i, &j, &k);
      double s[3];
      long c27[27];
      st27(S, L, g, i, j, k, s, c27);
      for (int q = 0; q < 27; q++)
        if (cls[c27[q]] == C_BODY) {
          cls[c27[q]] = C_GHOST;
          changed = 1;
        }
    }
  }
  for (long p = 0; p < P; p++)
    if (cls[p] == C_BODY) cls[p] = C_INACTIVE;
  /* 3. rows of ghosts and wall ghosts */
  int ng = 0;
  for (long p = 0; p < P; p++)
    if (cls[p] == C_GHOST || cls[p] == C_WALLG) ng++;
  L->ng = ng;
  L->g_pt = (int *)xcalloc(ng, sizeof(int));
  L->g_col = (int *)xcalloc(27L * ng, sizeof(int));
  L->g_w = (double *)xcalloc(27L * ng, sizeof(double));
  L->g_dtau = (double *)xcalloc(ng, sizeof(double));
  L->g_B = (double *)xcalloc(3L * ng, sizeof(double));
  L->g_th = (double *)xcalloc(3L * ng, sizeof(double));
  for (long p = 0; p < P; p++) L->rowof[p] = -1;
  int r = 0;
  for (long p = 0; p < P; p++) {
    if (!(cls[p] == C_GHOST || cls[p] == C_WALLG)) continue;
    int g, i, j, k;
    unpack(L, p, &g, &i, &j, &k);
    L->g_pt[r] = (int)p;
    L->rowof[p] = r;
    int *col = &L->g_col[27L * r];
    double *w = &L->g_w[27L * r];
    for (int q = 0; q < 27; q++) {
      col[q] = (int)p;
      w[q] = 0;
    }
    if (cls[p] == C_WALLG) {
      /* (3/8) x_G + (3/4) x_1 - (1/8) x_2 = b: the wall lies half a step from G (theta 1/2 along the normal) */
      int I[3] = {i, j, k}, d0 = -1;
      for (int d = 0; d < 3; d++)
        if (I[d] < 0 || I[d] > (d == g ? N : N - 1)) d0 = d;
      int st = I[d0] < 0 ? 1 : -1;
      double T[3];
      T3(0.5, T);
      for (int m = 0; m < 3; m++) {
        int J[3] = {i, j, k};
        J[d0] += st * m;
        col[m] = (int)gi3(L, g, J[0], J[1], J[2]);
        w[m] = T[m];
      }
      L->g_dtau[r] = S->dtau_dir;
      double X[3];
      node_xyz(L, g, i, j, k, X);
      X[d0] = I[d0] < 0 ? -1.0 : 1.0;
      for (int d = 0; d < 3; d++) L->g_B[3 * r + d] = X[d];
      r++;
      continue;
    }
    double G[3], B[3], s[3], th[3], n[3];
    long c27[27];
    node_xyz(L, g, i, j, k, G);
    int a = 2 * i + (g == 0 ? 0 : 1), b = 2 * j + (g == 1 ? 0 : 1), c = 2 * k + (g == 2 ? 0 : 1);
    double phig = lat(S, L, a, b, c);
    int ok = st27(S, L, g, i, j, k, s, c27);
    ok = boundary_point3(S, L, G, phig, B) && ok;
    for (int d = 0; d < 3; d++) th[d] = s[d] * (G[d] - B[d]) / L->h;
    for (int q = 0; q < 27; q++)
      if (!valued(cls[c27[q]]) || cls[c27[q]] == C_WALLG) ok = 0;
    for (int d = 0; d < 3; d++)
      if (!(th[d] > -0.5 && th[d] < 1.0)) ok = 0;
    double wt[27];
    if (g < 3) {
      o3_st27_dirichlet(th, wt);
      L->g_dtau[r] = S->dtau_dir;
    } else {
      normal3(S, L, B, n);
      o3_st27_neumann(th, s, n, L->h, wt);
      L->g_dtau[r] = S->dtau_neu_over_h * L->h;
    }
    double diag = g < 3 ? wt[0] : wt[0] * L->h;
    if (!(diag > (l == 0 ? 0.0 : S->cg_min))) ok = 0;
    for (int d = 0; d < 3; d++) {
      L->g_B[3 * r + d] = B[d];
      L->g_th[3 * r + d] = th[d];
    }
    if (ok) {
      for (int q = 0; q < 27; q++) {
        col[q] = (int)c27[q];
        w[q] = wt[q];
      }
    } else {
      cls[p] = C_GHOSTX;
    }
    r++;
  }
  /* 3b. extrapolation rows for the unusable ghosts (identity on coarse levels without sources) */
  for (int q = 0; q < ng; q++) {
    long p = L->g_pt[q];
    if (cls[p] != C_GHOSTX) continue;
    int g, i, j, k;
    unpack(L, p, &g, &i, &j, &k);
    int *col = &L->g_col[27L * q];
    double *w = &L->g_w[27L * q];
    long c3[3];
    double w3[3];
    L->g_dtau[q] = 1.0;
    if (extrap_row(S, L, g, i, j, k, c3, w3)) {
      w[0] = 1.0;
      col[0] = (int)p;
      for (int m = 0; m < 3; m++) {
        col[1 + m] = (int)c3[m];
        w[1 + m] = -w3[m];
      }
    } else {
      if (l == 0) return E_GEOM;
      w[0] = 1.0;
      col[0] = (int)p;
    }
  }
  /* 4. internal pressure count; every internal cell needs an internal face */
  L->Mp = 0;
  for (int k = 0; k < N; k++)
    for (int j = 0; j < N; j++)
      for (int i = 0; i < N; i++) {
        if (cls[gi3(L, 3, i, j, k)] != C_INT) continue;
        L->Mp++;
        long f[6] = {gi3(L, 0, i, j, k), gi3(L, 0, i + 1, j, k), gi3(L, 1, i, j, k),
                     gi3(L, 1, i, j + 1, k), gi3(L, 2, i, j, k), gi3(L, 2, i, j, k + 1)};
        int any = 0;
        for (int q = 0; q < 6; q++) any |= cls[f[q]] == C_INT;
        if (!any) return E_GEOM;
      }
  if (L->Mp == 0) return E_GEOM;
  return OK;
}

/* ------------------------------------------------------------------------- */
/* rows                                                                       */
/* ------------------------------------------------------------------------- */
static double aco(const S3 *S, const L3 *L) { return S->alpha / (L->h * L->h); }
/* (M x)_p for the row of point p (0 for points without a row); the mean row is separate */
static double row_dot(const S3 *S, const L3 *L, long p, const double *x) {
  int c = L->cls[p];
  if (c == C_WALLD) return x[p];
  if (rowed(c)) {
    int r = L->rowof[p];
    double s = 0;
    for (int q = 0; q < 27; q++) s += L->g_w[27L * r + q] * x[L->g_col[27L * r + q]];
    return s;
  }
  if (c != C_INT) return 0.0;
  int g, i, j, k;
  unpack(L, p, &g, &i, &j, &k);
  double a = aco(S, L), d = 1.0 + 6.0 * a, ih = 1.0 / L->h;
  if (g < 3) {
    double nb = x[gi3(L, g, i + 1, j, k)] + x[gi3(L, g, i - 1, j, k)] + x[gi3(L, g, i, j + 1, k)] +
                x[gi3(L, g, i, j - 1, k)] + x[gi3(L, g, i, j, k + 1)] + x[gi3(L, g, i, j, k - 1)];
    double pe = x[gi3(L, 3, i, j, k)], pw = x[gi3(L, 3, i - (g == 0), j - (g == 1), k - (g == 2))];
    return d * x[p] - a * nb + (pe - pw) * ih;
  }
  double div = x[gi3(L, 0, i + 1, j, k)] - x[gi3(L, 0, i, j, k)] + x[gi3(L, 1, i, j + 1, k)] - x[gi3(L, 1, i, j, k)] +
               x[gi3(L, 2, i, j, k + 1)] - x[gi3(L, 2, i, j, k)];
  return div * ih - x[4 * L->W3];
}
/* coefficient of unknown q in the row of p */
static double row_coef(const S3 *S, const L3 *L, long p, long q) {
  int c = L->cls[p];
  if (c == C_WALLD) return p == q ? 1.0 : 0.0;
  if (rowed(c)) {
    int r = L->rowof[p];
    double s = 0;
    for (int z = 0; z < 27; z++)
      if (L->g_col[27L * r + z] == q) s += L->g_w[27L * r + z];
    return s;
  }
  if (c != C_INT) return 0.0;
  int g, i, j, k;
  unpack(L, p, &g, &i, &j, &k);
  double a = aco(S, L), d = 1.0 + 6.0 * a, ih = 1.0 / L->h;
  if (q == 4 * L->W3) return g == 3 ? -1.0 : 0.0;
  if (g < 3) {
    if (q == p) return d;
    static const int d6[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    for (int z = 0; z < 6; z++)
      if (q == gi3(L, g, i + d6[z][0], j + d6[z][1], k + d6[z][2])) return -a;
    if (q == gi3(L, 3, i, j, k)) return ih;
    if (q == gi3(L, 3, i - (g == 0), j - (g == 1), k - (g == 2))) return -ih;
    return 0.0;
  }
  if (q == gi3(L, 0, i + 1, j, k) || q == gi3(L, 1, i, j + 1, k) || q == gi3(L, 2, i, j, k + 1)) return ih;
  if (q == gi3(L, 0, i, j, k) || q == gi3(L, 1, i, j, k) || q == gi3(L, 2, i, j, k)) return -ih;
  return 0.0;
}
static double mean_row(const L3 *L, const double *x) {
  double s = 0;
  for (long q = 3 * L->W3; q < 4 * L->W3; q++)
    if (L->cls[q] == C_INT) s += x[q];
  return s / L->Mp;
}
/* residual of every row; the mean-row residual in r[4 W^3]; returns the max norm */
static double residual(const S3 *S, L3 *L, const double *x, const double *b, double *r) {
  double m = 0;
  for (long p = 0; p < 4 * L->W3; p++) {
    int c = L->cls[p];
    r[p] = (c == C_INT || c == C_WALLD || rowed(c)) ? b[p] - row_dot(S, L, p, x) : 0.0;
    if (fabs(r[p]) > m || r[p] != r[p]) m = fabs(r[p]);
  }
  r[4 * L->W3] = b[4 * L->W3] - mean_row(L, x);
  if (fabs(r[4 * L->W3]) > m) m = fabs(r[4 * L->W3]);
  return m;
}

/* ------------------------------------------------------------------------- */
/* relaxation (Sect. 4.1 in 3-D)                                              */
/* ------------------------------------------------------------------------- */
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
/* the box of cell (i, j, k): its internal faces and pressure solved from their rows, everything else fixed */
static void box_relax(const S3 *S, L3 *L, int i, int j, int k) {
  long cand[7] = {gi3(L, 0, i, j, k), gi3(L, 0, i + 1, j, k), gi3(L, 1, i, j, k), gi3(L, 1, i, j + 1, k),
                  gi3(L, 2, i, j, k), gi3(L, 2, i, j, k + 1), gi3(L, 3, i, j, k)};
  long U[7];
  int m = 0;
  for (int q = 0; q < 7; q++)
    if (L->cls[cand[q]] == C_INT) U[m++] = cand[q];
  if (!m) return;
  double A[49], rhs[7];
  for (int a = 0; a < m; a++) {
    double t = L->b[U[a]] - row_dot(S, L, U[a], L->x);
    for (int c = 0; c < m; c++) {
      A[a * m + c] = row_coef(S, L, U[a], U[c]);
      t += A[a * m + c] * L->x[U[c]];
    }
    rhs[a] = t;
  }
  if (!dense_solve(m, A, rhs)) return;
  for (int a = 0; a < m; a++) L->x[U[a]] = rhs[a];
}
static void ghost_sweeps(const S3 *S, L3 *L) {
  double *nv = (double *)xcalloc(L->ng, sizeof(double));
  for (int it = 0; it < S->lam; it++) {
    for (int r = 0; r < L->ng; r++) {
      long p = L->g_pt[r];
      nv[r] = L->x[p] + L->g_dtau[r] * (L->b[p] - row_dot(S, L, p, L->x));
    }
    for (int r = 0; r < L->ng; r++) L->x[L->g_pt[r]] = nv[r];
  }
  free(nv);
}
/* xi <- mean over the internal cells of (div_h u - g): the continuity residuals then sum to zero */
static void xi_update(const S3 *S, L3 *L) {
  double s = 0;
  long xi = 4 * L->W3;
  for (long q = 3 * L->W3; q < 4 * L->W3; q++)
    if (L->cls[q] == C_INT) s += (row_dot(S, L, q, L->x) + L->x[xi]) - L->b[q];
  L->x[xi] = s / L->Mp;
}
/* one relaxation step: boxes in the colour order (i + 2j + 3k) mod 7, lambda ghost sweeps, xi */
static void relax_step(const S3 *S, L3 *L) {
  int N = L->N;
  for (int col = 0; col < 7; col++)
    for (int k = 0; k < N; k++)
      for (int j = 0; j < N; j++)
        for (int i = 0; i < N; i++)
          if ((i + 2 * j + 3 * k) % 7 == col) box_relax(S, L, i, j, k);
  ghost_sweeps(S, L);
  xi_update(S, L);
}
static void set_wall_dirichlet(L3 *L) {
  for (long p = 0; p < 4 * L->W3; p++)
    if (L->cls[p] == C_WALLD) L->x[p] = L->b[p];
}

/* ------------------------------------------------------------------------- */
/* transfers (Sect. 4.2 - 4.3 in 3-D)                                         */
/* ------------------------------------------------------------------------- */
/* restriction of the fine residual to the coarse right-hand side: the staggered weights (1 2 1)/4 along the
 * grid's own axis and 1/2, 1/2 across (1/8 for the cell centres) where every fine point of the stencil exists and
 * has the coarse point's class; otherwise the plain mean over the fine points that do; none: 0 */
static void restrict3(const L3 *F, const double *rf, L3 *C, double *bc) {
  for (long q = 0; q < 4 * C->W3; q++) {
    bc[q] = 0;
    int cc = C->cls[q];
    if (!(cc == C_INT || cc == C_GHOST)) continue;
    int g, I, J, K;
    unpack(C, q, &g, &I, &J, &K);
    int IJK[3] = {I, J, K};
    int lo[3], n3[3];
    double wts[3][3];
    for (int d = 0; d < 3; d++) {
      if (g == d) {
        lo[d] = 2 * IJK[d] - 1;
        n3[d] = 3;
        wts[d][0] = 0.25;
        wts[d][1] = 0.5;
        wts[d][2] = 0.25;
      } else {
        lo[d] = 2 * IJK[d];
        n3[d] = 2;
        wts[d][0] = wts[d][1] = 0.5;
      }
    }
    double s = 0, sw = 0, su = 0;
    int all = 1, cnt = 0;
    for (int c = 0; c < n3[2]; c++)
      for (int b = 0; b < n3[1]; b++)
        for (int a = 0; a < n3[0]; a++) {
          int i = lo[0] + a, j = lo[1] + b, k = lo[2] + c;
          if (!in3(F, i, j, k) || F->cls[gi3(F, g, i, j, k)] != cc) {
            all = 0;
            continue;
          }
          double v = rf[gi3(F, g, i, j, k)];
          s += wts[0][a] * wts[1][b] * wts[2][c] * v;
          sw += wts[0][a] * wts[1][b] * wts[2][c];
          su += v;
          cnt++;
        }
    (void)sw;
    bc[q] = all ? s : (cnt ? su / cnt : 0.0);
  }
  bc[4 * C->W3] = 0.0;
}
/* prolongation of the coarse correction, added to the fine internal and ghost values: trilinear staggered
 * weights (1 or 1/2, 1/2 along the grid's own axis, 3/4, 1/4 across), renormalised over the coarse points that
 * carry a value; the pressure outside the box takes the nearest cell (mirror); xi with weight 1 */
static void prolong3(const L3 *C, const double *ec, L3 *F, double *xf) {
  for (long p = 0; p < 4 * F->W3; p++) {
    int cf = F->cls[p];
    if (!(cf == C_INT || cf == C_GHOST || cf == C_GHOSTX)) continue;
    int g, i, j, k;
    unpack(F, p, &g, &i, &j, &k);
    int IJK[3] = {i, j, k}, ci[3][2], nn[3];
    double cw[3][2];
    for (int d = 0; d < 3; d++) {
      int f = IJK[d];
      if (g == d) {
        if ((f & 1) == 0) {
          ci[d][0] = f / 2;
          cw[d][0] = 1;
          nn[d] = 1;
        } else {
          ci[d][0] = (f - 1) / 2;
          ci[d][1] = (f + 1) / 2;
          cw[d][0] = cw[d][1] = 0.5;
          nn[d] = 2;
        }
      } else {
        int c0 = (f >= 0) ? f / 2 : -1;
        ci[d][0] = c0;
        ci[d][1] = ((f & 1) == 0) ? c0 - 1 : c0 + 1;
        cw[d][0] = 0.75;
        cw[d][1] = 0.25;
        nn[d] = 2;
      }
    }
    double s = 0, sw = 0;
    for (int c = 0; c < nn[2]; c++)
      for (int b = 0; b < nn[1]; b++)
        for (int a = 0; a < nn[0]; a++) {
          int I = ci[0][a], J = ci[1][b], K = ci[2][c];
          if (g == 3) {
            I = I < 0 ? 0 : (I > C->N - 1 ? C->N - 1 : I);
            J = J < 0 ? 0 : (J > C->N - 1 ? C->N - 1 : J);
            K = K < 0 ? 0 : (K > C->N - 1 ? C->N - 1 : K);
          }
          if (!in3(C, I, J, K)) continue;
          long q = gi3(C, g, I, J, K);
          if (!valued(C->cls[q])) continue;
          double w = cw[0][a] * cw[1][b] * cw[2][c];
          s += w * ec[q];
          sw += w;
        }
    if (sw > 0) xf[p] += s / sw;
  }
  xf[4 * F->W3] += ec[4 * C->W3];
}

/* ------------------------------------------------------------------------- */
/* coarsest level: dense LU of the whole system (unknowns: rowed or internal points, and xi)                 */
/* ------------------------------------------------------------------------- */
static int coarse_factor(S3 *S) {
  L3 *L = &S->lev[S->L - 1];
  long P = 4 * L->W3;
  free(L->c_map);
  free(L->c_LU);
  free(L->c_piv);
  L->c_map = (int *)xcalloc(P + 1, sizeof(int));
  int n = 0;
  for (long p = 0; p < P; p++) {
    int c = L->cls[p];
    L->c_map[p] = (c == C_INT || c == C_WALLD || rowed(c)) ? n++ : -1;
  }
  L->c_map[P] = n++;
  L->nc = n;
  double *A = (double *)xcalloc((size_t)n * n, sizeof(double));
  double *e = (double *)xcalloc(P + 1, sizeof(double));
  /* column by column: A e_q */
  for (long q = 0; q <= P; q++) {
    if (L->c_map[q] < 0) continue;
    e[q] = 1.0;
    for (long p = 0; p < P; p++)
      if (L->c_map[p] >= 0) {
        double v = (q == P) ? row_coef(S, L, p, P) : row_coef(S, L, p, q);
        if (v != 0.0) A[(size_t)L->c_map[p] * n + L->c_map[q]] = v;
      }
    if (q < P && q >= 3 * L->W3 && L->cls[q] == C_INT) A[(size_t)L->c_map[P] * n + L->c_map[q]] = 1.0 / L->Mp;
    e[q] = 0.0;
  }
  free(e);
  /* LU with partial pivoting */
  int *piv = (int *)xcalloc(n, sizeof(int));
  for (int k = 0; k < n; k++) {
    int p = k;
    for (int i = k + 1; i < n; i++)
      if (fabs(A[(size_t)i * n + k]) > fabs(A[(size_t)p * n + k])) p = i;
    piv[k] = p;
    if (A[(size_t)p * n + k] == 0.0) {
      free(A);
      free(piv);
      return E_GEOM;
    }
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
  L->c_LU = A;
  L->c_piv = piv;
  return OK;
}
static void coarse_solve(S3 *S) {
  L3 *L = &S->lev[S->L - 1];
  long P = 4 * L->W3;
  int n = L->nc;
  double *y = (double *)xcalloc(n, sizeof(double));
  for (long p = 0; p <= P; p++)
    if (L->c_map[p] >= 0) y[L->c_map[p]] = L->b[p];
  for (int k = 0; k < n; k++)
    if (L->c_piv[k] != k) {
      double t = y[k];
      y[k] = y[L->c_piv[k]];
      y[L->c_piv[k]] = t;
    }
  for (int i = 0; i < n; i++)
    for (int c = 0; c < i; c++) y[i] -= L->c_LU[(size_t)i * n + c] * y[c];
  for (int i = n - 1; i >= 0; i--) {
    for (int c = i + 1; c < n; c++) y[i] -= L->c_LU[(size_t)i * n + c] * y[c];
    y[i] /= L->c_LU[(size_t)i * n + i];
  }
  for (long p = 0; p <= P; p++) L->x[p] = L->c_map[p] >= 0 ? y[L->c_map[p]] : 0.0;
  free(y);
}

/* ------------------------------------------------------------------------- */
/* cycle and solver                                                           */
/* ------------------------------------------------------------------------- */
static void mean_project(L3 *L) {
  double m = mean_row(L, L->x);
  for (long q = 3 * L->W3; q < 4 * L->W3; q++) {
    int c = L->cls[q];
    if (c == C_INT || c == C_GHOST || c == C_GHOSTX) L->x[q] -= m;
  }
}
static void cycle(S3 *S, int l) {
  if (l == S->L - 1) {
    coarse_solve(S);
    return;
  }
  L3 *F = &S->lev[l], *C = &S->lev[l + 1];
  for (int q = 0; q < S->nu1; q++) relax_step(S, F);
  residual(S, F, F->x, F->b, F->r);
  restrict3(F, F->r, C, C->b);
  memset(C->x, 0, sizeof(double) * C->n);
  int reps = (l + 1 == S->L - 1) ? 1 : S->gamma;
  for (int q = 0; q < reps; q++) cycle(S, l + 1);
  prolong3(C, C->x, F, F->x);
  for (int q = 0; q < S->nu2; q++) relax_step(S, F);
}
/* B'(r): one cycle from zero on M e = r, mean projection, and the mean-row column (a constant pressure) */
static void precond(S3 *S, const double *r, double *z) {
  L3 *L = &S->lev[0];
  double *sb = L->b, *sx = L->x;
  L->b = (double *)r;
  L->x = z;
  memset(z, 0, sizeof(double) * L->n);
  set_wall_dirichlet(L);
  cycle(S, 0);
  mean_project(L);
  for (long q = 3 * L->W3; q < 4 * L->W3; q++) {
    int c = L->cls[q];
    if (c == C_INT || c == C_GHOST || c == C_GHOSTX) z[q] += r[4 * L->W3];
  }
  for (long q = 0; q < 4 * L->W3; q++) {
    int c = L->cls[q];
    if (!(c == C_INT || rowed(c) || c == C_WALLD)) z[q] = 0.0;
  }
  L->b = sb;
  L->x = sx;
}
static void apply(const S3 *S, L3 *L, const double *x, double *y) {
  for (long p = 0; p < 4 * L->W3; p++) {
    int c = L->cls[p];
    y[p] = (c == C_INT || c == C_WALLD || rowed(c)) ? row_dot(S, L, p, x) : 0.0;
  }
  y[4 * L->W3] = mean_row(L, x);
}
static double norm_inf(const double *v, long n) {
  double m = 0;
  for (long i = 0; i < n; i++)
    if (fabs(v[i]) > m || v[i] != v[i]) m = fabs(v[i]);
  return m;
}

/* Solve to ||r||_inf <= tol max(1, ||b||_inf): krylov = 0 plain cycles, krylov = m > 0 the cycle as the
 * preconditioner of GCR restarted after m directions (as in the 2-D oracle).  stats: cycles, res0, res, rho. */
int o3_solve(void *h, double tol, int max_cycles, double *stats) {
  S3 *S = (S3 *)h;
  if (!S->have_geom) return E_INVAL;
  L3 *L = &S->lev[0];
  long n = L->n;
  set_wall_dirichlet(L);
  double r0 = residual(S, L, L->x, L->b, L->r), bn = norm_inf(L->b, n), thr = tol * (bn > 1 ? bn : 1);
  double rn = r0, rp = r0, rho = 0;
  int c = 0, status = r0 == r0 ? OK : E_DIVERGED;
  S->nhist = 0;
  S->hist[S->nhist++] = r0;
  if (status == OK && S->krylov <= 0) {
    while (rn > thr && c < max_cycles) {
      cycle(S, 0);
      mean_project(L);
      rp = rn;
      rn = residual(S, L, L->x, L->b, L->r);
      rho = rn / rp;
      c++;
      if (S->nhist < 512) S->hist[S->nhist++] = rn;
      if (!(rn == rn) || rn > 1e6 * (r0 > 1 ? r0 : 1)) {
        status = E_DIVERGED;
        break;
      }
    }
  } else if (status == OK) {
    int m = S->krylov, k = 0;
    double *r = (double *)xcalloc(n, sizeof(double)), *z = (double *)xcalloc(n, sizeof(double));
    double *q = (double *)xcalloc(n, sizeof(double));
    double *Q = (double *)xcalloc((size_t)m * n, sizeof(double)), *Z = (double *)xcalloc((size_t)m * n, sizeof(double));
    double *nq = (double *)xcalloc(m, sizeof(double));
    memcpy(r, L->r, sizeof(double) * n);
    while (rn > thr && c < max_cycles) {
      precond(S, r, z);
      apply(S, L, z, q);
      /* classical Gram-Schmidt: every coefficient from the new image before any is subtracted */
      double beta[64];
      for (int i = 0; i < k; i++) {
        double d = 0;
        for (long e = 0; e < n; e++) d += Q[(size_t)i * n + e] * q[e];
        beta[i] = d / nq[i];
      }
      for (int i = 0; i < k; i++)
        for (long e = 0; e < n; e++) {
          q[e] -= beta[i] * Q[(size_t)i * n + e];
          z[e] -= beta[i] * Z[(size_t)i * n + e];
        }
      double qq = 0, rq = 0;
      for (long e = 0; e < n; e++) {
        qq += q[e] * q[e];
        rq += r[e] * q[e];
      }
      double gam = qq > 0 ? rq / qq : 0;
      for (long e = 0; e < n; e++) {
        L->x[e] += gam * z[e];
        r[e] -= gam * q[e];
        Q[(size_t)k * n + e] = q[e];
        Z[(size_t)k * n + e] = z[e];
      }
      nq[k] = qq;
      k++;
      c++;
      rp = rn;
      rn = norm_inf(r, n);
      if (rn <= thr || k == m) {
        rn = residual(S, L, L->x, L->b, r);
        k = 0;
      }
      rho = rn / rp;
      if (S->nhist < 512) S->hist[S->nhist++] = rn;
      if (!(rn == rn) || rn > 1e6 * (r0 > 1 ? r0 : 1)) {
        status = E_DIVERGED;
        break;
      }
    }
    free(r);
    free(z);
    free(q);
    free(Q);
    free(Z);
    free(nq);
  }
  if (status == OK && rn > thr) status = E_NOCONV;
  if (stats) {
    stats[0] = c;
    stats[1] = r0;
    stats[2] = rn;
    stats[3] = rho;
  }
  return status;
}

/* ------------------------------------------------------------------------- */
/* interface                                                                  */
/* ------------------------------------------------------------------------- */
/* iparams: nu1 nu2 gamma lambda coarsest_n march_max krylov; dparams: dtau_dir dtau_neu_over_h eps_over_h
 * cg_min */
void *o3_create(int N, const int *ip, const double *dp) {
  if (N < 4 || (N & (N - 1))) return NULL;
  S3 *S = (S3 *)xcalloc(1, sizeof(S3));
  S->N = N;
  S->nu1 = ip[0];
  S->nu2 = ip[1];
  S->gamma = ip[2];
  S->lam = ip[3];
  S->coarsest_n = ip[4];
  S->march_max = ip[5];
  S->krylov = ip[6] > 64 ? 64 : ip[6];
  S->dtau_dir = dp[0];
  S->dtau_neu_over_h = dp[1];
  S->eps_over_h = dp[2];
  S->cg_min = dp[3];
  S->nbis = (int)ceil(log2(0.5 / S->eps_over_h) - 1e-12);
  if (S->coarsest_n < 2 || S->coarsest_n > N) {
    free(S);
    return NULL;
  }
  int L = 0;
  for (int n = N; n >= S->coarsest_n; n /= 2) L++;
  S->L = L;
  for (int l = 0; l < L; l++) {
    L3 *V = &S->lev[l];
    V->N = N >> l;
    V->W = V->N + 2;
    V->W3 = (long)V->W * V->W * V->W;
    V->n = 4 * V->W3 + 1;
    V->h = 2.0 / V->N;
    V->lstride = 1 << l;
  }
  S->phi = (double *)xcalloc((size_t)(2 * N + 1) * (2 * N + 1) * (2 * N + 1), sizeof(double));
  return S;
}
void o3_destroy(void *h) {
  S3 *S = (S3 *)h;
  if (!S) return;
  for (int l = 0; l < S->L; l++) free_level(&S->lev[l]);
  free(S->phi);
  free(S);
}
int o3_num_levels(void *h) { return ((S3 *)h)->L; }
int o3_level_n(void *h, int l) { return ((S3 *)h)->lev[l].N; }

/* analytic level sets on the (2N + 1)^3 lattice: kind 0 sphere R - |x - c|, kind 1 ellipsoid
 * 1 - sqrt(sum ((x - c)_d / A_d)^2); p = {R or A_x, A_y, A_z, c_x, c_y, c_z} */
int o3_levelset_analytic(int kind, const double *p, int N, double *phi) {
  int n = 2 * N + 1;
  double hl = 1.0 / N;
  for (int c = 0; c < n; c++)
    for (int b = 0; b < n; b++)
      for (int a = 0; a < n; a++) {
        double X = -1 + a * hl - p[3], Y = -1 + b * hl - p[4], Z = -1 + c * hl - p[5];
        double v;
        if (kind == 0)
          v = p[0] - sqrt(X * X + Y * Y + Z * Z);
        else if (kind == 1)
          v = 1.0 - sqrt(X * X / (p[0] * p[0]) + Y * Y / (p[1] * p[1]) + Z * Z / (p[2] * p[2]));
        else
          return E_INVAL;
        phi[((size_t)c * n + b) * n + a] = v;
      }
  return OK;
}

int o3_set_levelset(void *h, const double *phi) {
  S3 *S = (S3 *)h;
  size_t nl = (size_t)(2 * S->N + 1);
  memcpy(S->phi, phi, nl * nl * nl * sizeof(double));
  for (int l = 0; l < S->L; l++) {
    L3 *V = &S->lev[l];
    int N = V->N;
    free_level(V);
    V->N = N;
    V->W = N + 2;
    V->W3 = (long)V->W * V->W * V->W;
    V->n = 4 * V->W3 + 1;
    V->h = 2.0 / N;
    V->lstride = 1 << l;
    V->cls = (unsigned char *)xcalloc(4 * V->W3, 1);
    V->x = (double *)xcalloc(V->n, sizeof(double));
    V->b = (double *)xcalloc(V->n, sizeof(double));
    V->r = (double *)xcalloc(V->n, sizeof(double));
    V->rowof = (int *)xcalloc(4 * V->W3, sizeof(int));
    int st = build_level(S, l);
    if (st) {
      S->have_geom = 0;
      return st;
    }
  }
  S->have_geom = 1;
  return S->alpha > 0 ? coarse_factor(S) : OK;
}
int o3_set_alpha(void *h, double alpha) {
  S3 *S = (S3 *)h;
  S->alpha = alpha;
  return S->have_geom ? coarse_factor(S) : OK;
}
int o3_get_classes(void *h, int l, unsigned char *out) {
  S3 *S = (S3 *)h;
  if (!S->have_geom) return E_INVAL;
  memcpy(out, S->lev[l].cls, 4 * S->lev[l].W3);
  return OK;
}
/* per point (4 W^3): boundary point (3), theta (3), 27 weights, 27 columns, dtau; NaN / -1 without a row */
int o3_get_ghost_rows(void *h, int l, double *B, double *th, double *w27, int *c27, double *dtau) {
  S3 *S = (S3 *)h;
  if (!S->have_geom) return E_INVAL;
  L3 *L = &S->lev[l];
  for (long p = 0; p < 4 * L->W3; p++) {
    int r = L->rowof[p];
    for (int d = 0; d < 3; d++) {
      B[3 * p + d] = r >= 0 ? L->g_B[3 * r + d] : NAN;
      th[3 * p + d] = r >= 0 ? L->g_th[3 * r + d] : NAN;
    }
    for (int q = 0; q < 27; q++) {
      w27[27 * p + q] = r >= 0 ? L->g_w[27L * r + q] : NAN;
      c27[27 * p + q] = r >= 0 ? L->g_col[27L * r + q] : -1;
    }
    dtau[p] = r >= 0 ? L->g_dtau[r] : NAN;
  }
  return OK;
}
/* boundary data on full grids (W^3 each, any may be NULL): values at ghost, wall-ghost and wall points */
void o3_set_boundary_values(void *h, const double *bu, const double *bv, const double *bw, const double *bp) {
  S3 *S = (S3 *)h;
  L3 *L = &S->lev[0];
  const double *src[4] = {bu, bv, bw, bp};
  for (int g = 0; g < 4; g++) {
    if (!src[g]) continue;
    for (long q = 0; q < L->W3; q++) {
      long p = g * L->W3 + q;
      int c = L->cls[p];
      if (c == C_GHOST || c == C_WALLG || c == C_WALLD) L->b[p] = src[g][q];
      if (c == C_GHOSTX) L->b[p] = 0.0;
    }
  }
}
/* right-hand sides of the internal rows (u, v, w momentum and continuity), mean row 0 */
void o3_set_rhs(void *h, const double *fu, const double *fv, const double *fw, const double *g) {
  S3 *S = (S3 *)h;
  L3 *L = &S->lev[0];
  const double *src[4] = {fu, fv, fw, g};
  for (int gg = 0; gg < 4; gg++)
    for (long q = 0; q < L->W3; q++) {
      long p = gg * L->W3 + q;
      if (L->cls[p] == C_INT) L->b[p] = src[gg] ? src[gg][q] : 0.0;
    }
  L->b[4 * L->W3] = 0.0;
}
void o3_set_x(void *h, const double *x) {
  L3 *L = &((S3 *)h)->lev[0];
  memcpy(L->x, x, sizeof(double) * L->n);
}
void o3_get_x(void *h, double *x) {
  L3 *L = &((S3 *)h)->lev[0];
  memcpy(x, L->x, sizeof(double) * L->n);
}
void o3_get_b(void *h, double *b) {
  L3 *L = &((S3 *)h)->lev[0];
  memcpy(b, L->b, sizeof(double) * L->n);
}
int o3_relax(void *h, int l, int steps) {
  S3 *S = (S3 *)h;
  if (!S->have_geom) return E_INVAL;
  for (int q = 0; q < steps; q++) relax_step(S, &S->lev[l]);
  return OK;
}
int o3_residual(void *h, double *r, double *res_inf) {
  S3 *S = (S3 *)h;
  if (!S->have_geom) return E_INVAL;
  L3 *L = &S->lev[0];
  double m = residual(S, L, L->x, L->b, L->r);
  if (r) memcpy(r, L->r, sizeof(double) * L->n);
  if (res_inf) *res_inf = m;
  return OK;
}
int o3_res_history(void *h, double *out, int n) {
  S3 *S = (S3 *)h;
  int m = S->nhist < n ? S->nhist : n;
  memcpy(out, S->hist, sizeof(double) * m);
  return m;
}
/* the finest matrix in CSR (rows and columns: the 4 W^3 + 1 entries; rows without an equation are identity
 * rows with a zero right-hand side, so the matrix is square and nonsingular) */
int o3_csr_size(void *h, int *n, long *nnz) {
  S3 *S = (S3 *)h;
  if (!S->have_geom) return E_INVAL;
  L3 *L = &S->lev[0];
  long cnt = 0;
  for (long p = 0; p < 4 * L->W3; p++) {
    int c = L->cls[p];
    cnt += rowed(c) ? 27 : (c == C_INT ? 10 : 1);
  }
  cnt += L->Mp;
  *n = (int)L->n;
  *nnz = cnt;
  return OK;
}
int o3_csr(void *h, long *rp, int *ci, double *va, double *b) {
  S3 *S = (S3 *)h;
  if (!S->have_geom) return E_INVAL;
  L3 *L = &S->lev[0];
  long P = 4 * L->W3, e = 0;
  for (long p = 0; p < P; p++) {
    rp[p] = e;
    int c = L->cls[p];
    b[p] = L->b[p];
    if (rowed(c)) {
      int r = L->rowof[p];
      for (int q = 0; q < 27; q++) {
        ci[e] = L->g_col[27L * r + q];
        va[e++] = L->g_w[27L * r + q];
      }
    } else if (c == C_INT) {
      int g, i, j, k;
      unpack(L, p, &g, &i, &j, &k);
      long cols[9];
      int m = int_row_cols(L, g, i, j, k, cols);
      for (int q = 0; q < m; q++) {
        ci[e] = (int)cols[q];
        va[e++] = row_coef(S, L, p, cols[q]);
      }
      if (g == 3) {
        ci[e] = (int)P;
        va[e++] = -1.0;
      }
    } else {
      ci[e] = (int)p;
      va[e++] = 1.0;
      if (c != C_WALLD) b[p] = 0.0;
    }
  }
  rp[P] = e;
  for (long q = 3 * L->W3; q < P; q++)
    if (L->cls[q] == C_INT) {
      ci[e] = (int)q;
      va[e++] = 1.0 / L->Mp;
    }
  b[P] = L->b[P];
  rp[P + 1] = e;
  return OK;
}
