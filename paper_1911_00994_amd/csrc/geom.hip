// Geometry on the device: level-set sampling, classification of the three staggered grids, ghost closure,
// Alg. 1 boundary points, ghost rows (eq. (BCu) and its normal derivative), extension points, and the exact
// factorisation of the coarsest system.  Arithmetic is kept in FP64 everywhere (small cut cells make the
// ghost coefficients ill-conditioned); this file is built with FMA contraction off so that the branch
// decisions of the bisection see the same roundings as a plain IEEE evaluation.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>

#include <thread>

#include "internal.h"

namespace gpmg {

// ---------------------------------------------------------------------------------------------------------
// lattice view of one level: phi of the level at lattice index (kx, ky), kx, ky in [0, 2N]
// ---------------------------------------------------------------------------------------------------------
struct Lat {
  const double *phi;
  int Lf;  // fine lattice points per axis
  int s;   // stride
  int N;   // level cells
  double h;
};

__device__ __forceinline__ double lat_at(const Lat &L, int kx, int ky) {
  return L.phi[(size_t)(ky * L.s) * L.Lf + (size_t)(kx * L.s)];
}

__device__ __forceinline__ double sgn1(double z) { return z >= 0.0 ? 1.0 : -1.0; }

// bilinear interpolant of phi on the lattice cell containing (x, y) (half-open cells, clamped), value and gradient
__device__ void bilin(const Lat &L, double x, double y, double *val, double *gx, double *gy) {
  const double hl = 0.5 * L.h;
  const int nl = 2 * L.N + 1;
  double fx = (x + 1.0) / hl, fy = (y + 1.0) / hl;
  int kx = (int)floor(fx), ky = (int)floor(fy);
  kx = kx < 0 ? 0 : (kx > nl - 2 ? nl - 2 : kx);
  ky = ky < 0 ? 0 : (ky > nl - 2 ? nl - 2 : ky);
  double tx = fx - kx, ty = fy - ky;
  double p00 = lat_at(L, kx, ky), p10 = lat_at(L, kx + 1, ky), p01 = lat_at(L, kx, ky + 1), p11 = lat_at(L, kx + 1, ky + 1);
  if (val) *val = (1 - tx) * (1 - ty) * p00 + tx * (1 - ty) * p10 + (1 - tx) * ty * p01 + tx * ty * p11;
  if (gx) *gx = ((1 - ty) * (p10 - p00) + ty * (p11 - p01)) / hl;
  if (gy) *gy = ((1 - tx) * (p01 - p00) + tx * (p11 - p10)) / hl;
}

__device__ void normal_at(const Lat &L, double x, double y, double *nx, double *ny) {
  double gx, gy;
  bilin(L, x, y, nullptr, &gx, &gy);
  double m = sqrt(gx * gx + gy * gy);
  if (m > 0) {
    *nx = gx / m;
    *ny = gy / m;
  } else {
    *nx = 0;
    *ny = 0;
  }
}

// node (g, i, j): coordinates and lattice indices
__device__ __forceinline__ void node_pos(int g, int i, int j, double h, double *x, double *y) {
  *x = (g == 0) ? -1.0 + i * h : -1.0 + (i + 0.5) * h;
  *y = (g == 1) ? -1.0 + j * h : -1.0 + (j + 0.5) * h;
}
__device__ __forceinline__ void node_lat(int g, int i, int j, int *kx, int *ky) {
  *kx = (g == 0) ? 2 * i : 2 * i + 1;
  *ky = (g == 1) ? 2 * j : 2 * j + 1;
}
__device__ __forceinline__ bool inside(int N, int i, int j) { return i >= -1 && i <= N && j >= -1 && j <= N; }
__device__ __forceinline__ int gix(int W, int g, int i, int j) { return g * W * W + (j + 1) * W + (i + 1); }
__device__ __forceinline__ uint8_t cls_of(const uint8_t *cls, int N, int W, int g, int i, int j) {
  return inside(N, i, j) ? cls[gix(W, g, i, j)] : (uint8_t)K_INACTIVE;
}
__device__ __forceinline__ bool has_value(uint8_t c) {
  return c == K_INT || c == K_GHOST || c == K_WALLD || c == K_WALLG || c == K_GHOSTX;
}

// ---------------------------------------------------------------------------------------------------------
// level set (Sect. 3.1; shapes of eq. (eq:domains); rigid motion of Sect. 5)
// ---------------------------------------------------------------------------------------------------------
__device__ double shape_value(int kind, double a0, double a1, double a2, double a3, double xb, double yb) {
  if (kind == 0) return a0 - sqrt(xb * xb + yb * yb);
  if (kind == 1) return a0 * a0 - (xb * xb + yb * yb);
  if (kind == 2 || kind == 3) {
    double c = cos(a2), s = sin(a2);
    double xr = c * xb - s * yb, yr = s * xb + c * yb;
    double q = xr * xr / (a0 * a0) + yr * yr / (a1 * a1);
    return kind == 2 ? 1.0 - q : 1.0 - sqrt(q);
  }
  if (kind == 4) {
    double r = sqrt(xb * xb + yb * yb);
    if (r == 0.0) return a0 + a1;
    return a0 + a1 * cos(a3 * (atan2(yb, xb) - a2)) - r;
  }
  return -1.0;
}

__global__ void k_levelset(double *phi, int N, int kind, double a0, double a1, double a2, double a3, double X, double Y,
                           double ang) {
  int nl = 2 * N + 1;
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)nl * nl) return;
  int kx = (int)(t % nl), ky = (int)(t / nl);
  double hl = 1.0 / N;
  double x = -1.0 + kx * hl - X, y = -1.0 + ky * hl - Y;
  double c = cos(ang), s = sin(ang);
  phi[t] = shape_value(kind, a0, a1, a2, a3, c * x + s * y, -s * x + c * y);
}

// ---------------------------------------------------------------------------------------------------------
// classification (Alg. LS: internal iff phi(P) < 0, each grid on its own)
// ---------------------------------------------------------------------------------------------------------
__global__ void k_classify(Lat L, uint8_t *cls, int W, int finest, int *flags) {
  int N = L.N;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * W * W) return;
  int g = t / (W * W), loc = t % (W * W), j = loc / W - 1, i = loc % W - 1;
  uint8_t c = K_INACTIVE;
  int kx, ky;
  node_lat(g, i, j, &kx, &ky);
  if (g == 0) {
    if ((i == 0 || i == N) && j >= 0 && j <= N - 1)
      c = K_WALLD;
    else if ((j == -1 || j == N) && i >= 1 && i <= N - 1)
      c = K_WALLG;
    else if (i >= 1 && i <= N - 1 && j >= 0 && j <= N - 1)
      c = lat_at(L, kx, ky) < 0 ? K_INT : K_BODY;
  } else if (g == 1) {
    if ((j == 0 || j == N) && i >= 0 && i <= N - 1)
      c = K_WALLD;
    else if ((i == -1 || i == N) && j >= 1 && j <= N - 1)
      c = K_WALLG;
    else if (i >= 0 && i <= N - 1 && j >= 1 && j <= N - 1)
      c = lat_at(L, kx, ky) < 0 ? K_INT : K_BODY;
  } else {
    if (i >= 0 && i <= N - 1 && j >= 0 && j <= N - 1) c = lat_at(L, kx, ky) < 0 ? K_INT : K_BODY;
  }
  if (finest && c == K_WALLD && lat_at(L, kx, ky) >= 0) atomicOr(&flags[1], 1);
  cls[t] = c;
}

__device__ __forceinline__ void to_ghost(uint8_t *cls, int N, int W, int g, int i, int j, int *changed) {
  if (!inside(N, i, j)) return;
  int k = gix(W, g, i, j);
  if (cls[k] == K_BODY) {
    cls[k] = K_GHOST;
    if (changed) *changed = 1;
  }
}

// external points used by internal equations become ghosts (Sect. 3.3)
__global__ void k_seed(uint8_t *cls, int N, int W) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * W * W) return;
  if (cls[t] != K_INT) return;
  int g = t / (W * W), loc = t % (W * W), j = loc / W - 1, i = loc % W - 1;
  if (g == 0) {
    to_ghost(cls, N, W, 0, i - 1, j, nullptr);
    to_ghost(cls, N, W, 0, i + 1, j, nullptr);
    to_ghost(cls, N, W, 0, i, j - 1, nullptr);
    to_ghost(cls, N, W, 0, i, j + 1, nullptr);
    to_ghost(cls, N, W, 2, i - 1, j, nullptr);
    to_ghost(cls, N, W, 2, i, j, nullptr);
  } else if (g == 1) {
    to_ghost(cls, N, W, 1, i - 1, j, nullptr);
    to_ghost(cls, N, W, 1, i + 1, j, nullptr);
    to_ghost(cls, N, W, 1, i, j - 1, nullptr);
    to_ghost(cls, N, W, 1, i, j + 1, nullptr);
    to_ghost(cls, N, W, 2, i, j - 1, nullptr);
    to_ghost(cls, N, W, 2, i, j, nullptr);
  } else {
    to_ghost(cls, N, W, 0, i, j, nullptr);
    to_ghost(cls, N, W, 0, i + 1, j, nullptr);
    to_ghost(cls, N, W, 1, i, j, nullptr);
    to_ghost(cls, N, W, 1, i, j + 1, nullptr);
  }
}

// external points of the upwind nine-point stencil of a ghost are ghosts too (closure, Sect. 3.3)
__global__ void k_closure(Lat L, uint8_t *cls, int W, int *changed) {
  int N = L.N;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * W * W) return;
  if (cls[t] != K_GHOST) return;
  int g = t / (W * W), loc = t % (W * W), j = loc / W - 1, i = loc % W - 1;
  double x, y, nx, ny;
  node_pos(g, i, j, L.h, &x, &y);
  normal_at(L, x, y, &nx, &ny);
  int sx = (int)sgn1(nx), sy = (int)sgn1(ny);
  for (int ky = 0; ky < 3; ky++)
    for (int kx = 0; kx < 3; kx++) to_ghost(cls, N, W, g, i - sx * kx, j - sy * ky, changed);
}

// external points within R index steps (max norm) of an internal point of the same grid carry extension values;
// the window is taken in two passes: rowint = an internal point within R steps along the row (k_ext_rows_int),
// then a body point is near if rowint holds within R steps along its column (k_ext_mark)
__global__ void k_ext_rows_int(const uint8_t *cls, int N, int W, int R, uint8_t *rowint) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * W * W) return;
  int g = t / (W * W), loc = t % (W * W), j = loc / W - 1, i = loc % W - 1;
  bool any = false;
  for (int di = -R; di <= R; di++) any = any || cls_of(cls, N, W, g, i + di, j) == K_INT;
  rowint[t] = any ? 1 : 0;
}
__global__ void k_ext_mark(uint8_t *cls, int N, int W, int R, const uint8_t *rowint) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * W * W) return;
  if (cls[t] != K_BODY) return;
  int g = t / (W * W), loc = t % (W * W), j = loc / W - 1, i = loc % W - 1;
  bool near = false;
  for (int dj = -R; dj <= R && !near; dj++) near = inside(N, i, j + dj) && rowint[gix(W, g, i, j + dj)];
  // a point never reads another point's BODY/EXT state here, so the in-place update is race free
  cls[t] = near ? K_EXT : K_BODY;
}
__global__ void k_body_to_inactive(uint8_t *cls, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n && cls[t] == K_BODY) cls[t] = K_INACTIVE;
}

// compaction (order does not matter: every consumer of these lists is order independent)
__global__ void k_compact(const uint8_t *cls, int n, int mode, int *list, int cap, int *counter) {
  __shared__ int woff[TPB / 64];
  __shared__ int bbase;
  const int t = blockIdx.x * blockDim.x + threadIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  bool take = false;
  if (t < n) {
    const uint8_t c = cls[t];
    take = (mode == 0) ? (c == K_GHOST || c == K_WALLG) : (c == K_EXT);
  }
  // one atomic per block: the block's takers get consecutive slots, wavefront by wavefront
  const unsigned long long m = __ballot(take);
  if (lane == 0) woff[wv] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < TPB / 64; w++) {
      const int c = woff[w];
      woff[w] = tot;
      tot += c;
    }
    bbase = tot ? atomicAdd(counter, tot) : 0;
  }
  __syncthreads();
  if (take) {
    const int slot = bbase + woff[wv] + __popcll(m & ((1ull << lane) - 1));
    if (slot < cap) list[slot] = t;
  }
}

// ---------------------------------------------------------------------------------------------------------
// ghost rows
// ---------------------------------------------------------------------------------------------------------
__device__ __forceinline__ void lagr3(double t, double T[3]) {
  T[0] = (1 - t) * (2 - t) / 2;
  T[1] = t * (2 - t);
  T[2] = t * (t - 1) / 2;
}
__device__ __forceinline__ void dlagr3(double t, double D[3]) {
  D[0] = t - 1.5;
  D[1] = 2 - 2 * t;
  D[2] = t - 0.5;
}

// Alg. 1 (march along the bilinear normal by h/2, then bisection on the last segment); returns success.  With rec
// given, the discrete path is recorded: rec[0] = march steps (+ 65536 when the march ends exactly on the zero set),
// rec[1] bit q set when bisection step q moved the inner end of the bracket
__device__ bool boundary_point(const Lat &L, double xg, double yg, double phig, int march_max, int nbis, double *Bx,
                               double *By, unsigned *rec = nullptr) {
  double hx = xg, hy = yg, ph = phig, kx = xg, ky = yg;
  int it = 0;
  while (ph > 0) {
    if (it == march_max) return false;
    kx = hx;
    ky = hy;
    double nx, ny;
    normal_at(L, hx, hy, &nx, &ny);
    hx = hx - 0.5 * L.h * nx;
    hy = hy - 0.5 * L.h * ny;
    bilin(L, hx, hy, &ph, nullptr, nullptr);
    it++;
  }
  if (rec) {
    rec[0] = (unsigned)it + (ph == 0.0 ? 65536u : 0u);
    rec[1] = 0;
  }
  if (it == 0 || ph == 0.0) {
    *Bx = hx;
    *By = hy;
    return true;
  }
  double bx = hx, by = hy;
  for (int q = 0; q < nbis; q++) {
    bx = 0.5 * (hx + kx);
    by = 0.5 * (hy + ky);
    double pb;
    bilin(L, bx, by, &pb, nullptr, nullptr);
    if (pb * ph < 0) {
      kx = bx;
      ky = by;
      if (rec) rec[1] |= 1u << q;
    } else {
      hx = bx;
      hy = by;
      ph = pb;
    }
  }
  *Bx = bx;
  *By = by;
  return true;
}

struct RowArgs {
  int *g_pt, *g_col;
  double *g_w, *g_dtau, *g_B, *g_nB, *g_th;
  int8_t *g_kind;
  int ng;
};

// pass A: wall-ghost rows and boundary-condition rows; unusable rows turn their point into GHOSTX
__global__ void k_ghost_rows(Lat L, uint8_t *cls, int W, RowArgs R, int march_max, int nbis, double cg_min,
                             double dtau_dir, double dtau_neu) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R.ng) return;
  int N = L.N;
  double h = L.h;
  int k = R.g_pt[r];
  int g = k / (W * W), loc = k % (W * W), j = loc / W - 1, i = loc % W - 1;
  uint8_t c = cls[k];
  int col[9];
  double w[9];
  for (int q = 0; q < 9; q++) {
    col[q] = k;
    w[q] = 0;
  }
  double xg, yg;
  node_pos(g, i, j, h, &xg, &yg);
  bool ok = true;
  double Bx = xg, By = yg, nbx = 0, nby = 0, thx = 0, thy = 0, dtau = dtau_dir;
  if (c == K_WALLG) {
    // tangential velocity on the box wall: eq. (BCu) with exact wall geometry (theta_n = 1/2, theta_t = 0)
    int di = 0, dj = 0;
    if (g == 0) {
      dj = (j == -1) ? 1 : -1;
      By = (j == -1) ? -1.0 : 1.0;
      nby = (j == -1) ? -1.0 : 1.0;
      thy = 0.5;
    } else {
      di = (i == -1) ? 1 : -1;
      Bx = (i == -1) ? -1.0 : 1.0;
      nbx = (i == -1) ? -1.0 : 1.0;
      thx = 0.5;
    }
    double T[3];
    lagr3(0.5, T);
    for (int q = 0; q < 3; q++) {
      col[q] = gix(W, g, i + q * di, j + q * dj);
      w[q] = T[q];
      if (q > 0 && cls[col[q]] != K_INT) ok = false;
    }
  } else {
    int kx, ky;
    node_lat(g, i, j, &kx, &ky);
    double phig = lat_at(L, kx, ky);
    double ngx, ngy;
    normal_at(L, xg, yg, &ngx, &ngy);
    double sx = sgn1(ngx), sy = sgn1(ngy);
    ok = boundary_point(L, xg, yg, phig, march_max, nbis, &Bx, &By);
    thx = sx * (xg - Bx) / h;
    thy = sy * (yg - By) / h;
    normal_at(L, Bx, By, &nbx, &nby);
    for (int ky2 = 0; ky2 < 3; ky2++)
      for (int kx2 = 0; kx2 < 3; kx2++) {
        int ii = i - (int)sx * kx2, jj = j - (int)sy * ky2;
        if (!inside(N, ii, jj)) {
          ok = false;
          continue;
        }
        col[ky2 * 3 + kx2] = gix(W, g, ii, jj);
        if (!has_value(cls[col[ky2 * 3 + kx2]])) ok = false;
      }
    double Tx[3], Ty[3];
    lagr3(thx, Tx);
    lagr3(thy, Ty);
    if (g < 2) {
      for (int ky2 = 0; ky2 < 3; ky2++)
        for (int kx2 = 0; kx2 < 3; kx2++) w[ky2 * 3 + kx2] = Tx[kx2] * Ty[ky2];
    } else {
      double Dx[3], Dy[3];
      dlagr3(thx, Dx);
      dlagr3(thy, Dy);
      for (int ky2 = 0; ky2 < 3; ky2++)
        for (int kx2 = 0; kx2 < 3; kx2++)
          w[ky2 * 3 + kx2] = -(nbx * sx * Dx[kx2] * Ty[ky2] + nby * sy * Tx[kx2] * Dy[ky2]) / h;
      dtau = dtau_neu;
    }
    if (!(thx > -0.5 && thx < 1.0 && thy > -0.5 && thy < 1.0)) ok = false;
    if (!((g < 2 ? w[0] : w[0] * h) > cg_min)) ok = false;
  }
  for (int q = 0; q < 9; q++) {
    R.g_col[9 * r + q] = col[q];
    R.g_w[9 * r + q] = w[q];
  }
  R.g_dtau[r] = dtau;
  R.g_B[2 * r] = Bx;
  R.g_B[2 * r + 1] = By;
  R.g_nB[2 * r] = nbx;
  R.g_nB[2 * r + 1] = nby;
  R.g_th[2 * r] = thx;
  R.g_th[2 * r + 1] = thy;
  R.g_kind[r] = ok ? 1 : 0;
  if (!ok) cls[k] = K_GHOSTX;
}

// quadratic extrapolation from the first three internal / boundary-condition points met towards the fluid,
// along the grid axis closest to the normal (the other axis as a second choice)
__device__ bool extrap_src(const Lat &L, const uint8_t *cls, int W, int g, int i, int j, int src[3], double w[3]) {
  int N = L.N;
  double x, y, nx, ny;
  node_pos(g, i, j, L.h, &x, &y);
  normal_at(L, x, y, &nx, &ny);
  int first = fabs(nx) >= fabs(ny) ? 0 : 1;
  for (int a = 0; a < 2; a++) {
    int ax = (a == 0) ? first : 1 - first;
    int s = (int)sgn1(ax == 0 ? nx : ny);
    int di = ax == 0 ? -s : 0, dj = ax == 1 ? -s : 0;
    int k0 = 0;
    for (int q = 1; q <= 4; q++) {
      uint8_t c = cls_of(cls, N, W, g, i + q * di, j + q * dj);
      if (c == K_INT || c == K_GHOST) {
        k0 = q;
        break;
      }
    }
    if (!k0) continue;
    bool good = true;
    for (int q = 0; q < 3; q++) {
      uint8_t c = cls_of(cls, N, W, g, i + (k0 + q) * di, j + (k0 + q) * dj);
      if (!(c == K_INT || c == K_GHOST)) good = false;
    }
    if (!good) continue;
    double kk = k0;
    w[0] = (kk + 1) * (kk + 2) / 2;
    w[1] = -kk * (kk + 2);
    w[2] = kk * (kk + 1) / 2;
    for (int q = 0; q < 3; q++) src[q] = gix(W, g, i + (k0 + q) * di, j + (k0 + q) * dj);
    return true;
  }
  return false;
}

// pass B: extrapolation rows x_G - sum w x_src = 0 for GHOSTX points (identity x_G = 0 when no source exists)
__global__ void k_ghostx_rows(Lat L, const uint8_t *cls, int W, RowArgs R, int finest, int *flags) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R.ng) return;
  int k = R.g_pt[r];
  if (cls[k] != K_GHOSTX) return;
  int g = k / (W * W), loc = k % (W * W), j = loc / W - 1, i = loc % W - 1;
  for (int q = 0; q < 9; q++) {
    R.g_col[9 * r + q] = k;
    R.g_w[9 * r + q] = 0;
  }
  R.g_w[9 * r] = 1.0;
  R.g_dtau[r] = 1.0;
  int src[3];
  double w[3];
  if (extrap_src(L, cls, W, g, i, j, src, w)) {
    for (int q = 0; q < 3; q++) {
      R.g_col[9 * r + 1 + q] = src[q];
      R.g_w[9 * r + 1 + q] = -w[q];
    }
    R.g_kind[r] = 2;
  } else {
    R.g_kind[r] = 0;
    if (finest) atomicAdd(&flags[4], 1);
  }
}

__global__ void k_ext_rows(Lat L, uint8_t *cls, int W, const int *e_pt, int ne, int *e_src, double *e_w) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int k = e_pt[e];
  int g = k / (W * W), loc = k % (W * W), j = loc / W - 1, i = loc % W - 1;
  int src[3];
  double w[3];
  if (extrap_src(L, cls, W, g, i, j, src, w)) {
    for (int q = 0; q < 3; q++) {
      e_src[3 * e + q] = src[q];
      e_w[3 * e + q] = w[q];
    }
  } else {
    for (int q = 0; q < 3; q++) {
      e_src[3 * e + q] = -1;
      e_w[3 * e + q] = 0;
    }
  }
}
// points whose extension has no source carry no value (separate pass: extrap_src above reads only INT/GHOST)
__global__ void k_ext_fail(uint8_t *cls, const int *e_pt, int ne, const int *e_src) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  if (e_src[3 * e] < 0) cls[e_pt[e]] = K_INACTIVE;
}

__global__ void k_count_mp(const uint8_t *cls, int W, int *mp) {
  int n = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < W * W; t += gridDim.x * blockDim.x)
    n += cls[2 * W * W + t] == K_INT;
  for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
  __shared__ int sn[TPB / 64];
  if ((threadIdx.x & 63) == 0) sn[threadIdx.x >> 6] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0;
    for (int q = 0; q < TPB / 64; q++) c += sn[q];
    if (c) atomicAdd(mp, c);
  }
}

// finest level: every internal cell needs an internal face (else its box has no velocity unknown)
__global__ void k_empty_cells(const uint8_t *cls, int N, int W, int *flags) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * N) return;
  int i = t % N, j = t / N;
  if (cls[gix(W, 2, i, j)] != K_INT) return;
  int nf = (cls[gix(W, 0, i, j)] == K_INT) + (cls[gix(W, 0, i + 1, j)] == K_INT) + (cls[gix(W, 1, i, j)] == K_INT) +
           (cls[gix(W, 1, i, j + 1)] == K_INT);
  if (nf == 0) atomicOr(&flags[1], 2);
}

// boundary band: cells with at least one internal box unknown within R cells (max norm) of a cell touching the
// body (one of its five box unknowns is neither internal nor a wall point); counted / listed per colour
__device__ bool cut_cell(const uint8_t *cls, int W, int i, int j) {
  int WW = W * W, c = (j + 1) * W + (i + 1);
  uint8_t k[5] = {cls[c], cls[c + 1], cls[WW + c], cls[WW + c + W], cls[2 * WW + c]};
  for (int q = 0; q < 5; q++)
    if (k[q] != K_INT && k[q] != K_WALLD) return true;
  return false;
}
// exclusive prefix sum over the block (and the block's total): wavefront shuffles, then the wavefronts' sums
__device__ int block_excl_scan(int v, int *total) {
  __shared__ int ws[TPB / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) ws[wv] = x;
  __syncthreads();
  int off = 0, tot = 0;
  for (int w = 0; w < TPB / 64; w++) {
    if (w < wv) off += ws[w];
    tot += ws[w];
  }
  *total = tot;
  __syncthreads();  // ws is reused by the next call
  return off + x - v;
}
// cut flags of the cells (one byte each), then each cell's band colour from them (-1: not in the band)
__global__ void k_band_cut(const uint8_t *cls, int N, int W, uint8_t *cut) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N * N) cut[t] = cut_cell(cls, W, t % N, t / N) ? 1 : 0;
}
__device__ __forceinline__ int band_colour(const uint8_t *cls, const uint8_t *cut, int N, int W, int R, int t) {
  int i = t % N, j = t / N, WW = W * W, c = (j + 1) * W + (i + 1);
  bool any = cls[c] == K_INT || cls[c + 1] == K_INT || cls[WW + c] == K_INT || cls[WW + c + W] == K_INT ||
             cls[2 * WW + c] == K_INT;
  if (!any) return -1;
  for (int dj = -R; dj <= R; dj++) {
    const int b = j + dj;
    if (b < 0 || b >= N) continue;
    for (int di = -R; di <= R; di++) {
      const int a = i + di;
      if (a >= 0 && a < N && cut[b * N + a]) return (i + 2 * j) % 5;
    }
  }
  return -1;
}
// this thread's rank among the block's cells of its colour (index order) and, in tot, the block's count per
// colour: wavefront ballots, then the wavefronts' counts in order
__device__ __forceinline__ int colour_rank(int col, int tot[5]) {
  __shared__ int wc[5][TPB / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int rank = 0;
  unsigned long long mine = 0;
  for (int c = 0; c < 5; c++) {
    const unsigned long long m = __ballot(col == c);
    if (lane == 0) wc[c][wv] = __popcll(m);
    if (col == c) mine = m;
  }
  __syncthreads();
  for (int c = 0; c < 5; c++) {
    int t = 0;
    for (int w = 0; w < TPB / 64; w++) {
      if (c == col && w < wv) rank += wc[c][w];
      t += wc[c][w];
    }
    tot[c] = t;
  }
  __syncthreads();
  return rank + (col >= 0 ? __popcll(mine & ((1ull << lane) - 1)) : 0);
}

// deterministic compaction: per-block counts, one scan of the block counts (k_scan_blocks), fill in index order;
// the colours go to col8 between the two passes
__global__ void __launch_bounds__(TPB) k_band_count(const uint8_t *cls, const uint8_t *cut, int N, int W, int R, int nb,
                                                    int *bcnt, int8_t *col8) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  const int col = t < N * N ? band_colour(cls, cut, N, W, R, t) : -1;
  if (t < N * N) col8[t] = (int8_t)col;
  int tot[5];
  (void)colour_rank(col, tot);
  if (threadIdx.x == 0)
    for (int c = 0; c < 5; c++) bcnt[c * nb + blockIdx.x] = tot[c];
}
// band cells grouped by colour, ascending cell index within a colour
__global__ void __launch_bounds__(TPB) k_band_fill(int N, int nb, const int8_t *col8, const int *boff, int *band) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  const int col = t < N * N ? col8[t] : -1;
  int tot[5];
  const int r = colour_rank(col, tot);
  if (col >= 0) band[boff[col * nb + blockIdx.x] + r] = t;
}
// colour offsets of the band (from the scanned counts) into out[0..5]
__global__ void k_band_offsets(const int *boff, int nb, int *out) {
  int c = threadIdx.x;
  if (c < 5) out[c] = boff[c * nb];
  if (c == 5) out[5] = boff[5 * nb];
}

// ---- boundary region tables for the LDS band kernel ----
// the 21 values a box update reads around cell index c (u: W E WW EE WS WN ES EN; v: S N SS NN SW SE NW NE;
// p: c W E S N) as global indices
__device__ __forceinline__ void box_points(int W, int c, int out[21]) {
  int WW = W * W;
  int q = 0;
  out[q++] = c;          // uW
  out[q++] = c + 1;      // uE
  out[q++] = c - 1;      // uWW
  out[q++] = c + 2;      // uEE
  out[q++] = c - W;      // uWS
  out[q++] = c + W;      // uWN
  out[q++] = c + 1 - W;  // uES
  out[q++] = c + 1 + W;  // uEN
  out[q++] = WW + c;          // vS
  out[q++] = WW + c + W;      // vN
  out[q++] = WW + c - W;      // vSS
  out[q++] = WW + c + 2 * W;  // vNN
  out[q++] = WW + c - 1;      // vSW
  out[q++] = WW + c + 1;      // vSE
  out[q++] = WW + c + W - 1;  // vNW
  out[q++] = WW + c + W + 1;  // vNE
  out[q++] = 2 * WW + c;      // p
  out[q++] = 2 * WW + c - 1;  // pW
  out[q++] = 2 * WW + c + 1;  // pE
  out[q++] = 2 * WW + c - W;  // pS
  out[q++] = 2 * WW + c + W;  // pN
}

__global__ void k_row_of(const int *g_pt, int ng, int *row_of) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < ng) row_of[g_pt[r]] = r;
}
// column-major copies of the ghost rows' columns (by row) and weights
__global__ void k_rows_t(const int *g_colr, const double *g_w, int ng, int *colr_t, double *w_t) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 9 * ng) return;
  const int r = e / 9, z = e - 9 * r;
  colr_t[(size_t)z * ng + r] = g_colr[e];
  w_t[(size_t)z * ng + r] = g_w[e];
}
// the columns of the ghost rows with every ghost point replaced by -(its row + 1) (row_of from k_row_of; every
// ghost, extrapolated-ghost and wall-ghost point has a row; a column whose row cannot be confirmed is reported)
__global__ void k_colr(const uint8_t *cls, const int *g_pt, const int *g_col, int ng, const int *row_of, int *g_colr,
                       int *bad) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 9 * ng) return;
  int c = g_col[e];
  uint8_t k = cls[c];
  if (k == K_GHOST || k == K_GHOSTX || k == K_WALLG) {
    int r = row_of[c];
    if (r >= 0 && r < ng && g_pt[r] == c) {
      g_colr[e] = -(r + 1);
      return;
    }
    atomicOr(bad, 1);
  }
  g_colr[e] = c;
}
__global__ void k_region_clear(int *map, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) map[t] = -1;
}
// mark: map[k] = -3 for every point the band kernel reads (the 21 values of a band box, the 9 columns of a body
// ghost row), wall ghost points excluded: the kernel's other workgroups write them.  Launched before k_region_mark,
// which marks the written points over these.
__global__ void k_region_mark_reads(const uint8_t *cls, int N, int W, const int *band, int nband, const int *g_pt,
                                    const int *g_col, int ng, int *map) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nband) {
    int cell = band[t], i = cell % N, j = cell / N, c = (j + 1) * W + (i + 1);
    int pts[21];
    box_points(W, c, pts);
    for (int q = 0; q < 21; q++)
      if (cls[pts[q]] != K_WALLG) map[pts[q]] = -3;
  } else if (t < nband + ng) {
    int r = t - nband;
    if (cls[g_pt[r]] == K_WALLG) return;
    for (int q = 0; q < 9; q++) {
      int c = g_col[9 * r + q];
      if (cls[c] != K_WALLG) map[c] = -3;
    }
  }
}
// mark: map[k] = -2 for every point the band kernel writes (the five unknowns of a band box, body ghost points);
// the points it only reads are constant during the kernel
__global__ void k_region_mark(const uint8_t *cls, int N, int W, const int *band, int nband, const int *g_pt, int ng,
                              int *map) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int WW = W * W;
  if (t < nband) {
    int cell = band[t], i = cell % N, j = cell / N, c = (j + 1) * W + (i + 1);
    map[c] = -2;
    map[c + 1] = -2;
    map[WW + c] = -2;
    map[WW + c + W] = -2;
    map[2 * WW + c] = -2;
  } else if (t < nband + ng) {
    int r = t - nband;
    if (cls[g_pt[r]] == K_WALLG) return;
    map[g_pt[r]] = -2;
  }
}
// written region points (mode 0), body ghost points (mode 1) and read-only region points (mode 2), each in
// ascending index order
__device__ __forceinline__ bool region_pred(int mode, const int *map, const uint8_t *cls, int t) {
  return mode == 0 ? map[t] == -2 : mode == 2 ? map[t] == -3 : (cls[t] == K_GHOST || cls[t] == K_GHOSTX);
}
__global__ void __launch_bounds__(TPB) k_pred_count(int mode, int n, const int *map, const uint8_t *cls, int *bcnt) {
  int t = blockIdx.x * TPB + threadIdx.x;
  int tot;
  block_excl_scan(t < n && region_pred(mode, map, cls, t) ? 1 : 0, &tot);
  if (threadIdx.x == 0) bcnt[blockIdx.x] = tot;
}
// out[*base + rank] = t for the points that satisfy the predicate (base: a device count, or null for 0)
__global__ void __launch_bounds__(TPB) k_pred_fill(int mode, int n, const int *map, const uint8_t *cls, const int *boff,
                                                   int cap, int *out, const int *base) {
  int t = blockIdx.x * TPB + threadIdx.x;
  bool take = t < n && region_pred(mode, map, cls, t);
  int tot;
  int q = (base ? *base : 0) + boff[blockIdx.x] + block_excl_scan(take ? 1 : 0, &tot);
  if (take && q < cap) out[q] = t;
}
__global__ void k_region_slots(const int *reg_pt, int nreg, int *map) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nreg) map[reg_pt[q]] = q;
}
// per band box, fields stored field-major (field f of box q at f * cap + q): the local indices of its 21 values
// (LDS slot, or -(global index + 1) for a point the kernel only reads), the flags of its free unknowns (bits
// W E S N P) and its cell index
__global__ void k_region_boxes(const uint8_t *cls, int N, int W, const int *band, int nband, const int *map, int cap,
                               int *bbox, int *bad) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nband) return;
  int cell = band[t], i = cell % N, j = cell / N, WW = W * W, c = (j + 1) * W + (i + 1);
  int pts[21];
  box_points(W, c, pts);
  for (int q = 0; q < 21; q++) {
    int l = map[pts[q]];
    bbox[q * cap + t] = l >= 0 ? l : -(pts[q] + 1);
    if (cls[pts[q]] == K_WALLG) atomicOr(bad, 8);  // wall ghosts are swept apart from the band
  }
  int f = (cls[c] == K_INT ? 1 : 0) | (cls[c + 1] == K_INT ? 2 : 0) | (cls[WW + c] == K_INT ? 4 : 0) |
          (cls[WW + c + W] == K_INT ? 8 : 0) | (cls[2 * WW + c] == K_INT ? 16 : 0);
  bbox[21 * cap + t] = f;
  bbox[22 * cap + t] = cell;
}
// body ghost rows in point order, fields stored field-major: bg_loc (own slot, then the 9 stencil entries as
// local indices), bg_w (9 weights), bg_dt, and bg_k (the point, for its right-hand side); a body row that would
// read a wall ghost is reported (the LDS kernel then does not apply)
__global__ void k_region_rows(const uint8_t *cls, const int *g_col, const double *g_w, const double *g_dtau,
                              const int *row_of, const int *map, int nbg, int cap, const int *bg_k, int *bg_loc,
                              double *bg_w, double *bg_dt, int *bad) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nbg) return;
  int k = bg_k[s], r = row_of[k];
  bg_loc[s] = map[k];
  for (int q = 0; q < 9; q++) {
    int c = g_col[9 * r + q], l = map[c];
    if (cls[c] == K_WALLG) atomicOr(bad, 4);
    bg_loc[(1 + q) * cap + s] = l >= 0 ? l : -(c + 1);
    bg_w[q * cap + s] = g_w[9 * r + q];
  }
  bg_dt[s] = g_dtau[r];
}
// wall ghost rows (order free: each is relaxed on its own); a wall row whose nodes a band box writes or whose
// stencil holds another ghost is reported
__global__ void k_wall_rows(const uint8_t *cls, const int *g_pt, const int *g_col, int ng, const int *map, int nw,
                            int *wg_rows, int *count, int *bad) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ng) return;
  int k = g_pt[r];
  if (cls[k] != K_WALLG) return;
  auto written = [&](int c) { return map[c] >= 0 && map[c] < nw; };  // slots past nw are only read
  for (int q = 0; q < 9; q++) {
    int c = g_col[9 * r + q];
    if (c != k && (written(c) || cls[c] == K_GHOST || cls[c] == K_GHOSTX || cls[c] == K_WALLG)) atomicOr(bad, 2);
  }
  if (map[k] >= 0) atomicOr(bad, 2);  // no wall ghost point is in the region
  wg_rows[atomicAdd(count, 1)] = r;
}

// ---- faces on the boundary of the internal pressure cells ----
// The divergences of the internal cells sum to (sum over these faces of +-u) / h: every face shared by two
// internal cells enters twice with opposite signs.  The list is built in a fixed order (cell index, then E W N S)
// by a per-block count, a scan of the block counts and a fill.
// Wall Dirichlet faces are left out: their values are fixed during a solve, and their part of the sum is added
// to the sum of the continuity right-hand sides instead.
__device__ __forceinline__ int face_mask(const uint8_t *cls, int W, int i, int j) {
  const int WW = W * W, c = (j + 1) * W + (i + 1), cp = 2 * WW + c;
  if (cls[cp] != K_INT) return 0;
  return (cls[cp + 1] != K_INT && cls[c + 1] != K_WALLD ? 1 : 0) | (cls[cp - 1] != K_INT && cls[c] != K_WALLD ? 2 : 0) |
         (cls[cp + W] != K_INT && cls[WW + c + W] != K_WALLD ? 4 : 0) |
         (cls[cp - W] != K_INT && cls[WW + c] != K_WALLD ? 8 : 0);
}
__global__ void __launch_bounds__(TPB) k_face_count(const uint8_t *cls, int N, int W, int *bcnt) {
  int t = blockIdx.x * TPB + threadIdx.x;
  int m = t < N * N ? face_mask(cls, W, t % N, t / N) : 0;
  int tot;
  block_excl_scan(__popc(m), &tot);
  if (threadIdx.x == 0) bcnt[blockIdx.x] = tot;
}
// exclusive scan of nb block counts in place (one workgroup); the total goes to bcnt[nb]
constexpr int SCAN_T = 1024;
__global__ void __launch_bounds__(SCAN_T) k_scan_blocks(int *bcnt, int nb) {
  __shared__ int s[SCAN_T];
  int per = (nb + SCAN_T - 1) / SCAN_T, lo = threadIdx.x * per, hi = min(nb, lo + per);
  int sum = 0;
  for (int q = lo; q < hi; q++) sum += bcnt[q];
  s[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < SCAN_T; o <<= 1) {
    int a = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += a;
    __syncthreads();
  }
  int run = s[threadIdx.x] - sum;
  for (int q = lo; q < hi; q++) {
    int c = bcnt[q];
    bcnt[q] = run;
    run += c;
  }
  if (threadIdx.x == SCAN_T - 1) bcnt[nb] = s[SCAN_T - 1];
}
__global__ void __launch_bounds__(TPB) k_face_fill(const uint8_t *cls, int N, int W, const int *boff, int cap, int *f_code) {
  int t = blockIdx.x * TPB + threadIdx.x;
  int i = t % N, j = t / N;
  int m = t < N * N ? face_mask(cls, W, i, j) : 0;
  int tot;
  int q = boff[blockIdx.x] + block_excl_scan(__popc(m), &tot);
  if (!m) return;
  const int WW = W * W, c = (j + 1) * W + (i + 1);
  // E (u, +), W (u, -), N (v, +), S (v, -)
  if ((m & 1) && q < cap) f_code[q++] = 2 * (c + 1);
  if ((m & 2) && q < cap) f_code[q++] = 2 * c + 1;
  if ((m & 4) && q < cap) f_code[q++] = 2 * (WW + c + W);
  if ((m & 8) && q < cap) f_code[q++] = 2 * (WW + c) + 1;
}
__global__ void k_face_loc(const int *f_code, int nf, const int *map, int *f_loc) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nf) return;
  int g = f_code[q] >> 1, l = map[g];
  f_loc[q] = l >= 0 ? l : -(g + 1);
}

// ---------------------------------------------------------------------------------------------------------
// boundary data of the finest level
// ---------------------------------------------------------------------------------------------------------
// body rows: u_b(B) = V + omega x (B - X(t)) with the path X(t) = X0 + U t (V = U plus the boundary-velocity offset)
__global__ void k_bvals_rows(const uint8_t *cls, int W, RowArgs R, double *b, double X0x, double X0y, double Ux, double Uy,
                             double om, double t, double Vx, double Vy, double wbu, double wtu, double wlv, double wrv) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R.ng) return;
  int k = R.g_pt[r];
  int g = k / (W * W), loc = k % (W * W), j = loc / W - 1, i = loc % W - 1;
  uint8_t c = cls[k];
  double val = 0;
  if (c == K_GHOST) {
    double X = X0x + Ux * t, Y = X0y + Uy * t;
    double Bx = R.g_B[2 * r], By = R.g_B[2 * r + 1];
    if (g == 0) val = Vx - om * (By - Y);
    if (g == 1) val = Vy + om * (Bx - X);
  } else if (c == K_WALLG) {
    if (g == 0) val = (j == -1) ? wbu : wtu;
    if (g == 1) val = (i == -1) ? wlv : wrv;
  }
  b[k] = val;
}
__global__ void k_bvals_points(const uint8_t *cls, int N, int W, double *b, double *x, double wlu, double wru, double wbv,
                               double wtv) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * W * W) return;
  uint8_t c = cls[t];
  if (c == K_INACTIVE || c == K_EXT) {
    b[t] = 0;
    return;
  }
  if (c != K_WALLD) return;
  int g = t / (W * W), loc = t % (W * W), j = loc / W - 1, i = loc % W - 1;
  double val = (g == 0) ? ((i == 0) ? wlu : wru) : ((j == 0) ? wbv : wtv);
  b[t] = val;
  x[t] = val;
  (void)N;
}

// ---------------------------------------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------------------------------------
// ---------------------------------------------------------------------------------------------------------
// coupled ghost boxes: a cell's box (Sect. 4.1.1: its pressure and its four faces) relaxed together with the body
// ghosts whose boundary rows weigh one of its internal unknowns.  Where such a weight dominates the ghost's own
// diagonal, the ghost row fixes the internal value and the internal equations fix the ghost value, and neither
// the box alone nor the fictitious-time step of eq. (ghostrelax) can resolve the pair.
// ---------------------------------------------------------------------------------------------------------
constexpr int XB_MAXM = 32;  // unknowns of one coupled box, at most
constexpr int XB_GCAP = 48;  // ghost entries gathered per box before duplicates are removed

// the cells whose box holds the internal point k: a u face separates cells (i-1, j) and (i, j), a v face (i, j-1)
// and (i, j); a pressure point belongs to its own cell
__device__ __forceinline__ int box_cells(int N, int W, int k, int cells[2]) {
  const int WW = W * W, g = k / WW, loc = k - g * WW, j = loc / W - 1, i = loc % W - 1;
  int n = 0;
  const int ci[2] = {g == 0 ? i - 1 : i, i}, cj[2] = {g == 1 ? j - 1 : j, j};
  for (int z = (g == 2 ? 1 : 0); z < 2; z++)
    if (ci[z] >= 0 && cj[z] >= 0 && ci[z] < N && cj[z] < N) cells[n++] = cj[z] * N + ci[z];
  return n;
}
__device__ __forceinline__ int cell_colour(int N, int cell) { return (cell % N + 2 * (cell / N)) % 5; }

// cells holding an internal column of a body ghost row
__global__ void k_xb_mark(const uint8_t *cls, int N, int W, const int *g_pt, const int *g_col, const double *g_w, int ng,
                          uint8_t *flag) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ng || cls[g_pt[r]] != K_GHOST) return;
  for (int z = 0; z < 9; z++) {
    const int c = g_col[9 * r + z];
    if (g_w[9 * r + z] == 0.0 || cls[c] != K_INT) continue;
    int cells[2];
    const int n = box_cells(N, W, c, cells);
    for (int q = 0; q < n; q++) flag[cells[q]] = 1;
  }
}
// per-block counts of the marked cells per colour (then k_scan_blocks over the 5 nb counts, colour-major)
__global__ void __launch_bounds__(TPB) k_xb_count(const uint8_t *flag, int N, int nb, int *bcnt) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  const int col = t < N * N && flag[t] ? cell_colour(N, t) : -1;
  int tot[5];
  (void)colour_rank(col, tot);
  if (threadIdx.x == 0)
    for (int c = 0; c < 5; c++) bcnt[c * nb + blockIdx.x] = tot[c];
}
// boxes in colour order, ascending cell within a colour; cellbox[cell] = its box or -1
__global__ void __launch_bounds__(TPB) k_xb_fill(const uint8_t *flag, int N, int nb, const int *boff, int *xb_cell,
                                                 int *cellbox, int cap, int *over) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  const int col = t < N * N && flag[t] ? cell_colour(N, t) : -1;
  int tot[5];
  const int r = colour_rank(col, tot);
  if (t >= N * N) return;
  int b = -1;
  if (col >= 0) {
    b = boff[col * nb + blockIdx.x] + r;
    if (b < cap)
      xb_cell[b] = t;
    else {
      atomicOr(over, 1);
      b = -1;
    }
  }
  cellbox[t] = b;
}
// each body ghost row appended to the boxes of the cells its internal columns border (duplicates removed later)
__global__ void k_xb_gather(const uint8_t *cls, int N, int W, const int *g_pt, const int *g_col, const double *g_w,
                            int ng, const int *cellbox, int *gcnt, int *gtmp, int *over) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ng) return;
  const int G = g_pt[r];
  if (cls[G] != K_GHOST) return;
  for (int z = 0; z < 9; z++) {
    const int c = g_col[9 * r + z];
    if (g_w[9 * r + z] == 0.0 || cls[c] != K_INT) continue;
    int cells[2];
    const int n = box_cells(N, W, c, cells);
    for (int q = 0; q < n; q++) {
      const int b = cellbox[cells[q]];
      if (b < 0) continue;
      const int slot = atomicAdd(&gcnt[b], 1);
      if (slot < XB_GCAP)
        gtmp[b * XB_GCAP + slot] = G;
      else
        atomicOr(over, 1);
    }
  }
}
__device__ __forceinline__ int box_unknowns(const uint8_t *cls, int N, int W, int cell, int U[5]) {
  const int WW = W * W, i = cell % N, j = cell / N, c = (j + 1) * W + (i + 1);
  const int cand[5] = {c, c + 1, WW + c, WW + c + W, 2 * WW + c};
  int m = 0;
  for (int q = 0; q < 5; q++)
    if (cls[cand[q]] == K_INT) U[m++] = cand[q];
  return m;
}
// per box: its ghosts sorted and distinct (count back into gcnt), its unknown count m and m^2 (scanned next)
__global__ void k_xb_size(const uint8_t *cls, int N, int W, const int *xb_cell, int nxb, int *gcnt, int *gtmp, int *mcnt,
                          int *sqcnt, int *over) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nxb) return;
  int *lst = gtmp + (size_t)b * XB_GCAP;
  const int n = min(gcnt[b], XB_GCAP);
  for (int q = 1; q < n; q++) {  // insertion sort (a few dozen entries)
    const int v = lst[q];
    int z = q - 1;
    while (z >= 0 && lst[z] > v) {
      lst[z + 1] = lst[z];
      z--;
    }
    lst[z + 1] = v;
  }
  int u = 0;
  for (int q = 0; q < n; q++)
    if (q == 0 || lst[q] != lst[q - 1]) lst[u++] = lst[q];
  gcnt[b] = u;
  int U[5];
  int m = box_unknowns(cls, N, W, xb_cell[b], U) + u;
  if (m > XB_MAXM) {
    atomicOr(over, 2);
    m = 0;
  }
  mcnt[b] = m;
  sqcnt[b] = m * m;
}
__global__ void k_xb_slots(const uint8_t *cls, int N, int W, const int *xb_cell, int nxb, const int *gcnt,
                           const int *gtmp, const int *xb_off, int *xb_idx, int *xb_box) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nxb) return;
  const int o = xb_off[b];
  if (xb_off[b + 1] == o) return;
  int U[5];
  const int m0 = box_unknowns(cls, N, W, xb_cell[b], U);
  for (int a = 0; a < m0; a++) {
    xb_idx[o + a] = U[a];
    xb_box[o + a] = b;
  }
  for (int a = 0; a < gcnt[b]; a++) {
    xb_idx[o + m0 + a] = gtmp[(size_t)b * XB_GCAP + a];
    xb_box[o + m0 + a] = b;
  }
}
__global__ void k_xb_own_clear(int *own, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) own[t] = 0x7fffffff;
}
// the first box of a colour that holds a ghost (the boxes are in colour order, so the smallest index)
__global__ void k_xb_own(const uint8_t *cls, int N, const int *xb_idx, const int *xb_box, const int *xb_cell, int nxs,
                         const int *g_rowof, int ng, int *own) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nxs) return;
  const int k = xb_idx[t];
  if (cls[k] != K_GHOST) return;
  const int b = xb_box[t];
  atomicMin(&own[cell_colour(N, xb_cell[b]) * ng + g_rowof[k]], b);
}
__global__ void k_xb_wr(const uint8_t *cls, int N, const int *xb_idx, const int *xb_box, const int *xb_cell, int nxs,
                        const int *g_rowof, int ng, const int *own, uint8_t *wr) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nxs) return;
  const int k = xb_idx[t], b = xb_box[t];
  wr[t] = cls[k] == K_INT ? 1 : (uint8_t)(own[cell_colour(N, xb_cell[b]) * ng + g_rowof[k]] == b);
}
__global__ void k_xb_soff(const int *xb_off, const int *co, int *out) {
  const int c = threadIdx.x;
  if (c < 6) out[c] = xb_off[co[c]];
}
// flat per-slot row tables (see Geo::xb_gc): the 9 columns and weights of each ghost slot's row, -1 for internal slots
__global__ void k_xb_flat_rows(const uint8_t *cls, const int *xb_idx, int nxs, int scap, const int *g_rowof,
                               const int *g_col, const double *g_w, int *gc, double *gw) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nxs) return;
  const int k = xb_idx[s];
  const bool ghost = cls[k] != K_INT;
  const int r = ghost ? g_rowof[k] : 0;
  for (int z = 0; z < 9; z++) {
    gc[(size_t)z * scap + s] = ghost ? g_col[9 * r + z] : -1;
    gw[(size_t)z * scap + s] = ghost ? g_w[9 * r + z] : 0.0;
  }
}
// flat per-slot write tables (see Geo::xb_uk), after the inverses (which decide which blocks are usable)
__global__ void k_xb_flat_write(const int *xb_idx, const int *xb_box, const int *xb_off, const int *xb_ioff,
                                const uint8_t *xb_wr, const uint8_t *xb_ok, int nxs, int *uk, int *uo, int *ub, int *um) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nxs) return;
  const int bx = xb_box[s], o = xb_off[bx], m = xb_off[bx + 1] - o;
  uk[s] = (xb_wr[s] && xb_ok[bx]) ? xb_idx[s] : -1;
  uo[s] = xb_ioff[bx] + (s - o) * m;
  ub[s] = o;
  um[s] = m;
}

// coefficient of unknown c in the row of point k (internal momentum or continuity row of Sect. 3.2, or the ghost
// row of k); the xi column of the continuity rows is not a box unknown
__device__ double xb_coef(const uint8_t *cls, int W, double h, double a, double d, const int *g_rowof, const int *g_col,
                          const double *g_w, int k, int c) {
  const int WW = W * W;
  if (cls[k] == K_INT) {
    const int g = k / WW, q = k - g * WW;
    const double ih = 1.0 / h;
    if (g < 2) {
      if (c == k) return d;
      if (c == k - 1 || c == k + 1 || c == k - W || c == k + W) return -a;
      if (c == 2 * WW + q) return ih;
      if (c == 2 * WW + q - (g == 0 ? 1 : W)) return -ih;
      return 0.0;
    }
    if (c == q + 1 || c == WW + q + W) return ih;
    if (c == q || c == WW + q) return -ih;
    return 0.0;
  }
  const int r = g_rowof[k];
  double s = 0;
  for (int z = 0; z < 9; z++)
    if (g_col[9 * r + z] == c) s += g_w[9 * r + z];
  return s;
}
// inverse of each box's block by Gauss-Jordan elimination with partial pivoting, one wavefront per box, the
// augmented block [A | I] in LDS
constexpr int XF_T = 64;
__global__ void __launch_bounds__(XF_T) k_xb_factor(const uint8_t *cls, int W, double h, double a, double d,
                                                    const int *xb_off, const int *xb_ioff, const int *xb_idx,
                                                    const int *g_rowof, const int *g_col, const double *g_w,
                                                    double *xb_inv, uint8_t *xb_ok) {
  __shared__ double A[XB_MAXM][2 * XB_MAXM + 1];
  __shared__ double colk[XB_MAXM];
  __shared__ int U[XB_MAXM];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int o = xb_off[b], m = xb_off[b + 1] - o, m2 = 2 * m;
  if (m == 0) {
    if (tid == 0) xb_ok[b] = 0;
    return;
  }
  if (tid < m) U[tid] = xb_idx[o + tid];
  __syncthreads();
  for (int e = tid; e < m * m; e += XF_T) {
    const int r = e / m, c = e - r * m;
    A[r][c] = xb_coef(cls, W, h, a, d, g_rowof, g_col, g_w, U[r], U[c]);
    A[r][m + c] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  bool ok = true;
  for (int k = 0; k < m; k++) {
    // pivot: the largest |A[r][k]|, r >= k (the smaller row on ties)
    double v = (tid >= k && tid < m) ? fabs(A[tid][k]) : -1.0;
    int ir = tid;
    for (int off = 32; off > 0; off >>= 1) {
      const double v2 = __shfl_xor(v, off, 64);
      const int i2 = __shfl_xor(ir, off, 64);
      if (v2 > v || (v2 == v && i2 < ir)) {
        v = v2;
        ir = i2;
      }
    }
    if (!(v > 0.0)) {
      ok = false;
      break;
    }
    if (ir != k)
      for (int c = tid; c < m2; c += XF_T) {
        const double t = A[k][c];
        A[k][c] = A[ir][c];
        A[ir][c] = t;
      }
    __syncthreads();
    const double piv = A[k][k];
    __syncthreads();
    for (int c = tid; c < m2; c += XF_T) A[k][c] /= piv;
    __syncthreads();
    if (tid < m) colk[tid] = A[tid][k];
    __syncthreads();
    for (int e = tid; e < m * m2; e += XF_T) {
      const int r = e / m2, c = e - r * m2;
      if (r != k) A[r][c] -= colk[r] * A[k][c];
    }
    __syncthreads();
  }
  double *out = xb_inv + xb_ioff[b];
  if (ok)
    for (int e = tid; e < m * m; e += XF_T) {
      const int r = e / m, c = e - r * m;
      out[e] = A[r][m + c];
    }
  if (tid == 0) xb_ok[b] = ok ? 1 : 0;
}

static Lat make_lat(Ctx *ctx, int l) {
  Lat L;
  L.phi = ctx->phi;
  L.Lf = 2 * ctx->N + 1;
  L.s = ctx->geo[l].lstride;
  L.N = ctx->geo[l].N;
  L.h = ctx->geo[l].h;
  return L;
}
static RowArgs row_args(Geo &G) {
  RowArgs R;
  R.g_pt = G.g_pt;
  R.g_col = G.g_col;
  R.g_w = G.g_w;
  R.g_dtau = G.g_dtau;
  R.g_B = G.g_B;
  R.g_nB = G.g_nB;
  R.g_th = G.g_th;
  R.g_kind = G.g_kind;
  R.ng = G.ng;
  return R;
}

gp_status levelset_analytic(Ctx *ctx, const gp_shape *sh, double t, const gp_rigid *mo) {
  int N = ctx->N, nl = 2 * N + 1;
  gp_rigid m{};
  if (mo) m = *mo;
  k_levelset<<<nblk((long)nl * nl), TPB, 0, ctx->stream>>>(ctx->phi, N, sh->kind, sh->p[0], sh->p[1], sh->p[2], sh->p[3],
                                                           m.X0x + m.Ux * t, m.X0y + m.Uy * t, m.omega * t);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

// Read-backs of the build without a blocking runtime call: k_publish (one wavefront) copies up to four ranges
// of device words into the level's pinned host buffer and then sets its sequence number there (system-scope
// release); the host polls that number, and the stream now and then, so that a failed launch ends the wait.
// (A copy to pageable memory and a stream synchronisation per read-back, a dozen per level and eight levels
// building at once, kept the threads waiting on each other in the runtime.)
struct PubSrc {
  const int *p[4];
  int n[4];
  int k;
};
__global__ void __launch_bounds__(64) k_publish(PubSrc src, int *dst, unsigned *seqp, unsigned seq) {
  int off = 0;
  for (int q = 0; q < src.k; q++) {
    for (int w = threadIdx.x; w < src.n[q]; w += 64) dst[off + w] = src.p[q][w];
    off += src.n[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(seqp, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
struct Words {
  const void *p;
  int n;  // 4-byte words
};
static gp_status fetch(Ctx *ctx, BuildRes &B, std::initializer_list<Words> src, void *out) {
  PubSrc ps{};
  int tot = 0;
  for (const Words &w : src) {
    ps.p[ps.k] = static_cast<const int *>(w.p);
    ps.n[ps.k] = w.n;
    ps.k++;
    tot += w.n;
  }
  const unsigned seq = ++B.seq;
  k_publish<<<1, 64, 0, B.s>>>(ps, B.hbuf, B.hseq, seq);
  GP_HIP(hipGetLastError());
  for (long it = 1;; it++) {
    if (__atomic_load_n(B.hseq, __ATOMIC_ACQUIRE) == seq) break;
    if ((it & 255) == 0) {
      const hipError_t e = hipStreamQuery(B.s);
      if (e == hipSuccess && __atomic_load_n(B.hseq, __ATOMIC_ACQUIRE) != seq) {
        std::lock_guard<std::mutex> lk(ctx->err_mu);
        ctx->hip_err = "a read-back of the geometry build did not arrive";
        return GP_EHIP;
      }
      if (e != hipSuccess && e != hipErrorNotReady) GP_HIP(e);
    }
  }
  std::memcpy(out, B.hbuf, (size_t)tot * sizeof(int));
  return GP_OK;
}
static gp_status read_flags(Ctx *ctx, BuildRes &B, int *h) { return fetch(ctx, B, {{B.flags, 8}}, h); }

// ---------------------------------------------------------------------------------------------------------
// angular sectors of a large boundary band (one workgroup each in the band relaxation).  Angles are taken about
// the mean of the band cells' centres.  A relaxation step's band work reaches R cells from a written point (the
// reach of each ghost sweep and each band colour, summed); two points within Euclidean distance d, both at least
// r_min from the centre, differ in angle by at most 2 asin(d / (2 r_min)), so with Delta that bound for
// d = R sqrt(2) h, a sector whose workgroup computes every band box and ghost row within Delta of its angles
// (redundantly with its neighbours) gets its own points exactly as the whole band would.
// ---------------------------------------------------------------------------------------------------------
__device__ __forceinline__ void sec_xy(int k, int W, double h, double &x, double &y) {
  const int q = k % (W * W), j = q / W - 1, i = q % W - 1;
  x = -1.0 + (i + 0.5) * h;
  y = -1.0 + (j + 0.5) * h;
}
__device__ __forceinline__ int sec_cheb(int a, int b, int W) {
  const int WW = W * W, qa = a % WW, qb = b % WW;
  return max(abs(qa / W - qb / W), abs(qa % W - qb % W));
}
struct SecGeo {
  double cx, cy, delta, w;
  int S;
};
__device__ __forceinline__ int sec_of(double x, double y, const SecGeo &sg) {
  const double th = atan2(y - sg.cy, x - sg.cx) + M_PI;
  int s = (int)floor(th / sg.w);
  return ((s % sg.S) + sg.S) % sg.S;
}
// bit mask of the sectors within delta of angle at (x, y)
__device__ __forceinline__ unsigned sec_bits(double x, double y, const SecGeo &sg) {
  const double th = atan2(y - sg.cy, x - sg.cx) + M_PI;
  const int lo = (int)floor((th - sg.delta) / sg.w), hi = (int)floor((th + sg.delta) / sg.w);
  unsigned m = 0;
  for (int k = lo; k <= hi; k++) m |= 1u << (((k % sg.S) + sg.S) % sg.S);
  return m;
}
// sums of the band cells' column and row numbers (integers in acc[0], acc[1], so the sum does not depend on the
// order of the additions); reach of the body ghost rows in cells (reach)
__global__ void k_sec_centre(const int *band, int nband, int N, double h, const int *bg_k, const int *bg_loc, int nbg,
                             int gcap, const int *reg_pt, int W, double *acc, int *reach) {
  (void)h;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nband) {
    const int cell = band[t];
    atomicAdd((unsigned long long *)&acc[0], (unsigned long long)(cell % N));
    atomicAdd((unsigned long long *)&acc[1], (unsigned long long)(cell / N));
  } else if (t < nband + nbg) {
    const int s2 = t - nband, k = bg_k[s2];
    int m = 0;
    for (int z = 1; z < 10; z++) m = max(m, sec_cheb(k, reg_pt[bg_loc[z * gcap + s2]], W));
    atomicMax(reach, m);
  }
}
// smallest distance from the centre over the region points (as the bits of a non-negative double)
__global__ void k_sec_rmin(const int *reg_pt, int nreg, int W, double h, double cx, double cy, unsigned long long *out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nreg) return;
  double x, y;
  sec_xy(reg_pt[g], W, h, x, y);
  atomicMin(out, (unsigned long long)__double_as_longlong(sqrt((x - cx) * (x - cx) + (y - cy) * (y - cy))));
}
__device__ __forceinline__ int band_colour_of(int q, const int *off) {
  int c = 0;
  while (c < 4 && q >= off[c + 1]) c++;
  return c;
}
struct SecOff {
  int p[SEC_MAX + 1], b[5 * SEC_MAX + 1], g[SEC_MAX + 1], o[SEC_MAX + 1];
};
// Counters per sector are aggregated per workgroup in LDS (one global atomic per sector and workgroup); the
// fills reserve a range per workgroup and sector the same way (the order within a sector is free: nothing
// depends on it but LDS slot numbers).
constexpr int SEC_CNT = 6 * SEC_MAX;  // 5 per sector for boxes by colour, 1 for rows
// memberships of the band boxes and body ghost rows, marked on the region points they name; counts per sector
__global__ void __launch_bounds__(TPB) k_sec_mark(const int *band, int nband, const int *boff, const int *bbox, int bcap,
                                                  int N, double h, const int *bg_k, const int *bg_loc, int nbg, int gcap,
                                                  int W, SecGeo sg, int *smask, int *cnt_b, int *cnt_g) {
  __shared__ int lc[SEC_CNT];
  for (int q = threadIdx.x; q < SEC_CNT; q += TPB) lc[q] = 0;
  __syncthreads();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nband) {
    const int cell = band[t];
    const unsigned m = sec_bits(-1.0 + (cell % N + 0.5) * h, -1.0 + (cell / N + 0.5) * h, sg);
    const int c = band_colour_of(t, boff);
    for (int s = 0; s < sg.S; s++)
      if (m >> s & 1u) atomicAdd(&lc[5 * s + c], 1);
    for (int z = 0; z < 21; z++) atomicOr(&smask[bbox[z * bcap + t]], (int)m);
  } else if (t < nband + nbg) {
    const int s2 = t - nband;
    double x, y;
    sec_xy(bg_k[s2], W, h, x, y);
    const unsigned m = sec_bits(x, y, sg);
    for (int s = 0; s < sg.S; s++)
      if (m >> s & 1u) atomicAdd(&lc[5 * SEC_MAX + s], 1);
    for (int z = 0; z < 10; z++) atomicOr(&smask[bg_loc[z * gcap + s2]], (int)m);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 5 * sg.S; q += TPB)
    if (lc[q]) atomicAdd(&cnt_b[q], lc[q]);
  for (int q = threadIdx.x; q < sg.S; q += TPB)
    if (lc[5 * SEC_MAX + q]) atomicAdd(&cnt_g[q], lc[5 * SEC_MAX + q]);
}
// points per sector, owned written points per sector (the sector of the point's own angle); bad: a point in more
// than four sectors, or a written point outside the region of its owner
__global__ void __launch_bounds__(TPB) k_sec_count(const int *smask, int nreg, int nregw, const int *reg_pt, int W,
                                                   double h, SecGeo sg, int *cnt_p, int *cnt_o, int *bad) {
  __shared__ int lp[SEC_MAX], lo[SEC_MAX];
  if (threadIdx.x < SEC_MAX) lp[threadIdx.x] = lo[threadIdx.x] = 0;
  __syncthreads();
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < nreg) {
    const unsigned m = (unsigned)smask[g];
    if (__popc(m) > 4) atomicOr(bad, 1);
    for (int s = 0; s < sg.S; s++)
      if (m >> s & 1u) atomicAdd(&lp[s], 1);
    if (g < nregw) {
      double x, y;
      sec_xy(reg_pt[g], W, h, x, y);
      const int o = sec_of(x, y, sg);
      if (!(m >> o & 1u)) atomicOr(bad, 2);
      atomicAdd(&lo[o], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x < sg.S) {
    if (lp[threadIdx.x]) atomicAdd(&cnt_p[threadIdx.x], lp[threadIdx.x]);
    if (lo[threadIdx.x]) atomicAdd(&cnt_o[threadIdx.x], lo[threadIdx.x]);
  }
}
__global__ void __launch_bounds__(TPB) k_sec_fill_pts(const int *smask, int nreg, int nregw, const int *reg_pt, int W,
                                                      double h, SecGeo sg, SecOff off, int *cur_p, int *cur_o,
                                                      int *sec_pt, int *lmap, int *own_loc, int *own_g) {
  __shared__ int lc[2 * SEC_MAX], base[2 * SEC_MAX];
  for (int q = threadIdx.x; q < 2 * SEC_MAX; q += TPB) lc[q] = 0;
  __syncthreads();
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned m = 0;
  int o = -1;
  if (g < nreg) {
    m = (unsigned)smask[g];
    for (int s = 0; s < sg.S; s++)
      if (m >> s & 1u) atomicAdd(&lc[s], 1);
    if (g < nregw) {
      double x, y;
      sec_xy(reg_pt[g], W, h, x, y);
      o = sec_of(x, y, sg);
      atomicAdd(&lc[SEC_MAX + o], 1);
    }
  }
  // one reservation per counter: points (cur_p) then owned (cur_o)
  __syncthreads();
  for (int q = threadIdx.x; q < 2 * SEC_MAX; q += TPB) {
    base[q] = (q % SEC_MAX < sg.S && lc[q]) ? atomicAdd(q < SEC_MAX ? &cur_p[q] : &cur_o[q - SEC_MAX], lc[q]) : 0;
    lc[q] = 0;
  }
  __syncthreads();
  if (g < nreg) {
    int r = 0;
    for (int s = 0; s < sg.S; s++)
      if (m >> s & 1u) {
        const int k = base[s] + atomicAdd(&lc[s], 1);
        sec_pt[off.p[s] + k] = reg_pt[g];
        lmap[4 * g + r++] = k;
      }
    if (o >= 0) {
      const int k = base[SEC_MAX + o] + atomicAdd(&lc[SEC_MAX + o], 1);
      own_loc[off.o[o] + k] = lmap[4 * g + __popc(m & ((1u << o) - 1u))];
      own_g[off.o[o] + k] = g;
    }
  }
}
__device__ __forceinline__ int sec_local(const int *smask, const int *lmap, int g, int s) {
  return lmap[4 * g + __popc((unsigned)smask[g] & ((1u << s) - 1u))];
}
__global__ void __launch_bounds__(TPB) k_sec_fill_tabs(const int *band, int nband, const int *boff, const int *bbox,
                                                       int bcap, int N, double h, const int *bg_k, const int *bg_loc,
                                                       const double *bg_w, const double *bg_dt, int nbg, int gcap, int W,
                                                       SecGeo sg, SecOff off, const int *smask, const int *lmap,
                                                       int *cur_b, int *cur_g, uint16_t *bsl, int *bfl, int *bcell,
                                                       int bstride, uint16_t *gl, double *gw, double *gdt, int *gk,
                                                       int gstride) {
  __shared__ int lc[SEC_CNT], base[SEC_CNT];
  for (int q = threadIdx.x; q < SEC_CNT; q += TPB) lc[q] = 0;
  __syncthreads();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned m = 0;
  int c = 0, s2 = -1;
  double x = 0, y = 0;
  if (t < nband) {
    const int cell = band[t];
    x = -1.0 + (cell % N + 0.5) * h;
    y = -1.0 + (cell / N + 0.5) * h;
    m = sec_bits(x, y, sg);
    c = band_colour_of(t, boff);
    for (int s = 0; s < sg.S; s++)
      if (m >> s & 1u) atomicAdd(&lc[5 * s + c], 1);
  } else if (t < nband + nbg) {
    s2 = t - nband;
    sec_xy(bg_k[s2], W, h, x, y);
    m = sec_bits(x, y, sg);
    for (int s = 0; s < sg.S; s++)
      if (m >> s & 1u) atomicAdd(&lc[5 * SEC_MAX + s], 1);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < SEC_CNT; q += TPB) {
    const bool box = q < 5 * SEC_MAX;
    const bool live = box ? q < 5 * sg.S : q - 5 * SEC_MAX < sg.S;
    base[q] = (live && lc[q]) ? atomicAdd(box ? &cur_b[q] : &cur_g[q - 5 * SEC_MAX], lc[q]) : 0;
    lc[q] = 0;
  }
  __syncthreads();
  if (t < nband) {
    for (int s = 0; s < sg.S; s++)
      if (m >> s & 1u) {
        const int idx = off.b[5 * s + c] + base[5 * s + c] + atomicAdd(&lc[5 * s + c], 1);
        for (int z = 0; z < 21; z++) bsl[z * bstride + idx] = (uint16_t)sec_local(smask, lmap, bbox[z * bcap + t], s);
        bfl[idx] = bbox[21 * bcap + t];
        bcell[idx] = band[t];
      }
  } else if (s2 >= 0) {
    for (int s = 0; s < sg.S; s++)
      if (m >> s & 1u) {
        const int idx = off.g[s] + base[5 * SEC_MAX + s] + atomicAdd(&lc[5 * SEC_MAX + s], 1);
        for (int z = 0; z < 10; z++) gl[z * gstride + idx] = (uint16_t)sec_local(smask, lmap, bg_loc[z * gcap + s2], s);
        for (int z = 0; z < 9; z++) gw[z * gstride + idx] = bg_w[z * gcap + s2];
        gdt[idx] = bg_dt[s2];
        gk[idx] = bg_k[s2];
      }
  }
}

// the sectors of level l, or sec_S = 0 where they do not apply (too close to the centre, a point in more than four
// sectors, a table over its capacity, a sector too large for LDS)
gp_status sector_build(Ctx *ctx, int l) {
  Geo &G = ctx->geo[l];
  BuildRes &B = ctx->bres[l];
  hipStream_t s = B.s;
  const int W = G.W, nt = G.nband + G.nbg;
  G.sec_S = 0;
  double *acc = B.red;  // [0], [1] centre sums, [2] r_min bits
  int *ic = B.bcnt;     // int counters
  GP_HIP(hipMemsetAsync(acc, 0, 2 * sizeof(double), s));
  GP_HIP(hipMemsetAsync(ic, 0, 4 * sizeof(int), s));
  k_sec_centre<<<nblk(nt), TPB, 0, s>>>(G.band, G.nband, G.N, G.h, G.bg_k, G.bg_loc, G.nbg, G.gcap, G.reg_pt, W, acc, ic);
  GP_HIP(hipGetLastError());
  unsigned long long hacc[2];
  int reach = 0;
  {
    int w[5];
    gp_status fs = fetch(ctx, B, {{acc, 4}, {ic, 1}}, w);
    if (fs) return fs;
    std::memcpy(hacc, w, 2 * sizeof(unsigned long long));
    reach = w[4];
  }
  SecGeo sg;  // the mean of the band cells' centres
  sg.cx = -1.0 + ((double)hacc[0] / G.nband + 0.5) * G.h;
  sg.cy = -1.0 + ((double)hacc[1] / G.nband + 0.5) * G.h;
  GP_HIP(hipMemsetAsync(acc + 2, 0x7f, sizeof(double), s));  // 0x7f7f...: ~1.4e306, above any distance here
  k_sec_rmin<<<nblk(G.nreg), TPB, 0, s>>>(G.reg_pt, G.nreg, W, G.h, sg.cx, sg.cy, (unsigned long long *)(acc + 2));
  GP_HIP(hipGetLastError());
  double rmin = 0;
  {
    gp_status fs = fetch(ctx, B, {{acc + 2, 2}}, &rmin);
    if (fs) return fs;
  }
  // reach of one relaxation step's band work in cells: each ghost sweep the ghost rows' reach (+1 for the
  // staggering), each band colour 3 (a box reads 2 cells away, +1), and 2 more for the written points themselves
  const int lam = ctx->prm.lambda_ghost, nsw = ctx->prm.bnd_sweeps;
  const double R = (lam * (reach + 1) + nsw * (5 * 3 + lam * (reach + 1)) + 2) * std::sqrt(2.0) * G.h;
  if (!(rmin > 0) || R >= 2.0 * rmin) return GP_OK;
  sg.delta = 2.0 * std::asin(R / (2.0 * rmin));
  // SEC_MAX sectors where no point falls in more than four of them (smaller regions to stage per workgroup),
  // else 8
  sg.S = SEC_MAX;
  sg.w = 2.0 * M_PI / sg.S;
  if (2.0 * sg.delta > 2.5 * sg.w) {
    sg.S = 8;
    sg.w = 2.0 * M_PI / sg.S;
  }
  if (2.0 * sg.delta > 2.5 * sg.w) return GP_OK;  // more than four sectors per point
  const int S = sg.S;
  int *cnt_b = ic, *cnt_g = ic + 5 * S, *cnt_p = ic + 6 * S, *cnt_o = ic + 7 * S, *bad = ic + 8 * S;
  int *cur = ic + 8 * S + 1;  // 8 S cursors
  GP_HIP(hipMemsetAsync(ic, 0, (16 * S + 1) * sizeof(int), s));
  GP_HIP(hipMemsetAsync(G.sec_mask, 0, (size_t)G.nreg * sizeof(int), s));
  k_sec_mark<<<nblk(nt), TPB, 0, s>>>(G.band, G.nband, G.d_band_off, G.bbox, G.bcap, G.N, G.h, G.bg_k, G.bg_loc, G.nbg,
                                      G.gcap, W, sg, G.sec_mask, cnt_b, cnt_g);
  k_sec_count<<<nblk(G.nreg), TPB, 0, s>>>(G.sec_mask, G.nreg, G.nregw, G.reg_pt, W, G.h, sg, cnt_p, cnt_o, bad);
  GP_HIP(hipGetLastError());
  std::vector<int> hc(8 * S + 1);
  {
    gp_status fs = fetch(ctx, B, {{ic, (int)hc.size()}}, hc.data());
    if (fs) return fs;
  }
  if (hc[8 * S]) return GP_OK;
  SecOff off{};
  int maxreg = 0, maxrow = 0;
  for (int q = 0; q < S; q++) {
    off.p[q + 1] = off.p[q] + hc[6 * S + q];
    off.g[q + 1] = off.g[q] + hc[5 * S + q];
    off.o[q + 1] = off.o[q] + hc[7 * S + q];
    maxreg = std::max(maxreg, hc[6 * S + q]);
    maxrow = std::max(maxrow, hc[5 * S + q]);
  }
  for (int q = 0; q < 5 * S; q++) off.b[q + 1] = off.b[q] + hc[q];
  if (off.p[S] > G.sec_pcap || off.b[5 * S] > G.sec_bcap || off.g[S] > G.sec_gcap || off.o[S] != G.nregw ||
      maxreg >= 65536 || (size_t)maxreg * sizeof(double) + 2 * (size_t)maxrow * sizeof(double) + 2048 > ctx->max_lds)
    return GP_OK;
  k_sec_fill_pts<<<nblk(G.nreg), TPB, 0, s>>>(G.sec_mask, G.nreg, G.nregw, G.reg_pt, W, G.h, sg, off, cur, cur + S,
                                              G.sec_pt, G.sec_lmap, G.sec_own_loc, G.sec_own_g);
  k_sec_fill_tabs<<<nblk(nt), TPB, 0, s>>>(G.band, G.nband, G.d_band_off, G.bbox, G.bcap, G.N, G.h, G.bg_k, G.bg_loc,
                                           G.bg_w, G.bg_dt, G.nbg, G.gcap, W, sg, off, G.sec_mask, G.sec_lmap,
                                           cur + 2 * S, cur + 7 * S, G.sec_bsl, G.sec_bfl, G.sec_bcell, G.sec_bcap,
                                           G.sec_gl, G.sec_gw, G.sec_gdt, G.sec_gk, G.sec_gcap);
  GP_HIP(hipGetLastError());
  for (int q = 0; q <= S; q++) {
    G.sec_poff[q] = off.p[q];
    G.sec_goff[q] = off.g[q];
    G.sec_ooff[q] = off.o[q];
  }
  for (int q = 0; q <= 5 * S; q++) G.sec_boff[q] = off.b[q];
  G.sec_maxreg = maxreg;
  G.sec_maxrow = maxrow;
  G.sec_S = S;
  return GP_OK;
}

// coupled-box tables of level l (after its ghost rows, their row map and the classes are final)
static gp_status xb_build(Ctx *ctx, int l, BuildRes &B) {
  Geo &G = ctx->geo[l];
  const int N = G.N, W = G.W;
  hipStream_t s = B.s;
  G.nxb = G.nxs = G.xb_maxs = 0;
  for (int c = 0; c < 6; c++) G.xb_coff[c] = G.xb_soff[c] = 0;
  G.xb_alpha = -1;
  if (!G.ng || !G.xb_cell) return GP_OK;
  int *cellbox = B.iscr;                                               // N^2 ints
  uint8_t *flag = reinterpret_cast<uint8_t *>(B.iscr + (size_t)N * N);  // N^2 bytes after them
  int *over = B.flags + 13;
  GP_HIP(hipMemsetAsync(flag, 0, (size_t)N * N, s));
  GP_HIP(hipMemsetAsync(over, 0, sizeof(int), s));
  k_xb_mark<<<nblk(G.ng), TPB, 0, s>>>(G.cls, N, W, G.g_pt, G.g_col, G.g_w, G.ng, flag);
  const int nb = nblk((long)N * N);
  k_xb_count<<<nb, TPB, 0, s>>>(flag, N, nb, B.bcnt);
  k_scan_blocks<<<1, SCAN_T, 0, s>>>(B.bcnt, 5 * nb);
  k_band_offsets<<<1, 64, 0, s>>>(B.bcnt, nb, G.d_xb_co);
  k_xb_fill<<<nb, TPB, 0, s>>>(flag, N, nb, B.bcnt, G.xb_cell, cellbox, G.xb_bcap, over);
  GP_HIP(hipGetLastError());
  int hco[6];
  gp_status fs = fetch(ctx, B, {{G.d_xb_co, 6}}, hco);
  if (fs) return fs;
  const int nxb = hco[5];
  if (nxb > G.xb_bcap) return GP_ENOMEM;
  if (nxb == 0) return GP_OK;
  GP_HIP(hipMemsetAsync(G.xb_gcnt, 0, (size_t)nxb * sizeof(int), s));
  k_xb_gather<<<nblk(G.ng), TPB, 0, s>>>(G.cls, N, W, G.g_pt, G.g_col, G.g_w, G.ng, cellbox, G.xb_gcnt, G.xb_gtmp, over);
  k_xb_size<<<nblk(nxb), TPB, 0, s>>>(G.cls, N, W, G.xb_cell, nxb, G.xb_gcnt, G.xb_gtmp, G.xb_off, G.xb_ioff, over);
  k_scan_blocks<<<1, SCAN_T, 0, s>>>(G.xb_off, nxb);
  k_scan_blocks<<<1, SCAN_T, 0, s>>>(G.xb_ioff, nxb);
  k_xb_soff<<<1, 64, 0, s>>>(G.xb_off, G.d_xb_co, G.d_xb_co + 8);
  GP_HIP(hipGetLastError());
  int w[9];
  fs = fetch(ctx, B, {{G.d_xb_co + 8, 6}, {G.xb_ioff + nxb, 1}, {over, 1}}, w);
  if (fs) return fs;
  if (w[7]) return GP_ENOMEM;  // a box with more ghosts or unknowns than the tables hold
  const int nxs = w[5];
  if (nxs > G.xb_scap || (long)w[6] > G.xb_icap) return GP_ENOMEM;
  k_xb_slots<<<nblk(nxb), TPB, 0, s>>>(G.cls, N, W, G.xb_cell, nxb, G.xb_gcnt, G.xb_gtmp, G.xb_off, G.xb_idx, G.xb_box);
  k_xb_own_clear<<<nblk(5L * G.ng), TPB, 0, s>>>(G.xb_own, 5 * G.ng);
  if (nxs) {
    k_xb_own<<<nblk(nxs), TPB, 0, s>>>(G.cls, N, G.xb_idx, G.xb_box, G.xb_cell, nxs, G.g_rowof, G.ng, G.xb_own);
    k_xb_wr<<<nblk(nxs), TPB, 0, s>>>(G.cls, N, G.xb_idx, G.xb_box, G.xb_cell, nxs, G.g_rowof, G.ng, G.xb_own, G.xb_wr);
    k_xb_flat_rows<<<nblk(nxs), TPB, 0, s>>>(G.cls, G.xb_idx, nxs, G.xb_scap, G.g_rowof, G.g_col, G.g_w, G.xb_gc,
                                             G.xb_gw);
  }
  GP_HIP(hipGetLastError());
  G.nxb = nxb;
  G.nxs = nxs;
  for (int c = 0; c < 6; c++) {
    G.xb_coff[c] = hco[c];
    G.xb_soff[c] = w[c];
  }
  for (int c = 0; c < 5; c++) G.xb_maxs = std::max(G.xb_maxs, G.xb_soff[c + 1] - G.xb_soff[c]);
  return GP_OK;
}

// the inverses of level l's coupled boxes for the current alpha, on stream s
gp_status xb_factor(Ctx *ctx, int l, hipStream_t s) {
  Geo &G = ctx->geo[l];
  if (G.nxb) {
    const double a = ctx->alpha / (G.h * G.h), d = 1.0 + 4.0 * a;
    k_xb_factor<<<G.nxb, XF_T, 0, s>>>(G.cls, G.W, G.h, a, d, G.xb_off, G.xb_ioff, G.xb_idx, G.g_rowof, G.g_col, G.g_w,
                                       G.xb_inv, G.xb_ok);
    if (G.nxs)
      k_xb_flat_write<<<nblk(G.nxs), TPB, 0, s>>>(G.xb_idx, G.xb_box, G.xb_off, G.xb_ioff, G.xb_wr, G.xb_ok, G.nxs,
                                                   G.xb_uk, G.xb_uo, G.xb_ub, G.xb_um);
    GP_HIP(hipGetLastError());
  }
  G.xb_alpha = ctx->alpha;
  return GP_OK;
}
gp_status ensure_xb(Ctx *ctx) {
  if (!ctx->have_geom || !ctx->prm.ghost_boxes) return GP_OK;
  for (int l = 0; l < ctx->L; l++)
    if (ctx->geo[l].nxb && ctx->geo[l].xb_alpha != ctx->alpha) {
      gp_status st = xb_factor(ctx, l, ctx->stream);
      if (st) return st;
    }
  return GP_OK;
}

static std::atomic<long> geo_gen_counter{0};

static gp_status build_level(Ctx *ctx, int l) {
  Geo &G = ctx->geo[l];
  G.gen = ++geo_gen_counter;  // tables derived from this level's (the reverse mode's) are rebuilt on a change
  BuildRes &B = ctx->bres[l];
  Lat L = make_lat(ctx, l);
  int W = G.W, P = 3 * W * W;
  hipStream_t s = B.s;
  int hf[8];
  GP_HIP(hipMemsetAsync(B.flags, 0, 8 * sizeof(int), s));
  k_classify<<<nblk(P), TPB, 0, s>>>(L, G.cls, W, l == 0, B.flags);
  k_seed<<<nblk(P), TPB, 0, s>>>(G.cls, G.N, W);
  for (int it = 0;; it += 2) {  // two closure passes per read-back: a pass that changes nothing is a fixpoint
    GP_HIP(hipMemsetAsync(B.flags, 0, sizeof(int), s));
    k_closure<<<nblk(P), TPB, 0, s>>>(L, G.cls, W, B.flags);
    GP_HIP(hipMemsetAsync(B.flags + 7, 0, sizeof(int), s));
    k_closure<<<nblk(P), TPB, 0, s>>>(L, G.cls, W, B.flags + 7);
    gp_status st = read_flags(ctx, B, hf);
    if (st) return st;
    if (!hf[7]) break;
    if (it > 64) return GP_EGEOM;
  }
  {
    uint8_t *rowint = reinterpret_cast<uint8_t *>(B.iscr);  // 3 W^2 bytes
    k_ext_rows_int<<<nblk(P), TPB, 0, s>>>(G.cls, G.N, W, ctx->prm.ext_radius, rowint);
    k_ext_mark<<<nblk(P), TPB, 0, s>>>(G.cls, G.N, W, ctx->prm.ext_radius, rowint);
  }
  k_body_to_inactive<<<nblk(P), TPB, 0, s>>>(G.cls, P);
  // ghost rows
  GP_HIP(hipMemsetAsync(B.flags + 2, 0, 2 * sizeof(int), s));
  k_compact<<<nblk(P), TPB, 0, s>>>(G.cls, P, 0, G.g_pt, G.gcap, B.flags + 2);
  k_compact<<<nblk(P), TPB, 0, s>>>(G.cls, P, 1, G.e_pt, G.ecap, B.flags + 3);
  gp_status st = read_flags(ctx, B, hf);
  if (st) return st;
  if (hf[2] > G.gcap || hf[3] > G.ecap) return GP_ENOMEM;
  G.ng = hf[2];
  G.ne = hf[3];
  RowArgs R = row_args(G);
  double nbis_d = ceil(log2(0.5 / ctx->prm.bisect_eps_over_h) - 1e-12);
  if (G.ng) {
    // the finest level keeps every row with a positive diagonal; coarse levels replace small ones (cg_min)
    k_ghost_rows<<<nblk(G.ng), TPB, 0, s>>>(L, G.cls, W, R, ctx->prm.march_max, (int)nbis_d, l == 0 ? 0.0 : ctx->prm.cg_min,
                                            ctx->prm.dtau_dir, ctx->prm.dtau_neu_over_h * G.h);
    k_ghostx_rows<<<nblk(G.ng), TPB, 0, s>>>(L, G.cls, W, R, l == 0, B.flags);
  }
  if (G.ne) {
    k_ext_rows<<<nblk(G.ne), TPB, 0, s>>>(L, G.cls, W, G.e_pt, G.ne, G.e_src, G.e_w);
    k_ext_fail<<<nblk(G.ne), TPB, 0, s>>>(G.cls, G.e_pt, G.ne, G.e_src);
    k_row_of<<<nblk(G.ne), TPB, 0, s>>>(G.e_pt, G.ne, G.e_rowof);
  }
  if (G.ng) k_row_of<<<nblk(G.ng), TPB, 0, s>>>(G.g_pt, G.ng, G.g_rowof);
  if (ctx->prm.ghost_boxes && l < ctx->prm.ghost_box_levels) {
    gp_status xs = xb_build(ctx, l, B);
    if (xs) return xs;
  } else {
    G.nxb = G.nxs = G.xb_maxs = 0;
  }
  GP_HIP(hipMemsetAsync(G.d_mp, 0, sizeof(int), s));
  k_count_mp<<<std::min(256, nblk(W * W)), TPB, 0, s>>>(G.cls, W, G.d_mp);
  // boundary band: cells grouped by colour, ascending cell index within a colour
  {
    int nb = nblk((long)G.N * G.N);
    int hoff[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (ctx->prm.bnd_sweeps > 0) {
      uint8_t *cut = reinterpret_cast<uint8_t *>(B.iscr);  // N^2 cut flags, then N^2 colours
      int8_t *col8 = reinterpret_cast<int8_t *>(cut + (size_t)G.N * G.N);
      k_band_cut<<<nb, TPB, 0, s>>>(G.cls, G.N, W, cut);
      k_band_count<<<nb, TPB, 0, s>>>(G.cls, cut, G.N, W, ctx->prm.bnd_radius, nb, B.bcnt, col8);
      k_scan_blocks<<<1, SCAN_T, 0, s>>>(B.bcnt, 5 * nb);
      k_band_offsets<<<1, 64, 0, s>>>(B.bcnt, nb, G.d_band_off);
      k_band_fill<<<nb, TPB, 0, s>>>(G.N, nb, col8, B.bcnt, G.band);
      GP_HIP(hipGetLastError());
      gp_status fs = fetch(ctx, B, {{G.d_band_off, 6}}, hoff);
      if (fs) return fs;
    }
    G.nband = hoff[5];
    for (int c = 0; c < 8; c++) G.hband_off[c] = hoff[c];
  }
  // boundary region of the LDS band kernel
  G.lds_ok = 0;
  G.nreg = G.nregw = G.nbg = G.nwg = 0;
  if (G.nband > 0 && G.nband <= G.bcap) {
    const int P3 = 3 * W * W, nbr = nblk(P3);
    const int regcap = G.gcap * 12 + 32 * G.N + 4096;
    int *cnt2 = B.bcnt + nbr + 1;  // block counts of the read-only points
    k_region_clear<<<nblk(P3 + 1), TPB, 0, s>>>(G.reg_map, P3 + 1);
    k_region_mark_reads<<<nblk(G.nband + G.ng), TPB, 0, s>>>(G.cls, G.N, W, G.band, G.nband, G.g_pt, G.g_col, G.ng,
                                                             G.reg_map);
    k_region_mark<<<nblk(G.nband + G.ng), TPB, 0, s>>>(G.cls, G.N, W, G.band, G.nband, G.g_pt, G.ng, G.reg_map);
    // the written points, then the read-only points after them
    k_pred_count<<<nbr, TPB, 0, s>>>(0, P3, G.reg_map, G.cls, B.bcnt);
    k_scan_blocks<<<1, SCAN_T, 0, s>>>(B.bcnt, nbr);
    k_pred_fill<<<nbr, TPB, 0, s>>>(0, P3, G.reg_map, G.cls, B.bcnt, regcap, G.reg_pt, nullptr);
    k_pred_count<<<nbr, TPB, 0, s>>>(2, P3, G.reg_map, G.cls, cnt2);
    k_scan_blocks<<<1, SCAN_T, 0, s>>>(cnt2, nbr);
    k_pred_fill<<<nbr, TPB, 0, s>>>(2, P3, G.reg_map, G.cls, cnt2, regcap, G.reg_pt, B.bcnt + nbr);
    GP_HIP(hipGetLastError());
    int nr = 0;
    {
      int w[2];
      gp_status fs = fetch(ctx, B, {{B.bcnt + nbr, 1}, {cnt2 + nbr, 1}}, w);
      if (fs) return fs;
      G.nregw = w[0];
      nr = w[1];
    }
    // the read-only points are staged too when they fit (FP64 values, and the body ghost rows' new values and
    // right-hand sides in LDS); otherwise their map entries stay negative and the kernel reads them from global
    // memory
    const bool want_sec = G.sec_pcap > 0 && G.nband >= ctx->band_sector_min;  // sectors need every point staged
    const bool rd = G.nregw + nr <= regcap &&
                    (want_sec || (size_t)(G.nregw + nr) * sizeof(double) + 2 * (size_t)G.ng * sizeof(double) + 2048 <=
                                     ctx->max_lds);
    G.nreg = rd ? G.nregw + nr : G.nregw;
    if (G.nreg <= regcap) {
      GP_HIP(hipMemsetAsync(B.flags + 10, 0, 2 * sizeof(int), s));
      k_region_slots<<<nblk(G.nreg), TPB, 0, s>>>(G.reg_pt, G.nreg, G.reg_map);
      k_region_boxes<<<nblk(G.nband), TPB, 0, s>>>(G.cls, G.N, W, G.band, G.nband, G.reg_map, G.bcap, G.bbox,
                                                   B.flags + 11);
      // body ghost rows in point order
      k_pred_count<<<nbr, TPB, 0, s>>>(1, P3, G.reg_map, G.cls, B.bcnt);
      k_scan_blocks<<<1, SCAN_T, 0, s>>>(B.bcnt, nbr);
      k_pred_fill<<<nbr, TPB, 0, s>>>(1, P3, G.reg_map, G.cls, B.bcnt, G.gcap, G.bg_k, nullptr);
      if (G.ng) k_row_of<<<nblk(G.ng), TPB, 0, s>>>(G.g_pt, G.ng, B.iscr);
      GP_HIP(hipGetLastError());
      gp_status fs = fetch(ctx, B, {{B.bcnt + nbr, 1}}, &G.nbg);
      if (fs) return fs;
      if (G.nbg > G.gcap) return GP_ENOMEM;
      if (G.nbg)
        k_region_rows<<<nblk(G.nbg), TPB, 0, s>>>(G.cls, G.g_col, G.g_w, G.g_dtau, B.iscr, G.reg_map, G.nbg, G.gcap,
                                                  G.bg_k, G.bg_loc, G.bg_w, G.bg_dt, B.flags + 11);
      if (G.ng)
        k_wall_rows<<<nblk(G.ng), TPB, 0, s>>>(G.cls, G.g_pt, G.g_col, G.ng, G.reg_map, G.nregw, G.wg_rows,
                                               B.flags + 10, B.flags + 11);
      GP_HIP(hipGetLastError());
      int hr[2];
      fs = fetch(ctx, B, {{B.flags + 10, 2}}, hr);
      if (fs) return fs;
      G.nwg = hr[0];
      G.lds_ok = hr[1] == 0 ? 1 : 0;
    }
  }
  G.sec_S = 0;
  if (G.lds_ok && G.sec_pcap > 0 && G.nband >= ctx->band_sector_min && G.nreg > G.nregw && G.nbg > 0) {
    gp_status sst = sector_build(ctx, l);
    if (sst) return sst;
  }
  // ghost columns by row (the double-buffered ghost sweeps of the device-wide band path)
  if (G.ng) {
    GP_HIP(hipMemsetAsync(B.flags + 12, 0, sizeof(int), s));
    k_row_of<<<nblk(G.ng), TPB, 0, s>>>(G.g_pt, G.ng, B.iscr);
    k_colr<<<nblk(9L * G.ng), TPB, 0, s>>>(G.cls, G.g_pt, G.g_col, G.ng, B.iscr, G.g_colr, B.flags + 12);
    k_rows_t<<<nblk(9L * G.ng), TPB, 0, s>>>(G.g_colr, G.g_w, G.ng, G.g_colrT, G.g_wT);
  }
  // boundary faces of the internal pressure cells (and their band-region entries)
  {
    int nb = nblk((long)G.N * G.N);
    k_face_count<<<nb, TPB, 0, s>>>(G.cls, G.N, W, B.bcnt);
    k_scan_blocks<<<1, SCAN_T, 0, s>>>(B.bcnt, nb);
    k_face_fill<<<nb, TPB, 0, s>>>(G.cls, G.N, W, B.bcnt, G.fcap, G.f_code);
    GP_HIP(hipGetLastError());
    int w[2];
    gp_status fs = fetch(ctx, B, {{B.bcnt + nb, 1}, {B.flags + 12, 1}}, w);
    if (fs) return fs;
    G.nf = w[0];
    const int cb = G.ng ? w[1] : 1;
    G.colr_ok = G.ng > 0 && cb == 0;
    if (G.nf > G.fcap) return GP_ENOMEM;
    if (G.lds_ok && G.nf) k_face_loc<<<nblk(G.nf), TPB, 0, s>>>(G.f_code, G.nf, G.reg_map, G.f_loc);
  }
  if (l == 0) k_empty_cells<<<nblk(G.N * G.N), TPB, 0, s>>>(G.cls, G.N, W, B.flags);
  GP_HIP(hipGetLastError());
  {
    int w[9];
    st = fetch(ctx, B, {{G.d_mp, 1}, {B.flags, 8}}, w);
    if (st) return st;
    G.mp = w[0];
    for (int q = 0; q < 8; q++) hf[q] = w[1 + q];
  }
  if (G.mp == 0) return GP_EGEOM;
  if (l == 0 && (hf[1] || hf[4])) return GP_EGEOM;
  return GP_OK;
}

// The levels are independent of each other (each samples the level set on its own lattice), so they are built
// concurrently: level 0 on the context's stream by the calling thread, every other level on a stream of its own
// by a host thread of its own, each with its own scratch (BuildRes).  Their many small launches and read-backs
// then overlap instead of adding up.  The context's stream waits for all of them before anything after the build.
gp_status geometry_build(Ctx *ctx) {
  ctx->have_geom = 0;
  ctx->c_ok = 0;
  const int L = ctx->L;
  GP_HIP(hipEventRecord(ctx->bres[0].ev, ctx->stream));  // the level set and anything before it
  for (int l = 1; l < L; l++) GP_HIP(hipStreamWaitEvent(ctx->bres[l].s, ctx->bres[0].ev, 0));
  std::vector<gp_status> st(L, GP_OK);
  std::vector<std::thread> th;
  th.reserve(L);
  for (int l = L - 1; l >= 1; l--)  // the coarsest first: its exact inverse follows its build
    th.emplace_back([ctx, l, L, &st]() {
      if (hipSetDevice(ctx->device) != hipSuccess) {
        st[l] = GP_EHIP;
        return;
      }
      st[l] = build_level(ctx, l);
      // the coupled-box inverses for the current alpha (a stale alpha is caught by ensure_xb)
      if (st[l] == GP_OK && ctx->alpha > 0 && ctx->prm.ghost_boxes) st[l] = xb_factor(ctx, l, ctx->bres[l].s);
      // the coarsest level: its exact inverse for the current alpha too, while the finer levels still build (a
      // failure leaves c_ok = 0, and the solver factors again and reports it)
      if (l == L - 1 && st[l] == GP_OK && ctx->alpha > 0) (void)coarse_factor(ctx, ctx->bres[l]);
    });
  st[0] = build_level(ctx, 0);
  if (st[0] == GP_OK && ctx->alpha > 0 && ctx->prm.ghost_boxes) st[0] = xb_factor(ctx, 0, ctx->stream);
  for (auto &t : th) t.join();
  for (int l = 0; l < L; l++)
    if (st[l]) return st[l];
  for (int l = 1; l < L; l++) {
    GP_HIP(hipEventRecord(ctx->bres[l].ev, ctx->bres[l].s));
    GP_HIP(hipStreamWaitEvent(ctx->stream, ctx->bres[l].ev, 0));
  }
  ctx->have_geom = 1;
  return GP_OK;
}

gp_status default_boundary_values(Ctx *ctx) {
  Geo &G = ctx->geo[0];
  int W = G.W;
  RowArgs R = row_args(G);
  const double *w = ctx->walls;
  const gp_rigid &m = ctx->motion;
  if (G.ng)
    k_bvals_rows<<<nblk(G.ng), TPB, 0, ctx->stream>>>(G.cls, W, R, ctx->v64[0].b, m.X0x, m.X0y, m.Ux, m.Uy, m.omega,
                                                      ctx->t_geom, m.Ux + ctx->ub_off[0], m.Uy + ctx->ub_off[1], w[0],
                                                      w[4], w[7], w[3]);
  k_bvals_points<<<nblk(3 * W * W), TPB, 0, ctx->stream>>>(G.cls, G.N, W, ctx->v64[0].b, ctx->v64[0].x, w[6], w[2], w[1],
                                                           w[5]);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

// ---------------------------------------------------------------------------------------------------------
// coarsest level: dense matrix of the active unknowns and its inverse (Gauss-Jordan with partial pivoting)
// ---------------------------------------------------------------------------------------------------------
// the active unknowns of the coarsest level in index order (one workgroup of CM_T threads, a chunk of CM_T
// points at a time: wavefront ballots, then the wavefronts' offsets in order)
constexpr int CM_T = 1024;
__global__ void __launch_bounds__(CM_T) k_coarse_map(const uint8_t *cls, int P, int *map, int *inv, int *count) {
  __shared__ int wcount[CM_T / 64];
  __shared__ int base;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) base = 0;
  __syncthreads();
  for (int k0 = 0; k0 < P; k0 += CM_T) {
    const int k = k0 + tid;
    bool act = false;
    if (k < P) {
      const uint8_t c = cls[k];
      act = c == K_INT || c == K_GHOST || c == K_GHOSTX || c == K_WALLG;
    }
    const unsigned long long m = __ballot(act);
    if (lane == 0) wcount[wv] = __popcll(m);
    __syncthreads();
    int off = base;
    for (int w = 0; w < wv; w++) off += wcount[w];
    if (k < P) {
      if (act) {
        const int n = off + __popcll(m & ((1ull << lane) - 1));
        map[n] = k;
        inv[k] = n;
      } else {
        inv[k] = -1;
      }
    }
    __syncthreads();
    if (tid == 0)
      for (int w = 0; w < CM_T / 64; w++) base += wcount[w];
    __syncthreads();
  }
  if (tid == 0) {
    map[base] = P;  // xi
    inv[P] = base;
    *count = base + 1;
  }
}

__global__ void k_coarse_fill(const uint8_t *cls, int N, int W, double h, double a, double d, const int *map,
                              const int *inv, int nc, const int *row_of, const int *g_col, const double *g_w, int mp,
                              double *A) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  double *row = A + (size_t)q * nc;  // zeroed before the launch
  int P = 3 * W * W;
  int k = map[q];
  auto put = [&](int col, double v) {
    int ci = inv[col];
    if (ci >= 0) row[ci] += v;
  };
  if (k == P) {  // mean row
    for (int t = 2 * W * W; t < P; t++)
      if (cls[t] == K_INT) put(t, 1.0 / mp);
    return;
  }
  int g = k / (W * W), loc = k % (W * W), j = loc / W - 1, i = loc % W - 1;
  uint8_t c = cls[k];
  if (c == K_INT) {
    if (g == 0) {
      put(k, d);
      put(gix(W, 0, i - 1, j), -a);
      put(gix(W, 0, i + 1, j), -a);
      put(gix(W, 0, i, j - 1), -a);
      put(gix(W, 0, i, j + 1), -a);
      put(gix(W, 2, i, j), 1.0 / h);
      put(gix(W, 2, i - 1, j), -1.0 / h);
    } else if (g == 1) {
      put(k, d);
      put(gix(W, 1, i - 1, j), -a);
      put(gix(W, 1, i + 1, j), -a);
      put(gix(W, 1, i, j - 1), -a);
      put(gix(W, 1, i, j + 1), -a);
      put(gix(W, 2, i, j), 1.0 / h);
      put(gix(W, 2, i, j - 1), -1.0 / h);
    } else {
      put(gix(W, 0, i + 1, j), 1.0 / h);
      put(gix(W, 0, i, j), -1.0 / h);
      put(gix(W, 1, i, j + 1), 1.0 / h);
      put(gix(W, 1, i, j), -1.0 / h);
      put(P, -1.0);
    }
  } else {
    int r = row_of[k];
    for (int z = 0; z < 9; z++)
      if (g_w[9 * r + z] != 0.0) put(g_col[9 * r + z], g_w[9 * r + z]);
  }
  (void)N;
}


// Blocked Gauss-Jordan inversion with partial pivoting (ties: smallest row).  The matrix is kept in the current
// row order (row interchanges applied); per panel of nb columns [k0, k0+nb):
//  - k_gj_panel (one workgroup, the n x nb panel in LDS) runs the nb elimination steps on the panel columns: pivot
//    search, interchange, the pivot row scaled, every other row eliminated, the pivot column replaced by the
//    inverse column (-f/piv, and 1/piv at the pivot);
//  - k_gj_trail applies the same nb steps to every other column at once: with P the nb pivot rows before the
//    panel, new column = (rows outside P: old row through the interchanges) + K_new * old(P rows of the column),
//    K_new being the panel's new columns.
// The interchanges are not undone on the matrix: the column order of the result is folded into bmap, so that
// x[map[q]] = sum_j A[q][j] b[bmap[j]] applies the inverse.
constexpr int GJ_T = 1024;
__global__ void __launch_bounds__(GJ_T) k_gj_panel(const double *__restrict__ Ain, double *Aout, int n, int k0, int nb,
                                                   int *spv, int *perm, int *fail) {
  // panel, column-major: column j at pl[j * n]; then fcol (n), rowk (nb), oldk (nb)
  extern __shared__ double pl[];
  __shared__ int lperm[1024];
  __shared__ double wbest[GJ_T / 64];
  __shared__ int wbi[GJ_T / 64];
  double *fcol = pl + (size_t)nb * n, *rowk = fcol + n, *oldk = rowk + nb;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (*fail) return;  // an earlier panel found no pivot
  for (int e = tid; e < n * nb; e += GJ_T) {
    int i = e / nb, j = e - i * nb;
    pl[j * n + i] = Ain[(size_t)i * n + k0 + j];
  }
  for (int i = tid; i < n; i += GJ_T) lperm[i] = i;
  __syncthreads();
  // the update's thread map: column uj, rows ui, ui + 32, ... (consecutive threads on consecutive rows)
  const int uj = tid >> 5, ui = tid & 31;
  for (int j = 0; j < nb; j++) {
    const int k = k0 + j;
    const double *cj = pl + (size_t)j * n;
    // pivot: the largest |entry| of column j at or below k (ties to the smaller row)
    double best = -1;
    int bi = n;
    for (int i = k + tid; i < n; i += GJ_T) {
      double av = fabs(cj[i]);
      if (av > best) {
        best = av;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      double ob = __shfl_xor(best, o, 64);
      int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      wbest[wv] = best;
      wbi[wv] = bi;
    }
    __syncthreads();
    // every wavefront reduces the GJ_T / 64 wave results the same way (lane w holds result w % (GJ_T / 64))
    double bb = wbest[lane % (GJ_T / 64)];
    int p = wbi[lane % (GJ_T / 64)];
    for (int o = GJ_T / 128; o > 0; o >>= 1) {
      const double ob = __shfl_xor(bb, o, 64);
      const int oi = __shfl_xor(p, o, 64);
      if (ob > bb || (ob == bb && oi < p)) {
        bb = ob;
        p = oi;
      }
    }
    if (!(bb > 0) || p >= n) {
      if (tid == 0) *fail = 1;
      return;
    }
    // rows k and p interchanged (row p's values scaled into rowk, row k's kept in oldk for position p), and the
    // pivot column after the interchange, all read before anything is written
    const double cjk = cj[k], cjp = cj[p], inv = 1.0 / cjp;
    for (int i = tid; i < n; i += GJ_T) fcol[i] = i == k ? cjp : (i == p ? cjk : cj[i]);
    for (int jj = tid; jj < nb; jj += GJ_T) {
      rowk[jj] = (jj == j) ? inv : pl[jj * n + p] * inv;
      oldk[jj] = pl[jj * n + k];
    }
    if (tid == 0) {
      spv[k] = p;
      const int t = lperm[k];
      lperm[k] = lperm[p];
      lperm[p] = t;
    }
    __syncthreads();
    if (uj < nb) {
      double *col = pl + (size_t)uj * n;
      const double rk = rowk[uj], ok = oldk[uj];
      for (int i0 = ui; i0 < n; i0 += 8 * 32) {  // eight rows' loads before any store (col and fcol share pl)
        double cv[8], fv[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const int i = i0 + 32 * u;
          cv[u] = i < n ? col[i] : 0.0;
          fv[u] = i < n ? fcol[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const int i = i0 + 32 * u;
          if (i >= n) break;
          col[i] = i == k ? rk : ((uj == j) ? -fv[u] * inv : (i == p ? ok : cv[u]) - fv[u] * rk);
        }
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < n * nb; e += GJ_T) {
    int i = e / nb, j = e - i * nb;
    Aout[(size_t)i * n + k0 + j] = pl[j * n + i];
  }
  for (int i = tid; i < n; i += GJ_T) perm[i] = lperm[i];
}
__global__ void k_gj_trail(const double *__restrict__ Ain, double *Aout, int n, int k0, int nb, const int *__restrict__ perm,
                           const int *__restrict__ fail) {
  long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * n || *fail) return;
  int i = (int)(e / n), c = (int)(e - (long)i * n);
  if (c >= k0 && c < k0 + nb) return;
  double s = (i < k0 || i >= k0 + nb) ? Ain[(size_t)perm[i] * n + c] : 0.0;
  for (int t = 0; t < nb; t++) s += Aout[(size_t)i * n + k0 + t] * Ain[(size_t)perm[k0 + t] * n + c];
  Aout[(size_t)i * n + c] = s;
}
// undoing the interchanges as column interchanges in reverse order puts result column c at column lab[c]
__global__ void __launch_bounds__(GJ_T) k_gj_finish(const int *__restrict__ spv, int n, const int *__restrict__ map,
                                                    int *bmap, const int *__restrict__ fail) {
  __shared__ int lab[1024];
  if (*fail) return;
  if (threadIdx.x == 0) {
    for (int c = 0; c < n; c++) lab[c] = c;
    for (int k = n - 1; k >= 0; k--) {
      int t = lab[k];
      lab[k] = lab[spv[k]];
      lab[spv[k]] = t;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += GJ_T) bmap[lab[c]] = map[c];
}

gp_status coarse_factor(Ctx *ctx) { return coarse_factor(ctx, ctx->bres[0]); }
// on the stream and flags of B (the coarsest level's, when the geometry build factors it early)
gp_status coarse_factor(Ctx *ctx, BuildRes &B) {
  int l = ctx->L - 1;
  Geo &G = ctx->geo[l];
  int W = G.W, P = 3 * W * W;
  hipStream_t s = B.s;
  int *inv = (int *)ctx->c_work;  // scratch (P+1 ints fit easily)
  int *row_of = inv + (P + 1);
  k_coarse_map<<<1, CM_T, 0, s>>>(G.cls, P, ctx->c_map, inv, B.flags + 5);
  if (G.ng) k_row_of<<<nblk(G.ng), TPB, 0, s>>>(G.g_pt, G.ng, row_of);
  int hf[8];
  gp_status st = read_flags(ctx, B, hf);
  if (st) return st;
  ctx->nc = hf[5];
  if (ctx->nc > 1024) return GP_EINVAL;
  double a = ctx->alpha / (G.h * G.h), d = 1.0 + 4.0 * a;
  GP_HIP(hipMemsetAsync(ctx->c_A, 0, (size_t)ctx->nc * ctx->nc * sizeof(double), s));
  k_coarse_fill<<<nblk(ctx->nc), TPB, 0, s>>>(G.cls, G.N, W, G.h, a, d, ctx->c_map, inv, ctx->nc, row_of, G.g_col, G.g_w,
                                             G.mp, ctx->c_A);
  GP_HIP(hipMemsetAsync(B.flags + 6, 0, sizeof(int), s));
  {
    const int n = ctx->nc;
    int nb = std::min(32, std::max(1, 15000 / n - 1));
    int *spv = (int *)(ctx->c_work) + 2 * (P + 1), *perm = spv + 1024;
    double *Ain = ctx->c_A, *Aout = ctx->c_B;
    for (int k0 = 0; k0 < n; k0 += nb) {
      int w = std::min(nb, n - k0);
      size_t lds = ((size_t)w * n + n + 2 * w) * sizeof(double);
      k_gj_panel<<<1, GJ_T, lds, s>>>(Ain, Aout, n, k0, w, spv, perm, B.flags + 6);
      k_gj_trail<<<nblk((long)n * n), TPB, 0, s>>>(Ain, Aout, n, k0, w, perm, B.flags + 6);
      std::swap(Ain, Aout);
    }
    ctx->c_inv = Ain;
    k_gj_finish<<<1, GJ_T, 0, s>>>(spv, n, ctx->c_map, ctx->c_bmap, B.flags + 6);
  }
  GP_HIP(hipGetLastError());
  st = read_flags(ctx, B, hf);
  if (st) return st;
  if (hf[6]) return GP_EGEOM;
  ctx->c_ok = 1;
  return GP_OK;
}


// ---------------------------------------------------------------------------------------------------------
// derivative of the finest boundary rows with respect to the body position (reverse mode, body velocity along
// the path).  With the discrete decisions of the geometry frozen (classes, ghost points, the upwind stencils, the
// number of march steps and the bisection branches of Alg. 1), the rows eq. (BCu) of the body ghosts and their
// boundary data are smooth functions of the body position P = X(t).  The lattice samples move with it,
// d phi_k / dP = -R(-omega t)^T grad phi0, and B, theta, n_B and the weights follow by forward-mode
// differentiation (D2: a value and its two partials) along the recorded path.
// ---------------------------------------------------------------------------------------------------------
namespace {
struct D2 {
  double v, x, y;
};
__device__ __forceinline__ D2 dc(double v) { return {v, 0.0, 0.0}; }
__device__ __forceinline__ D2 operator+(D2 a, D2 b) { return {a.v + b.v, a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ D2 operator-(D2 a, D2 b) { return {a.v - b.v, a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ D2 operator-(D2 a) { return {-a.v, -a.x, -a.y}; }
__device__ __forceinline__ D2 operator*(D2 a, D2 b) { return {a.v * b.v, a.x * b.v + a.v * b.x, a.y * b.v + a.v * b.y}; }
__device__ __forceinline__ D2 operator*(double c, D2 a) { return {c * a.v, c * a.x, c * a.y}; }
__device__ __forceinline__ D2 operator/(D2 a, D2 b) {
  const double q = a.v / b.v;
  return {q, (a.x - q * b.x) / b.v, (a.y - q * b.y) / b.v};
}
__device__ __forceinline__ D2 operator/(D2 a, double c) { return {a.v / c, a.x / c, a.y / c}; }
__device__ __forceinline__ D2 dsqrt(D2 a) {
  const double r = sqrt(a.v);
  return {r, r > 0 ? a.x / (2 * r) : 0.0, r > 0 ? a.y / (2 * r) : 0.0};
}
__device__ __forceinline__ D2 dcos(D2 a) { return {cos(a.v), -sin(a.v) * a.x, -sin(a.v) * a.y}; }
__device__ __forceinline__ D2 datan2(D2 y, D2 x) {
  const double d = x.v * x.v + y.v * y.v;
  return {atan2(y.v, x.v), (x.v * y.x - y.v * x.x) / d, (x.v * y.y - y.v * x.y) / d};
}

struct ShapeArg {
  int kind;
  double a0, a1, a2, a3;
  double X, Y, c, s;  // body position and the cosine and sine of its angle
};
// the shapes of shape_value on D2 arguments
__device__ D2 shape_d2(const ShapeArg &S, D2 xb, D2 yb) {
  const int kind = S.kind;
  if (kind == 0) return dc(S.a0) - dsqrt(xb * xb + yb * yb);
  if (kind == 1) return dc(S.a0 * S.a0) - (xb * xb + yb * yb);
  if (kind == 2 || kind == 3) {
    const double c = cos(S.a2), s = sin(S.a2);
    const D2 xr = c * xb - s * yb, yr = s * xb + c * yb;
    const D2 q = xr * xr / (S.a0 * S.a0) + yr * yr / (S.a1 * S.a1);
    return kind == 2 ? dc(1.0) - q : dc(1.0) - dsqrt(q);
  }
  if (kind == 4) {
    const D2 r = dsqrt(xb * xb + yb * yb);
    if (r.v == 0.0) return dc(S.a0 + S.a1);
    return dc(S.a0) + S.a1 * dcos(S.a3 * (datan2(yb, xb) - dc(S.a2))) - r;
  }
  return dc(-1.0);
}
// a finest lattice sample: the stored value and its partials along the body position
__device__ D2 lat_d2(const Lat &L, const ShapeArg &S, int kx, int ky) {
  const double hl = 0.5 * L.h;
  const D2 x = {-1.0 + kx * hl - S.X, -1.0, 0.0}, y = {-1.0 + ky * hl - S.Y, 0.0, -1.0};
  const D2 p = shape_d2(S, S.c * x + S.s * y, S.c * y - S.s * x);
  return {lat_at(L, kx, ky), p.x, p.y};
}
// bilin on D2 positions (the cell of the interpolation is frozen)
__device__ void bilin_d2(const Lat &L, const ShapeArg &S, D2 x, D2 y, D2 *val, D2 *gx, D2 *gy) {
  const double hl = 0.5 * L.h;
  const int nl = 2 * L.N + 1;
  const D2 fx = (x + dc(1.0)) / hl, fy = (y + dc(1.0)) / hl;
  int kx = (int)floor(fx.v), ky = (int)floor(fy.v);
  kx = kx < 0 ? 0 : (kx > nl - 2 ? nl - 2 : kx);
  ky = ky < 0 ? 0 : (ky > nl - 2 ? nl - 2 : ky);
  const D2 tx = fx - dc(kx), ty = fy - dc(ky), ux = dc(1.0) - tx, uy = dc(1.0) - ty;
  const D2 p00 = lat_d2(L, S, kx, ky), p10 = lat_d2(L, S, kx + 1, ky), p01 = lat_d2(L, S, kx, ky + 1),
           p11 = lat_d2(L, S, kx + 1, ky + 1);
  if (val) *val = ux * uy * p00 + tx * uy * p10 + ux * ty * p01 + tx * ty * p11;
  if (gx) *gx = (uy * (p10 - p00) + ty * (p11 - p01)) / hl;
  if (gy) *gy = (ux * (p01 - p00) + tx * (p11 - p10)) / hl;
}
__device__ void normal_d2(const Lat &L, const ShapeArg &S, D2 x, D2 y, D2 *nx, D2 *ny) {
  D2 gx, gy;
  bilin_d2(L, S, x, y, nullptr, &gx, &gy);
  const D2 m = dsqrt(gx * gx + gy * gy);
  if (m.v > 0) {
    *nx = gx / m;
    *ny = gy / m;
  } else {
    *nx = dc(0.0);
    *ny = dc(0.0);
  }
}
// Alg. 1 along a recorded path (boundary_point's rec)
__device__ void boundary_point_d2(const Lat &L, const ShapeArg &S, double xg, double yg, int nbis, const unsigned rec[2],
                                  D2 *Bx, D2 *By) {
  D2 hx = dc(xg), hy = dc(yg), kx = hx, ky = hy;
  const int nm = (int)(rec[0] & 65535u);
  for (int it = 0; it < nm; it++) {
    kx = hx;
    ky = hy;
    D2 nx, ny;
    normal_d2(L, S, hx, hy, &nx, &ny);
    hx = hx - (0.5 * L.h) * nx;
    hy = hy - (0.5 * L.h) * ny;
  }
  if (nm == 0 || rec[0] >= 65536u) {
    *Bx = hx;
    *By = hy;
    return;
  }
  D2 bx = hx, by = hy;
  for (int q = 0; q < nbis; q++) {
    bx = 0.5 * (hx + kx);
    by = 0.5 * (hy + ky);
    if (rec[1] >> q & 1u) {
      kx = bx;
      ky = by;
    } else {
      hx = bx;
      hy = by;
    }
  }
  *Bx = bx;
  *By = by;
}
__device__ __forceinline__ void lagr3_d2(D2 t, D2 T[3]) {
  T[0] = 0.5 * ((dc(1.0) - t) * (dc(2.0) - t));
  T[1] = t * (dc(2.0) - t);
  T[2] = 0.5 * (t * (t - dc(1.0)));
}
__device__ __forceinline__ void dlagr3_d2(D2 t, D2 D[3]) {
  D[0] = t - dc(1.5);
  D[1] = dc(2.0) - 2.0 * t;
  D[2] = t - dc(0.5);
}

// per body ghost row (finest level, eq. (BCu) rows): lam_G times the partials of its residual b_G - sum w x along
// the body position, into cx[k], cy[k] at the ghost's point k (other points untouched); mism counts rows whose
// recomputed boundary point is not the stored one
__global__ void k_path_rows(Lat L, ShapeArg S, double om, const uint8_t *__restrict__ cls, int W, RowArgs R,
                            int march_max, int nbis, const double *__restrict__ x, const double *__restrict__ lam,
                            double *cx, double *cy, int *mism) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R.ng) return;
  const int k = R.g_pt[r];
  if (cls[k] != K_GHOST || R.g_kind[r] != 1) return;
  const double h = L.h;
  const int g = k / (W * W), loc = k % (W * W), j = loc / W - 1, i = loc % W - 1;
  double xg, yg;
  node_pos(g, i, j, h, &xg, &yg);
  int kx, ky;
  node_lat(g, i, j, &kx, &ky);
  double ngx, ngy;
  normal_at(L, xg, yg, &ngx, &ngy);
  const double sx = sgn1(ngx), sy = sgn1(ngy);
  double Bx, By;
  unsigned rec[2];
  if (!boundary_point(L, xg, yg, lat_at(L, kx, ky), march_max, nbis, &Bx, &By, rec) || Bx != R.g_B[2 * r] ||
      By != R.g_B[2 * r + 1]) {
    atomicAdd(mism, 1);
    return;
  }
  D2 BX, BY;
  boundary_point_d2(L, S, xg, yg, nbis, rec, &BX, &BY);
  const D2 thx = (sx / h) * (dc(xg) - BX), thy = (sy / h) * (dc(yg) - BY);
  D2 Tx[3], Ty[3], w[9];
  lagr3_d2(thx, Tx);
  lagr3_d2(thy, Ty);
  if (g < 2) {
    for (int b = 0; b < 3; b++)
      for (int a = 0; a < 3; a++) w[b * 3 + a] = Tx[a] * Ty[b];
  } else {
    D2 nbx, nby, Dx[3], Dy[3];
    normal_d2(L, S, BX, BY, &nbx, &nby);
    dlagr3_d2(thx, Dx);
    dlagr3_d2(thy, Dy);
    for (int b = 0; b < 3; b++)
      for (int a = 0; a < 3; a++) w[b * 3 + a] = -(1.0 / h) * (sx * (nbx * Dx[a] * Ty[b]) + sy * (nby * Tx[a] * Dy[b]));
  }
  double dx = 0, dy = 0;
  for (int z = 0; z < 9; z++) {
    const double xv = x[R.g_col[9 * r + z]];
    dx -= w[z].x * xv;
    dy -= w[z].y * xv;
  }
  // boundary data of the velocity rows, u_b = V + omega x (B - P)
  if (g == 0) {
    dx += -om * BY.x;
    dy += -om * (BY.y - 1.0);
  } else if (g == 1) {
    dx += om * (BX.x - 1.0);
    dy += om * BX.y;
  }
  const double l = lam[k];
  cx[k] = l * dx;
  cy[k] = l * dy;
}
__global__ void k_zero2(double *a, double *b, long n) {
  const long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (q < n) a[q] = b[q] = 0.0;
}
// acc[0..1] += scale * (sum of cx, sum of cy) over the points, in a fixed order: PS_B block partials of a fixed
// grid-stride split (k_path_part), then their sum in block order (k_path_fin)
constexpr int PS_B = 256, PS_T = 256;
__global__ void __launch_bounds__(PS_T) k_path_part(const double *__restrict__ cx, const double *__restrict__ cy, long n,
                                                    double *part) {
  __shared__ double sa[PS_T], sb[PS_T];
  double a = 0, b = 0;
  for (long q = blockIdx.x * (long)PS_T + threadIdx.x; q < n; q += (long)PS_B * PS_T) {
    a += cx[q];
    b += cy[q];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int o = PS_T / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sa[threadIdx.x] += sa[threadIdx.x + o];
      sb[threadIdx.x] += sb[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sa[0];
    part[PS_B + blockIdx.x] = sb[0];
  }
}
__global__ void __launch_bounds__(PS_B) k_path_fin(const double *__restrict__ part, double scale, double *acc) {
  __shared__ double sa[PS_B], sb[PS_B];
  sa[threadIdx.x] = part[threadIdx.x];
  sb[threadIdx.x] = part[PS_B + threadIdx.x];
  __syncthreads();
  for (int o = PS_B / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sa[threadIdx.x] += sa[threadIdx.x + o];
      sb[threadIdx.x] += sb[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    acc[0] += scale * sa[0];
    acc[1] += scale * sb[0];
  }
}
}  // namespace

gp_status path_terms(Ctx *ctx, const gp_shape &sh, const gp_rigid &mo, double t, const double *x, const double *lam,
                     double *cx, double *cy, double *acc, int *mism) {
  Geo &G = ctx->geo[0];
  if (!G.ng) return GP_OK;
  hipStream_t s = ctx->stream;
  Lat L = make_lat(ctx, 0);
  ShapeArg S;
  S.kind = sh.kind;
  S.a0 = sh.p[0];
  S.a1 = sh.p[1];
  S.a2 = sh.p[2];
  S.a3 = sh.p[3];
  S.X = mo.X0x + mo.Ux * t;
  S.Y = mo.X0y + mo.Uy * t;
  S.c = cos(mo.omega * t);
  S.s = sin(mo.omega * t);
  const long n = 3L * G.WW;
  k_zero2<<<nblk(n), TPB, 0, s>>>(cx, cy, n);
  const double nbis_d = ceil(log2(0.5 / ctx->prm.bisect_eps_over_h) - 1e-12);
  k_path_rows<<<nblk(G.ng), TPB, 0, s>>>(L, S, mo.omega, G.cls, G.W, row_args(G), ctx->prm.march_max, (int)nbis_d, x,
                                          lam, cx, cy, mism);
  // X(t) = X0 + U t: the partials along the position times t are those along U
  k_path_part<<<PS_B, PS_T, 0, s>>>(cx, cy, n, ctx->d_red);
  k_path_fin<<<1, PS_B, 0, s>>>(ctx->d_red, t, acc);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

}  // namespace gpmg
