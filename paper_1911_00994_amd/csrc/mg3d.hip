// The 3-D form of the solver (include/gpmg3.h): geometry of Sect. 3.1 - 3.3 carried to three dimensions (trilinear
// level set on the half-step lattice, Alg. 1, triquadratic ghost rows on the 27-point upwind stencil), the
// relaxation of Sect. 4.1 with a 7-unknown box per cell in the colour order (i + 2j + 3k) mod 7, fictitious-time
// ghost sweeps, xi and the mean-pressure row, staggered restriction and trilinear prolongation, an exact coarsest
// solve (explicit inverse), and GCR around the cycle.  Every array is a full grid (4 W^3 + 1 doubles per vector);
// ghost rows are a compact structure of arrays numbered in point order.  All arithmetic FP64; the file is compiled
// without FMA contraction so that the geometry decisions (Alg. 1's sign tests) follow the plain FP64 order.
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gpmg3.h"
#include "internal.h"

namespace gpmg {
namespace d3 {

enum : uint8_t { C_INACTIVE = 0, C_INT = 1, C_GHOST = 2, C_WALLD = 3, C_WALLG = 4, C_BODY = 6, C_GHOSTX = 7 };
constexpr int T3 = 256;
constexpr int RB = 1024;  // blocks of the grid reductions
inline int nb3(long n) { return (int)((n + T3 - 1) / T3); }

struct LevelView {
  int N, W, Nf, lstride;
  long W3;
  double h;
  const double *phi;
};

struct Lev {
  int N = 0, W = 0, lstride = 1;
  long W3 = 0, n = 0;
  double h = 0;
  uint8_t *cls = nullptr;
  double *x = nullptr, *b = nullptr, *r = nullptr;
  int *rowof = nullptr;
  int ng = 0, gcap = 0;
  int *g_pt = nullptr, *g_col = nullptr;
  double *g_w = nullptr, *g_dtau = nullptr, *g_B = nullptr, *g_th = nullptr, *g_tmp = nullptr;
  int Mp = 0;
  LevelView view(const double *phi, int Nf) const { return LevelView{N, W, Nf, lstride, W3, h, phi}; }
};

}  // namespace d3
}  // namespace gpmg

struct gp3_ctx {
  int N = 0, L = 0;
  gp3_params prm{};
  double alpha = 0;
  int nbis = 6;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string hip_err;
  std::mutex err_mu;
  gpmg::d3::Lev lev[12];
  double *phi = nullptr;
  int have_geom = 0;
  // device scratch: flags / counters, reduction partials, scalars
  int *d_flags = nullptr;
  double *d_part = nullptr, *d_scal = nullptr;
  int *d_bcnt = nullptr;
  // coarsest level: dense map, matrix and its inverse
  int nc = 0, c_ok = 0;
  int *c_map = nullptr;
  double *c_A = nullptr, *c_inv = nullptr, *c_b = nullptr, *c_x = nullptr;
  // GCR workspace
  int kr_m = 0;
  double *kr_r = nullptr, *kr_z = nullptr, *kr_q = nullptr, *kr_Q = nullptr, *kr_Z = nullptr, *kr_zero = nullptr;
  double *kr_s = nullptr;
};

namespace gpmg {
namespace d3 {

using Ctx3 = gp3_ctx;

#define G3_HIP(call)                                                    \
  do {                                                                  \
    hipError_t e_ = (call);                                             \
    if (e_ != hipSuccess) {                                             \
      std::lock_guard<std::mutex> lk_(ctx->err_mu);                     \
      ctx->hip_err = std::string(#call) + ": " + hipGetErrorString(e_); \
      return GP_EHIP;                                                   \
    }                                                                   \
  } while (0)

// ---------------------------------------------------------------------------------------------------------
// indexing and the level set
// ---------------------------------------------------------------------------------------------------------
__device__ __forceinline__ long gi(const LevelView &L, int g, int i, int j, int k) {
  return g * L.W3 + ((long)(k + 1) * L.W + (j + 1)) * L.W + (i + 1);
}
__device__ __forceinline__ bool in3(const LevelView &L, int i, int j, int k) {
  return i >= -1 && i <= L.N && j >= -1 && j <= L.N && k >= -1 && k <= L.N;
}
__device__ __forceinline__ void unpack(const LevelView &L, long p, int &g, int &i, int &j, int &k) {
  g = (int)(p / L.W3);
  long q = p - g * L.W3;
  k = (int)(q / ((long)L.W * L.W)) - 1;
  q -= (long)(k + 1) * L.W * L.W;
  j = (int)(q / L.W) - 1;
  i = (int)(q - (long)(j + 1) * L.W) - 1;
}
__device__ __forceinline__ double ofs(int g, int d) { return (g == d) ? 0.0 : 0.5; }
__device__ __forceinline__ void node_xyz(const LevelView &L, int g, int i, int j, int k, double X[3]) {
  X[0] = -1.0 + (i + ofs(g, 0)) * L.h;
  X[1] = -1.0 + (j + ofs(g, 1)) * L.h;
  X[2] = -1.0 + (k + ofs(g, 2)) * L.h;
}
__device__ __forceinline__ bool valued(int c) {
  return c == C_INT || c == C_GHOST || c == C_GHOSTX || c == C_WALLD || c == C_WALLG;
}
__device__ __forceinline__ bool rowed(int c) { return c == C_GHOST || c == C_GHOSTX || c == C_WALLG; }
__device__ __forceinline__ double lat(const LevelView &L, int a, int b, int c) {
  const long n = 2L * L.Nf + 1, s = L.lstride;
  return L.phi[((long)c * s * n + (long)b * s) * n + (long)a * s];
}
// value and gradient of the trilinear interpolant on the lattice cell holding X (half-open, clamped)
__device__ void trilin(const LevelView &L, const double X[3], double *val, double g[3]) {
  const double hl = 0.5 * L.h;
  const int nl = 2 * L.N + 1;
  int c[3];
  double t[3];
  for (int d = 0; d < 3; d++) {
    const double f = (X[d] + 1.0) / hl;
    c[d] = (int)floor(f);
    if (c[d] < 0) c[d] = 0;
    if (c[d] > nl - 2) c[d] = nl - 2;
    t[d] = f - c[d];
  }
  double v[2][2][2];
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++)
      for (int e = 0; e < 2; e++) v[e][b][a] = lat(L, c[0] + a, c[1] + b, c[2] + e);
  double s = 0, gx = 0, gy = 0, gz = 0;
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++)
      for (int e = 0; e < 2; e++) {
        const double wx = a ? t[0] : 1 - t[0], wy = b ? t[1] : 1 - t[1], wz = e ? t[2] : 1 - t[2];
        const double dx = a ? 1 : -1, dy = b ? 1 : -1, dz = e ? 1 : -1;
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
__device__ void normal_at(const LevelView &L, const double X[3], double n[3]) {
  double g[3];
  trilin(L, X, nullptr, g);
  const double m = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  for (int d = 0; d < 3; d++) n[d] = m > 0 ? g[d] / m : 0.0;
}
// Alg. 1 in 3-D: march against the normal by h/2 while the interpolant is positive (at most march_max steps),
// then nbis halvings of the last step; the boundary point is the last midpoint
__device__ bool boundary_point(const LevelView &L, const double G[3], double phig, int march_max, int nbis, double B[3]) {
  double H[3] = {G[0], G[1], G[2]}, K[3] = {G[0], G[1], G[2]}, ph = phig;
  int it = 0;
  while (ph > 0) {
    if (it == march_max) return false;
    double n[3];
    for (int d = 0; d < 3; d++) K[d] = H[d];
    normal_at(L, H, n);
    for (int d = 0; d < 3; d++) H[d] -= 0.5 * L.h * n[d];
    trilin(L, H, &ph, nullptr);
    it++;
  }
  if (it == 0 || ph == 0.0) {
    for (int d = 0; d < 3; d++) B[d] = H[d];
    return true;
  }
  double M[3] = {H[0], H[1], H[2]};
  for (int q = 0; q < nbis; q++) {
    for (int d = 0; d < 3; d++) M[d] = 0.5 * (H[d] + K[d]);
    double pm;
    trilin(L, M, &pm, nullptr);
    if (pm * ph < 0) {
      for (int d = 0; d < 3; d++) K[d] = M[d];
    } else {
      for (int d = 0; d < 3; d++) H[d] = M[d];
      ph = pm;
    }
  }
  for (int d = 0; d < 3; d++) B[d] = M[d];
  return true;
}
__device__ __forceinline__ void lag3(double t, double T[3]) {
  T[0] = (1 - t) * (2 - t) / 2;
  T[1] = t * (2 - t);
  T[2] = t * (t - 1) / 2;
}
__device__ __forceinline__ void dlag3(double t, double D[3]) {
  D[0] = t - 1.5;
  D[1] = 2 - 2 * t;
  D[2] = t - 0.5;
}
// the 27-point upwind stencil of (g, i, j, k): the signs of the normal there and the columns (false if it leaves
// the arrays; such columns point at the ghost itself)
__device__ bool stencil27(const LevelView &L, int g, int i, int j, int k, double s[3], long col[27]) {
  double X[3], n[3];
  node_xyz(L, g, i, j, k, X);
  normal_at(L, X, n);
  for (int d = 0; d < 3; d++) s[d] = n[d] >= 0 ? 1.0 : -1.0;
  bool ok = true;
  for (int c = 0; c < 3; c++)
    for (int b = 0; b < 3; b++)
      for (int a = 0; a < 3; a++) {
        const int ii = i - (int)s[0] * a, jj = j - (int)s[1] * b, kk = k - (int)s[2] * c;
        if (!in3(L, ii, jj, kk)) {
          ok = false;
          col[(c * 3 + b) * 3 + a] = gi(L, g, i, j, k);
        } else {
          col[(c * 3 + b) * 3 + a] = gi(L, g, ii, jj, kk);
        }
      }
  return ok;
}
// columns of the internal row of (g, i, j, k): u, v, w rows read 7 own values and 2 pressures, the continuity row
// the 6 faces
__device__ int int_cols(const LevelView &L, int g, int i, int j, int k, long *cols) {
  int m = 0;
  if (g < 3) {
    cols[m++] = gi(L, g, i, j, k);
    cols[m++] = gi(L, g, i + 1, j, k);
    cols[m++] = gi(L, g, i - 1, j, k);
    cols[m++] = gi(L, g, i, j + 1, k);
    cols[m++] = gi(L, g, i, j - 1, k);
    cols[m++] = gi(L, g, i, j, k + 1);
    cols[m++] = gi(L, g, i, j, k - 1);
    cols[m++] = gi(L, 3, i, j, k);
    cols[m++] = gi(L, 3, i - (g == 0), j - (g == 1), k - (g == 2));
  } else {
    cols[m++] = gi(L, 0, i, j, k);
    cols[m++] = gi(L, 0, i + 1, j, k);
    cols[m++] = gi(L, 1, i, j, k);
    cols[m++] = gi(L, 1, i, j + 1, k);
    cols[m++] = gi(L, 2, i, j, k);
    cols[m++] = gi(L, 2, i, j, k + 1);
  }
  return m;
}

// ---------------------------------------------------------------------------------------------------------
// geometry kernels
// ---------------------------------------------------------------------------------------------------------
__global__ void k_sample(int kind, double p0, double p1, double p2, double c0, double c1, double c2, int N, double *phi) {
  const long n = 2L * N + 1, t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= n * n * n) return;
  const int a = (int)(t % n), b = (int)((t / n) % n), c = (int)(t / (n * n));
  const double hl = 1.0 / N;
  const double X = -1 + a * hl - c0, Y = -1 + b * hl - c1, Z = -1 + c * hl - c2;
  phi[t] = kind == 0 ? p0 - sqrt(X * X + Y * Y + Z * Z)
                     : 1.0 - sqrt(X * X / (p0 * p0) + Y * Y / (p1 * p1) + Z * Z / (p2 * p2));
}

__global__ void k_classify(LevelView L, uint8_t *cls) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p >= 4 * L.W3) return;
  int g, i, j, k;
  unpack(L, p, g, i, j, k);
  const int I[3] = {i, j, k}, N = L.N;
  int out = 0, ring = -1;
  bool normal_wall = false;
  for (int d = 0; d < 3; d++) {
    const int hi = (g < 3 && d == g) ? N : N - 1;
    if (I[d] < 0 || I[d] > hi) {
      out++;
      ring = d;
    }
    if (g < 3 && d == g && (I[d] == 0 || I[d] == N)) normal_wall = true;
  }
  uint8_t c = C_INACTIVE;
  if (g == 3) {
    if (out) {
      cls[p] = C_INACTIVE;
      return;
    }
  } else {
    if (out >= 2) {
      cls[p] = C_INACTIVE;
      return;
    }
    if (out == 1) {
      cls[p] = ring != g ? C_WALLG : C_INACTIVE;
      return;
    }
    if (normal_wall) {
      cls[p] = C_WALLD;
      return;
    }
  }
  const int a = 2 * i + (g == 0 ? 0 : 1), b = 2 * j + (g == 1 ? 0 : 1), cc = 2 * k + (g == 2 ? 0 : 1);
  c = lat(L, a, b, cc) < 0 ? C_INT : C_BODY;
  cls[p] = c;
}
// ghosts: body points read by internal rows
__global__ void k_seed(LevelView L, uint8_t *cls) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p >= 4 * L.W3 || cls[p] != C_INT) return;
  int g, i, j, k;
  unpack(L, p, g, i, j, k);
  long cols[9];
  const int m = int_cols(L, g, i, j, k, cols);
  for (int q = 0; q < m; q++)
    if (cls[cols[q]] == C_BODY) cls[cols[q]] = C_GHOST;
}
// closure under the ghosts' 27-point stencils (repeated until nothing changes)
__global__ void k_closure(LevelView L, uint8_t *cls, int *changed) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p >= 4 * L.W3 || cls[p] != C_GHOST) return;
  int g, i, j, k;
  unpack(L, p, g, i, j, k);
  double s[3];
  long col[27];
  stencil27(L, g, i, j, k, s, col);
  for (int q = 0; q < 27; q++)
    if (cls[col[q]] == C_BODY) {
      cls[col[q]] = C_GHOST;
      *changed = 1;
    }
}
__global__ void k_body_off(long P, uint8_t *cls) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p < P && cls[p] == C_BODY) cls[p] = C_INACTIVE;
}
// row numbering in point order: per-block counts, one-block scan, per-block assignment
constexpr int NB_T = 1024;
__global__ void __launch_bounds__(NB_T) k_row_count(long P, const uint8_t *cls, int *bcnt) {
  __shared__ int sm[NB_T / 64];
  const long p = blockIdx.x * (long)NB_T + threadIdx.x;
  const bool f = p < P && (cls[p] == C_GHOST || cls[p] == C_WALLG);
  const unsigned long long bal = __ballot(f);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int q = 0; q < NB_T / 64; q++) t += sm[q];
    bcnt[blockIdx.x] = t;
  }
}
__global__ void __launch_bounds__(NB_T) k_scan(int *bcnt, int nb, int *total) {
  __shared__ int sm[NB_T];
  int run = 0;
  for (int o = 0; o < nb; o += NB_T) {
    const int t = o + threadIdx.x;
    const int v = t < nb ? bcnt[t] : 0;
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int s = 1; s < NB_T; s <<= 1) {
      const int a = threadIdx.x >= s ? sm[threadIdx.x - s] : 0;
      __syncthreads();
      sm[threadIdx.x] += a;
      __syncthreads();
    }
    if (t < nb) bcnt[t] = run + sm[threadIdx.x] - v;
    run += sm[NB_T - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = run;
}
__global__ void __launch_bounds__(NB_T) k_row_assign(long P, const uint8_t *cls, const int *boff, int *rowof, int *g_pt,
                                                     int gcap) {
  __shared__ int sm[NB_T / 64];
  const long p = blockIdx.x * (long)NB_T + threadIdx.x;
  const bool f = p < P && (cls[p] == C_GHOST || cls[p] == C_WALLG);
  const unsigned long long bal = __ballot(f);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sm[wv] = __popcll(bal);
  __syncthreads();
  int before = 0;
  for (int q = 0; q < wv; q++) before += sm[q];
  const int mine = __popcll(bal & ((1ull << lane) - 1ull));
  if (p < P) {
    if (f) {
      const int r = boff[blockIdx.x] + before + mine;
      rowof[p] = r;
      if (r < gcap) g_pt[r] = (int)p;  // more rows than the tables hold: the caller reports it
    } else {
      rowof[p] = -1;
    }
  }
}
struct RowArgs {
  int ng, level, march_max, nbis;
  double dtau_dir, dtau_neu, cg_min;
  int *g_pt, *g_col;
  double *g_w, *g_dtau, *g_B, *g_th;
};
// the rows of ghosts and wall ghosts; an unusable body row turns its point into an extrapolation ghost
__global__ void k_rows(LevelView L, uint8_t *cls, RowArgs A) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= A.ng) return;
  const long p = A.g_pt[r];
  int g, i, j, k;
  unpack(L, p, g, i, j, k);
  int *col = A.g_col + 27L * r;
  double *w = A.g_w + 27L * r;
  for (int q = 0; q < 27; q++) {
    col[q] = (int)p;
    w[q] = 0.0;
  }
  const int N = L.N;
  if (cls[p] == C_WALLG) {
    const int I[3] = {i, j, k};
    int d0 = -1;
    for (int d = 0; d < 3; d++)
      if (I[d] < 0 || I[d] > (d == g ? N : N - 1)) d0 = d;
    const int st = I[d0] < 0 ? 1 : -1;
    double T[3];
    lag3(0.5, T);
    for (int m = 0; m < 3; m++) {
      int J[3] = {i, j, k};
      J[d0] += st * m;
      col[m] = (int)gi(L, g, J[0], J[1], J[2]);
      w[m] = T[m];
    }
    A.g_dtau[r] = A.dtau_dir;
    double X[3];
    node_xyz(L, g, i, j, k, X);
    X[d0] = I[d0] < 0 ? -1.0 : 1.0;
    for (int d = 0; d < 3; d++) {
      A.g_B[3 * r + d] = X[d];
      A.g_th[3 * r + d] = 0.0;
    }
    return;
  }
  double G[3], B[3] = {0, 0, 0}, s[3], th[3], n[3];
  long c27[27];
  node_xyz(L, g, i, j, k, G);
  const int a = 2 * i + (g == 0 ? 0 : 1), b = 2 * j + (g == 1 ? 0 : 1), c = 2 * k + (g == 2 ? 0 : 1);
  const double phig = lat(L, a, b, c);
  bool ok = stencil27(L, g, i, j, k, s, c27);
  ok = boundary_point(L, G, phig, A.march_max, A.nbis, B) && ok;
  for (int d = 0; d < 3; d++) th[d] = s[d] * (G[d] - B[d]) / L.h;
  for (int q = 0; q < 27; q++) {
    const int cq = cls[c27[q]];
    if (!valued(cq) || cq == C_WALLG) ok = false;
  }
  for (int d = 0; d < 3; d++)
    if (!(th[d] > -0.5 && th[d] < 1.0)) ok = false;
  double wt[27];
  double T[3][3];
  for (int d = 0; d < 3; d++) lag3(th[d], T[d]);
  if (g < 3) {
    for (int cc = 0; cc < 3; cc++)
      for (int bb = 0; bb < 3; bb++)
        for (int aa = 0; aa < 3; aa++) wt[(cc * 3 + bb) * 3 + aa] = T[0][aa] * T[1][bb] * T[2][cc];
    A.g_dtau[r] = A.dtau_dir;
  } else {
    double D[3][3];
    for (int d = 0; d < 3; d++) dlag3(th[d], D[d]);
    normal_at(L, B, n);
    for (int cc = 0; cc < 3; cc++)
      for (int bb = 0; bb < 3; bb++)
        for (int aa = 0; aa < 3; aa++)
          wt[(cc * 3 + bb) * 3 + aa] =
              -(n[0] * s[0] * D[0][aa] * T[1][bb] * T[2][cc] + n[1] * s[1] * T[0][aa] * D[1][bb] * T[2][cc] +
                n[2] * s[2] * T[0][aa] * T[1][bb] * D[2][cc]) / L.h;
    A.g_dtau[r] = A.dtau_neu;
  }
  const double diag = g < 3 ? wt[0] : wt[0] * L.h;
  if (!(diag > (A.level == 0 ? 0.0 : A.cg_min))) ok = false;
  for (int d = 0; d < 3; d++) {
    A.g_B[3 * r + d] = B[d];
    A.g_th[3 * r + d] = th[d];
  }
  if (ok) {
    for (int q = 0; q < 27; q++) {
      col[q] = (int)c27[q];
      w[q] = wt[q];
    }
  } else {
    cls[p] = C_GHOSTX;
  }
}
// extrapolation rows x_G - sum w x_q = 0 of the unusable ghosts: along the grid axis closest to the normal (then the
// others), from the first three consecutive internal / ghost / wall points towards the fluid; without sources the
// identity on coarse levels and a geometry error on the finest
__global__ void k_extrap(LevelView L, const uint8_t *cls, RowArgs A, int *bad) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= A.ng) return;
  const long p = A.g_pt[r];
  if (cls[p] != C_GHOSTX) return;
  int g, i, j, k;
  unpack(L, p, g, i, j, k);
  int *col = A.g_col + 27L * r;
  double *w = A.g_w + 27L * r;
  A.g_dtau[r] = 1.0;
  double X[3], n[3];
  node_xyz(L, g, i, j, k, X);
  normal_at(L, X, n);
  int order[3] = {0, 1, 2};
  for (int a = 0; a < 3; a++)
    for (int b = a + 1; b < 3; b++)
      if (fabs(n[order[b]]) > fabs(n[order[a]])) {
        const int t = order[a];
        order[a] = order[b];
        order[b] = t;
      }
  for (int q = 0; q < 3; q++) {
    const int ax = order[q], sg = n[ax] >= 0 ? 1 : -1;
    int di[3] = {0, 0, 0};
    di[ax] = -sg;
    for (int k0 = 1; k0 <= 4; k0++) {
      bool okk = true;
      long c3[3];
      for (int m = 0; m < 3; m++) {
        const int ii = i + di[0] * (k0 + m), jj = j + di[1] * (k0 + m), kk = k + di[2] * (k0 + m);
        if (!in3(L, ii, jj, kk)) {
          okk = false;
          break;
        }
        const long pp = gi(L, g, ii, jj, kk);
        const int c = cls[pp];
        if (!(c == C_INT || c == C_GHOST || c == C_WALLD)) {
          okk = false;
          break;
        }
        c3[m] = pp;
      }
      if (!okk) continue;
      const double t0 = k0, t1 = k0 + 1, t2 = k0 + 2;
      const double w0 = (0 - t1) * (0 - t2) / ((t0 - t1) * (t0 - t2));
      const double w1 = (0 - t0) * (0 - t2) / ((t1 - t0) * (t1 - t2));
      const double w2 = (0 - t0) * (0 - t1) / ((t2 - t0) * (t2 - t1));
      w[0] = 1.0;
      col[0] = (int)p;
      col[1] = (int)c3[0];
      col[2] = (int)c3[1];
      col[3] = (int)c3[2];
      w[1] = -w0;
      w[2] = -w1;
      w[3] = -w2;
      return;
    }
  }
  w[0] = 1.0;
  col[0] = (int)p;
  if (A.level == 0) atomicOr(bad, 1);
}
// internal pressure count, and the flag of an internal cell without an internal face
__global__ void k_cells(LevelView L, const uint8_t *cls, int *mp, int *bad) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int N = L.N;
  if (t >= (long)N * N * N) return;
  const int i = (int)(t % N), j = (int)((t / N) % N), k = (int)(t / ((long)N * N));
  if (cls[gi(L, 3, i, j, k)] != C_INT) return;
  atomicAdd(mp, 1);
  const long f[6] = {gi(L, 0, i, j, k), gi(L, 0, i + 1, j, k), gi(L, 1, i, j, k),
                     gi(L, 1, i, j + 1, k), gi(L, 2, i, j, k), gi(L, 2, i, j, k + 1)};
  bool any = false;
  for (int q = 0; q < 6; q++) any |= cls[f[q]] == C_INT;
  if (!any) atomicOr(bad, 2);
}

// ---------------------------------------------------------------------------------------------------------
// rows, residual, relaxation
// ---------------------------------------------------------------------------------------------------------
struct RowTab {
  const uint8_t *cls;
  const int *rowof, *g_col;
  const double *g_w;
  double a, d, ih;
};
// (M x)_p of the row of point p (0 without a row; the mean row is separate)
__device__ double row_dot(const LevelView &L, const RowTab &R, long p, const double *x) {
  const int c = R.cls[p];
  if (c == C_WALLD) return x[p];
  if (rowed(c)) {
    const int r = R.rowof[p];
    double s = 0;
    for (int q = 0; q < 27; q++) s += R.g_w[27L * r + q] * x[R.g_col[27L * r + q]];
    return s;
  }
  if (c != C_INT) return 0.0;
  int g, i, j, k;
  unpack(L, p, g, i, j, k);
  if (g < 3) {
    const double nb = x[gi(L, g, i + 1, j, k)] + x[gi(L, g, i - 1, j, k)] + x[gi(L, g, i, j + 1, k)] +
                      x[gi(L, g, i, j - 1, k)] + x[gi(L, g, i, j, k + 1)] + x[gi(L, g, i, j, k - 1)];
    const double pe = x[gi(L, 3, i, j, k)], pw = x[gi(L, 3, i - (g == 0), j - (g == 1), k - (g == 2))];
    return R.d * x[p] - R.a * nb + (pe - pw) * R.ih;
  }
  const double div = x[gi(L, 0, i + 1, j, k)] - x[gi(L, 0, i, j, k)] + x[gi(L, 1, i, j + 1, k)] - x[gi(L, 1, i, j, k)] +
                     x[gi(L, 2, i, j, k + 1)] - x[gi(L, 2, i, j, k)];
  return div * R.ih - x[4 * L.W3];
}

// block partials of a sum (slot 0) and a max (slot 1) over RB blocks, then the totals
__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wmax(double v) {
  for (int o = 32; o > 0; o >>= 1) {
    const double u = __shfl_xor(v, o, 64);
    v = (u > v || u != u) ? u : v;
  }
  return v;
}
// r = b - M x on every point row; part[blk] = max |r| of the block, part[RB + blk] = sum of the internal p of the
// block (for the mean row)
__global__ void __launch_bounds__(T3) k_resid(LevelView L, RowTab R, const double *x, const double *b, double *r,
                                              double *part, int store) {
  __shared__ double sm[2][T3 / 64];
  const long P = 4 * L.W3;
  double m = 0, ps = 0;
  for (long p = blockIdx.x * (long)T3 + threadIdx.x; p < P; p += (long)RB * T3) {
    const int c = R.cls[p];
    const double v = (c == C_INT || c == C_WALLD || rowed(c)) ? b[p] - row_dot(L, R, p, x) : 0.0;
    if (store) r[p] = v;
    const double av = fabs(v);
    m = (av > m || av != av) ? av : m;
    if (p >= 3 * L.W3 && c == C_INT) ps += x[p];
  }
  m = wmax(m);
  ps = wsum(ps);
  if ((threadIdx.x & 63) == 0) {
    sm[0][threadIdx.x >> 6] = m;
    sm[1][threadIdx.x >> 6] = ps;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, s = 0;
    for (int q = 0; q < T3 / 64; q++) {
      a = (sm[0][q] > a || sm[0][q] != sm[0][q]) ? sm[0][q] : a;
      s += sm[1][q];
    }
    part[blockIdx.x] = a;
    part[RB + blockIdx.x] = s;
  }
}
// the mean row's residual and the max norm: out[0] = max norm, r[P] = b[P] - (sum p) / Mp
__global__ void __launch_bounds__(RB) k_resid_fin(const double *part, double bmean, int mp, double *r, long P,
                                                  double *out, int store) {
  __shared__ double sm[2][RB / 64];
  double m = part[threadIdx.x], s = part[RB + threadIdx.x];
  m = wmax(m);
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) {
    sm[0][threadIdx.x >> 6] = m;
    sm[1][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, t = 0;
    for (int q = 0; q < RB / 64; q++) {
      a = (sm[0][q] > a || sm[0][q] != sm[0][q]) ? sm[0][q] : a;
      t += sm[1][q];
    }
    const double rm = bmean - t / mp;
    if (store) r[P] = rm;
    const double ar = fabs(rm);
    out[0] = (ar > a || ar != ar) ? ar : a;
  }
}

// the box of cell (i, j, k): pairs of opposite faces solved in terms of the cell's pressure, then the pressure from
// the continuity row (the block's exact solution; faces and pressure that are not internal are held fixed)
__device__ void box_update(const LevelView &L, const RowTab &R, double *x, const double *b, int i, int j, int k) {
  const long W3 = L.W3;
  const long c0 = gi(L, 3, i, j, k), pc = c0;
  const double a = R.a, d = R.d, ih = R.ih;
  // faces: lo / hi of axis e are the points (e, cell) and (e, cell + 1 along e)
  long lo[3], hi[3];
  bool flo[3], fhi[3];
  for (int e = 0; e < 3; e++) {
    lo[e] = gi(L, e, i, j, k);
    hi[e] = gi(L, e, i + (e == 0), j + (e == 1), k + (e == 2));
    flo[e] = R.cls[lo[e]] == C_INT;
    fhi[e] = R.cls[hi[e]] == C_INT;
  }
  const bool fP = R.cls[pc] == C_INT;
  if (!(fP || flo[0] || fhi[0] || flo[1] || fhi[1] || flo[2] || fhi[2])) return;
  const double xi = x[4 * W3], p0 = x[pc];
  double A_lo[3], B_lo[3], A_hi[3], B_hi[3];
  for (int e = 0; e < 3; e++) {
    const long st = (e == 0) ? 1 : (e == 1 ? L.W : (long)L.W * L.W);
    const long f0 = lo[e] - e * W3, f1 = hi[e] - e * W3;  // position within the grid
    const double *u = x + e * W3;
    // lateral neighbours (the two other axes) of each face; only the rows of internal faces are formed (their
    // stencils stay inside the padded grids)
    const long s1 = (e == 0) ? L.W : 1, s2 = (e == 2) ? L.W : (long)L.W * L.W;
    double Rlo = 0, Rhi = 0;
    if (flo[e]) {
      // row of the lo face: d u_lo - a (u_lo-1 + u_hi + lateral) + ih (p_c - p beyond) = b_lo
      const double lat0 = u[f0 + s1] + u[f0 - s1] + u[f0 + s2] + u[f0 - s2];
      Rlo = b[lo[e]] + a * (u[f0 - st] + lat0) + ih * x[3 * W3 + f0 - st];
      if (!fhi[e]) Rlo += a * u[f1];
      if (!fP) Rlo -= ih * p0;
    }
    if (fhi[e]) {
      // row of the hi face: d u_hi - a (u_hi+1 + u_lo + lateral) + ih (p beyond - p_c) = b_hi
      const double lat1 = u[f1 + s1] + u[f1 - s1] + u[f1 + s2] + u[f1 - s2];
      Rhi = b[hi[e]] + a * (u[f1 + st] + lat1) - ih * x[3 * W3 + f1];
      if (!flo[e]) Rhi += a * u[f0];
      if (!fP) Rhi += ih * p0;
    }
    A_lo[e] = B_lo[e] = A_hi[e] = B_hi[e] = 0;
    if (flo[e] && fhi[e]) {
      const double det = d * d - a * a;
      A_lo[e] = (d * Rlo + a * Rhi) / det;
      A_hi[e] = (a * Rlo + d * Rhi) / det;
      B_lo[e] = -ih / (d + a);
      B_hi[e] = ih / (d + a);
    } else if (flo[e]) {
      A_lo[e] = Rlo / d;
      B_lo[e] = -ih / d;
    } else if (fhi[e]) {
      A_hi[e] = Rhi / d;
      B_hi[e] = ih / d;
    }
  }
  double pn = p0;
  if (fP) {
    double SA = 0, SB = 0;
    for (int e = 0; e < 3; e++) {
      SA += (fhi[e] ? A_hi[e] : x[hi[e]]) - (flo[e] ? A_lo[e] : x[lo[e]]);
      SB += (fhi[e] ? B_hi[e] : 0.0) - (flo[e] ? B_lo[e] : 0.0);
    }
    if (SB == 0.0) return;  // no internal face: the block is singular, the box is skipped
    pn = ((b[pc] + xi) * L.h - SA) / SB;
    x[pc] = pn;
  }
  for (int e = 0; e < 3; e++) {
    const double bp = fP ? pn : 0.0;
    if (flo[e]) x[lo[e]] = A_lo[e] + B_lo[e] * bp;
    if (fhi[e]) x[hi[e]] = A_hi[e] + B_hi[e] * bp;
  }
  (void)c0;
}
// the boxes of one colour (i + 2j + 3k) mod 7 = col: thread t -> row (j, k) and the m-th cell of the colour in it
__global__ void k_box(LevelView L, RowTab R, double *x, const double *b, int col) {
  const int N = L.N, K7 = N / 7 + 1;
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)K7 * N * N) return;
  const int m = (int)(t % K7), jk = (int)(t / K7), j = jk % N, k = jk / N;
  const int i = ((col - 2 * j - 3 * k) % 7 + 7) % 7 + 7 * m;
  if (i >= N) return;
  box_update(L, R, x, b, i, j, k);
}
// fictitious-time sweep of every ghost row (eq. (ghostrelax)), simultaneous: new values first, then written
__global__ void k_ghost_a(LevelView L, RowTab R, const int *g_pt, const double *dtau, int ng, const double *x,
                          const double *b, double *tmp) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ng) return;
  const long p = g_pt[r];
  tmp[r] = x[p] + dtau[r] * (b[p] - row_dot(L, R, p, x));
}
__global__ void k_ghost_b(const int *g_pt, int ng, const double *tmp, double *x) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < ng) x[g_pt[r]] = tmp[r];
}
// xi <- mean over the internal cells of (div_h u - g): block partials, then the total
__global__ void __launch_bounds__(T3) k_xi_part(LevelView L, RowTab R, const double *x, const double *b, double *part) {
  __shared__ double sm[T3 / 64];
  double s = 0;
  for (long q = blockIdx.x * (long)T3 + threadIdx.x; q < L.W3; q += (long)RB * T3) {
    const long p = 3 * L.W3 + q;
    if (R.cls[p] == C_INT) s += (row_dot(L, R, p, x) + x[4 * L.W3]) - b[p];
  }
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int q = 0; q < T3 / 64; q++) t += sm[q];
    part[blockIdx.x] = t;
  }
}
__global__ void __launch_bounds__(RB) k_sum_fin(const double *part, double scale, double *out) {
  __shared__ double sm[RB / 64];
  double s = wsum(part[threadIdx.x]);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int q = 0; q < RB / 64; q++) t += sm[q];
    *out = t * scale;
  }
}
// mean of the internal pressure (block partials) and the shift of every pressure unknown by it
__global__ void __launch_bounds__(T3) k_pmean_part(LevelView L, const uint8_t *cls, const double *x, double *part) {
  __shared__ double sm[T3 / 64];
  double s = 0;
  for (long q = blockIdx.x * (long)T3 + threadIdx.x; q < L.W3; q += (long)RB * T3)
    if (cls[3 * L.W3 + q] == C_INT) s += x[3 * L.W3 + q];
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int q = 0; q < T3 / 64; q++) t += sm[q];
    part[blockIdx.x] = t;
  }
}
__global__ void k_pshift(LevelView L, const uint8_t *cls, double *x, const double *mean, const double *extra) {
  const long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (q >= L.W3) return;
  const int c = cls[3 * L.W3 + q];
  if (c == C_INT || c == C_GHOST || c == C_GHOSTX) x[3 * L.W3 + q] += (extra ? *extra : 0.0) - *mean;
}
__global__ void k_set_walld(long P, const uint8_t *cls, double *x, const double *b) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p < P && cls[p] == C_WALLD) x[p] = b[p];
}
__global__ void k_fill(double *x, long n, double v) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < n) x[t] = v;
}
// entries without an equation set to zero
__global__ void k_mask(long P, const uint8_t *cls, double *z) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int c = cls[p];
  if (!(c == C_INT || rowed(c) || c == C_WALLD)) z[p] = 0.0;
}

// ---------------------------------------------------------------------------------------------------------
// transfers
// ---------------------------------------------------------------------------------------------------------
// restriction of the fine residual to the coarse right-hand side (internal and boundary-condition ghost rows):
// staggered weights (1 2 1)/4 along the grid's own axis, 1/2, 1/2 across, where every fine point exists and has the
// coarse point's class; otherwise the mean over the fine points that do; none: 0
__global__ void k_restrict(LevelView F, const uint8_t *clsf, const double *rf, LevelView C, const uint8_t *clsc,
                           double *bc) {
  const long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long PC = 4 * C.W3;
  if (q > PC) return;
  if (q == PC) {
    bc[q] = 0.0;
    return;
  }
  bc[q] = 0.0;
  const int cc = clsc[q];
  if (!(cc == C_INT || cc == C_GHOST)) return;
  int g, I, J, K;
  unpack(C, q, g, I, J, K);
  const int IJK[3] = {I, J, K};
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
      wts[d][2] = 0;
    }
  }
  double s = 0, su = 0;
  bool all = true;
  int cnt = 0;
  for (int c = 0; c < n3[2]; c++)
    for (int b = 0; b < n3[1]; b++)
      for (int a = 0; a < n3[0]; a++) {
        const int i = lo[0] + a, j = lo[1] + b, k = lo[2] + c;
        if (!in3(F, i, j, k) || clsf[gi(F, g, i, j, k)] != cc) {
          all = false;
          continue;
        }
        const double v = rf[gi(F, g, i, j, k)];
        s += wts[0][a] * wts[1][b] * wts[2][c] * v;
        su += v;
        cnt++;
      }
  bc[q] = all ? s : (cnt ? su / cnt : 0.0);
}
// prolongation of the coarse correction, added to the fine internal and ghost values: trilinear staggered weights
// renormalised over the coarse points that carry a value; the pressure outside the box takes the nearest cell
__global__ void k_prolong(LevelView C, const uint8_t *clsc, const double *ec, LevelView F, const uint8_t *clsf,
                          double *xf) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long PF = 4 * F.W3;
  if (p > PF) return;
  if (p == PF) {
    xf[p] += ec[4 * C.W3];
    return;
  }
  const int cf = clsf[p];
  if (!(cf == C_INT || cf == C_GHOST || cf == C_GHOSTX)) return;
  int g, i, j, k;
  unpack(F, p, g, i, j, k);
  const int IJK[3] = {i, j, k};
  int ci[3][2], nn[3];
  double cw[3][2];
  for (int d = 0; d < 3; d++) {
    const int f = IJK[d];
    if (g == d) {
      if ((f & 1) == 0) {
        ci[d][0] = f / 2;
        ci[d][1] = 0;
        cw[d][0] = 1;
        cw[d][1] = 0;
        nn[d] = 1;
      } else {
        ci[d][0] = (f - 1) / 2;
        ci[d][1] = (f + 1) / 2;
        cw[d][0] = cw[d][1] = 0.5;
        nn[d] = 2;
      }
    } else {
      const int c0 = (f >= 0) ? f / 2 : -1;
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
          I = I < 0 ? 0 : (I > C.N - 1 ? C.N - 1 : I);
          J = J < 0 ? 0 : (J > C.N - 1 ? C.N - 1 : J);
          K = K < 0 ? 0 : (K > C.N - 1 ? C.N - 1 : K);
        }
        if (!in3(C, I, J, K)) continue;
        const long q = gi(C, g, I, J, K);
        if (!valued(clsc[q])) continue;
        const double w = cw[0][a] * cw[1][b] * cw[2][c];
        s += w * ec[q];
        sw += w;
      }
  if (sw > 0) xf[p] += s / sw;
}

// ---------------------------------------------------------------------------------------------------------
// coarsest level: dense map (point order), matrix, Gauss-Jordan inverse, product
// ---------------------------------------------------------------------------------------------------------
__global__ void k_cmap(long P, const uint8_t *cls, int *map, int *nc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int n = 0;
  for (long p = 0; p < P; p++) {
    const int c = cls[p];
    map[p] = (c == C_INT || c == C_WALLD || rowed(c)) ? n++ : -1;
  }
  map[P] = n++;
  *nc = n;
}
__global__ void k_cfill(LevelView L, RowTab R, const int *map, int nc, int mp, double *A) {
  const long P = 4 * L.W3;
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p > P) return;
  const int row = map[p];
  if (row < 0) return;
  double *Ar = A + (size_t)row * nc;
  if (p == P) {  // the mean row
    for (long q = 3 * L.W3; q < P; q++)
      if (R.cls[q] == C_INT) Ar[map[q]] = 1.0 / mp;
    return;
  }
  const int c = R.cls[p];
  if (c == C_WALLD) {
    Ar[row] = 1.0;
    return;
  }
  if (rowed(c)) {
    const int r = R.rowof[p];
    for (int q = 0; q < 27; q++) {
      const int col = map[R.g_col[27L * r + q]];
      if (col >= 0) Ar[col] += R.g_w[27L * r + q];
    }
    return;
  }
  int g, i, j, k;
  unpack(L, p, g, i, j, k);
  long cols[9];
  const int m = int_cols(L, g, i, j, k, cols);
  if (g < 3) {
    const double co[9] = {R.d, -R.a, -R.a, -R.a, -R.a, -R.a, -R.a, R.ih, -R.ih};
    for (int q = 0; q < m; q++)
      if (map[cols[q]] >= 0) Ar[map[cols[q]]] += co[q];
  } else {
    const double co[6] = {-R.ih, R.ih, -R.ih, R.ih, -R.ih, R.ih};
    for (int q = 0; q < m; q++)
      if (map[cols[q]] >= 0) Ar[map[cols[q]]] += co[q];
    Ar[map[P]] += -1.0;
  }
}
// Gauss-Jordan step k on the augmented [A | I] (n x 2n, row-major): the pivot row found and swapped in by one
// workgroup, then every other row eliminated by the grid
constexpr int GJ_T = 1024;
__global__ void __launch_bounds__(GJ_T) k_gj_pivot(double *M, int n, int k, int *fail) {
  __shared__ double sv[GJ_T / 64];
  __shared__ int si[GJ_T / 64];
  __shared__ int piv;
  double best = -1;
  int bi = -1;
  for (int r = k + threadIdx.x; r < n; r += GJ_T) {
    const double v = fabs(M[(size_t)r * 2 * n + k]);
    if (v > best) {
      best = v;
      bi = r;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double v2 = __shfl_xor(best, o, 64);
    const int i2 = __shfl_xor(bi, o, 64);
    if (v2 > best || (v2 == best && i2 >= 0 && (bi < 0 || i2 < bi))) {
      best = v2;
      bi = i2;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    sv[threadIdx.x >> 6] = best;
    si[threadIdx.x >> 6] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = -1;
    int i = -1;
    for (int q = 0; q < GJ_T / 64; q++)
      if (sv[q] > b || (sv[q] == b && si[q] >= 0 && (i < 0 || si[q] < i))) {
        b = sv[q];
        i = si[q];
      }
    piv = i;
    if (!(b > 0)) *fail = 1;
  }
  __syncthreads();
  const int pr = piv;
  if (pr < 0) return;
  const size_t w = 2 * (size_t)n;
  if (pr != k)
    for (size_t c = threadIdx.x; c < w; c += GJ_T) {
      const double t = M[(size_t)k * w + c];
      M[(size_t)k * w + c] = M[(size_t)pr * w + c];
      M[(size_t)pr * w + c] = t;
    }
  __syncthreads();
  const double pv = M[(size_t)k * w + k];
  __syncthreads();
  if (pv != 0.0)
    for (size_t c = threadIdx.x; c < w; c += GJ_T) M[(size_t)k * w + c] /= pv;
}
__global__ void k_gj_elim(double *M, int n, int k) {
  const size_t w = 2 * (size_t)n;
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * (long)w) return;
  const int r = (int)(t / (long)w);
  const size_t c = t - (size_t)r * w;
  if (r == k || c == (size_t)k) return;  // column k is cleared below, after every row has read it
  const double f = M[(size_t)r * w + k];
  if (f != 0.0) M[(size_t)r * w + c] -= f * M[(size_t)k * w + c];
}
__global__ void k_gj_clear(double *M, int n, int k) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n && r != k) M[(size_t)r * 2 * n + k] = 0.0;
}
__global__ void k_augment(const double *A, int n, double *M) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * 2 * n) return;
  const int r = (int)(t / (2L * n)), c = (int)(t - (long)r * 2 * n);
  M[t] = c < n ? A[(size_t)r * n + c] : (c - n == r ? 1.0 : 0.0);
}
__global__ void k_take_inv(const double *M, int n, double *inv) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * n) return;
  const int r = (int)(t / n), c = (int)(t - (long)r * n);
  inv[t] = M[(size_t)r * 2 * n + n + c];
}
// x = inv b on the coarsest level (one workgroup of 64 per row)
__global__ void __launch_bounds__(64) k_capply(const double *inv, const int *map, int nc, long P, const double *b,
                                               double *x, const double *bvec) {
  (void)bvec;
  const int row = blockIdx.x;
  if (row >= nc) return;
  // gather: the dense right-hand side is b at the mapped points (built by k_cgather into x's spare buffer)
  double s = 0;
  for (int c = threadIdx.x; c < nc; c += 64) s += inv[(size_t)row * nc + c] * b[c];
  s = wsum(s);
  if (threadIdx.x == 0) x[row] = s;
  (void)map;
  (void)P;
}
__global__ void k_cgather(long P, const int *map, const double *b, double *bd) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p <= P && map[p] >= 0) bd[map[p]] = b[p];
}
__global__ void k_cscatter(long P, const int *map, const double *xd, double *x) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p <= P) x[p] = map[p] >= 0 ? xd[map[p]] : 0.0;
}

// ---------------------------------------------------------------------------------------------------------
// GCR kernels (vectors of n doubles; block partials over RB blocks, summed in block order)
// ---------------------------------------------------------------------------------------------------------
constexpr int KMAX = 32;
// part[i * RB + blk] = (Q_i . q) over the block, i < k
__global__ void __launch_bounds__(T3) k_dots(const double *Q, long n, int k, const double *q, double *part) {
  __shared__ double sm[T3 / 64];
  for (int i = 0; i < k; i++) {
    double s = 0;
    for (long e = blockIdx.x * (long)T3 + threadIdx.x; e < n; e += (long)RB * T3) s += Q[(size_t)i * n + e] * q[e];
    s = wsum(s);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0;
      for (int w = 0; w < T3 / 64; w++) t += sm[w];
      part[(size_t)i * RB + blockIdx.x] = t;
    }
    __syncthreads();
  }
}
// out[i] = (sum of part[i]) / div[i]  (div null: no division)
__global__ void __launch_bounds__(RB) k_sums(const double *part, int cnt, const double *div, double *out) {
  __shared__ double sm[RB / 64];
  for (int i = 0; i < cnt; i++) {
    const double s = wsum(part[(size_t)i * RB + threadIdx.x]);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0;
      for (int w = 0; w < RB / 64; w++) t += sm[w];
      out[i] = div ? t / div[i] : t;
    }
    __syncthreads();
  }
}
// q -= sum beta_i Q_i, z -= sum beta_i Z_i (stored as Q_k, Z_k); partials of |q|^2 and r . q
__global__ void __launch_bounds__(T3) k_orth(const double *Q, const double *Z, long n, int k, const double *beta,
                                             const double *q, const double *z, const double *r, double *Qk, double *Zk,
                                             double *part) {
  __shared__ double sm[2][T3 / 64];
  double s2 = 0, sr = 0;
  for (long e = blockIdx.x * (long)T3 + threadIdx.x; e < n; e += (long)RB * T3) {
    double qq = q[e], zz = z[e];
    for (int i = 0; i < k; i++) {
      qq -= beta[i] * Q[(size_t)i * n + e];
      zz -= beta[i] * Z[(size_t)i * n + e];
    }
    Qk[e] = qq;
    Zk[e] = zz;
    s2 += qq * qq;
    sr += r[e] * qq;
  }
  s2 = wsum(s2);
  sr = wsum(sr);
  if ((threadIdx.x & 63) == 0) {
    sm[0][threadIdx.x >> 6] = s2;
    sm[1][threadIdx.x >> 6] = sr;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0;
    for (int w = 0; w < T3 / 64; w++) {
      a += sm[0][w];
      b += sm[1][w];
    }
    part[blockIdx.x] = a;
    part[RB + blockIdx.x] = b;
  }
}
// the stored images are Q_k = -M Z_k, so with g = (r . Q_k) / |Q_k|^2 the step is x -= g Z_k, r -= g Q_k; block
// maxima of |r|
__global__ void __launch_bounds__(T3) k_step(long n, const double *sc, const double *Qk, const double *Zk, double *x,
                                             double *r, double *part) {
  __shared__ double sm[T3 / 64];
  const double g = sc[0] > 0 ? sc[1] / sc[0] : 0.0;
  double m = 0;
  for (long e = blockIdx.x * (long)T3 + threadIdx.x; e < n; e += (long)RB * T3) {
    x[e] -= g * Zk[e];
    const double rr = r[e] - g * Qk[e];
    r[e] = rr;
    const double a = fabs(rr);
    m = (a > m || a != a) ? a : m;
  }
  m = wmax(m);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0;
    for (int w = 0; w < T3 / 64; w++) a = (sm[w] > a || sm[w] != sm[w]) ? sm[w] : a;
    part[blockIdx.x] = a;
  }
}
__global__ void __launch_bounds__(RB) k_maxfin(const double *part, double *out) {
  __shared__ double sm[RB / 64];
  double m = wmax(part[threadIdx.x]);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0;
    for (int w = 0; w < RB / 64; w++) a = (sm[w] > a || sm[w] != sm[w]) ? sm[w] : a;
    *out = a;
  }
}
// max |b| over a vector (block partials)
__global__ void __launch_bounds__(T3) k_absmax_part(const double *v, long n, double *part) {
  __shared__ double sm[T3 / 64];
  double m = 0;
  for (long e = blockIdx.x * (long)T3 + threadIdx.x; e < n; e += (long)RB * T3) {
    const double a = fabs(v[e]);
    m = (a > m || a != a) ? a : m;
  }
  m = wmax(m);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0;
    for (int w = 0; w < T3 / 64; w++) a = (sm[w] > a || sm[w] != sm[w]) ? sm[w] : a;
    part[blockIdx.x] = a;
  }
}

// ---------------------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------------------
static RowTab rowtab(const Ctx3 *ctx, const Lev &V) {
  const double a = ctx->alpha / (V.h * V.h);
  return RowTab{V.cls, V.rowof, V.g_col, V.g_w, a, 1.0 + 6.0 * a, 1.0 / V.h};
}
static gp_status read_ints(Ctx3 *ctx, const int *d, int *h, int n) {
  G3_HIP(hipMemcpyAsync(h, d, n * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  G3_HIP(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}
static gp_status read_double(Ctx3 *ctx, const double *d, double *h) {
  G3_HIP(hipMemcpyAsync(h, d, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  G3_HIP(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}

static gp_status coarse_factor(Ctx3 *ctx) {
  Lev &V = ctx->lev[ctx->L - 1];
  hipStream_t s = ctx->stream;
  const long P = 4 * V.W3;
  int *d_nc = ctx->d_flags + 4;
  k_cmap<<<1, 1, 0, s>>>(P, V.cls, ctx->c_map, d_nc);
  int nc = 0;
  gp_status st = read_ints(ctx, d_nc, &nc, 1);
  if (st) return st;
  if (nc > 4096) return GP_EINVAL;
  ctx->nc = nc;
  double *M = ctx->c_A;                    // augmented n x 2n
  double *A = ctx->c_inv + (size_t)nc * nc;  // the plain matrix after the inverse's slot
  k_fill<<<nb3((long)nc * nc), T3, 0, s>>>(A, (long)nc * nc, 0.0);
  const LevelView LV = V.view(ctx->phi, ctx->N);
  k_cfill<<<nb3(P + 1), T3, 0, s>>>(LV, rowtab(ctx, V), ctx->c_map, nc, V.Mp, A);
  k_augment<<<nb3((long)nc * 2 * nc), T3, 0, s>>>(A, nc, M);
  int *fail = ctx->d_flags + 5;
  G3_HIP(hipMemsetAsync(fail, 0, sizeof(int), s));
  for (int k = 0; k < nc; k++) {
    k_gj_pivot<<<1, GJ_T, 0, s>>>(M, nc, k, fail);
    k_gj_elim<<<nb3((long)nc * 2 * nc), T3, 0, s>>>(M, nc, k);
    k_gj_clear<<<nb3(nc), T3, 0, s>>>(M, nc, k);
  }
  k_take_inv<<<nb3((long)nc * nc), T3, 0, s>>>(M, nc, ctx->c_inv);
  G3_HIP(hipGetLastError());
  int f = 0;
  if ((st = read_ints(ctx, fail, &f, 1))) return st;
  if (f) return GP_EGEOM;
  ctx->c_ok = 1;
  return GP_OK;
}

static gp_status build_level(Ctx3 *ctx, int l) {
  Lev &V = ctx->lev[l];
  hipStream_t s = ctx->stream;
  const LevelView LV = V.view(ctx->phi, ctx->N);
  const long P = 4 * V.W3;
  k_classify<<<nb3(P), T3, 0, s>>>(LV, V.cls);
  k_seed<<<nb3(P), T3, 0, s>>>(LV, V.cls);
  for (int it = 0; it < 64; it++) {
    G3_HIP(hipMemsetAsync(ctx->d_flags, 0, sizeof(int), s));
    k_closure<<<nb3(P), T3, 0, s>>>(LV, V.cls, ctx->d_flags);
    int ch = 0;
    gp_status st = read_ints(ctx, ctx->d_flags, &ch, 1);
    if (st) return st;
    if (!ch) break;
  }
  k_body_off<<<nb3(P), T3, 0, s>>>(P, V.cls);
  const int nbk = (int)((P + NB_T - 1) / NB_T);
  k_row_count<<<nbk, NB_T, 0, s>>>(P, V.cls, ctx->d_bcnt);
  k_scan<<<1, NB_T, 0, s>>>(ctx->d_bcnt, nbk, ctx->d_flags + 1);
  k_row_assign<<<nbk, NB_T, 0, s>>>(P, V.cls, ctx->d_bcnt, V.rowof, V.g_pt, V.gcap);
  int ng = 0;
  gp_status st = read_ints(ctx, ctx->d_flags + 1, &ng, 1);
  if (st) return st;
  if (ng > V.gcap) return GP_ENOMEM;
  V.ng = ng;
  RowArgs A{ng, l, ctx->prm.march_max, ctx->nbis, ctx->prm.dtau_dir, ctx->prm.dtau_neu_over_h * V.h, ctx->prm.cg_min,
            V.g_pt, V.g_col, V.g_w, V.g_dtau, V.g_B, V.g_th};
  G3_HIP(hipMemsetAsync(ctx->d_flags + 2, 0, 2 * sizeof(int), s));
  if (ng) {
    k_rows<<<nb3(ng), T3, 0, s>>>(LV, V.cls, A);
    k_extrap<<<nb3(ng), T3, 0, s>>>(LV, V.cls, A, ctx->d_flags + 3);
  }
  k_cells<<<nb3((long)V.N * V.N * V.N), T3, 0, s>>>(LV, V.cls, ctx->d_flags + 2, ctx->d_flags + 3);
  G3_HIP(hipGetLastError());
  int hf[2];
  if ((st = read_ints(ctx, ctx->d_flags + 2, hf, 2))) return st;
  V.Mp = hf[0];
  if (hf[1] || V.Mp == 0) return GP_EGEOM;
  return GP_OK;
}

static gp_status geometry(Ctx3 *ctx) {
  ctx->have_geom = 0;
  ctx->c_ok = 0;
  for (int l = 0; l < ctx->L; l++) {
    gp_status st = build_level(ctx, l);
    if (st) return st;
  }
  ctx->have_geom = 1;
  if (ctx->alpha > 0) return coarse_factor(ctx);
  return GP_OK;
}

static void relax_step(Ctx3 *ctx, int l) {
  Lev &V = ctx->lev[l];
  hipStream_t s = ctx->stream;
  const LevelView LV = V.view(ctx->phi, ctx->N);
  const RowTab R = rowtab(ctx, V);
  const long cells = (long)(V.N / 7 + 1) * V.N * V.N;
  for (int c = 0; c < 7; c++) k_box<<<nb3(cells), T3, 0, s>>>(LV, R, V.x, V.b, c);
  for (int it = 0; it < ctx->prm.lambda_ghost && V.ng; it++) {
    k_ghost_a<<<nb3(V.ng), T3, 0, s>>>(LV, R, V.g_pt, V.g_dtau, V.ng, V.x, V.b, V.g_tmp);
    k_ghost_b<<<nb3(V.ng), T3, 0, s>>>(V.g_pt, V.ng, V.g_tmp, V.x);
  }
  k_xi_part<<<RB, T3, 0, s>>>(LV, R, V.x, V.b, ctx->d_part);
  k_sum_fin<<<1, RB, 0, s>>>(ctx->d_part, 1.0 / V.Mp, V.x + 4 * V.W3);
}
static void residual(Ctx3 *ctx, int l, const double *x, const double *b, double *r, double *out, bool store) {
  Lev &V = ctx->lev[l];
  const LevelView LV = V.view(ctx->phi, ctx->N);
  k_resid<<<RB, T3, 0, ctx->stream>>>(LV, rowtab(ctx, V), x, b, r, ctx->d_part, store ? 1 : 0);
  // the mean row's right-hand side is zero on every level (only the finest one carries data, set to zero)
  k_resid_fin<<<1, RB, 0, ctx->stream>>>(ctx->d_part, 0.0, V.Mp, r, 4 * V.W3, out, store ? 1 : 0);
}
static void coarse_solve(Ctx3 *ctx) {
  Lev &V = ctx->lev[ctx->L - 1];
  hipStream_t s = ctx->stream;
  const long P = 4 * V.W3;
  double *bd = ctx->c_b, *xd = ctx->c_x;
  k_cgather<<<nb3(P + 1), T3, 0, s>>>(P, ctx->c_map, V.b, bd);
  k_capply<<<ctx->nc, 64, 0, s>>>(ctx->c_inv, ctx->c_map, ctx->nc, P, bd, xd, nullptr);
  k_cscatter<<<nb3(P + 1), T3, 0, s>>>(P, ctx->c_map, xd, V.x);
}
static void cycle(Ctx3 *ctx, int l) {
  if (l == ctx->L - 1) {
    coarse_solve(ctx);
    return;
  }
  Lev &F = ctx->lev[l], &C = ctx->lev[l + 1];
  hipStream_t s = ctx->stream;
  for (int q = 0; q < ctx->prm.nu1; q++) relax_step(ctx, l);
  residual(ctx, l, F.x, F.b, F.r, ctx->d_scal + 2, true);
  const LevelView FV = F.view(ctx->phi, ctx->N), CV = C.view(ctx->phi, ctx->N);
  k_restrict<<<nb3(C.n), T3, 0, s>>>(FV, F.cls, F.r, CV, C.cls, C.b);
  k_fill<<<nb3(C.n), T3, 0, s>>>(C.x, C.n, 0.0);
  const int reps = (l + 1 == ctx->L - 1) ? 1 : ctx->prm.gamma;
  for (int q = 0; q < reps; q++) cycle(ctx, l + 1);
  k_prolong<<<nb3(F.n), T3, 0, s>>>(CV, C.cls, C.x, FV, F.cls, F.x);
  for (int q = 0; q < ctx->prm.nu2; q++) relax_step(ctx, l);
}
static void mean_project(Ctx3 *ctx, double *x, const double *extra) {
  Lev &V = ctx->lev[0];
  const LevelView LV = V.view(ctx->phi, ctx->N);
  k_pmean_part<<<RB, T3, 0, ctx->stream>>>(LV, V.cls, x, ctx->d_part);
  k_sum_fin<<<1, RB, 0, ctx->stream>>>(ctx->d_part, 1.0 / V.Mp, ctx->d_scal + 4);
  k_pshift<<<nb3(V.W3), T3, 0, ctx->stream>>>(LV, V.cls, x, ctx->d_scal + 4, extra);
}
static gp_status resnorm(Ctx3 *ctx, double *out) {
  Lev &V = ctx->lev[0];
  residual(ctx, 0, V.x, V.b, V.r, ctx->d_scal + 1, true);
  G3_HIP(hipGetLastError());
  return read_double(ctx, ctx->d_scal + 1, out);
}
static gp_status bnorm(Ctx3 *ctx, double *out) {
  Lev &V = ctx->lev[0];
  k_absmax_part<<<RB, T3, 0, ctx->stream>>>(V.b, V.n, ctx->d_part);
  k_maxfin<<<1, RB, 0, ctx->stream>>>(ctx->d_part, ctx->d_scal + 3);
  G3_HIP(hipGetLastError());
  return read_double(ctx, ctx->d_scal + 3, out);
}

static gp_status gcr_alloc(Ctx3 *ctx) {
  const int m = std::max(1, std::min(KMAX, ctx->prm.krylov));
  if (ctx->kr_r && ctx->kr_m == m) return GP_OK;
  for (double **p : {&ctx->kr_r, &ctx->kr_z, &ctx->kr_q, &ctx->kr_Q, &ctx->kr_Z, &ctx->kr_zero, &ctx->kr_s}) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  const size_t n = ctx->lev[0].n;
  G3_HIP(hipMalloc((void **)&ctx->kr_r, n * sizeof(double)));
  G3_HIP(hipMalloc((void **)&ctx->kr_z, n * sizeof(double)));
  G3_HIP(hipMalloc((void **)&ctx->kr_q, n * sizeof(double)));
  G3_HIP(hipMalloc((void **)&ctx->kr_Q, (size_t)m * n * sizeof(double)));
  G3_HIP(hipMalloc((void **)&ctx->kr_Z, (size_t)m * n * sizeof(double)));
  G3_HIP(hipMalloc((void **)&ctx->kr_zero, n * sizeof(double)));
  G3_HIP(hipMalloc((void **)&ctx->kr_s, (2 * KMAX + 8) * sizeof(double)));
  k_fill<<<nb3((long)n), T3, 0, ctx->stream>>>(ctx->kr_zero, (long)n, 0.0);
  G3_HIP(hipGetLastError());
  ctx->kr_m = m;
  return GP_OK;
}

// z = B' r: one cycle from zero on M e = r, the mean projection and the mean-row column (a constant pressure),
// zero where no equation
static void precond(Ctx3 *ctx, const double *r, double *z) {
  Lev &V = ctx->lev[0];
  hipStream_t s = ctx->stream;
  double *X0 = V.x, *B0 = V.b;
  V.x = z;
  V.b = const_cast<double *>(r);
  k_fill<<<nb3(V.n), T3, 0, s>>>(z, V.n, 0.0);
  k_set_walld<<<nb3(4 * V.W3), T3, 0, s>>>(4 * V.W3, V.cls, z, r);
  cycle(ctx, 0);
  mean_project(ctx, z, r + 4 * V.W3);
  k_mask<<<nb3(4 * V.W3), T3, 0, s>>>(4 * V.W3, V.cls, z);
  V.x = X0;
  V.b = B0;
}

gp_status solve(Ctx3 *ctx, double tol, int max_cycles, gp_stats *stt) {
  auto t0 = std::chrono::steady_clock::now();
  Lev &V = ctx->lev[0];
  hipStream_t s = ctx->stream;
  const long n = V.n;
  k_set_walld<<<nb3(4 * V.W3), T3, 0, s>>>(4 * V.W3, V.cls, V.x, V.b);
  double r0, bn;
  gp_status st = resnorm(ctx, &r0);
  if (st) return st;
  if (!(r0 == r0)) return GP_EDIVERGED;
  if ((st = bnorm(ctx, &bn))) return st;
  const double thr = tol * (bn > 1 ? bn : 1), lim = 1e6 * (r0 > 1 ? r0 : 1);
  double rn = r0, rp = r0, rho = 0;
  int c = 0;
  gp_status out = GP_OK;
  if (ctx->prm.krylov <= 0) {
    while (rn > thr && c < max_cycles) {
      cycle(ctx, 0);
      mean_project(ctx, V.x, nullptr);
      rp = rn;
      if ((st = resnorm(ctx, &rn))) return st;
      rho = rn / rp;
      c++;
      if (!(rn == rn) || rn > lim) {
        out = GP_EDIVERGED;
        break;
      }
    }
  } else {
    if ((st = gcr_alloc(ctx))) return st;
    const int m = ctx->kr_m;
    G3_HIP(hipMemcpyAsync(ctx->kr_r, V.r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    double *beta = ctx->kr_s, *sc = ctx->kr_s + KMAX, *nq = ctx->kr_s + KMAX + 4;
    int k = 0;
    while (rn > thr && c < max_cycles) {
      double *Qk = ctx->kr_Q + (size_t)k * n, *Zk = ctx->kr_Z + (size_t)k * n;
      precond(ctx, ctx->kr_r, ctx->kr_z);
      // q = -M z: the residual of z with a zero right-hand side
      residual(ctx, 0, ctx->kr_z, ctx->kr_zero, ctx->kr_q, ctx->d_scal + 5, true);
      if (k) {
        k_dots<<<RB, T3, 0, s>>>(ctx->kr_Q, n, k, ctx->kr_q, ctx->d_part);
        k_sums<<<1, RB, 0, s>>>(ctx->d_part, k, nq, beta);
      }
      k_orth<<<RB, T3, 0, s>>>(ctx->kr_Q, ctx->kr_Z, n, k, beta, ctx->kr_q, ctx->kr_z, ctx->kr_r, Qk, Zk, ctx->d_part);
      k_sums<<<1, RB, 0, s>>>(ctx->d_part, 2, nullptr, sc);
      k_sums<<<1, RB, 0, s>>>(ctx->d_part, 1, nullptr, nq + k);  // |Q_k|^2, kept for the later coefficients
      k_step<<<RB, T3, 0, s>>>(n, sc, Qk, Zk, V.x, ctx->kr_r, ctx->d_part);
      k_maxfin<<<1, RB, 0, s>>>(ctx->d_part, ctx->d_scal + 1);
      G3_HIP(hipGetLastError());
      if ((st = read_double(ctx, ctx->d_scal + 1, &rn))) return st;
      c++;
      k++;
      if (!(rn == rn) || rn > lim) {
        out = GP_EDIVERGED;
        break;
      }
      if (rn <= thr || k == m) {
        if ((st = resnorm(ctx, &rn))) return st;
        G3_HIP(hipMemcpyAsync(ctx->kr_r, V.r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        k = 0;
      }
      rho = rn / rp;
      rp = rn;
    }
  }
  if (out == GP_OK && rn > thr) out = GP_ENOCONV;
  if (stt) {
    stt->cycles = c;
    stt->outer = 0;
    stt->res0 = r0;
    stt->res = rn;
    stt->rho = rho;
    stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stt->bytes_alg = 0;
  }
  return out;
}

}  // namespace d3
}  // namespace gpmg

using namespace gpmg::d3;

extern "C" {

void gp3_default_params(gp3_params *p) {
  if (!p) return;
  p->nu1 = 2;
  p->nu2 = 2;
  p->gamma = 1;
  p->lambda_ghost = 2;
  p->coarsest_n = 4;
  p->march_max = 8;
  p->krylov = 8;
  p->dtau_dir = 0.9;
  p->dtau_neu_over_h = 0.6;
  p->bisect_eps_over_h = 0.01;
  p->cg_min = 0.1;
}

void gp3_destroy(gp3_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  auto fr = [](void *p) {
    if (p) (void)hipFree(p);
  };
  for (int l = 0; l < ctx->L; l++) {
    Lev &V = ctx->lev[l];
    for (void *p : {(void *)V.cls, (void *)V.x, (void *)V.b, (void *)V.r, (void *)V.rowof, (void *)V.g_pt,
                    (void *)V.g_col, (void *)V.g_w, (void *)V.g_dtau, (void *)V.g_B, (void *)V.g_th, (void *)V.g_tmp})
      fr(p);
  }
  for (void *p : {(void *)ctx->phi, (void *)ctx->d_flags, (void *)ctx->d_part, (void *)ctx->d_scal,
                  (void *)ctx->d_bcnt, (void *)ctx->c_map, (void *)ctx->c_A, (void *)ctx->c_inv, (void *)ctx->c_b,
                  (void *)ctx->c_x, (void *)ctx->kr_r,
                  (void *)ctx->kr_z, (void *)ctx->kr_q, (void *)ctx->kr_Q, (void *)ctx->kr_Z, (void *)ctx->kr_zero,
                  (void *)ctx->kr_s})
    fr(p);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

gp_status gp3_setup_grid(gp3_ctx **out, int N, const gp3_params *prm, void *hip_stream) {
  if (!out) return GP_EINVAL;
  *out = nullptr;
  gp3_params P;
  if (prm)
    P = *prm;
  else
    gp3_default_params(&P);
  if (N < 8 || (N & (N - 1)) || P.coarsest_n < 2 || P.coarsest_n > N / 2 || (P.coarsest_n & (P.coarsest_n - 1)) ||
      P.nu1 < 0 || P.nu2 < 0 || P.gamma < 1 || P.lambda_ghost < 0 || P.krylov < 0 || P.krylov > KMAX ||
      !(P.dtau_neu_over_h > 0) || !(P.bisect_eps_over_h > 0))
    return GP_EINVAL;
  gp3_ctx *ctx = new gp3_ctx();
  ctx->N = N;
  ctx->prm = P;
  ctx->nbis = (int)std::ceil(std::log2(0.5 / P.bisect_eps_over_h) - 1e-12);
  ctx->stream = (hipStream_t)hip_stream;
  gp_status st = GP_OK;
  auto fail = [&](gp_status s) {
    gp3_destroy(ctx);
    return s;
  };
  if (!ctx->stream) {
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamDefault) != hipSuccess) return fail(GP_EHIP);
    ctx->own_stream = true;
  }
  int L = 0;
  for (int n = N; n >= P.coarsest_n; n /= 2) L++;
  ctx->L = L;
  const size_t nl = 2 * (size_t)N + 1;
  auto al = [&](void **p, size_t bytes) -> bool { return hipMalloc(p, bytes ? bytes : 1) == hipSuccess; };
  if (!al((void **)&ctx->phi, nl * nl * nl * sizeof(double))) return fail(GP_ENOMEM);
  size_t maxbcnt = 0;
  for (int l = 0; l < L; l++) {
    Lev &V = ctx->lev[l];
    V.N = N >> l;
    V.W = V.N + 2;
    V.W3 = (long)V.W * V.W * V.W;
    V.n = 4 * V.W3 + 1;
    V.h = 2.0 / V.N;
    V.lstride = 1 << l;
    // ghost rows: the points within a few cells of the body and the walls' rings, bounded by the grid
    V.gcap = (int)std::min<long>(4 * V.W3, 64L * V.W * V.W + 4096);
    if (!al((void **)&V.cls, 4 * V.W3) || !al((void **)&V.x, V.n * sizeof(double)) ||
        !al((void **)&V.b, V.n * sizeof(double)) || !al((void **)&V.r, V.n * sizeof(double)) ||
        !al((void **)&V.rowof, 4 * V.W3 * sizeof(int)) || !al((void **)&V.g_pt, V.gcap * sizeof(int)) ||
        !al((void **)&V.g_col, 27L * V.gcap * sizeof(int)) || !al((void **)&V.g_w, 27L * V.gcap * sizeof(double)) ||
        !al((void **)&V.g_dtau, V.gcap * sizeof(double)) || !al((void **)&V.g_B, 3L * V.gcap * sizeof(double)) ||
        !al((void **)&V.g_th, 3L * V.gcap * sizeof(double)) || !al((void **)&V.g_tmp, V.gcap * sizeof(double)))
      return fail(GP_ENOMEM);
    (void)hipMemsetAsync(V.x, 0, V.n * sizeof(double), ctx->stream);
    (void)hipMemsetAsync(V.b, 0, V.n * sizeof(double), ctx->stream);
    maxbcnt = std::max(maxbcnt, (size_t)((4 * V.W3 + NB_T - 1) / NB_T));
  }
  const Lev &Cl = ctx->lev[L - 1];
  const size_t cmax = 4 * Cl.W3 + 1;  // dense size bound
  if (!al((void **)&ctx->d_flags, 16 * sizeof(int)) || !al((void **)&ctx->d_part, (KMAX + 2) * RB * sizeof(double)) ||
      !al((void **)&ctx->d_scal, 16 * sizeof(double)) || !al((void **)&ctx->d_bcnt, maxbcnt * sizeof(int)) ||
      !al((void **)&ctx->c_map, (cmax + 1) * sizeof(int)) || !al((void **)&ctx->c_A, 2 * cmax * cmax * sizeof(double)) ||
      !al((void **)&ctx->c_inv, 2 * cmax * cmax * sizeof(double)) || !al((void **)&ctx->c_b, cmax * sizeof(double)) ||
      !al((void **)&ctx->c_x, cmax * sizeof(double)))
    return fail(GP_ENOMEM);
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(GP_EHIP);
  (void)st;
  *out = ctx;
  return GP_OK;
}

int gp3_num_levels(const gp3_ctx *ctx) { return ctx ? ctx->L : 0; }
const char *gp3_last_hip_error(const gp3_ctx *ctx) { return ctx ? ctx->hip_err.c_str() : ""; }

gp_status gp3_set_levelset(gp3_ctx *ctx, const double *phi, int on_device) {
  if (!ctx || !phi) return GP_EINVAL;
  const size_t nl = 2 * (size_t)ctx->N + 1;
  G3_HIP(hipMemcpyAsync(ctx->phi, phi, nl * nl * nl * sizeof(double),
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->stream));
  return geometry(ctx);
}
gp_status gp3_set_levelset_analytic(gp3_ctx *ctx, int kind, const double *p) {
  if (!ctx || !p || (kind != 0 && kind != 1)) return GP_EINVAL;
  const long nl = 2L * ctx->N + 1;
  k_sample<<<nb3(nl * nl * nl), T3, 0, ctx->stream>>>(kind, p[0], p[1], p[2], p[3], p[4], p[5], ctx->N, ctx->phi);
  G3_HIP(hipGetLastError());
  return geometry(ctx);
}
gp_status gp3_set_alpha(gp3_ctx *ctx, double alpha) {
  if (!ctx || !(alpha >= 0)) return GP_EINVAL;
  ctx->alpha = alpha;
  ctx->c_ok = 0;
  if (ctx->have_geom && alpha > 0) return coarse_factor(ctx);
  return GP_OK;
}

static gp_status stage_grids(gp3_ctx *ctx, const double *const src[4], int on_device, double *dst_tmp) {
  const Lev &V = ctx->lev[0];
  for (int g = 0; g < 4; g++) {
    if (!src[g]) {
      k_fill<<<nb3(V.W3), T3, 0, ctx->stream>>>(dst_tmp + g * V.W3, V.W3, 0.0);
      continue;
    }
    G3_HIP(hipMemcpyAsync(dst_tmp + g * V.W3, src[g], V.W3 * sizeof(double),
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->stream));
  }
  return GP_OK;
}
__global__ void k_take_rhs(long P, const uint8_t *cls, const double *src, double *b, int which) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p > P) return;
  if (p == P) {
    if (which == 0) b[P] = 0.0;
    return;
  }
  const int c = cls[p];
  if (which == 0 && c == C_INT) b[p] = src[p];
  if (which == 1) {
    if (c == C_GHOST || c == C_WALLG || c == C_WALLD) b[p] = src[p];
    if (c == C_GHOSTX) b[p] = 0.0;
  }
}
gp_status gp3_set_rhs(gp3_ctx *ctx, const double *fu, const double *fv, const double *fw, const double *g, int on_device) {
  if (!ctx || !ctx->have_geom) return GP_EINVAL;
  Lev &V = ctx->lev[0];
  const double *src[4] = {fu, fv, fw, g};
  gp_status st = stage_grids(ctx, src, on_device, V.r);
  if (st) return st;
  k_take_rhs<<<nb3(4 * V.W3 + 1), T3, 0, ctx->stream>>>(4 * V.W3, V.cls, V.r, V.b, 0);
  G3_HIP(hipGetLastError());
  return GP_OK;
}
gp_status gp3_set_boundary_values(gp3_ctx *ctx, const double *bu, const double *bv, const double *bw, const double *bp,
                                  int on_device) {
  if (!ctx || !ctx->have_geom) return GP_EINVAL;
  Lev &V = ctx->lev[0];
  const double *src[4] = {bu, bv, bw, bp};
  gp_status st = stage_grids(ctx, src, on_device, V.r);
  if (st) return st;
  k_take_rhs<<<nb3(4 * V.W3 + 1), T3, 0, ctx->stream>>>(4 * V.W3, V.cls, V.r, V.b, 1);
  G3_HIP(hipGetLastError());
  return GP_OK;
}
gp_status gp3_set_x(gp3_ctx *ctx, const double *x, int on_device) {
  if (!ctx || !x) return GP_EINVAL;
  Lev &V = ctx->lev[0];
  G3_HIP(hipMemcpyAsync(V.x, x, V.n * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        ctx->stream));
  return GP_OK;
}
gp_status gp3_get_x(gp3_ctx *ctx, double *x, int on_device) {
  if (!ctx || !x) return GP_EINVAL;
  Lev &V = ctx->lev[0];
  G3_HIP(hipMemcpyAsync(x, V.x, V.n * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        ctx->stream));
  G3_HIP(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}
gp_status gp3_get_classes(gp3_ctx *ctx, int level, unsigned char *cls) {
  if (!ctx || !cls || level < 0 || level >= ctx->L || !ctx->have_geom) return GP_EINVAL;
  Lev &V = ctx->lev[level];
  G3_HIP(hipMemcpyAsync(cls, V.cls, 4 * V.W3, hipMemcpyDeviceToHost, ctx->stream));
  G3_HIP(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}
gp_status gp3_get_ghost_rows(gp3_ctx *ctx, int level, double *B, double *th, double *w27, int *c27, double *dtau) {
  if (!ctx || level < 0 || level >= ctx->L || !ctx->have_geom) return GP_EINVAL;
  Lev &V = ctx->lev[level];
  const long P = 4 * V.W3;
  std::vector<int> rowof(P), pt(V.ng), col(27L * V.ng);
  std::vector<double> gB(3L * V.ng), gth(3L * V.ng), gw(27L * V.ng), gdt(V.ng);
  hipStream_t s = ctx->stream;
  G3_HIP(hipMemcpyAsync(rowof.data(), V.rowof, P * sizeof(int), hipMemcpyDeviceToHost, s));
  if (V.ng) {
    G3_HIP(hipMemcpyAsync(col.data(), V.g_col, col.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    G3_HIP(hipMemcpyAsync(gw.data(), V.g_w, gw.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    G3_HIP(hipMemcpyAsync(gB.data(), V.g_B, gB.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    G3_HIP(hipMemcpyAsync(gth.data(), V.g_th, gth.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    G3_HIP(hipMemcpyAsync(gdt.data(), V.g_dtau, gdt.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  G3_HIP(hipStreamSynchronize(s));
  for (long p = 0; p < P; p++) {
    const int r = rowof[p];
    for (int d = 0; d < 3; d++) {
      if (B) B[3 * p + d] = r >= 0 ? gB[3L * r + d] : NAN;
      if (th) th[3 * p + d] = r >= 0 ? gth[3L * r + d] : NAN;
    }
    for (int q = 0; q < 27; q++) {
      if (w27) w27[27 * p + q] = r >= 0 ? gw[27L * r + q] : NAN;
      if (c27) c27[27 * p + q] = r >= 0 ? col[27L * r + q] : -1;
    }
    if (dtau) dtau[p] = r >= 0 ? gdt[r] : NAN;
  }
  return GP_OK;
}
gp_status gp3_relax(gp3_ctx *ctx, int steps) {
  if (!ctx || !ctx->have_geom || steps < 0) return GP_EINVAL;
  for (int q = 0; q < steps; q++) relax_step(ctx, 0);
  G3_HIP(hipGetLastError());
  G3_HIP(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}
gp_status gp3_cycle(gp3_ctx *ctx, double *res_inf) {
  if (!ctx || !ctx->have_geom) return GP_EINVAL;
  if (!ctx->c_ok) {
    if (!(ctx->alpha > 0)) return GP_EINVAL;
    gp_status st = coarse_factor(ctx);
    if (st) return st;
  }
  Lev &V = ctx->lev[0];
  k_set_walld<<<nb3(4 * V.W3), T3, 0, ctx->stream>>>(4 * V.W3, V.cls, V.x, V.b);
  cycle(ctx, 0);
  mean_project(ctx, V.x, nullptr);
  G3_HIP(hipGetLastError());
  double r = 0;
  gp_status st = resnorm(ctx, &r);
  if (st) return st;
  if (res_inf) *res_inf = r;
  return GP_OK;
}
gp_status gp3_solve(gp3_ctx *ctx, double tol, int max_cycles, gp_stats *st) {
  if (!ctx || !ctx->have_geom || !(tol > 0) || max_cycles < 0) return GP_EINVAL;
  if (!ctx->c_ok) {
    if (!(ctx->alpha > 0)) return GP_EINVAL;
    gp_status s = coarse_factor(ctx);
    if (s) return s;
  }
  return solve(ctx, tol, max_cycles, st);
}
gp_status gp3_residual(gp3_ctx *ctx, double *r, double *res_inf) {
  if (!ctx || !ctx->have_geom) return GP_EINVAL;
  Lev &V = ctx->lev[0];
  double ri = 0;
  gp_status st = resnorm(ctx, &ri);
  if (st) return st;
  if (res_inf) *res_inf = ri;
  if (r) {
    G3_HIP(hipMemcpyAsync(r, V.r, V.n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    G3_HIP(hipStreamSynchronize(ctx->stream));
  }
  return GP_OK;
}

}  // extern "C"
