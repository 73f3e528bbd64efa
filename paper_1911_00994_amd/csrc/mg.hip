// Multigrid of Sect. 4 on the device: 5-colour box relaxation, fictitious-time ghost sweeps, the scalar
// unknown xi, residual, boundary-aware restriction, extension fill, bilinear prolongation, exact coarsest solve
// and the cycle driver.  Vectors are templated on the storage type T (double for the FP64 solver, float for the
// inner cycles of the mixed-precision solver); all arithmetic inside a kernel is FP64 and ghost-row
// coefficients are always FP64.
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>

#include <hip/hip_ext.h>

#include "internal.h"

namespace gpmg {

__device__ __forceinline__ int pidx(int W, int i, int j) { return (j + 1) * W + (i + 1); }

// ---------------------------------------------------------------------------------------------------------
// box relaxation of all cells of one colour (i + 2j) mod 5 (Sect. 4.1.1; the colour order replaces the
// lexicographic order, same-colour boxes share no unknown and read nothing another one writes).
// Box unknowns: p_ij and the four faces, those that are internal points; everything else is held fixed.
// With the faces W/E coupled through -a and S/N likewise, each free face is affine in p:
//   both free:  [d -a; -a d] [uW; uE] = [RW - p/h; RE + p/h]
//   one free:   d uW = RW + a uE - p/h   (resp. d uE = RE + a uW + p/h)
// and the continuity row fixes p.
// ---------------------------------------------------------------------------------------------------------

// new values of a box from its 21 neighbouring values and 5 right-hand sides; skip = the box is left unchanged
struct BoxNew {
  double p, uW, uE, vS, vN;
  bool skip;
};
__device__ __forceinline__ BoxNew box_core(const BoxK &K, bool fW, bool fE, bool fS, bool fN, bool fP, double uW, double uE,
                                           double uWW, double uEE, double uWS, double uWN, double uES, double uEN, double vS,
                                           double vN, double vSS, double vNN, double vSW, double vSE, double vNW, double vNE,
                                           double pc, double pW, double pE, double pS, double pN, double bW_, double bE_,
                                           double bS_, double bN_, double bP_, double xi) {
  // the pressure's denominator is Du + Dv, each 0, ihd or 2 bp by the free faces of the pair; it is divided
  // here (a table indexed by lane-varying values would be a memory load on the critical path)
  BoxNew o;
  o.skip = false;
  const double a = K.a, ih = K.ih;
  double aW = uW, bW = 0, aE = uE, bE = 0, aS = vS, bS = 0, aN = vN, bN = 0, Du = 0, Dv = 0;
  {
    const double RW = bW_ + a * (uWW + uWS + uWN) + pW * ih;
    const double RE = bE_ + a * (uEE + uES + uEN) - pE * ih;
    if (fW && fE) {
      aW = K.q1 * RW + K.q2 * RE;
      bW = -K.bp;
      aE = K.q2 * RW + K.q1 * RE;
      bE = K.bp;
      Du = 2.0 * K.bp;
    } else if (fW) {
      aW = (RW + a * uE) * K.id;
      bW = -K.ihd;
      Du = K.ihd;
    } else if (fE) {
      aE = (RE + a * uW) * K.id;
      bE = K.ihd;
      Du = K.ihd;
    }
  }
  {
    const double RS = bS_ + a * (vSS + vSW + vSE) + pS * ih;
    const double RN = bN_ + a * (vNN + vNW + vNE) - pN * ih;
    if (fS && fN) {
      aS = K.q1 * RS + K.q2 * RN;
      bS = -K.bp;
      aN = K.q2 * RS + K.q1 * RN;
      bN = K.bp;
      Dv = 2.0 * K.bp;
    } else if (fS) {
      aS = (RS + a * vN) * K.id;
      bS = -K.ihd;
      Dv = K.ihd;
    } else if (fN) {
      aN = (RN + a * vS) * K.id;
      bN = K.ihd;
      Dv = K.ihd;
    }
  }
  double pn = pc;
  if (fP) {
    const double den = Du + Dv;
    if (den == 0.0) {  // no free face: the block is singular, the box is skipped
      o.skip = true;
      return o;
    }
    pn = (K.h * (xi + bP_) - (aE - aW + aN - aS)) * (1.0 / den);
  }
  o.p = pn;
  o.uW = aW + bW * pn;
  o.uE = aE + bE * pn;
  o.vS = aS + bS * pn;
  o.vN = aN + bN * pn;
  return o;
}

template <typename T>
__device__ __forceinline__ void box_update(int W, const BoxK &K, const uint8_t *__restrict__ cls, T *__restrict__ x,
                                           const T *__restrict__ b, int i, int j) {
  const int WW = W * W;
  T *u = x, *v = x + WW, *p = x + 2 * WW;
  const T *bu = b, *bv = b + WW, *bp = b + 2 * WW;
  const int c = (j + 1) * W + (i + 1);
  // every load is issued up front (all indices stay inside the padded arrays for 0 <= i, j < N); the
  // classes then decide which values enter the box
  const uint8_t kW = cls[c], kE = cls[c + 1], kS = cls[WW + c], kN = cls[WW + c + W], kP = cls[2 * WW + c];
  const double uW = u[c], uE = u[c + 1], vS = v[c], vN = v[c + W], pc = p[c];
  const double uWW = u[c - 1], uEE = u[c + 2], uWS = u[c - W], uWN = u[c + W], uES = u[c + 1 - W], uEN = u[c + 1 + W];
  const double vSS = v[c - W], vNN = v[c + 2 * W], vSW = v[c - 1], vSE = v[c + 1], vNW = v[c + W - 1], vNE = v[c + W + 1];
  const double pW = p[c - 1], pE = p[c + 1], pS = p[c - W], pN = p[c + W];
  const double bW_ = bu[c], bE_ = bu[c + 1], bS_ = bv[c], bN_ = bv[c + W], bP_ = bp[c];
  const double xi = (double)x[3 * WW];
  const bool fW = kW == K_INT, fE = kE == K_INT, fS = kS == K_INT, fN = kN == K_INT, fP = kP == K_INT;
  if (!(fW || fE || fS || fN || fP)) return;
  const BoxNew o = box_core(K, fW, fE, fS, fN, fP, uW, uE, uWW, uEE, uWS, uWN, uES, uEN, vS, vN, vSS, vNN, vSW, vSE, vNW,
                            vNE, pc, pW, pE, pS, pN, bW_, bE_, bS_, bN_, bP_, xi);
  if (o.skip) return;
  if (fP) p[c] = (T)o.p;
  if (fW) u[c] = (T)o.uW;
  if (fE) u[c + 1] = (T)o.uE;
  if (fS) v[c] = (T)o.vS;
  if (fN) v[c + W] = (T)o.vN;
}

// the same update with the five right-hand sides of the box passed in (W E S N P)
template <typename T>
__device__ __forceinline__ void box_update_rb(int W, const BoxK &K, const uint8_t *__restrict__ cls, T *__restrict__ x,
                                              const double (&bb)[5], int i, int j) {
  const int WW = W * W;
  T *u = x, *v = x + WW, *p = x + 2 * WW;
  const int c = (j + 1) * W + (i + 1);
  const uint8_t kW = cls[c], kE = cls[c + 1], kS = cls[WW + c], kN = cls[WW + c + W], kP = cls[2 * WW + c];
  const double uW = u[c], uE = u[c + 1], vS = v[c], vN = v[c + W], pc = p[c];
  const double uWW = u[c - 1], uEE = u[c + 2], uWS = u[c - W], uWN = u[c + W], uES = u[c + 1 - W], uEN = u[c + 1 + W];
  const double vSS = v[c - W], vNN = v[c + 2 * W], vSW = v[c - 1], vSE = v[c + 1], vNW = v[c + W - 1], vNE = v[c + W + 1];
  const double pW = p[c - 1], pE = p[c + 1], pS = p[c - W], pN = p[c + W];
  const double xi = (double)x[3 * WW];
  const bool fW = kW == K_INT, fE = kE == K_INT, fS = kS == K_INT, fN = kN == K_INT, fP = kP == K_INT;
  if (!(fW || fE || fS || fN || fP)) return;
  const BoxNew o = box_core(K, fW, fE, fS, fN, fP, uW, uE, uWW, uEE, uWS, uWN, uES, uEN, vS, vN, vSS, vNN, vSW, vSE, vNW,
                            vNE, pc, pW, pE, pS, pN, bb[0], bb[1], bb[2], bb[3], bb[4], xi);
  if (o.skip) return;
  if (fP) p[c] = (T)o.p;
  if (fW) u[c] = (T)o.uW;
  if (fE) u[c + 1] = (T)o.uE;
  if (fS) v[c] = (T)o.vS;
  if (fN) v[c + W] = (T)o.vN;
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_box(int N, int W, BoxK BK, const uint8_t *__restrict__ cls,
                                             T *__restrict__ x, const T *__restrict__ b, int colour) {
  const int K = N / 5 + 1;
  // workgroups are dealt to the 8 XCDs round robin: remap so that each XCD works on one contiguous band of
  // rows and its L2 sees the row halos of its own band
  const int nb = gridDim.x, per = (nb + 7) / 8;
  const int lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  int t = lb * blockDim.x + threadIdx.x;
  int j = t / K, kk = t - j * K;
  if (j >= N) return;
  int i = ((colour - 2 * j) % 5 + 5) % 5 + 5 * kk;
  if (i >= N) return;
  box_update<T>(W, BK, cls, x, b, i, j);
}

// ---------------------------------------------------------------------------------------------------------
// all five colours of a box sweep in one launch (temporal blocking).  A workgroup owns a BT x BT tile of cells
// and stages x and the classes of the points of the tile widened by BH = 10 cells in LDS.  Pass k (colour k)
// updates the boxes of colour k within 1 + 2 (4 - k) cells of the tile: a box depends only on boxes within 2
// cells written in earlier passes, so every box computed in pass k sees exactly the values the colour-by-colour
// sweep gives it, and the boxes that write the tile's own points (u, v, p of its cells: the west and south faces
// and the centre) are all computed in every pass.  A pass has at most 500 boxes, one per thread, so each thread
// loads the right-hand sides of its five boxes into registers while the tile is staged (b needs no LDS, and two
// workgroups fit on a compute unit).  The sweep reads x and writes a second buffer y: every point is owned by
// one tile (the border rows and columns -1 and N by the tiles next to them), so y receives every point once,
// and no workgroup can see another one's new values while staging its halo.  The caller swaps x and y.
// Tiles are dealt to the 8 XCDs in contiguous runs (when their number is a multiple of 8), so the halos that
// neighbouring tiles share are fetched into the same L2.
// ---------------------------------------------------------------------------------------------------------
// BT = 32 on the large levels (53 x 53 staged points), 16 where 32-cell tiles would leave most compute units idle
constexpr int BH = 10;
constexpr int B5_T = 512;
template <int BT>
constexpr int box5_rw() { return BT + 2 * BH + 1; }
static_assert((32 + 2 * (1 + 2 * 4) + 4) / 5 * (32 + 2 * (1 + 2 * 4)) <= B5_T, "one box per thread and pass");
template <typename T, int BT>
__host__ __device__ constexpr size_t box5_lds() {
  return ((3 * box5_rw<BT>() * box5_rw<BT>() + 1) * sizeof(T) + 15) / 16 * 16 + 3 * box5_rw<BT>() * box5_rw<BT>();
}
static inline int box5_tile(int N) { return (N / 16) * (N / 16) <= 512 ? 16 : 32; }
template <typename T, int BT>
__global__ void __launch_bounds__(B5_T, 2) k_box5(int N, int W, BoxK K, const uint8_t *__restrict__ cls,
                                                  const T *__restrict__ x, const T *__restrict__ b, T *__restrict__ y,
                                                  const unsigned long long *__restrict__ go, double go_lo,
                                                  double go_hi) {
  if (go) {  // queued before the host's convergence test: run only if go_lo < norm <= go_hi (norm as bits)
    const double r = __longlong_as_double((long long)*go);
    if (!(r > go_lo && r <= go_hi)) return;
  }
  constexpr int BRW = box5_rw<BT>(), BRWW = BRW * BRW;
  extern __shared__ unsigned char lds_raw[];
  T *xs = reinterpret_cast<T *>(lds_raw);
  uint8_t *cs = lds_raw + ((3 * BRWW + 1) * sizeof(T) + 15) / 16 * 16;
  const int WW = W * W, nt = (N + BT - 1) / BT, ntt = nt * nt;
  const int tile = (ntt & 7) ? blockIdx.x : (blockIdx.x & 7) * (ntt >> 3) + (blockIdx.x >> 3);
  const int i0 = (tile % nt) * BT, j0 = (tile / nt) * BT;
  const int gi0 = i0 - BH, gj0 = j0 - BH;  // point (gi0, gj0) sits at LDS point (0, 0)
  // this thread's box in each pass (cell i, j; i = -1 for none) and its right-hand sides
  int bi[5], bj[5];
  double bb[5][5];
#pragma unroll
  for (int k = 0; k < 5; k++) {
    const int ex = 1 + 2 * (4 - k);
    const int ilo = max(0, i0 - ex), ihi = min(N, i0 + BT + ex), jlo = max(0, j0 - ex), jhi = min(N, j0 + BT + ex);
    const int per = (ihi - ilo + 4) / 5;  // colour-k cells per row, at most
    const int t = threadIdx.x, r = t / max(per, 1), m = t - r * per, j = jlo + r;
    const int i = ilo + ((k - (ilo + 2 * j)) % 5 + 5) % 5 + 5 * m;
    const bool on = per > 0 && j < jhi && i < ihi;
    bi[k] = on ? i : -1;
    bj[k] = j;
    const int c = on ? (j + 1) * W + (i + 1) : 0;
    bb[k][0] = (double)b[c];
    bb[k][1] = (double)b[c + 1];
    bb[k][2] = (double)b[WW + c];
    bb[k][3] = (double)b[WW + c + W];
    bb[k][4] = (double)b[2 * WW + c];
  }
  // staging: batches of B5_B points per thread, all their loads issued before any LDS store
  constexpr int B5_B = 9;
  for (int e0 = threadIdx.x; e0 < 3 * BRWW; e0 += B5_B * B5_T) {
    int kk[B5_B];
    T xv[B5_B];
    uint8_t cv[B5_B];
#pragma unroll
    for (int u = 0; u < B5_B; u++) {
      int e = e0 + u * B5_T;
      int g = e / BRWW, q = e - g * BRWW, pj = q / BRW, pi = q - pj * BRW;
      int gi = gi0 + pi, gj = gj0 + pj;
      kk[u] = (e < 3 * BRWW && gi >= -1 && gi <= N && gj >= -1 && gj <= N) ? g * WW + (gj + 1) * W + (gi + 1) : -1;
    }
#pragma unroll
    for (int u = 0; u < B5_B; u++) {
      int k = kk[u] >= 0 ? kk[u] : 0;
      xv[u] = x[k];
      cv[u] = cls[k];
    }
#pragma unroll
    for (int u = 0; u < B5_B; u++) {
      int e = e0 + u * B5_T;
      if (e >= 3 * BRWW) continue;
      bool in = kk[u] >= 0;
      xs[e] = in ? xv[u] : (T)0;
      cs[e] = in ? cv[u] : (uint8_t)K_INACTIVE;
    }
  }
  if (threadIdx.x == 0) xs[3 * BRWW] = x[3 * WW];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 5; k++) {
    // LDS cell coordinates: point index of cell i is i - gi0, and the update takes the cell as point - 1
    if (bi[k] >= 0) box_update_rb<T>(BRW, K, cs, xs, bb[k], bi[k] - gi0 - 1, bj[k] - gj0 - 1);
    __syncthreads();
  }
  // owned points: the tile's cells, plus the border row / column -1 or N next to it
  const int ib = i0 == 0 ? -1 : i0, ie = min(N, i0 + BT) + (i0 + BT >= N ? 1 : 0);
  const int jb = j0 == 0 ? -1 : j0, je = min(N, j0 + BT) + (j0 + BT >= N ? 1 : 0);
  const int ow = ie - ib, oh = je - jb;
  for (int e = threadIdx.x; e < 3 * ow * oh; e += B5_T) {
    int g = e / (ow * oh), q = e - g * ow * oh, lj = q / ow, li = q - lj * ow;
    int gi = ib + li, gj = jb + lj;
    y[g * WW + (gj + 1) * W + (gi + 1)] = xs[g * BRWW + (gj - gj0) * BRW + (gi - gi0)];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) y[3 * WW] = xs[3 * BRWW];
}

// box relaxation of the band cells band[lo, hi) (one colour), spread over the whole device
template <typename T>
__global__ void __launch_bounds__(TPB) k_box_list(int N, int W, BoxK K, const uint8_t *__restrict__ cls,
                                                  T *__restrict__ x, const T *__restrict__ b, const int *__restrict__ band,
                                                  int lo, int hi) {
  int t = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= hi) return;
  int cell = band[t];
  box_update<T>(W, K, cls, x, b, cell % N, cell / N);
}

// fictitious-time relaxation of every ghost row at once (eq. ghostrelax, Jacobi): w += dtau (g - B w)
template <typename T>
__global__ void k_ghost_a(const int *__restrict__ pt, const int *__restrict__ col, const double *__restrict__ w,
                          const double *__restrict__ dtau, int ng, const T *__restrict__ x, const T *__restrict__ b,
                          double *__restrict__ tmp) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ng) return;
  int k = pt[r];
  double s = 0;
#pragma unroll
  for (int q = 0; q < 9; q++) s += w[9 * r + q] * (double)x[col[9 * r + q]];
  tmp[r] = (double)x[k] + dtau[r] * ((double)b[k] - s);
}
template <typename T>
__global__ void k_ghost_b(const int *__restrict__ pt, int ng, const double *__restrict__ tmp, T *__restrict__ x) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < ng) x[pt[r]] = (T)tmp[r];
}

// one simultaneous sweep of every ghost row reading the old ghost values from prev (row-indexed; null: from x)
// and writing the new ones to next (row-indexed, stored as T values; null: into x).  With prev given, every ghost
// value the sweep reads comes from prev (colr gives ghost columns as -(row + 1)), so writing x in place is safe;
// the arithmetic is that of k_ghost_a followed by k_ghost_b.
template <typename T>
__global__ void __launch_bounds__(TPB) k_ghost_sweep2(const int *__restrict__ pt, const int *__restrict__ col,
                                                      const int *__restrict__ colr, const double *__restrict__ w,
                                                      const double *__restrict__ dtau, int ng, T *x,
                                                      const T *__restrict__ b, const double *__restrict__ prev,
                                                      double *__restrict__ next) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ng) return;
  int k = pt[r];
  double sum = 0;
  if (prev) {
#pragma unroll
    for (int z = 0; z < 9; z++) {
      int c = colr[9 * r + z];
      sum += w[9 * r + z] * (c < 0 ? prev[-c - 1] : (double)x[c]);
    }
  } else {
#pragma unroll
    for (int z = 0; z < 9; z++) sum += w[9 * r + z] * (double)x[col[9 * r + z]];
  }
  const double old = prev ? prev[r] : (double)x[k];
  const T nv = (T)(old + dtau[r] * ((double)b[k] - sum));
  if (next)
    next[r] = (double)nv;
  else
    x[k] = nv;
}

// all lambda sweeps in one workgroup: Jacobi phases separated by barriers (global memory, same CU)
constexpr int GH_T = 1024;
template <typename T>
__global__ void __launch_bounds__(GH_T) k_ghost_sweeps(const int *__restrict__ pt, const int *__restrict__ col,
                                                       const double *__restrict__ w, const double *__restrict__ dtau, int ng,
                                                       T *x, const T *__restrict__ b, double *tmp, int sweeps) {
  for (int it = 0; it < sweeps; it++) {
    for (int r = threadIdx.x; r < ng; r += GH_T) {
      int k = pt[r];
      double s = 0;
#pragma unroll
      for (int q = 0; q < 9; q++) s += w[9 * r + q] * (double)x[col[9 * r + q]];
      tmp[r] = (double)x[k] + dtau[r] * ((double)b[k] - s);
    }
    __syncthreads();
    for (int r = threadIdx.x; r < ng; r += GH_T) x[pt[r]] = (T)tmp[r];
    __syncthreads();
  }
}

// extra relaxation of the boundary band (one workgroup): `sweeps` times the box sweep over the band cells in
// the colour order, each followed by lambda ghost sweeps
constexpr int BAND_T = 1024;
template <typename T>
__global__ void __launch_bounds__(BAND_T) k_band_sweeps(int N, int W, BoxK K,
                                                        const uint8_t *__restrict__ cls, T *x, const T *__restrict__ b,
                                                        const int *__restrict__ band, const int *__restrict__ off,
                                                        const int *__restrict__ pt, const int *__restrict__ col,
                                                        const double *__restrict__ w, const double *__restrict__ dtau,
                                                        int ng, double *tmp, int sweeps, int lambda, int ghosts_first) {
  if (ghosts_first) {
    for (int it = 0; it < lambda; it++) {
      for (int r = threadIdx.x; r < ng; r += BAND_T) {
        int k = pt[r];
        double sum = 0;
#pragma unroll
        for (int z = 0; z < 9; z++) sum += w[9 * r + z] * (double)x[col[9 * r + z]];
        tmp[r] = (double)x[k] + dtau[r] * ((double)b[k] - sum);
      }
      __syncthreads();
      for (int r = threadIdx.x; r < ng; r += BAND_T) x[pt[r]] = (T)tmp[r];
      __syncthreads();
    }
  }
  for (int s = 0; s < sweeps; s++) {
    for (int c = 0; c < 5; c++) {
      int lo = off[c], hi = off[c + 1];
      for (int q = lo + threadIdx.x; q < hi; q += BAND_T) {
        int cell = band[q];
        box_update<T>(W, K, cls, x, b, cell % N, cell / N);
      }
      __syncthreads();
    }
    for (int it = 0; it < lambda; it++) {
      for (int r = threadIdx.x; r < ng; r += BAND_T) {
        int k = pt[r];
        double sum = 0;
#pragma unroll
        for (int z = 0; z < 9; z++) sum += w[9 * r + z] * (double)x[col[9 * r + z]];
        tmp[r] = (double)x[k] + dtau[r] * ((double)b[k] - sum);
      }
      __syncthreads();
      for (int r = threadIdx.x; r < ng; r += BAND_T) x[pt[r]] = (T)tmp[r];
      __syncthreads();
    }
  }
}

// wall ghost rows: all their Jacobi sweeps at once, each row independent of every other ghost
template <typename T>
__device__ __forceinline__ void wall_ghost_row(int r, const int *__restrict__ g_pt, const int *__restrict__ g_col,
                                               const double *__restrict__ g_w, const double *__restrict__ g_dtau, T *x,
                                               const T *__restrict__ b, int sweeps) {
  int k = g_pt[r];
  double rest = 0, w0 = 0;
#pragma unroll
  for (int z = 0; z < 9; z++) {
    int c = g_col[9 * r + z];
    if (c == k)
      w0 += g_w[9 * r + z];
    else
      rest += g_w[9 * r + z] * (double)x[c];
  }
  double xv = (double)x[k], bb = (double)b[k], dt = g_dtau[r];
  for (int it = 0; it < sweeps; it++) xv = xv + dt * (bb - (w0 * xv + rest));
  x[k] = (T)xv;
}
// sum over a workgroup of BAND_T threads (every thread gets the total; fixed order)
__device__ double band_block_sum(double v) {
  __shared__ double s[BAND_T / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0;
  for (int q = 0; q < BAND_T / 64; q++) t += s[q];
  return t;
}

// G, the sum over a level's internal cells of the continuity right-hand sides (less the wall Dirichlet faces'
// share), which every xi update of the level subtracts, comes as ngp partial sums: one (k_gsum) on a level whose
// right-hand side the caller set, the block sums of k_resid_restrict on a coarse level.  A 1024-thread workgroup
// issues its loads early (gp_start: two per thread, in flight with what the kernel loads next) and sums them in
// a fixed order when it needs G (gp_total).
struct GpPre {
  double a, b;
};
__device__ __forceinline__ GpPre gp_start(const double *__restrict__ gp, int ngp) {
  const int t = threadIdx.x;
  return {t < ngp ? gp[t] : 0.0, t + BAND_T < ngp ? gp[t + BAND_T] : 0.0};
}
__device__ __forceinline__ double gp_total(GpPre pre, const double *__restrict__ gp, int ngp) {
  double v = pre.a + pre.b;
  for (int q = threadIdx.x + 2 * BAND_T; q < ngp; q += BAND_T) v += gp[q];
  return band_block_sum(v);
}

// One relaxation step's work after the five box sweeps, in one workgroup:
//  - workgroup 0: the body ghost rows and the band boxes as in k_band_sweeps, with the values the kernel writes
//    staged in LDS (region slots [0, nregw), written back at the end) and, when they fit, the values it only reads
//    (slots [nregw, nreg); they are constant during the kernel, and any others come from global memory), then
//    xi <- mean over internal cells of (div u - g) from the boundary faces of the internal cells;
//  - the other workgroups: the wall ghost rows, all lambda (1 + sweeps) of their Jacobi sweeps at once (they read
//    only internal points next to the walls, which no band box writes, and neither a body ghost row nor a listed
//    face reads them).
constexpr int BATCH = 8;
struct BandOff {
  int o[6];
};
// Staging modes of k_band_lds, each one also staging what the ones before it stage:
//   0: the written points only (every other point comes from global memory);
//   1: also the points the box and ghost tables only read (every table entry is an LDS slot);
//   2: also the body ghost rows' tables (slots as 16-bit numbers, weights, dtau);
//   3: also the band boxes' tables (slots, flags, cell) and their right-hand sides.
// LDS after the region, 8-byte aligned: nv, gb (new values and right-hand sides of the ghost rows), then for mode
// >= 2: gw (9 nbg), gdt (nbg), gl (10 nbg 16-bit), and for mode 3: bbv (5 nb), bcl (nb), bfl (nb), bsl (21 nb 16-bit)
__host__ __device__ inline size_t band_lds_bytes(int mode, size_t region_bytes, int nbg, int nb) {
  size_t o = (region_bytes + 7) & ~(size_t)7;
  o += 2 * (size_t)nbg * 8;
  if (mode >= 2) o = (o + 10 * (size_t)nbg * 8 + 10 * (size_t)nbg * 2 + 7) & ~(size_t)7;
  if (mode >= 3) o += 5 * (size_t)nb * 8 + 2 * (size_t)nb * 4 + 21 * (size_t)nb * 2;
  return o;
}
template <typename T, int MODE>
__global__ void __launch_bounds__(BAND_T) k_band_lds(int N, int W, BoxK K, T *x, const T *__restrict__ b,
                                                     BandOff off, const int *__restrict__ bbox, int bcap,
                                                     const int *__restrict__ reg_pt, int nreg, int nregw,
                                                     const int *__restrict__ bg_k,
                                                     const int *__restrict__ bg_loc, const double *__restrict__ bg_w,
                                                     const double *__restrict__ bg_dt, int nbg, int gcap,
                                                     const int *__restrict__ g_pt, const int *__restrict__ g_col,
                                                     const double *__restrict__ g_w, const double *__restrict__ g_dtau,
                                                     const int *__restrict__ wg_rows, int nwg, int sweeps, int lambda,
                                                     const int *__restrict__ f_code, const int *__restrict__ f_loc, int nf,
                                                     const double *__restrict__ gp, int ngp, const int *__restrict__ mp) {
  extern __shared__ unsigned char lds_raw[];
  T *xs = reinterpret_cast<T *>(lds_raw);
  const int nb = off.o[5];
  double *nv = reinterpret_cast<double *>(lds_raw + ((nreg * sizeof(T) + 7) & ~(size_t)7));
  double *gb = nv + nbg;
  double *gw = gb + nbg, *gdt = gw + 9 * nbg;
  uint16_t *gl = reinterpret_cast<uint16_t *>(gdt + nbg);
  double *bbv = reinterpret_cast<double *>(lds_raw + band_lds_bytes(2, nreg * sizeof(T), nbg, nb));
  int *bcl = reinterpret_cast<int *>(bbv + 5 * nb), *bfl = bcl + nb;
  uint16_t *bsl = reinterpret_cast<uint16_t *>(bfl + nb);
  const int WW = W * W;
  // value of a table entry: local LDS slot (written by this kernel) or -(global index + 1) (read only).  From
  // mode 1 on every point the box and ghost tables name is staged (the face list may still name others).
  auto val = [&](int e) -> double { return e >= 0 ? (double)xs[e] : (double)x[-e - 1]; };
  auto tval = [&](int e) -> double { return MODE >= 1 ? (double)xs[e] : val(e); };
  const int tid = threadIdx.x;
  if (blockIdx.x > 0) {
    // the other workgroups of the launch take the wall ghost rows, on other compute units
    for (int q = (blockIdx.x - 1) * BAND_T + tid; q < nwg; q += (gridDim.x - 1) * BAND_T)
      wall_ghost_row<T>(wg_rows[q], g_pt, g_col, g_w, g_dtau, x, b, lambda * (1 + sweeps));
    return;
  }
  // G's partials early where registers allow (modes 0 and 1 hold more of the region's values in registers)
  const GpPre gpre = MODE >= 2 ? gp_start(gp, ngp) : GpPre{0.0, 0.0};
  // mode 3 (small bands): this thread's face and written points' positions load with the staging, when there is
  // at most one face and WB_PRE written points per thread
  constexpr int WB_PRE = 4;
  const bool fpre = MODE == 3 && nf <= BAND_T, wpre = MODE == 3 && nregw <= WB_PRE * BAND_T;
  int pfe = 0, pfc = -1, pw[WB_PRE];
  if (fpre && tid < nf) {
    pfe = f_loc[tid];
    pfc = f_code[tid];
  }
#pragma unroll
  for (int u = 0; u < WB_PRE; u++) pw[u] = (wpre && tid + u * BAND_T < nregw) ? reg_pt[tid + u * BAND_T] : -1;
  // stage the region: batches of BATCH loads in flight per thread (16 at once measured slower on one CU)
  for (int q0 = tid; q0 < nreg; q0 += BATCH * BAND_T) {
    int gi[BATCH];
    T vv[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; u++) gi[u] = q0 + u * BAND_T < nreg ? reg_pt[q0 + u * BAND_T] : 0;
#pragma unroll
    for (int u = 0; u < BATCH; u++) vv[u] = x[gi[u]];
#pragma unroll
    for (int u = 0; u < BATCH; u++)
      if (q0 + u * BAND_T < nreg) xs[q0 + u * BAND_T] = vv[u];
  }
  for (int s2 = tid; s2 < nbg; s2 += BAND_T) {
    gb[s2] = (double)b[bg_k[s2]];
    if (MODE >= 2) {
#pragma unroll
      for (int z = 0; z < 9; z++) gw[z * nbg + s2] = bg_w[z * gcap + s2];
      gdt[s2] = bg_dt[s2];
#pragma unroll
      for (int z = 0; z < 10; z++) gl[z * nbg + s2] = (uint16_t)bg_loc[z * gcap + s2];
    }
  }
  if (MODE >= 3) {
    for (int q = tid; q < nb; q += BAND_T) {
      const int cell = bbox[22 * bcap + q], i = cell % N, j = cell / N, cg = (j + 1) * W + (i + 1);
      bcl[q] = cell;
      bfl[q] = bbox[21 * bcap + q];
#pragma unroll
      for (int z = 0; z < 21; z++) bsl[z * nb + q] = (uint16_t)bbox[z * bcap + q];
      bbv[q] = (double)b[cg];
      bbv[nb + q] = (double)b[cg + 1];
      bbv[2 * nb + q] = (double)b[WW + cg];
      bbv[3 * nb + q] = (double)b[WW + cg + W];
      bbv[4 * nb + q] = (double)b[2 * WW + cg];
    }
  }
  // the cell of this thread's first box of the next colour is loaded one colour ahead, so that the right-hand
  // sides of the box can be loaded together with its table
  int next_cell = MODE < 3 && off.o[0] + tid < off.o[1] ? bbox[22 * bcap + off.o[0] + tid] : 0;
  const double xi = (double)x[3 * WW];
  __syncthreads();
  // Jacobi sweeps of the body ghost rows; each new value goes through nv (written and read back by the same
  // thread), so no row data is held across the barrier
  auto ghost_block = [&]() {
    for (int it = 0; it < lambda; it++) {
      if (MODE >= 2) {
        for (int s2 = tid; s2 < nbg; s2 += BAND_T) {
          double sum = 0;
#pragma unroll
          for (int z = 0; z < 9; z++) sum += gw[z * nbg + s2] * (double)xs[gl[(1 + z) * nbg + s2]];
          nv[s2] = (double)xs[gl[s2]] + gdt[s2] * (gb[s2] - sum);
        }
      } else {
        for (int s0 = tid; s0 < nbg; s0 += 2 * BAND_T) {  // two rows per thread at a time: their loads overlap
          const int s1 = s0 + BAND_T, t1 = s1 < nbg ? s1 : s0;
          double sum0 = 0, sum1 = 0;
#pragma unroll
          for (int z = 0; z < 9; z++) {
            sum0 += bg_w[z * gcap + s0] * tval(bg_loc[(1 + z) * gcap + s0]);
            sum1 += bg_w[z * gcap + t1] * tval(bg_loc[(1 + z) * gcap + t1]);
          }
          nv[s0] = (double)xs[bg_loc[s0]] + bg_dt[s0] * (gb[s0] - sum0);
          if (s1 < nbg) nv[s1] = (double)xs[bg_loc[s1]] + bg_dt[s1] * (gb[s1] - sum1);
        }
      }
      __syncthreads();
      for (int s2 = tid; s2 < nbg; s2 += BAND_T) xs[MODE >= 2 ? (int)gl[s2] : bg_loc[s2]] = (T)nv[s2];
      __syncthreads();
    }
  };
  // one band box: table entry fld (0..20 slots, 21 flags) and right-hand side k (W E S N P)
  auto band_box = [&](auto TB, auto RB) {
    const int f = TB(21);
    const bool fW = f & 1, fE = f & 2, fS = f & 4, fN = f & 8, fP = f & 16;
    double uW = tval(TB(0)), uE = tval(TB(1)), uWW = tval(TB(2)), uEE = tval(TB(3)), uWS = tval(TB(4)),
           uWN = tval(TB(5)), uES = tval(TB(6)), uEN = tval(TB(7));
    double vS = tval(TB(8)), vN = tval(TB(9)), vSS = tval(TB(10)), vNN = tval(TB(11)), vSW = tval(TB(12)),
           vSE = tval(TB(13)), vNW = tval(TB(14)), vNE = tval(TB(15));
    double pc = tval(TB(16)), pW = tval(TB(17)), pE = tval(TB(18)), pS = tval(TB(19)), pN = tval(TB(20));
    const BoxNew o = box_core(K, fW, fE, fS, fN, fP, uW, uE, uWW, uEE, uWS, uWN, uES, uEN, vS, vN, vSS, vNN, vSW, vSE,
                              vNW, vNE, pc, pW, pE, pS, pN, RB(0), RB(1), RB(2), RB(3), RB(4), xi);
    if (!o.skip) {
      if (fP) xs[TB(16)] = (T)o.p;
      if (fW) xs[TB(0)] = (T)o.uW;
      if (fE) xs[TB(1)] = (T)o.uE;
      if (fS) xs[TB(8)] = (T)o.vS;
      if (fN) xs[TB(9)] = (T)o.vN;
    }
  };
  ghost_block();
  for (int sw = 0; sw < sweeps; sw++) {
    for (int c = 0; c < 5; c++) {
      if (MODE >= 3) {
        for (int q = off.o[c] + tid; q < off.o[c + 1]; q += BAND_T)
          band_box([&](int fld) { return fld == 21 ? bfl[q] : (int)bsl[fld * nb + q]; },
                   [&](int k) { return bbv[k * nb + q]; });
      } else {
        const int first_cell = next_cell, cn = c == 4 ? 0 : c + 1;
        next_cell = off.o[cn] + tid < off.o[cn + 1] ? bbox[22 * bcap + off.o[cn] + tid] : 0;
        for (int q = off.o[c] + tid; q < off.o[c + 1]; q += BAND_T) {
          const int cell = q == off.o[c] + tid ? first_cell : bbox[22 * bcap + q];
          const int i = cell % N, j = cell / N, cg = (j + 1) * W + (i + 1);
          const double rb[5] = {(double)b[cg], (double)b[cg + 1], (double)b[WW + cg], (double)b[WW + cg + W],
                                (double)b[2 * WW + cg]};
          band_box([&](int fld) { return bbox[fld * bcap + q]; }, [&](int k) { return rb[k]; });
        }
      }
      __syncthreads();
    }
    ghost_block();
  }
  double fs = 0;
  if (fpre) {
    if (pfc >= 0) {
      const double v = val(pfe);
      fs = (pfc & 1) ? -v : v;
    }
  } else {
    for (int q0 = tid; q0 < nf; q0 += BATCH * BAND_T) {
      int e[BATCH], cd[BATCH];
      double v[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; u++) {
        bool in = q0 + u * BAND_T < nf;
        e[u] = in ? f_loc[q0 + u * BAND_T] : 0;
        cd[u] = in ? f_code[q0 + u * BAND_T] : -1;
      }
#pragma unroll
      for (int u = 0; u < BATCH; u++) v[u] = val(e[u]);
#pragma unroll
      for (int u = 0; u < BATCH; u++)
        if (cd[u] >= 0) fs += (cd[u] & 1) ? -v[u] : v[u];
    }
  }
  fs = band_block_sum(fs);
  const double gsum = gp_total(MODE >= 2 ? gpre : gp_start(gp, ngp), gp, ngp);
  if (wpre) {
#pragma unroll
    for (int u = 0; u < WB_PRE; u++)
      if (pw[u] >= 0) x[pw[u]] = xs[tid + u * BAND_T];
  } else {
    for (int q0 = tid; q0 < nregw; q0 += BATCH * BAND_T) {  // only the written points go back
      int gi[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; u++) gi[u] = q0 + u * BAND_T < nregw ? reg_pt[q0 + u * BAND_T] : -1;
#pragma unroll
      for (int u = 0; u < BATCH; u++)
        if (gi[u] >= 0) x[gi[u]] = xs[q0 + u * BAND_T];
    }
  }
  if (tid == 0) x[3 * WW] = (T)((fs / K.h - gsum) / *mp);
}

// xi <- mean over internal cells of (div u - g), from the boundary faces of the internal cells (one workgroup)
template <typename T>
__global__ void __launch_bounds__(BAND_T) k_xi_faces(int WW, double h, T *x, const int *__restrict__ f_code, int nf,
                                                     const double *__restrict__ gp, int ngp, const int *__restrict__ mp) {
  const GpPre gpre = gp_start(gp, ngp);
  double fs = 0;
  for (int q = threadIdx.x; q < nf; q += BAND_T) {
    double v = (double)x[f_code[q] >> 1];
    fs += (f_code[q] & 1) ? -v : v;
  }
  fs = band_block_sum(fs);
  const double gsum = gp_total(gpre, gp, ngp);
  if (threadIdx.x == 0) x[3 * WW] = (T)((fs / h - gsum) / *mp);
}

// One relaxation step's band work over angular sectors (built by sector_build), one workgroup per sector: the
// sector's region is staged in LDS, its ghost rows and band boxes (those within reach of its own points, some
// also computed by the neighbouring sectors) are relaxed as in k_band_lds, and the values of the written points
// it owns go to out (by region index); workgroups S and on take the wall ghost rows.  k_band_sec_fin then moves
// out into x and updates xi.  Nothing reads x while this kernel writes it: the sectors write out only.
// lambda Jacobi sweeps of all ghost rows (eq. (ghostrelax)) and then xi from the boundary faces of the internal
// cells, in one workgroup (levels without the extra band relaxation, at most 2 BAND_T ghost rows).  Each thread
// keeps the tables of its rows in registers for every sweep and its new values in registers between the read and
// the write phase of a sweep; the face codes are loaded with the tables.
constexpr int GX_F = 4;  // face codes per thread loaded ahead
// R rows per thread (ng <= R * BAND_T)
template <typename T, int R>
__global__ void __launch_bounds__(BAND_T) k_ghost_xi(const int *__restrict__ pt, const int *__restrict__ col,
                                                     const int *__restrict__ colr, const int *__restrict__ colr_t,
                                                     const double *__restrict__ w_t, const double *__restrict__ w,
                                                     const double *__restrict__ dtau, int ng, T *x,
                                                     const T *__restrict__ b, int sweeps, int WW, double h,
                                                     const uint8_t *__restrict__ cls, const int *__restrict__ rowof,
                                                     const int *__restrict__ f_code, int nf,
                                                     const double *__restrict__ gp, int ngp, const int *__restrict__ mp) {
  // with colr (every ghost column given as -(its row + 1)) the ghost values live in LDS by row during the sweeps:
  // the other columns do not change in a ghost sweep, so every global load goes out before the first sweep and
  // the sweeps and the face sum read registers and LDS only
  __shared__ double gv[R * BAND_T];
  const int tid = threadIdx.x;
  const GpPre gpre = gp_start(gp, ngp);
  int fc[GX_F];
#pragma unroll
  for (int j = 0; j < GX_F; j++) fc[j] = tid + j * BAND_T < nf ? f_code[tid + j * BAND_T] : 0;
  // a thread without a second row computes a dummy one (point 0, weights 0) and does not store it, so that the
  // loads of both rows go out together
  int kk[R], cc[R][9];
  double ww[R][9], dt[R];
  bool has[R];
  const int *cs = (R == 1 && colr) ? colr : col;
#pragma unroll
  for (int i = 0; i < R; i++) {
    const int r = tid + i * BAND_T;
    has[i] = r < ng;
    kk[i] = has[i] ? pt[r] : 0;
    dt[i] = has[i] ? dtau[r] : 0.0;
#pragma unroll
    for (int z = 0; z < 9; z++) {  // column-major tables (colr_t, w_t) when given: coalesced over the rows
      cc[i][z] = has[i] ? (colr_t ? colr_t[(size_t)z * ng + r] : cs[9 * r + z]) : 0;
      ww[i][z] = has[i] ? (w_t ? w_t[(size_t)z * ng + r] : w[9 * r + z]) : 0.0;
    }
  }
  if (R == 1 && colr) {
    double xv[R][9], bb[R];
    int fr[GX_F];
    double fv[GX_F];
#pragma unroll
    for (int i = 0; i < R; i++) {
#pragma unroll
      for (int z = 0; z < 9; z++) xv[i][z] = cc[i][z] >= 0 ? (double)x[cc[i][z]] : 0.0;
      bb[i] = (double)b[kk[i]];
      if (has[i]) gv[tid + i * BAND_T] = (double)x[kk[i]];
    }
#pragma unroll
    for (int j = 0; j < GX_F; j++) {
      fr[j] = -1;
      fv[j] = 0.0;
      if (tid + j * BAND_T < nf) {
        const int k = fc[j] >> 1;
        const uint8_t c = cls[k];
        if (c == K_GHOST || c == K_GHOSTX || c == K_WALLG)
          fr[j] = rowof[k];
        else
          fv[j] = (double)x[k];
      }
    }
    __syncthreads();
    for (int it = 0; it < sweeps; it++) {
      double nv[R];
#pragma unroll
      for (int i = 0; i < R; i++) {
        double s = 0;
#pragma unroll
        for (int z = 0; z < 9; z++) s += ww[i][z] * (cc[i][z] >= 0 ? xv[i][z] : gv[-cc[i][z] - 1]);
        nv[i] = (has[i] ? gv[tid + i * BAND_T] : 0.0) + dt[i] * (bb[i] - s);
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < R; i++)
        if (has[i]) gv[tid + i * BAND_T] = (double)(T)nv[i];
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < R; i++)
      if (has[i]) x[kk[i]] = (T)gv[tid + i * BAND_T];
    double fs = 0;
#pragma unroll
    for (int j = 0; j < GX_F; j++)
      if (tid + j * BAND_T < nf) {
        const double v = fr[j] >= 0 ? gv[fr[j]] : fv[j];
        fs += (fc[j] & 1) ? -v : v;
      }
    for (int q = tid + GX_F * BAND_T; q < nf; q += BAND_T) {
      const int k = f_code[q] >> 1;
      const uint8_t c = cls[k];
      const double v = (c == K_GHOST || c == K_GHOSTX || c == K_WALLG) ? gv[rowof[k]] : (double)x[k];
      fs += (f_code[q] & 1) ? -v : v;
    }
    fs = band_block_sum(fs);
    const double gsum = gp_total(gpre, gp, ngp);
    if (tid == 0) x[3 * WW] = (T)((fs / h - gsum) / *mp);
    return;
  }
  for (int it = 0; it < sweeps; it++) {
    double nv[R];
#pragma unroll
    for (int i = 0; i < R; i++) {
      double s = 0;
#pragma unroll
      for (int z = 0; z < 9; z++) s += ww[i][z] * (double)x[cc[i][z]];
      nv[i] = (double)x[kk[i]] + dt[i] * ((double)b[kk[i]] - s);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; i++)
      if (has[i]) x[kk[i]] = (T)nv[i];
    __syncthreads();
  }
  // faces (some are ghost points the sweeps wrote): the codes loaded ahead, then any beyond them
  double fs = 0;
#pragma unroll
  for (int j = 0; j < GX_F; j++)
    if (tid + j * BAND_T < nf) {
      const double v = (double)x[fc[j] >> 1];
      fs += (fc[j] & 1) ? -v : v;
    }
  for (int q = tid + GX_F * BAND_T; q < nf; q += BAND_T) {
    const double v = (double)x[f_code[q] >> 1];
    fs += (f_code[q] & 1) ? -v : v;
  }
  fs = band_block_sum(fs);
  const double gsum = gp_total(gpre, gp, ngp);
  if (tid == 0) x[3 * WW] = (T)((fs / h - gsum) / *mp);
}
// The ghost sweeps and xi with two rows a thread (BAND_T < ng <= 2 BAND_T) from the column-major row tables (ghost
// columns by row): each row's fixed columns are summed once (they do not change in the sweeps) and its ghost
// columns kept as (weight, LDS row), weight zero for the others, so that the sweeps read registers and LDS only
template <typename T>
__global__ void __launch_bounds__(BAND_T) k_ghost_xi2(const int *__restrict__ pt, const int *__restrict__ colr_t,
                                                      const double *__restrict__ w_t, const double *__restrict__ dtau,
                                                      int ng, T *x, const T *__restrict__ b, int sweeps, int WW, double h,
                                                      const uint8_t *__restrict__ cls, const int *__restrict__ rowof,
                                                      const int *__restrict__ f_code, int nf,
                                                      const double *__restrict__ gp, int ngp, const int *__restrict__ mp) {
  __shared__ double gv[2 * BAND_T];
  const int tid = threadIdx.x;
  const GpPre gpre = gp_start(gp, ngp);
  double sf[2], bb[2], dt[2], wg[2][9];
  int kk[2], ix[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // LDS rows of the ghost columns, row 0's in the low 16 bits
  bool has[2];
#pragma unroll
  for (int i = 0; i < 2; i++) {
    const int r = tid + i * BAND_T;
    has[i] = r < ng;
    kk[i] = has[i] ? pt[r] : 0;
    dt[i] = has[i] ? dtau[r] : 0.0;
    int cz[9];
    double wz[9], xz[9];
#pragma unroll
    for (int z = 0; z < 9; z++) {
      cz[z] = has[i] ? colr_t[(size_t)z * ng + r] : 0;
      wz[z] = has[i] ? w_t[(size_t)z * ng + r] : 0.0;
    }
#pragma unroll
    for (int z = 0; z < 9; z++) xz[z] = cz[z] >= 0 ? (double)x[cz[z]] : 0.0;
    bb[i] = (double)b[kk[i]];
    if (has[i]) gv[r] = (double)x[kk[i]];
    sf[i] = 0.0;
#pragma unroll
    for (int z = 0; z < 9; z++) {
      const bool gz = cz[z] < 0;
      if (!gz) sf[i] += wz[z] * xz[z];
      wg[i][z] = gz ? wz[z] : 0.0;
      ix[z] |= (gz ? -cz[z] - 1 : 0) << (16 * i);
    }
  }
  __syncthreads();
  for (int it = 0; it < sweeps; it++) {
    double nv[2];
#pragma unroll
    for (int i = 0; i < 2; i++) {
      double s = sf[i];
#pragma unroll
      for (int z = 0; z < 9; z++) s += wg[i][z] * gv[(ix[z] >> (16 * i)) & 0xffff];
      nv[i] = (has[i] ? gv[tid + i * BAND_T] : 0.0) + dt[i] * (bb[i] - s);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; i++)
      if (has[i]) gv[tid + i * BAND_T] = (double)(T)nv[i];
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; i++)
    if (has[i]) x[kk[i]] = (T)gv[tid + i * BAND_T];
  // xi: the boundary faces, ghost ones from LDS (the sweeps change only ghost points)
  double fs = 0;
  for (int q = tid; q < nf; q += BAND_T) {
    const int k = f_code[q] >> 1;
    const uint8_t c = cls[k];
    const double v = (c == K_GHOST || c == K_GHOSTX || c == K_WALLG) ? gv[rowof[k]] : (double)x[k];
    fs += (f_code[q] & 1) ? -v : v;
  }
  fs = band_block_sum(fs);
  const double gsum = gp_total(gpre, gp, ngp);
  if (tid == 0) x[3 * WW] = (T)((fs / h - gsum) / *mp);
}

struct SecTabs {
  int poff[SEC_MAX + 1], boff[5 * SEC_MAX + 1], goff[SEC_MAX + 1], ooff[SEC_MAX + 1];
};
// GST: the sector's ghost-row tables are staged in LDS with the region (the sweeps then read no global memory)
template <typename T, bool GST>
__global__ void __launch_bounds__(BAND_T) k_band_sec(int N, int W, BoxK K, const T *x, T *xw,
                                                     const T *__restrict__ b, int S, SecTabs tb,
                                                     const int *__restrict__ spt, const uint16_t *__restrict__ bsl,
                                                     const int *__restrict__ bfl, const int *__restrict__ bcell,
                                                     int bstride, const uint16_t *__restrict__ gl,
                                                     const double *__restrict__ gw, const double *__restrict__ gdt,
                                                     const int *__restrict__ gk, int gstride,
                                                     const int *__restrict__ own_loc, const int *__restrict__ own_g,
                                                     double *__restrict__ out, const int *__restrict__ g_pt,
                                                     const int *__restrict__ g_col, const double *__restrict__ g_w,
                                                     const double *__restrict__ g_dtau, const int *__restrict__ wg_rows,
                                                     int nwg, int sweeps, int lambda) {
  extern __shared__ unsigned char lds_raw[];
  const int tid = threadIdx.x, sec = blockIdx.x;
  if (sec >= S) {
    for (int q = (sec - S) * BAND_T + tid; q < nwg; q += (gridDim.x - S) * BAND_T)
      wall_ghost_row<T>(wg_rows[q], g_pt, g_col, g_w, g_dtau, xw, b, lambda * (1 + sweeps));
    return;
  }
  const int p0 = tb.poff[sec], np = tb.poff[sec + 1] - p0, g0 = tb.goff[sec], ng = tb.goff[sec + 1] - g0;
  const int WW = W * W;
  T *xs = reinterpret_cast<T *>(lds_raw);
  double *nv = reinterpret_cast<double *>(lds_raw + ((np * sizeof(T) + 7) & ~(size_t)7));
  double *gb = nv + ng;
  double *gws = gb + ng, *gdts = gws + 9 * ng;              // GST: 9 weights field-major, dtau
  uint16_t *gls = reinterpret_cast<uint16_t *>(gdts + ng);  // GST: own + 9 column slots, field-major
  for (int q0 = tid; q0 < np; q0 += BATCH * BAND_T) {
    int gi[BATCH];
    T vv[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; u++) gi[u] = q0 + u * BAND_T < np ? spt[p0 + q0 + u * BAND_T] : 0;
#pragma unroll
    for (int u = 0; u < BATCH; u++) vv[u] = x[gi[u]];
#pragma unroll
    for (int u = 0; u < BATCH; u++)
      if (q0 + u * BAND_T < np) xs[q0 + u * BAND_T] = vv[u];
  }
  for (int k = tid; k < ng; k += BAND_T) {
    gb[k] = (double)b[gk[g0 + k]];
    if (GST) {
#pragma unroll
      for (int z = 0; z < 9; z++) gws[z * ng + k] = gw[z * gstride + g0 + k];
#pragma unroll
      for (int z = 0; z < 10; z++) gls[z * ng + k] = gl[z * gstride + g0 + k];
      gdts[k] = gdt[g0 + k];
    }
  }
  // the cell of this thread's first box of the next colour is loaded one colour ahead, so that the right-hand
  // sides of the box go out together with its table
  auto first_cell_of = [&](int c) {
    const int q = tb.boff[5 * sec + c] + tid;
    return q < tb.boff[5 * sec + c + 1] ? bcell[q] : 0;
  };
  int next_cell = first_cell_of(0);
  const double xi = (double)x[3 * WW];
  __syncthreads();
  auto ghost_block = [&]() {
    for (int it = 0; it < lambda; it++) {
      for (int k = tid; k < ng; k += BAND_T) {
        double sum = 0;
        if (GST) {
#pragma unroll
          for (int z = 0; z < 9; z++) sum += gws[z * ng + k] * (double)xs[gls[(1 + z) * ng + k]];
          nv[k] = (double)xs[gls[k]] + gdts[k] * (gb[k] - sum);
        } else {
          const int idx = g0 + k;
#pragma unroll
          for (int z = 0; z < 9; z++) sum += gw[z * gstride + idx] * (double)xs[gl[(1 + z) * gstride + idx]];
          nv[k] = (double)xs[gl[idx]] + gdt[idx] * (gb[k] - sum);
        }
      }
      __syncthreads();
      for (int k = tid; k < ng; k += BAND_T) xs[GST ? gls[k] : gl[g0 + k]] = (T)nv[k];
      __syncthreads();
    }
  };
  ghost_block();
  for (int sw = 0; sw < sweeps; sw++) {
    for (int c = 0; c < 5; c++) {
      const int first_cell = next_cell;
      next_cell = first_cell_of(c == 4 ? 0 : c + 1);
      for (int q = tb.boff[5 * sec + c] + tid; q < tb.boff[5 * sec + c + 1]; q += BAND_T) {
        auto TB = [&](int fld) { return (int)bsl[fld * bstride + q]; };
        const int cell = q == tb.boff[5 * sec + c] + tid ? first_cell : bcell[q];
        const int i = cell % N, j = cell / N, cg = (j + 1) * W + (i + 1);
        const int f = bfl[q];
        const bool fW = f & 1, fE = f & 2, fS = f & 4, fN = f & 8, fP = f & 16;
        const double bW_ = b[cg], bE_ = b[cg + 1], bS_ = b[WW + cg], bN_ = b[WW + cg + W], bP_ = b[2 * WW + cg];
        double uW = xs[TB(0)], uE = xs[TB(1)], uWW = xs[TB(2)], uEE = xs[TB(3)], uWS = xs[TB(4)], uWN = xs[TB(5)],
               uES = xs[TB(6)], uEN = xs[TB(7)];
        double vS = xs[TB(8)], vN = xs[TB(9)], vSS = xs[TB(10)], vNN = xs[TB(11)], vSW = xs[TB(12)],
               vSE = xs[TB(13)], vNW = xs[TB(14)], vNE = xs[TB(15)];
        double pc = xs[TB(16)], pW = xs[TB(17)], pE = xs[TB(18)], pS = xs[TB(19)], pN = xs[TB(20)];
        const BoxNew o = box_core(K, fW, fE, fS, fN, fP, uW, uE, uWW, uEE, uWS, uWN, uES, uEN, vS, vN, vSS, vNN, vSW, vSE,
                                  vNW, vNE, pc, pW, pE, pS, pN, bW_, bE_, bS_, bN_, bP_, xi);
        if (!o.skip) {
          if (fP) xs[TB(16)] = (T)o.p;
          if (fW) xs[TB(0)] = (T)o.uW;
          if (fE) xs[TB(1)] = (T)o.uE;
          if (fS) xs[TB(8)] = (T)o.vS;
          if (fN) xs[TB(9)] = (T)o.vN;
        }
      }
      __syncthreads();
    }
    ghost_block();
  }
  for (int k = tb.ooff[sec] + tid; k < tb.ooff[sec + 1]; k += BAND_T) out[own_g[k]] = (double)xs[own_loc[k]];
}
// the written points from out into x (region index -> point; workgroups 1 and on), and xi from the boundary
// faces of the internal cells as in k_xi_faces (workgroup 0; a written face takes its value from out, as the
// others write it into x)
template <typename T>
__global__ void __launch_bounds__(BAND_T) k_band_sec_fin(const int *__restrict__ reg_pt, int nregw,
                                                         const double *__restrict__ out, T *x, int WW, double h,
                                                         const int *__restrict__ f_code, const int *__restrict__ f_loc,
                                                         int nf, const double *__restrict__ gp, int ngp,
                                                         const int *__restrict__ mp) {
  if (blockIdx.x > 0) {
    for (int g = (blockIdx.x - 1) * BAND_T + threadIdx.x; g < nregw; g += (gridDim.x - 1) * BAND_T)
      x[reg_pt[g]] = (T)out[g];
    return;
  }
  const GpPre gpre = gp_start(gp, ngp);
  double fs = 0;
  for (int q = threadIdx.x; q < nf; q += BAND_T) {
    const int e = f_loc[q];
    const double v = (e >= 0 && e < nregw) ? (double)(T)out[e] : (double)x[f_code[q] >> 1];
    fs += (f_code[q] & 1) ? -v : v;
  }
  fs = band_block_sum(fs);
  const double gsum = gp_total(gpre, gp, ngp);
  if (threadIdx.x == 0) x[3 * WW] = (T)((fs / h - gsum) / *mp);
}



// ---------------------------------------------------------------------------------------------------------
// deterministic grid reductions: fixed grid, fixed per-thread ranges, tree in LDS, the last block sums the
// block partials in a fixed order
// ---------------------------------------------------------------------------------------------------------

__device__ double block_sum(double v) {
  __shared__ double s[TPB];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = TPB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  double r = s[0];
  __syncthreads();
  return r;
}

// The reductions of whole levels below run on at most RD_B workgroups of RD_T threads, each thread with RD_U
// elements' loads in flight: the ticket (rd_last_total) costs one contended atomic and a fence per workgroup,
// which with 512 workgroups of 256 threads took longer than reading the data.
constexpr int RD_T = 1024, RD_B = 128, RD_U = 8;
static_assert(RD_B <= TPB, "pmean_total reads one partial per thread");
static inline int rd_blocks(long n) {
  return (int)std::max(1L, std::min((long)RD_B, (n + (long)RD_T * RD_U - 1) / ((long)RD_T * RD_U)));
}
__device__ bool rd_last_total(double mine, double *part, unsigned *ticket, double *total) {
  __shared__ bool last;
  const double bs = band_block_sum(mine);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = bs;
    __threadfence();
    last = atomicAdd(ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  const double v = threadIdx.x < gridDim.x
                       ? __hip_atomic_load(&part[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                       : 0.0;
  *total = band_block_sum(v);
  if (threadIdx.x == 0) *ticket = 0;
  return true;
}

// G = sum over the internal cells of (g - (wall Dirichlet faces of the cell, with their divergence signs) / h); the
// xi update then needs only the faces of the boundary list: xi = (sum over the listed faces of +-u / h - G) / mp
template <typename T>
__global__ void __launch_bounds__(RD_T) k_gsum(int W, double h, const uint8_t *__restrict__ cls, const T *__restrict__ x,
                                               const T *__restrict__ b, double *part, unsigned *ticket, double *out) {
  const int WW = W * W, stride = gridDim.x * RD_T;
  double s = 0;
  for (int t0 = blockIdx.x * RD_T + threadIdx.x; t0 < WW; t0 += RD_U * stride) {
    uint8_t c[RD_U];
    double g[RD_U];
#pragma unroll
    for (int u = 0; u < RD_U; u++) {
      const int t = t0 + u * stride;
      c[u] = t < WW ? cls[2 * WW + t] : (uint8_t)K_INACTIVE;
      g[u] = t < WW ? (double)b[2 * WW + t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < RD_U; u++) {
      if (c[u] != K_INT) continue;
      const int t = t0 + u * stride;
      double wf = 0;
      if (cls[t + 1] == K_WALLD) wf += (double)x[t + 1];
      if (cls[t] == K_WALLD) wf -= (double)x[t];
      if (cls[WW + t + W] == K_WALLD) wf += (double)x[WW + t + W];
      if (cls[WW + t] == K_WALLD) wf -= (double)x[WW + t];
      s += g[u] - wf / h;
    }
  }
  double tot;
  if (rd_last_total(s, part, ticket, &tot) && threadIdx.x == 0) *out = tot;
}

// mean of the internal pressure (row eq:midpoint) as block partials part[0, gridDim.x): every block of the
// consumer adds them (pmean_total), which costs less than electing a last block with a ticket (a device-scope fence
// per block)
template <typename T>
__global__ void __launch_bounds__(RD_T) k_pmean(int W, const uint8_t *__restrict__ cls, const T *__restrict__ x,
                                                double *part) {
  const int WW = W * W, stride = gridDim.x * RD_T;
  double s = 0;
  for (int t0 = blockIdx.x * RD_T + threadIdx.x; t0 < WW; t0 += RD_U * stride) {
    uint8_t c[RD_U];
    double v[RD_U];
#pragma unroll
    for (int u = 0; u < RD_U; u++) {  // loads at a clamped position: none waits for a test
      const int t = t0 + u * stride, tc = min(t, WW - 1);
      const uint8_t cv = cls[2 * WW + tc];
      v[u] = (double)x[2 * WW + tc];
      c[u] = t < WW ? cv : (uint8_t)K_INACTIVE;
    }
#pragma unroll
    for (int u = 0; u < RD_U; u++)
      if (c[u] == K_INT) s += v[u];
  }
  const double bs = band_block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = bs;
}
// the mean from k_pmean's np <= TPB block partials, in a fixed order, in every block of a TPB-thread consumer (all
// its threads call it); block 0 also stores it to *out
__device__ double pmean_total(const double *__restrict__ part, int np, const int *__restrict__ mp, double *out) {
  __shared__ double sm[TPB / 64];
  double v = (int)threadIdx.x < np ? part[threadIdx.x] : 0.0;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0;
  for (int q = 0; q < TPB / 64; q++) t += sm[q];
  const double m = t / *mp;
  if (blockIdx.x == 0 && threadIdx.x == 0) *out = m;
  return m;
}
template <typename T>
__global__ void __launch_bounds__(TPB) k_pshift(int W, const uint8_t *__restrict__ cls, T *__restrict__ x,
                                                const double *__restrict__ part, int np, const int *__restrict__ mp,
                                                double *mean) {
  const int WW = W * W;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int tc = min(t, WW - 1);
  const uint8_t c = cls[2 * WW + tc];
  const double v = (double)x[2 * WW + tc];  // loaded with the partials
  const double m = pmean_total(part, np, mp, mean);
  if (t >= WW) return;
  if (c == K_INT || c == K_GHOST || c == K_GHOSTX) x[2 * WW + t] = (T)(v - m);
}

// ---------------------------------------------------------------------------------------------------------
// residual r = b - M x
// ---------------------------------------------------------------------------------------------------------
// residual of the point rows (internal momentum and continuity rows, wall identity rows; 0 for every other
// point, whose row, if any, is a ghost row handled by k_resid_ghost)
template <typename T, int G>
__device__ __forceinline__ double resid_int(int W, double h, double a, double d, const T *__restrict__ x,
                                            const T *__restrict__ b, int t) {
  // the residual of the internal row t of component G (any padded position at least one cell inside the ring
  // reads only entries of x)
  const int WW = W * W, q = t - G * WW;
  const T *u = x, *v = x + WW, *p = x + 2 * WW;
  double ih = 1.0 / h;
  if (G == 0)
    return (double)b[t] - (d * (double)u[q] - a * ((double)u[q - 1] + (double)u[q + 1] + (double)u[q - W] + (double)u[q + W]) +
                           ((double)p[q] - (double)p[q - 1]) * ih);
  if (G == 1)
    return (double)b[t] - (d * (double)v[q] - a * ((double)v[q - 1] + (double)v[q + 1] + (double)v[q - W] + (double)v[q + W]) +
                           ((double)p[q] - (double)p[q - W]) * ih);
  return (double)b[t] - (((double)u[q + 1] - (double)u[q] + (double)v[q + W] - (double)v[q]) * ih - (double)x[3 * WW]);
}
template <typename T>
__device__ __forceinline__ double resid_point(int W, double h, double a, double d, const uint8_t *__restrict__ cls,
                                              const T *__restrict__ x, const T *__restrict__ b, int t) {
  const int WW = W * W;
  uint8_t c = cls[t];
  if (c == K_INT) {
    const int g = t / WW;
    if (g == 0) return resid_int<T, 0>(W, h, a, d, x, b, t);
    if (g == 1) return resid_int<T, 1>(W, h, a, d, x, b, t);
    return resid_int<T, 2>(W, h, a, d, x, b, t);
  }
  if (c == K_WALLD) return (double)b[t] - (double)x[t];
  return 0.0;
}
// ---------------------------------------------------------------------------------------------------------
// coupled ghost boxes (tables and block inverses from the geometry build): after the box sweep, colour by colour,
// every coupled box of the colour forms the residuals of its rows from the values at the start of the colour,
// then adds its inverse times them to the unknowns it writes.  Phase one reads, phase two writes, so the boxes of
// one colour never see each other's updates.
// ---------------------------------------------------------------------------------------------------------
struct XbTab {
  const int *idx;
  const double *inv;
  int S;                   // stride of the field-major row tables (the level's slot capacity)
  const int *gc;           // 9 columns per ghost slot (gc[s] = -1: internal slot)
  const double *gw;        // 9 weights per ghost slot
  const int *uk, *uo, *ub, *um;  // write tables: target point (-1: none), inverse row, box's first slot, box size
};
static inline XbTab xb_tab(const Geo &G) {
  return XbTab{G.xb_idx, G.xb_inv, G.xb_scap, G.xb_gc, G.xb_gw, G.xb_uk, G.xb_uo, G.xb_ub, G.xb_um};
}
// residual of the row of slot s (its point's internal row, or the point's ghost row); every table entry it needs
// is one load away from s
template <typename T>
__device__ __forceinline__ double xb_slot_res(int W, double h, double a, double d, const T *x, const T *b,
                                              const XbTab &X, int s) {
  // every table entry of the slot at once (an internal slot's ghost entries are not used)
  const int k = X.idx[s];
  int c[9];
  double w[9];
#pragma unroll
  for (int z = 0; z < 9; z++) {
    c[z] = X.gc[(size_t)z * X.S + s];
    w[z] = X.gw[(size_t)z * X.S + s];
  }
  if (c[0] < 0) {
    const int g = k / (W * W);
    if (g == 0) return resid_int<T, 0>(W, h, a, d, x, b, k);
    if (g == 1) return resid_int<T, 1>(W, h, a, d, x, b, k);
    return resid_int<T, 2>(W, h, a, d, x, b, k);
  }
  double sw = 0;
#pragma unroll
  for (int z = 0; z < 9; z++) sw += w[z] * (double)x[c[z]];
  return (double)b[k] - sw;
}
// the new value of slot s (when its box writes it): x + (row s of the inverse) . (the box's residuals), the
// residual of slot q of the box at rs[q - rbase]
template <typename T>
__device__ __forceinline__ void xb_slot_write(const XbTab &X, T *x, const double *rs, int rbase, int s) {
  const int k = X.uk[s];
  if (k < 0) return;
  const int m = X.um[s];
  const double *iv = X.inv + X.uo[s];
  const double *r = rs + (X.ub[s] - rbase);
  double v = 0;
#pragma unroll 8
  for (int c = 0; c < m; c++) v += iv[c] * r[c];
  x[k] = (T)((double)x[k] + v);
}
template <typename T>
__global__ void __launch_bounds__(TPB) k_xb_res(int lo, int hi, int W, double h, double a, double d,
                                                const uint8_t *__restrict__ cls, const T *x, const T *b, XbTab X,
                                                double *rs) {
  const int s = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (s < hi) rs[s] = xb_slot_res<T>(W, h, a, d, x, b, X, s);
}
template <typename T>
__global__ void __launch_bounds__(TPB) k_xb_upd(int lo, int hi, T *x, XbTab X, const double *rs) {
  const int s = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (s < hi) xb_slot_write<T>(X, x, rs, 0, s);
}
struct XbOff {
  int o[6];
};
// all five colours in one workgroup (levels whose colours have few slots)
constexpr int XW_T = 1024;
template <typename T>
__global__ void __launch_bounds__(XW_T) k_xb_wg(XbOff so, int W, double h, double a, double d,
                                                const uint8_t *__restrict__ cls, T *x, const T *b, XbTab X, double *rs) {
  for (int c = 0; c < 5; c++) {
    for (int s = so.o[c] + threadIdx.x; s < so.o[c + 1]; s += XW_T) rs[s] = xb_slot_res<T>(W, h, a, d, x, b, X, s);
    __syncthreads();
    for (int s = so.o[c] + threadIdx.x; s < so.o[c + 1]; s += XW_T) xb_slot_write<T>(X, x, rs, 0, s);
    __syncthreads();
  }
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_resid_pts(int N, int W, double h, double a, double d,
                                                   const uint8_t *__restrict__ cls, const T *__restrict__ x,
                                                   const T *__restrict__ b, T *__restrict__ r, unsigned long long *rmax) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * W * W) return;
  r[t] = (T)resid_point<T>(W, h, a, d, cls, x, b, t);
  (void)N;
  (void)rmax;
}
// residual of the point rows, one point per thread in the first nbp blocks, and of the ghost rows (pt, col, w:
// ng rows of nine columns), one row per thread in the blocks after them (the point blocks leave those points'
// entries to them), stored in r when store is set (an FP64 solve needs only the norm); each block leaves the largest |residual| (as the bits of the double, which order like the
// values; NaN above everything) in part[gridDim + block] and its sum of the internal pressures in part[block],
// for k_resid_mean_row (no atomics and no grid-wide fence: the kernel writes the whole residual)
template <typename T>
__global__ void __launch_bounds__(TPB) k_resid_pts_norm(int W, double h, double a, double d,
                                                        const uint8_t *__restrict__ cls, const T *__restrict__ x,
                                                        const T *__restrict__ b, T *__restrict__ r, int nbp,
                                                        const int *__restrict__ pt, const int *__restrict__ col,
                                                        const double *__restrict__ w, int ng, double *part, int store) {
  __shared__ unsigned long long sm[TPB / 64];
  const int WW = W * W;
  double res = 0, ps = 0;
  if ((int)blockIdx.x < nbp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 3 * WW) {
      // the loads of the internal row go out with the class (at a fixed internal position where this point's
      // row would read outside its component), then the class picks the row
      const int g = t / WW, q = t - g * WW;
      const int k = q > W && q < WW - W - 1 ? t : g * WW + W + 1;
      const uint8_t c = cls[t];
      const double bt = (double)b[t], xt = (double)x[t];
      const double ri = g == 0 ? resid_int<T, 0>(W, h, a, d, x, b, k)
                                : (g == 1 ? resid_int<T, 1>(W, h, a, d, x, b, k) : resid_int<T, 2>(W, h, a, d, x, b, k));
      if (c != K_GHOST && c != K_GHOSTX && c != K_WALLG) {
        res = c == K_INT ? ri : (c == K_WALLD ? bt - xt : 0.0);
        if (store) r[t] = (T)res;
        if (t >= 2 * WW && c == K_INT) ps += xt;
      }
    }
  } else {
    const int q = (blockIdx.x - nbp) * blockDim.x + threadIdx.x;
    if (q < ng) {
      const int k = pt[q];
      double sw = 0;
#pragma unroll
      for (int z = 0; z < 9; z++) sw += w[9 * q + z] * (double)x[col[9 * q + z]];
      res = (double)b[k] - sw;
      if (store) r[k] = (T)res;
    }
  }
  unsigned long long m = (unsigned long long)__double_as_longlong(fabs(res));
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long q = __shfl_xor(m, o, 64);
    m = q > m ? q : m;
  }
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  ps = block_sum(ps);  // its barriers also publish sm
  if (threadIdx.x == 0) {
    for (int q = 0; q < TPB / 64; q++) m = sm[q] > m ? sm[q] : m;
    part[blockIdx.x] = ps;
    part[gridDim.x + blockIdx.x] = __longlong_as_double((long long)m);
  }
}
// the mean-pressure row's residual -mean(p) from the block sums of k_resid_pts_norm (fixed order), into r[3WW], and
// the max norm of the whole residual into *rmax (as bits), and into *hmax when given (pinned host memory, so that
// the host can poll it without a copy).  1024 threads, eight loads in flight per thread.
constexpr int RM_T = 1024;
template <typename T>
__global__ void __launch_bounds__(RM_T) k_resid_mean_row(const double *__restrict__ part, int nb, const int *mp,
                                                         T *r3, unsigned long long *rmax,
                                                         unsigned long long *hmax) {
  __shared__ double ssum[RM_T / 64];
  __shared__ unsigned long long smax[RM_T / 64];
  double v = 0;
  unsigned long long m = 0;
  for (int q0 = threadIdx.x; q0 < nb; q0 += 8 * RM_T) {
    double ps[8], pm[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int q = q0 + u * RM_T;
      ps[u] = q < nb ? part[q] : 0.0;
      pm[u] = q < nb ? part[nb + q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      v += ps[u];
      const unsigned long long z = (unsigned long long)__double_as_longlong(pm[u]);
      m = z > m ? z : m;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    v += __shfl_xor(v, o, 64);
    const unsigned long long q = __shfl_xor(m, o, 64);
    m = q > m ? q : m;
  }
  if ((threadIdx.x & 63) == 0) {
    ssum[threadIdx.x >> 6] = v;
    smax[threadIdx.x >> 6] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0;
    for (int q = 0; q < RM_T / 64; q++) {
      tot += ssum[q];
      m = smax[q] > m ? smax[q] : m;
    }
    const double res = -tot / *mp;
    *r3 = (T)res;
    const unsigned long long z = (unsigned long long)__double_as_longlong(fabs(res));
    *rmax = z > m ? z : m;
    if (hmax) *hmax = z > m ? z : m;  // host memory the solver polls
  }
}
template <typename T>
__global__ void k_resid_ghost(const int *__restrict__ pt, const int *__restrict__ col, const double *__restrict__ w, int ng,
                              const T *__restrict__ x, const T *__restrict__ b, T *__restrict__ r, unsigned long long *rmax) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ng) return;
  int k = pt[q];
  double s = 0;
#pragma unroll
  for (int z = 0; z < 9; z++) s += w[9 * q + z] * (double)x[col[9 * q + z]];
  double res = (double)b[k] - s;
  r[k] = (T)res;
}
// max |b| over a vector (wavefront reduction, one atomic per wavefront)
template <typename T>
__global__ void k_absmax(const T *__restrict__ v, long n, unsigned long long *out) {
  const long st = (long)gridDim.x * blockDim.x;
  double a = 0;
  for (long t0 = blockIdx.x * (long)blockDim.x + threadIdx.x; t0 < n; t0 += 8 * st) {
    double w[8];
#pragma unroll
    for (int u = 0; u < 8; u++) w[u] = t0 + u * st < n ? fabs((double)v[t0 + u * st]) : 0.0;
#pragma unroll
    for (int u = 0; u < 8; u++) a = fmax(a, w[u]);
  }
  // one atomic per block (contended atomics on one address cost ~10 ns each)
  __shared__ unsigned long long sm[TPB / 64];
  unsigned long long z = (unsigned long long)__double_as_longlong(a);
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long q = __shfl_xor(z, o, 64);
    z = q > z ? q : z;
  }
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = z;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < TPB / 64; q++) z = sm[q] > z ? sm[q] : z;
    if (z) atomicMax(out, z);
  }
}

template <typename T>
__global__ void k_set_walld(int n, const uint8_t *cls, T *x, const T *b) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n && cls[t] == K_WALLD) x[t] = b[t];
}

template <typename T>
__global__ void k_fill(T *x, long n, T val) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < n) x[t] = val;
}

// ---------------------------------------------------------------------------------------------------------
// boundary-aware restriction (eqs. restop, restop5)
// ---------------------------------------------------------------------------------------------------------
// boundary-aware restriction of the fine residual to coarse entry t (t = 3 WWc is the mean row: 0); the fine
// residual at point kf of class cc is rv(kf, cc)
template <typename RV>
__device__ __forceinline__ double restrict_core(int Nf, int Wf, const uint8_t *__restrict__ clsf, int Nc, int Wc,
                                                const uint8_t *__restrict__ clsc, int t, RV rvf) {
  const int WWc = Wc * Wc, WWf = Wf * Wf;
  if (t == 3 * WWc) return 0.0;
  int g = t / WWc, q = t - g * WWc, jc = q / Wc - 1, ic = q % Wc - 1;
  uint8_t cc = clsc[t];
  if (!(cc == K_INT || cc == K_GHOST || cc == K_WALLG)) return 0.0;
  int fi[6], fj[6];
  double fw[6];
  int m = 0;
  if (g == 0) {
    for (int dy = 0; dy < 2; dy++)
      for (int dx = -1; dx <= 1; dx++) {
        fi[m] = 2 * ic + dx;
        fj[m] = 2 * jc + dy;
        fw[m] = (dx == 0 ? 0.25 : 0.125);
        m++;
      }
  } else if (g == 1) {
    for (int dy = -1; dy <= 1; dy++)
      for (int dx = 0; dx < 2; dx++) {
        fi[m] = 2 * ic + dx;
        fj[m] = 2 * jc + dy;
        fw[m] = (dy == 0 ? 0.25 : 0.125);
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
  bool all = true;
  int cnt = 0;
  double sw = 0, sa = 0;
  for (int z = 0; z < m; z++) {
    if (fi[z] < -1 || fi[z] > Nf || fj[z] < -1 || fj[z] > Nf) {
      all = false;
      continue;
    }
    int kf = g * WWf + pidx(Wf, fi[z], fj[z]);
    if (clsf[kf] == cc) {
      double rv = rvf(kf, cc);
      cnt++;
      sw += fw[z] * rv;
      sa += rv;
    } else
      all = false;
  }
  return all ? sw : (cnt ? sa / cnt : 0.0);
}
template <typename TF>
__device__ __forceinline__ double restrict_value(int Nf, int Wf, const uint8_t *__restrict__ clsf, const TF *__restrict__ rf,
                                                 int Nc, int Wc, const uint8_t *__restrict__ clsc, int t) {
  return restrict_core(Nf, Wf, clsf, Nc, Wc, clsc, t, [&](int kf, uint8_t) { return (double)rf[kf]; });
}
// residual and restriction in one pass: the residual of an internal, ghost or wall-ghost fine row is formed where
// the restriction needs it (rounded to T, as the stored residual would be; growof: the ghost row of each ghost
// point, whose residual is formed as in k_resid_ghost).  Also the zero initial guess of the coarse correction,
// and the coarse level's G (see
// gp_start) as block partials: gpart[block - b0] = the sum of the restricted continuity right-hand sides of the
// block's internal cells, for the blocks b0 = 2 Wc^2 / TPB and on (those holding pressure entries; with x = 0
// the wall Dirichlet faces add nothing).
// the restricted residual of coarse entry t (restrict_core with the residual formed inline): the classes of the
// entry's fine points are loaded together, then the values of all its internal ones together (a fine point that is
// not taken reads a fixed internal position instead), so an entry costs three dependent loads whatever its mix of
// classes; the sums are formed in restrict_core's order.
template <typename T>
__device__ __forceinline__ double resid_restrict_entry(int Nf, int Wf, double h, double a, double d,
                                                       const uint8_t *__restrict__ clsf, const T *__restrict__ xf,
                                                       const T *__restrict__ bf, const int *__restrict__ growof,
                                                       const int *__restrict__ gcol, const double *__restrict__ gw,
                                                       int Wc, const uint8_t *__restrict__ clsc, int t) {
  const int WWc = Wc * Wc, WWf = Wf * Wf;
  const bool xi_entry = t == 3 * WWc;  // the entry of xi restricts to 0
  const int tt = xi_entry ? 0 : t;
  const int g = tt / WWc, q = tt - g * WWc, jc = q / Wc - 1, ic = q % Wc - 1;
  const uint8_t cc = clsc[tt];  // loaded together with the fine classes below (no branch between)
  const bool taken = !xi_entry && (cc == K_INT || cc == K_GHOST || cc == K_WALLG);
  const int m = g < 2 ? 6 : 4, safe = g * WWf + pidx(Wf, 0, 0);
  int kf[6];
  bool ok[6];
  double fw[6], rv[6];
#pragma unroll
  for (int z = 0; z < 6; z++) {  // u: 2 rows of 3, v: 3 rows of 2, p: 2 x 2
    const int dx = g == 0 ? z % 3 - 1 : z % 2, dy = g == 0 ? z / 3 : (g == 1 ? z / 2 - 1 : z / 2);
    const int fi = 2 * ic + dx, fj = 2 * jc + dy;
    fw[z] = g == 2 ? 0.25 : ((g == 0 ? dx : dy) == 0 ? 0.25 : 0.125);
    const bool in = z < m && fi >= -1 && fi <= Nf && fj >= -1 && fj <= Nf;
    kf[z] = in ? g * WWf + pidx(Wf, fi, fj) : safe;
    ok[z] = in;
  }
#pragma unroll
  for (int z = 0; z < 6; z++) {
    const uint8_t cz = clsf[kf[z]];  // loaded for every slot (no short circuit)
    ok[z] = ok[z] & taken & (cz == cc);
  }
  if (cc == K_INT) {  // one branch per component, each slot's loads straight-line
    if (g == 0) {
#pragma unroll
      for (int z = 0; z < 6; z++) rv[z] = (double)(T)resid_int<T, 0>(Wf, h, a, d, xf, bf, ok[z] ? kf[z] : safe);
    } else if (g == 1) {
#pragma unroll
      for (int z = 0; z < 6; z++) rv[z] = (double)(T)resid_int<T, 1>(Wf, h, a, d, xf, bf, ok[z] ? kf[z] : safe);
    } else {
#pragma unroll
      for (int z = 0; z < 4; z++) rv[z] = (double)(T)resid_int<T, 2>(Wf, h, a, d, xf, bf, ok[z] ? kf[z] : safe);
      rv[4] = rv[5] = 0.0;
    }
  } else {
#pragma unroll
    for (int z = 0; z < 6; z++) {
      rv[z] = 0.0;
      if (ok[z]) {
        const int r = growof[kf[z]];
        double sw = 0;
#pragma unroll
        for (int e = 0; e < 9; e++) sw += gw[9 * r + e] * (double)xf[gcol[9 * r + e]];
        rv[z] = (double)(T)((double)bf[kf[z]] - sw);
      }
    }
  }
  if (!taken) return 0.0;
  bool all = true;
  int cnt = 0;
  double sw = 0, sa = 0;
#pragma unroll
  for (int z = 0; z < 6; z++) {
    if (z >= m) break;
    if (ok[z]) {
      cnt++;
      sw += fw[z] * rv[z];
      sa += rv[z];
    } else
      all = false;
  }
  return all ? sw : (cnt ? sa / cnt : 0.0);
}
template <typename T>
__global__ void __launch_bounds__(TPB) k_resid_restrict(int Nf, int Wf, double h, double a, double d,
                                                        const uint8_t *__restrict__ clsf, const T *__restrict__ xf,
                                                        const T *__restrict__ bf, const int *__restrict__ growof,
                                                        const int *__restrict__ gcol, const double *__restrict__ gw,
                                                        int Nc, int Wc, const uint8_t *__restrict__ clsc,
                                                        T *__restrict__ bc, T *__restrict__ xc, double *__restrict__ gpart) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x, WWc = Wc * Wc;
  double gs = 0;
  if (t <= 3 * WWc) {
    const T v = (T)resid_restrict_entry<T>(Nf, Wf, h, a, d, clsf, xf, bf, growof, gcol, gw, Wc, clsc, t);
    bc[t] = v;
    xc[t] = (T)0;
    if (t >= 2 * WWc && t < 3 * WWc && clsc[t] == K_INT) gs = (double)v;
  }
  const int b0 = 2 * WWc / TPB;
  if ((int)blockIdx.x >= b0) {  // the same for the whole block
    gs = block_sum(gs);
    if (threadIdx.x == 0) gpart[blockIdx.x - b0] = gs;
  }
}
// restriction of a stored residual (and, when xc is given, the zero initial guess of the coarse correction)
template <typename TF, typename TC>
__global__ void __launch_bounds__(TPB) k_restrict(int Nf, int Wf, const uint8_t *__restrict__ clsf, const TF *__restrict__ rf,
                                                  int Nc, int Wc, const uint8_t *__restrict__ clsc, TC *__restrict__ bc,
                                                  TC *__restrict__ xc) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > 3 * Wc * Wc) return;
  bc[t] = (TC)restrict_value<TF>(Nf, Wf, clsf, rf, Nc, Wc, clsc, t);
  if (xc) xc[t] = (TC)0;
}

// extension values: quadratic extrapolation from the sources (Sect. 4.3)
template <typename T>
__global__ void k_ext_fill(const int *__restrict__ e_pt, const int *__restrict__ e_src, const double *__restrict__ e_w, int ne,
                           T *__restrict__ x) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  if (e_src[3 * e] < 0) return;
  double v = e_w[3 * e] * (double)x[e_src[3 * e]] + e_w[3 * e + 1] * (double)x[e_src[3 * e + 1]] +
             e_w[3 * e + 2] * (double)x[e_src[3 * e + 2]];
  x[e_pt[e]] = (T)v;
}

// bilinear prolongation of the coarse correction to fine entry t (internal, ghost, extrapolated and wall-ghost
// points and xi; 0 elsewhere), coarse pressure mirrored outside the box (Sect. 4.3); xcv(kc) is the coarse value
// the coarse points of fine entry t (an entry of component g below 3 Wf^2) and their bilinear weights, in the
// order the sum takes them: slot 2 aa + bb for the y offset aa and x offset bb; ok: the slot is used
struct ProlongSlots {
  int kc[4];
  double w[4];
  bool ok[4];
};
__device__ __forceinline__ ProlongSlots prolong_slots(int Nf, int Wf, int Nc, int Wc, int t) {
  const int WWf = Wf * Wf, WWc = Wc * Wc;
  int g = t / WWf, q = t - g * WWf, j = q / Wf - 1, i = q % Wf - 1;
  int xi_[2], yi_[2];
  double xw[2], yw[2];
  int nx, ny;
  if (g == 0) {  // faces along x
    if ((i & 1) == 0) {
      xi_[0] = xi_[1] = i / 2;
      xw[0] = 1;
      xw[1] = 0;
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
  if (g == 1) {  // faces along y
    if ((j & 1) == 0) {
      yi_[0] = yi_[1] = j / 2;
      yw[0] = 1;
      yw[1] = 0;
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
  ProlongSlots S;
#pragma unroll
  for (int aa = 0; aa < 2; aa++)
#pragma unroll
    for (int bb = 0; bb < 2; bb++) {
      const int z = 2 * aa + bb;
      int ic = xi_[bb], jc = yi_[aa];
      if (g == 2) {  // pressure outside the box mirrored
        ic = ic < 0 ? 0 : (ic > Nc - 1 ? Nc - 1 : ic);
        jc = jc < 0 ? 0 : (jc > Nc - 1 ? Nc - 1 : jc);
      }
      S.ok[z] = aa < ny && bb < nx && ic >= -1 && ic <= Nc && jc >= -1 && jc <= Nc;
      S.kc[z] = g * WWc + (S.ok[z] ? pidx(Wc, ic, jc) : pidx(Wc, 0, 0));
      S.w[z] = xw[bb] * yw[aa];
    }
  return S;
}
template <typename XV>
__device__ __forceinline__ double prolong_value(int Nf, int Wf, const uint8_t *__restrict__ clsf, int Nc, int Wc,
                                                XV xcv, int t) {
  const int WWf = Wf * Wf, WWc = Wc * Wc;
  if (t == 3 * WWf) return xcv(3 * WWc);
  uint8_t c = clsf[t];
  if (!(c == K_INT || c == K_GHOST || c == K_GHOSTX || c == K_WALLG)) return 0.0;
  const ProlongSlots S = prolong_slots(Nf, Wf, Nc, Wc, t);
  double e = 0;
#pragma unroll
  for (int z = 0; z < 4; z++)
    if (S.ok[z]) e += S.w[z] * xcv(S.kc[z]);
  return e;
}
// With erow, the coarse extension points take their extrapolation from the sources here, rounded to TC as
// k_ext_fill stores it (erow: the extension row of each such point); without, xc already holds them.  The
// class test costs more than the k_ext_fill launch on the largest fine levels (PROLONG_EXT_INLINE_MAX cells).
constexpr long PROLONG_EXT_INLINE_MAX = 1L << 19;
template <typename TC, typename TF>
__global__ void __launch_bounds__(TPB) k_prolong(int Nf, int Wf, const uint8_t *__restrict__ clsf, TF *__restrict__ xf,
                                                 int Nc, int Wc, const TC *__restrict__ xc, const uint8_t *__restrict__ clsc,
                                                 const int *__restrict__ erow, const int *__restrict__ esrc,
                                                 const double *__restrict__ ew) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int WWf = Wf * Wf;
  if (t > 3 * WWf) return;
  if (t == 3 * WWf) {  // xi
    xf[t] = (TF)((double)xf[t] + (double)xc[3 * Wc * Wc]);
    return;
  }
  // every load of the entry is issued before any test (a slot that is not used reads a fixed coarse point)
  const ProlongSlots S = prolong_slots(Nf, Wf, Nc, Wc, t);
  const uint8_t c = clsf[t];
  const double xft = (double)xf[t];
  double xv[4];
  bool ext[4];
#pragma unroll
  for (int z = 0; z < 4; z++) {
    xv[z] = (double)xc[S.kc[z]];
    ext[z] = erow != nullptr && clsc[S.kc[z]] == K_EXT;
  }
  if (!(c == K_INT || c == K_GHOST || c == K_GHOSTX || c == K_WALLG)) return;
  double e = 0;
#pragma unroll
  for (int z = 0; z < 4; z++) {
    if (!S.ok[z]) continue;
    double v = xv[z];
    if (ext[z]) {
      const int r = erow[S.kc[z]];
      v = (double)(TC)(ew[3 * r] * (double)xc[esrc[3 * r]] + ew[3 * r + 1] * (double)xc[esrc[3 * r + 1]] +
                       ew[3 * r + 2] * (double)xc[esrc[3 * r + 2]]);
    }
    e += S.w[z] * v;
  }
  if (e != 0.0) xf[t] = (TF)(xft + e);
}

// exact coarsest solve with the stored inverse: x[map[q]] = sum_r Ainv[q][r] b[map[r]] (one wavefront per row)
template <typename T>
__global__ void __launch_bounds__(64) k_coarse_apply(const double *__restrict__ Ainv, const int *__restrict__ map,
                                                     const int *__restrict__ bmap, int nc, const T *__restrict__ b,
                                                     T *__restrict__ x) {
  int q = blockIdx.x;
  double s = 0;
  for (int r = threadIdx.x; r < nc; r += 64) s += Ainv[(size_t)q * nc + r] * (double)b[bmap[r]];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (threadIdx.x == 0) x[map[q]] = (T)s;
}


// ---------------------------------------------------------------------------------------------------------
// the small levels in one workgroup: the whole V cycle from level l0 (N <= 32 at the default sizes) down to the
// coarsest, with x, b, r and the classes of every level in LDS.  Same operations and arithmetic as the per-level
// kernels (the box update, residual, restriction, prolongation and coarsest product are shared); xi is taken
// from the direct sum over the internal cells.
// ---------------------------------------------------------------------------------------------------------
constexpr int SC_T = 1024;
constexpr int SC_MAXL = 4;
struct SmallLevel {
  int N, W, n, ng, ne, nband, mp;
  double h, a, d;
  BoxK K;
  const uint8_t *cls;
  const int *g_pt, *g_col, *e_pt, *e_src, *band;
  const double *g_w, *g_dtau, *e_w;
  int boff[6];
  int ox, ob, orr, oc;  // LDS offsets (bytes) of x, b, r and the classes
  int ogw, ogc, ogp, ogd;  // LDS offsets of the ghost rows, field-major: 9 weights, 9 columns, point, dtau
  int obl;                 // LDS offset of the band cells
  int nxb;                 // coupled boxes (tables in global memory), slot offsets per colour
  int xso[6];
  XbTab xb;
};
struct SmallCycle {
  int nl;  // fused levels; the last one is the coarsest
  SmallLevel lv[SC_MAXL];
  const double *Ainv;
  const int *map, *bmap;
  int nc, nu1, nu2, lambda, bnd, onv;
  int oxr;  // LDS offset of the coupled boxes' residuals (one colour)
};

__device__ double sc_block_sum(double v) {
  __shared__ double s[SC_T / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0;
  for (int q = 0; q < SC_T / 64; q++) t += s[q];
  return t;
}

// ghost rows of a level staged in LDS, field-major
struct ScRows {
  const double *w, *dt;
  const int *col, *pt;
};

template <typename T>
__device__ void sc_ghosts(const SmallLevel &L, const ScRows &G, T *x, const T *b, double *nv, int lambda) {
  const int ng = L.ng;
  for (int it = 0; it < lambda; it++) {
    for (int r = threadIdx.x; r < ng; r += SC_T) {
      double sum = 0;
#pragma unroll
      for (int z = 0; z < 9; z++) sum += G.w[z * ng + r] * (double)x[G.col[z * ng + r]];
      int k = G.pt[r];
      nv[r] = (double)x[k] + G.dt[r] * ((double)b[k] - sum);
    }
    __syncthreads();
    for (int r = threadIdx.x; r < ng; r += SC_T) x[G.pt[r]] = (T)nv[r];
    __syncthreads();
  }
}

template <typename T>
__device__ void sc_relax(const SmallCycle &P, const SmallLevel &L, const ScRows &G, T *x, const T *b, const uint8_t *cls,
                         double *nv, const int *band, double *xr) {
  const int K = L.N / 5 + 1;
  for (int c = 0; c < 5; c++) {
    for (int t = threadIdx.x; t < K * L.N; t += SC_T) {
      int j = t / K, kk = t - j * K;
      int i = ((c - 2 * j) % 5 + 5) % 5 + 5 * kk;
      if (i < L.N) box_update<T>(L.W, L.K, cls, x, b, i, j);
    }
    __syncthreads();
  }
  if (L.nxb)
    for (int c = 0; c < 5; c++) {
      for (int s = L.xso[c] + threadIdx.x; s < L.xso[c + 1]; s += SC_T)
        xr[s - L.xso[c]] = xb_slot_res<T>(L.W, L.h, L.a, L.d, x, b, L.xb, s);
      __syncthreads();
      for (int s = L.xso[c] + threadIdx.x; s < L.xso[c + 1]; s += SC_T) xb_slot_write<T>(L.xb, x, xr, L.xso[c], s);
      __syncthreads();
    }
  sc_ghosts<T>(L, G, x, b, nv, P.lambda);
  if (P.bnd > 0 && L.nband > 0) {
    for (int q = 0; q < P.bnd; q++) {
      for (int c = 0; c < 5; c++) {
        for (int t = L.boff[c] + threadIdx.x; t < L.boff[c + 1]; t += SC_T) {
          int cell = band[t];
          box_update<T>(L.W, L.K, cls, x, b, cell % L.N, cell / L.N);
        }
        __syncthreads();
      }
      sc_ghosts<T>(L, G, x, b, nv, P.lambda);
    }
  }
  // xi <- mean over internal cells of (div u - g)
  const int WW = L.W * L.W;
  double s = 0;
  for (int t = threadIdx.x; t < L.N * L.N; t += SC_T) {
    int i = t % L.N, j = t / L.N, c = pidx(L.W, i, j);
    if (cls[2 * WW + c] != K_INT) continue;
    s += ((double)x[c + 1] - (double)x[c] + (double)x[WW + c + L.W] - (double)x[WW + c]) / L.h - (double)b[2 * WW + c];
  }
  s = sc_block_sum(s);
  if (threadIdx.x == 0) x[3 * WW] = (T)(s / L.mp);
  __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(SC_T) k_small_cycle(SmallCycle P, T *xg, const T *__restrict__ bg) {
  extern __shared__ unsigned char lds_raw[];
  auto X = [&](int m) { return reinterpret_cast<T *>(lds_raw + P.lv[m].ox); };
  auto B = [&](int m) { return reinterpret_cast<T *>(lds_raw + P.lv[m].ob); };
  auto R = [&](int m) { return reinterpret_cast<T *>(lds_raw + P.lv[m].orr); };
  auto C = [&](int m) { return reinterpret_cast<uint8_t *>(lds_raw + P.lv[m].oc); };
  double *nv = reinterpret_cast<double *>(lds_raw + P.onv);
  double *xr = reinterpret_cast<double *>(lds_raw + P.oxr);
  auto GR = [&](int m) {
    const SmallLevel &L = P.lv[m];
    return ScRows{reinterpret_cast<const double *>(lds_raw + L.ogw), reinterpret_cast<const double *>(lds_raw + L.ogd),
                  reinterpret_cast<const int *>(lds_raw + L.ogc), reinterpret_cast<const int *>(lds_raw + L.ogp)};
  };
  const int tid = threadIdx.x;
  for (int m = 0; m < P.nl; m++) {
    const SmallLevel &L = P.lv[m];
    for (int t = tid; t < 3 * L.W * L.W; t += SC_T) C(m)[t] = L.cls[t];
    if (m < P.nl - 1) {
      double *gw = reinterpret_cast<double *>(lds_raw + L.ogw), *gd = reinterpret_cast<double *>(lds_raw + L.ogd);
      int *gc = reinterpret_cast<int *>(lds_raw + L.ogc), *gp = reinterpret_cast<int *>(lds_raw + L.ogp);
      for (int e = tid; e < 9 * L.ng; e += SC_T) {  // contiguous reads of the row-major tables
        int r = e / 9, z = e - 9 * r;
        gw[z * L.ng + r] = L.g_w[e];
        gc[z * L.ng + r] = L.g_col[e];
      }
      for (int r = tid; r < L.ng; r += SC_T) {
        gp[r] = L.g_pt[r];
        gd[r] = L.g_dtau[r];
      }
      int *bl = reinterpret_cast<int *>(lds_raw + L.obl);
      for (int q = tid; q < L.nband; q += SC_T) bl[q] = L.band[q];
    }
    for (int t = tid; t < L.n; t += SC_T) {
      X(m)[t] = m == 0 ? xg[t] : (T)0;
      B(m)[t] = m == 0 ? bg[t] : (T)0;
    }
  }
  __syncthreads();
  const int bot = P.nl - 1;
  for (int m = 0; m < bot; m++) {
    const SmallLevel &L = P.lv[m], &Cl = P.lv[m + 1];
    const ScRows G = GR(m);
    const int *bl = reinterpret_cast<const int *>(lds_raw + L.obl);
    for (int q = 0; q < P.nu1; q++) sc_relax<T>(P, L, G, X(m), B(m), C(m), nv, bl, xr);
    for (int t = tid; t < 3 * L.W * L.W; t += SC_T) R(m)[t] = (T)resid_point<T>(L.W, L.h, L.a, L.d, C(m), X(m), B(m), t);
    __syncthreads();
    for (int r = tid; r < L.ng; r += SC_T) {
      double sum = 0;
#pragma unroll
      for (int z = 0; z < 9; z++) sum += G.w[z * L.ng + r] * (double)X(m)[G.col[z * L.ng + r]];
      int k = G.pt[r];
      R(m)[k] = (T)((double)B(m)[k] - sum);
    }
    __syncthreads();
    for (int t = tid; t <= 3 * Cl.W * Cl.W; t += SC_T)
      B(m + 1)[t] = (T)restrict_value<T>(L.N, L.W, C(m), R(m), Cl.N, Cl.W, C(m + 1), t);
    __syncthreads();
  }
  // coarsest: x[map[q]] = sum_j Ainv[q][j] b[bmap[j]], one wavefront per row.  Up to 256 unknowns, a wavefront
  // takes eight rows at a time with all 32 loads of a lane issued together (the rows' latencies overlap); the
  // sum of each row is formed in the same order as in the one-row loop below and in k_coarse_apply.
  if (P.nc <= 256) {
    constexpr int CK = 4, RB = 8;
    const int lane = tid & 63, wave = tid >> 6, last = P.nc - 1;
    double bv[CK];
#pragma unroll
    for (int k = 0; k < CK; k++) {
      int r = lane + 64 * k;
      bv[k] = r < P.nc ? (double)B(bot)[P.bmap[r]] : 0.0;  // columns past the end add +0
    }
    for (int q0 = wave; q0 < P.nc; q0 += RB * (SC_T / 64)) {
      double a[RB][CK];
#pragma unroll
      for (int g = 0; g < RB; g++) {
        const int q = min(q0 + g * (SC_T / 64), last);
#pragma unroll
        for (int k = 0; k < CK; k++) a[g][k] = P.Ainv[(size_t)q * P.nc + min(lane + 64 * k, last)];
      }
#pragma unroll
      for (int g = 0; g < RB; g++) {
        double s = 0;
#pragma unroll
        for (int k = 0; k < CK; k++) s += a[g][k] * bv[k];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
        const int q = q0 + g * (SC_T / 64);
        if (lane == 0 && q < P.nc) X(bot)[P.map[q]] = (T)s;
      }
    }
    __syncthreads();
  } else {
    const int lane = tid & 63;
    for (int q = tid >> 6; q < P.nc; q += SC_T / 64) {
      double s = 0;
      for (int r = lane; r < P.nc; r += 64) s += P.Ainv[(size_t)q * P.nc + r] * (double)B(bot)[P.bmap[r]];
      for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
      if (lane == 0) X(bot)[P.map[q]] = (T)s;
    }
    __syncthreads();
  }
  for (int m = bot - 1; m >= 0; m--) {
    const SmallLevel &L = P.lv[m], &Cl = P.lv[m + 1];
    T *xc = X(m + 1);
    for (int e = tid; e < Cl.ne; e += SC_T) {
      if (Cl.e_src[3 * e] < 0) continue;
      xc[Cl.e_pt[e]] = (T)(Cl.e_w[3 * e] * (double)xc[Cl.e_src[3 * e]] + Cl.e_w[3 * e + 1] * (double)xc[Cl.e_src[3 * e + 1]] +
                           Cl.e_w[3 * e + 2] * (double)xc[Cl.e_src[3 * e + 2]]);
    }
    __syncthreads();
    for (int t = tid; t <= 3 * L.W * L.W; t += SC_T) {
      double e = prolong_value(L.N, L.W, C(m), Cl.N, Cl.W, [&](int kc) -> double { return (double)xc[kc]; }, t);
      if (e != 0.0 || t == 3 * L.W * L.W) X(m)[t] = (T)((double)X(m)[t] + e);
    }
    __syncthreads();
    for (int q = 0; q < P.nu2; q++)
      sc_relax<T>(P, L, GR(m), X(m), B(m), C(m), nv, reinterpret_cast<const int *>(lds_raw + L.obl), xr);
  }
  for (int t = tid; t < P.lv[0].n; t += SC_T) xg[t] = X(0)[t];
}

// ---------------------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------------------
template <typename T>
static Vec<T> &vec(Ctx *ctx, int l);
template <>
Vec<double> &vec<double>(Ctx *ctx, int l) {
  return ctx->v64[l];
}
template <>
Vec<float> &vec<float>(Ctx *ctx, int l) {
  return ctx->v32[l];
}

static inline int box_grid(int K, int N) { return ((nblk((long)K * N) + 7) / 8) * 8; }

static inline double coef_a(Ctx *ctx, int l) { return ctx->alpha / (ctx->geo[l].h * ctx->geo[l].h); }

template <typename T>
static void relax_ghosts(Ctx *ctx, int l) {
  Geo &G = ctx->geo[l];
  Vec<T> &V = vec<T>(ctx, l);
  hipStream_t s = ctx->stream;
  if (G.ng && ctx->prm.lambda_ghost > 0) {
    if (G.ng <= 4 * GH_T) {
      k_ghost_sweeps<T><<<1, GH_T, 0, s>>>(G.g_pt, G.g_col, G.g_w, G.g_dtau, G.ng, V.x, V.b, ctx->gtmp,
                                           ctx->prm.lambda_ghost);
    } else {
      for (int it = 0; it < ctx->prm.lambda_ghost; it++) {
        k_ghost_a<T><<<nblk(G.ng), TPB, 0, s>>>(G.g_pt, G.g_col, G.g_w, G.g_dtau, G.ng, V.x, V.b, ctx->gtmp);
        k_ghost_b<T><<<nblk(G.ng), TPB, 0, s>>>(G.g_pt, G.ng, ctx->gtmp, V.x);
      }
    }
  }
}
static void relax_ghost_only(Ctx *ctx, int l) { relax_ghosts<double>(ctx, l); }

// one five-colour sweep x -> y; with events, they take the start and end times of the dispatch
template <typename T>
static void box5_launch(const Geo &G, const BoxK &BK, const Vec<T> &V, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                        const unsigned long long *go = nullptr, double go_lo = 0, double go_hi = 0) {
  const int bt = box5_tile(G.N), nt = (G.N + bt - 1) / bt;
  auto kern = bt == 16 ? k_box5<T, 16> : k_box5<T, 32>;
  const std::uint32_t lds = (std::uint32_t)(bt == 16 ? box5_lds<T, 16>() : box5_lds<T, 32>());
  if (e0)
    hipExtLaunchKernelGGL(kern, dim3(nt * nt), dim3(B5_T), lds, s, e0, e1, 0u, G.N, G.W, BK, (const uint8_t *)G.cls,
                          (const T *)V.x, (const T *)V.b, V.y, go, go_lo, go_hi);
  else
    kern<<<nt * nt, B5_T, lds, s>>>(G.N, G.W, BK, G.cls, V.x, V.b, V.y, go, go_lo, go_hi);
}
template <typename T>
static bool box5_applies(Ctx *ctx, int l) {
  return ctx->box_tiles && vec<T>(ctx, l).y && box5_lds<T, 32>() + 1024 <= ctx->max_lds;
}
// the finest five-colour sweep of a relaxation step (through the launch probe while it has events left); with
// go, the guarded launch of queue_head
static void box5_finest(Ctx *ctx, const BoxK &BK, const unsigned long long *go, double lo, double hi, bool *probed) {
  Geo &G = ctx->geo[0];
  const bool probe = 2 * ctx->probe_n < (int)ctx->probe_ev.size() && ctx->probe_seq % ctx->probe_every == 0;
  if (!ctx->probe_ev.empty()) ctx->probe_seq++;
  if (probe) {  // the events take the start and end times of the dispatch itself
    hipEvent_t e0 = ctx->probe_ev[2 * ctx->probe_n], e1 = ctx->probe_ev[2 * ctx->probe_n + 1];
    ctx->probe_n++;
    box5_launch<double>(G, BK, ctx->v64[0], ctx->stream, e0, e1, go, lo, hi);
  } else {
    box5_launch<double>(G, BK, ctx->v64[0], ctx->stream, nullptr, nullptr, go, lo, hi);
  }
  if (probed) *probed = probe;
}

// the coupled boxes of level l after its box sweep: one workgroup for all five colours where every colour has
// fewer than band_split_min slots, else two launches per colour (residuals, then writes)
template <typename T>
static void xb_relax(Ctx *ctx, int l) {
  Geo &G = ctx->geo[l];
  if (!ctx->prm.ghost_boxes || !G.nxb) return;
  Vec<T> &V = vec<T>(ctx, l);
  hipStream_t s = ctx->stream;
  const double a = coef_a(ctx, l), d = 1.0 + 4.0 * a;
  const XbTab X = xb_tab(G);
  if (G.xb_maxs <= XW_T) {  // at most one slot per thread and colour: one workgroup, no launch per phase
    XbOff so;
    for (int c = 0; c < 6; c++) so.o[c] = G.xb_soff[c];
    k_xb_wg<T><<<1, XW_T, 0, s>>>(so, G.W, G.h, a, d, G.cls, V.x, V.b, X, G.xb_r);
    return;
  }
  for (int c = 0; c < 5; c++) {
    const int lo = G.xb_soff[c], hi = G.xb_soff[c + 1];
    if (hi == lo) continue;
    k_xb_res<T><<<nblk(hi - lo), TPB, 0, s>>>(lo, hi, G.W, G.h, a, d, G.cls, V.x, V.b, X, G.xb_r);
    k_xb_upd<T><<<nblk(hi - lo), TPB, 0, s>>>(lo, hi, V.x, X, G.xb_r);
  }
}

template <typename T>
static void relax(Ctx *ctx, int l) {
  Geo &G = ctx->geo[l];
  Vec<T> &V = vec<T>(ctx, l);
  hipStream_t s = ctx->stream;
  double a = coef_a(ctx, l), d = 1.0 + 4.0 * a;
  const BoxK BK = box_consts(G.h, a, d);
  int K = G.N / 5 + 1;
  if (box5_applies<T>(ctx, l)) {
    if (sizeof(T) == 8 && l == 0) {
      if (ctx->head_queued)  // issued ahead by queue_head (the host has seen that the solve goes on)
        ctx->head_queued = false;
      else
        box5_finest(ctx, BK, nullptr, 0, 0, nullptr);
    } else {
      box5_launch<T>(G, BK, V, s, nullptr, nullptr);
    }
    std::swap(V.x, V.y);
  } else {
    for (int col = 0; col < 5; col++) k_box<T><<<box_grid(K, G.N), TPB, 0, s>>>(G.N, G.W, BK, G.cls, V.x, V.b, col);
  }
  xb_relax<T>(ctx, l);
  const bool band = ctx->prm.bnd_sweeps > 0 && G.nband > 0;
  const size_t lds_bytes = (size_t)G.nreg * sizeof(T);
  const size_t sec_base = ((G.sec_maxreg * sizeof(T) + 7) & ~(size_t)7) + 2 * (size_t)G.sec_maxrow * sizeof(double);
  if (band && G.sec_S > 0 && sec_base + 1024 <= ctx->max_lds) {
    // a large band over angular sectors, one workgroup each, plus the wall rows; then write-back and xi
    SecTabs tb;
    for (int q = 0; q <= G.sec_S; q++) {
      tb.poff[q] = G.sec_poff[q];
      tb.goff[q] = G.sec_goff[q];
      tb.ooff[q] = G.sec_ooff[q];
    }
    for (int q = 0; q <= 5 * G.sec_S; q++) tb.boff[q] = G.sec_boff[q];
    // the ghost-row tables join the region in LDS where they fit (9 weights and dtau, 10 slots per row)
    const size_t lds_g = sec_base + (size_t)G.sec_maxrow * (10 * sizeof(double) + 10 * sizeof(uint16_t));
    const bool gst = lds_g + 1024 <= ctx->max_lds;
    const size_t lds = gst ? lds_g : sec_base;
    const int nwb = (G.nwg + BAND_T - 1) / BAND_T;
    auto kern = gst ? k_band_sec<T, true> : k_band_sec<T, false>;
    kern<<<G.sec_S + nwb, BAND_T, lds, s>>>(
        G.N, G.W, BK, V.x, V.x, V.b, G.sec_S, tb, G.sec_pt, G.sec_bsl, G.sec_bfl, G.sec_bcell, G.sec_bcap, G.sec_gl,
        G.sec_gw, G.sec_gdt, G.sec_gk, G.sec_gcap, G.sec_own_loc, G.sec_own_g, G.sec_out, G.g_pt, G.g_col, G.g_w,
        G.g_dtau, G.wg_rows, G.nwg, ctx->prm.bnd_sweeps, ctx->prm.lambda_ghost);
    const int nfb = 1 + std::min(64, (G.nregw + BAND_T - 1) / BAND_T);
    k_band_sec_fin<T><<<nfb, BAND_T, 0, s>>>(G.reg_pt, G.nregw, G.sec_out, V.x, G.WW, G.h, G.f_code, G.f_loc, G.nf,
                                             ctx->gs_ptr[l], ctx->gs_n[l], G.d_mp);
    return;
  }
  if (band && G.nband >= ctx->band_split_min) {
    // a large band: ghost sweeps and band colours as device-wide launches
    auto sweeps = [&]() {
      const int lam = ctx->prm.lambda_ghost;
      if (lam >= 2 && G.colr_ok) {  // one launch per sweep: the sweeps between go through two row buffers
        double *buf[2] = {ctx->gtmp, ctx->gtmp2};
        for (int it = 0; it < lam; it++) {
          const double *prev = it == 0 ? nullptr : buf[(it - 1) & 1];
          double *next = it == lam - 1 ? nullptr : buf[it & 1];
          k_ghost_sweep2<T><<<nblk(G.ng), TPB, 0, s>>>(G.g_pt, G.g_col, G.g_colr, G.g_w, G.g_dtau, G.ng, V.x, V.b, prev,
                                                     next);
        }
        return;
      }
      for (int it = 0; it < lam; it++) {
        k_ghost_a<T><<<nblk(G.ng), TPB, 0, s>>>(G.g_pt, G.g_col, G.g_w, G.g_dtau, G.ng, V.x, V.b, ctx->gtmp);
        k_ghost_b<T><<<nblk(G.ng), TPB, 0, s>>>(G.g_pt, G.ng, ctx->gtmp, V.x);
      }
    };
    if (G.ng) sweeps();
    for (int q = 0; q < ctx->prm.bnd_sweeps; q++) {
      for (int c = 0; c < 5; c++) {
        int lo = G.hband_off[c], hi = G.hband_off[c + 1];
        if (hi > lo) k_box_list<T><<<nblk(hi - lo), TPB, 0, s>>>(G.N, G.W, BK, G.cls, V.x, V.b, G.band, lo, hi);
      }
      if (G.ng) sweeps();
    }
    k_xi_faces<T><<<1, BAND_T, 0, s>>>(G.WW, G.h, V.x, G.f_code, G.nf, ctx->gs_ptr[l], ctx->gs_n[l], G.d_mp);
    return;
  }
  const size_t with_nv = band_lds_bytes(1, lds_bytes, G.nbg, G.nband);
  if (band && G.lds_ok && with_nv + 1024 <= ctx->max_lds) {
    // wall ghosts, body ghosts, band boxes and xi in one workgroup; the most staging that fits in LDS (16-bit
    // slot numbers need fewer than 65536 region points)
    int nwb = (G.nwg + BAND_T - 1) / BAND_T;
    BandOff bo;
    for (int c = 0; c < 6; c++) bo.o[c] = G.hband_off[c];
    int mode = G.nreg > G.nregw ? 1 : 0;
    if (mode == 1 && G.nreg < 65536) {
      if (band_lds_bytes(3, lds_bytes, G.nbg, G.nband) + 1024 <= ctx->max_lds)
        mode = 3;
      else if (band_lds_bytes(2, lds_bytes, G.nbg, G.nband) + 1024 <= ctx->max_lds)
        mode = 2;
    }
    auto kern = mode == 3 ? k_band_lds<T, 3> : mode == 2 ? k_band_lds<T, 2> : mode == 1 ? k_band_lds<T, 1> : k_band_lds<T, 0>;
    kern<<<1 + nwb, BAND_T, band_lds_bytes(mode, lds_bytes, G.nbg, G.nband), s>>>(G.N, G.W, BK, V.x, V.b, bo, G.bbox, G.bcap, G.reg_pt, G.nreg, G.nregw, G.bg_k,
                                          G.bg_loc, G.bg_w, G.bg_dt, G.nbg, G.gcap, G.g_pt, G.g_col, G.g_w, G.g_dtau,
                                          G.wg_rows, G.nwg, ctx->prm.bnd_sweeps, ctx->prm.lambda_ghost, G.f_code, G.f_loc,
                                          G.nf, ctx->gs_ptr[l], ctx->gs_n[l], G.d_mp);
    return;
  }
  if (!band && G.ng <= 2 * BAND_T) {
    // the ghost sweeps and xi in one workgroup (a few rows per thread)
    // one row per thread: the sweeps run from registers and LDS (below 128 registers); two: from global memory
    if (G.ng <= BAND_T)
      k_ghost_xi<T, 1><<<1, BAND_T, 0, s>>>(G.g_pt, G.g_col, G.colr_ok ? G.g_colr : nullptr,
                                             G.colr_ok ? G.g_colrT : nullptr, G.colr_ok ? G.g_wT : nullptr, G.g_w,
                                             G.g_dtau, G.ng,
                                             V.x, V.b, ctx->prm.lambda_ghost, G.WW, G.h, G.cls, G.g_rowof, G.f_code,
                                             G.nf, ctx->gs_ptr[l], ctx->gs_n[l], G.d_mp);
    else if (G.colr_ok)
      k_ghost_xi2<T><<<1, BAND_T, 0, s>>>(G.g_pt, G.g_colrT, G.g_wT, G.g_dtau, G.ng, V.x, V.b, ctx->prm.lambda_ghost,
                                          G.WW, G.h, G.cls, G.g_rowof, G.f_code, G.nf, ctx->gs_ptr[l], ctx->gs_n[l],
                                          G.d_mp);
    else
      k_ghost_xi<T, 2><<<1, BAND_T, 0, s>>>(G.g_pt, G.g_col, nullptr, nullptr, nullptr, G.g_w, G.g_dtau, G.ng, V.x, V.b,
                                             ctx->prm.lambda_ghost, G.WW, G.h, G.cls, G.g_rowof, G.f_code, G.nf,
                                             ctx->gs_ptr[l], ctx->gs_n[l], G.d_mp);
    return;
  }
  if (!band && G.ng) {
    // many ghost rows: one device-wide launch per sweep (the sweeps between go through two row buffers), then xi
    // (some of its faces are ghost points the last sweep writes)
    const int lam = ctx->prm.lambda_ghost;
    if (G.colr_ok) {
      double *buf[2] = {ctx->gtmp, ctx->gtmp2};
      for (int it = 0; it < lam; it++) {
        const double *prev = it == 0 ? nullptr : buf[(it - 1) & 1];
        double *next = it == lam - 1 ? nullptr : buf[it & 1];
        k_ghost_sweep2<T><<<nblk(G.ng), TPB, 0, s>>>(G.g_pt, G.g_col, G.g_colr, G.g_w, G.g_dtau, G.ng, V.x, V.b, prev,
                                                   next);
      }
    } else {
      relax_ghosts<T>(ctx, l);
    }
    k_xi_faces<T><<<1, BAND_T, 0, s>>>(G.WW, G.h, V.x, G.f_code, G.nf, ctx->gs_ptr[l], ctx->gs_n[l], G.d_mp);
    return;
  }
  if (band && G.ng <= 4 * GH_T) {
    // ghost sweeps and the band sweeps in one workgroup
    k_band_sweeps<T><<<1, BAND_T, 0, s>>>(G.N, G.W, BK, G.cls, V.x, V.b, G.band, G.d_band_off, G.g_pt, G.g_col,
                                          G.g_w, G.g_dtau, G.ng, ctx->gtmp, ctx->prm.bnd_sweeps, ctx->prm.lambda_ghost, 1);
  } else {
    relax_ghosts<T>(ctx, l);
    if (band)
      k_band_sweeps<T><<<1, BAND_T, 0, s>>>(G.N, G.W, BK, G.cls, V.x, V.b, G.band, G.d_band_off, G.g_pt, G.g_col,
                                            G.g_w, G.g_dtau, G.ng, ctx->gtmp, ctx->prm.bnd_sweeps, ctx->prm.lambda_ghost, 0);
  }
  k_xi_faces<T><<<1, BAND_T, 0, s>>>(G.WW, G.h, V.x, G.f_code, G.nf, ctx->gs_ptr[l], ctx->gs_n[l], G.d_mp);
}

// sum of the continuity right-hand sides of level l (read by the xi updates of its relaxation steps)
template <typename T>
static void gsum(Ctx *ctx, int l) {
  Geo &G = ctx->geo[l];
  ctx->gs_ptr[l] = ctx->d_lev + l;
  ctx->gs_n[l] = 1;
  k_gsum<T><<<rd_blocks(G.WW), RD_T, 0, ctx->stream>>>(G.W, G.h, G.cls, vec<T>(ctx, l).x, vec<T>(ctx, l).b, ctx->d_red, ctx->d_ticket,
                                         ctx->d_lev + l);
}

template <typename T>
static void residual(Ctx *ctx, int l, unsigned long long *rmax, unsigned long long *hmax = nullptr, bool store = true) {
  Geo &G = ctx->geo[l];
  Vec<T> &V = vec<T>(ctx, l);
  hipStream_t s = ctx->stream;
  double a = coef_a(ctx, l), d = 1.0 + 4.0 * a;
  if (rmax) {
    // two partials per block in d_red (2 (nblk(3 (N+2)^2) + nblk(gcap)) + 16 slots)
    const int nbp = nblk(3L * G.WW), nb = nbp + (G.ng ? nblk(G.ng) : 0);
    k_resid_pts_norm<T><<<nb, TPB, 0, s>>>(G.W, G.h, a, d, G.cls, V.x, V.b, V.r, nbp, G.g_pt, G.g_col, G.g_w, G.ng,
                                           ctx->d_red, store ? 1 : 0);
    k_resid_mean_row<T><<<1, RM_T, 0, s>>>(ctx->d_red, nb, G.d_mp, V.r + 3L * G.WW, rmax, hmax);
  } else {
    k_resid_pts<T><<<nblk(3L * G.WW), TPB, 0, s>>>(G.N, G.W, G.h, a, d, G.cls, V.x, V.b, V.r, nullptr);
    if (G.ng) k_resid_ghost<T><<<nblk(G.ng), TPB, 0, s>>>(G.g_pt, G.g_col, G.g_w, G.ng, V.x, V.b, V.r, nullptr);
  }

}

template <typename T>
static void coarse_solve(Ctx *ctx) {
  int l = ctx->L - 1;
  Vec<T> &V = vec<T>(ctx, l);
  k_coarse_apply<T><<<ctx->nc, 64, 0, ctx->stream>>>(ctx->c_inv, ctx->c_map, ctx->c_bmap, ctx->nc, V.b, V.x);
}

// the V cycle from level l down in one workgroup, if those levels fit in LDS (gamma = 1 only)
template <typename T>
static size_t small_cycle_setup(Ctx *ctx, int l, SmallCycle &P) {
  if (ctx->prm.gamma != 1 || ctx->nc <= 0 || !ctx->c_ok) return 0;
  P.nl = ctx->L - l;
  if (P.nl < 2 || P.nl > SC_MAXL) return 0;
  size_t off = 0;
  int maxng = 0, maxxs = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 15) & ~(size_t)15;
    return (int)o;
  };
  for (int m = 0; m < P.nl; m++) {
    Geo &G = ctx->geo[l + m];
    SmallLevel &S = P.lv[m];
    S.N = G.N;
    S.W = G.W;
    S.n = G.n;
    S.ng = G.ng;
    S.ne = G.ne;
    S.nband = (ctx->prm.bnd_sweeps > 0) ? G.nband : 0;
    S.mp = G.mp;
    S.h = G.h;
    S.a = ctx->alpha / (G.h * G.h);
    S.d = 1.0 + 4.0 * S.a;
    S.K = box_consts(S.h, S.a, S.d);
    S.cls = G.cls;
    S.g_pt = G.g_pt;
    S.g_col = G.g_col;
    S.g_w = G.g_w;
    S.g_dtau = G.g_dtau;
    S.e_pt = G.e_pt;
    S.e_src = G.e_src;
    S.e_w = G.e_w;
    S.band = G.band;
    for (int c = 0; c < 6; c++) S.boff[c] = G.hband_off[c];
    const bool bottom = m == P.nl - 1;
    S.ox = take((size_t)G.n * sizeof(T));
    S.ob = take((size_t)G.n * sizeof(T));
    S.orr = bottom ? 0 : take((size_t)G.n * sizeof(T));
    S.oc = take((size_t)3 * G.WW);
    S.ogw = bottom ? 0 : take((size_t)9 * G.ng * sizeof(double));
    S.ogd = bottom ? 0 : take((size_t)G.ng * sizeof(double));
    S.ogc = bottom ? 0 : take((size_t)9 * G.ng * sizeof(int));
    S.ogp = bottom ? 0 : take((size_t)G.ng * sizeof(int));
    S.obl = bottom ? 0 : take((size_t)S.nband * sizeof(int));
    S.nxb = (!bottom && ctx->prm.ghost_boxes) ? G.nxb : 0;
    for (int c = 0; c < 6; c++) S.xso[c] = G.xb_soff[c];
    S.xb = xb_tab(G);
    if (!bottom) maxng = std::max(maxng, G.ng);
    if (S.nxb) maxxs = std::max(maxxs, G.xb_maxs);
  }
  P.onv = take((size_t)maxng * sizeof(double));
  P.oxr = take((size_t)std::max(1, maxxs) * sizeof(double));
  if (off + 2048 > ctx->max_lds) return 0;
  P.Ainv = ctx->c_inv;
  P.map = ctx->c_map;
  P.bmap = ctx->c_bmap;
  P.nc = ctx->nc;
  P.nu1 = ctx->prm.nu1;
  P.nu2 = ctx->prm.nu2;
  P.lambda = ctx->prm.lambda_ghost;
  P.bnd = ctx->prm.bnd_sweeps;
  return off;
}

template <typename T>
static void cycle(Ctx *ctx, int l) {
  if (l == ctx->L - 1) {
    coarse_solve<T>(ctx);
    return;
  }
  if (ctx->small_cycles && ctx->geo[l].N <= 32) {
    SmallCycle P{};
    size_t lds = small_cycle_setup<T>(ctx, l, P);
    if (lds) {
      Vec<T> &V = vec<T>(ctx, l);
      k_small_cycle<T><<<1, SC_T, lds, ctx->stream>>>(P, V.x, V.b);
      return;
    }
  }
  Geo &F = ctx->geo[l], &C = ctx->geo[l + 1];
  Vec<T> &VF = vec<T>(ctx, l), &VC = vec<T>(ctx, l + 1);
  hipStream_t s = ctx->stream;
  for (int q = 0; q < ctx->prm.nu1; q++) relax<T>(ctx, l);
  {
    const double a = coef_a(ctx, l), d = 1.0 + 4.0 * a;
    k_resid_restrict<T><<<nblk(3L * C.WW + 1), TPB, 0, s>>>(F.N, F.W, F.h, a, d, F.cls, VF.x, VF.b, F.g_rowof, F.g_col,
                                                          F.g_w, C.N, C.W, C.cls, VC.b, VC.x, ctx->d_gpart + C.gp_off);
    ctx->gs_ptr[l + 1] = ctx->d_gpart + C.gp_off;
    ctx->gs_n[l + 1] = C.gp_n;
  }
  int reps = (l + 1 == ctx->L - 1) ? 1 : ctx->prm.gamma;
  for (int q = 0; q < reps; q++) cycle<T>(ctx, l + 1);
  const bool ext_inline = (long)F.N * F.N <= PROLONG_EXT_INLINE_MAX;
  if (C.ne && !ext_inline) k_ext_fill<T><<<nblk(C.ne), TPB, 0, s>>>(C.e_pt, C.e_src, C.e_w, C.ne, VC.x);
  k_prolong<T, T><<<nblk(3L * F.WW + 1), TPB, 0, s>>>(F.N, F.W, F.cls, VF.x, C.N, C.W, VC.x, C.cls,
                                                     C.ne && ext_inline ? C.e_rowof : nullptr, C.e_src, C.e_w);
  for (int q = 0; q < ctx->prm.nu2; q++) relax<T>(ctx, l);
}

template <typename T>
static void mean_project(Ctx *ctx) {
  Geo &G = ctx->geo[0];
  Vec<T> &V = vec<T>(ctx, 0);
  const int np = rd_blocks(G.WW);
  k_pmean<T><<<np, RD_T, 0, ctx->stream>>>(G.W, G.cls, V.x, ctx->d_red);
  k_pshift<T><<<nblk(G.WW), TPB, 0, ctx->stream>>>(G.W, G.cls, V.x, ctx->d_red, np, G.d_mp, ctx->d_scal);
}

// The finest residual norm reaches the host through pinned memory: norm_launch clears the host slot to a value no
// norm has (the bits of a negative NaN; the kernel stores |r| as bits) and issues the residual kernels, whose last
// one also stores the norm there; wait_norm polls the slot, and now and then the stream, so that a failed launch
// ends the wait (once the stream is idle the store has landed; else the device copy is read).
constexpr unsigned long long NORM_PENDING = ~0ull;
// algorithmic bytes of one cycle from the finest level (the compulsory traffic model of the kernels: per cell of a
// level, 65 B per relaxation step in FP64 storage (33 in FP32), 53 B (27) for the residual with the restriction and
// the prolongation; a level below is visited gamma times as often on a quarter of the cells) and of one residual
// norm (41 B per cell)
double cycle_bytes(const Ctx *ctx, bool fp32) {
  const double step = fp32 ? 33.0 : 65.0, tr = fp32 ? 27.0 : 53.0;
  double b = 0, wgt = 1;
  for (int l = 0; l + 1 < ctx->L; l++) {
    const double cells = (double)ctx->geo[l].N * ctx->geo[l].N;
    b += wgt * cells * ((ctx->prm.nu1 + ctx->prm.nu2) * step + tr);
    wgt *= (l + 2 == ctx->L) ? 1.0 : (double)ctx->prm.gamma;
  }
  return b;
}
static double norm_bytes(const Ctx *ctx) { return 41.0 * ctx->geo[0].N * ctx->geo[0].N; }

static void norm_launch(Ctx *ctx, bool store = true) {
  __atomic_store_n(ctx->h_rmax, NORM_PENDING, __ATOMIC_RELEASE);
  residual<double>(ctx, 0, (unsigned long long *)(ctx->d_scal + 1), ctx->h_rmax, store);
}
static gp_status wait_norm(Ctx *ctx, double *out) {
  unsigned long long v = NORM_PENDING;
  for (long it = 1;; it++) {
    v = __atomic_load_n(ctx->h_rmax, __ATOMIC_ACQUIRE);
    if (v != NORM_PENDING) break;
    if ((it & 255) == 0) {
      const hipError_t e = hipStreamQuery(ctx->stream);
      if (e == hipSuccess) {
        v = __atomic_load_n(ctx->h_rmax, __ATOMIC_ACQUIRE);
        if (v == NORM_PENDING)
          GP_HIP(hipMemcpy(&v, ctx->d_scal + 1, sizeof(v), hipMemcpyDeviceToHost));
        break;
      }
      if (e != hipErrorNotReady) GP_HIP(e);
    }
  }
  std::memcpy(out, &v, sizeof(double));
  return GP_OK;
}
static gp_status resnorm64(Ctx *ctx, double *out) {
  norm_launch(ctx);
  GP_HIP(hipGetLastError());
  return wait_norm(ctx, out);
}

static gp_status bnorm64(Ctx *ctx, double *out) {
  // max |b| over the finest vector (entries without an equation are zero)
  Geo &G = ctx->geo[0];
  unsigned long long *m = (unsigned long long *)(ctx->d_scal + 3);
  k_fill<unsigned long long><<<1, 1, 0, ctx->stream>>>(m, 1, 0ull);
  k_absmax<double><<<std::min(1024, nblk(G.n)), TPB, 0, ctx->stream>>>(ctx->v64[0].b, G.n, m);
  GP_HIP(hipGetLastError());
  unsigned long long hv = 0;
  GP_HIP(hipMemcpyAsync(&hv, m, sizeof(hv), hipMemcpyDeviceToHost, ctx->stream));
  GP_HIP(hipStreamSynchronize(ctx->stream));
  std::memcpy(out, &hv, sizeof(double));
  return GP_OK;
}

gp_status set_wall_dirichlet(Ctx *ctx) {
  Geo &G = ctx->geo[0];
  k_set_walld<double><<<nblk(3L * G.WW), TPB, 0, ctx->stream>>>(3 * G.WW, G.cls, ctx->v64[0].x, ctx->v64[0].b);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

gp_status relax64(Ctx *ctx, int level, int steps) {
  gp_status st = ensure_xb(ctx);
  if (st) return st;
  gsum<double>(ctx, level);
  for (int q = 0; q < steps; q++) relax<double>(ctx, level);
  GP_HIP(hipGetLastError());
  GP_HIP(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}

gp_status time_kernel(Ctx *ctx, int which, int l, int reps, double *avg_us) {
  Geo &G = ctx->geo[l];
  Vec<double> &V = ctx->v64[l];
  hipStream_t s = ctx->stream;
  double a = coef_a(ctx, l), d = 1.0 + 4.0 * a;
  hipEvent_t e0, e1;
  GP_HIP(hipEventCreate(&e0));
  GP_HIP(hipEventCreate(&e1));
  int K = G.N / 5 + 1;
  int launches = 0;
  GP_HIP(hipEventRecord(e0, s));
  for (int q = 0; q < reps; q++) {
    if (which == 0) {
      for (int col = 0; col < 5; col++)
        k_box<double><<<box_grid(K, G.N), TPB, 0, s>>>(G.N, G.W, box_consts(G.h, a, d), G.cls, V.x, V.b, col);
      launches += 5;
    } else if (which == 1) {
      k_resid_pts<double><<<nblk(3L * G.WW), TPB, 0, s>>>(G.N, G.W, G.h, a, d, G.cls, V.x, V.b, V.r, nullptr);
      launches++;
    } else if (which == 2 && l + 1 < ctx->L) {
      Geo &C = ctx->geo[l + 1];
      k_restrict<double, double><<<nblk(3L * C.WW + 1), TPB, 0, s>>>(G.N, G.W, G.cls, V.r, C.N, C.W, C.cls, ctx->v64[l + 1].b,
                                                                     nullptr);
      launches++;
    } else if (which == 3 && l + 1 < ctx->L) {
      Geo &C = ctx->geo[l + 1];
      k_fill<double><<<nblk(C.n), TPB, 0, s>>>(ctx->v64[l + 1].x, C.n, 0.0);  // zero correction: x unchanged
      k_prolong<double, double><<<nblk(3L * G.WW + 1), TPB, 0, s>>>(G.N, G.W, G.cls, V.x, C.N, C.W, ctx->v64[l + 1].x,
                                                                    C.cls, C.ne ? C.e_rowof : nullptr, C.e_src, C.e_w);
      launches++;
    } else if (which == 4) {
      relax_ghost_only(ctx, l);
      launches++;
    } else if (which == 5 && V.y && box5_lds<double, 32>() + 1024 <= ctx->max_lds) {
      box5_launch<double>(G, box_consts(G.h, a, d), V, s, nullptr, nullptr);
      std::swap(V.x, V.y);
      launches++;
    } else {
      return GP_EINVAL;
    }
  }
  GP_HIP(hipEventRecord(e1, s));
  GP_HIP(hipEventSynchronize(e1));
  float ms = 0;
  GP_HIP(hipEventElapsedTime(&ms, e0, e1));
  GP_HIP(hipEventDestroy(e0));
  GP_HIP(hipEventDestroy(e1));
  *avg_us = launches ? 1000.0 * ms / launches : 0.0;
  return GP_OK;
}

gp_status probe_start(Ctx *ctx, int max_launches, int every) {
  double dummy;
  int n;
  if (!ctx->probe_ev.empty()) probe_stop(ctx, &dummy, &n);
  ctx->probe_ev.assign(2 * (size_t)max_launches, nullptr);
  ctx->probe_n = 0;
  ctx->probe_every = every;
  ctx->probe_seq = 0;
  for (auto &e : ctx->probe_ev) GP_HIP(hipEventCreate(&e));
  return GP_OK;
}

gp_status probe_stop(Ctx *ctx, double *avg_us, int *launches) {
  double total = 0;
  gp_status st = GP_OK;
  if (ctx->probe_n > 0 && hipEventSynchronize(ctx->probe_ev[2 * ctx->probe_n - 1]) != hipSuccess) st = GP_EHIP;
  for (int q = 0; q < ctx->probe_n && st == GP_OK; q++) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, ctx->probe_ev[2 * q], ctx->probe_ev[2 * q + 1]) != hipSuccess) st = GP_EHIP;
    total += ms;
  }
  *launches = ctx->probe_n;
  *avg_us = ctx->probe_n ? 1000.0 * total / ctx->probe_n : 0.0;
  for (auto &e : ctx->probe_ev)
    if (e) (void)hipEventDestroy(e);
  ctx->probe_ev.clear();
  ctx->probe_n = 0;
  if (st) ctx->hip_err = "event timing of the probed launches failed";
  return st;
}

gp_status residual64(Ctx *ctx, int level, double *res_inf) {
  (void)level;
  return resnorm64(ctx, res_inf);
}

gp_status mg_cycle64(Ctx *ctx, double *res_inf) {
  gp_status st = set_wall_dirichlet(ctx);
  if (st) return st;
  if ((st = ensure_xb(ctx))) return st;
  gsum<double>(ctx, 0);
  cycle<double>(ctx, 0);
  mean_project<double>(ctx);
  GP_HIP(hipGetLastError());
  if (res_inf) return resnorm64(ctx, res_inf);
  GP_HIP(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}

// ---------------------------------------------------------------------------------------------------------
// mixed precision: FP64 iterative refinement around FP32 cycles
//   r = b - M x (FP64), solve M e = r approximately by k FP32 cycles (FP64 arithmetic inside the kernels,
//   FP64 ghost coefficients, FP64 reductions and coarsest solve), x += e, p <- p - mean(p) (FP64)
// ---------------------------------------------------------------------------------------------------------
__global__ void k_cast_rhs(const double *__restrict__ r, float *__restrict__ b, long n) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < n) b[t] = (t == n - 1) ? 0.0f : (float)r[t];  // the mean row is restored by the FP64 projection
}
__global__ void k_add_correction(const uint8_t *__restrict__ cls, long n, const float *__restrict__ e, double *__restrict__ x) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  if (t == n - 1) {
    x[t] += (double)e[t];
    return;
  }
  uint8_t c = cls[t];
  if (c == K_INT || c == K_GHOST || c == K_GHOSTX || c == K_WALLG) x[t] += (double)e[t];
}

static gp_status ensure_fp32(Ctx *ctx) {
  for (int l = 0; l < ctx->L; l++) {
    Vec<float> &V = ctx->v32[l];
    if (V.x) continue;
    size_t n = ctx->geo[l].n;
    GP_HIP(hipMalloc((void **)&V.x, n * sizeof(float)));
    GP_HIP(hipMalloc((void **)&V.b, n * sizeof(float)));
    GP_HIP(hipMalloc((void **)&V.r, n * sizeof(float)));
    if (ctx->geo[l].N >= 64) GP_HIP(hipMalloc((void **)&V.y, n * sizeof(float)));
    GP_HIP(hipMemsetAsync(V.x, 0, n * sizeof(float), ctx->stream));
    GP_HIP(hipMemsetAsync(V.b, 0, n * sizeof(float), ctx->stream));
    GP_HIP(hipMemsetAsync(V.r, 0, n * sizeof(float), ctx->stream));
  }
  return GP_OK;
}

// one refinement step; the FP64 residual of the current x must be in v64[0].r
static void refine_step(Ctx *ctx, int inner) {
  Geo &G = ctx->geo[0];
  hipStream_t s = ctx->stream;
  Vec<float> &E = ctx->v32[0];
  k_cast_rhs<<<nblk(G.n), TPB, 0, s>>>(ctx->v64[0].r, E.b, G.n);
  k_fill<float><<<nblk(G.n), TPB, 0, s>>>(E.x, G.n, 0.0f);
  gsum<float>(ctx, 0);  // b of the inner cycles is fixed for the whole refinement step
  for (int q = 0; q < inner; q++) {
    cycle<float>(ctx, 0);
    mean_project<float>(ctx);
  }
  k_add_correction<<<nblk(G.n), TPB, 0, s>>>(G.cls, G.n, E.x, ctx->v64[0].x);
  mean_project<double>(ctx);
}

// The launches of one solver iteration (an FP64 cycle and the mean projection, or one refinement step) followed
// by the residual norm into d_scal[1], captured as a graph: most launches of a cycle are a few microseconds
// long, shorter than the host needs to issue them one by one.  Captured at the start of every solve (the
// geometry, alpha and buffers may have changed since the last one); the executable graph of the previous solve
// is updated in place when the launch sequence has the same shape, else instantiated anew.
static void iteration_launches(Ctx *ctx, int precision) {
  if (precision == GP_FP64) {
    cycle<double>(ctx, 0);
    mean_project<double>(ctx);
  } else {
    refine_step(ctx, ctx->prm.mixed_inner_cycles);
  }
  residual<double>(ctx, 0, (unsigned long long *)(ctx->d_scal + 1), ctx->h_rmax, precision != GP_FP64);
}

static gp_status capture_iteration(Ctx *ctx, int precision) {
  hipStream_t s = ctx->stream;
  hipGraphExec_t &ex = ctx->g_iter[precision == GP_FP64 ? 0 : 1];
  hipGraph_t g = nullptr;
  GP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  iteration_launches(ctx, precision);
  hipError_t el = hipGetLastError();
  hipError_t ec = hipStreamEndCapture(s, &g);
  if (el != hipSuccess || ec != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    ctx->hip_err = std::string("capture of a solver iteration: ") + hipGetErrorString(el != hipSuccess ? el : ec);
    return GP_EHIP;
  }
  if (ex) {
    hipGraphNode_t bad = nullptr;
    hipGraphExecUpdateResult ur = hipGraphExecUpdateError;
    if (hipGraphExecUpdate(ex, g, &bad, &ur) != hipSuccess || ur != hipGraphExecUpdateSuccess) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(ex);
      ex = nullptr;
    }
  }
  hipError_t ei = ex ? hipSuccess : hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    ex = nullptr;
    ctx->hip_err = std::string("hipGraphInstantiate: ") + hipGetErrorString(ei);
    return GP_EHIP;
  }
  return GP_OK;
}

// The first box sweep of the next FP64 cycle, queued behind the residual norm of this one before the host has
// read it: its workgroups return at once unless lo < norm <= hi, the condition under which the solve goes on, so
// the device need not wait for the host's test and its next launches.  relax() takes it as its first sweep when
// the host goes on; when the solve stops, drop_head() forgets it (and its probe events).
static void queue_head(Ctx *ctx, double lo, double hi) {
  Geo &G = ctx->geo[0];
  const double a = coef_a(ctx, 0), d = 1.0 + 4.0 * a;
  box5_finest(ctx, box_consts(G.h, a, d), (const unsigned long long *)(ctx->d_scal + 1), lo, hi, &ctx->head_probe);
  ctx->head_queued = true;
}
static void drop_head(Ctx *ctx) {
  if (!ctx->head_queued) return;
  ctx->head_queued = false;
  if (!ctx->probe_ev.empty()) ctx->probe_seq--;
  if (ctx->head_probe) ctx->probe_n--;
}

// ---------------------------------------------------------------------------------------------------------
// generalized conjugate residual iteration (GCR) around the cycle.  Per iteration: z = B' r (the preconditioner),
// q = M z, q and z orthogonalised against the stored images Q_i = M Z_i and directions Z_i (classical Gram-Schmidt,
// one pass: q -= sum (Q_i . q / |Q_i|^2) Q_i, z likewise with Z_i), stored as Q_k, Z_k, then x += (r . Q_k / |Q_k|^2)
// Z_k, r -= (r . Q_k / |Q_k|^2) Q_k.  The vectors are the finest level's full unknown vectors (3 W^2 + 1 doubles,
// zero where no equation); every reduction runs over GR_B fixed blocks summed in block order, so the iteration is
// deterministic.  The image is formed as -M z (the residual kernel with a zero right-hand side), so the stored
// images are -M Z_i; the signs cancel in every coefficient.
// ---------------------------------------------------------------------------------------------------------
constexpr int GR_B = 1024, GR_T = 256, KR_MAX = 64;

// partials of the k dot products (Q_i . qn), i < k: part[i * GR_B + block]
__global__ void __launch_bounds__(GR_T) k_gcr_dots(const double *__restrict__ Q, long n, int k, const double *__restrict__ qn,
                                                   double *part) {
  __shared__ double sm[GR_T];
  double acc[KR_MAX / 4];
  for (int i0 = 0; i0 < k; i0 += KR_MAX / 4) {
    const int kk = min(KR_MAX / 4, k - i0);
    for (int i = 0; i < KR_MAX / 4; i++) acc[i] = 0;
    for (long e = blockIdx.x * (long)GR_T + threadIdx.x; e < n; e += (long)GR_B * GR_T) {
      const double q = qn[e];
#pragma unroll
      for (int i = 0; i < KR_MAX / 4; i++)
        if (i < kk) acc[i] += Q[(size_t)(i0 + i) * n + e] * q;
    }
    for (int i = 0; i < kk; i++) {
      sm[threadIdx.x] = acc[i];
      __syncthreads();
      for (int o = GR_T / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
        __syncthreads();
      }
      if (threadIdx.x == 0) part[(size_t)(i0 + i) * GR_B + blockIdx.x] = sm[0];
      __syncthreads();
    }
  }
}
// out[i] = (sum_b part[i * GR_B + b]) / div[i] for i < cnt (div may be null: no division); with nu2 set, also
// nu2[0] = out[0] (the squared norm of the new image, kept for the later projections)
__global__ void __launch_bounds__(GR_B) k_gcr_sum(const double *__restrict__ part, int cnt, const double *__restrict__ div,
                                                  double *out, double *nu2) {
  __shared__ double sm[GR_B];
  for (int i = 0; i < cnt; i++) {
    sm[threadIdx.x] = part[(size_t)i * GR_B + threadIdx.x];
    __syncthreads();
    for (int o = GR_B / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double v = div ? sm[0] / div[i] : sm[0];
      out[i] = v;
      if (nu2 && i == 0) *nu2 = v;
    }
    __syncthreads();
  }
}
// Gram-Schmidt step into the k-th slots: Qk = qn - sum_i b_i Q_i, Zk = z - sum_i b_i Z_i (b_i = Q_i . qn / |Q_i|^2),
// and the partials of |Qk|^2 and r . Qk into part[block], part[GR_B + block]
__global__ void __launch_bounds__(GR_T) k_gcr_orth(const double *__restrict__ Q, const double *__restrict__ Z, long n,
                                                   int k, const double *__restrict__ beta, const double *__restrict__ qn,
                                                   const double *__restrict__ z, const double *__restrict__ r, double *Qk,
                                                   double *Zk, double *part) {
  __shared__ double sm[GR_T];
  double s2 = 0, sr = 0;
  for (long e = blockIdx.x * (long)GR_T + threadIdx.x; e < n; e += (long)GR_B * GR_T) {
    double q = qn[e], zz = z[e];
    for (int i = 0; i < k; i++) {
      const double b = beta[i];
      q -= b * Q[(size_t)i * n + e];
      zz -= b * Z[(size_t)i * n + e];
    }
    Qk[e] = q;
    Zk[e] = zz;
    s2 += q * q;
    sr += r[e] * q;
  }
  for (int w = 0; w < 2; w++) {
    sm[threadIdx.x] = w == 0 ? s2 : sr;
    __syncthreads();
    for (int o = GR_T / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)w * GR_B + blockIdx.x] = sm[0];
    __syncthreads();
  }
}
// the step with g = (r . Qk) / |Qk|^2 (sc[0] = |Qk|^2, sc[1] = r . Qk): the image of Zk is -Qk, so the coefficient
// of the direction is -g: x -= g Zk, r -= g Qk; block maxima of |r| into part[block]
__global__ void __launch_bounds__(GR_T) k_gcr_step(long n, const double *__restrict__ sc, const double *__restrict__ Qk,
                                                   const double *__restrict__ Zk, double *x, double *r, double *part) {
  __shared__ double sm[GR_T];
  const double nu2 = sc[0], g = nu2 > 0 ? sc[1] / nu2 : 0.0;
  double m = 0;
  for (long e = blockIdx.x * (long)GR_T + threadIdx.x; e < n; e += (long)GR_B * GR_T) {
    x[e] -= g * Zk[e];
    const double rr = r[e] - g * Qk[e];
    r[e] = rr;
    const double a = fabs(rr);
    m = (a > m || a != a) ? a : m;
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int o = GR_T / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double v = sm[threadIdx.x + o];
      if (v > sm[threadIdx.x] || v != v) sm[threadIdx.x] = v;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}
// max of the block maxima into *dmax (as bits) and *hmax (pinned host memory)
__global__ void __launch_bounds__(GR_B) k_gcr_max(const double *__restrict__ part, unsigned long long *dmax,
                                                  unsigned long long *hmax) {
  __shared__ double sm[GR_B];
  sm[threadIdx.x] = part[threadIdx.x];
  __syncthreads();
  for (int o = GR_B / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double v = sm[threadIdx.x + o];
      if (v > sm[threadIdx.x] || v != v) sm[threadIdx.x] = v;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(sm[0]);
    *dmax = b;
    if (hmax) __hip_atomic_store(hmax, b, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}
// preconditioner input: z = 0 except at the wall Dirichlet rows, where the cycle's x equals its right-hand side
// r; and, for the xi updates of the cycle, G = the sum over the internal cells of the continuity right-hand sides
// less the wall Dirichlet faces' share (as k_gsum forms it from x = z and b = r), as PC_B block partials in part.
// Thread t of the grid-stride loop covers the three grid entries at t (and the xi entry, t = 0) and cell t.
constexpr int PC_B = 256, PC_T = 1024;
__global__ void __launch_bounds__(PC_T) k_pc_in(const uint8_t *__restrict__ cls, int W, double h,
                                                const double *__restrict__ r, double *z, double *part) {
  __shared__ double sm[PC_T / 64];
  const int WW = W * W;
  double s = 0;
  for (int t = blockIdx.x * PC_T + threadIdx.x; t < WW; t += PC_B * PC_T) {
    const uint8_t cu = cls[t], cv = cls[WW + t], cp = cls[2 * WW + t];
    z[t] = cu == K_WALLD ? r[t] : 0.0;
    z[WW + t] = cv == K_WALLD ? r[WW + t] : 0.0;
    z[2 * WW + t] = cp == K_WALLD ? r[2 * WW + t] : 0.0;
    if (t == 0) z[3 * WW] = 0.0;
    if (cp == K_INT) {
      double wf = 0;
      if (cls[t + 1] == K_WALLD) wf += r[t + 1];
      if (cu == K_WALLD) wf -= r[t];
      if (cls[WW + t + W] == K_WALLD) wf += r[WW + t + W];
      if (cv == K_WALLD) wf -= r[WW + t];
      s += r[2 * WW + t] - wf / h;
    }
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int q = 0; q < PC_T / 64; q++) t += sm[q];
    part[blockIdx.x] = t;
  }
}
// preconditioner output (FP64, in place): the pressure unknowns shifted by -mean + (mean-row entry of r), which is
// the cycle's mean projection followed by the mean-row column of B' (a constant pressure changes no other row)
__global__ void __launch_bounds__(TPB) k_pc_shift(const uint8_t *__restrict__ cls, int WW, const double *__restrict__ part,
                                                  int np, const int *__restrict__ mp, double *mean,
                                                  const double *__restrict__ r, double *z) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const double m = pmean_total(part, np, mp, mean);
  if (t >= WW) return;
  const uint8_t c = cls[2 * WW + t];
  if (c == K_INT || c == K_GHOST || c == K_GHOSTX) z[2 * WW + t] += r[3 * WW] - m;
}

gp_status gcr_alloc(Ctx *ctx) {
  const int m = std::max(1, ctx->prm.krylov);
  GcrWs &w = ctx->kr;
  if (w.r && w.m == m) return GP_OK;
  const size_t n = ctx->geo[0].n;
  for (double **p : {&w.r, &w.z, &w.Q, &w.Z, &w.zero, &w.s, &w.part}) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  w.m = 0;
  GP_HIP(hipMalloc((void **)&w.r, n * sizeof(double)));
  GP_HIP(hipMalloc((void **)&w.z, n * sizeof(double)));
  GP_HIP(hipMalloc((void **)&w.Q, (size_t)m * n * sizeof(double)));
  GP_HIP(hipMalloc((void **)&w.Z, (size_t)m * n * sizeof(double)));
  GP_HIP(hipMalloc((void **)&w.zero, n * sizeof(double)));
  GP_HIP(hipMalloc((void **)&w.s, (2 * KR_MAX + 8) * sizeof(double)));
  GP_HIP(hipMalloc((void **)&w.part, (size_t)(KR_MAX + 2) * GR_B * sizeof(double)));
  k_fill<double><<<nblk((long)n), TPB, 0, ctx->stream>>>(w.zero, (long)n, 0.0);
  GP_HIP(hipGetLastError());
  w.m = m;
  return GP_OK;
}

gp_status gcr_solve(Ctx *ctx, const GcrWs &ws, GcrOps &ops, double *x, double *r, double r0, double thr, double lim,
                    int max_it, int *iters, double *res, double *rho, int *status, double *kbytes) {
  hipStream_t s = ctx->stream;
  const long n = ctx->geo[0].n;
  const int m = ws.m;
  double *beta = ws.s, *sc = ws.s + KR_MAX, *nu2 = ws.s + KR_MAX + 8;
  double rn = r0, rp = r0;
  int c = 0, k = 0;
  gp_status st = GP_OK;
  *status = GP_OK;
  *rho = 0;
  double kb = 0;
  while (rn > thr && c < max_it) {
    double *z = ws.z, *qn = ctx->v64[0].r;
    double *Qk = ws.Q + (size_t)k * n, *Zk = ws.Z + (size_t)k * n;
    ops.precond(r, z);
    ops.apply_neg(z, qn);  // qn = -M z
    if (k) {
      k_gcr_dots<<<GR_B, GR_T, 0, s>>>(ws.Q, n, k, qn, ws.part);
      k_gcr_sum<<<1, GR_B, 0, s>>>(ws.part, k, nu2, beta, nullptr);
    }
    k_gcr_orth<<<GR_B, GR_T, 0, s>>>(ws.Q, ws.Z, n, k, beta, qn, z, r, Qk, Zk, ws.part);
    k_gcr_sum<<<1, GR_B, 0, s>>>(ws.part, 2, nullptr, sc, nu2 + k);
    k_gcr_step<<<GR_B, GR_T, 0, s>>>(n, sc, Qk, Zk, x, r, ws.part);
    __atomic_store_n(ctx->h_rmax, NORM_PENDING, __ATOMIC_RELEASE);
    k_gcr_max<<<1, GR_B, 0, s>>>(ws.part, (unsigned long long *)(ctx->d_scal + 1), ctx->h_rmax);
    GP_HIP(hipGetLastError());
    if ((st = wait_norm(ctx, &rn))) return st;
    kb += (3.0 * k + 12.0) * 8.0 * (double)n;
    c++;
    k++;
    if (!(rn == rn) || rn > lim) {
      *status = GP_EDIVERGED;
      break;
    }
    if (rn <= thr || k == m) {  // confirm with the true residual, or restart from it
      if ((st = ops.residual(&rn))) return st;
      k = 0;
    }
    *rho = rn / rp;
    rp = rn;
  }
  *iters = c;
  *res = rn;
  if (kbytes) *kbytes = kb;
  return GP_OK;
}

// the cycle's result as a preconditioner output: pressure unknowns shifted by the mean-row entry of r (the cycle
// itself leaves the mean at zero; a constant pressure changes no other row), zero where no equation
template <typename T>
__global__ void k_pc_out(const uint8_t *__restrict__ cls, int WW, const T *xin, const double *__restrict__ r, double *z) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > 3 * WW) return;
  if (t == 3 * WW) {
    z[t] = (double)xin[t];
    return;
  }
  const uint8_t c = cls[t];
  const bool eq = c == K_INT || c == K_GHOST || c == K_GHOSTX || c == K_WALLG || c == K_WALLD;
  const bool pu = t >= 2 * WW && (c == K_INT || c == K_GHOST || c == K_GHOSTX);
  z[t] = eq ? (double)xin[t] + (pu ? r[3 * WW] : 0.0) : 0.0;
}

// GCR around the FP64 cycle (precision GP_FP64) or the FP32 cycle (GP_MIXED: the preconditioner runs in FP32
// storage, everything else in FP64)
static gp_status gcr_mg_solve(Ctx *ctx, const GcrWs &ws, int precision, double tol, int max_cycles, gp_stats *stt) {
  auto t0 = std::chrono::steady_clock::now();
  gp_status st = set_wall_dirichlet(ctx);
  if (st) return st;
  if ((st = ensure_xb(ctx))) return st;
  if (precision != GP_FP64 && (st = ensure_fp32(ctx))) return st;
  Geo &G = ctx->geo[0];
  Vec<double> &V = ctx->v64[0];
  hipStream_t s = ctx->stream;
  const long n = G.n;
  double *X0 = V.x, *B0 = V.b;
  double r0, bn;
  if ((st = resnorm64(ctx, &r0))) return st;  // V.r = b - M x
  if (!(r0 == r0)) return GP_EDIVERGED;        // NaN or Inf in the data
  GP_HIP(hipMemcpyAsync(ws.r, V.r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  if ((st = bnorm64(ctx, &bn))) return st;
  const double thr = tol * (bn > 1 ? bn : 1), lim = 1e6 * (r0 > 1 ? r0 : 1);
  GcrOps ops;
  ops.precond = [&](const double *r, double *z) {
    if (precision == GP_FP64) {
      double *Y0 = V.y;
      V.x = z;
      V.b = const_cast<double *>(r);
      // z and the finest level's G (block partials in the workspace's reduction slots, which the GCR kernels
      // only use after the cycle)
      k_pc_in<<<PC_B, PC_T, 0, s>>>(G.cls, G.W, G.h, r, z, ws.part);
      ctx->gs_ptr[0] = ws.part;
      ctx->gs_n[0] = PC_B;
      cycle<double>(ctx, 0);
      if (V.x != z) {  // an odd number of finest sweeps leaves the result in the second buffer
        (void)hipMemcpyAsync(z, V.x, n * sizeof(double), hipMemcpyDeviceToDevice, s);
      }
      V.x = X0;
      V.b = B0;
      V.y = Y0;
      // the mean projection and the mean-row column in one pass
      const int np = rd_blocks(G.WW);
      k_pmean<double><<<np, RD_T, 0, s>>>(G.W, G.cls, z, ctx->d_red);
      k_pc_shift<<<nblk(G.WW), TPB, 0, s>>>(G.cls, G.WW, ctx->d_red, np, G.d_mp, ctx->d_scal, r, z);
    } else {
      Vec<float> &E = ctx->v32[0];
      k_cast_rhs<<<nblk(n), TPB, 0, s>>>(r, E.b, n);
      k_fill<float><<<nblk(n), TPB, 0, s>>>(E.x, n, 0.0f);
      k_set_walld<float><<<nblk(3L * G.WW), TPB, 0, s>>>(3 * G.WW, G.cls, E.x, E.b);
      gsum<float>(ctx, 0);
      cycle<float>(ctx, 0);
      mean_project<float>(ctx);
      k_pc_out<float><<<nblk(n), TPB, 0, s>>>(G.cls, G.WW, E.x, r, z);
    }
  };
  ops.apply_neg = [&](const double *z, double *q) {
    V.x = const_cast<double *>(z);
    V.b = ws.zero;
    double *R0 = V.r;
    V.r = q;
    residual<double>(ctx, 0, (unsigned long long *)(ctx->d_scal + 2), nullptr, true);
    V.x = X0;
    V.b = B0;
    V.r = R0;
  };
  ops.residual = [&](double *rinf) -> gp_status {
    gp_status e = resnorm64(ctx, rinf);
    if (e) return e;
    GP_HIP(hipMemcpyAsync(ws.r, V.r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    return GP_OK;
  };
  int iters = 0, status = GP_OK;
  double res = r0, rho = 0;
  double kb = 0;
  st = gcr_solve(ctx, ws, ops, X0, ws.r, r0, thr, lim, max_cycles, &iters, &res, &rho, &status, &kb);
  V.x = X0;
  V.b = B0;
  if (st) return st;
  gp_status out = status;
  if (out == GP_OK && res > thr) out = GP_ENOCONV;
  ctx->last_cycles = iters;
  if (stt) {
    stt->cycles = iters;
    stt->bytes_alg = iters * (cycle_bytes(ctx, precision != GP_FP64) + norm_bytes(ctx)) + kb;
    stt->outer = 0;
    stt->res0 = r0;
    stt->res = res;
    stt->rho = rho;
    stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return out;
}

static gp_status plain_mg_solve(Ctx *ctx, int precision, double tol, int max_cycles, gp_stats *stt);

gp_status mg_solve(Ctx *ctx, int precision, double tol, int max_cycles, gp_stats *stt) {
  if (ctx->prm.krylov <= 0) return plain_mg_solve(ctx, precision, tol, max_cycles, stt);
  gp_status st = gcr_alloc(ctx);
  if (st) return st;
  return gcr_mg_solve(ctx, ctx->kr, precision, tol, max_cycles, stt);
}

static gp_status plain_mg_solve(Ctx *ctx, int precision, double tol, int max_cycles, gp_stats *stt) {
  auto t0 = std::chrono::steady_clock::now();
  gp_status st = set_wall_dirichlet(ctx);
  if (st) return st;
  if ((st = ensure_xb(ctx))) return st;
  double r0, bn;
  if ((st = resnorm64(ctx, &r0))) return st;
  if (!(r0 == r0)) return GP_EDIVERGED;  // NaN or Inf in the data
  if ((st = bnorm64(ctx, &bn))) return st;
  double thr = tol * (bn > 1 ? bn : 1);
  double r = r0, rho = 0;
  int c = 0, outer = 0;
  gp_status out = GP_OK;
  // the launch probe records events around launches, which a replayed graph would not repeat
  const bool graph = ctx->graphs && ctx->probe_ev.empty() && r > thr && max_cycles > 0;
  if (precision != GP_FP64 && (st = ensure_fp32(ctx))) return st;
  if (precision == GP_FP64) gsum<double>(ctx, 0);  // b and the wall values are fixed during the solve
  if (graph && (st = capture_iteration(ctx, precision))) return st;
  hipGraphExec_t ex = ctx->g_iter[precision == GP_FP64 ? 0 : 1];
  const double lim = 1e6 * (r0 > 1 ? r0 : 1);  // divergence
  if (precision == GP_FP64) {
    // the loop goes on while thr < r <= lim (r not NaN) and c < max_cycles: the guard of queue_head
    const bool ahead = ctx->queue_ahead && !graph && ctx->prm.nu1 > 0 && ctx->L > 1 &&
                       !(ctx->small_cycles && ctx->geo[0].N <= 32) && box5_applies<double>(ctx, 0);
    while (r > thr && c < max_cycles) {
      double rp = r;
      if (graph) {
        __atomic_store_n(ctx->h_rmax, NORM_PENDING, __ATOMIC_RELEASE);
        GP_HIP(hipGraphLaunch(ex, ctx->stream));
        if ((st = wait_norm(ctx, &r))) return st;
      } else {
        cycle<double>(ctx, 0);
        mean_project<double>(ctx);
        norm_launch(ctx, false);  // the cycles form their own residuals; only the norm is needed
        GP_HIP(hipGetLastError());
        if (ahead && c + 1 < max_cycles) queue_head(ctx, thr, lim);
        GP_HIP(hipGetLastError());
        st = wait_norm(ctx, &r);
        if (st) {
          drop_head(ctx);
          return st;
        }
      }
      c++;
      rho = r / rp;
      const bool diverged = !(r == r) || r > lim;
      if (diverged || !(r > thr) || c >= max_cycles) drop_head(ctx);
      if (diverged) {
        out = GP_EDIVERGED;
        break;
      }
    }
  } else {
    int k = ctx->prm.mixed_inner_cycles;
    while (r > thr && c < max_cycles) {
      double rp = r;
      if (graph) {  // v64[0].r holds the residual of the last norm
        __atomic_store_n(ctx->h_rmax, NORM_PENDING, __ATOMIC_RELEASE);
        GP_HIP(hipGraphLaunch(ex, ctx->stream));
        if ((st = wait_norm(ctx, &r))) return st;
      } else {
        refine_step(ctx, k);
        if ((st = resnorm64(ctx, &r))) return st;
      }
      c += k;
      outer++;
      rho = r / rp;
      if (!(r == r) || r > lim) {
        out = GP_EDIVERGED;
        break;
      }
    }
  }
  if (out == GP_OK && r > thr) out = GP_ENOCONV;
  ctx->last_cycles = c;
  if (stt) {
    stt->cycles = c;
    stt->bytes_alg = c * (cycle_bytes(ctx, precision != GP_FP64) + norm_bytes(ctx));
    stt->outer = outer;
    stt->res0 = r0;
    stt->res = r;
    stt->rho = rho;
    stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return out;
}


// ---------------------------------------------------------------------------------------------------------
// gp_solve_noalloc: the FP64 solve of gp_solve with its GCR workspace taken from a static device array instead of
// device memory the context allocates at its first solve.  Every device the library runs on holds one copy of the
// array (SCRATCH_BYTES) until the process ends; its address on a device is taken once, by scratch_init with that
// device current (context set-up), and kept per device.  Host code never uses the array's name as an address: on
// the host the name stands for a host-side shadow, which a kernel cannot dereference.
// ---------------------------------------------------------------------------------------------------------
constexpr size_t SCRATCH_BYTES = size_t(64) << 20;
constexpr size_t SCRATCH_DOUBLES = SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];
constexpr int SCRATCH_MAX_DEV = 64;
static std::mutex scratch_mu;
static double *scratch_dev[SCRATCH_MAX_DEV];
static bool scratch_done[SCRATCH_MAX_DEV];

gp_status scratch_init(Ctx *ctx) {
  const int dev = ctx->device;
  if (dev < 0 || dev >= SCRATCH_MAX_DEV) return GP_EINVAL;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (scratch_done[dev]) return scratch_dev[dev] ? GP_OK : GP_EHIP;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  scratch_done[dev] = true;
  if (e != hipSuccess || !p) {
    ctx->hip_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return GP_EHIP;
  }
  scratch_dev[dev] = (double *)p;
  return GP_OK;
}

// doubles of a GCR workspace with m directions over vectors of n doubles, each piece starting on a 256-byte boundary
static size_t gcr_ws_doubles(long n, int m) {
  auto up = [](size_t v) { return (v + 31) & ~(size_t)31; };
  return 3 * up((size_t)n) + 2 * up((size_t)m * n) + up(2 * KR_MAX + 8) + up((size_t)(KR_MAX + 2) * GR_B);
}

gp_status mg_solve_noalloc(Ctx *ctx, double tol, int max_cycles, gp_stats *stt) {
  const bool graphs = ctx->graphs;
  ctx->graphs = 0;  // instantiating a graph allocates
  gp_status st = GP_OK;
  if (ctx->prm.krylov <= 0) {  // the plain cycle iteration uses no workspace
    st = plain_mg_solve(ctx, GP_FP64, tol, max_cycles, stt);
    ctx->graphs = graphs;
    return st;
  }
  ctx->graphs = graphs;
  double *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (ctx->device >= 0 && ctx->device < SCRATCH_MAX_DEV) base = scratch_dev[ctx->device];
  }
  if (!base) {
    if (ctx->hip_err.empty()) ctx->hip_err = "gp_solve_noalloc: the static scratch array has no address on this device";
    return GP_EHIP;
  }
  const long n = ctx->geo[0].n;
  const int m = ctx->prm.krylov;
  const size_t need = gcr_ws_doubles(n, m);
  if (need > SCRATCH_DOUBLES) {
    ctx->hip_err = "gp_solve_noalloc: GCR workspace of " + std::to_string(need * sizeof(double)) + " bytes (N = " +
                   std::to_string(ctx->N) + ", krylov = " + std::to_string(m) + ") exceeds the static scratch of " +
                   std::to_string(SCRATCH_BYTES) + " bytes";
    return GP_ESCRATCH;
  }
  auto up = [](size_t v) { return (v + 31) & ~(size_t)31; };
  GcrWs w;
  w.m = m;
  double *p = base;
  w.r = p, p += up((size_t)n);
  w.z = p, p += up((size_t)n);
  w.zero = p, p += up((size_t)n);
  w.Q = p, p += up((size_t)m * n);
  w.Z = p, p += up((size_t)m * n);
  w.s = p, p += up(2 * KR_MAX + 8);
  w.part = p;
  // the array keeps whatever the last call on this device left in it: the zero vector is cleared by a fill kernel
  // (every other piece is written before it is read)
  k_fill<double><<<nblk(n), TPB, 0, ctx->stream>>>(w.zero, n, 0.0);
  GP_HIP(hipGetLastError());
  return gcr_mg_solve(ctx, w, GP_FP64, tol, max_cycles, stt);
}

}  // namespace gpmg
