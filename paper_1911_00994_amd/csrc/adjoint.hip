// Reverse mode of the solver: the transposed system M^T lam = g, solved with the transpose of the multigrid
// cycle, and the adjoint of the Crank-Nicolson step (gradients of a function of the final velocity with respect
// to the forcing and to the rigid-body velocity).  Everything here is FP64.
//
// The cycle is an affine map x_out = C x_in + B b.  The transposed cycle applies B'^T, the exact transpose of
// B' = B + s e_mean^T, where s is the indicator of the pressure unknowns that the mean projection shifts: B' is
// what the cycle computes for a mean-row right-hand side b_mean (the cycle itself only handles b_mean = 0, and
// the shift by b_mean is exact because the gradient, Neumann and extrapolation rows do not see a constant
// pressure).  lam <- lam + B'^T (g - M^T lam) then has the error propagator (I - M B')^T, with the spectrum of
// the forward iteration's I - B' M.  Each elementary operation of the cycle is transposed on its own, in reverse
// order:
//   box colour      x_F <- A_F^{-1} (b_F - M_{F,~F} x)   ->  s = A_F^{-T} xbar_F, bbar_F += s, xbar_F = 0,
//                                                          xbar_k -= M_{F,k} s for the other columns k;
//                   A_F^T = S A_F S with S = diag(1, 1, 1, 1, -1) (the pressure row and column change sign)
//   ghost sweep     x_G <- x_G + dtau (b_G - B_G x)        ->  t = dtau xbar_G, bbar_G += t, xbar -= B^T t
//   xi update       xi = mean over internal cells of (div u - g)
//   residual        r = b - M x                            ->  bbar += rbar, xbar -= M^T rbar
//   restriction, prolongation, extension fill, coarsest inverse, mean projection, wall identity rows.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace gpmg {

namespace {

constexpr int ARED = 512;  // blocks of the deterministic reductions here

__device__ __forceinline__ int aix(int W, int i, int j) { return (j + 1) * W + (i + 1); }

__device__ double ablock_sum(double v) {
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
// deterministic grid sum: block partials, the last block to finish adds them in block order
__device__ bool alast_total(double mine, double *part, unsigned *ticket, double *total) {
  __shared__ bool last;
  double bs = ablock_sum(mine);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = bs;
    __threadfence();
    unsigned tk = atomicAdd(ticket, 1u);
    last = (tk == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double v = 0;
  for (int q = threadIdx.x; q < (int)gridDim.x; q += TPB) v += __hip_atomic_load(&part[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  *total = ablock_sum(v);
  if (threadIdx.x == 0) *ticket = 0;
  return true;
}

// ---------------------------------------------------------------------------------------------------------
// y = base + sgn * M^T lam.  Point part: each unknown gathers the coefficients of the internal momentum and
// continuity rows, the wall identity row and the mean row that reference it.
// ---------------------------------------------------------------------------------------------------------
__global__ void k_mt_pts(int N, int W, double h, double a, double d, const uint8_t *__restrict__ cls,
                         const double *__restrict__ lam, const double *base, double sgn, double *y, double inv_mp) {
  const int WW = W * W;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * WW) return;
  const int g = t / WW, q = t - g * WW, j = q / W - 1, i = q % W - 1;
  const uint8_t *cu = cls, *cv = cls + WW, *cp = cls + 2 * WW;
  const double *lu = lam, *lv = lam + WW, *lp = lam + 2 * WW;
  const double ih = 1.0 / h;
  const bool hasW = i - 1 >= -1, hasE = i + 1 <= N, hasS = j - 1 >= -1, hasN = j + 1 <= N;
  double s = 0;
  if (g == 0) {
    if (cu[q] == K_INT) s += d * lu[q];
    if (hasW && cu[q - 1] == K_INT) s -= a * lu[q - 1];
    if (hasE && cu[q + 1] == K_INT) s -= a * lu[q + 1];
    if (hasS && cu[q - W] == K_INT) s -= a * lu[q - W];
    if (hasN && cu[q + W] == K_INT) s -= a * lu[q + W];
    if (hasW && cp[q - 1] == K_INT) s += ih * lp[q - 1];  // E face of cell (i-1, j)
    if (cp[q] == K_INT) s -= ih * lp[q];                  // W face of cell (i, j)
    if (cu[q] == K_WALLD) s += lu[q];
  } else if (g == 1) {
    if (cv[q] == K_INT) s += d * lv[q];
    if (hasW && cv[q - 1] == K_INT) s -= a * lv[q - 1];
    if (hasE && cv[q + 1] == K_INT) s -= a * lv[q + 1];
    if (hasS && cv[q - W] == K_INT) s -= a * lv[q - W];
    if (hasN && cv[q + W] == K_INT) s -= a * lv[q + W];
    if (hasS && cp[q - W] == K_INT) s += ih * lp[q - W];  // N face of cell (i, j-1)
    if (cp[q] == K_INT) s -= ih * lp[q];                  // S face of cell (i, j)
    if (cv[q] == K_WALLD) s += lv[q];
  } else {
    if (cu[q] == K_INT) s += ih * lu[q];                 // u(i,j) row: (p(i,j) - p(i-1,j)) / h
    if (hasE && cu[q + 1] == K_INT) s -= ih * lu[q + 1];
    if (cv[q] == K_INT) s += ih * lv[q];
    if (hasN && cv[q + W] == K_INT) s -= ih * lv[q + W];
    if (cp[q] == K_INT) s += lam[3 * WW] * inv_mp;       // mean row
  }
  y[t] = base[t] + sgn * s;
}
// ghost rows: y[col] += sgn * w * lam_G
__global__ void k_mt_ghost(const int *__restrict__ pt, const int *__restrict__ col, const double *__restrict__ w, int ng,
                           const double *__restrict__ lam, double sgn, double *y) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ng) return;
  double lg = sgn * lam[pt[r]];
  if (lg == 0.0) return;
#pragma unroll
  for (int z = 0; z < 9; z++) atomicAdd(&y[col[9 * r + z]], w[9 * r + z] * lg);
}
// xi column: -1 in every internal continuity row
__global__ void __launch_bounds__(TPB) k_mt_xi(int W, const uint8_t *__restrict__ cls, const double *__restrict__ lam,
                                               const double *base, double sgn, double *y, double *part, unsigned *ticket) {
  const int WW = W * W;
  double s = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < WW; t += gridDim.x * blockDim.x)
    if (cls[2 * WW + t] == K_INT) s += lam[2 * WW + t];
  double tot;
  if (alast_total(s, part, ticket, &tot) && threadIdx.x == 0) y[3 * WW] = base[3 * WW] - sgn * tot;
}

// ---------------------------------------------------------------------------------------------------------
// transposed box colour.  Free unknowns F of the box (internal ones); s = A_F^{-T} y solved as S A_F^{-1} S y
// with the closed form of the forward box solve (fixed unknowns enter with zero); then bbar_F += s, xbar_F = 0
// and xbar_k -= M_{F,k} s over the columns outside F (atomics: same-colour boxes share read-only neighbours,
// never unknowns).  The xi column collects sum of s_P (grid sum, added to xbar_xi by the last block).
// ---------------------------------------------------------------------------------------------------------
__device__ __forceinline__ double box_adj(int N, int W, double h, double a, double d, const uint8_t *__restrict__ cls,
                                          double *xb, double *bb, int i, int j) {
  const int WW = W * W, c = (j + 1) * W + (i + 1);
  const bool fW = cls[c] == K_INT, fE = cls[c + 1] == K_INT, fS = cls[WW + c] == K_INT, fN = cls[WW + c + W] == K_INT,
             fP = cls[2 * WW + c] == K_INT;
  if (!(fW || fE || fS || fN || fP)) return 0.0;
  const double ih = 1.0 / h, det = d * d - a * a;
  // right-hand side S y
  const double rW = fW ? xb[c] : 0.0, rE = fE ? xb[c + 1] : 0.0, rS = fS ? xb[WW + c] : 0.0, rN = fN ? xb[WW + c + W] : 0.0,
               rP = fP ? -xb[2 * WW + c] : 0.0;
  double aW = 0, bW = 0, aE = 0, bE = 0, aS = 0, bS = 0, aN = 0, bN = 0;
  if (fW && fE) {
    aW = (d * rW + a * rE) / det;
    bW = -ih / (d + a);
    aE = (a * rW + d * rE) / det;
    bE = ih / (d + a);
  } else if (fW) {
    aW = rW / d;
    bW = -ih / d;
  } else if (fE) {
    aE = rE / d;
    bE = ih / d;
  }
  if (fS && fN) {
    aS = (d * rS + a * rN) / det;
    bS = -ih / (d + a);
    aN = (a * rS + d * rN) / det;
    bN = ih / (d + a);
  } else if (fS) {
    aS = rS / d;
    bS = -ih / d;
  } else if (fN) {
    aN = rN / d;
    bN = ih / d;
  }
  double zP = 0;
  if (fP) {
    const double den = bE - bW + bN - bS;
    if (den == 0.0) return 0.0;  // the forward sweep skips this box
    zP = (h * rP - (aE - aW + aN - aS)) / den;
  }
  const double sW = fW ? aW + bW * zP : 0.0, sE = fE ? aE + bE * zP : 0.0, sS = fS ? aS + bS * zP : 0.0,
               sN = fN ? aN + bN * zP : 0.0, sP = fP ? -zP : 0.0;
  double *xu = xb, *xv = xb + WW, *xp = xb + 2 * WW;
  if (fW) {
    bb[c] += sW;
    xu[c] = 0;
    atomicAdd(&xu[c - 1], a * sW);
    atomicAdd(&xu[c - W], a * sW);
    atomicAdd(&xu[c + W], a * sW);
    if (!fE) atomicAdd(&xu[c + 1], a * sW);
    atomicAdd(&xp[c - 1], ih * sW);
    if (!fP) atomicAdd(&xp[c], -ih * sW);
  }
  if (fE) {
    bb[c + 1] += sE;
    xu[c + 1] = 0;
    atomicAdd(&xu[c + 2], a * sE);
    atomicAdd(&xu[c + 1 - W], a * sE);
    atomicAdd(&xu[c + 1 + W], a * sE);
    if (!fW) atomicAdd(&xu[c], a * sE);
    atomicAdd(&xp[c + 1], -ih * sE);
    if (!fP) atomicAdd(&xp[c], ih * sE);
  }
  if (fS) {
    bb[WW + c] += sS;
    xv[c] = 0;
    atomicAdd(&xv[c - W], a * sS);
    atomicAdd(&xv[c - 1], a * sS);
    atomicAdd(&xv[c + 1], a * sS);
    if (!fN) atomicAdd(&xv[c + W], a * sS);
    atomicAdd(&xp[c - W], ih * sS);
    if (!fP) atomicAdd(&xp[c], -ih * sS);
  }
  if (fN) {
    bb[WW + c + W] += sN;
    xv[c + W] = 0;
    atomicAdd(&xv[c + 2 * W], a * sN);
    atomicAdd(&xv[c + W - 1], a * sN);
    atomicAdd(&xv[c + W + 1], a * sN);
    if (!fS) atomicAdd(&xv[c], a * sN);
    atomicAdd(&xp[c + W], -ih * sN);
    if (!fP) atomicAdd(&xp[c], ih * sN);
  }
  if (fP) {
    bb[2 * WW + c] += sP;
    xp[c] = 0;
    if (!fE) atomicAdd(&xu[c + 1], -ih * sP);
    if (!fW) atomicAdd(&xu[c], ih * sP);
    if (!fN) atomicAdd(&xv[c + W], -ih * sP);
    if (!fS) atomicAdd(&xv[c], ih * sP);
  }
  (void)N;
  return sP;
}
// one colour over all cells (list == nullptr) or over the band cells list[lo, hi)
__global__ void __launch_bounds__(TPB) k_box_adj(int N, int W, double h, double a, double d, const uint8_t *__restrict__ cls,
                                                 double *xb, double *bb, int colour, const int *__restrict__ list, int lo,
                                                 int hi, double *part, unsigned *ticket) {
  const int K = N / 5 + 1;
  const long total = list ? (long)(hi - lo) : (long)K * N;
  double sp = 0;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    int i, j;
    if (list) {
      int cell = list[lo + t];
      i = cell % N;
      j = cell / N;
    } else {
      j = (int)(t / K);
      int kk = (int)(t - (long)j * K);
      i = ((colour - 2 * j) % 5 + 5) % 5 + 5 * kk;
      if (i >= N) continue;
    }
    sp += box_adj(N, W, h, a, d, cls, xb, bb, i, j);
  }
  double tot;
  if (alast_total(sp, part, ticket, &tot) && threadIdx.x == 0) xb[3 * W * W] += tot;
}

// transposed Jacobi sweep of all ghost rows
__global__ void k_gadj_a(const int *__restrict__ pt, const double *__restrict__ dtau, int ng, const double *__restrict__ xb,
                         double *bb, double *tmp) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ng) return;
  double t = dtau[r] * xb[pt[r]];
  tmp[r] = t;
  bb[pt[r]] += t;
}
__global__ void k_gadj_b(const int *__restrict__ col, const double *__restrict__ w, int ng, const double *__restrict__ tmp,
                         double *xb) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ng) return;
  double t = tmp[r];
  if (t == 0.0) return;
#pragma unroll
  for (int z = 0; z < 9; z++) atomicAdd(&xb[col[9 * r + z]], -w[9 * r + z] * t);
}

// transposed xi update: xi = (sum over internal cells of (div u - g)) / mp
__global__ void k_take(double *src, double *dst) {
  *dst = *src;
  *src = 0.0;
}
__global__ void k_xi_adj(int N, int W, double h, const uint8_t *__restrict__ cls, double *xb, double *bb,
                         const double *__restrict__ xibar, double inv_mp) {
  const int WW = W * W;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * WW) return;
  const double c = *xibar * inv_mp;
  if (c == 0.0) return;
  const int g = t / WW, q = t - g * WW, j = q / W - 1, i = q % W - 1;
  const uint8_t *cp = cls + 2 * WW;
  if (g == 0) {
    double f = (i - 1 >= -1 && cp[q - 1] == K_INT ? 1.0 : 0.0) - (cp[q] == K_INT ? 1.0 : 0.0);
    if (f != 0.0) xb[t] += f * c / h;
  } else if (g == 1) {
    double f = (j - 1 >= -1 && cp[q - W] == K_INT ? 1.0 : 0.0) - (cp[q] == K_INT ? 1.0 : 0.0);
    if (f != 0.0) xb[t] += f * c / h;
  } else if (cp[q] == K_INT) {
    bb[t] -= c;
  }
  (void)N;
}

// transposed residual: bbar += rbar (the M^T part is k_mt_* with sgn = -1)
__global__ void k_add(double *y, const double *__restrict__ x, long n) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < n) y[t] += x[t];
}

// transposed restriction (gather over the coarse parents of each fine point, with the forward weights)
__device__ __forceinline__ double restrict_weight(int g, int Nf, int Wf, const uint8_t *__restrict__ clsf, int ic, int jc,
                                                  uint8_t cc, int dxs, int dys) {
  const int WWf = Wf * Wf;
  bool all = true;
  int cnt = 0;
  double wsel = 0;
  for (int dy = (g == 1 ? -1 : 0); dy <= 1; dy++)
    for (int dx = (g == 0 ? -1 : 0); dx <= 1; dx++) {
      double fw = g == 0 ? (dx == 0 ? 0.25 : 0.125) : (g == 1 ? (dy == 0 ? 0.25 : 0.125) : 0.25);
      int fi = 2 * ic + dx, fj = 2 * jc + dy;
      if (fi < -1 || fi > Nf || fj < -1 || fj > Nf) {
        all = false;
        continue;
      }
      if (clsf[g * WWf + aix(Wf, fi, fj)] == cc) {
        cnt++;
        if (dx == dxs && dy == dys) wsel = fw;
      } else
        all = false;
    }
  return all ? wsel : (cnt ? 1.0 / cnt : 0.0);
}
__global__ void k_restrict_adj(int Nf, int Wf, const uint8_t *__restrict__ clsf, double *rbf, int Nc, int Wc,
                               const uint8_t *__restrict__ clsc, const double *__restrict__ bbc) {
  const int WWf = Wf * Wf, WWc = Wc * Wc;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 3 * WWf) {
    rbf[t] = 0.0;
    return;
  }
  if (t > 3 * WWf) return;
  const int g = t / WWf, q = t - g * WWf, j = q / Wf - 1, i = q % Wf - 1;
  const uint8_t cf = clsf[t];
  double acc = 0;
  if (cf == K_INT || cf == K_GHOST || cf == K_WALLG) {
    for (int dy = (g == 1 ? -1 : 0); dy <= 1; dy++)
      for (int dx = (g == 0 ? -1 : 0); dx <= 1; dx++) {
        if (((i - dx) & 1) || ((j - dy) & 1)) continue;
        int ic = (i - dx) / 2, jc = (j - dy) / 2;
        if (ic < -1 || ic > Nc || jc < -1 || jc > Nc) continue;
        int kc = g * WWc + aix(Wc, ic, jc);
        if (clsc[kc] != cf) continue;
        acc += restrict_weight(g, Nf, Wf, clsf, ic, jc, cf, dx, dy) * bbc[kc];
      }
  }
  rbf[t] = acc;
}

// transposed prolongation: each coarse point gathers the weights with which the fine points of its window read it
__device__ __forceinline__ int prolong_parents(int g, int i, int j, int Nc, int pi[4], int pj[4], double pw[4]) {
  int xi_[2], yi_[2], nx, ny;
  double xw[2], yw[2];
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
  int m = 0;
  for (int aa = 0; aa < ny; aa++)
    for (int bb = 0; bb < nx; bb++) {
      int ic = xi_[bb], jc = yi_[aa];
      if (g == 2) {
        ic = ic < 0 ? 0 : (ic > Nc - 1 ? Nc - 1 : ic);
        jc = jc < 0 ? 0 : (jc > Nc - 1 ? Nc - 1 : jc);
      }
      if (ic < -1 || ic > Nc || jc < -1 || jc > Nc) continue;
      pi[m] = ic;
      pj[m] = jc;
      pw[m] = xw[bb] * yw[aa];
      m++;
    }
  return m;
}
__global__ void k_prolong_adj(int Nf, int Wf, const uint8_t *__restrict__ clsf, const double *__restrict__ xbf, int Nc,
                              int Wc, double *xbc) {
  const int WWf = Wf * Wf, WWc = Wc * Wc;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 3 * WWc) {
    xbc[t] = xbf[3 * WWf];
    return;
  }
  if (t > 3 * WWc) return;
  const int g = t / WWc, q = t - g * WWc, jc = q / Wc - 1, ic = q % Wc - 1;
  double acc = 0;
  for (int j = 2 * jc - 1; j <= 2 * jc + 2; j++)
    for (int i = 2 * ic - 1; i <= 2 * ic + 2; i++) {
      if (i < -1 || i > Nf || j < -1 || j > Nf) continue;
      int kf = g * WWf + aix(Wf, i, j);
      uint8_t c = clsf[kf];
      if (!(c == K_INT || c == K_GHOST || c == K_GHOSTX || c == K_WALLG)) continue;
      int pi[4], pj[4];
      double pw[4];
      int m = prolong_parents(g, i, j, Nc, pi, pj, pw);
      for (int z = 0; z < m; z++)
        if (pi[z] == ic && pj[z] == jc) acc += pw[z] * xbf[kf];
    }
  xbc[t] = acc;
}

// transposed extension fill (sources are internal or ghost points, never extension points)
__global__ void k_ext_adj(const int *__restrict__ e_pt, const int *__restrict__ e_src, const double *__restrict__ e_w, int ne,
                          double *xb) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne || e_src[3 * e] < 0) return;
  double v = xb[e_pt[e]];
  xb[e_pt[e]] = 0.0;
  if (v == 0.0) return;
  for (int q = 0; q < 3; q++) atomicAdd(&xb[e_src[3 * e + q]], e_w[3 * e + q] * v);
}

// transposed coarsest solve: bbar[bmap[j]] += sum_q Ainv[q][j] xbar[map[q]] (one wavefront per column), then
// xbar[map[q]] = 0
__global__ void __launch_bounds__(64) k_coarse_t(const double *__restrict__ Ainv, const int *__restrict__ map,
                                                 const int *__restrict__ bmap, int nc, const double *__restrict__ xb,
                                                 double *bb) {
  int jcol = blockIdx.x;
  double s = 0;
  for (int q = threadIdx.x; q < nc; q += 64) s += Ainv[(size_t)q * nc + jcol] * xb[map[q]];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (threadIdx.x == 0) bb[bmap[jcol]] += s;
}
__global__ void k_zero_at(const int *__restrict__ idx, int n, double *x) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) x[idx[q]] = 0.0;
}

// transposed mean projection (p -= mean over internal p, on internal, ghost and extrapolated p), plus the
// mean-row column of B': sigma = sum over those p of xbar_p goes to bbar_mean and, divided by mp, is taken
// from xbar on the internal p
__global__ void __launch_bounds__(TPB) k_mean_sum(int W, const uint8_t *__restrict__ cls, const double *__restrict__ xb,
                                                  double *part, unsigned *ticket, double *out) {
  const int WW = W * W;
  double s = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < WW; t += gridDim.x * blockDim.x) {
    uint8_t c = cls[2 * WW + t];
    if (c == K_INT || c == K_GHOST || c == K_GHOSTX) s += xb[2 * WW + t];
  }
  double tot;
  if (alast_total(s, part, ticket, &tot) && threadIdx.x == 0) *out = tot;
}
__global__ void k_mean_apply(int W, const uint8_t *__restrict__ cls, double *xb, double *bb, const double *__restrict__ sig,
                             double inv_mp) {
  const int WW = W * W;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == WW) bb[3 * WW] += *sig;
  if (t >= WW) return;
  if (cls[2 * WW + t] == K_INT) xb[2 * WW + t] -= *sig * inv_mp;
}

// transposed wall identity rows (x_walld = b_walld before the cycle)
__global__ void k_walld_adj(int n, const uint8_t *__restrict__ cls, double *xb, double *bb) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n || cls[t] != K_WALLD) return;
  bb[t] += xb[t];
  xb[t] = 0.0;
}

// the mean-row column of B': the pressures the mean projection shifts move by b_mean
__global__ void k_mean_shift(int W, const uint8_t *__restrict__ cls, double *x, const double *__restrict__ b) {
  const int WW = W * W;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= WW) return;
  uint8_t c = cls[2 * WW + t];
  if (c == K_INT || c == K_GHOST || c == K_GHOSTX) x[2 * WW + t] += b[3 * WW];
}

__global__ void k_fill0(double *x, long n) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < n) x[t] = 0.0;
}
__global__ void k_copy(double *y, const double *__restrict__ x, long n) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < n) y[t] = x[t];
}
// unknowns of the system: internal, ghost, extrapolated, wall ghost and wall Dirichlet points, and xi
__global__ void k_mask_unknowns(int n3, const uint8_t *__restrict__ cls, double *x) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n3) return;
  uint8_t c = cls[t];
  if (!(c == K_INT || c == K_GHOST || c == K_GHOSTX || c == K_WALLG || c == K_WALLD)) x[t] = 0.0;
}
__global__ void k_absmax_d(const double *__restrict__ v, long n, unsigned long long *out) {
  double m = 0;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    double a = fabs(v[t]);
    m = (a > m || a != a) ? a : m;
  }
  unsigned long long b = (unsigned long long)__double_as_longlong(m);
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long c = __shfl_xor(b, o, 64);
    b = c > b ? c : b;
  }
  if ((threadIdx.x & 63) == 0 && b) atomicMax(out, b);
}

}  // namespace

// ---------------------------------------------------------------------------------------------------------
// host side: transposed cycle
// ---------------------------------------------------------------------------------------------------------
gp_status adjoint_alloc(Ctx *ctx) {
  if (ctx->adj[0].x) return GP_OK;
  for (int l = 0; l < ctx->L; l++) {
    size_t n = ctx->geo[l].n;
    Vec<double> &A = ctx->adj[l];
    GP_HIP(hipMalloc((void **)&A.x, n * sizeof(double)));
    GP_HIP(hipMalloc((void **)&A.b, n * sizeof(double)));
    GP_HIP(hipMalloc((void **)&A.r, n * sizeof(double)));
    k_fill0<<<nblk(n), TPB, 0, ctx->stream>>>(A.x, n);
    k_fill0<<<nblk(n), TPB, 0, ctx->stream>>>(A.b, n);
    k_fill0<<<nblk(n), TPB, 0, ctx->stream>>>(A.r, n);
  }
  size_t n0 = ctx->geo[0].n;
  GP_HIP(hipMalloc((void **)&ctx->a_g, n0 * sizeof(double)));
  GP_HIP(hipMalloc((void **)&ctx->a_lam, n0 * sizeof(double)));
  GP_HIP(hipGetLastError());
  return GP_OK;
}

static inline double coef_a_l(Ctx *ctx, int l) { return ctx->alpha / (ctx->geo[l].h * ctx->geo[l].h); }

// y = base + sgn M^T lam on level l
static void mt_apply(Ctx *ctx, int l, const double *lam, const double *base, double sgn, double *y) {
  Geo &G = ctx->geo[l];
  hipStream_t s = ctx->stream;
  double a = coef_a_l(ctx, l), d = 1.0 + 4.0 * a;
  // every entry of y is written by one thread from the same entry of base, so y may alias base
  k_mt_xi<<<std::min(ARED, nblk(G.WW)), TPB, 0, s>>>(G.W, G.cls, lam, base, sgn, y, ctx->d_red, ctx->d_ticket);
  k_mt_pts<<<nblk(3L * G.WW), TPB, 0, s>>>(G.N, G.W, G.h, a, d, G.cls, lam, base, sgn, y, 1.0 / G.mp);
  if (G.ng) k_mt_ghost<<<nblk(G.ng), TPB, 0, s>>>(G.g_pt, G.g_col, G.g_w, G.ng, lam, sgn, y);
}

static void box_colour_t(Ctx *ctx, int l, int colour, bool band) {
  Geo &G = ctx->geo[l];
  Vec<double> &A = ctx->adj[l];
  double a = coef_a_l(ctx, l), d = 1.0 + 4.0 * a;
  long total;
  const int *list = nullptr;
  int lo = 0, hi = 0;
  if (band) {
    lo = G.hband_off[colour];
    hi = G.hband_off[colour + 1];
    if (hi <= lo) return;
    list = G.band;
    total = hi - lo;
  } else {
    total = (long)(G.N / 5 + 1) * G.N;
  }
  int nb = std::min(4096, nblk(total));
  k_box_adj<<<nb, TPB, 0, ctx->stream>>>(G.N, G.W, G.h, a, d, G.cls, A.x, A.b, colour, list, lo, hi, ctx->d_red, ctx->d_ticket);
}

static void ghost_sweep_t(Ctx *ctx, int l) {
  Geo &G = ctx->geo[l];
  if (!G.ng) return;
  Vec<double> &A = ctx->adj[l];
  k_gadj_a<<<nblk(G.ng), TPB, 0, ctx->stream>>>(G.g_pt, G.g_dtau, G.ng, A.x, A.b, ctx->gtmp);
  k_gadj_b<<<nblk(G.ng), TPB, 0, ctx->stream>>>(G.g_col, G.g_w, G.ng, ctx->gtmp, A.x);
}

// reverse of: box colours 0..4, lambda ghost sweeps, [band colours 0..4, lambda ghost sweeps] x bnd_sweeps, xi
static void relax_t(Ctx *ctx, int l) {
  Geo &G = ctx->geo[l];
  Vec<double> &A = ctx->adj[l];
  hipStream_t s = ctx->stream;
  double *xib = ctx->d_scal + 8;
  k_take<<<1, 1, 0, s>>>(A.x + 3 * (size_t)G.WW, xib);
  k_xi_adj<<<nblk(3L * G.WW), TPB, 0, s>>>(G.N, G.W, G.h, G.cls, A.x, A.b, xib, 1.0 / G.mp);
  const int lam = ctx->prm.lambda_ghost;
  if (ctx->prm.bnd_sweeps > 0 && G.nband > 0) {
    for (int q = 0; q < ctx->prm.bnd_sweeps; q++) {
      for (int it = 0; it < lam; it++) ghost_sweep_t(ctx, l);
      for (int c = 4; c >= 0; c--) box_colour_t(ctx, l, c, true);
    }
  }
  for (int it = 0; it < lam; it++) ghost_sweep_t(ctx, l);
  for (int c = 4; c >= 0; c--) box_colour_t(ctx, l, c, false);
}

static void cycle_t(Ctx *ctx, int l) {
  hipStream_t s = ctx->stream;
  if (l == ctx->L - 1) {
    Vec<double> &A = ctx->adj[l];
    k_coarse_t<<<ctx->nc, 64, 0, s>>>(ctx->c_A, ctx->c_map, ctx->c_bmap, ctx->nc, A.x, A.b);
    k_zero_at<<<nblk(ctx->nc), TPB, 0, s>>>(ctx->c_map, ctx->nc, A.x);
    return;
  }
  Geo &F = ctx->geo[l], &C = ctx->geo[l + 1];
  Vec<double> &AF = ctx->adj[l], &AC = ctx->adj[l + 1];
  for (int q = 0; q < ctx->prm.nu2; q++) relax_t(ctx, l);
  k_prolong_adj<<<nblk(3L * C.WW + 1), TPB, 0, s>>>(F.N, F.W, F.cls, AF.x, C.N, C.W, AC.x);
  if (C.ne) k_ext_adj<<<nblk(C.ne), TPB, 0, s>>>(C.e_pt, C.e_src, C.e_w, C.ne, AC.x);
  k_fill0<<<nblk(C.n), TPB, 0, s>>>(AC.b, C.n);
  int reps = (l + 1 == ctx->L - 1) ? 1 : ctx->prm.gamma;
  for (int q = 0; q < reps; q++) cycle_t(ctx, l + 1);
  // x_{l+1} was set to zero before the coarse cycles: its adjoint is dropped
  k_restrict_adj<<<nblk(3L * F.WW + 1), TPB, 0, s>>>(F.N, F.W, F.cls, AF.r, C.N, C.W, C.cls, AC.b);
  k_add<<<nblk(F.n), TPB, 0, s>>>(AF.b, AF.r, F.n);
  mt_apply(ctx, l, AF.r, AF.x, -1.0, AF.x);
  for (int q = 0; q < ctx->prm.nu1; q++) relax_t(ctx, l);
}

// bbar = B'^T xbar with xbar in adj[0].x (consumed) and the result in adj[0].b
static void apply_cycle_t(Ctx *ctx) {
  Geo &G = ctx->geo[0];
  Vec<double> &A = ctx->adj[0];
  hipStream_t s = ctx->stream;
  k_fill0<<<nblk(G.n), TPB, 0, s>>>(A.b, G.n);
  k_mean_sum<<<std::min(ARED, nblk(G.WW)), TPB, 0, s>>>(G.W, G.cls, A.x, ctx->d_red, ctx->d_ticket, ctx->d_scal + 9);
  k_mean_apply<<<nblk(G.WW + 1), TPB, 0, s>>>(G.W, G.cls, A.x, A.b, ctx->d_scal + 9, 1.0 / G.mp);
  cycle_t(ctx, 0);
  k_walld_adj<<<nblk(3L * G.WW), TPB, 0, s>>>(3 * G.WW, G.cls, A.x, A.b);
}

static gp_status ready(Ctx *ctx) {
  if (!ctx->have_geom) return GP_EINVAL;
  if (!ctx->c_ok) {
    gp_status st = coarse_factor(ctx);
    if (st) return st;
  }
  return adjoint_alloc(ctx);
}

static gp_status absmax_dev(Ctx *ctx, const double *v, long n, double *out) {
  unsigned long long *m = (unsigned long long *)(ctx->d_scal + 10);
  k_fill0<<<1, 1, 0, ctx->stream>>>((double *)m, 1);
  k_absmax_d<<<std::min(1024, nblk(n)), TPB, 0, ctx->stream>>>(v, n, m);
  GP_HIP(hipGetLastError());
  unsigned long long hv;
  GP_HIP(hipMemcpyAsync(&hv, m, sizeof(hv), hipMemcpyDeviceToHost, ctx->stream));
  GP_HIP(hipStreamSynchronize(ctx->stream));
  std::memcpy(out, &hv, sizeof(double));
  return GP_OK;
}

// M^T lam = g on the finest level, g in ctx->a_g (masked to the unknowns), lam in ctx->a_lam (initial guess in)
gp_status adjoint_solve_dev(Ctx *ctx, double tol, int max_cycles, gp_stats *stt) {
  auto t0 = std::chrono::steady_clock::now();
  Geo &G = ctx->geo[0];
  Vec<double> &A = ctx->adj[0];
  hipStream_t s = ctx->stream;
  k_mask_unknowns<<<nblk(3L * G.WW), TPB, 0, s>>>(3 * G.WW, G.cls, ctx->a_g);
  double gn, r0 = 0, r = 0, rho = 0;
  gp_status st;
  if ((st = absmax_dev(ctx, ctx->a_g, G.n, &gn))) return st;
  const double thr = tol * (gn > 1 ? gn : 1);
  int c = 0;
  gp_status out = GP_OK;
  for (;;) {
    mt_apply(ctx, 0, ctx->a_lam, ctx->a_g, -1.0, A.x);  // A.x = g - M^T lam
    double rp = r;
    if ((st = absmax_dev(ctx, A.x, G.n, &r))) return st;
    if (c == 0) r0 = r;
    else rho = r / rp;
    if (!(r == r) || r > 1e6 * (r0 > 1 ? r0 : 1)) {
      out = GP_EDIVERGED;
      break;
    }
    if (r <= thr || c >= max_cycles) break;
    apply_cycle_t(ctx);
    k_add<<<nblk(G.n), TPB, 0, s>>>(ctx->a_lam, A.b, G.n);
    c++;
  }
  GP_HIP(hipGetLastError());
  if (out == GP_OK && r > thr) out = GP_ENOCONV;
  if (stt) {
    stt->cycles = c;
    stt->outer = 0;
    stt->res0 = r0;
    stt->res = r;
    stt->rho = rho;
    stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return out;
}

}  // namespace gpmg

using namespace gpmg;

static gp_status copy_in(gp_ctx *ctx, double *dst, const double *src, size_t n, int on_device) {
  GP_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        ctx->stream));
  return GP_OK;
}
static gp_status copy_out(gp_ctx *ctx, double *dst, const double *src, size_t n, int on_device) {
  GP_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        ctx->stream));
  GP_HIP(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}

extern "C" gp_status gp_apply_mt(gp_ctx *ctx, const double *lam, double *y, int on_device) {
  if (!ctx || !lam || !y) return GP_EINVAL;
  gp_status st = ready(ctx);
  if (st) return st;
  Geo &G = ctx->geo[0];
  if ((st = copy_in(ctx, ctx->a_lam, lam, G.n, on_device))) return st;
  k_fill0<<<nblk(G.n), TPB, 0, ctx->stream>>>(ctx->a_g, G.n);
  mt_apply(ctx, 0, ctx->a_lam, ctx->a_g, 1.0, ctx->adj[0].r);
  GP_HIP(hipGetLastError());
  return copy_out(ctx, y, ctx->adj[0].r, G.n, on_device);
}

extern "C" gp_status gp_apply_cycle(gp_ctx *ctx, const double *b, double *x, int on_device) {
  if (!ctx || !b || !x) return GP_EINVAL;
  gp_status st = ready(ctx);
  if (st) return st;
  Geo &G = ctx->geo[0];
  Vec<double> &V = ctx->v64[0];
  if ((st = copy_in(ctx, V.b, b, G.n, on_device))) return st;
  k_fill0<<<nblk(G.n), TPB, 0, ctx->stream>>>(V.x, G.n);
  if ((st = mg_cycle64(ctx, nullptr))) return st;
  // the mean-row column of B': shift the projected pressures by b_mean
  k_mean_shift<<<nblk(G.WW), TPB, 0, ctx->stream>>>(G.W, G.cls, V.x, V.b);
  GP_HIP(hipGetLastError());
  return copy_out(ctx, x, V.x, G.n, on_device);
}

extern "C" gp_status gp_apply_cycle_t(gp_ctx *ctx, const double *xbar, double *bbar, int on_device) {
  if (!ctx || !xbar || !bbar) return GP_EINVAL;
  gp_status st = ready(ctx);
  if (st) return st;
  Geo &G = ctx->geo[0];
  if ((st = copy_in(ctx, ctx->adj[0].x, xbar, G.n, on_device))) return st;
  apply_cycle_t(ctx);
  GP_HIP(hipGetLastError());
  return copy_out(ctx, bbar, ctx->adj[0].b, G.n, on_device);
}

extern "C" gp_status gp_adjoint_solve(gp_ctx *ctx, const double *g, double *lam, int on_device, double tol, int max_cycles,
                                      gp_stats *stats) {
  if (!ctx || !g || !lam || !(tol > 0) || max_cycles < 0) return GP_EINVAL;
  gp_status st = ready(ctx);
  if (st) return st;
  Geo &G = ctx->geo[0];
  if ((st = copy_in(ctx, ctx->a_g, g, G.n, on_device))) return st;
  k_fill0<<<nblk(G.n), TPB, 0, ctx->stream>>>(ctx->a_lam, G.n);
  gp_status out = adjoint_solve_dev(ctx, tol, max_cycles, stats);
  if (out != GP_OK && out != GP_ENOCONV) return out;
  if ((st = copy_out(ctx, lam, ctx->a_lam, G.n, on_device))) return st;
  return out;
}
