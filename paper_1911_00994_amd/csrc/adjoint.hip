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

// grid sums over two kernels: each block of the producer writes its block sum to part[blockIdx.x]; one block of
// the next kernel adds part[0, np) in a fixed order.  The kernel boundary orders the two, where the ticket of
// alast_total costs a device-scope fence per block (an L2 write-back on a chip of several L2s) and a contended
// atomic, which grows with the grid.
__device__ void ablock_part(double v, double *part) {
  const double bs = ablock_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = bs;
}
__device__ double apart_total(const double *__restrict__ part, int np) {
  double v = 0;
  for (int q = threadIdx.x; q < np; q += TPB) v += part[q];
  return ablock_sum(v);
}
__global__ void __launch_bounds__(TPB) k_part_total(const double *__restrict__ part, int np, double *out, int add) {
  const double t = apart_total(part, np);
  if (threadIdx.x == 0) *out = add ? *out + t : t;
}

// ---------------------------------------------------------------------------------------------------------
// y = base + sgn * M^T lam.  Point part: each unknown gathers the coefficients of the internal momentum and
// continuity rows, the wall identity row and the mean row that reference it.
// ---------------------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(TPB) k_mt_pts(int N, int W, double h, double a, double d, const uint8_t *__restrict__ cls,
                                                const double *__restrict__ lam, const double *base, double sgn, double *y,
                                                double inv_mp, const double *__restrict__ part, int np) {
  const int WW = W * W;
  if (blockIdx.x == 0) {  // the xi entry: k_mt_xi's partials
    const double tot = apart_total(part, np);
    if (threadIdx.x == 0) y[3 * WW] = base[3 * WW] - sgn * tot;
  }
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
// ghost rows: y[col] += sgn * w * lam_G, gathered per column from the ghost-row table
__global__ void k_gt_mt(const int *__restrict__ tl, const int *__restrict__ off, const int *__restrict__ ent,
                        const int *__restrict__ nt, const int *__restrict__ pt, const double *__restrict__ w,
                        const double *__restrict__ lam, double sgn, double *y) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= *nt) return;
  double acc = 0;
  for (int q = off[s]; q < off[s + 1]; q++) {
    const int e = ent[q];
    acc += w[e] * (sgn * lam[pt[e / 9]]);
  }
  y[tl[s]] += acc;
}
// xi column: -1 in every internal continuity row
__global__ void __launch_bounds__(TPB) k_mt_xi(int W, const uint8_t *__restrict__ cls, const double *__restrict__ lam,
                                               double *part) {
  const int WW = W * W;
  double s = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < WW; t += gridDim.x * blockDim.x)
    if (cls[2 * WW + t] == K_INT) s += lam[2 * WW + t];
  ablock_part(s, part);
}

// ---------------------------------------------------------------------------------------------------------
// transposed box colour.  Free unknowns F of the box (internal ones); s = A_F^{-T} y solved as S A_F^{-1} S y
// with the closed form of the forward box solve (fixed unknowns enter with zero); then bbar_F += s, xbar_F = 0,
// and the box's five values go to S (zero for fixed unknowns).  k_box_adj_g then forms xbar_k -= M_{F,k} s for the
// columns outside F as a gather: every point adds, in a fixed order, the terms of the colour's boxes whose rows
// reference it (same-colour boxes share read-only neighbours, never unknowns, so an unknown of F gathers nothing).
// The xi column collects sum of s_P (grid sum, added to xbar_xi by the last block).
// ---------------------------------------------------------------------------------------------------------
// the scatter of the transposed box colour as a gather.  A box at cell c with values sW, sE, sS, sN, sP (its W, E,
// S, N faces and pressure) adds to the points c + o of the terms below (coefficient, and a condition on the box's
// own unknowns where a face or the pressure is a fixed unknown of the box); point q gathers them from the boxes
// c = q - o of the colour.
//   u:  sW a at -1, -W, +W and at +1 (E fixed);  sE a at +2, +1-W, +1+W and at 0 (W fixed);
//       sP -1/h at +1 (E fixed), +1/h at 0 (W fixed)
//   v:  sS a at -W, -1, +1 and at +W (N fixed);  sN a at +2W, +W-1, +W+1 and at 0 (S fixed);
//       sP -1/h at +W (N fixed), +1/h at 0 (S fixed)
//   p:  sW +1/h at -1, -1/h at 0 (P fixed);  sE -1/h at +1, +1/h at 0 (P fixed);  sS +1/h at -W, -1/h at 0 (P fixed);
//       sN -1/h at +W, +1/h at 0 (P fixed)
template <bool CMP>
__device__ __forceinline__ double box_gather(int N, int W, double ih, double a, const uint8_t *__restrict__ cls,
                                             const double *__restrict__ S, int colour, int t) {
  const int WW = W * W, K = N / 5 + 1, sst = CMP ? K * N : WW;
  const int g = t / WW, q = t - g * WW;
  const double *sW = S, *sE = S + sst, *sS = S + 2 * sst, *sN = S + 3 * sst, *sP = S + 4 * sst;
  const int qi = q % W - 1, qj = q / W - 1;
  // the box at cell (qi - di, qj - dj) has the colour when di + 2 dj = m (mod 5)
  const int m = ((qi + 2 * qj - colour) % 5 + 5) % 5;
  // index in S of that box (cell q - o, o = dj W + di; or its slot j K + i / 5 in the per-colour layout), or -1
  // when it is outside the grid or of another colour
  auto at = [&](int di, int dj) -> int {
    const int i = qi - di, j = qj - dj;
    if (m != ((di + 2 * dj) % 5 + 5) % 5 || i < 0 || i >= N || j < 0 || j >= N) return -1;
    return CMP ? j * K + (int)((unsigned)i / 5u) : q - dj * W - di;
  };
  auto fixed = [&](int k) { return cls[k] != K_INT; };
  double acc = 0;
  int k;
  if (g == 0) {
    const bool fq = fixed(q);
    if ((k = at(-1, 0)) >= 0) acc += a * sW[k];
    if ((k = at(0, -1)) >= 0) acc += a * sW[k];
    if ((k = at(0, 1)) >= 0) acc += a * sW[k];
    if ((k = at(1, 0)) >= 0 && fq) acc += a * sW[k];  // E face of box q - 1 is q
    if ((k = at(2, 0)) >= 0) acc += a * sE[k];
    if ((k = at(1, -1)) >= 0) acc += a * sE[k];
    if ((k = at(1, 1)) >= 0) acc += a * sE[k];
    if ((k = at(0, 0)) >= 0 && fq) acc += a * sE[k];  // W face of box q is q
    if ((k = at(1, 0)) >= 0 && fq) acc += -ih * sP[k];
    if ((k = at(0, 0)) >= 0 && fq) acc += ih * sP[k];
  } else if (g == 1) {
    const bool fq = fixed(WW + q);
    if ((k = at(0, -1)) >= 0) acc += a * sS[k];
    if ((k = at(-1, 0)) >= 0) acc += a * sS[k];
    if ((k = at(1, 0)) >= 0) acc += a * sS[k];
    if ((k = at(0, 1)) >= 0 && fq) acc += a * sS[k];  // N face of box q - W is q
    if ((k = at(0, 2)) >= 0) acc += a * sN[k];
    if ((k = at(-1, 1)) >= 0) acc += a * sN[k];
    if ((k = at(1, 1)) >= 0) acc += a * sN[k];
    if ((k = at(0, 0)) >= 0 && fq) acc += a * sN[k];  // S face of box q is q
    if ((k = at(0, 1)) >= 0 && fq) acc += -ih * sP[k];
    if ((k = at(0, 0)) >= 0 && fq) acc += ih * sP[k];
  } else {
    const bool pf = fixed(2 * WW + q);
    if ((k = at(-1, 0)) >= 0) acc += ih * sW[k];
    if ((k = at(0, 0)) >= 0 && pf) acc += -ih * sW[k];
    if ((k = at(1, 0)) >= 0) acc += -ih * sE[k];
    if ((k = at(0, 0)) >= 0 && pf) acc += ih * sE[k];
    if ((k = at(0, -1)) >= 0) acc += ih * sS[k];
    if ((k = at(0, 0)) >= 0 && pf) acc += -ih * sS[k];
    if ((k = at(0, 1)) >= 0) acc += -ih * sN[k];
    if ((k = at(0, 0)) >= 0 && pf) acc += ih * sN[k];
  }
  return acc;
}
// the transposed solve of the box at cell (i, j); its five values go to S[f sst + si] for the faces f = W, E, S, N
// and the pressure, and the return value is sP (for the xi column)
__device__ __forceinline__ double box_adj(int W, const BoxK &BK, const uint8_t *__restrict__ cls, double *xb, double *bb,
                                          double *S, int si, int sst, int i, int j) {
  const int WW = W * W, c = (j + 1) * W + (i + 1);
  const int k0 = c, k1 = c + 1, k2 = WW + c, k3 = WW + c + W, k4 = 2 * WW + c;
  // every load up front (all five indices are points of the level), so that they are in flight together
  const uint8_t c0 = cls[k0], c1 = cls[k1], c2 = cls[k2], c3 = cls[k3], c4 = cls[k4];
  const double x0 = xb[k0], x1 = xb[k1], x2 = xb[k2], x3 = xb[k3], x4 = xb[k4];
  const double b0 = bb[k0], b1 = bb[k1], b2 = bb[k2], b3 = bb[k3], b4 = bb[k4];
  const bool fW = c0 == K_INT, fE = c1 == K_INT, fS = c2 == K_INT, fN = c3 == K_INT, fP = c4 == K_INT;
  if (!(fW || fE || fS || fN || fP)) {
    for (int f = 0; f < 5; f++) S[f * sst + si] = 0.0;
    return 0.0;
  }
  // right-hand side S y
  const double rW = fW ? x0 : 0.0, rE = fE ? x1 : 0.0, rS = fS ? x2 : 0.0, rN = fN ? x3 : 0.0, rP = fP ? -x4 : 0.0;
  double aW = 0, bW = 0, aE = 0, bE = 0, aS = 0, bS = 0, aN = 0, bN = 0;
  if (fW && fE) {
    aW = BK.q1 * rW + BK.q2 * rE;
    bW = -BK.bp;
    aE = BK.q2 * rW + BK.q1 * rE;
    bE = BK.bp;
  } else if (fW) {
    aW = rW * BK.id;
    bW = -BK.ihd;
  } else if (fE) {
    aE = rE * BK.id;
    bE = BK.ihd;
  }
  if (fS && fN) {
    aS = BK.q1 * rS + BK.q2 * rN;
    bS = -BK.bp;
    aN = BK.q2 * rS + BK.q1 * rN;
    bN = BK.bp;
  } else if (fS) {
    aS = rS * BK.id;
    bS = -BK.ihd;
  } else if (fN) {
    aN = rN * BK.id;
    bN = BK.ihd;
  }
  double zP = 0;
  if (fP) {
    const double den = bE - bW + bN - bS;
    if (den == 0.0) {  // the forward sweep skips this box
      for (int f = 0; f < 5; f++) S[f * sst + si] = 0.0;
      return 0.0;
    }
    zP = (BK.h * rP - (aE - aW + aN - aS)) / den;
  }
  const double sW = fW ? aW + bW * zP : 0.0, sE = fE ? aE + bE * zP : 0.0, sS = fS ? aS + bS * zP : 0.0,
               sN = fN ? aN + bN * zP : 0.0, sP = fP ? -zP : 0.0;
  if (fW) {
    bb[k0] = b0 + sW;
    xb[k0] = 0;
  }
  if (fE) {
    bb[k1] = b1 + sE;
    xb[k1] = 0;
  }
  if (fS) {
    bb[k2] = b2 + sS;
    xb[k2] = 0;
  }
  if (fN) {
    bb[k3] = b3 + sN;
    xb[k3] = 0;
  }
  if (fP) {
    bb[k4] = b4 + sP;
    xb[k4] = 0;
  }
  S[si] = sW;
  S[sst + si] = sE;
  S[2 * sst + si] = sS;
  S[3 * sst + si] = sN;
  S[4 * sst + si] = sP;
  return sP;
}
// one colour over all cells (list == nullptr) or over the band cells list[lo, hi)
__global__ void __launch_bounds__(TPB) k_box_adj(int N, int W, BoxK BK, const uint8_t *__restrict__ cls,
                                                 double *xb, double *bb, double *S, int colour, const int *__restrict__ list,
                                                 int lo, int hi, double *part) {
  // all cells, one a thread (the boxes of the colour, one in five, read neighbouring cache lines together)
  const long total = list ? (long)(hi - lo) : (long)N * N;
  double sp = 0;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    int i, j;
    if (list) {
      int cell = list[lo + t];
      i = cell % N;
      j = cell / N;
    } else {
      j = (int)(t / N);
      i = (int)(t - (long)j * N);
      if ((i + 2 * j) % 5 != colour) continue;
    }
    sp += box_adj(W, BK, cls, xb, bb, S, (j + 1) * W + (i + 1), W * W, i, j);
  }
  ablock_part(sp, part);
}
__global__ void __launch_bounds__(TPB) k_box_adj_g(int N, int W, double ih, double a, const uint8_t *__restrict__ cls,
                                                   const double *__restrict__ S, int colour, double *xb,
                                                   const double *__restrict__ part, int np) {
  if (blockIdx.x == 0) {  // the xi column: k_box_adj's partials of sP
    const double tot = apart_total(part, np);
    if (threadIdx.x == 0) xb[3 * W * W] += tot;
  }
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * W * W) return;
  const double acc = box_gather<false>(N, W, ih, a, cls, S, colour, t);
  if (acc != 0.0) xb[t] += acc;
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
// xbar[col] -= w * t, gathered per column from the ghost-row table
__global__ void k_gt_sweep(const int *__restrict__ tl, const int *__restrict__ off, const int *__restrict__ ent,
                           const int *__restrict__ nt, const double *__restrict__ w, const double *__restrict__ tmp,
                           double *xb) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= *nt) return;
  double acc = 0;
  for (int q = off[s]; q < off[s + 1]; q++) {
    const int e = ent[q];
    acc += -w[e] * tmp[e / 9];
  }
  if (acc != 0.0) xb[tl[s]] += acc;
}

// transposed coupled boxes of one colour.  Forward: x_k <- x_k + sum_c Ainv[a_k][c] r_c over the written slots k of
// each box, r = b - M x on the box's rows, all boxes of the colour from the same x.  Transposed: t_c = sum over the
// written slots k of Ainv[a_k][c] xbar_k (all boxes first), then bbar on row c += t_c and xbar -= t_c (row c of M).
// t of the slots [lo, hi), XL lanes per slot (a fixed shuffle tree adds their parts), and the xi column: the sum of
// t over the slots on internal continuity rows, added to xbar_xi by the last block
constexpr int XL = 8;
__global__ void __launch_bounds__(TPB) k_xbt_t(int lo, int hi, int W, const uint8_t *__restrict__ cls,
                                               const int *__restrict__ idx, const int *__restrict__ box,
                                               const int *__restrict__ off, const int *__restrict__ ioff,
                                               const uint8_t *__restrict__ wr, const uint8_t *__restrict__ ok,
                                               const double *__restrict__ inv, double *xb, double *t, double *part) {
  const int WW = W * W;
  const long n = (long)XL * (hi - lo);
  double acc = 0;
  for (long g0 = (long)blockIdx.x * blockDim.x; g0 < n; g0 += (long)gridDim.x * blockDim.x) {
    const long g = g0 + threadIdx.x;
    const int s = lo + (int)(g / XL), ln = (int)(g % XL);
    double v = 0;
    if (g < n) {
      const int bx = box[s], o = off[bx], m = off[bx + 1] - o, c = s - o;
      if (ok[bx]) {
        const double *iv = inv + ioff[bx];
        for (int q = ln; q < m; q += XL) {
          const double w = iv[(size_t)q * m + c], xv = xb[idx[o + q]];  // idx is a point of the level for every slot
          if (wr[o + q]) v += w * xv;
        }
      }
    }
    for (int d = XL / 2; d > 0; d >>= 1) v += __shfl_xor(v, d);
    if (g < n && ln == 0) {
      t[s] = v;
      const int k = idx[s];
      if (k >= 2 * WW && cls[k] == K_INT) acc += v;
    }
  }
  ablock_part(acc, part);
}
// the scatter of the transposed coupled boxes as a gather over the slot table: entry z = 0 of slot s is bbar on its
// point (+t_s); entries z = 1.. are the columns of its row (xbar -= t_s times the row's coefficient): the internal
// momentum row (d on itself, -a on the four neighbours, the pressure difference / h), the internal continuity row
// (the four face differences / h; its -1 for xi is summed in k_xbt_t), or a ghost row (its 9 weights)
__device__ __forceinline__ double xt_coef(int k, int z, int W, double h, double a, double d,
                                          const uint8_t *__restrict__ cls, const int *__restrict__ g_rowof,
                                          const double *__restrict__ g_w) {
  const int WW = W * W;
  if (cls[k] != K_INT) return -g_w[9 * g_rowof[k] + z - 1];
  const double ih = 1.0 / h;
  if (k / WW < 2) return z == 1 ? -d : (z <= 5 ? a : (z == 6 ? -ih : ih));
  return (z & 1) ? -ih : ih;
}
// the xi column of the transposed coupled boxes: xbar_xi += sum of t_s over the internal continuity slots of
// [lo, hi) (block partials in slot order, summed by the last block)
// the coefficient of every entry of a coupled-box table (the slot's row, column z), for k_xt_apply
__global__ void k_xt_coef(int lo, const int *__restrict__ off, const int *__restrict__ ent, const int *__restrict__ nt,
                          int W, double h, double a, double d, const uint8_t *__restrict__ cls,
                          const int *__restrict__ idx, const int *__restrict__ g_rowof, const double *__restrict__ g_w,
                          double *coef) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= *nt) return;
  for (int q = off[s]; q < off[s + 1]; q++) {
    const int e = ent[q], sl = lo + e / 10, z = e % 10;
    coef[q] = z == 0 ? 1.0 : xt_coef(idx[sl], z, W, h, a, d, cls, g_rowof, g_w);
  }
}
__global__ void __launch_bounds__(TPB) k_xt_apply(int lo, const int *__restrict__ tl, const int *__restrict__ off,
                                                  const int *__restrict__ ent, const int *__restrict__ nt,
                                                  const double *__restrict__ coef, const double *__restrict__ t,
                                                  double *xb, double *bb, int W, const double *__restrict__ part,
                                                  int np) {
  if (blockIdx.x == 0) {  // the xi column: k_xbt_t's partials
    const double tot = apart_total(part, np);
    if (threadIdx.x == 0) xb[3 * W * W] += tot;
  }
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= *nt) return;
  double accb = 0, accx = 0;
  bool any = false;
  for (int q = off[s]; q < off[s + 1]; q++) {
    const int e = ent[q];
    const double v = t[lo + e / 10], w = coef[q];
    if (v == 0.0) continue;
    any = true;
    if (e % 10 == 0)
      accb += v;
    else
      accx += w * v;
  }
  if (any) {
    bb[tl[s]] += accb;
    xb[tl[s]] += accx;
  }
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

// One transposed relaxation of a small level in one workgroup: the xi update, the lambda ghost sweeps and the box
// colours 4..0 of relax_t, with xbar, bbar, the classes, the ghost sweep's row values and the box values in LDS
// (the box values of one colour in the per-colour layout, slot j K + i / 5) and a barrier after every grid-wide
// step.  On a small level the separate launches (about 16 per relaxation) cost more than their work.
constexpr int RT_T = 1024;
struct RelaxT {
  int N, W, lam, ng;
  BoxK BK;
  double inv_mp;
  const uint8_t *cls;
  const int *g_pt, *tl, *off, *ent, *nt;
  const double *g_dtau, *g_w;
  double *xb, *bb;
};
// LDS bytes of k_relax_t_wg on a level of size N
inline size_t relax_t_lds(int N, int ng) {
  const size_t W = N + 2, WW = W * W, K = N / 5 + 1;
  return (6 * WW + 1 + 5 * K * N + ng) * sizeof(double) + ((3 * WW + 15) & ~(size_t)15);
}
__global__ void __launch_bounds__(RT_T) k_relax_t_wg(RelaxT P) {
  extern __shared__ __align__(16) unsigned char rt_lds[];
  __shared__ double red[RT_T / 64];
  const int tid = threadIdx.x, N = P.N, W = P.W, WW = W * W, K = N / 5 + 1, KN = K * N;
  double *xs = reinterpret_cast<double *>(rt_lds);
  double *bb = xs + 3 * WW + 1;
  double *Sc = bb + 3 * WW;
  double *gt = Sc + 5 * KN;
  uint8_t *cl = reinterpret_cast<uint8_t *>(gt + P.ng);
  for (int t = tid; t <= 3 * WW; t += RT_T) xs[t] = P.xb[t];
  for (int t = tid; t < 3 * WW; t += RT_T) {
    bb[t] = P.bb[t];
    cl[t] = P.cls[t];
  }
  __syncthreads();
  // xi: take xibar, then its contributions to the divergence columns and the continuity right-hand sides
  const double c = xs[3 * WW] * P.inv_mp, ih = P.BK.ih;
  __syncthreads();
  if (tid == 0) xs[3 * WW] = 0.0;
  if (c != 0.0) {
    const uint8_t *cp = cl + 2 * WW;
    for (int t = tid; t < 3 * WW; t += RT_T) {
      const int g = t / WW, q = t - g * WW, j = q / W - 1, i = q % W - 1;
      if (g == 0) {
        const double f = (i - 1 >= -1 && cp[q - 1] == K_INT ? 1.0 : 0.0) - (cp[q] == K_INT ? 1.0 : 0.0);
        if (f != 0.0) xs[t] += f * c / P.BK.h;
      } else if (g == 1) {
        const double f = (j - 1 >= -1 && cp[q - W] == K_INT ? 1.0 : 0.0) - (cp[q] == K_INT ? 1.0 : 0.0);
        if (f != 0.0) xs[t] += f * c / P.BK.h;
      } else if (cp[q] == K_INT) {
        bb[t] -= c;
      }
    }
  }
  __syncthreads();
  // ghost sweeps: t = dtau xbar_G, bbar_G += t, then xbar -= B^T t gathered per column
  if (P.ng) {
    const int nt = *P.nt;
    for (int it = 0; it < P.lam; it++) {
      for (int r = tid; r < P.ng; r += RT_T) {
        const double t = P.g_dtau[r] * xs[P.g_pt[r]];
        gt[r] = t;
        bb[P.g_pt[r]] += t;
      }
      __syncthreads();
      for (int s = tid; s < nt; s += RT_T) {
        double acc = 0;
        for (int q = P.off[s]; q < P.off[s + 1]; q++) {
          const int e = P.ent[q];
          acc += -P.g_w[e] * gt[e / 9];
        }
        if (acc != 0.0) xs[P.tl[s]] += acc;
      }
      __syncthreads();
    }
  }
  // box colours 4..0: the box solves of the colour, then the gather of their scatter
  for (int colour = 4; colour >= 0; colour--) {
    double sp = 0;
    for (int t = tid; t < KN; t += RT_T) {
      const int j = t / K, kk = t - j * K;
      const int i = ((colour - 2 * j) % 5 + 5) % 5 + 5 * kk;
      if (i < N) sp += box_adj(W, P.BK, cl, xs, bb, Sc, t, KN, i, j);
    }
    for (int o = 32; o > 0; o >>= 1) sp += __shfl_xor(sp, o);
    if ((tid & 63) == 0) red[tid >> 6] = sp;
    __syncthreads();
    if (tid == 0) {
      double tot = 0;
      for (int w = 0; w < RT_T / 64; w++) tot += red[w];
      xs[3 * WW] += tot;
    }
    for (int t = tid; t < 3 * WW; t += RT_T) {
      const double acc = box_gather<true>(N, W, ih, P.BK.a, cl, Sc, colour, t);
      if (acc != 0.0) xs[t] += acc;
    }
    __syncthreads();
  }
  for (int t = tid; t <= 3 * WW; t += RT_T) P.xb[t] = xs[t];
  for (int t = tid; t < 3 * WW; t += RT_T) P.bb[t] = bb[t];
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

// transposed extension fill (sources are internal or ghost points, never extension points): every source gathers
// w * xbar of the extension points that read it (table entries 3 e + q), then the extension points' xbar are zeroed
__global__ void k_et_apply(const int *__restrict__ tl, const int *__restrict__ off, const int *__restrict__ ent,
                           const int *__restrict__ nt, const int *__restrict__ e_pt, const double *__restrict__ e_w,
                           double *xb) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= *nt) return;
  double acc = 0;
  for (int q = off[s]; q < off[s + 1]; q++) {
    const int e = ent[q];
    acc += e_w[e] * xb[e_pt[e / 3]];
  }
  if (acc != 0.0) xb[tl[s]] += acc;
}
__global__ void k_et_zero(const int *__restrict__ e_pt, const int *__restrict__ e_src, int ne, double *xb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne || e_src[3 * e] < 0) return;
  xb[e_pt[e]] = 0.0;
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
                                                  double *part) {
  const int WW = W * W;
  double s = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < WW; t += gridDim.x * blockDim.x) {
    uint8_t c = cls[2 * WW + t];
    if (c == K_INT || c == K_GHOST || c == K_GHOSTX) s += xb[2 * WW + t];
  }
  ablock_part(s, part);
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
// transposed scatter tables (TTab): entry targets, then count, list, offsets, fill and per-target sort
// ---------------------------------------------------------------------------------------------------------
namespace {
__global__ void k_izero(int *x, long n) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}
__global__ void k_tt_tgt_ghost(const int *__restrict__ col, int n, int *tgt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) tgt[e] = col[e];
}
__global__ void k_tt_tgt_ext(const int *__restrict__ src, int n, int *tgt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) tgt[e] = src[3 * (e / 3)] < 0 ? -1 : src[e];
}
// entries 10 (s - lo) + z of the slots s in [lo, lo + ns)
__global__ void k_tt_tgt_xb(int lo, int ns, int W, const uint8_t *__restrict__ cls, const int *__restrict__ idx,
                            const int *__restrict__ g_rowof, const int *__restrict__ g_col, int *tgt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 10 * ns) return;
  const int sl = lo + e / 10, z = e % 10, k = idx[sl], WW = W * W;
  int t = -1;
  if (z == 0) {
    t = k;
  } else if (cls[k] != K_INT) {
    t = g_col[9 * g_rowof[k] + z - 1];
  } else {
    const int g = k / WW, q = k - g * WW;
    if (g < 2) {
      const int tt[7] = {k, k - 1, k + 1, k - W, k + W, 2 * WW + q, 2 * WW + q - (g == 0 ? 1 : W)};
      if (z <= 7) t = tt[z - 1];
    } else {
      // the xi column (every internal continuity row) is summed in k_xbt_t: a table segment that long would be
      // slow to order
      const int tt[4] = {q + 1, q, WW + q + W, WW + q};
      if (z <= 4) t = tt[z - 1];
    }
  }
  tgt[e] = t;
}
__global__ void k_tt_count(const int *__restrict__ tgt, int n, int *cnt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n && tgt[e] >= 0) atomicAdd(&cnt[tgt[e]], 1);
}
// the targets with entries, in any order (each target's sum does not depend on where it sits in the list)
__global__ void k_tt_list(const int *__restrict__ cnt, int T, int *tl, int *tc, int *pos, int *nt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T || cnt[t] == 0) return;
  const int sl = atomicAdd(nt, 1);
  tl[sl] = t;
  tc[sl] = cnt[t];
  pos[t] = sl;
}
// exclusive scan of the counts tc[0 .. nt) into off (one workgroup); cur (the fill cursors) cleared
__global__ void __launch_bounds__(1024) k_tt_scan(const int *__restrict__ nt_p, int *tc, int *off) {
  __shared__ int part[1024];
  const int nt = *nt_p, T = blockDim.x, tid = threadIdx.x;
  const int per = (nt + T - 1) / T, lo = tid * per, hi = min(nt, lo + per);
  int sum = 0;
  for (int q = lo; q < hi; q++) sum += tc[q];
  part[tid] = sum;
  __syncthreads();
  for (int o = 1; o < T; o <<= 1) {  // inclusive scan of the partials
    int v = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = part[tid] - sum;
  for (int q = lo; q < hi; q++) {
    const int c = tc[q];
    off[q] = run;
    run += c;
    tc[q] = 0;
  }
  if (tid == T - 1) off[nt] = part[T - 1];
}
__global__ void k_tt_fill(const int *__restrict__ tgt, int n, const int *__restrict__ pos, const int *__restrict__ off,
                          int *cur, int *ent) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n || tgt[e] < 0) return;
  const int sl = pos[tgt[e]];
  ent[off[sl] + atomicAdd(&cur[sl], 1)] = e;
}
// each target's entries in ascending order of their keys; the point counts cleared for the next table.  The key of
// entry e is e, or with `pt` given pt[e / K] K + e % K: the entry's item named by its point, so that the order does
// not depend on how a geometry build numbered the items (ghost rows and extension points are numbered in the order
// a compaction met them)
__global__ void k_tt_sort(const int *__restrict__ nt_p, const int *__restrict__ tl, const int *__restrict__ off,
                          const int *__restrict__ pt, int K, int *ent, int *cnt) {
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= *nt_p) return;
  const int lo = off[sl], hi = off[sl + 1];
  auto key = [&](int e) { return pt ? pt[e / K] * K + e % K : e; };
  for (int q = lo + 1; q < hi; q++) {
    const int v = ent[q], kv = key(v);
    int r = q - 1;
    while (r >= lo && key(ent[r]) > kv) {
      ent[r + 1] = ent[r];
      r--;
    }
    ent[r + 1] = v;
  }
  cnt[tl[sl]] = 0;
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
  GP_HIP(hipMalloc((void **)&ctx->a_S, 5 * (size_t)ctx->geo[0].WW * sizeof(double)));
  GP_HIP(hipGetLastError());
  return GP_OK;
}

static void ifree(int *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// regroup the entries whose targets the launch `tgt_fn` writes into ctx->tt_tgt (n entries, targets below T)
template <class F>
static gp_status tt_build(Ctx *ctx, TTab &tab, int n, int T, const int *pt, int K, F tgt_fn) {
  hipStream_t s = ctx->stream;
  tab.ne = n;
  if (n == 0) return GP_OK;
  if (T > ctx->tt_ccap) {
    ifree(ctx->tt_cnt);
    ifree(ctx->tt_pos);
    GP_HIP(hipMalloc((void **)&ctx->tt_cnt, (size_t)T * sizeof(int)));
    GP_HIP(hipMalloc((void **)&ctx->tt_pos, (size_t)T * sizeof(int)));
    k_izero<<<nblk(T), TPB, 0, s>>>(ctx->tt_cnt, T);
    ctx->tt_ccap = T;
  }
  if (n > ctx->tt_tcap) {
    ifree(ctx->tt_tgt);
    GP_HIP(hipMalloc((void **)&ctx->tt_tgt, (size_t)n * sizeof(int)));
    ctx->tt_tcap = n;
  }
  const int mt = std::min(n, T);
  if (mt + 1 > tab.cap_t) {
    ifree(tab.tl);
    ifree(tab.off);
    ifree(tab.cur);
    GP_HIP(hipMalloc((void **)&tab.tl, (size_t)(mt + 1) * sizeof(int)));
    GP_HIP(hipMalloc((void **)&tab.off, (size_t)(mt + 2) * sizeof(int)));
    GP_HIP(hipMalloc((void **)&tab.cur, (size_t)(mt + 1) * sizeof(int)));
    tab.cap_t = mt + 1;
  }
  if (n > tab.cap_e) {
    ifree(tab.ent);
    GP_HIP(hipMalloc((void **)&tab.ent, (size_t)n * sizeof(int)));
    tab.cap_e = n;
  }
  if (!tab.d_nt) GP_HIP(hipMalloc((void **)&tab.d_nt, sizeof(int)));
  tgt_fn(ctx->tt_tgt);
  k_tt_count<<<nblk(n), TPB, 0, s>>>(ctx->tt_tgt, n, ctx->tt_cnt);
  k_izero<<<1, 1, 0, s>>>(tab.d_nt, 1);
  k_tt_list<<<nblk(T), TPB, 0, s>>>(ctx->tt_cnt, T, tab.tl, tab.cur, ctx->tt_pos, tab.d_nt);
  k_tt_scan<<<1, 1024, 0, s>>>(tab.d_nt, tab.cur, tab.off);
  k_tt_fill<<<nblk(n), TPB, 0, s>>>(ctx->tt_tgt, n, ctx->tt_pos, tab.off, tab.cur, tab.ent);
  k_tt_sort<<<nblk(mt), TPB, 0, s>>>(tab.d_nt, tab.tl, tab.off, pt, K, tab.ent, ctx->tt_cnt);
  GP_HIP(hipGetLastError());
  return GP_OK;
}

// the transposed scatter tables of every level for its current geometry
static gp_status ensure_tabs(Ctx *ctx) {
  hipStream_t s = ctx->stream;
  for (int l = 0; l < ctx->L; l++) {
    Geo &G = ctx->geo[l];
    AdjTabs &A = ctx->atab[l];
    if (A.gen == G.gen) continue;
    const int T = 3 * G.WW + 1;
    gp_status st = tt_build(ctx, A.gt, 9 * G.ng, T, G.g_pt, 9, [&](int *tgt) {
      k_tt_tgt_ghost<<<nblk(9 * G.ng), TPB, 0, s>>>(G.g_col, 9 * G.ng, tgt);
    });
    if (st) return st;
    st = tt_build(ctx, A.et, 3 * G.ne, T, G.e_pt, 3, [&](int *tgt) {
      k_tt_tgt_ext<<<nblk(3 * G.ne), TPB, 0, s>>>(G.e_src, 3 * G.ne, tgt);
    });
    if (st) return st;
    const bool xb = ctx->prm.ghost_boxes && G.nxb;
    for (int c = 0; c < 5; c++) {
      const int lo = G.xb_soff[c], ns = xb ? G.xb_soff[c + 1] - lo : 0;
      st = tt_build(ctx, A.xt[c], 10 * ns, T, nullptr, 10, [&](int *tgt) {
        k_tt_tgt_xb<<<nblk(10 * ns), TPB, 0, s>>>(lo, ns, G.W, G.cls, G.xb_idx, G.g_rowof, G.g_col, tgt);
      });
      if (st) return st;
      TTab &X = A.xt[c];
      if (X.ne > X.cap_c) {
        if (X.coef) (void)hipFree(X.coef);
        X.coef = nullptr;
        X.cap_c = 0;
        GP_HIP(hipMalloc((void **)&X.coef, (size_t)X.ne * sizeof(double)));
        X.cap_c = X.ne;
      }
    }
    A.xok = false;
    A.gen = G.gen;
  }
  return GP_OK;
}
void adjoint_free_tabs(Ctx *ctx) {
  for (int l = 0; l < MAXLEV; l++)
    for (TTab *t : {&ctx->atab[l].gt, &ctx->atab[l].et, &ctx->atab[l].xt[0], &ctx->atab[l].xt[1], &ctx->atab[l].xt[2],
                     &ctx->atab[l].xt[3], &ctx->atab[l].xt[4]}) {
      ifree(t->tl);
      ifree(t->off);
      ifree(t->ent);
      ifree(t->cur);
      ifree(t->d_nt);
      if (t->coef) (void)hipFree(t->coef);
      *t = TTab();
    }
  ifree(ctx->tt_cnt);
  ifree(ctx->tt_pos);
  ifree(ctx->tt_tgt);
  ctx->tt_ccap = ctx->tt_tcap = 0;
  for (int l = 0; l < MAXLEV; l++) ctx->atab[l].xok = false;
  if (ctx->a_S) (void)hipFree(ctx->a_S);
  ctx->a_S = nullptr;
}
// launch size covering every target of a table
static inline int tt_blocks(const TTab &t, int T) { return nblk(std::min(t.ne, T)); }

// transposed extension fill of level l on x
static void ext_fill_t(Ctx *ctx, int l, double *x) {
  Geo &G = ctx->geo[l];
  const TTab &E = ctx->atab[l].et;
  if (!G.ne || !E.ne) return;
  hipStream_t s = ctx->stream;
  k_et_apply<<<tt_blocks(E, 3 * G.WW + 1), TPB, 0, s>>>(E.tl, E.off, E.ent, E.d_nt, G.e_pt, G.e_w, x);
  k_et_zero<<<nblk(G.ne), TPB, 0, s>>>(G.e_pt, G.e_src, G.ne, x);
}

static inline double coef_a_l(Ctx *ctx, int l) { return ctx->alpha / (ctx->geo[l].h * ctx->geo[l].h); }

// y = base + sgn M^T lam on level l
static void mt_apply(Ctx *ctx, int l, const double *lam, const double *base, double sgn, double *y) {
  Geo &G = ctx->geo[l];
  hipStream_t s = ctx->stream;
  double a = coef_a_l(ctx, l), d = 1.0 + 4.0 * a;
  // every entry of y is written by one thread from the same entry of base, so y may alias base
  const int np = std::min(ARED, nblk(G.WW));
  k_mt_xi<<<np, TPB, 0, s>>>(G.W, G.cls, lam, ctx->d_red);
  k_mt_pts<<<nblk(3L * G.WW), TPB, 0, s>>>(G.N, G.W, G.h, a, d, G.cls, lam, base, sgn, y, 1.0 / G.mp, ctx->d_red, np);
  const TTab &GT = ctx->atab[l].gt;
  if (G.ng && GT.ne)
    k_gt_mt<<<tt_blocks(GT, 3 * G.WW + 1), TPB, 0, s>>>(GT.tl, GT.off, GT.ent, GT.d_nt, G.g_pt, G.g_w, lam, sgn, y);
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
    total = (long)G.N * G.N;
  }
  int nb = std::min(4096, nblk(total));
  // a band colour writes the values of its listed boxes only: the others of the colour must read zero
  if (band) k_fill0<<<nblk(5L * G.WW), TPB, 0, ctx->stream>>>(ctx->a_S, 5L * G.WW);
  k_box_adj<<<nb, TPB, 0, ctx->stream>>>(G.N, G.W, box_consts(G.h, a, d), G.cls, A.x, A.b, ctx->a_S, colour, list, lo, hi,
                                         ctx->d_red);
  k_box_adj_g<<<nblk(3L * G.WW), TPB, 0, ctx->stream>>>(G.N, G.W, 1.0 / G.h, a, G.cls, ctx->a_S, colour, A.x, ctx->d_red,
                                                        nb);
}

static void ghost_sweep_t(Ctx *ctx, int l) {
  Geo &G = ctx->geo[l];
  if (!G.ng) return;
  Vec<double> &A = ctx->adj[l];
  k_gadj_a<<<nblk(G.ng), TPB, 0, ctx->stream>>>(G.g_pt, G.g_dtau, G.ng, A.x, A.b, ctx->gtmp);
  const TTab &GT = ctx->atab[l].gt;
  k_gt_sweep<<<tt_blocks(GT, 3 * G.WW + 1), TPB, 0, ctx->stream>>>(GT.tl, GT.off, GT.ent, GT.d_nt, G.g_w, ctx->gtmp, A.x);
}

// reverse of the coupled boxes of level l (colours 4..0)
static void xb_relax_t(Ctx *ctx, int l) {
  Geo &G = ctx->geo[l];
  if (!ctx->prm.ghost_boxes || !G.nxb) return;
  Vec<double> &A = ctx->adj[l];
  hipStream_t s = ctx->stream;
  const double a = coef_a_l(ctx, l), d = 1.0 + 4.0 * a;
  AdjTabs &AT = ctx->atab[l];
  if (!AT.xok || AT.xa != a) {
    for (int c = 0; c < 5; c++) {
      const TTab &X = AT.xt[c];
      if (X.ne)
        k_xt_coef<<<tt_blocks(X, 3 * G.WW + 1), TPB, 0, s>>>(G.xb_soff[c], X.off, X.ent, X.d_nt, G.W, G.h, a, d, G.cls,
                                                            G.xb_idx, G.g_rowof, G.g_w, X.coef);
    }
    AT.xa = a;
    AT.xok = true;
  }
  for (int c = 4; c >= 0; c--) {
    const int lo = G.xb_soff[c], hi = G.xb_soff[c + 1];
    if (hi == lo) continue;
    const int np = std::min(ARED, nblk((long)XL * (hi - lo)));
    k_xbt_t<<<np, TPB, 0, s>>>(lo, hi, G.W, G.cls, G.xb_idx, G.xb_box, G.xb_off, G.xb_ioff, G.xb_wr, G.xb_ok, G.xb_inv,
                               A.x, G.xb_r, ctx->d_red);
    const TTab &X = ctx->atab[l].xt[c];
    if (X.ne)
      k_xt_apply<<<tt_blocks(X, 3 * G.WW + 1), TPB, 0, s>>>(lo, X.tl, X.off, X.ent, X.d_nt, X.coef, G.xb_r, A.x, A.b, G.W,
                                                           ctx->d_red, np);
    else
      k_part_total<<<1, TPB, 0, s>>>(ctx->d_red, np, A.x + 3 * (size_t)G.WW, 1);
  }
}

// reverse of: box colours 0..4, coupled boxes, lambda ghost sweeps, [band colours 0..4, lambda ghost sweeps] x
// bnd_sweeps, xi
// levels up to this size relax in one workgroup (k_relax_t_wg), when its LDS fits
constexpr int RT_MAXN = 32;

static void relax_t(Ctx *ctx, int l) {
  Geo &G = ctx->geo[l];
  Vec<double> &A = ctx->adj[l];
  hipStream_t s = ctx->stream;
  const bool band = ctx->prm.bnd_sweeps > 0 && G.nband > 0, xbx = ctx->prm.ghost_boxes && G.nxb;
  if (G.N <= RT_MAXN && !band && !xbx && relax_t_lds(G.N, G.ng) + 1024 <= ctx->max_lds) {
    const TTab &GT = ctx->atab[l].gt;
    RelaxT P;
    P.N = G.N;
    P.W = G.W;
    P.lam = ctx->prm.lambda_ghost;
    P.ng = G.ng;
    const double a = coef_a_l(ctx, l);
    P.BK = box_consts(G.h, a, 1.0 + 4.0 * a);
    P.inv_mp = 1.0 / G.mp;
    P.cls = G.cls;
    P.g_pt = G.g_pt;
    P.tl = GT.tl;
    P.off = GT.off;
    P.ent = GT.ent;
    P.nt = GT.d_nt;
    P.g_dtau = G.g_dtau;
    P.g_w = G.g_w;
    P.xb = A.x;
    P.bb = A.b;
    k_relax_t_wg<<<1, RT_T, relax_t_lds(G.N, G.ng), s>>>(P);
    return;
  }
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
  xb_relax_t(ctx, l);
  for (int c = 4; c >= 0; c--) box_colour_t(ctx, l, c, false);
}

static void cycle_t(Ctx *ctx, int l) {
  hipStream_t s = ctx->stream;
  if (l == ctx->L - 1) {
    Vec<double> &A = ctx->adj[l];
    k_coarse_t<<<ctx->nc, 64, 0, s>>>(ctx->c_inv, ctx->c_map, ctx->c_bmap, ctx->nc, A.x, A.b);
    k_zero_at<<<nblk(ctx->nc), TPB, 0, s>>>(ctx->c_map, ctx->nc, A.x);
    return;
  }
  Geo &F = ctx->geo[l], &C = ctx->geo[l + 1];
  Vec<double> &AF = ctx->adj[l], &AC = ctx->adj[l + 1];
  for (int q = 0; q < ctx->prm.nu2; q++) relax_t(ctx, l);
  k_prolong_adj<<<nblk(3L * C.WW + 1), TPB, 0, s>>>(F.N, F.W, F.cls, AF.x, C.N, C.W, AC.x);
  ext_fill_t(ctx, l + 1, AC.x);
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
  const int np = std::min(ARED, nblk(G.WW));
  k_mean_sum<<<np, TPB, 0, s>>>(G.W, G.cls, A.x, ctx->d_red);
  k_part_total<<<1, TPB, 0, s>>>(ctx->d_red, np, ctx->d_scal + 9, 0);
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
  gp_status st = ensure_xb(ctx);
  if (st) return st;
  if ((st = adjoint_alloc(ctx))) return st;
  return ensure_tabs(ctx);
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
  double kb = 0;
  gp_status out = GP_OK;
  if (ctx->prm.krylov > 0) {
    // GCR with the transposed cycle as the preconditioner (the transpose of the forward solve's iteration)
    if ((st = gcr_alloc(ctx))) return st;
    const long n = G.n;
    mt_apply(ctx, 0, ctx->a_lam, ctx->a_g, -1.0, ctx->kr.r);
    if ((st = absmax_dev(ctx, ctx->kr.r, n, &r0))) return st;
    GcrOps ops;
    ops.precond = [&](const double *r, double *z) {
      k_copy<<<nblk(n), TPB, 0, s>>>(A.x, r, n);
      apply_cycle_t(ctx);
      k_copy<<<nblk(n), TPB, 0, s>>>(z, A.b, n);
      k_mask_unknowns<<<nblk(3L * G.WW), TPB, 0, s>>>(3 * G.WW, G.cls, z);
    };
    ops.apply_neg = [&](const double *z, double *q) {
      mt_apply(ctx, 0, z, ctx->kr.zero, -1.0, q);
      k_mask_unknowns<<<nblk(3L * G.WW), TPB, 0, s>>>(3 * G.WW, G.cls, q);
    };
    ops.residual = [&](double *rinf) -> gp_status {
      mt_apply(ctx, 0, ctx->a_lam, ctx->a_g, -1.0, ctx->kr.r);
      return absmax_dev(ctx, ctx->kr.r, n, rinf);
    };
    int status = GP_OK;
    const double lim = 1e6 * (r0 > 1 ? r0 : 1);
    if ((st = gcr_solve(ctx, ctx->kr, ops, ctx->a_lam, ctx->kr.r, r0, thr, lim, max_cycles, &c, &r, &rho, &status,
                        &kb)))
      return st;
    out = status;
  }
  for (; ctx->prm.krylov == 0;) {
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
    stt->bytes_alg = c * cycle_bytes(ctx, false) + kb;
    stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return out;
}


// ---------------------------------------------------------------------------------------------------------
// reverse mode of the Crank-Nicolson step (Sect. 2): the right-hand side of step n on the internal momentum
// rows of Omega^{n+1} is u^n + alpha lap u^n + dt f - dt C with C = c^n + c^{n-1}/2 - c^{n-2}/2 (extrapolation)
// or C = (c^n + c(u^{n+1}))/2 (converged fixed-point iteration of the first two steps)
// ---------------------------------------------------------------------------------------------------------
namespace {

// xb += J_c(y)^T cbar: transpose of the Jacobian of c(u) = u du/dx + vbar du/dy (and its v counterpart) at the
// state y, gathered at every u and v node from the convection nodes whose stencil holds it
__global__ void k_conv_jt(int N, int W, double h, const double *__restrict__ y, const double *__restrict__ cbu,
                          const double *__restrict__ cbv, double *xb) {
  const int WW = W * W;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * WW) return;
  const int g = t / WW, q = t - g * WW, b = q / W - 1, a = q % W - 1;
  const double *U = y, *V = y + WW;
  auto in = [&](int i, int j) { return i >= -1 && i <= N && j >= -1 && j <= N; };
  auto CU = [&](int i, int j) { return in(i, j) ? cbu[aix(W, i, j)] : 0.0; };
  auto CV = [&](int i, int j) { return in(i, j) ? cbv[aix(W, i, j)] : 0.0; };
  auto Uv = [&](int i, int j) { return in(i, j) ? U[aix(W, i, j)] : 0.0; };
  auto Vv = [&](int i, int j) { return in(i, j) ? V[aix(W, i, j)] : 0.0; };
  auto vbar = [&](int i, int j) { return 0.25 * (Vv(i - 1, j) + Vv(i, j) + Vv(i - 1, j + 1) + Vv(i, j + 1)); };
  auto ubar = [&](int i, int j) { return 0.25 * (Uv(i, j - 1) + Uv(i + 1, j - 1) + Uv(i, j) + Uv(i + 1, j)); };
  const double i2h = 0.5 / h;
  double s = 0, c;
  if (g == 0) {
    if ((c = CU(a, b)) != 0.0) s += c * (Uv(a + 1, b) - Uv(a - 1, b)) * i2h;
    if ((c = CU(a - 1, b)) != 0.0) s += c * Uv(a - 1, b) * i2h;
    if ((c = CU(a + 1, b)) != 0.0) s -= c * Uv(a + 1, b) * i2h;
    if ((c = CU(a, b - 1)) != 0.0) s += c * vbar(a, b - 1) * i2h;
    if ((c = CU(a, b + 1)) != 0.0) s -= c * vbar(a, b + 1) * i2h;
    const int ci[4] = {a, a - 1, a, a - 1}, cj[4] = {b + 1, b + 1, b, b};
    for (int z = 0; z < 4; z++)
      if ((c = CV(ci[z], cj[z])) != 0.0) s += c * 0.25 * (Vv(ci[z] + 1, cj[z]) - Vv(ci[z] - 1, cj[z])) * i2h;
  } else {
    if ((c = CV(a, b)) != 0.0) s += c * (Vv(a, b + 1) - Vv(a, b - 1)) * i2h;
    if ((c = CV(a - 1, b)) != 0.0) s += c * ubar(a - 1, b) * i2h;
    if ((c = CV(a + 1, b)) != 0.0) s -= c * ubar(a + 1, b) * i2h;
    if ((c = CV(a, b - 1)) != 0.0) s += c * Vv(a, b - 1) * i2h;
    if ((c = CV(a, b + 1)) != 0.0) s -= c * Vv(a, b + 1) * i2h;
    const int ci[4] = {a + 1, a, a + 1, a}, cj[4] = {b, b, b - 1, b - 1};
    for (int z = 0; z < 4; z++)
      if ((c = CU(ci[z], cj[z])) != 0.0) s += c * 0.25 * (Uv(ci[z], cj[z] + 1) - Uv(ci[z], cj[z] - 1)) * i2h;
  }
  if (s != 0.0) xb[t] += s;
}

// from the adjoint lam of the step's right-hand side (P lam = lam on the internal momentum rows):
// xbn = P lam + alpha lap^T (P lam) (adjoint of u^n), fb += dt P lam, and the convection-history adjoints
__global__ void k_step_adj(int N, int W, double h, double alpha, double dt, const uint8_t *__restrict__ cls,
                           const double *__restrict__ lam, double *xbn, double *fb, double *r1, double *r2, double *r3,
                           int extrap) {
  const int WW = W * W;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * WW) return;
  const int g = t / WW, q = t - g * WW, j = q / W - 1, i = q % W - 1;
  const uint8_t *cg = cls + g * WW;
  const double *lg = lam + g * WW;
  auto P = [&](int a, int b) {
    return (a >= -1 && a <= N && b >= -1 && b <= N && cg[aix(W, a, b)] == K_INT) ? lg[aix(W, a, b)] : 0.0;
  };
  const double pc = P(i, j);
  const double lapt = P(i - 1, j) + P(i + 1, j) + P(i, j - 1) + P(i, j + 1) - 4.0 * pc;
  xbn[t] = pc + alpha / (h * h) * lapt;
  if (pc == 0.0) return;
  fb[t] += dt * pc;
  if (extrap) {
    r1[t] -= dt * pc;
    r2[t] -= 0.5 * dt * pc;
    r3[t] += 0.5 * dt * pc;
  } else {
    r1[t] -= 0.5 * dt * pc;
  }
}

// cb = scale * P lam (u and v)
__global__ void k_pscale(int W, const uint8_t *__restrict__ cls, const double *__restrict__ lam, double scale, double *cb) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * W * W) return;
  cb[t] = cls[t] == K_INT ? scale * lam[t] : 0.0;
}

// ub[comp] += sum of lam over the body boundary-condition rows of grid comp
__global__ void __launch_bounds__(TPB) k_ub_sum(int W, int comp, const uint8_t *__restrict__ cls, const double *__restrict__ lam,
                                                double *part, unsigned *ticket, double *ub) {
  const int WW = W * W;
  double s = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < WW; t += gridDim.x * blockDim.x)
    if (cls[comp * WW + t] == K_GHOST) s += lam[comp * WW + t];
  double tot;
  if (alast_total(s, part, ticket, &tot) && threadIdx.x == 0) ub[comp] += tot;
}

__global__ void k_diffmax(const double *__restrict__ a, const double *__restrict__ b, long n, unsigned long long *out) {
  double m = 0;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    double d = fabs(a[t] - b[t]);
    m = (d > m || d != d) ? d : m;
  }
  unsigned long long bb = (unsigned long long)__double_as_longlong(m);
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long c = __shfl_xor(bb, o, 64);
    bb = c > bb ? c : bb;
  }
  if ((threadIdx.x & 63) == 0 && bb) atomicMax(out, bb);
}

}  // namespace

// ---- tape ----
static size_t snap_len(const Ctx *ctx) { return 11 * (size_t)ctx->geo[0].WW + 1; }

static gp_status snap_alloc(Ctx *ctx, CnSnap &sn) {
  if (!sn.buf) GP_HIP(hipMalloc((void **)&sn.buf, snap_len(ctx) * sizeof(double)));
  return GP_OK;
}
static gp_status snap_save(Ctx *ctx, CnSnap &sn) {
  gp_status st = snap_alloc(ctx, sn);
  if (st) return st;
  const size_t WW = ctx->geo[0].WW, n = 3 * WW + 1;
  hipStream_t s = ctx->stream;
  GP_HIP(hipMemcpyAsync(sn.buf, ctx->v64[0].x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  for (int k = 0; k < 3; k++) {
    GP_HIP(hipMemcpyAsync(sn.buf + n + (2 * k) * WW, ctx->cu[k], WW * sizeof(double), hipMemcpyDeviceToDevice, s));
    GP_HIP(hipMemcpyAsync(sn.buf + n + (2 * k + 1) * WW, ctx->cv[k], WW * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  GP_HIP(hipMemcpyAsync(sn.buf + n + 6 * WW, ctx->lapu, WW * sizeof(double), hipMemcpyDeviceToDevice, s));
  GP_HIP(hipMemcpyAsync(sn.buf + n + 7 * WW, ctx->lapv, WW * sizeof(double), hipMemcpyDeviceToDevice, s));
  sn.nstep = ctx->nstep;
  return GP_OK;
}
static gp_status snap_restore(Ctx *ctx, const CnSnap &sn) {
  const size_t WW = ctx->geo[0].WW, n = 3 * WW + 1;
  hipStream_t s = ctx->stream;
  GP_HIP(hipMemcpyAsync(ctx->v64[0].x, sn.buf, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  for (int k = 0; k < 3; k++) {
    GP_HIP(hipMemcpyAsync(ctx->cu[k], sn.buf + n + (2 * k) * WW, WW * sizeof(double), hipMemcpyDeviceToDevice, s));
    GP_HIP(hipMemcpyAsync(ctx->cv[k], sn.buf + n + (2 * k + 1) * WW, WW * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  GP_HIP(hipMemcpyAsync(ctx->lapu, sn.buf + n + 6 * WW, WW * sizeof(double), hipMemcpyDeviceToDevice, s));
  GP_HIP(hipMemcpyAsync(ctx->lapv, sn.buf + n + 7 * WW, WW * sizeof(double), hipMemcpyDeviceToDevice, s));
  ctx->nstep = sn.nstep;
  return GP_OK;
}

void tape_free(Ctx *ctx) {
  Tape &T = ctx->tape;
  for (auto &sn : T.ckpt) (void)hipFree(sn.buf);
  for (auto &sn : T.seg) (void)hipFree(sn.buf);
  (void)hipFree(T.last.buf);
  T.last.buf = nullptr;
  T.ckpt.clear();
  T.seg.clear();
  if (T.d_mism) (void)hipFree(T.d_mism);
  T.d_mism = nullptr;
  for (double **p : {&T.fu, &T.fv, &T.xb, &T.yb, &T.xbn, &T.lamp, &T.ring, &T.fb, &T.tcb, &T.ub, &T.upath, &T.pcx, &T.pcy})
    if (*p) {
      (void)hipFree(*p);
      *p = nullptr;
    }
  T.valid = 0;
}

// geometry of step n (t^{n+1}) with the tape's boundary-velocity offset
static gp_status tape_geometry(Ctx *ctx, int n) {
  Tape &T = ctx->tape;
  ctx->ub_off[0] = T.ub_off[0];
  ctx->ub_off[1] = T.ub_off[1];
  return gp_set_levelset_analytic(static_cast<gp_ctx *>(ctx), &T.shape, T.t0 + (n + 1) * T.dt, &T.motion);
}

static gp_status tape_step(Ctx *ctx, int n, gp_stats *st) {
  Tape &T = ctx->tape;
  gp_status s = tape_geometry(ctx, n);
  if (s) return s;
  return gp_cn_step(static_cast<gp_ctx *>(ctx), T.dt, T.fu, T.fv, nullptr, 1, GP_FP64, T.tol, T.max_cycles, T.picard_eps,
                    T.picard_max, st);
}

// reverse of step n; the context holds the geometry of t^{n+1}, post = the state after step n, pre.nstep tells
// which convection form the step used
static gp_status adjoint_step(Ctx *ctx, const CnSnap &pre, const CnSnap &post, double tol, int max_cycles,
                              gp_stats *acc) {
  Tape &T = ctx->tape;
  Geo &G = ctx->geo[0];
  hipStream_t s = ctx->stream;
  const size_t WW = G.WW, n = G.n;
  gp_status st = GP_OK;
  const double alpha = T.dt / (2.0 * ctx->Re);
  if (alpha != ctx->alpha) ctx->c_ok = 0;  // the geometry build factored the coarsest system for the current alpha
  ctx->alpha = alpha;
  if ((st = ready(ctx))) return st;
  const double *y = post.buf;  // x^{n+1} (extension values filled)
  double *R[4];  // adjoints of c^{n+1}, c^n, c^{n-1}, c^{n-2} (u grid, then v grid)
  for (int k = 0; k < 4; k++) R[k] = T.ring + (size_t)((T.ring_head + k) & 3) * 2 * WW;
  const int extrap = pre.nstep >= 2;
  // adjoint of c^{n+1} = c(x^{n+1})
  k_conv_jt<<<nblk(2L * WW), TPB, 0, s>>>(G.N, G.W, G.h, y, R[0], R[0] + WW, T.xb);
  if (!extrap) k_copy<<<nblk(n), TPB, 0, s>>>(T.yb, T.xb, n);
  // adjoint of the extension fill, then of the solve
  ext_fill_t(ctx, 0, T.xb);
  k_copy<<<nblk(n), TPB, 0, s>>>(ctx->a_g, T.xb, n);
  // the previous step's adjoint as the initial guess (steps change smoothly; the first reversed step starts at 0)
  k_mask_unknowns<<<nblk(3L * G.WW), TPB, 0, s>>>(3 * G.WW, G.cls, ctx->a_lam);
  gp_stats sub{};
  st = adjoint_solve_dev(ctx, tol, max_cycles, &sub);
  if (st != GP_OK && st != GP_ENOCONV) return st;
  acc->cycles += sub.cycles;
  acc->outer++;
  if (!extrap) {
    // fixed point lam = M^{-T} E^T (ybar - dt/2 J_c^T P lam)
    for (int it = 0; it < T.picard_max; it++) {
      k_pscale<<<nblk(2L * WW), TPB, 0, s>>>(G.W, G.cls, ctx->a_lam, -0.5 * T.dt, T.tcb);
      k_copy<<<nblk(n), TPB, 0, s>>>(ctx->a_g, T.yb, n);
      k_conv_jt<<<nblk(2L * WW), TPB, 0, s>>>(G.N, G.W, G.h, y, T.tcb, T.tcb + WW, ctx->a_g);
      ext_fill_t(ctx, 0, ctx->a_g);
      k_copy<<<nblk(n), TPB, 0, s>>>(T.lamp, ctx->a_lam, n);
      st = adjoint_solve_dev(ctx, tol, max_cycles, &sub);  // warm start from the previous lam
      if (st != GP_OK && st != GP_ENOCONV) return st;
      acc->cycles += sub.cycles;
      acc->outer++;
      unsigned long long *m = (unsigned long long *)(ctx->d_scal + 11);
      k_fill0<<<1, 1, 0, s>>>((double *)m, 1);
      k_diffmax<<<std::min(1024, nblk(n)), TPB, 0, s>>>(ctx->a_lam, T.lamp, n, m);
      double dl, ln;
      unsigned long long hv;
      GP_HIP(hipMemcpyAsync(&hv, m, sizeof(hv), hipMemcpyDeviceToHost, s));
      GP_HIP(hipStreamSynchronize(s));
      std::memcpy(&dl, &hv, sizeof(double));
      if ((st = absmax_dev(ctx, ctx->a_lam, n, &ln))) return st;
      if (!(dl == dl)) return GP_EDIVERGED;
      if (dl <= T.picard_eps * (ln > 1 ? ln : 1)) break;
    }
  }
  // adjoints of u^n, of the forcing, of the convection history and of the boundary velocity
  k_step_adj<<<nblk(2L * WW), TPB, 0, s>>>(G.N, G.W, G.h, ctx->alpha, T.dt, G.cls, ctx->a_lam, T.xbn, T.fb, R[1], R[2],
                                          R[3], extrap);
  for (int comp = 0; comp < 2; comp++)
    k_ub_sum<<<std::min(ARED, nblk(WW)), TPB, 0, s>>>(G.W, comp, G.cls, ctx->a_lam, ctx->d_red, ctx->d_ticket, T.ub);
  // and of the body position along the path (the rows of this step's geometry at t = ctx->t_geom)
  if ((st = path_terms(ctx, T.shape, T.motion, ctx->t_geom, y, ctx->a_lam, T.pcx, T.pcy, T.upath, T.d_mism))) return st;
  // rotate the ring: c^{n+1} is done (its slot becomes the zeroed c^{n-3}), c^n is the next step's first entry
  k_fill0<<<nblk(2L * WW), TPB, 0, s>>>(R[0], 2 * WW);
  T.ring_head = (T.ring_head + 1) & 3;
  k_fill0<<<nblk(n), TPB, 0, s>>>(T.xb, n);
  k_copy<<<nblk(2L * WW), TPB, 0, s>>>(T.xb, T.xbn, 2 * WW);
  GP_HIP(hipGetLastError());
  return GP_OK;
}


static gp_status dalloc0(Ctx *ctx, double **p, size_t n) {
  if (!*p) GP_HIP(hipMalloc((void **)p, n * sizeof(double)));
  k_fill0<<<nblk((long)n), TPB, 0, ctx->stream>>>(*p, (long)n);
  return GP_OK;
}

gp_status tape_forward(Ctx *ctx, const gp_shape *shape, const gp_rigid *motion, double t0, double dt, int nsteps,
                       const double *fu, const double *fv, int on_device, const double *ub_off, double tol, int max_cycles,
                       double picard_eps, int picard_max, int K, gp_stats *stt) {
  Tape &T = ctx->tape;
  const size_t WW = ctx->geo[0].WW;
  T.valid = 0;
  if (T.K != K || (int)T.ckpt.size() < (nsteps + K - 1) / K) {
    for (auto &sn : T.seg) (void)hipFree(sn.buf);
    T.seg.clear();
  }
  T.nsteps = nsteps;
  T.K = K;
  T.shape = *shape;
  T.motion = motion ? *motion : gp_rigid{0, 0, 0, 0, 0};
  T.t0 = t0;
  T.dt = dt;
  T.ub_off[0] = ub_off ? ub_off[0] : 0.0;
  T.ub_off[1] = ub_off ? ub_off[1] : 0.0;
  T.tol = tol;
  T.max_cycles = max_cycles;
  T.picard_eps = picard_eps;
  T.picard_max = picard_max;
  gp_status st;
  if ((st = dalloc0(ctx, &T.fu, WW)) || (st = dalloc0(ctx, &T.fv, WW))) return st;
  hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (fu) GP_HIP(hipMemcpyAsync(T.fu, fu, WW * sizeof(double), kind, ctx->stream));
  if (fv) GP_HIP(hipMemcpyAsync(T.fv, fv, WW * sizeof(double), kind, ctx->stream));
  const int nseg = (nsteps + K - 1) / K;
  if ((int)T.ckpt.size() < nseg) T.ckpt.resize(nseg);
  gp_stats acc{}, sub{};
  auto t0c = std::chrono::steady_clock::now();
  for (int n = 0; n < nsteps; n++) {
    if (n % K == 0 && (st = snap_save(ctx, T.ckpt[n / K]))) return st;
    st = tape_step(ctx, n, &sub);
    if (st) return st;
    acc.cycles += sub.cycles;
    acc.outer += sub.outer;
    acc.res = sub.res;
  }
  if ((st = snap_save(ctx, T.last))) return st;
  ctx->ub_off[0] = ctx->ub_off[1] = 0.0;
  GP_HIP(hipStreamSynchronize(ctx->stream));
  acc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0c).count();
  if (stt) *stt = acc;
  T.valid = 1;
  return GP_OK;
}

gp_status tape_backward(Ctx *ctx, const double *seed_u, const double *seed_v, int on_device, double tol, int max_cycles,
                        double *dfu, double *dfv, double *dU, double *du0, double *dv0, gp_stats *stt) {
  Tape &T = ctx->tape;
  Geo &G = ctx->geo[0];
  const size_t WW = G.WW, n = G.n;
  hipStream_t s = ctx->stream;
  gp_status st;
  if (!T.valid) return GP_EINVAL;
  if ((st = adjoint_alloc(ctx))) return st;
  if ((st = dalloc0(ctx, &T.xb, n)) || (st = dalloc0(ctx, &T.yb, n)) || (st = dalloc0(ctx, &T.xbn, 2 * WW)) ||
      (st = dalloc0(ctx, &T.lamp, n)) || (st = dalloc0(ctx, &T.ring, 8 * WW)) || (st = dalloc0(ctx, &T.fb, 2 * WW)) ||
      (st = dalloc0(ctx, &T.tcb, 2 * WW)) || (st = dalloc0(ctx, &T.ub, 2)) || (st = dalloc0(ctx, &T.upath, 2)) ||
      (st = dalloc0(ctx, &T.pcx, 3 * WW)) || (st = dalloc0(ctx, &T.pcy, 3 * WW)))
    return st;
  if (!T.d_mism) GP_HIP(hipMalloc((void **)&T.d_mism, sizeof(int)));
  k_izero<<<1, 1, 0, s>>>(T.d_mism, 1);
  T.ring_head = 0;
  k_fill0<<<nblk((long)n), TPB, 0, s>>>(ctx->a_lam, (long)n);
  hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (seed_u) GP_HIP(hipMemcpyAsync(T.xb, seed_u, WW * sizeof(double), kind, s));
  if (seed_v) GP_HIP(hipMemcpyAsync(T.xb + WW, seed_v, WW * sizeof(double), kind, s));
  const int K = T.K, nseg = (T.nsteps + K - 1) / K;
  if ((int)T.seg.size() < K + 1) T.seg.resize(K + 1);
  gp_stats acc{}, sub{};
  auto t0c = std::chrono::steady_clock::now();
  for (int sg = nseg - 1; sg >= 0; sg--) {
    const int s0 = sg * K, s1 = std::min(s0 + K, T.nsteps);
    if ((st = snap_restore(ctx, T.ckpt[sg]))) return st;
    // the states inside the segment are replayed; the state after its last step is the next checkpoint (or the
    // end of the run), which the forward run kept (the steps are deterministic, so a replay would reproduce it)
    for (int m = s0; m < s1 - 1; m++) {
      if ((st = snap_save(ctx, T.seg[m - s0]))) return st;
      if ((st = tape_step(ctx, m, &sub))) return st;
    }
    if ((st = snap_save(ctx, T.seg[s1 - 1 - s0]))) return st;
    const CnSnap &end = sg + 1 < nseg ? T.ckpt[sg + 1] : T.last;
    for (int m = s1 - 1; m >= s0; m--) {
      if ((st = tape_geometry(ctx, m))) return st;
      const CnSnap &post = m == s1 - 1 ? end : T.seg[m + 1 - s0];
      if ((st = adjoint_step(ctx, T.seg[m - s0], post, tol, max_cycles, &acc))) return st;
    }
  }
  // c^0 = c(u^0) entered the first steps: its adjoint goes to u^0
  {
    double *R0 = T.ring + (size_t)(T.ring_head & 3) * 2 * WW;
    k_conv_jt<<<nblk(2L * WW), TPB, 0, s>>>(G.N, G.W, G.h, T.ckpt[0].buf, R0, R0 + WW, T.xb);
  }
  // the context is left at the end of the run
  if ((st = tape_geometry(ctx, T.nsteps - 1)) || (st = snap_restore(ctx, T.last))) return st;
  ctx->ub_off[0] = ctx->ub_off[1] = 0.0;
  hipMemcpyKind ok = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (dfu) GP_HIP(hipMemcpyAsync(dfu, T.fb, WW * sizeof(double), ok, s));
  if (dfv) GP_HIP(hipMemcpyAsync(dfv, T.fb + WW, WW * sizeof(double), ok, s));
  if (du0) GP_HIP(hipMemcpyAsync(du0, T.xb, WW * sizeof(double), ok, s));
  if (dv0) GP_HIP(hipMemcpyAsync(dv0, T.xb + WW, WW * sizeof(double), ok, s));
  if (dU) GP_HIP(hipMemcpyAsync(dU, T.ub, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  GP_HIP(hipMemcpyAsync(T.h_upath, T.upath, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  GP_HIP(hipMemcpyAsync(&T.h_mism, T.d_mism, sizeof(int), hipMemcpyDeviceToHost, s));
  GP_HIP(hipStreamSynchronize(s));
  acc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0c).count();
  if (stt) *stt = acc;
  return GP_OK;
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

extern "C" gp_status gp_tape_forward(gp_ctx *ctx, const gp_shape *shape, const gp_rigid *motion, double t0, double dt,
                                     int nsteps, const double *fu, const double *fv, int on_device, const double *ub_offset,
                                     double tol, int max_cycles, double picard_eps, int picard_max, int checkpoint_every,
                                     gp_stats *st) {
  if (!ctx || !shape || !ctx->have_geom || !(dt > 0) || nsteps < 1 || checkpoint_every < 1 || !(tol > 0) ||
      max_cycles < 1 || picard_max < 1)
    return GP_EINVAL;
  return tape_forward(ctx, shape, motion, t0, dt, nsteps, fu, fv, on_device, ub_offset, tol, max_cycles, picard_eps,
                      picard_max, checkpoint_every, st);
}

extern "C" gp_status gp_tape_backward(gp_ctx *ctx, const double *seed_u, const double *seed_v, int on_device, double tol,
                                      int max_cycles, double *dJdfu, double *dJdfv, double *dJdU, double *dJdu0,
                                      double *dJdv0, gp_stats *st) {
  if (!ctx || !(tol > 0) || max_cycles < 1) return GP_EINVAL;
  return tape_backward(ctx, seed_u, seed_v, on_device, tol, max_cycles, dJdfu, dJdfv, dJdU, dJdu0, dJdv0, st);
}

extern "C" gp_status gp_tape_path_gradient(gp_ctx *ctx, double *dJdU_path, int *unmatched) {
  if (!ctx || !dJdU_path || !ctx->tape.valid) return GP_EINVAL;
  dJdU_path[0] = ctx->tape.h_upath[0];
  dJdU_path[1] = ctx->tape.h_upath[1];
  if (unmatched) *unmatched = ctx->tape.h_mism;
  return GP_OK;
}
