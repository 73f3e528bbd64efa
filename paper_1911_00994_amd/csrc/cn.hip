// Crank-Nicolson time step (Sect. 2) on a possibly moving domain (Sect. 3.4).
//   f~ = u^n + alpha lap u^n + dt f^{n+1/2} - dt C  on the internal points of Omega^{n+1}, alpha = dt / (2 Re),
//   C = c^n + c^{n-1}/2 - c^{n-2}/2 (eq. extrUdU) from the third step on, and the fixed-point iteration of
//   eq. (NSitconv) with C = (c^n + c(u^{n+1,k}))/2 for the first two steps, stopped by eq. (iterativeNS).
// c(u) = u du/dx + v_bar du/dy with the central differences of Sect. 3.2 and v_bar the average of the four
// surrounding v nodes; the history holds NaN where the stencil had no value, so a missing value shows up as a
// NaN right-hand side and the step is rejected.
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>

#include "internal.h"

namespace gpmg {

__device__ __forceinline__ bool valued(uint8_t c) {
  return c == K_INT || c == K_GHOST || c == K_GHOSTX || c == K_WALLD || c == K_WALLG || c == K_EXT;
}

// convection and Laplacian of the state at every u and v node whose stencil carries values
__global__ void k_conv_lap(int N, int W, double h, const uint8_t *__restrict__ cls, const double *__restrict__ x,
                           double *cu, double *cv, double *lu, double *lv) {
  int WW = W * W;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= WW) return;
  int j = t / W - 1, i = t % W - 1;
  const double *u = x, *v = x + WW;
  const double nan = __builtin_nan("");
  auto VU = [&](int a, int b) { return a >= -1 && a <= N && b >= -1 && b <= N && valued(cls[(b + 1) * W + (a + 1)]); };
  auto VV = [&](int a, int b) { return a >= -1 && a <= N && b >= -1 && b <= N && valued(cls[WW + (b + 1) * W + (a + 1)]); };
  auto U = [&](int a, int b) { return u[(b + 1) * W + (a + 1)]; };
  auto V = [&](int a, int b) { return v[(b + 1) * W + (a + 1)]; };
  double cuv = nan, luv = nan, cvv = nan, lvv = nan;
  if (VU(i, j) && VU(i - 1, j) && VU(i + 1, j) && VU(i, j - 1) && VU(i, j + 1)) {
    luv = (U(i - 1, j) + U(i + 1, j) + U(i, j - 1) + U(i, j + 1) - 4 * U(i, j)) / (h * h);
    if (VV(i - 1, j) && VV(i, j) && VV(i - 1, j + 1) && VV(i, j + 1)) {
      double vb = 0.25 * (V(i - 1, j) + V(i, j) + V(i - 1, j + 1) + V(i, j + 1));
      cuv = U(i, j) * (U(i + 1, j) - U(i - 1, j)) / (2 * h) + vb * (U(i, j + 1) - U(i, j - 1)) / (2 * h);
    }
  }
  if (VV(i, j) && VV(i - 1, j) && VV(i + 1, j) && VV(i, j - 1) && VV(i, j + 1)) {
    lvv = (V(i - 1, j) + V(i + 1, j) + V(i, j - 1) + V(i, j + 1) - 4 * V(i, j)) / (h * h);
    if (VU(i, j - 1) && VU(i + 1, j - 1) && VU(i, j) && VU(i + 1, j)) {
      double ub = 0.25 * (U(i, j - 1) + U(i + 1, j - 1) + U(i, j) + U(i + 1, j));
      cvv = ub * (V(i + 1, j) - V(i - 1, j)) / (2 * h) + V(i, j) * (V(i, j + 1) - V(i, j - 1)) / (2 * h);
    }
  }
  cu[t] = cuv;
  cv[t] = cvv;
  if (lu) lu[t] = luv;
  if (lv) lv[t] = lvv;
}

// the largest |v| of a block into *m (as bits, which order like the values; NaN above everything): wavefront
// maximum, then one atomic per block; the kernels below loop over their points with at most MAXB_BLOCKS blocks
// (contended atomics on one address cost ~10 ns each; one per element took a third of a millisecond).  Every
// thread of the block calls it.
constexpr int MAXB_BLOCKS = 1024;
__device__ __forceinline__ unsigned long long abits(double v) {
  return (unsigned long long)__double_as_longlong(fabs(v));
}
__device__ __forceinline__ void bmax(unsigned long long *m, unsigned long long a) {
  __shared__ unsigned long long sm[TPB / 64];
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long b = __shfl_xor(a, o, 64);
    a = b > a ? b : a;
  }
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < (int)(blockDim.x >> 6); q++) a = sm[q] > a ? sm[q] : a;
    if (a) atomicMax(m, a);
  }
}

// explicit part on the internal velocity points; NaN marks a missing history value
__global__ void k_fbase(int W, const uint8_t *__restrict__ cls, const double *__restrict__ x, const double *__restrict__ lu,
                        const double *__restrict__ lv, const double *__restrict__ f, double alpha, double dt, double *fb,
                        unsigned long long *fmax) {
  const int WW = W * W;
  unsigned long long m = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < 2 * WW; t += gridDim.x * blockDim.x) {
    double val = 0;
    if (cls[t] == K_INT) {
      const double lap = t < WW ? lu[t] : lv[t - WW];
      val = x[t] + alpha * lap + dt * (f ? f[t] : 0.0);
    }
    fb[t] = val;
    m = max(m, abits(val));
  }
  bmax(fmax, m);
}

// momentum right-hand side with the extrapolated convection (n >= 2) or c^n (first Picard iterate)
__global__ void k_rhs_conv(int W, const uint8_t *__restrict__ cls, const double *__restrict__ fb, const double *c0u,
                           const double *c0v, const double *c1u, const double *c1v, const double *c2u, const double *c2v,
                           int extrap, double dt, double *b, unsigned long long *bad) {
  int WW = W * W;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * WW) return;
  if (cls[t] != K_INT) return;
  int q = t < WW ? t : t - WW;
  const double *c0 = t < WW ? c0u : c0v, *c1 = t < WW ? c1u : c1v, *c2 = t < WW ? c2u : c2v;
  double C = extrap ? c0[q] + 0.5 * c1[q] - 0.5 * c2[q] : c0[q];
  double val = fb[t] - dt * C;
  b[t] = val;
  if (val != val) atomicOr((unsigned int *)bad, 1u);
}

// Picard update: b = f~ - dt (c^n + c(u^{n+1,k})) / 2 and the residual of eq. (iterativeNS) at the new iterate
__global__ void k_picard(int N, int W, double h, double a, double d, const uint8_t *__restrict__ cls,
                         const double *__restrict__ x, const double *__restrict__ fb, const double *c0u, const double *c0v,
                         const double *cku, const double *ckv, double dt, double *b, unsigned long long *rmax) {
  const int WW = W * W;
  unsigned long long m = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < 2 * WW; t += gridDim.x * blockDim.x) {
    if (cls[t] != K_INT) continue;
    const int g = t < WW ? 0 : 1, q = t - g * WW;
    const double C = 0.5 * (g == 0 ? c0u[q] + cku[q] : c0v[q] + ckv[q]);
    const double bn = fb[t] - dt * C;
    const double *u = x + g * WW, *p = x + 2 * WW;
    const double ih = 1.0 / h;
    const double Mx =
        d * u[q] - a * (u[q - 1] + u[q + 1] + u[q - W] + u[q + W]) + (p[q] - (g == 0 ? p[q - 1] : p[q - W])) * ih;
    const double r = bn - Mx;
    b[t] = bn;
    m = max(m, abits(r));
  }
  bmax(rmax, m);
  (void)N;
}

__global__ void k_rhs_cont(int W, const uint8_t *__restrict__ cls, const double *g, double *b) {
  int WW = W * W;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == WW) {
    b[3 * WW] = 0;
    return;
  }
  if (t > WW) return;
  if (cls[2 * WW + t] == K_INT) b[2 * WW + t] = g ? g[t] : 0.0;
}

__global__ void k_fill_nan(double *a, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) a[t] = __builtin_nan("");
}
__global__ void k_zero_u64(unsigned long long *p, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0ull;
}

template <typename T>
__global__ void k_ext_fill_cn(const int *__restrict__ e_pt, const int *__restrict__ e_src, const double *__restrict__ e_w,
                              int ne, T *__restrict__ x) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  if (e_src[3 * e] < 0) return;
  x[e_pt[e]] = (T)(e_w[3 * e] * (double)x[e_src[3 * e]] + e_w[3 * e + 1] * (double)x[e_src[3 * e + 1]] +
                   e_w[3 * e + 2] * (double)x[e_src[3 * e + 2]]);
}

static double u64_to_d(unsigned long long v) {
  double d;
  std::memcpy(&d, &v, sizeof(d));
  return d;
}

gp_status cn_set_state_finish(Ctx *ctx) {
  Geo &G = ctx->geo[0];
  hipStream_t s = ctx->stream;
  k_conv_lap<<<nblk(G.WW), TPB, 0, s>>>(G.N, G.W, G.h, G.cls, ctx->v64[0].x, ctx->cu[0], ctx->cv[0], ctx->lapu, ctx->lapv);
  for (int k = 1; k < 3; k++) {
    k_fill_nan<<<nblk(G.WW), TPB, 0, s>>>(ctx->cu[k], G.WW);
    k_fill_nan<<<nblk(G.WW), TPB, 0, s>>>(ctx->cv[k], G.WW);
  }
  ctx->nstep = 0;
  GP_HIP(hipGetLastError());
  GP_HIP(hipStreamSynchronize(s));
  return GP_OK;
}

gp_status cn_step(Ctx *ctx, double dt, const double *fu, const double *fv, const double *g, int precision, double tol,
                  int max_cycles, double picard_eps, int picard_max, gp_stats *stt) {
  auto t0 = std::chrono::steady_clock::now();
  Geo &G = ctx->geo[0];
  hipStream_t s = ctx->stream;
  int WW = G.WW;
  double alpha = dt / (2.0 * ctx->Re);
  if (alpha != ctx->alpha) ctx->c_ok = 0;
  ctx->alpha = alpha;
  if (!ctx->c_ok) {
    gp_status st = coarse_factor(ctx);
    if (st) return st;
  }
  unsigned long long *flags = (unsigned long long *)(ctx->d_scal + 4);  // [0] |fb| max, [1] NaN flag, [2] picard res
  k_zero_u64<<<1, 4, 0, s>>>(flags, 4);
  // forcing staged in fwork by the caller: u grid, v grid, continuity right-hand side
  (void)fu;
  (void)fv;
  k_fbase<<<std::min(MAXB_BLOCKS, nblk(2L * WW)), TPB, 0, s>>>(G.W, G.cls, ctx->v64[0].x, ctx->lapu, ctx->lapv, ctx->fwork, alpha, dt,
                                       ctx->fbase, flags);
  k_rhs_cont<<<nblk(WW + 1), TPB, 0, s>>>(G.W, G.cls, g ? ctx->fwork + 2 * (size_t)WW : nullptr, ctx->v64[0].b);
  int extrap = ctx->nstep >= 2;
  k_rhs_conv<<<nblk(2L * WW), TPB, 0, s>>>(G.W, G.cls, ctx->fbase, ctx->cu[0], ctx->cv[0], ctx->cu[1], ctx->cv[1],
                                          ctx->cu[2], ctx->cv[2], extrap, dt, ctx->v64[0].b, flags + 1);
  GP_HIP(hipGetLastError());
  unsigned long long hf[4];
  GP_HIP(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
  GP_HIP(hipStreamSynchronize(s));
  double fbn = u64_to_d(hf[0]);
  if (hf[1] || !(fbn == fbn)) return GP_EGEOM;  // an internal point of the new domain lacks step-n values
  gp_stats sub{};
  int total = 0, picard = 0;
  double bytes = 0;
  gp_status st = GP_OK;
  if (extrap) {
    st = mg_solve(ctx, precision, tol, max_cycles, &sub);
    total = sub.cycles;
    bytes = sub.bytes_alg;
  } else {
    double h = G.h, a = alpha / (h * h), d = 1.0 + 4.0 * a;
    for (;;) {
      st = mg_solve(ctx, precision, tol, max_cycles, &sub);
      total += sub.cycles;
      bytes += sub.bytes_alg;
      picard++;
      if (st != GP_OK && st != GP_ENOCONV) break;
      if (G.ne) k_ext_fill_cn<double><<<nblk(G.ne), TPB, 0, s>>>(G.e_pt, G.e_src, G.e_w, G.ne, ctx->v64[0].x);
      k_conv_lap<<<nblk(WW), TPB, 0, s>>>(G.N, G.W, G.h, G.cls, ctx->v64[0].x, ctx->cku, ctx->ckv, nullptr, nullptr);
      k_zero_u64<<<1, 1, 0, s>>>(flags + 2, 1);
      k_picard<<<std::min(MAXB_BLOCKS, nblk(2L * WW)), TPB, 0, s>>>(G.N, G.W, G.h, a, d, G.cls, ctx->v64[0].x, ctx->fbase, ctx->cu[0], ctx->cv[0],
                                            ctx->cku, ctx->ckv, dt, ctx->v64[0].b, flags + 2);
      GP_HIP(hipGetLastError());
      unsigned long long rv;
      GP_HIP(hipMemcpyAsync(&rv, flags + 2, sizeof(rv), hipMemcpyDeviceToHost, s));
      GP_HIP(hipStreamSynchronize(s));
      double rn = u64_to_d(rv);
      double thr = picard_eps * (fbn > 1 ? fbn : 1);
      if (!(rn == rn)) {
        st = GP_EDIVERGED;
        break;
      }
      if (rn < thr || picard >= picard_max) break;
    }
  }
  // finish: extension values, history shift, convection and Laplacian of the new state
  if (G.ne) k_ext_fill_cn<double><<<nblk(G.ne), TPB, 0, s>>>(G.e_pt, G.e_src, G.e_w, G.ne, ctx->v64[0].x);
  double *ou = ctx->cu[2], *ov = ctx->cv[2];
  ctx->cu[2] = ctx->cu[1];
  ctx->cv[2] = ctx->cv[1];
  ctx->cu[1] = ctx->cu[0];
  ctx->cv[1] = ctx->cv[0];
  ctx->cu[0] = ou;
  ctx->cv[0] = ov;
  k_conv_lap<<<nblk(WW), TPB, 0, s>>>(G.N, G.W, G.h, G.cls, ctx->v64[0].x, ctx->cu[0], ctx->cv[0], ctx->lapu, ctx->lapv);
  GP_HIP(hipGetLastError());
  GP_HIP(hipStreamSynchronize(s));
  ctx->nstep++;
  if (stt) {
    *stt = sub;
    stt->cycles = total;
    stt->bytes_alg = bytes;
    stt->outer = picard;
    stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return st;
}

}  // namespace gpmg

using namespace gpmg;

extern "C" gp_status gp_set_state(gp_ctx *ctx, const double *u, const double *v, const double *p, double xi, int on_device) {
  gp_status st = gp_set_x(ctx, u, v, p, xi, on_device);
  if (st) return st;
  if (!ctx->have_geom) return GP_EINVAL;
  return cn_set_state_finish(ctx);
}

extern "C" gp_status gp_cn_step(gp_ctx *ctx, double dt, const double *fu, const double *fv, const double *g, int on_device,
                                int precision, double tol, int max_cycles, double picard_eps, int picard_max, gp_stats *st) {
  if (!ctx || !ctx->have_geom || !(dt > 0) || !(tol > 0) || max_cycles < 0 || picard_max < 1 ||
      (precision != GP_FP64 && precision != GP_MIXED))
    return GP_EINVAL;
  Geo &G = ctx->geo[0];
  hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (fu) GP_HIP(hipMemcpyAsync(ctx->fwork, fu, G.WW * sizeof(double), k, ctx->stream));
  else GP_HIP(hipMemsetAsync(ctx->fwork, 0, G.WW * sizeof(double), ctx->stream));
  if (fv) GP_HIP(hipMemcpyAsync(ctx->fwork + G.WW, fv, G.WW * sizeof(double), k, ctx->stream));
  else GP_HIP(hipMemsetAsync(ctx->fwork + G.WW, 0, G.WW * sizeof(double), ctx->stream));
  if (g) GP_HIP(hipMemcpyAsync(ctx->fwork + 2 * (size_t)G.WW, g, G.WW * sizeof(double), k, ctx->stream));
  return cn_step(ctx, dt, fu, fv, g, precision, tol, max_cycles, picard_eps, picard_max, st);
}
