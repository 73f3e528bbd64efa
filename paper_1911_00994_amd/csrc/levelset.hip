// Level-set reinitialisation of Sect. 3.1, eq. (sdf), on the half-step lattice of a context: the steady state of
// d(phi_d)/d(mu) = sgn(phi) (1 - |grad phi_d|), phi_d = phi at mu = 0 (the step before the solver path for a
// deforming body, whose level set is no longer a distance function).  Discretisation (the paper fixes only the
// equation): explicit Euler steps in mu of size cfl * dx; |grad phi_d| by the first-order Godunov upwind
// approximation (nearest lattice value repeated beyond the lattice); at the points next to the interface the
// distance estimate D = dx phi / |Delta phi| of the initial data replaces the upwind step, so the interface does not
// move; sgn(0) = 0.
//
// Layout and schedule: the lattice is cut into RT_T x RT_T output tiles; one workgroup stages its tile with a halo of
// RT_K points in LDS (two buffers) and runs up to RT_K steps there before writing its tile back, so one launch does
// RT_K steps with one pass over HBM.  A point's class (sign, next to the interface) and D stay in registers of the
// thread that owns it for all steps of a launch.  Values computed near the staged border use clamped neighbours
// that are not the lattice's; that error moves one point per step and never reaches the tile after RT_K steps.
#include "internal.h"

namespace gpmg {

constexpr int RT_T = 48, RT_K = 8, RT_S = RT_T + 2 * RT_K, RT_THR = 1024, RT_PPT = (RT_S * RT_S + RT_THR - 1) / RT_THR;

// per lattice point: code bit 0/1 the sign of phi (1: positive, 2: negative, 0: zero), bit 2 next to the interface;
// D the interface distance estimate
__global__ void k_reinit_prep(const double *__restrict__ phi0, int n, double dx, int8_t *code, double *D) {
  const long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= (long)n * n) return;
  const int j = (int)(k / n), i = (int)(k - (long)j * n);
  const int im = i > 0 ? i - 1 : i, ip = i < n - 1 ? i + 1 : i, jm = j > 0 ? j - 1 : j, jp = j < n - 1 ? j + 1 : j;
  const double p = phi0[k], pw = phi0[(long)j * n + im], pe = phi0[(long)j * n + ip], ps = phi0[(long)jm * n + i],
               pn = phi0[(long)jp * n + i];
  const bool cross = p == 0.0 || p * pw < 0 || p * pe < 0 || p * ps < 0 || p * pn < 0;
  int8_t c = p > 0 ? 1 : (p < 0 ? 2 : 0);
  double d = 0;
  if (cross) {
    c |= 4;
    const double ex = fmax(fmax(fabs(pe - pw) / 2, fabs(pe - p)), fabs(p - pw));
    const double ey = fmax(fmax(fabs(pn - ps) / 2, fabs(pn - p)), fabs(p - ps));
    double len = sqrt(ex * ex + ey * ey);
    if (len < 1e-300) len = 1e-300;
    d = dx * p / len;
  }
  code[k] = c;
  D[k] = d;
}

// one pseudo-time step of point value p with its four neighbours (west, east, south, north)
__device__ __forceinline__ double reinit_point(double p, double pw, double pe, double ps, double pn, int8_t c, double D,
                                               double dx, double cfl) {
  const int sg = (c & 3) == 1 ? 1 : ((c & 3) == 2 ? -1 : 0);
  if (sg == 0) return p;
  const double dmu = cfl * dx;
  if (c & 4) return p - (dmu / dx) * (sg * fabs(p) - D);
  const double a = (p - pw) / dx, b = (pe - p) / dx, cc = (p - ps) / dx, d = (pn - p) / dx;
  double gx, gy;
  if (sg > 0) {
    const double a1 = a > 0 ? a : 0, b1 = b < 0 ? b : 0, c1 = cc > 0 ? cc : 0, d1 = d < 0 ? d : 0;
    gx = a1 * a1 > b1 * b1 ? a1 * a1 : b1 * b1;
    gy = c1 * c1 > d1 * d1 ? c1 * c1 : d1 * d1;
  } else {
    const double a1 = a < 0 ? a : 0, b1 = b > 0 ? b : 0, c1 = cc < 0 ? cc : 0, d1 = d > 0 ? d : 0;
    gx = a1 * a1 > b1 * b1 ? a1 * a1 : b1 * b1;
    gy = c1 * c1 > d1 * d1 ? c1 * c1 : d1 * d1;
  }
  return p - dmu * sg * (sqrt(gx + gy) - 1.0);
}

// steps (<= RT_K) pseudo-time steps of every tile; cur -> nxt
__global__ void __launch_bounds__(RT_THR) k_reinit_tile(const double *__restrict__ cur, double *__restrict__ nxt,
                                                        const int8_t *__restrict__ code, const double *__restrict__ D,
                                                        int n, int tiles_x, double dx, double cfl, int steps) {
  __shared__ double buf[2][RT_S * RT_S];
  const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
  const int x0 = tx * RT_T - RT_K, y0 = ty * RT_T - RT_K;  // lattice position of staged point (0, 0)
  // staged region clipped to the lattice: local [lx0, lx1) x [ly0, ly1)
  const int lx0 = x0 < 0 ? -x0 : 0, ly0 = y0 < 0 ? -y0 : 0;
  const int lx1 = min(RT_S, n - x0), ly1 = min(RT_S, n - y0);
  int8_t cc[RT_PPT];
  double dd[RT_PPT];
#pragma unroll
  for (int u = 0; u < RT_PPT; u++) {
    const int q = threadIdx.x + u * RT_THR;
    const int ly = q / RT_S, lx = q - ly * RT_S;
    const bool in = q < RT_S * RT_S && lx >= lx0 && lx < lx1 && ly >= ly0 && ly < ly1;
    const long g = (long)(y0 + ly) * n + (x0 + lx);
    cc[u] = in ? code[g] : (int8_t)0;
    dd[u] = in ? D[g] : 0.0;
    if (q < RT_S * RT_S) buf[0][q] = in ? cur[g] : 0.0;
  }
  __syncthreads();
  int src = 0;
  for (int s = 0; s < steps; s++) {
#pragma unroll
    for (int u = 0; u < RT_PPT; u++) {
      const int q = threadIdx.x + u * RT_THR;
      if (q >= RT_S * RT_S) continue;
      const int ly = q / RT_S, lx = q - ly * RT_S;
      if (lx < lx0 || lx >= lx1 || ly < ly0 || ly >= ly1) continue;
      const double *b = buf[src];
      // neighbours: the lattice's edge repeats the point itself; the staged border does too (its values are
      // wrong, but do not reach the tile within RT_K steps)
      const int qw = lx > lx0 ? q - 1 : q, qe = lx + 1 < lx1 ? q + 1 : q;
      const int qs = ly > ly0 ? q - RT_S : q, qn = ly + 1 < ly1 ? q + RT_S : q;
      buf[src ^ 1][q] = reinit_point(b[q], b[qw], b[qe], b[qs], b[qn], cc[u], dd[u], dx, cfl);
    }
    __syncthreads();
    src ^= 1;
  }
#pragma unroll
  for (int u = 0; u < RT_PPT; u++) {
    const int q = threadIdx.x + u * RT_THR;
    if (q >= RT_S * RT_S) continue;
    const int ly = q / RT_S, lx = q - ly * RT_S;
    if (lx < RT_K || lx >= RT_K + RT_T || ly < RT_K || ly >= RT_K + RT_T) continue;
    if (lx >= lx1 || ly >= ly1) continue;
    nxt[(long)(y0 + ly) * n + (x0 + lx)] = buf[src][q];
  }
}

gp_status reinit_levelset(Ctx *ctx, double *phi, int on_device, int iters, double cfl) {
  const int n = 2 * ctx->N + 1;
  const size_t nn = (size_t)n * n;
  hipStream_t s = ctx->stream;
  if (!ctx->rl_a) {
    GP_HIP(hipMalloc((void **)&ctx->rl_a, nn * sizeof(double)));
    GP_HIP(hipMalloc((void **)&ctx->rl_b, nn * sizeof(double)));
    GP_HIP(hipMalloc((void **)&ctx->rl_d, nn * sizeof(double)));
    GP_HIP(hipMalloc((void **)&ctx->rl_c, nn));
  }
  const double dx = 0.5 * ctx->geo[0].h;
  GP_HIP(hipMemcpyAsync(ctx->rl_a, phi, nn * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        s));
  k_reinit_prep<<<nblk((long)nn), TPB, 0, s>>>(ctx->rl_a, n, dx, ctx->rl_c, ctx->rl_d);
  const int tiles_x = (n + RT_T - 1) / RT_T;
  double *a = ctx->rl_a, *b = ctx->rl_b;
  for (int done = 0; done < iters; done += RT_K) {
    const int steps = std::min(RT_K, iters - done);
    k_reinit_tile<<<tiles_x * tiles_x, RT_THR, 0, s>>>(a, b, ctx->rl_c, ctx->rl_d, n, tiles_x, dx, cfl, steps);
    std::swap(a, b);
  }
  GP_HIP(hipGetLastError());
  GP_HIP(hipMemcpyAsync(phi, a, nn * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  GP_HIP(hipStreamSynchronize(s));
  return GP_OK;
}

}  // namespace gpmg
