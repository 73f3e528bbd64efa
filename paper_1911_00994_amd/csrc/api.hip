// C-ABI entry points of the gpmg library: context, geometry, linear-system and inspection calls.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>

#include "internal.h"

using namespace gpmg;


namespace {

template <typename T>
gp_status dalloc(Ctx *ctx, T **p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void **)p, n * sizeof(T));
  if (e != hipSuccess) {
    ctx->hip_err = std::string("hipMalloc: ") + hipGetErrorString(e);
    *p = nullptr;
    return GP_ENOMEM;
  }
  return GP_OK;
}

void dfree(void *p) {
  if (p) (void)hipFree(p);
}

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

__global__ void k_scatter_pts(const uint8_t *cls, int n, int mode, const double *src, double *b, double *x) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  uint8_t c = cls[t];
  if (mode == 0) {  // boundary data
    if (c == K_GHOST || c == K_WALLG || c == K_WALLD) b[t] = src[t];
    if (c == K_WALLD) x[t] = src[t];
  } else {  // internal right-hand side
    if (c == K_INT) b[t] = src[t];
  }
}
__global__ void k_zero_int(const uint8_t *cls, int lo, int hi, double *b) {
  int t = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (t < hi && cls[t] == K_INT) b[t] = 0;
}

gp_status stage_in(Ctx *ctx, const double *src, int on_device, double *dst, size_t n) {
  GP_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        ctx->stream));
  return GP_OK;
}

gp_status ensure_coarse(Ctx *ctx) {
  if (!ctx->have_geom) return GP_EINVAL;
  if (ctx->c_ok) return GP_OK;
  return coarse_factor(ctx);
}

// wait for a background geometry build (gp_prepare_levelset_analytic) and forget it
void prep_discard(Ctx *ctx) {
  if (!ctx->prep_active) return;
  ctx->prep.join();
  ctx->prep_active = false;
}
bool same_shape(const gp_shape &a, const gp_shape &b) {
  return a.kind == b.kind && a.p[0] == b.p[0] && a.p[1] == b.p[1] && a.p[2] == b.p[2] && a.p[3] == b.p[3];
}
bool same_motion(const gp_rigid &a, const gp_rigid &b) {
  return a.X0x == b.X0x && a.X0y == b.X0y && a.Ux == b.Ux && a.Uy == b.Uy && a.omega == b.omega;
}
// the prepared geometry becomes the context's: the two contexts exchange their levels' tables, level set and
// coarsest inverse (the shadow keeps the old ones, which the next preparation overwrites)
void take_prepared(Ctx *ctx) {
  Ctx *sh = ctx->shadow;
  for (int l = 0; l < ctx->L; l++) std::swap(ctx->geo[l], sh->geo[l]);
  std::swap(ctx->phi, sh->phi);
  std::swap(ctx->nc, sh->nc);
  std::swap(ctx->c_map, sh->c_map);
  std::swap(ctx->c_bmap, sh->c_bmap);
  std::swap(ctx->c_A, sh->c_A);
  std::swap(ctx->c_B, sh->c_B);
  std::swap(ctx->c_inv, sh->c_inv);
  std::swap(ctx->c_work, sh->c_work);
  std::swap(ctx->c_ok, sh->c_ok);
  ctx->c_ok = ctx->c_ok && ctx->prep_alpha == ctx->alpha;  // factored for the alpha of the time of preparation
  ctx->have_geom = 1;
}

gp_status after_geometry(Ctx *ctx) {
  gp_status st = geometry_build(ctx);  // also the coarsest inverse where it can (c_ok)
  if (st) return st;
  st = default_boundary_values(ctx);
  if (st) return st;
  return GP_OK;
}

}  // namespace

extern "C" {

void gp_default_params(gp_params *p) {
  if (!p) return;
  p->nu1 = 2;
  p->nu2 = 2;
  p->gamma = 1;
  p->lambda_ghost = 2;
  p->coarsest_n = 8;
  p->march_max = 8;
  p->ext_radius = 4;
  p->dtau_dir = 0.9;
  p->dtau_neu_over_h = 0.9;
  p->bisect_eps_over_h = 0.01;
  p->cg_min = 0.1;
  p->mixed_inner_cycles = 2;
  p->bnd_sweeps = 0;
  p->bnd_radius = 2;
  p->fuse_small_levels = 1;
  p->band_split_min = 3000;
  p->graph_iterations = 0;
  p->band_sector_min = 1500;
  p->queue_ahead = 1;
  p->ghost_boxes = 1;
  p->krylov = 8;
  p->ghost_box_levels = 1;
}

const char *gp_strerror(gp_status st) {
  switch (st) {
    case GP_OK: return "ok";
    case GP_EINVAL: return "invalid argument";
    case GP_ENOMEM: return "out of memory";
    case GP_EHIP: return "HIP runtime error";
    case GP_EGEOM: return "geometry rejected";
    case GP_ENOCONV: return "no convergence within max_cycles";
    case GP_EDIVERGED: return "iteration diverged";
    case GP_ESCRATCH: return "problem too large for the static scratch of gp_solve_noalloc";
    default: return "unknown status";
  }
}

const char *gp_last_hip_error(const gp_ctx *ctx) { return ctx ? ctx->hip_err.c_str() : ""; }

int gp_num_levels(const gp_ctx *ctx) { return ctx ? ctx->L : 0; }

gp_status gp_get_band_layout(gp_ctx *ctx, int level, int *out) {
  if (!ctx || !out || level < 0 || level >= ctx->L || !ctx->have_geom) return GP_EINVAL;
  const Geo &G = ctx->geo[level];
  out[0] = G.nband;
  out[1] = G.nbg;
  out[2] = G.sec_S;
  out[3] = G.lds_ok;
  return GP_OK;
}

gp_status gp_get_coupled_boxes(gp_ctx *ctx, int level, int *counts, int *cell, int *off, int *idx, unsigned char *wr,
                               int *colour_off) {
  if (!ctx || !counts || level < 0 || level >= ctx->L || !ctx->have_geom) return GP_EINVAL;
  const Geo &G = ctx->geo[level];
  counts[0] = G.nxb;
  counts[1] = G.nxs;
  if (colour_off)
    for (int c = 0; c < 6; c++) colour_off[c] = G.xb_coff[c];
  if (G.nxb == 0) return GP_OK;
  if (cell) GP_HIP(hipMemcpyAsync(cell, G.xb_cell, (size_t)G.nxb * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  if (off) GP_HIP(hipMemcpyAsync(off, G.xb_off, (size_t)(G.nxb + 1) * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  if (idx) GP_HIP(hipMemcpyAsync(idx, G.xb_idx, (size_t)G.nxs * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  if (wr) GP_HIP(hipMemcpyAsync(wr, G.xb_wr, (size_t)G.nxs, hipMemcpyDeviceToHost, ctx->stream));
  GP_HIP(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}

void gp_destroy(gp_ctx *ctx) {
  if (!ctx) return;
  prep_discard(ctx);
  if (ctx->shadow) gp_destroy(static_cast<gp_ctx *>(ctx->shadow));
  if (ctx->prep_start) (void)hipEventDestroy(ctx->prep_start);
  if (ctx->prep_done) (void)hipEventDestroy(ctx->prep_done);
  (void)hipStreamSynchronize(ctx->stream);
  for (int l = 0; l < ctx->L; l++) {
    Geo &G = ctx->geo[l];
    dfree(G.cls);
    dfree(G.xb_cell);
    dfree(G.xb_off);
    dfree(G.xb_ioff);
    dfree(G.xb_gcnt);
    dfree(G.xb_gtmp);
    dfree(G.xb_ok);
    dfree(G.xb_idx);
    dfree(G.xb_box);
    dfree(G.xb_wr);
    dfree(G.xb_r);
    dfree(G.xb_inv);
    for (void *q : {(void *)G.xb_gc, (void *)G.xb_gw, (void *)G.xb_uk, (void *)G.xb_uo, (void *)G.xb_ub, (void *)G.xb_um})
      dfree(q);
    dfree(G.xb_own);
    dfree(G.d_xb_co);
    dfree(G.sec_pt);
    dfree(G.sec_bfl);
    dfree(G.sec_bcell);
    dfree(G.sec_gk);
    dfree(G.sec_own_loc);
    dfree(G.sec_own_g);
    dfree(G.sec_mask);
    dfree(G.sec_lmap);
    dfree(G.sec_bsl);
    dfree(G.sec_gl);
    dfree(G.sec_gw);
    dfree(G.sec_gdt);
    dfree(G.sec_out);
    dfree(G.g_pt);
    dfree(G.g_col);
    dfree(G.g_colr);
    dfree(G.g_colrT);
    dfree(G.g_wT);
    dfree(G.g_w);
    dfree(G.g_dtau);
    dfree(G.g_B);
    dfree(G.g_nB);
    dfree(G.g_th);
    dfree(G.g_kind);
    dfree(G.e_pt);
    dfree(G.e_src);
    dfree(G.e_w);
    dfree(G.d_mp);
    dfree(G.band);
    dfree(G.d_band_off);
    dfree(G.reg_map);
    dfree(G.reg_pt);
    dfree(G.bbox);
    dfree(G.bg_k);
    dfree(G.bg_loc);
    dfree(G.bg_w);
    dfree(G.bg_dt);
    dfree(G.wg_rows);
    dfree(G.f_code);
    dfree(G.f_loc);
    dfree(G.g_rowof);
    dfree(G.e_rowof);
    dfree(ctx->v64[l].x);
    dfree(ctx->v64[l].b);
    dfree(ctx->v64[l].r);
    dfree(ctx->v64[l].y);
    dfree(ctx->v32[l].y);
    dfree(ctx->v32[l].x);
    dfree(ctx->v32[l].b);
    dfree(ctx->v32[l].r);
    dfree(ctx->adj[l].x);
    dfree(ctx->adj[l].b);
    dfree(ctx->adj[l].r);
  }
  dfree(ctx->a_g);
  dfree(ctx->a_lam);
  adjoint_free_tabs(ctx);
  tape_free(ctx);
  for (auto &g : ctx->g_iter)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto e : ctx->probe_ev)
    if (e) (void)hipEventDestroy(e);
  ctx->probe_ev.clear();
  if (ctx->h_rmax) (void)hipHostFree(ctx->h_rmax);
  dfree(ctx->phi);
  dfree(ctx->gtmp);
  dfree(ctx->gtmp2);
  dfree(ctx->d_red);
  dfree(ctx->d_ticket);
  dfree(ctx->d_scal);
  dfree(ctx->d_lev);
  dfree(ctx->d_gpart);
  dfree(ctx->d_bcnt);
  dfree(ctx->d_iscr);
  dfree(ctx->d_flags);
  for (int l = 0; l < MAXLEV; l++) {
    BuildRes &B = ctx->bres[l];
    if (B.ev) (void)hipEventDestroy(B.ev);
    if (B.hbuf) (void)hipHostFree(B.hbuf);
    if (l == 0) continue;
    dfree(B.flags);
    dfree(B.bcnt);
    dfree(B.iscr);
    dfree(B.red);
    if (B.s) (void)hipStreamDestroy(B.s);
  }
  dfree(ctx->c_map);
  dfree(ctx->c_A);
  dfree(ctx->c_B);
  dfree(ctx->c_bmap);
  dfree(ctx->c_work);
  for (int k = 0; k < 3; k++) {
    dfree(ctx->cu[k]);
    dfree(ctx->cv[k]);
  }
  dfree(ctx->lapu);
  dfree(ctx->lapv);
  dfree(ctx->fbase);
  dfree(ctx->cku);
  dfree(ctx->ckv);
  dfree(ctx->fwork);
  for (double *p : {ctx->kr.r, ctx->kr.z, ctx->kr.Q, ctx->kr.Z, ctx->kr.zero, ctx->kr.s, ctx->kr.part}) dfree(p);
  for (void *p : {(void *)ctx->rl_a, (void *)ctx->rl_b, (void *)ctx->rl_d, (void *)ctx->rl_c}) dfree(p);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

gp_status gp_setup_grid(gp_ctx **out, int N, double Re, const gp_params *prm, void *hip_stream) {
  if (!out) return GP_EINVAL;
  *out = nullptr;
  gp_params P;
  if (prm)
    P = *prm;
  else
    gp_default_params(&P);
  if (!pow2(N) || N < 16 || !pow2(P.coarsest_n) || P.coarsest_n < 4 || P.coarsest_n > N / 2 || P.nu1 < 0 || P.nu2 < 0 ||
      P.gamma < 1 || P.lambda_ghost < 0 || P.march_max < 1 || P.ext_radius < 1 || !(Re > 0) || P.mixed_inner_cycles < 1 ||
      P.bnd_sweeps < 0 || P.bnd_radius < 0 || P.band_split_min < 1 || P.band_sector_min < 1 ||
      (P.ghost_boxes != 0 && P.ghost_boxes != 1) || P.krylov < 0 || P.krylov > 64 ||
      P.ghost_box_levels < 0)
    return GP_EINVAL;
  gp_ctx *ctx = new gp_ctx();
  ctx->N = N;
  ctx->Re = Re;
  ctx->prm = P;
  ctx->small_cycles = P.fuse_small_levels ? 1 : 0;
  ctx->band_split_min = P.band_split_min;
  ctx->graphs = P.graph_iterations ? 1 : 0;
  ctx->band_sector_min = P.band_sector_min;
  ctx->queue_ahead = P.queue_ahead ? 1 : 0;
  ctx->stream = (hipStream_t)hip_stream;
  if (!ctx->stream) {  // graphs are captured from the context's stream, which cannot be the null stream
    if (hipStreamCreate(&ctx->stream) != hipSuccess) {
      delete ctx;
      return GP_EHIP;
    }
    ctx->own_stream = true;
  }
  int L = 0;
  for (int n = N; n >= P.coarsest_n; n /= 2) {
    Geo &G = ctx->geo[L];
    G.N = n;
    G.W = n + 2;
    G.WW = G.W * G.W;
    G.n = 3 * G.WW + 1;
    G.h = 2.0 / n;
    G.lstride = N / n;
    G.gcap = 48 * n + 4096;
    G.ecap = 96 * n + 4096;
    G.fcap = 4 * G.gcap + 8 * n + 4096;
    G.bcap = 24 * n + 4096;
    L++;
  }
  ctx->L = L;
  gp_status st = GP_OK;
#define ALLOC(p, n)                      \
  if ((st = dalloc(ctx, &(p), (n)))) { \
    gp_destroy(ctx);                     \
    return st;                           \
  }
  size_t gmax = 0;
  for (int l = 0; l < L; l++) {
    Geo &G = ctx->geo[l];
    ALLOC(G.cls, (size_t)3 * G.WW);
    ALLOC(G.g_pt, (size_t)G.gcap);
    ALLOC(G.g_col, (size_t)9 * G.gcap);
    ALLOC(G.g_colr, (size_t)9 * G.gcap);
    ALLOC(G.g_colrT, (size_t)9 * G.gcap);
    ALLOC(G.g_wT, (size_t)9 * G.gcap);
    ALLOC(G.g_w, (size_t)9 * G.gcap);
    ALLOC(G.g_dtau, (size_t)G.gcap);
    ALLOC(G.g_B, (size_t)2 * G.gcap);
    ALLOC(G.g_nB, (size_t)2 * G.gcap);
    ALLOC(G.g_th, (size_t)2 * G.gcap);
    ALLOC(G.g_kind, (size_t)G.gcap);
    ALLOC(G.e_pt, (size_t)G.ecap);
    ALLOC(G.e_src, (size_t)3 * G.ecap);
    ALLOC(G.e_w, (size_t)3 * G.ecap);
    ALLOC(G.d_mp, 1);
    ALLOC(G.band, (size_t)G.N * G.N);
    ALLOC(G.d_band_off, 8);
    ALLOC(G.reg_map, (size_t)3 * G.WW + 1);
    ALLOC(G.reg_pt, (size_t)G.gcap * 12 + (size_t)32 * G.N + 4096);
    ALLOC(G.bbox, (size_t)23 * G.bcap);
    ALLOC(G.bg_k, (size_t)G.gcap);
    ALLOC(G.bg_loc, (size_t)10 * G.gcap);
    ALLOC(G.bg_w, (size_t)9 * G.gcap);
    ALLOC(G.bg_dt, (size_t)G.gcap);
    ALLOC(G.wg_rows, (size_t)G.gcap);
    ALLOC(G.f_code, (size_t)G.fcap);
    if (G.N >= 256) {  // band sectors (large bands only)
      const size_t regcap = (size_t)G.gcap * 12 + (size_t)32 * G.N + 4096;
      G.sec_rcap = (int)regcap;
      G.sec_pcap = (int)(4 * regcap);
      G.sec_bcap = 4 * G.bcap;
      G.sec_gcap = 4 * G.gcap;
      ALLOC(G.sec_pt, (size_t)G.sec_pcap);
      ALLOC(G.sec_mask, regcap);
      ALLOC(G.sec_lmap, 4 * regcap);
      ALLOC(G.sec_out, regcap);
      ALLOC(G.sec_own_loc, regcap);
      ALLOC(G.sec_own_g, regcap);
      ALLOC(G.sec_bsl, (size_t)21 * G.sec_bcap);
      ALLOC(G.sec_bfl, (size_t)G.sec_bcap);
      ALLOC(G.sec_bcell, (size_t)G.sec_bcap);
      ALLOC(G.sec_gl, (size_t)10 * G.sec_gcap);
      ALLOC(G.sec_gw, (size_t)9 * G.sec_gcap);
      ALLOC(G.sec_gdt, (size_t)G.sec_gcap);
      ALLOC(G.sec_gk, (size_t)G.sec_gcap);
    }
    ALLOC(G.f_loc, (size_t)G.fcap);
    if (P.ghost_boxes && l < P.ghost_box_levels) {  // coupled ghost boxes
      G.xb_bcap = G.gcap;
      G.xb_scap = 8 * G.gcap;
      G.xb_icap = 24L * G.gcap;
      ALLOC(G.xb_cell, (size_t)G.xb_bcap);
      ALLOC(G.xb_off, (size_t)G.xb_bcap + 1);
      ALLOC(G.xb_ioff, (size_t)G.xb_bcap + 1);
      ALLOC(G.xb_gcnt, (size_t)G.xb_bcap);
      ALLOC(G.xb_gtmp, (size_t)48 * G.xb_bcap);
      ALLOC(G.xb_ok, (size_t)G.xb_bcap);
      ALLOC(G.xb_idx, (size_t)G.xb_scap);
      ALLOC(G.xb_box, (size_t)G.xb_scap);
      ALLOC(G.xb_wr, (size_t)G.xb_scap);
      ALLOC(G.xb_r, (size_t)G.xb_scap);
      ALLOC(G.xb_inv, (size_t)G.xb_icap);
      ALLOC(G.xb_gc, (size_t)9 * G.xb_scap);
      ALLOC(G.xb_gw, (size_t)9 * G.xb_scap);
      ALLOC(G.xb_uk, (size_t)G.xb_scap);
      ALLOC(G.xb_uo, (size_t)G.xb_scap);
      ALLOC(G.xb_ub, (size_t)G.xb_scap);
      ALLOC(G.xb_um, (size_t)G.xb_scap);
      ALLOC(G.xb_own, (size_t)5 * G.gcap);
      ALLOC(G.d_xb_co, 16);
    }
    ALLOC(G.g_rowof, (size_t)G.n);
    ALLOC(G.e_rowof, (size_t)G.n);
    ALLOC(ctx->v64[l].x, (size_t)G.n);
    ALLOC(ctx->v64[l].b, (size_t)G.n);
    ALLOC(ctx->v64[l].r, (size_t)G.n);
    if (G.N >= 64) ALLOC(ctx->v64[l].y, (size_t)G.n);
    gmax = std::max(gmax, (size_t)G.gcap);
    GP_HIP(hipMemsetAsync(ctx->v64[l].x, 0, G.n * sizeof(double), ctx->stream));
    GP_HIP(hipMemsetAsync(ctx->v64[l].b, 0, G.n * sizeof(double), ctx->stream));
    GP_HIP(hipMemsetAsync(ctx->v64[l].r, 0, G.n * sizeof(double), ctx->stream));
  }
  ALLOC(ctx->phi, (size_t)(2 * N + 1) * (2 * N + 1));
  ALLOC(ctx->gtmp, gmax);
  ALLOC(ctx->gtmp2, gmax);
  // block partials: two per block of the finest residual norm (points and ghost rows)
  ALLOC(ctx->d_red, std::max<size_t>(8192, 2 * ((size_t)nblk(3L * (N + 2) * (N + 2)) + (size_t)nblk((long)gmax)) + 16));
  {
    void *hp = nullptr;
    GP_HIP(hipHostMalloc(&hp, 64, hipHostMallocCoherent));
    ctx->h_rmax = (unsigned long long *)hp;
  }
  ALLOC(ctx->d_ticket, 4);
  ALLOC(ctx->d_scal, 16);
  ALLOC(ctx->d_lev, 2 * MAXLEV);
  {  // block partials of G written by the restriction onto each coarse level (see k_resid_restrict)
    size_t tot = 16;
    for (int l = 1; l < L; l++) {
      Geo &G = ctx->geo[l];
      G.gp_off = (int)tot;
      G.gp_n = nblk(3L * G.WW + 1) - 2 * G.WW / TPB;
      tot += (size_t)G.gp_n + 16;
    }
    ALLOC(ctx->d_gpart, tot);
    for (int l = 0; l < L; l++) {
      ctx->gs_ptr[l] = ctx->d_lev + l;
      ctx->gs_n[l] = 1;
    }
  }
  ALLOC(ctx->d_bcnt, (size_t)8 * nblk((long)(N + 2) * (N + 2)) + 16);  // two scans of 3 (N+2)^2 points, or 5 colours
  ALLOC(ctx->d_iscr, (size_t)3 * (N + 2) * (N + 2) + 1);
  ALLOC(ctx->d_flags, 16);
  // geometry build resources: level 0 the context's own, the others a stream, event and scratch each
  GP_HIP(hipGetDevice(&ctx->device));
  (void)scratch_init(ctx);  // address of the static scratch on this device (gp_solve_noalloc reports a failure)
  for (int l = 0; l < L; l++) {
    BuildRes &B = ctx->bres[l];
    GP_HIP(hipEventCreateWithFlags(&B.ev, hipEventDisableTiming));
    {
      void *hp = nullptr;
      GP_HIP(hipHostMalloc(&hp, 4096, hipHostMallocCoherent));
      B.hbuf = (int *)hp;
      B.hseq = (unsigned *)(B.hbuf + 1020);
      *B.hseq = 0;
      B.seq = 0;
    }
    if (l == 0) {
      B.s = ctx->stream;
      B.flags = ctx->d_flags;
      B.bcnt = ctx->d_bcnt;
      B.iscr = ctx->d_iscr;
      B.red = ctx->d_red;
      continue;
    }
    const long WWl = (long)ctx->geo[l].WW;
    GP_HIP(hipStreamCreate(&B.s));
    ALLOC(B.flags, 16);
    ALLOC(B.bcnt, (size_t)8 * nblk(WWl) + 16);
    ALLOC(B.iscr, (size_t)3 * WWl + 1);
    ALLOC(B.red, 16);
  }
  GP_HIP(hipMemsetAsync(ctx->d_ticket, 0, 4 * sizeof(unsigned), ctx->stream));
  GP_HIP(hipMemsetAsync(ctx->d_lev, 0, 2 * MAXLEV * sizeof(double), ctx->stream));
  Geo &C = ctx->geo[L - 1];
  ALLOC(ctx->c_map, (size_t)3 * C.WW + 2);
  ALLOC(ctx->c_A, (size_t)1024 * 1024);
  ALLOC(ctx->c_B, (size_t)1024 * 1024);
  ALLOC(ctx->c_bmap, 1024);
  ALLOC(ctx->c_work, (size_t)4 * (3 * C.WW + 1) + 2048);
  int WW = ctx->geo[0].WW;
  for (int k = 0; k < 3; k++) {
    ALLOC(ctx->cu[k], (size_t)WW);
    ALLOC(ctx->cv[k], (size_t)WW);
  }
  ALLOC(ctx->lapu, (size_t)WW);
  ALLOC(ctx->lapv, (size_t)WW);
  ALLOC(ctx->fbase, (size_t)2 * WW);
  ALLOC(ctx->cku, (size_t)WW);
  ALLOC(ctx->ckv, (size_t)WW);
  ALLOC(ctx->fwork, (size_t)3 * WW + 1);
#undef ALLOC
  {
    int dev = 0, lds = 0;
    GP_HIP(hipGetDevice(&dev));
    GP_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    ctx->max_lds = (size_t)lds;
  }
  GP_HIP(hipStreamSynchronize(ctx->stream));
  *out = ctx;
  return GP_OK;
}

gp_status gp_set_levelset(gp_ctx *ctx, const double *phi, int on_device, double t, const gp_rigid *motion) {
  if (!ctx || !phi) return GP_EINVAL;
  prep_discard(ctx);
  size_t n = (size_t)(2 * ctx->N + 1) * (2 * ctx->N + 1);
  gp_status st = stage_in(ctx, phi, on_device, ctx->phi, n);
  if (st) return st;
  ctx->t_geom = t;
  ctx->motion = motion ? *motion : gp_rigid{0, 0, 0, 0, 0};
  return after_geometry(ctx);
}

gp_status gp_set_levelset_analytic(gp_ctx *ctx, const gp_shape *shape, double t, const gp_rigid *motion) {
  if (!ctx || !shape || shape->kind < 0 || shape->kind > 5) return GP_EINVAL;
  if (ctx->prep_active) {
    prep_discard(ctx);
    const gp_rigid mo = motion ? *motion : gp_rigid{0, 0, 0, 0, 0};
    if (ctx->prep_status == GP_OK && same_shape(*shape, ctx->prep_shape) && t == ctx->prep_t &&
        same_motion(mo, ctx->prep_motion)) {
      GP_HIP(hipStreamWaitEvent(ctx->stream, ctx->prep_done, 0));
      take_prepared(ctx);
      ctx->t_geom = t;
      ctx->motion = mo;
      return default_boundary_values(ctx);
    }
  }
  gp_status st = levelset_analytic(ctx, shape, t, motion);
  if (st) return st;
  ctx->t_geom = t;
  ctx->motion = motion ? *motion : gp_rigid{0, 0, 0, 0, 0};
  return after_geometry(ctx);
}

gp_status gp_prepare_levelset_analytic(gp_ctx *ctx, const gp_shape *shape, double t, const gp_rigid *motion) {
  if (!ctx || !shape || shape->kind < 0 || shape->kind > 5) return GP_EINVAL;
  prep_discard(ctx);
  if (!ctx->shadow) {
    gp_ctx *sh = nullptr;
    gp_status st = gp_setup_grid(&sh, ctx->N, ctx->Re, &ctx->prm, nullptr);
    if (st) return st;
    ctx->shadow = sh;
    GP_HIP(hipEventCreateWithFlags(&ctx->prep_start, hipEventDisableTiming));
    GP_HIP(hipEventCreateWithFlags(&ctx->prep_done, hipEventDisableTiming));
  }
  Ctx *sh = ctx->shadow;
  sh->alpha = ctx->alpha;  // for its early coarsest factorisation
  ctx->prep_shape = *shape;
  ctx->prep_t = t;
  ctx->prep_motion = motion ? *motion : gp_rigid{0, 0, 0, 0, 0};
  ctx->prep_alpha = ctx->alpha;
  // after all work queued on the context's stream so far: it may still read the geometry the shadow holds
  GP_HIP(hipEventRecord(ctx->prep_start, ctx->stream));
  GP_HIP(hipStreamWaitEvent(sh->stream, ctx->prep_start, 0));
  ctx->prep_status = GP_OK;
  ctx->prep_active = true;
  const gp_shape shp = *shape;
  const gp_rigid mo = ctx->prep_motion;
  ctx->prep = std::thread([ctx, sh, shp, t, mo]() {
    gp_status st = hipSetDevice(ctx->device) == hipSuccess ? GP_OK : GP_EHIP;
    if (!st) st = levelset_analytic(sh, &shp, t, &mo);
    if (!st) st = geometry_build(sh);
    if (!st && hipEventRecord(ctx->prep_done, sh->stream) != hipSuccess) st = GP_EHIP;
    ctx->prep_status = st;
  });
  return GP_OK;
}

gp_status gp_set_walls(gp_ctx *ctx, const double *w) {
  if (!ctx || !w) return GP_EINVAL;
  std::memcpy(ctx->walls, w, 8 * sizeof(double));
  if (ctx->have_geom) return default_boundary_values(ctx);
  return GP_OK;
}

gp_status gp_get_boundary_geometry(gp_ctx *ctx, double *B, double *nB) {
  if (!ctx || !ctx->have_geom || !B || !nB) return GP_EINVAL;
  Geo &G = ctx->geo[0];
  int P = 3 * G.WW;
  std::vector<int> pt(G.ng);
  std::vector<double> hB(2 * G.ng), hn(2 * G.ng);
  std::vector<uint8_t> cls(P);
  GP_HIP(hipMemcpyAsync(pt.data(), G.g_pt, G.ng * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  GP_HIP(hipMemcpyAsync(hB.data(), G.g_B, 2 * G.ng * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  GP_HIP(hipMemcpyAsync(hn.data(), G.g_nB, 2 * G.ng * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  GP_HIP(hipMemcpyAsync(cls.data(), G.cls, P, hipMemcpyDeviceToHost, ctx->stream));
  GP_HIP(hipStreamSynchronize(ctx->stream));
  const double nan = std::numeric_limits<double>::quiet_NaN();
  for (int k = 0; k < 2 * P; k++) B[k] = nB[k] = nan;
  for (int r = 0; r < G.ng; r++) {
    int k = pt[r];
    if (cls[k] == K_GHOSTX) continue;
    B[2 * k] = hB[2 * r];
    B[2 * k + 1] = hB[2 * r + 1];
    nB[2 * k] = hn[2 * r];
    nB[2 * k + 1] = hn[2 * r + 1];
  }
  for (int k = 0; k < P; k++) {
    if (cls[k] != K_WALLD) continue;
    int g = k / G.WW, q = k % G.WW, j = q / G.W - 1, i = q % G.W - 1;
    B[2 * k] = (g == 0) ? -1.0 + i * G.h : -1.0 + (i + 0.5) * G.h;
    B[2 * k + 1] = (g == 1) ? -1.0 + j * G.h : -1.0 + (j + 0.5) * G.h;
  }
  return GP_OK;
}

gp_status gp_set_boundary_values(gp_ctx *ctx, const double *bu, const double *bv, const double *bp, int on_device) {
  if (!ctx || !ctx->have_geom) return GP_EINVAL;
  Geo &G = ctx->geo[0];
  const double *src[3] = {bu, bv, bp};
  for (int g = 0; g < 3; g++) {
    if (!src[g]) continue;
    gp_status st = stage_in(ctx, src[g], on_device, ctx->fwork + (size_t)g * G.WW, G.WW);
    if (st) return st;
    k_scatter_pts<<<nblk(G.WW), TPB, 0, ctx->stream>>>(G.cls + g * G.WW, G.WW, 0, ctx->fwork + (size_t)g * G.WW,
                                                       ctx->v64[0].b + (size_t)g * G.WW, ctx->v64[0].x + (size_t)g * G.WW);
  }
  GP_HIP(hipGetLastError());
  GP_HIP(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}

gp_status gp_set_alpha(gp_ctx *ctx, double alpha) {
  if (!ctx || !(alpha >= 0)) return GP_EINVAL;
  if (alpha != ctx->alpha) ctx->c_ok = 0;
  ctx->alpha = alpha;
  return GP_OK;
}

gp_status gp_set_rhs(gp_ctx *ctx, const double *fu, const double *fv, const double *g, int on_device) {
  if (!ctx || !ctx->have_geom) return GP_EINVAL;
  Geo &G = ctx->geo[0];
  const double *src[3] = {fu, fv, g};
  for (int q = 0; q < 3; q++) {
    if (src[q]) {
      gp_status st = stage_in(ctx, src[q], on_device, ctx->fwork + (size_t)q * G.WW, G.WW);
      if (st) return st;
      k_scatter_pts<<<nblk(G.WW), TPB, 0, ctx->stream>>>(G.cls + q * G.WW, G.WW, 1, ctx->fwork + (size_t)q * G.WW,
                                                         ctx->v64[0].b + (size_t)q * G.WW, nullptr);
    } else {
      k_zero_int<<<nblk(G.WW), TPB, 0, ctx->stream>>>(G.cls, q * G.WW, (q + 1) * G.WW, ctx->v64[0].b);
    }
  }
  GP_HIP(hipMemsetAsync(ctx->v64[0].b + 3 * (size_t)G.WW, 0, sizeof(double), ctx->stream));
  GP_HIP(hipGetLastError());
  GP_HIP(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}

gp_status gp_set_x(gp_ctx *ctx, const double *u, const double *v, const double *p, double xi, int on_device) {
  if (!ctx || !u || !v || !p) return GP_EINVAL;
  Geo &G = ctx->geo[0];
  double *x = ctx->v64[0].x;
  gp_status st;
  if ((st = stage_in(ctx, u, on_device, x, G.WW))) return st;
  if ((st = stage_in(ctx, v, on_device, x + G.WW, G.WW))) return st;
  if ((st = stage_in(ctx, p, on_device, x + 2 * (size_t)G.WW, G.WW))) return st;
  GP_HIP(hipMemcpyAsync(x + 3 * (size_t)G.WW, &xi, sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  GP_HIP(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}

gp_status gp_get_x(gp_ctx *ctx, double *u, double *v, double *p, double *xi, int on_device) {
  if (!ctx) return GP_EINVAL;
  Geo &G = ctx->geo[0];
  double *x = ctx->v64[0].x;
  hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (u) GP_HIP(hipMemcpyAsync(u, x, G.WW * sizeof(double), k, ctx->stream));
  if (v) GP_HIP(hipMemcpyAsync(v, x + G.WW, G.WW * sizeof(double), k, ctx->stream));
  if (p) GP_HIP(hipMemcpyAsync(p, x + 2 * (size_t)G.WW, G.WW * sizeof(double), k, ctx->stream));
  if (xi) GP_HIP(hipMemcpyAsync(xi, x + 3 * (size_t)G.WW, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  GP_HIP(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}

gp_status gp_mg_vcycle(gp_ctx *ctx, int precision, double *res_inf) {
  if (!ctx || precision != GP_FP64) return GP_EINVAL;
  gp_status st = ensure_coarse(ctx);
  if (st) return st;
  return mg_cycle64(ctx, res_inf);
}

gp_status gp_solve(gp_ctx *ctx, int precision, double tol, int max_cycles, gp_stats *s) {
  if (!ctx || !(tol > 0) || max_cycles < 0 || (precision != GP_FP64 && precision != GP_MIXED)) return GP_EINVAL;
  gp_status st = ensure_coarse(ctx);
  if (st) return st;
  return mg_solve(ctx, precision, tol, max_cycles, s);
}

gp_status gp_reinit_levelset(gp_ctx *ctx, double *phi, int on_device, int iters, double cfl) {
  if (!ctx || !phi || iters < 0 || !(cfl > 0 && cfl <= 0.5)) return GP_EINVAL;
  return reinit_levelset(ctx, phi, on_device, iters, cfl);
}

gp_status gp_solve_noalloc(gp_ctx *ctx, double tol, int max_cycles, gp_stats *s) {
  if (!ctx || !(tol > 0) || max_cycles < 0) return GP_EINVAL;
  gp_status st = ensure_coarse(ctx);
  if (st) return st;
  return mg_solve_noalloc(ctx, tol, max_cycles, s);
}

gp_status gp_residual(gp_ctx *ctx, double *r, double *res_inf) {
  if (!ctx || !ctx->have_geom) return GP_EINVAL;
  double ri;
  gp_status st = residual64(ctx, 0, &ri);
  if (st) return st;
  if (res_inf) *res_inf = ri;
  if (r) {
    GP_HIP(hipMemcpyAsync(r, ctx->v64[0].r, ctx->geo[0].n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    GP_HIP(hipStreamSynchronize(ctx->stream));
  }
  return GP_OK;
}

gp_status gp_get_classes(gp_ctx *ctx, int level, unsigned char *cls) {
  if (!ctx || !cls || level < 0 || level >= ctx->L) return GP_EINVAL;
  Geo &G = ctx->geo[level];
  GP_HIP(hipMemcpyAsync(cls, G.cls, 3 * (size_t)G.WW, hipMemcpyDeviceToHost, ctx->stream));
  GP_HIP(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}

gp_status gp_get_ghost_rows(gp_ctx *ctx, int level, double *B, double *nB, double *th, double *w9, int *col9, double *dtau,
                            int *kind) {
  if (!ctx || level < 0 || level >= ctx->L || !B || !nB || !th || !w9 || !col9 || !dtau || !kind) return GP_EINVAL;
  Geo &G = ctx->geo[level];
  int P = 3 * G.WW, ng = G.ng;
  std::vector<int> pt(ng), col(9 * ng);
  std::vector<double> hB(2 * ng), hn(2 * ng), ht(2 * ng), hw(9 * ng), hd(ng);
  std::vector<int8_t> hk(ng);
  hipStream_t s = ctx->stream;
  GP_HIP(hipMemcpyAsync(pt.data(), G.g_pt, ng * sizeof(int), hipMemcpyDeviceToHost, s));
  GP_HIP(hipMemcpyAsync(col.data(), G.g_col, 9 * ng * sizeof(int), hipMemcpyDeviceToHost, s));
  GP_HIP(hipMemcpyAsync(hB.data(), G.g_B, 2 * ng * sizeof(double), hipMemcpyDeviceToHost, s));
  GP_HIP(hipMemcpyAsync(hn.data(), G.g_nB, 2 * ng * sizeof(double), hipMemcpyDeviceToHost, s));
  GP_HIP(hipMemcpyAsync(ht.data(), G.g_th, 2 * ng * sizeof(double), hipMemcpyDeviceToHost, s));
  GP_HIP(hipMemcpyAsync(hw.data(), G.g_w, 9 * ng * sizeof(double), hipMemcpyDeviceToHost, s));
  GP_HIP(hipMemcpyAsync(hd.data(), G.g_dtau, ng * sizeof(double), hipMemcpyDeviceToHost, s));
  GP_HIP(hipMemcpyAsync(hk.data(), G.g_kind, ng, hipMemcpyDeviceToHost, s));
  GP_HIP(hipStreamSynchronize(s));
  const double nan = std::numeric_limits<double>::quiet_NaN();
  for (int k = 0; k < P; k++) {
    for (int q = 0; q < 2; q++) B[2 * k + q] = nB[2 * k + q] = th[2 * k + q] = nan;
    for (int q = 0; q < 9; q++) {
      w9[9 * k + q] = nan;
      col9[9 * k + q] = -1;
    }
    dtau[k] = nan;
    kind[k] = -1;
  }
  for (int r = 0; r < ng; r++) {
    int k = pt[r];
    for (int q = 0; q < 2; q++) {
      B[2 * k + q] = hB[2 * r + q];
      nB[2 * k + q] = hn[2 * r + q];
      th[2 * k + q] = ht[2 * r + q];
    }
    for (int q = 0; q < 9; q++) {
      w9[9 * k + q] = hw[9 * r + q];
      col9[9 * k + q] = col[9 * r + q];
    }
    dtau[k] = hd[r];
    kind[k] = hk[r];
  }
  return GP_OK;
}

gp_status gp_get_ext_rows(gp_ctx *ctx, int level, int *src3, double *w3) {
  if (!ctx || level < 0 || level >= ctx->L || !src3 || !w3) return GP_EINVAL;
  Geo &G = ctx->geo[level];
  int P = 3 * G.WW, ne = G.ne;
  std::vector<int> pt(ne), src(3 * ne);
  std::vector<double> w(3 * ne);
  GP_HIP(hipMemcpyAsync(pt.data(), G.e_pt, ne * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  GP_HIP(hipMemcpyAsync(src.data(), G.e_src, 3 * ne * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  GP_HIP(hipMemcpyAsync(w.data(), G.e_w, 3 * ne * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  GP_HIP(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < 3 * P; k++) {
    src3[k] = -1;
    w3[k] = std::numeric_limits<double>::quiet_NaN();
  }
  for (int e = 0; e < ne; e++) {
    if (src[3 * e] < 0) continue;
    for (int q = 0; q < 3; q++) {
      src3[3 * pt[e] + q] = src[3 * e + q];
      w3[3 * pt[e] + q] = w[3 * e + q];
    }
  }
  return GP_OK;
}

gp_status gp_relax(gp_ctx *ctx, int level, int steps) {
  if (!ctx || !ctx->have_geom || level < 0 || level >= ctx->L || steps < 0) return GP_EINVAL;
  return relax64(ctx, level, steps);
}

gp_status gp_time_kernel(gp_ctx *ctx, int which, int level, int reps, double *avg_us) {
  if (!ctx || !ctx->have_geom || level < 0 || level >= ctx->L || reps < 1 || !avg_us) return GP_EINVAL;
  return time_kernel(ctx, which, level, reps, avg_us);
}

gp_status gp_probe_start(gp_ctx *ctx, int max_launches, int every) {
  if (!ctx || max_launches < 1 || max_launches > (1 << 16) || every < 1 || every > 64) return GP_EINVAL;
  return probe_start(ctx, max_launches, every);
}

gp_status gp_probe_stop(gp_ctx *ctx, double *avg_us, int *launches) {
  if (!ctx || !avg_us || !launches) return GP_EINVAL;
  return probe_stop(ctx, avg_us, launches);
}

}  // extern "C"
