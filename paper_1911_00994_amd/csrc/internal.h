// Internal declarations of the gpmg HIP library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "../../include/gpmg.h"

namespace gpmg {

// point classes (same numbering as the public GP_* class constants; BODY is transient)
enum : uint8_t {
  K_INACTIVE = 0,
  K_INT = 1,
  K_GHOST = 2,
  K_WALLD = 3,
  K_WALLG = 4,
  K_EXT = 5,
  K_BODY = 6,
  K_GHOSTX = 7
};

constexpr int SEC_MAX = 16;  // angular sectors of a band, at most
constexpr int MAXLEV = 16;
constexpr int TPB = 256;

// geometry of one level (device pointers), shared by the FP64 and FP32 hierarchies
struct Geo {
  int N = 0, W = 0, WW = 0, n = 0;  // n = 3*WW + 1 unknowns (xi last)
  double h = 0;
  int lstride = 1;                  // level lattice step in fine lattice steps
  uint8_t *cls = nullptr;           // 3*WW
  // ghost rows (GHOST, GHOSTX, WALLG): compact, unordered
  int ng = 0, gcap = 0;
  int *g_pt = nullptr;              // global unknown index
  int *g_col = nullptr;             // 9 per row
  int *g_colr = nullptr;            // g_col with every ghost point given as -(its row + 1)
  int *g_colrT = nullptr;           // g_colr and g_w column-major ([z ng + r]): a wavefront's loads of one column of
  double *g_wT = nullptr;           // consecutive rows are contiguous
  double *g_w = nullptr;            // 9 per row
  double *g_dtau = nullptr;
  double *g_B = nullptr, *g_nB = nullptr, *g_th = nullptr;  // 2 per row
  int8_t *g_kind = nullptr;         // 1 BC row, 2 extrapolation, 0 identity
  // extension points: compact
  int ne = 0, ecap = 0;
  int *e_pt = nullptr, *e_src = nullptr;  // 3 sources per point (-1 none)
  double *e_w = nullptr;
  int *d_mp = nullptr;              // device: number of internal pressure points
  int mp = 0;                       // host copy
  // cells of the boundary band, grouped by colour: band[band_off[c] .. band_off[c+1]) (cell index j*N + i)
  int *band = nullptr;
  int *d_band_off = nullptr;        // device: 6 offsets
  int nband = 0;                    // host copy of the total
  int hband_off[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // boundary region staged in LDS by the band kernel: region points (global index, ascending), global -> local
  // map, per band box (field-major, stride bcap) the local indices of its 21 values, its free-unknown flags and
  // its cell, body ghost rows in point order (field-major, stride gcap: point, 10 local indices, 9 weights,
  // fictitious time step), wall ghost rows (row ids)
  int *reg_pt = nullptr, *reg_map = nullptr, *bbox = nullptr, *bg_k = nullptr, *bg_loc = nullptr, *wg_rows = nullptr;
  double *bg_w = nullptr, *bg_dt = nullptr;
  int bcap = 0;
  int nreg = 0, nregw = 0, nbg = 0, nwg = 0;  // region points (the first nregw are written), body and wall rows
  int lds_ok = 0;                   // 1 when the LDS band kernel applies to this level
  // angular sectors of the band, one workgroup each (see sector_build): per sector s its region points
  // (sec_pt, global index; local slot = position), band boxes by colour (sec_bsl 21 local slots as 16-bit numbers,
  // field-major; sec_bfl flags; sec_bcell cell), body ghost rows (sec_gl own + 9 column local slots, 16-bit; sec_gw
  // 9 weights; sec_gdt; sec_gk the point, for its right-hand side) and owned written points (sec_own_loc local
  // slot, sec_own_g region index, whose value goes to sec_out[region index]); all field-major with the totals
  // as strides
  int sec_S = 0;
  int sec_poff[SEC_MAX + 1] = {0}, sec_boff[5 * SEC_MAX + 1] = {0}, sec_goff[SEC_MAX + 1] = {0},
      sec_ooff[SEC_MAX + 1] = {0};
  int sec_maxreg = 0, sec_maxrow = 0;  // largest region and row count of a sector
  int *sec_pt = nullptr, *sec_bfl = nullptr, *sec_bcell = nullptr, *sec_gk = nullptr, *sec_own_loc = nullptr,
      *sec_own_g = nullptr, *sec_mask = nullptr, *sec_lmap = nullptr;
  uint16_t *sec_bsl = nullptr, *sec_gl = nullptr;
  double *sec_gw = nullptr, *sec_gdt = nullptr, *sec_out = nullptr;
  int sec_pcap = 0, sec_bcap = 0, sec_gcap = 0, sec_rcap = 0;
  int colr_ok = 0;                  // 1 when g_colr holds the row of every ghost column
  int gp_off = 0, gp_n = 0;         // this level's block partials of G in Ctx::d_gpart (written by the restriction)
  // row of each ghost point in g_pt and of each extension point in e_pt (3 W^2 + 1 entries; others undefined)
  int *g_rowof = nullptr, *e_rowof = nullptr;
  // faces on the boundary of the internal pressure cells, cell-major order: code = 2 * (u or v index) + (1 if the
  // face enters the cell's divergence with a minus sign); f_loc = the same face as an LDS band-region entry
  int *f_code = nullptr, *f_loc = nullptr;
  int nf = 0, fcap = 0;
  // coupled ghost boxes: the cells whose internal unknowns appear in a body ghost row, each relaxed together with
  // those ghosts.  Boxes ordered by colour, then cell; per box its unknowns (slots xb_off[b] .. xb_off[b+1]: the
  // internal box unknowns W, E, S, N face, pressure, then its ghosts in point order), per slot the box and whether
  // the box writes the value (a ghost is written by the first box of a colour that holds it), per box the inverse
  // of its block (row-major, at xb_ioff[b]) for the alpha xb_alpha and a flag (0: singular block, not relaxed)
  int nxb = 0, nxs = 0;
  int xb_coff[6] = {0, 0, 0, 0, 0, 0}, xb_soff[6] = {0, 0, 0, 0, 0, 0};  // host: box and slot offsets per colour
  int xb_maxs = 0;                  // most slots of one colour
  int xb_bcap = 0, xb_scap = 0;
  long xb_icap = 0;
  int *xb_cell = nullptr, *xb_off = nullptr, *xb_ioff = nullptr, *xb_idx = nullptr, *xb_box = nullptr;
  int *xb_gcnt = nullptr, *xb_gtmp = nullptr, *xb_own = nullptr, *d_xb_co = nullptr;
  uint8_t *xb_wr = nullptr, *xb_ok = nullptr;
  double *xb_inv = nullptr, *xb_r = nullptr;
  // the same tables flattened per slot, so a relaxation kernel reaches everything it needs in one dependent load:
  // xb_gc / xb_gw the 9 columns and weights of a ghost slot's row (field-major, stride xb_scap; xb_gc[s] = -1 for
  // an internal slot), and for the write phase (refreshed with the inverses) xb_uk the point a slot writes (-1: the
  // box does not write it, or its block is singular), xb_uo the offset of its row of the inverse, xb_ub the box's
  // first slot and xb_um the box's size
  int *xb_gc = nullptr, *xb_uk = nullptr, *xb_uo = nullptr, *xb_ub = nullptr, *xb_um = nullptr;
  double *xb_gw = nullptr;
  double xb_alpha = -1;
  long gen = 0;                     // identity of this build of the level's tables (fresh on every build)
};

// transposed scatter table of the reverse mode.  A table of items with K entries each (entry e = item * K + z) and a
// target point per entry is regrouped by target: tl[0 .. nt) the targets that receive entries, ent[off[s] ..
// off[s + 1]) the entries of target tl[s] in ascending order, so that a gather over one target adds its entries in
// a fixed order (the scatter it replaces added them with atomics, in arrival order).  nt lives on the device.
struct TTab {
  int *tl = nullptr, *off = nullptr, *ent = nullptr, *cur = nullptr, *d_nt = nullptr;
  double *coef = nullptr;           // per entry: its matrix coefficient (coupled-box tables only)
  int cap_t = 0, cap_e = 0, cap_c = 0;
  int ne = 0;                       // entries of the table (host)
};
struct AdjTabs {
  long gen = -1;                    // Geo::gen of the tables below
  TTab gt, et, xt[5];               // ghost rows (K = 9), extension points (K = 3), coupled-box slots of each
                                    // colour (K = 10)
  double xa = 0;                    // the a of the coupled-box coefficients (valid when xok)
  bool xok = false;
};

// one precision's vectors on one level
template <typename T>
struct Vec {
  T *x = nullptr, *b = nullptr, *r = nullptr;
  T *y = nullptr;  // second buffer of x for sweeps that read one copy and write the other (swapped afterwards)
};

// saved time-stepping state of the finest level: x (3*WW + 1), then the convection history c^n, c^{n-1},
// c^{n-2} (u and v grids) and the Laplacian of u^n (u and v): 11*WW + 1 doubles
struct CnSnap {
  double *buf = nullptr;
  int nstep = 0;
};

// record of a run of Crank-Nicolson steps for the reverse pass (checkpoints every K steps)
struct Tape {
  int valid = 0, nsteps = 0, K = 8;
  gp_shape shape{};
  gp_rigid motion{};
  double t0 = 0, dt = 0, ub_off[2] = {0, 0};
  double tol = 1e-10, picard_eps = 1e-6;
  int max_cycles = 100, picard_max = 20;
  double *fu = nullptr, *fv = nullptr;  // forcing (device, W*W each)
  std::vector<CnSnap> ckpt;             // state before steps 0, K, 2K, ...
  std::vector<CnSnap> seg;              // K + 1 states of the segment being reversed
  CnSnap last;                          // state after the last step
  // reverse pass: adjoint of the state (full vector), of the filled state of a fixed-point step, ring of the
  // convection-history adjoints (c^{n+1}, c^n, c^{n-1}, c^{n-2}; u and v), forcing adjoint, scratch
  double *xb = nullptr, *yb = nullptr, *xbn = nullptr, *lamp = nullptr, *ring = nullptr, *fb = nullptr, *tcb = nullptr;
  double *ub = nullptr;                 // device [2]: adjoint of the boundary-velocity offset
  // device [2]: the part of dJ/dU that comes through the body path X(t) = X0 + U t (the rows' dependence on the
  // body position), its per-point scratch (3 W^2 each) and the count of rows whose path could not be replayed
  double *upath = nullptr, *pcx = nullptr, *pcy = nullptr;
  int *d_mism = nullptr;
  double h_upath[2] = {0, 0};
  int h_mism = 0;
  int ring_head = 0;
};

// a level's stream, event and scratch for the geometry build (level 0: the context's own)
struct BuildRes {
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  int *flags = nullptr, *bcnt = nullptr, *iscr = nullptr;
  double *red = nullptr;
  int *hbuf = nullptr;        // pinned host words for the read-backs (fetch)
  unsigned *hseq = nullptr;   // in hbuf: the sequence number of the last read-back that arrived
  unsigned seq = 0;           // the last one issued
};

// GCR workspace (gcr_solve): the residual, the preconditioned direction, m stored directions Z and their images
// Q, a zero vector (n doubles each), device scalars (the Gram-Schmidt coefficients, then |q|^2, (r, q) and the
// step) and the block partials of the reductions.  Either the context's own buffers (gcr_alloc) or slices of the
// library's static scratch array (gp_solve_noalloc).
struct GcrWs {
  int m = 0;
  double *r = nullptr, *z = nullptr, *Q = nullptr, *Z = nullptr, *zero = nullptr, *s = nullptr, *part = nullptr;
};

struct Ctx {
  int N = 0, L = 0;
  double Re = 100, alpha = 0;
  gp_params prm{};
  hipStream_t stream = nullptr;
  bool own_stream = false;  // created by the context (the caller passed none)
  std::string hip_err;
  std::mutex err_mu;
  int device = 0;                   // the device the context was set up on
  BuildRes bres[MAXLEV];
  Geo geo[MAXLEV];
  Vec<double> v64[MAXLEV];
  Vec<float> v32[MAXLEV];
  Vec<double> adj[MAXLEV];          // transposed cycle: x = adjoint of x, b = adjoint of b, r = adjoint of r
  double *a_g = nullptr, *a_lam = nullptr;  // transposed solve: right-hand side and solution (finest)
  AdjTabs atab[MAXLEV];             // transposed scatter tables per level
  int *tt_cnt = nullptr, *tt_pos = nullptr, *tt_tgt = nullptr;  // table build scratch (points; entries)
  int tt_ccap = 0, tt_tcap = 0;
  double *a_S = nullptr;            // transposed box colour: the five box values per cell (finest size)
  Tape tape;
  double *phi = nullptr;            // fine half lattice (2N+1)^2
  double *gtmp = nullptr, *gtmp2 = nullptr;  // ghost Jacobi scratch, row-indexed (max gcap each)
  // reductions / flags
  double *d_red = nullptr;          // partial sums (blocks) scratch
  unsigned int *d_ticket = nullptr; // last-block tickets
  double *d_lev = nullptr;          // per level: [l] sum of the continuity right-hand sides over internal cells
  int *d_bcnt = nullptr;            // per-block counts of the deterministic compactions
  int *d_iscr = nullptr;            // point-indexed int scratch (finest size)
  double *d_scal = nullptr;         // device scalars: [0] mean p, [1] res max (as bits), [2..] misc
  int *d_flags = nullptr;           // device flags: [0] changed, [1] geometry error bits, [2] ghost count, [3] ext count, [4] bad rows
  int have_geom = 0;
  double t_geom = 0;
  gp_rigid motion{};
  double ub_off[2] = {0, 0};        // offset added to the rigid boundary velocity of the body rows (path unchanged)
  double walls[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // coarsest exact solve: compacted active unknowns and explicit inverse (FP64)
  int nc = 0;                       // number of active unknowns on the coarsest level
  int *c_map = nullptr;             // nc: global index of each active unknown
  int *c_bmap = nullptr;            // nc: right-hand side index for each column of the stored inverse
  double *c_A = nullptr, *c_B = nullptr;  // nc*nc matrix and a second buffer (the blocked inversion alternates)
  double *c_inv = nullptr;          // the buffer holding the inverse (c_A or c_B)
  double *c_work = nullptr;         // nc*nc scratch
  int c_ok = 0;
  // time-stepping state (finest level)
  int nstep = 0;
  double *cu[3] = {nullptr, nullptr, nullptr}, *cv[3] = {nullptr, nullptr, nullptr};
  double *lapu = nullptr, *lapv = nullptr, *fbase = nullptr, *cku = nullptr, *ckv = nullptr;
  double *fwork = nullptr;          // 3*WW staging for inputs
  int last_cycles = 0;
  size_t max_lds = 65536;           // dynamic LDS a workgroup may use on this device
  int small_cycles = 1;             // run the levels with N <= 32 as one workgroup when they fit in LDS
  int band_split_min = 3000;        // bands with at least this many cells use device-wide launches
  int band_sector_min = 1500;       // bands with at least this many cells use angular sectors where possible
  int box_tiles = 1;                // all five colours of a box sweep in one launch (LDS tiles with halos)
  // launch probe: HIP event pairs around the finest-level five-colour box launches of the FP64 cycle
  std::vector<hipEvent_t> probe_ev;
  int probe_n = 0;
  int probe_every = 1, probe_seq = 0;  // events on launch probe_seq = 0, every, 2 every, ... (seq counts them all)
  // one solver iteration as an executable HIP graph, per precision (captured per solve, updated in place)
  int graphs = 1;
  hipGraphExec_t g_iter[2] = {nullptr, nullptr};
  // the finest residual norm for the host: k_resid_mean_row also stores it in pinned host memory (h_rmax), which
  // the solver polls
  unsigned long long *h_rmax = nullptr;
  // the first box sweep of the next FP64 cycle, queued before the host has the norm (queue_head); the device
  // skips it when the solve stops there
  int queue_ahead = 1;
  // G of each level (see gp_start): its partials and their number; d_lev + l (one) after gsum(l), the block sums
  // of the restriction onto level l after it (d_gpart + gp_off, gp_n)
  double *d_gpart = nullptr;
  const double *gs_ptr[MAXLEV] = {nullptr};
  int gs_n[MAXLEV] = {0};
  bool head_queued = false, head_probe = false;
  // generalized conjugate residual iteration around the cycle (finest-level vectors of n = 3 W^2 + 1 doubles):
  // the GCR workspace of gp_solve / gp_adjoint_solve (allocated at the first solve, gcr_alloc)
  GcrWs kr{};
  // level-set reinitialisation (gp_reinit_levelset, allocated at its first call): two lattices of values, the
  // interface distance estimates and the point codes, (2N+1)^2 each
  double *rl_a = nullptr, *rl_b = nullptr, *rl_d = nullptr;
  int8_t *rl_c = nullptr;
  // the geometry of a later time built in the background (gp_prepare_levelset_analytic) in a second context
  Ctx *shadow = nullptr;
  std::thread prep;
  bool prep_active = false;
  gp_status prep_status = GP_OK;
  gp_shape prep_shape{};
  double prep_t = 0, prep_alpha = 0;
  gp_rigid prep_motion{};
  hipEvent_t prep_start = nullptr, prep_done = nullptr;
};

// error handling (the message under a lock: the geometry build runs one host thread per level)
#define GP_HIP(call)                                                      \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess) {                                               \
      std::lock_guard<std::mutex> lk_(ctx->err_mu);                       \
      ctx->hip_err = std::string(#call) + ": " + hipGetErrorString(e_);   \
      return GP_EHIP;                                                     \
    }                                                                     \
  } while (0)

inline int nblk(long n) { return (int)((n + TPB - 1) / TPB); }

// per-level constants of the box solve (the quotients by d, d + a and d^2 - a^2)
struct BoxK {
  double h, ih, a, q1, q2, bp, id, ihd;  // q1 = d / det, q2 = a / det, bp = (1/h) / (d + a), id = 1 / d, ihd = (1/h) / d
};
inline BoxK box_consts(double h, double a, double d) {
  BoxK K;
  const double det = d * d - a * a;
  K.h = h;
  K.ih = 1.0 / h;
  K.a = a;
  K.q1 = d / det;
  K.q2 = a / det;
  K.bp = K.ih / (d + a);
  K.id = 1.0 / d;
  K.ihd = K.ih / d;
  return K;
}

// geometry (geom.hip)
gp_status geometry_build(Ctx *ctx);
gp_status levelset_analytic(Ctx *ctx, const gp_shape *shape, double t, const gp_rigid *mo);
gp_status default_boundary_values(Ctx *ctx);
gp_status coarse_factor(Ctx *ctx);
gp_status coarse_factor(Ctx *ctx, BuildRes &B);
gp_status sector_build(Ctx *ctx, int l);
gp_status xb_factor(Ctx *ctx, int l, hipStream_t s);
gp_status ensure_xb(Ctx *ctx);
void adjoint_free_tabs(Ctx *ctx);  // the reverse mode's scatter tables and scratch
// acc[0..1] += t * sum over the finest body ghost rows of lam_G d(b_G - M_G x)/dP (P the body position at time t,
// discrete decisions of the geometry frozen); mism counts rows whose Alg. 1 path was not reproduced
gp_status path_terms(Ctx *ctx, const gp_shape &sh, const gp_rigid &mo, double t, const double *x, const double *lam,
                     double *cx, double *cy, double *acc, int *mism);

// multigrid (mg.hip)
gp_status mg_cycle64(Ctx *ctx, double *res_inf);
gp_status mg_solve(Ctx *ctx, int precision, double tol, int max_cycles, gp_stats *st);
gp_status relax64(Ctx *ctx, int level, int steps);
gp_status residual64(Ctx *ctx, int level, double *res_inf);
gp_status set_wall_dirichlet(Ctx *ctx);
gp_status time_kernel(Ctx *ctx, int which, int level, int reps, double *avg_us);
gp_status probe_start(Ctx *ctx, int max_launches, int every);
gp_status probe_stop(Ctx *ctx, double *avg_us, int *launches);

// GCR (mg.hip): M x = b to ||r||_inf <= thr.  precond(r, z): z = B' r (the cycle as an operator, 0 where no
// equation); apply_neg(z, q): q = -M z; residual(x, r): r = b - M x (true residual) and its max norm.  x and r
// are the caller's device vectors (n doubles); r must hold b - M x on entry.
struct GcrOps {
  std::function<void(const double *r, double *z)> precond;
  std::function<void(const double *z, double *q)> apply_neg;
  std::function<gp_status(double *rinf)> residual;
};
gp_status gcr_solve(Ctx *ctx, const GcrWs &ws, GcrOps &ops, double *x, double *r, double r0, double thr, double lim,
                    int max_it, int *iters, double *res, double *rho, int *status, double *kbytes);
double cycle_bytes(const Ctx *ctx, bool fp32);
gp_status gcr_alloc(Ctx *ctx);
// the static scratch array of gp_solve_noalloc: its device address on the current device, taken once per device
// (scratch_init, at context set-up), and the FP64 solve with the GCR workspace carved from it
gp_status scratch_init(Ctx *ctx);
gp_status mg_solve_noalloc(Ctx *ctx, double tol, int max_cycles, gp_stats *st);

// level-set reinitialisation (levelset.hip)
gp_status reinit_levelset(Ctx *ctx, double *phi, int on_device, int iters, double cfl);

// adjoint (adjoint.hip)
gp_status adjoint_alloc(Ctx *ctx);
gp_status adjoint_solve_dev(Ctx *ctx, double tol, int max_cycles, gp_stats *st);
void tape_free(Ctx *ctx);

// time stepping (cn.hip)
gp_status cn_set_state_finish(Ctx *ctx);
gp_status cn_step(Ctx *ctx, double dt, const double *fu, const double *fv, const double *g, int precision, double tol,
                  int max_cycles, double picard_eps, int picard_max, gp_stats *st);

}  // namespace gpmg

// the opaque public handle is the context itself
struct gp_ctx : public gpmg::Ctx {};
