// C ABI of the light-field super-resolution solver (include/lfsr.h): parameter
// validation, tiling plan, workspace layout and the per-iteration launch
// schedule of the ADMM loop (arXiv 2206.05047, sec 5, Algorithms 1 and 2).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lfsr_handle.h"

using namespace lfsr;

namespace {

thread_local std::string g_thread_err = "no error";

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

bool fail(std::string* err, const char* msg) {
  if (err) *err = msg;
  return false;
}

// Tiling for the forward and adjoint kernels; false if the warp halo is too
// large for any LDS tile.
bool choose_tiles(Geom& g, std::string* err) {
  // forward: the largest LR tile whose LDS and per-thread slots fit
  const int fcand[6][2] = {{16, 16}, {16, 8}, {8, 8}, {8, 4}, {4, 4}, {4, 2}};
  bool ok = false;
  for (auto& c : fcand) {
    g.f_tly = c[0];
    g.f_tlx = c[1];
    if (forward_tile_ok(g)) {
      ok = true;
      break;
    }
  }
  if (!ok) return fail(err, "disp_bound too large: the forward warp halo does not fit in LDS");
  const long long ftiles = (long long)((g.sy + g.f_tly - 1) / g.f_tly) * ((g.sx + g.f_tlx - 1) / g.f_tlx);
  // views per block: whole angular rows when that still gives >= ~2048 blocks
  // (the vertical warp coordinate is then computed once per row)
  long long vpb = (ftiles * g.sk + 3071) / 3072;
  if (vpb < 1) vpb = 1;
  if (vpb >= g.V) vpb = (vpb / g.V) * g.V;
  else if (ftiles * ((g.sk + g.V - 1) / g.V) >= 2048) vpb = g.V;
  if (vpb > g.sk) vpb = g.sk;
  g.f_vpb = (int)vpb;
  if (forward_col_setup(g)) {
    // NW waves per block (8 for quad cells, 4 for the plain tile), each a view
    // at a time.  Views are split into groups so that a launch is about 1.5
    // rounds of resident blocks (2 or 4 per CU on 256 CUs): long view loops
    // amortise the tile staging, and the partial second round keeps the tail
    // short.
    const long long nw = g.f_col == 2 ? 8 : 4, slots = g.f_col == 2 ? 512 : 1024;
    const long long ct = (long long)((g.sy + g.f_tly - 1) / g.f_tly) * ((g.sx + g.f_tlx - 1) / g.f_tlx);
    long long groups = (3 * slots / 2 + ct / 2) / ct;
    const long long gmax = (g.sk + nw - 1) / nw;
    if (groups < 1) groups = 1;
    if (groups > gmax) groups = gmax;
    const long long vpw = (g.sk + nw * groups - 1) / (nw * groups);
    g.f_vpb = (int)(nw * vpw);
  }
  forward_orbit_setup(g);

  // adjoint: prefer >= 1024 tiles; the HR tile must be at least the halo
  const int acand[7][2] = {{16, 8}, {8, 8}, {8, 4}, {4, 8}, {4, 4}, {4, 2}, {4, 1}};
  int best = -1;
  for (int ci = 0; ci < 7; ++ci) {
    Geom t = g;
    t.a_tly = acand[ci][0];
    t.a_tlx = acand[ci][1];
    t.a_th = t.a_tly * g.zeta;
    t.a_tw = t.a_tlx * g.zeta;
    t.a_ey = t.a_th + 2 * g.halo;
    t.a_ex = t.a_tw + 2 * g.halo;
    if (!adjoint_tile_ok(t)) continue;
    const long long nt = (long long)((g.sy + t.a_tly - 1) / t.a_tly) * ((g.sx + t.a_tlx - 1) / t.a_tlx);
    best = ci;
    if (nt >= 1024) break;
  }
  if (best < 0) return fail(err, "disp_bound too large for the adjoint tiling (halo exceeds tile or LDS)");
  g.a_tly = acand[best][0];
  g.a_tlx = acand[best][1];
  g.a_th = g.a_tly * g.zeta;
  g.a_tw = g.a_tlx * g.zeta;
  g.a_ey = g.a_th + 2 * g.halo;
  g.a_ex = g.a_tw + 2 * g.halo;
  g.a_nty = (g.sy + g.a_tly - 1) / g.a_tly;
  g.a_ntx = (g.sx + g.a_tlx - 1) / g.a_tlx;
  g.a_inv_th = (float)(1.0 / g.a_th);
  g.a_inv_tw = (float)(1.0 / g.a_tw);
  g.a_col = 0;
  g.a_vg = 1;
  g.a_vpb = g.sk;
  (void)adjoint_col_setup(g);
  long long rbk = (g.p + 4 * kThreads - 1) / (4 * kThreads);
  g.red_blocks = (int)(rbk < kRedBlocks ? (rbk < 1 ? 1 : rbk) : kRedBlocks);
  return true;
}

bool make_plan(const lfsr_params* p, Plan* pl, std::string* err) {
  if (!p) return fail(err, "params is NULL");
  std::memset(pl, 0, sizeof(*pl));
  Geom& g = pl->g;
  if (p->ang_rows < 1 || p->ang_cols < 1 || p->ang_rows > 63 || p->ang_cols > 63)
    return fail(err, "ang_rows/ang_cols must be in 1..63");
  if (p->lr_h < 1 || p->lr_w < 1) return fail(err, "lr_h/lr_w must be >= 1");
  if (p->scale < 1 || p->scale > 8) return fail(err, "scale must be in 1..8");
  if ((long long)p->lr_h * p->scale > 32768 || (long long)p->lr_w * p->scale > 32768)
    return fail(err, "HR size above 32768 per side");
  // one HR plane stays below 1 GiB of floats (32-bit byte offsets in the kernels)
  if ((long long)p->lr_h * p->scale * (long long)p->lr_w * p->scale > (1LL << 28))
    return fail(err, "HR image above 2^28 pixels");
  if (p->n_disp != 1 && p->n_disp != p->ang_rows * p->ang_cols)
    return fail(err, "n_disp must be 1 (one map on the reference view) or ang_rows*ang_cols (one map per view)");
  if (!(std::isfinite(p->lambda1) && std::isfinite(p->lambda2)) || p->lambda1 < 0.f || p->lambda2 < 0.f ||
      p->lambda1 + p->lambda2 <= 0.f)
    return fail(err, "lambda1, lambda2 must be finite, >= 0 and not both 0");
  if (p->nltv_window < 1 || p->nltv_window > kMaxWin || p->nltv_window % 2 == 0)
    return fail(err, "nltv_window must be odd in 1..15");
  if (!(p->sigma_s > 0.f) || !std::isfinite(p->sigma_s)) return fail(err, "sigma_s must be finite and > 0");
  if (!(p->sigma_e > 0.f)) return fail(err, "sigma_e must be > 0 (+INF disables the edge weight)");
  if (!(p->admm_penalty > 0.f) || !std::isfinite(p->admm_penalty)) return fail(err, "admm_penalty must be > 0");
  if (p->admm_iters < 1 || p->admm_iters > 1000000) return fail(err, "admm_iters must be in 1..1e6");
  if (p->cg_iters < 0 || p->cg_iters > 100000) return fail(err, "cg_iters must be in 0..1e5");
  if (!(p->cg_tol >= 0.f) || !std::isfinite(p->cg_tol)) return fail(err, "cg_tol must be finite and >= 0");
  if (!(p->stop_tol >= 0.f) || !std::isfinite(p->stop_tol)) return fail(err, "stop_tol must be finite and >= 0");
  if (!(p->disp_bound > 0.f) || !std::isfinite(p->disp_bound) || p->disp_bound > 256.f)
    return fail(err, "disp_bound must be in (0, 256]");
  if (p->reweight != 0 && p->reweight != 1) return fail(err, "reweight must be 0 or 1");
  if (p->storage != LFSR_F32 && p->storage != LFSR_F16 && p->storage != LFSR_BF16)
    return fail(err, "storage must be LFSR_F32, LFSR_F16 or LFSR_BF16");
  if (p->spatial_weight != 0 && p->spatial_weight != 1) return fail(err, "spatial_weight must be 0 or 1");
  if (p->spatial_weight == 1 && !(p->sigma_s <= 1.f)) return fail(err, "BTV spatial weight needs 0 < sigma_s <= 1");

  g.U = p->ang_rows;
  g.V = p->ang_cols;
  g.sk = g.U * g.V;
  g.kref = ((g.U - 1) / 2) * g.V + (g.V - 1) / 2;  // the view with angular offset (0, 0)
  g.sy = p->lr_h;
  g.sx = p->lr_w;
  g.zeta = p->scale;
  g.H = g.zeta * g.sy;
  g.W = g.zeta * g.sx;
  g.q = (long long)g.sy * g.sx;
  g.p = (long long)g.H * g.W;

  // blur (sec 4.1): normalised Gaussian; sigma <= 0 -> sqrt(zeta^2-1)/4
  double sigma = p->blur_sigma;
  int kb = p->blur_size;
  if (!(sigma > 0.0)) {
    sigma = std::sqrt((double)g.zeta * g.zeta - 1.0) / 4.0;
    if (kb <= 0) kb = sigma > 0.0 ? 2 * (int)std::ceil(3.0 * sigma) + 1 : 1;
  } else if (kb <= 0) {
    kb = 2 * (int)std::ceil(3.0 * sigma) + 1;
  }
  if (!std::isfinite(sigma)) return fail(err, "blur_sigma must be finite");
  if (kb < 1 || kb > kMaxTaps || kb % 2 == 0) return fail(err, "blur_size must be odd in 1..31");
  g.kb = kb;
  g.rb = kb / 2;
  g.blur2d = p->blur_taps ? 1 : 0;
  if (g.blur2d) {  // an explicit kernel (sec 7.1: motion blur), used as given
    if (p->blur_size < 1 || p->blur_size > kMax2DTaps || p->blur_size % 2 == 0)
      return fail(err, "an explicit blur kernel needs an odd blur_size in 1..15");
    g.kb = p->blur_size;
    g.rb = g.kb / 2;
    for (int i = 0; i < g.kb * g.kb; ++i) {
      if (!std::isfinite(p->blur_taps[i])) return fail(err, "blur_taps must be finite");
      pl->taps2d[i] = p->blur_taps[i];
    }
  }
  {
    double s = 0.0, t[kMaxTaps];
    for (int a = 0; a < kb; ++a) {
      const double d = a - g.rb;
      t[a] = sigma > 0.0 ? std::exp(-d * d / (2.0 * sigma * sigma)) : (d == 0.0 ? 1.0 : 0.0);
      s += t[a];
    }
    for (int a = 0; a < kb; ++a) g.g[a] = (float)(t[a] / s);
  }

  // NLTV (sec 3.4, 4.1): offsets row-major over the window, centre skipped
  g.win = p->nltv_window;
  g.rw = g.win / 2;
  g.sd = g.win * g.win - 1;
  {
    const int half = (g.win * g.win) / 2;
    for (int d = 0; d < g.sd; ++d) {
      const int id = d < half ? d : d + 1;
      const int dy = id / g.win - g.rw, dx = id % g.win - g.rw;
      const double c = p->spatial_weight == 1 ? std::pow((double)p->sigma_s, (double)(std::abs(dy) + std::abs(dx)))
                                              : std::exp(-(double)(dy * dy + dx * dx) / (double)p->sigma_s);
      g.cd[d] = (float)c;
      g.cd2[d] = (float)(c * c);
      g.ody[d] = (signed char)dy;
      g.odx[d] = (signed char)dx;
    }
  }
  g.lambda1 = p->lambda1;
  g.lambda2 = p->lambda2;
  g.half_theta = 0.5f * p->admm_penalty;
  g.clip = (float)(1.0 / (double)p->admm_penalty);
  g.cA = (float)((double)p->lambda2 + 0.5 * (double)p->admm_penalty * (double)p->lambda1 * p->lambda1);
  g.use_edge = std::isfinite(p->sigma_e) ? 1 : 0;
  g.reweight = p->reweight;
  g.n_iter = p->admm_iters;
  g.inv_sigma_e = g.use_edge ? (float)(1.0 / (double)p->sigma_e) : 0.f;
  g.disp_bound = p->disp_bound;
  g.n_disp = p->n_disp;
  g.cg_tol = p->cg_tol;
  g.stop_tol = p->stop_tol;
  {
    const int tmax = g.U / 2 > g.V / 2 ? g.U / 2 : g.V / 2;  // largest |angular offset| (odd or even grid)
    g.halo = (int)std::ceil((double)tmax * (double)p->disp_bound) + 1;
  }
  if (!choose_tiles(g, err)) return false;

  // workspace layout; es = bytes per element of the storage type
  const size_t P = (size_t)g.p, Q = (size_t)g.q;
  const size_t es = p->storage == LFSR_F32 ? 4 : 2;
  size_t o = 0;
  auto take = [&](size_t n) {
    size_t at = o;
    o = align256(o + n);
    return at;
  };
  pl->off_sc = take(sizeof(DevScalars));
  pl->off_x = take(P * es);
  pl->off_dx = take(es == 4 ? 0 : P * 4);
  pl->off_m = take(P * 4);
  pl->off_vs = take(P * 4);
  pl->off_r = take(P * 4);
  pl->off_pv = take(P * 4);
  pl->off_hp = take(P * 4);
  pl->off_wd = take((size_t)g.sk * Q * es);
  pl->off_ws0 = take((size_t)g.sd * P * es);
  pl->off_ws1 = take((size_t)g.sd * P * es);
  pl->off_lr = take((size_t)g.sk * Q * es);
  pl->off_adj = take((size_t)g.a_vg * g.a_nty * g.a_ntx * g.a_ey * g.a_ex * 4);
  {
    const dim3 fg = forward_grid(g), tg = tv_grid(g);
    pl->off_pwzd = take((size_t)fg.x * fg.y * fg.z * 3 * sizeof(double));
    pl->off_ptv = take((size_t)tg.x * tg.y * 2 * sizeof(double));
    pl->off_prr0 = take((size_t)kRedBlocks * sizeof(double));
    pl->off_prr1 = take((size_t)kRedBlocks * sizeof(double));
    pl->off_pphp = take((size_t)tg.x * tg.y * sizeof(double));
    pl->off_pmax = take(std::max((size_t)fg.x * fg.y * fg.z, (size_t)kRedBlocks) * sizeof(float));
    const dim3 ag = adjoint_grid(g);
    pl->off_pcnt = take((size_t)ag.x * ag.y * ag.z * sizeof(int));
  }
  pl->off_stats = take((size_t)p->admm_iters * LFSR_NSTAT * sizeof(double));
  pl->off_taps = take(g.blur2d ? (size_t)g.kb * g.kb * sizeof(float) : 0);
  pl->bytes = o;
  return true;
}

}  // namespace

namespace {

lfsr_status set_err(lfsr_handle* h, lfsr_status st, const std::string& msg) {
  if (h) h->err = msg;
  else g_thread_err = msg;
  return st;
}

// Check for launch errors after enqueueing work.
lfsr_status check_hip(lfsr_handle* h, const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    h->broken = true;
    return set_err(h, LFSR_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
  }
  return LFSR_OK;
}

lfsr_status usable(lfsr_handle* h) {
  if (!h) return set_err(nullptr, LFSR_EINVAL, "handle is NULL");
  if (h->broken) return set_err(h, LFSR_ESTATE, "handle unusable after an earlier device error: " + h->err);
  return LFSR_OK;
}

hipStream_t S(void* s) { return (hipStream_t)s; }

// Bracket a launch with profiling events when its kind is being timed.
template <class F>
void timed(lfsr_handle* h, int kind, hipStream_t s, F&& launch) {
  Profile& pr = h->prof;
  const bool t = pr.on && (pr.mask >> kind & 1u) && (size_t)(2 * pr.used + 1) < pr.ev.size();
  if (t) (void)hipEventRecord(pr.ev[2 * pr.used], s);
  launch();
  if (t) {
    (void)hipEventRecord(pr.ev[2 * pr.used + 1], s);
    pr.kind[pr.used] = kind;
    ++pr.used;
  }
}

// One ADMM iteration (Algorithm 1 with the CG x-step of Algorithm 2).
void enqueue_iteration(lfsr_handle* h, hipStream_t s) {
  const Geom& g = h->plan.g;
  const Bufs& b = h->b;
  // weights from x^(n-1) (sec 7.1: recomputed every iteration when reweighting)
  timed(h, LFSR_K_OTHER, s, [&] { launch_edge(g, b.x, b.st, h->occ, b.m, s, b, kGateAdmm | kGateReweight); });
  // z/w-steps of both blocks; e and the NLTV divergence feed v
  timed(h, LFSR_K_FORWARD, s, [&] { launch_forward_wzd(g, h->disp, h->y, s, b); });
  if (g.sd > 0) timed(h, LFSR_K_NLTV, s, [&] { launch_tv(g, s, b); });
  timed(h, LFSR_K_ADJOINT, s, [&] { launch_adjoint(g, b.lr, b.st, h->disp, s, b, kGateAdmm, forward_blocks(g)); });
  // the CG start and the normal assembly gather the adjoint's partial images themselves when they can
  const int fuse = merge_fusable(g) ? 1 : 0;
  if (!fuse) timed(h, LFSR_K_OTHER, s, [&] { launch_merge(g, b.r, s, b, kGateAdmm); });
  timed(h, LFSR_K_CG, s, [&] { launch_cginit(g, s, b, fuse); });
  // x-step: K CG steps on G^T G delta = -v, accumulated straight into the FP32 estimate
  for (int k = 1; k <= h->prm.cg_iters; ++k) {
    timed(h, LFSR_K_FORWARD, s, [&] { launch_forward_cg(g, b.pv, h->disp, s, b, kGateAdmm | kGateCg); });
    timed(h, LFSR_K_ADJOINT, s,
          [&] { launch_adjoint(g, b.lr, b.st, h->disp, s, b, kGateAdmm | kGateCg, forward_blocks(g)); });
    if (!fuse) timed(h, LFSR_K_OTHER, s, [&] { launch_merge(g, b.hp, s, b, kGateAdmm | kGateCg); });
    timed(h, LFSR_K_NORMAL, s, [&] { launch_hp(g, b.pv, b.m, b.hp, s, b, kGateAdmm | kGateCg, 1, fuse); });
    timed(h, LFSR_K_CG, s, [&] { launch_cgupd(g, k, s, b); });
    // the direction after the last step is never read (the next x-step starts from p = r)
    if (k < h->prm.cg_iters) timed(h, LFSR_K_CG, s, [&] { launch_cgp(g, k, s, b); });
  }
  if (b.st != kStF32) timed(h, LFSR_K_CG, s, [&] { launch_fold(g, s, b); });
  timed(h, LFSR_K_OTHER, s, [&] { launch_iter_end(g, s, b); });
  h->n_done += 1;
}

// Workspace of lfsr_solve_noalloc: one array per GPU, resident for the life
// of the process.  Host code never uses this name as an address (on the host
// it only identifies the symbol); the device address of each GPU's copy is
// looked up once per device and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[LFSR_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the
// first call on that device); nullptr and *err set on failure.
void* scratch_ptr(std::string* err) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    *err = "device index beyond the scratch table";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

// The adjoint's fixed-point scale uses per-block contribution counts of the
// disparity map bound by lfsr_init.  An operator call with another map
// recounts for its own map; put the bound map's counts back afterwards.
void restore_counts(lfsr_handle* h, const float* d_disp, hipStream_t s) {
  if (h->disp && h->disp != d_disp) launch_adjcount(h->plan.g, h->disp, s, h->b);
}

// An explicit blur kernel lives in the workspace; every entry point that
// applies B enqueues its (tiny) upload first, so that it does not depend on
// which call came before.
void upload_taps(lfsr_handle* h, hipStream_t s) {
  if (h->plan.g.blur2d) launch_set_taps(h->plan.g, h->plan.taps2d, s);
}

// Carve a workspace into the buffers of a handle (the layout of make_plan).
void bind_workspace(lfsr_handle* h, const lfsr_params* p, const Plan& pl, char* w) {
  h->prm = *p;
  h->plan = pl;
  h->ws = w;
  h->b.sc = (DevScalars*)(w + pl.off_sc);
  h->b.st = p->storage;
  h->b.x = w + pl.off_x;
  h->b.dx = p->storage == LFSR_F32 ? nullptr : (float*)(w + pl.off_dx);
  h->b.m = (float*)(w + pl.off_m);
  h->b.vs = (float*)(w + pl.off_vs);
  h->b.r = (float*)(w + pl.off_r);
  h->b.pv = (float*)(w + pl.off_pv);
  h->b.hp = (float*)(w + pl.off_hp);
  h->b.wD = w + pl.off_wd;
  h->b.wS[0] = w + pl.off_ws0;
  h->b.wS[1] = w + pl.off_ws1;
  h->b.lr = w + pl.off_lr;
  h->b.adj = (float*)(w + pl.off_adj);
  h->b.p_wzd = (double*)(w + pl.off_pwzd);
  h->b.p_tv = (double*)(w + pl.off_ptv);
  h->b.p_rr[0] = (double*)(w + pl.off_prr0);
  h->b.p_rr[1] = (double*)(w + pl.off_prr1);
  h->b.p_php = (double*)(w + pl.off_pphp);
  h->b.p_max = (float*)(w + pl.off_pmax);
  h->b.p_cnt = (int*)(w + pl.off_pcnt);
  h->b.stats = (double*)(w + pl.off_stats);
  h->plan.g.taps2d = pl.g.blur2d ? (const float*)(w + pl.off_taps) : nullptr;
  h->n_done = 0;
  h->bound = false;
  h->broken = false;
  h->y = h->disp = h->occ = nullptr;
  h->err = "no error";
}

}  // namespace

extern "C" {

size_t lfsr_workspace_bytes(const lfsr_params* p) {
  Plan pl;
  std::string err;
  if (!make_plan(p, &pl, &err)) {
    g_thread_err = err;
    return 0;
  }
  return pl.bytes;
}

lfsr_status lfsr_create(const lfsr_params* p, void* d_workspace, size_t bytes, lfsr_handle** out) {
  if (!out) return set_err(nullptr, LFSR_EINVAL, "out is NULL");
  *out = nullptr;
  Plan pl;
  std::string err;
  if (!make_plan(p, &pl, &err)) return set_err(nullptr, LFSR_EINVAL, err);
  if (!d_workspace) return set_err(nullptr, LFSR_ENOMEM, "workspace is NULL");
  if (((uintptr_t)d_workspace & 255) != 0) return set_err(nullptr, LFSR_EINVAL, "workspace not 256-byte aligned");
  if (bytes < pl.bytes)
    return set_err(nullptr, LFSR_ENOMEM,
                   "workspace too small: need " + std::to_string(pl.bytes) + " bytes, got " + std::to_string(bytes));
  lfsr_handle* h = new (std::nothrow) lfsr_handle();
  if (!h) return set_err(nullptr, LFSR_ENOMEM, "host allocation of the handle failed");
  bind_workspace(h, p, pl, (char*)d_workspace);
  *out = h;
  return LFSR_OK;
}

void lfsr_destroy(lfsr_handle* h) {
  if (!h) return;
  for (hipEvent_t e : h->prof.ev) (void)hipEventDestroy(e);
  delete h;
}

const char* lfsr_last_error(const lfsr_handle* h) { return h ? h->err.c_str() : g_thread_err.c_str(); }

lfsr_status lfsr_init(lfsr_handle* h, const float* d_lr, const float* d_disp, const float* d_occ,
                      const float* d_x0, void* hip_stream) {
  lfsr_status st = usable(h);
  if (st) return st;
  if (!d_lr || !d_disp) return set_err(h, LFSR_EINVAL, "d_lr and d_disp are required");
  const Geom& g = h->plan.g;
  hipStream_t s = S(hip_stream);
  h->y = d_lr;
  h->disp = d_disp;
  h->occ = d_occ;
  upload_taps(h, s);
  launch_reset(0, s, h->b);
  launch_check(g, d_lr, d_disp, d_occ, s, h->b);
  launch_adjcount(g, d_disp, s, h->b);
  launch_zero(h->b.wD, h->b.st, (long long)g.sk * g.q, s);
  launch_zero(h->b.wS[0], h->b.st, (long long)g.sd * g.p, s);
  launch_fill(h->b.m, g.p, 1.f, s);
  // x0 in FP32 (into x, or into the remainder buffer and then split)
  float* x32 = h->b.st == kStF32 ? (float*)h->b.x : h->b.dx;
  if (d_x0) {
    if (hipMemcpyAsync(x32, d_x0, (size_t)g.p * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return check_hip(h, "lfsr_init copy x0");
  } else {
    launch_bicubic(g, d_lr + (size_t)g.kref * g.q, x32, s);
  }
  if (h->b.st != kStF32) launch_split(g, x32, s, h->b);
  h->n_done = 0;
  h->bound = true;
  return check_hip(h, "lfsr_init");
}

lfsr_status lfsr_iterate(lfsr_handle* h, int32_t count, void* hip_stream) {
  lfsr_status st = usable(h);
  if (st) return st;
  if (!h->bound) return set_err(h, LFSR_ESTATE, "lfsr_iterate before lfsr_init / lfsr_write_state");
  if (count < 0) return set_err(h, LFSR_EINVAL, "count must be >= 0");
  hipStream_t s = S(hip_stream);
  for (int i = 0; i < count; ++i) enqueue_iteration(h, s);
  return check_hip(h, "lfsr_iterate");
}

lfsr_status lfsr_read_state(lfsr_handle* h, float* d_x, float* d_wd, float* d_ws, float* d_m, void* hip_stream) {
  lfsr_status st = usable(h);
  if (st) return st;
  const Geom& g = h->plan.g;
  hipStream_t s = S(hip_stream);
  if (h->b.st == kStF32) {
    if (d_x && hipMemcpyAsync(d_x, h->b.x, (size_t)g.p * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return check_hip(h, "lfsr_read_state x");
    if (d_wd && hipMemcpyAsync(d_wd, h->b.wD, (size_t)g.sk * g.q * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return check_hip(h, "lfsr_read_state w_D");
  } else {
    if (d_x) launch_join(g, d_x, s, h->b);
    if (d_wd) launch_to_float(h->b.wD, h->b.st, d_wd, (long long)g.sk * g.q, s);
  }
  if (d_ws) launch_copy_ws(d_ws, (long long)g.sd * g.p, s, h->b);
  if (d_m && hipMemcpyAsync(d_m, h->b.m, (size_t)g.p * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return check_hip(h, "lfsr_read_state m");
  return check_hip(h, "lfsr_read_state");
}

lfsr_status lfsr_write_state(lfsr_handle* h, const float* d_x, const float* d_wd, const float* d_ws,
                             const float* d_m, int32_t n_done, void* hip_stream) {
  lfsr_status st = usable(h);
  if (st) return st;
  const Geom& g = h->plan.g;
  if (!d_x || !d_wd || (g.sd > 0 && !d_ws)) return set_err(h, LFSR_EINVAL, "d_x, d_wd and d_ws are required");
  if (!h->prm.reweight && n_done > 0 && !d_m) return set_err(h, LFSR_EINVAL, "d_m required when reweight = 0");
  if (n_done < 0) return set_err(h, LFSR_EINVAL, "n_done must be >= 0");
  if (!h->y) return set_err(h, LFSR_ESTATE, "lfsr_write_state needs inputs bound by lfsr_init first");
  hipStream_t s = S(hip_stream);
  upload_taps(h, s);
  launch_reset(n_done, s, h->b);
  if (h->b.st == kStF32) {
    if (hipMemcpyAsync(h->b.x, d_x, (size_t)g.p * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->b.wD, d_wd, (size_t)g.sk * g.q * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        (g.sd > 0 &&
         hipMemcpyAsync(h->b.wS[0], d_ws, (size_t)g.sd * g.p * 4, hipMemcpyDeviceToDevice, s) != hipSuccess))
      return check_hip(h, "lfsr_write_state copy");
  } else {  // x splits exactly; the duals round to the storage type
    launch_split(g, d_x, s, h->b);
    launch_from_float(d_wd, h->b.wD, h->b.st, (long long)g.sk * g.q, s);
    if (g.sd > 0) launch_from_float(d_ws, h->b.wS[0], h->b.st, (long long)g.sd * g.p, s);
  }
  if (d_m && hipMemcpyAsync(h->b.m, d_m, (size_t)g.p * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return check_hip(h, "lfsr_write_state copy m");
  h->n_done = n_done;
  h->bound = true;
  return check_hip(h, "lfsr_write_state");
}

lfsr_status lfsr_get_stats(lfsr_handle* h, lfsr_stats* out, void* hip_stream) {
  lfsr_status st = usable(h);
  if (st) return st;
  if (!out) return set_err(h, LFSR_EINVAL, "out is NULL");
  hipStream_t s = S(hip_stream);
  DevScalars sc;
  if (hipMemcpyAsync(&sc, h->b.sc, sizeof(sc), hipMemcpyDeviceToHost, s) != hipSuccess)
    return check_hip(h, "lfsr_get_stats copy");
  const int nrow = std::min(h->prm.admm_iters, std::max(h->n_done, 0));
  if (out->h_hist && nrow > 0 &&
      hipMemcpyAsync(out->h_hist, h->b.stats, (size_t)nrow * LFSR_NSTAT * sizeof(double), hipMemcpyDeviceToHost,
                     s) != hipSuccess)
    return check_hip(h, "lfsr_get_stats copy hist");
  if (hipStreamSynchronize(s) != hipSuccess) return check_hip(h, "lfsr_get_stats sync");
  out->iters_run = sc.iters_done;
  out->cg_steps = sc.cg_steps;
  out->cg_pi = sc.pi;
  out->objective = 0.0;
  out->primal_res = 0.0;
  const int last = std::min(sc.iters_done, h->prm.admm_iters) - 1;
  if (last >= 0) {
    double row[LFSR_NSTAT];
    if (hipMemcpy(row, h->b.stats + (size_t)last * LFSR_NSTAT, sizeof(row), hipMemcpyDeviceToHost) != hipSuccess)
      return check_hip(h, "lfsr_get_stats row");
    out->objective = row[0];
    out->primal_res = row[1];
  }
  if (sc.err_flags & 1) return set_err(h, LFSR_ENONFINITE, "non-finite value in the LR views, disparity or occlusion map");
  if (sc.err_flags & 2) return set_err(h, LFSR_EINVAL, "|disparity| exceeds disp_bound");
  return check_hip(h, "lfsr_get_stats");
}

lfsr_status lfsr_solve(lfsr_handle* h, const float* d_lr, const float* d_disp, const float* d_occ,
                       const float* d_x0, float* d_hr_out, lfsr_stats* h_stats, void* hip_stream) {
  lfsr_status st = usable(h);
  if (st) return st;
  if (!d_hr_out) return set_err(h, LFSR_EINVAL, "d_hr_out is NULL");
  st = lfsr_init(h, d_lr, d_disp, d_occ, d_x0, hip_stream);
  if (st) return st;
  st = lfsr_iterate(h, h->prm.admm_iters, hip_stream);
  if (st) return st;
  if (h->b.st != kStF32)
    launch_join(h->plan.g, d_hr_out, S(hip_stream), h->b);
  else if (hipMemcpyAsync(d_hr_out, h->b.x, (size_t)h->plan.g.p * 4, hipMemcpyDeviceToDevice, S(hip_stream)) !=
           hipSuccess)
    return check_hip(h, "lfsr_solve copy out");
  if (h_stats) return lfsr_get_stats(h, h_stats, hip_stream);
  return check_hip(h, "lfsr_solve");
}

lfsr_status lfsr_forward(lfsr_handle* h, const float* d_x, const float* d_disp, float* d_lr_out, void* hip_stream) {
  lfsr_status st = usable(h);
  if (st) return st;
  if (!d_x || !d_disp || !d_lr_out) return set_err(h, LFSR_EINVAL, "NULL pointer");
  upload_taps(h, S(hip_stream));
  launch_forward(h->plan.g, d_x, d_disp, d_lr_out, S(hip_stream), h->b, 0);
  return check_hip(h, "lfsr_forward");
}

lfsr_status lfsr_adjoint(lfsr_handle* h, const float* d_lr, const float* d_disp, float* d_hr_out, void* hip_stream) {
  lfsr_status st = usable(h);
  if (st) return st;
  if (!d_lr || !d_disp || !d_hr_out) return set_err(h, LFSR_EINVAL, "NULL pointer");
  const Geom& g = h->plan.g;
  upload_taps(h, S(hip_stream));
  const int npmax = launch_absmax(g, d_lr, (long long)g.sk * g.q, S(hip_stream), h->b);
  launch_adjcount(g, d_disp, S(hip_stream), h->b);
  launch_adjoint(g, d_lr, kStF32, d_disp, S(hip_stream), h->b, 0, npmax);
  launch_merge(g, d_hr_out, S(hip_stream), h->b, 0);
  restore_counts(h, d_disp, S(hip_stream));
  return check_hip(h, "lfsr_adjoint");
}

lfsr_status lfsr_normal(lfsr_handle* h, const float* d_p, const float* d_disp, const float* d_m, float* d_out,
                        void* hip_stream) {
  lfsr_status st = usable(h);
  if (st) return st;
  if (!d_p || !d_disp || !d_m || !d_out) return set_err(h, LFSR_EINVAL, "NULL pointer");
  if (d_out == d_p || d_out == d_m) return set_err(h, LFSR_EINVAL, "d_out must not alias d_p or d_m");
  const Geom& g = h->plan.g;
  hipStream_t s = S(hip_stream);
  upload_taps(h, s);
  launch_forward_cg(g, d_p, d_disp, s, h->b, 0);
  launch_adjcount(g, d_disp, s, h->b);
  launch_adjoint(g, h->b.lr, h->b.st, d_disp, s, h->b, 0, forward_blocks(g));
  const int fuse = merge_fusable(g) ? 1 : 0;
  if (!fuse) launch_merge(g, d_out, s, h->b, 0);
  launch_hp(g, d_p, d_m, d_out, s, h->b, 0, 0, fuse);
  restore_counts(h, d_disp, s);
  return check_hip(h, "lfsr_normal");
}

lfsr_status lfsr_edge_weight(lfsr_handle* h, const float* d_x, const float* d_occ, float* d_m_out, void* hip_stream) {
  lfsr_status st = usable(h);
  if (st) return st;
  if (!d_x || !d_m_out) return set_err(h, LFSR_EINVAL, "NULL pointer");
  launch_edge(h->plan.g, d_x, kStF32, d_occ, d_m_out, S(hip_stream), h->b, 0);
  return check_hip(h, "lfsr_edge_weight");
}

lfsr_status lfsr_occlusion_weight(lfsr_handle* h, const float* d_lr, const float* d_disp, float sigma_o1,
                                  float sigma_o2, float* d_occ_out, void* hip_stream) {
  lfsr_status st = usable(h);
  if (st) return st;
  if (!d_lr || !d_disp || !d_occ_out) return set_err(h, LFSR_EINVAL, "NULL pointer");
  if (!(sigma_o1 > 0.f) || !(sigma_o2 > 0.f))
    return set_err(h, LFSR_EINVAL, "sigma_o1 and sigma_o2 must be > 0 (+INF switches a factor off)");
  const Geom& g = h->plan.g;
  hipStream_t s = S(hip_stream);
  // the CG vectors are free outside an iteration: the up-sampled reference
  // view, the up-sampled view k and the running sum of squared errors
  float *lref = h->b.r, *lk = h->b.pv, *acc = h->b.hp;
  const float* dref = d_disp + (g.n_disp > 1 ? (size_t)g.kref * g.p : 0);  // the reference view's map
  launch_bicubic(g, d_lr + (size_t)g.kref * g.q, lref, s);
  launch_fill(acc, g.p, 0.f, s);
  for (int k = 0; k < g.sk; ++k) {
    if (k == g.kref) continue;
    launch_bicubic(g, d_lr + (size_t)k * g.q, lk, s);
    launch_occ_acc(g, lref, lk, dref, k, acc, s);
  }
  const float c1 = std::isinf(sigma_o1) ? 0.f : (float)(0.5 / ((double)sigma_o1 * sigma_o1));
  const float c2 = std::isinf(sigma_o2) ? 0.f : (float)(0.5 / ((double)sigma_o2 * sigma_o2));
  launch_occ_final(g, dref, acc, g.sk > 1 ? (float)(1.0 / (g.sk - 1)) : 0.f, c1, c2, d_occ_out, s);
  return check_hip(h, "lfsr_occlusion_weight");
}

lfsr_status lfsr_gd(lfsr_handle* h, int32_t iters, float step, int32_t line_search, double* h_hist,
                    void* hip_stream) {
  lfsr_status st = usable(h);
  if (st) return st;
  if (!h->bound) return set_err(h, LFSR_ESTATE, "lfsr_gd before lfsr_init");
  if (h->b.st != kStF32) return set_err(h, LFSR_EINVAL, "lfsr_gd needs FP32 storage");
  if (iters < 0 || !(step > 0.f) || !std::isfinite(step) || (line_search != 0 && line_search != 1))
    return set_err(h, LFSR_EINVAL, "lfsr_gd: iters >= 0, step > 0 and line_search 0 or 1 required");
  const Geom& g = h->plan.g;
  const Bufs& b = h->b;
  hipStream_t s = S(hip_stream);
  float* x = (float*)b.x;
  float* xc = b.vs;  // trial point of the line search
  double dev[2];
  auto read = [&](double* out) -> bool {  // (J, |g|^2) of the last evaluations
    if (hipMemcpyAsync(dev, &b.sc->gd_cost, 2 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return false;
    out[0] = dev[0];
    out[1] = dev[1];
    return true;
  };
  // weights fixed at the starting point (the cost every solver minimises here)
  launch_edge(g, x, kStF32, h->occ, b.m, s, b, 0);
  launch_gd_cost(g, x, h->disp, h->y, s, b);  // one CU: A and S
  launch_gd_grad(g, h->disp, s, b);           // one CU: A^T and S^T
  double cur[2];
  if (!read(cur)) return check_hip(h, "lfsr_gd read");
  double cu = 2.0, eta = step;
  if (h_hist) {
    h_hist[0] = cur[0];
    h_hist[1] = cu;
    h_hist[2] = 0.0;
  }
  for (int it = 1; it <= iters; ++it) {
    if (!line_search) {
      launch_gd_step(g, x, step, x, s, b);
      launch_gd_cost(g, x, h->disp, h->y, s, b);
      launch_gd_grad(g, h->disp, s, b);
      cu += 2.0;
      if (!read(cur)) return check_hip(h, "lfsr_gd read");
    } else {
      // backtracking by halves from twice the last accepted step; Armijo
      // sufficient decrease J(x - eta g) <= J(x) - 1e-4 eta |g|^2
      eta = it == 1 ? (double)step : 2.0 * eta;
      for (int trial = 0; trial < 30; ++trial) {
        launch_gd_step(g, x, (float)eta, xc, s, b);
        launch_gd_cost(g, xc, h->disp, h->y, s, b);
        cu += 1.0;
        double trial_val[2];
        if (!read(trial_val)) return check_hip(h, "lfsr_gd read");
        if (trial_val[0] <= cur[0] - 1e-4 * eta * cur[1]) {
          if (hipMemcpyAsync(x, xc, (size_t)g.p * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return check_hip(h, "lfsr_gd accept");
          launch_gd_grad(g, h->disp, s, b);
          cu += 1.0;
          if (!read(cur)) return check_hip(h, "lfsr_gd read");
          break;
        }
        eta *= 0.5;
      }
    }
    if (h_hist) {
      h_hist[3 * it + 0] = cur[0];
      h_hist[3 * it + 1] = cu;
      h_hist[3 * it + 2] = line_search ? eta : (double)step;
    }
  }
  return check_hip(h, "lfsr_gd");
}

lfsr_status lfsr_bicubic(lfsr_handle* h, const float* d_lr_view, float* d_hr_out, void* hip_stream) {
  lfsr_status st = usable(h);
  if (st) return st;
  if (!d_lr_view || !d_hr_out) return set_err(h, LFSR_EINVAL, "NULL pointer");
  launch_bicubic(h->plan.g, d_lr_view, d_hr_out, S(hip_stream));
  return check_hip(h, "lfsr_bicubic");
}

lfsr_status lfsr_profile_begin(lfsr_handle* h, uint32_t kind_mask, int32_t capacity) {
  lfsr_status st = usable(h);
  if (st) return st;
  if (h->prof.on) return set_err(h, LFSR_ESTATE, "a profile is already open");
  if (capacity < 1 || capacity > (1 << 20)) return set_err(h, LFSR_EINVAL, "capacity must be in 1..2^20");
  Profile& pr = h->prof;
  pr.ev.assign(2 * (size_t)capacity, nullptr);
  pr.kind.assign((size_t)capacity, 0);
  for (auto& e : pr.ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& f : pr.ev)
        if (f) (void)hipEventDestroy(f);
      pr.ev.clear();
      return check_hip(h, "lfsr_profile_begin event create");
    }
  }
  pr.mask = kind_mask;
  pr.used = 0;
  pr.on = true;
  return LFSR_OK;
}

lfsr_status lfsr_profile_end(lfsr_handle* h, double* h_total_ms, int32_t* h_launches) {
  lfsr_status st = usable(h);
  if (st) return st;
  Profile& pr = h->prof;
  if (!pr.on) return set_err(h, LFSR_ESTATE, "no profile is open");
  double tot[LFSR_K_COUNT] = {0};
  int cnt[LFSR_K_COUNT] = {0};
  lfsr_status res = LFSR_OK;
  if (pr.used > 0 && hipEventSynchronize(pr.ev[2 * pr.used - 1]) != hipSuccess) res = check_hip(h, "profile sync");
  for (int i = 0; i < pr.used && res == LFSR_OK; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pr.ev[2 * i], pr.ev[2 * i + 1]) != hipSuccess) {
      res = check_hip(h, "profile elapsed");
      break;
    }
    tot[pr.kind[i]] += ms;
    cnt[pr.kind[i]] += 1;
  }
  for (hipEvent_t e : pr.ev) (void)hipEventDestroy(e);
  pr.ev.clear();
  pr.kind.clear();
  pr.on = false;
  pr.used = 0;
  for (int k = 0; k < LFSR_K_COUNT; ++k) {
    if (h_total_ms) h_total_ms[k] = tot[k];
    if (h_launches) h_launches[k] = cnt[k];
  }
  return res;
}

lfsr_status lfsr_solve_noalloc(const lfsr_params* p, const float* d_lr, const float* d_disp, const float* d_occ,
                               const float* d_x0, float* d_hr_out, lfsr_stats* h_stats, void* hip_stream) {
  Plan pl;
  std::string err;
  if (!make_plan(p, &pl, &err)) return set_err(nullptr, LFSR_EINVAL, err);
  if (pl.bytes > LFSR_NOALLOC_MAX_BYTES)
    return set_err(nullptr, LFSR_ENOMEM,
                   "lfsr_solve_noalloc: the problem needs " + std::to_string(pl.bytes) +
                       " bytes of workspace, above the static scratch of " + std::to_string(LFSR_NOALLOC_MAX_BYTES) +
                       " bytes (use lfsr_create + lfsr_solve with a caller workspace)");
  char* ws = (char*)scratch_ptr(&err);
  if (!ws) return set_err(nullptr, LFSR_EDEVICE, "lfsr_solve_noalloc: " + err);
  // a handle for this call only: every kernel gets the scratch pointers by value
  lfsr_handle h{};
  bind_workspace(&h, p, pl, ws);
  const lfsr_status st = lfsr_solve(&h, d_lr, d_disp, d_occ, d_x0, d_hr_out, h_stats, hip_stream);
  if (st) set_err(nullptr, st, "lfsr_solve_noalloc: " + h.err);
  return st;
}

}  // extern "C"
