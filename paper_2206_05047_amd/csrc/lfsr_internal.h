// Internal types shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lfsr {

constexpr int kMaxTaps = 31;      // blur size limit
constexpr int kMax2DTaps = 15;    // size limit of an explicit (non-separable) blur kernel
constexpr int kMaxWin = 15;       // NLTV window limit
constexpr int kMaxOffsets = kMaxWin * kMaxWin - 1;
constexpr int kThreads = 256;     // kernels run 256-thread (4 x wave64) blocks, except the NLTV step:

// forward operator: blur positions, horizontal-pass outputs per thread
constexpr int kFwdSlots = 12;     // NY*NX <= 256*kFwdSlots
constexpr int kFwdHSlots = 5;     // NY*tlx <= 256*kFwdHSlots
// adjoint (per wave: a quarter of the tile's HR rows): HR pixels,
// vertical-pass outputs and staged LR values per lane
constexpr int kAdjSlots = 5;      // (TH/4)*TW <= 64*kAdjSlots
constexpr int kAdjVSlots = 4;     // (TH/4)*LX <= 64*kAdjVSlots
constexpr int kAdjESlots = 3;     // RL*LX <= 64*kAdjESlots

constexpr int kTvThreads = 512;   // eight waves on one NLTV tile
constexpr int kCgThreads = 512;   // CG element-wise kernels (2 rows per thread)
constexpr int kTvTileX = 64, kTvTileY = 16;  // NLTV / normal-operator tiles (4 rows per thread in the latter)
// LDS row pitch (floats) of the column-per-lane kernels' source tile and
// accumulator: tile width + 2 halo must fit (halo <= 32)
constexpr int kColPitch = 128;
constexpr int kRedBlocks = 512;   // max grid of the element-wise CG kernels (= partials per reduction)

// Problem geometry and model constants, passed by value to every kernel.
struct Geom {
  int U, V, sk, kref;         // angular grid, views, reference view (angular offset (0, 0))
  int sy, sx, zeta, H, W;     // LR size, scale, HR size
  long long q, p;             // LR and HR pixel counts
  int kb, rb;                 // blur size and radius
  float g[kMaxTaps];          // normalised 1-D Gaussian taps (2-D kernel = g x g)
  int blur2d;                 // 1: explicit kb x kb correlation kernel at taps2d (tiled kernels only)
  const float* taps2d;        // its device copy in the workspace (set when the workspace is bound)
  int win, rw, sd;            // NLTV window, radius, number of offsets
  float cd[kMaxOffsets];      // spatial weight exp(-|d|^2/sigma_s) of offset d
  float cd2[kMaxOffsets];     // its square
  signed char ody[kMaxOffsets], odx[kMaxOffsets];  // offset d = (dy, dx)
  float lambda1, lambda2;
  float half_theta;           // vartheta / 2
  float clip;                 // 1 / vartheta
  float cA;                   // lambda2 + vartheta lambda1^2 / 2
  float inv_sigma_e;          // 1/sigma_e (0 when the edge weight is off)
  int use_edge;
  int reweight;
  int n_disp;                 // 1: one disparity map for every view; sk: view k's own map ([k][H][W])
  int halo;                   // warp halo in HR px: ceil(max |theta| * disp_bound) + 1
  float disp_bound;
  float cg_tol;
  float stop_tol;
  int n_iter;                 // rows of the statistics history
  // forward-operator tiling: LR tile and views per block.  f_col selects the
  // column-per-lane kernel: 1 = plain tile, 4 waves; 2 = quad-cell tile, 8
  // waves (f_vpb = waves x views per wave).  f_orb = 1: the CG-form quad
  // kernel walks mirror orbits of views instead of single views (same grid)
  int f_tly, f_tlx, f_vpb;
  int f_col;
  int f_orb;
  // adjoint tiling: LR tile, HR tile, extended (haloed) tile, tile grid
  int a_tly, a_tlx, a_th, a_tw, a_ey, a_ex, a_nty, a_ntx;
  // a_col = 1: column-per-lane adjoint; views split into a_vg groups of a_vpb,
  // each group writing its own set of partial images
  int a_col, a_vg, a_vpb;
  float a_inv_th, a_inv_tw;   // 1/a_th, 1/a_tw (division-free tile lookup)
  int red_blocks;             // grid of the element-wise CG kernels
};

// Device-resident scalars of one handle (lives in the workspace).  Written by
// block 0 of a kernel and read by later kernels only (no intra-kernel
// cross-block communication, so no device-scope fences are needed).
struct DevScalars {
  double pi;        // final CG |r|^2 of the current x-step
  double res1;      // primal residual of the first iteration (stop test)
  int res1_set;
  int wcur;         // which NLTV dual buffer holds the current w_S
  int cg_done;      // CG of the current x-step has stopped
  int cg_steps;     // CG steps taken in the current x-step
  int admm_done;    // stop test met: later iterations are no-ops
  int stop_pending;
  int iters_done;
  int err_flags;    // bit 0: non-finite input, bit 1: |disp| > disp_bound
  double gd_cost;   // gradient-descent baselines: J at the last evaluated point
  double gd_gnorm;  // and |g|^2 of the last gradient
};

// Storage element types of the solver state (the values of lfsr_storage).
enum : int { kStF32 = 0, kStF16 = 1, kStBF16 = 2 };

// Device pointers of one handle's working set.  x, wD, wS and lr hold
// elements of the storage type `st`; everything else is float / double.
struct Bufs {
  int st;          // storage type of x, wD, wS, lr
  void* x;         // [H][W] HR estimate (16-bit storage: the rounded part)
  float* dx;       // [H][W] 16-bit storage only: FP32 remainder, x = x16 + dx; CG accumulates here
  float* m;        // [H][W] weight map w_e * occ
  float* vs;       // [H][W] NLTV divergence part of v
  float* r;        // [H][W] CG residual
  float* pv;       // [H][W] CG direction
  float* hp;       // [H][W] H p
  void* wD;        // [sk][sy][sx] data dual
  void* wS[2];     // [sd][H][W] NLTV dual, ping-pong
  void* lr;        // [sk][sy][sx] e (wz-step) or t = A p (CG)
  float* adj;      // [a_nty*a_ntx][a_ey][a_ex] per-tile adjoint partial images
  double* p_wzd;   // [forward blocks][3] data-block partial sums
  double* p_tv;    // [tv blocks][2] NLTV-block partial sums
  double* p_rr[2]; // [red_blocks] <r,r> partials (ping-pong over CG steps)
  double* p_php;   // [tv blocks] <p,Hp> partials
  float* p_max;    // [max(forward blocks, kRedBlocks)] per-block max |LR| (adjoint fixed-point scale)
  int* p_cnt;      // [adjoint blocks] most contributions any accumulator cell of the block receives
  double* stats;   // [n_iter][6]
  DevScalars* sc;
};

// gate bits of the iteration kernels
enum : int {
  kGateAdmm = 1,      // skip once the ADMM stop test has fired
  kGateCg = 2,        // skip once CG has stopped
  kGateReweight = 4,  // edge weight: skip when reweight = 0 and this is not the first iteration
};

// Launchers (lfsr_kernels.hip).
size_t forward_lds(const Geom& g);
size_t adjoint_lds(const Geom& g);
size_t tv_lds(const Geom& g);
bool forward_tile_ok(const Geom& g);
// switch g to the column-per-lane forward kernel when its shape is compiled
// and its tile fits (sets f_col, f_tly, f_tlx; the caller sets f_vpb)
bool forward_col_setup(Geom& g);
// set f_orb when the mirror-orbit walk of the CG-form forward is expected to
// shorten a block's slowest wave (after f_col and f_vpb are set)
void forward_orbit_setup(Geom& g);
bool adjoint_tile_ok(const Geom& g);
// switch g to the column-per-lane adjoint when its shape is compiled and its
// tile fits (sets a_col, the tile fields and the view groups)
bool adjoint_col_setup(Geom& g);
dim3 forward_grid(const Geom& g);
dim3 adjoint_grid(const Geom& g);
dim3 tv_grid(const Geom& g);
// FP32 operator: out = A src
void launch_forward(const Geom& g, const float* src, const float* disp, float* out, hipStream_t s,
                    const Bufs& b, int gate);
// CG product: b.lr (storage type) = A src
void launch_forward_cg(const Geom& g, const float* src, const float* disp, hipStream_t s, const Bufs& b, int gate);
// data-block wz-step from b.x: b.lr = e, b.wD updated
void launch_forward_wzd(const Geom& g, const float* disp, const float* y, hipStream_t s, const Bufs& b);
// lr holds elements of storage type lr_st.  npmax: number of per-block
// maxima of |lr| in b.p_max (forward_blocks(g) after a forward launch, or
// the return value of launch_absmax)
void launch_adjoint(const Geom& g, const void* lr, int lr_st, const float* disp, hipStream_t s, const Bufs& b,
                    int gate, int npmax);
int launch_absmax(const Geom& g, const float* v, long long n, hipStream_t s, const Bufs& b);
// contribution counts of the column adjoint for a disparity map (b.p_cnt);
// must run before launch_adjoint whenever the disparity changes (no-op for
// the general adjoint)
void launch_adjcount(const Geom& g, const float* disp, hipStream_t s, const Bufs& b);
int forward_blocks(const Geom& g);
// dense A^T e from the adjoint's partial images
void launch_merge(const Geom& g, float* out, hipStream_t s, const Bufs& b, int gate);
void launch_tv(const Geom& g, hipStream_t s, const Bufs& b);
// out: H pv on exit; on entry the merged A^T A pv, unless fused (then the
// kernel gathers it from the adjoint's partial images b.adj; only when
// merge_fusable(g))
void launch_hp(const Geom& g, const float* pv, const float* m, float* out, hipStream_t s, const Bufs& b, int gate,
               int with_dot, int fused);
bool merge_fusable(const Geom& g);
// r holds the merged A^T e on entry, unless fused (then gathered from b.adj;
// only when merge_fusable(g))
void launch_cginit(const Geom& g, hipStream_t s, const Bufs& b, int fused);
void launch_cgupd(const Geom& g, int step, hipStream_t s, const Bufs& b);
void launch_cgp(const Geom& g, int step, hipStream_t s, const Bufs& b);
void launch_iter_end(const Geom& g, hipStream_t s, const Bufs& b);
void launch_edge(const Geom& g, const void* x, int x_st, const float* occ, float* m, hipStream_t s, const Bufs& b,
                 int gate);
void launch_fold(const Geom& g, hipStream_t s, const Bufs& b);                     // x16 + dx -> x16, dx
void launch_split(const Geom& g, const float* src, hipStream_t s, const Bufs& b);  // src -> x16, dx
void launch_join(const Geom& g, float* out, hipStream_t s, const Bufs& b);         // x16 + dx -> out
void launch_to_float(const void* in, int st, float* out, long long n, hipStream_t s);
void launch_from_float(const float* in, void* out, int st, long long n, hipStream_t s);
void launch_zero(void* p, int st, long long n, hipStream_t s);
void launch_bicubic(const Geom& g, const float* lrv, float* out, hipStream_t s);
// gradient-descent baselines (FP32 state): cost parts at xp (J -> sc->gd_cost;
// q = lambda1 sgn(r) + 2 lambda2 r into b.lr over its t = A xp; S^T sgn(g)
// into b.hp); gradient g = b.r + b.hp into b.pv (|g|^2 -> sc->gd_gnorm);
// out = x - eta g
void launch_gd_cost(const Geom& g, const float* xp, const float* disp, const float* y, hipStream_t s, const Bufs& b);
void launch_gd_grad(const Geom& g, const float* disp, hipStream_t s, const Bufs& b);
void launch_gd_step(const Geom& g, const float* x, float eta, float* out, hipStream_t s, const Bufs& b);
// occlusion weight: acc += squared projection error of view k; then the weight
void launch_occ_acc(const Geom& g, const float* lref, const float* lk, const float* disp, int k, float* acc,
                    hipStream_t s);
void launch_occ_final(const Geom& g, const float* disp, const float* acc, float inv_views, float c1, float c2,
                      float* out, hipStream_t s);
void launch_check(const Geom& g, const float* y, const float* disp, const float* occ, hipStream_t s, const Bufs& b);
void launch_fill(float* p, long long n, float v, hipStream_t s);
// copy an explicit blur kernel (kb * kb floats, host) to g.taps2d
void launch_set_taps(const Geom& g, const float* host_taps, hipStream_t s);
void launch_reset(int n_done, hipStream_t s, const Bufs& b);
void launch_copy_ws(float* out, long long n, hipStream_t s, const Bufs& b);

}  // namespace lfsr
