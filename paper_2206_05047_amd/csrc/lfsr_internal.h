// Internal types shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lfsr {

constexpr int kMaxTaps = 31;      // blur size limit
constexpr int kMaxWin = 15;       // NLTV window limit
constexpr int kMaxOffsets = kMaxWin * kMaxWin - 1;
constexpr int kThreads = 256;     // every kernel runs 256-thread (4 x wave64) blocks
constexpr int kAdjMaxPix = 16;    // HR pixels per thread in the adjoint tile
constexpr int kTvTileX = 64, kTvTileY = 16;  // NLTV / normal-operator tiles
constexpr int kRedBlocks = 1024;  // grid of the element-wise reduction kernels

// Problem geometry and model constants, passed by value to every kernel.
struct Geom {
  int U, V, sk, kref;         // angular grid, views, reference (centre) view
  int sy, sx, zeta, H, W;     // LR size, scale, HR size
  long long q, p;             // LR and HR pixel counts
  int kb, rb;                 // blur size and radius
  float g[kMaxTaps];          // normalised 1-D Gaussian taps (2-D kernel = g x g)
  int win, rw, sd;            // NLTV window, radius, number of offsets
  float cd[kMaxOffsets];      // spatial weight exp(-|d|^2/sigma_s) of offset d
  float cd2[kMaxOffsets];     // its square
  float lambda1, lambda2;
  float half_theta;           // vartheta / 2
  float clip;                 // 1 / vartheta
  float cA;                   // lambda2 + vartheta lambda1^2 / 2
  float inv_sigma_e;          // 1/sigma_e (0 when the edge weight is off)
  int use_edge;
  int halo;                   // warp halo in HR px: ceil(max |theta| * disp_bound) + 1
  float disp_bound;
  float cg_tol;
  float stop_tol;
  // forward-operator tiling: LR tile and views per block
  int f_tly, f_tlx, f_vpb;
  // adjoint tiling: LR tile, HR tile, extended (haloed) tile, tile grid
  int a_tly, a_tlx, a_th, a_tw, a_ey, a_ex, a_nty, a_ntx;
  int a_npix;                 // HR pixels per thread (<= kAdjMaxPix)
};

// Device-resident scalars of one handle (lives in the workspace).
struct DevScalars {
  double pi;        // CG |r|^2
  double alpha, beta;
  double php;       // <p, Hp>
  double data_abs, data_sq, dwD2;   // wz-step data-block partial results
  double reg_abs, dwS2;             // wz-step NLTV-block partial results
  double res1;      // primal residual of the first iteration (stop test)
  int res1_set;
  int wcur;         // which NLTV dual buffer holds the current w_S
  int cg_done;      // CG of the current x-step has stopped
  int admm_done;    // stop test met: later iterations are no-ops
  int stop_pending;
  int cg_steps;
  int iters_done;
  int err_flags;    // bit 0: non-finite input, bit 1: |disp| > disp_bound
  unsigned counters[16];  // last-block counters, one per reduction site
};

enum Counter { kCntFwd = 0, kCntTv, kCntInit, kCntHp, kCntUpd, kCntCheck };

// Device pointers of one handle's working set.
struct Bufs {
  float* x;        // [H][W] HR estimate
  float* m;        // [H][W] weight map w_e * occ
  float* vs;       // [H][W] NLTV divergence part of v
  float* r;        // [H][W] CG residual
  float* pv;       // [H][W] CG direction
  float* hp;       // [H][W] H p
  float* wD;       // [sk][sy][sx] data dual
  float* wS[2];    // [sd][H][W] NLTV dual, ping-pong
  float* lr;       // [sk][sy][sx] e (wz-step) or t = A p (CG)
  float* adj;      // [a_nty*a_ntx][a_ey][a_ex] per-tile adjoint partial images
  double* part;    // per-block FP64 partial sums
  double* stats;   // [admm_iters][6]
  DevScalars* sc;
};

// Launchers (lfsr_kernels.hip).  gate bit 0: skip after the ADMM stop test
// fired, bit 1: skip after CG stopped (0 for the plain operator entry points).
size_t forward_lds(const Geom& g);
size_t adjoint_lds(const Geom& g);
size_t tv_lds(const Geom& g);
dim3 forward_grid(const Geom& g);
dim3 adjoint_grid(const Geom& g);
dim3 tv_grid(const Geom& g);
unsigned red_blocks(const Geom& g);
void launch_forward(const Geom& g, const float* src, const float* disp, float* out, hipStream_t s,
                    const Bufs& b, int gate);
void launch_forward_wzd(const Geom& g, const float* src, const float* disp, const float* y, hipStream_t s,
                        const Bufs& b);
void launch_adjoint(const Geom& g, const float* lr, const float* disp, hipStream_t s, const Bufs& b, int gate);
void launch_merge(const Geom& g, float* out, hipStream_t s, const Bufs& b);
void launch_tv(const Geom& g, hipStream_t s, const Bufs& b);
void launch_hp(const Geom& g, const float* pv, const float* m, float* out, hipStream_t s, const Bufs& b, int gate,
               int with_dot);
void launch_cginit(const Geom& g, double* stats_row, hipStream_t s, const Bufs& b);
void launch_cgupd(const Geom& g, hipStream_t s, const Bufs& b);
void launch_cgp(const Geom& g, hipStream_t s, const Bufs& b);
void launch_iter_end(const Geom& g, double* stats_row, hipStream_t s, const Bufs& b);
void launch_edge(const Geom& g, const float* x, const float* occ, float* m, hipStream_t s, const Bufs& b, int gate);
void launch_bicubic(const Geom& g, const float* lrv, float* out, hipStream_t s);
void launch_check(const Geom& g, const float* y, const float* disp, const float* occ, hipStream_t s, const Bufs& b);
void launch_fill(float* p, long long n, float v, hipStream_t s);
void launch_reset(int n_done, hipStream_t s, const Bufs& b);
void launch_copy_ws(float* out, long long n, hipStream_t s, const Bufs& b);

}  // namespace lfsr
