// HIP kernels (gfx950) for the ADMM light-field super-resolution iteration of
// arXiv 2206.05047: the forward model A_k = D B W_k and its exact adjoint
// (sec 3.1, 4.1), the fused z/w-steps of both dual blocks (sec 5, Algorithm 1),
// the weighted-NLTV normal operator and the CG x-step (sec 5, Algorithm 2).
//
// Design notes (MI355X / CDNA4):
//  * Every kernel runs 256-thread blocks (4 wave64).  Nothing here is a dense
//    contraction, so there is no MFMA; the warp/blur stencils are LDS-staged
//    and the dual-field streams are coalesced row-major passes.
//  * Forward operator: one block owns an LR tile and a group of views.  The HR
//    source tile (plus the blur radius and the warp halo) is staged in LDS once
//    and reused by every view of the group.  Per view the bilinear warp is
//    evaluated at every HR position the blur reads, then the separable blur is
//    evaluated only at the lattice points the decimation keeps.
//  * Adjoint: one block owns an HR tile and all views.  B D^T is applied as a
//    polyphase separable filter from an LDS copy of the LR tile, and W_k^T as a
//    scatter with the bilinear weights of W_k into per-wave LDS accumulators
//    (tile + warp halo).  Each block writes its haloed tile to a partial image;
//    the consumer kernel sums the (at most 9) overlapping tiles in a fixed
//    order, so the result is deterministic and needs no global atomics.
//  * Reductions: per-block FP64 partials, summed in a fixed order by the last
//    block to finish (device-scope fences + counter).  All control scalars
//    (CG alpha/beta/pi, stop flags) stay in device memory, so an ADMM
//    iteration never synchronises with the host.
#include "lfsr_internal.h"

namespace lfsr {

__device__ __forceinline__ int floordiv(int a, int b) {  // b > 0
  return a >= 0 ? a / b : -((-a + b - 1) / b);
}

__device__ __forceinline__ float clipf(float u, float c) { return fminf(fmaxf(u, -c), c); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum N doubles over the block; the result is valid in thread 0.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* sh /* [4*N] */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int n = 0; n < N; ++n) v[n] = wave_sum(v[n]);
  if (lane == 0) {
#pragma unroll
    for (int n = 0; n < N; ++n) sh[wid * N + n] = v[n];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] = ((sh[n] + sh[N + n]) + sh[2 * N + n]) + sh[3 * N + n];
  }
  __syncthreads();
}

// Publish this block's partials and report whether it is the last block of the
// grid to do so.  Release (writers) / acquire (last block) at device scope.
__device__ __forceinline__ bool last_block(unsigned* counter, unsigned nblocks) {
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned prev = atomicAdd(counter, 1u);
    s_last = (prev == nblocks - 1);
  }
  __syncthreads();
  if (s_last) __threadfence();
  return s_last != 0;
}

__device__ __forceinline__ double load_part(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Fixed-order reduction of nb blocks' N partials by the last block.
template <int N>
__device__ __forceinline__ void reduce_parts(const double* part, unsigned nb, double (&out)[N], double* sh) {
#pragma unroll
  for (int n = 0; n < N; ++n) out[n] = 0.0;
  for (unsigned b = threadIdx.x; b < nb; b += kThreads) {
#pragma unroll
    for (int n = 0; n < N; ++n) out[n] += load_part(part + (size_t)b * N + n);
  }
  block_sum<N>(out, sh);
}

__device__ __forceinline__ bool gated(const DevScalars* sc, int gate) {
  // gate bit 0: skip once the ADMM stop test has fired; bit 1: skip once CG has stopped
  return ((gate & 1) && sc->admm_done) || ((gate & 2) && sc->cg_done);
}

// Sum of the per-tile adjoint partial images that cover HR pixel (Y, X).
__device__ __forceinline__ float adj_merge(const Geom& g, const float* __restrict__ adj, int Y, int X) {
  const int ty = Y / g.a_th, tx = X / g.a_tw;
  const int ly = Y - ty * g.a_th, lx = X - tx * g.a_tw;
  const size_t tile = (size_t)g.a_ey * g.a_ex;
  float s = 0.f;
#pragma unroll
  for (int a = -1; a <= 1; ++a) {
    const int tty = ty + a;
    const int ey = ly - a * g.a_th + g.halo;
    if (tty < 0 || tty >= g.a_nty || ey < 0 || ey >= g.a_ey) continue;
#pragma unroll
    for (int b = -1; b <= 1; ++b) {
      const int ttx = tx + b;
      const int ex = lx - b * g.a_tw + g.halo;
      if (ttx < 0 || ttx >= g.a_ntx || ex < 0 || ex >= g.a_ex) continue;
      s += adj[((size_t)tty * g.a_ntx + ttx) * tile + (size_t)ey * g.a_ex + ex];
    }
  }
  return s;
}

// ---------------------------------------------------------------------------
// Forward operator t_k = D B W_k src for every view (sec 3.1, 4.1).
// WZD = true fuses the data-block z/w-steps of Algorithm 1: r = t - y,
// w_D' = clip(lambda1 r + w_D, +-1/vartheta) (= u - prox(u)), and the input of
// A^T, e = lambda2 r + (vartheta/2) lambda1 (2 w_D' - w_D), written to `out`.
// grid = (ceil(sx/f_tlx), ceil(sy/f_tly), ceil(sk/f_vpb)).
template <bool WZD>
__global__ __launch_bounds__(kThreads) void k_forward(Geom g, const float* __restrict__ src,
                                                      const float* __restrict__ disp, float* __restrict__ out,
                                                      const float* __restrict__ y, float* __restrict__ wD,
                                                      double* __restrict__ part, DevScalars* __restrict__ sc,
                                                      int gate) {
  if (gated(sc, gate)) return;
  extern __shared__ float smem[];
  const int zeta = g.zeta, rb = g.rb, h = g.halo;
  const int tly = g.f_tly, tlx = g.f_tlx;
  const int NY = (tly - 1) * zeta + 1 + 2 * rb;
  const int NX = (tlx - 1) * zeta + 1 + 2 * rb;
  const int SY = NY + 2 * h, SX = NX + 2 * h;
  float* xs = smem;          // [SY][SX] source tile, zero outside the image
  float* om = xs + SY * SX;  // [NY][NX] disparity at the blur positions
  float* wv = om + NY * NX;  // [NY][NX] warped values of the current view
  float* hb = wv + NY * NX;  // [NY][tlx] horizontal blur at lattice columns
  const int i0 = blockIdx.y * tly, j0 = blockIdx.x * tlx;
  const int Yp0 = i0 * zeta - rb, Xp0 = j0 * zeta - rb;
  const int tid = threadIdx.x;

  for (int idx = tid; idx < SY * SX; idx += kThreads) {
    const int ty = idx / SX, tx = idx - ty * SX;
    const int Y = Yp0 - h + ty, X = Xp0 - h + tx;
    xs[idx] = (Y >= 0 && Y < g.H && X >= 0 && X < g.W) ? src[(size_t)Y * g.W + X] : 0.f;
  }
  for (int idx = tid; idx < NY * NX; idx += kThreads) {
    const int py = idx / NX, px = idx - py * NX;
    const int Y = Yp0 + py, X = Xp0 + px;
    om[idx] = (Y >= 0 && Y < g.H && X >= 0 && X < g.W) ? disp[(size_t)Y * g.W + X] : 0.f;
  }
  __syncthreads();

  const int k0 = blockIdx.z * g.f_vpb;
  const int k1 = min(g.sk, k0 + g.f_vpb);
  const float hmin = (float)(-h), hmax = (float)(h - 1);
  double s_abs = 0.0, s_sq = 0.0, s_dw = 0.0;
  for (int k = k0; k < k1; ++k) {
    const float tau = (float)(k / g.V - (g.U - 1) / 2);
    const float rho = (float)(k % g.V - (g.V - 1) / 2);
    // W_k at every HR position the blur reads; zero outside the image
    for (int idx = tid; idx < NY * NX; idx += kThreads) {
      const int py = idx / NX, px = idx - py * NX;
      const int Y = Yp0 + py, X = Xp0 + px;
      float val = 0.f;
      if (Y >= 0 && Y < g.H && X >= 0 && X < g.W) {
        const float w = om[idx];
        const float sy = tau * w, sx = rho * w;
        float fy0 = floorf(sy), fx0 = floorf(sx);
        const float fy = sy - fy0, fx = sx - fx0;
        fy0 = fminf(fmaxf(fy0, hmin), hmax);  // memory safety only: |disp| <= disp_bound keeps it in range
        fx0 = fminf(fmaxf(fx0, hmin), hmax);
        const float* s = xs + (py + h + (int)fy0) * SX + (px + h + (int)fx0);
        const float a = s[0], b = s[1], c = s[SX], d = s[SX + 1];
        const float top = fmaf(fx, b - a, a);
        const float bot = fmaf(fx, d - c, c);
        val = fmaf(fy, bot - top, top);
      }
      wv[idx] = val;
    }
    __syncthreads();
    // B, horizontal pass, only at the lattice columns D keeps
    for (int idx = tid; idx < NY * tlx; idx += kThreads) {
      const int py = idx / tlx, j = idx - py * tlx;
      const float* s = wv + py * NX + j * zeta;
      float acc = 0.f;
      for (int b = 0; b < g.kb; ++b) acc = fmaf(g.g[b], s[b], acc);
      hb[idx] = acc;
    }
    __syncthreads();
    // B, vertical pass, only at the lattice rows; then the fused epilogue
    for (int idx = tid; idx < tly * tlx; idx += kThreads) {
      const int li = idx / tlx, lj = idx - li * tlx;
      const int i = i0 + li, j = j0 + lj;
      if (i >= g.sy || j >= g.sx) continue;
      const float* s = hb + li * zeta * tlx + lj;
      float t = 0.f;
      for (int a = 0; a < g.kb; ++a) t = fmaf(g.g[a], s[a * tlx], t);
      const size_t o = (size_t)k * g.q + (size_t)i * g.sx + j;
      if constexpr (!WZD) {
        out[o] = t;
      } else {
        const float r = t - y[o];
        const float w0 = wD[o];
        const float wn = clipf(fmaf(g.lambda1, r, w0), g.clip);
        out[o] = g.lambda2 * r + g.half_theta * g.lambda1 * (2.f * wn - w0);
        wD[o] = wn;
        const double rd = (double)r, dw = (double)wn - (double)w0;
        s_abs += fabs(rd);
        s_sq += rd * rd;
        s_dw += dw * dw;
      }
    }
  }
  if constexpr (WZD) {
    __shared__ double red[4 * 3];
    double v[3] = {s_abs, s_sq, s_dw};
    block_sum<3>(v, red);
    const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
    const unsigned bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    if (tid == 0) {
      part[(size_t)bid * 3 + 0] = v[0];
      part[(size_t)bid * 3 + 1] = v[1];
      part[(size_t)bid * 3 + 2] = v[2];
    }
    if (last_block(&sc->counters[kCntFwd], nb)) {
      double a[3];
      reduce_parts<3>(part, nb, a, red);
      if (tid == 0) {
        sc->data_abs = a[0];
        sc->data_sq = a[1];
        sc->dwD2 = a[2];
        sc->counters[kCntFwd] = 0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint sum_k A_k^T lr_k = sum_k W_k^T B^T D^T lr_k into per-tile partial
// images [tile][a_ey][a_ex] (HR tile + warp halo).  grid = (a_ntx, a_nty).
__global__ __launch_bounds__(kThreads) void k_adjoint(Geom g, const float* __restrict__ lr,
                                                      const float* __restrict__ disp, float* __restrict__ outp,
                                                      const DevScalars* __restrict__ sc, int gate) {
  if (gated(sc, gate)) return;
  extern __shared__ float smem[];
  const int zeta = g.zeta, rb = g.rb, h = g.halo;
  const int TH = g.a_th, TW = g.a_tw, EY = g.a_ey, EX = g.a_ex;
  const int ci = (rb + zeta - 1) / zeta;  // LR rows/cols of blur reach
  const int LY = g.a_tly + 2 * ci, LX = g.a_tlx + 2 * ci;
  float* acc = smem;                // [4][EY][EX] one accumulator per wave
  float* et = acc + 4 * EY * EX;    // [2][LY][LX] LR tile of the view (double buffered)
  float* hv = et + 2 * LY * LX;     // [2][TH][LX] vertical B^T pass
  const int ty = blockIdx.y, tx = blockIdx.x;
  const int i0 = ty * g.a_tly, j0 = tx * g.a_tlx;
  const int Y0 = i0 * zeta, X0 = j0 * zeta;
  const int tid = threadIdx.x, wave = tid >> 6;
  float* myacc = acc + wave * EY * EX;
  for (int idx = tid; idx < 4 * EY * EX; idx += kThreads) acc[idx] = 0.f;

  float omr[kAdjMaxPix];
#pragma unroll
  for (int s = 0; s < kAdjMaxPix; ++s) {
    const int idx = tid + s * kThreads;
    float w = 0.f;
    if (s < g.a_npix && idx < TH * TW) {
      const int ly = idx / TW, lx = idx - ly * TW;
      const int Y = Y0 + ly, X = X0 + lx;
      if (Y < g.H && X < g.W) w = disp[(size_t)Y * g.W + X];
    }
    omr[s] = w;
  }
  const float hmin = (float)(-h), hmax = (float)(h - 1);

  for (int k = 0; k < g.sk; ++k) {
    const int buf = k & 1;
    float* e_ = et + buf * LY * LX;
    float* h_ = hv + buf * TH * LX;
    const float* lk = lr + (size_t)k * g.q;
    for (int idx = tid; idx < LY * LX; idx += kThreads) {
      const int a = idx / LX, b = idx - a * LX;
      const int i = i0 - ci + a, j = j0 - ci + b;
      e_[idx] = (i >= 0 && i < g.sy && j >= 0 && j < g.sx) ? lk[(size_t)i * g.sx + j] : 0.f;
    }
    __syncthreads();
    // B^T D^T, vertical: every LR sample i with |Y - zeta i| <= rb feeds row Y
    for (int idx = tid; idx < TH * LX; idx += kThreads) {
      const int ly = idx / LX, b = idx - ly * LX;
      const int Y = Y0 + ly;
      const int ilo = floordiv(Y - rb + zeta - 1, zeta), ihi = floordiv(Y + rb, zeta);
      float a_ = 0.f;
      for (int i = ilo; i <= ihi; ++i) a_ = fmaf(g.g[Y - zeta * i + rb], e_[(i - i0 + ci) * LX + b], a_);
      h_[idx] = a_;
    }
    __syncthreads();
    const float tau = (float)(k / g.V - (g.U - 1) / 2);
    const float rho = (float)(k % g.V - (g.V - 1) / 2);
#pragma unroll
    for (int s = 0; s < kAdjMaxPix; ++s) {
      const int idx = tid + s * kThreads;
      if (s >= g.a_npix || idx >= TH * TW) break;
      const int ly = idx / TW, lx = idx - ly * TW;
      const int Y = Y0 + ly, X = X0 + lx;
      if (Y >= g.H || X >= g.W) continue;
      // B^T D^T, horizontal
      const int jlo = floordiv(X - rb + zeta - 1, zeta), jhi = floordiv(X + rb, zeta);
      float u = 0.f;
      for (int j = jlo; j <= jhi; ++j) u = fmaf(g.g[X - zeta * j + rb], h_[ly * LX + (j - j0 + ci)], u);
      // W_k^T: send u back to the four taps W_k read it from
      const float w = omr[s];
      const float sy = tau * w, sx = rho * w;
      float fy0 = floorf(sy), fx0 = floorf(sx);
      const float fy = sy - fy0, fx = sx - fx0;
      fy0 = fminf(fmaxf(fy0, hmin), hmax);
      fx0 = fminf(fmaxf(fx0, hmin), hmax);
      float* a = myacc + (ly + h + (int)fy0) * EX + (lx + h + (int)fx0);
      const float u0 = u * (1.f - fy), u1 = u * fy;
      atomicAdd(a, u0 * (1.f - fx));
      atomicAdd(a + 1, u0 * fx);
      atomicAdd(a + EX, u1 * (1.f - fx));
      atomicAdd(a + EX + 1, u1 * fx);
    }
  }
  __syncthreads();
  float* o = outp + ((size_t)ty * g.a_ntx + tx) * (size_t)(EY * EX);
  const int n = EY * EX;
  for (int idx = tid; idx < n; idx += kThreads)
    o[idx] = ((acc[idx] + acc[n + idx]) + acc[2 * n + idx]) + acc[3 * n + idx];
}

// out = sum of the adjoint partial images (the operator entry point).
__global__ __launch_bounds__(kThreads) void k_merge(Geom g, const float* __restrict__ adj, float* __restrict__ out) {
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < g.p; o += (long long)gridDim.x * kThreads) {
    const int Y = (int)(o / g.W), X = (int)(o - (long long)Y * g.W);
    out[o] = adj_merge(g, adj, Y, X);
  }
}

// ---------------------------------------------------------------------------
// NLTV block of the wz-step (sec 3.4, 4.1; Algorithm 1): for every offset d
//   g_d = c_d m (x - S_d x)  (dropped where z+d is outside),
//   w_S' = clip(g_d + w_S, +-1/vartheta),  f_d = 2 w_S' - w_S,
//   vs = S^T f = sum_d [c_d m(z) f_d(z) 1(z+d in) - c_d m(z-d) f_d(z-d) 1(z-d in)].
// The second term is pulled, recomputing f_d(z-d) from the previous dual
// (ping-pong buffers make that read race-free).  grid = (ceil(W/64), ceil(H/16)).
__global__ __launch_bounds__(kThreads) void k_tv(Geom g, const float* __restrict__ x, const float* __restrict__ m,
                                                 float* __restrict__ ws0, float* __restrict__ ws1,
                                                 float* __restrict__ vs, double* __restrict__ part,
                                                 DevScalars* __restrict__ sc) {
  if (sc->admm_done) return;
  extern __shared__ float smem[];
  const int rw = g.rw;
  const int LXd = kTvTileX + 2 * rw, LYd = kTvTileY + 2 * rw;
  float* xs = smem;
  float* ms = xs + LYd * LXd;
  const int X0 = blockIdx.x * kTvTileX, Y0 = blockIdx.y * kTvTileY;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < LYd * LXd; idx += kThreads) {
    const int a = idx / LXd, b = idx - a * LXd;
    const int Y = Y0 - rw + a, X = X0 - rw + b;
    const bool in = Y >= 0 && Y < g.H && X >= 0 && X < g.W;
    xs[idx] = in ? x[(size_t)Y * g.W + X] : 0.f;
    ms[idx] = in ? m[(size_t)Y * g.W + X] : 0.f;
  }
  __syncthreads();
  const float* wo = sc->wcur ? ws1 : ws0;
  float* wn_ = sc->wcur ? ws0 : ws1;
  const int lx = tid & 63, ly0 = tid >> 6;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  double s_abs = 0.0, s_dw = 0.0;
  const int half = (g.win * g.win) / 2;
  for (int d = 0; d < g.sd; ++d) {
    const int id = d < half ? d : d + 1;
    const int dy = id / g.win - rw, dx = id - (id / g.win) * g.win - rw;
    const float c = g.cd[d];
    const float* wod = wo + (size_t)d * g.p;
    float* wnd = wn_ + (size_t)d * g.p;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int ly = ly0 + 4 * rr;
      const int Y = Y0 + ly, X = X0 + lx;
      if (Y >= g.H || X >= g.W) continue;
      const size_t o = (size_t)Y * g.W + X;
      const int sl = (ly + rw) * LXd + (lx + rw);
      const float xz = xs[sl], mz = ms[sl];
      const bool fwd_in = Y + dy >= 0 && Y + dy < g.H && X + dx >= 0 && X + dx < g.W;
      const float gv = fwd_in ? c * mz * (xz - xs[sl + dy * LXd + dx]) : 0.f;
      const float w0 = wod[o];
      const float wn = clipf(gv + w0, g.clip);
      wnd[o] = wn;
      if (fwd_in) acc[rr] = fmaf(c * mz, 2.f * wn - w0, acc[rr]);
      const double dw = (double)wn - (double)w0;
      s_abs += fabs((double)gv);
      s_dw += dw * dw;
      const int Ym = Y - dy, Xm = X - dx;
      if (Ym >= 0 && Ym < g.H && Xm >= 0 && Xm < g.W) {
        const int sm = sl - dy * LXd - dx;
        const float mm = ms[sm];
        const float g2 = c * mm * (xs[sm] - xz);
        const float w2 = wod[(size_t)Ym * g.W + Xm];
        const float wn2 = clipf(g2 + w2, g.clip);
        acc[rr] = fmaf(-(c * mm), 2.f * wn2 - w2, acc[rr]);
      }
    }
  }
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int Y = Y0 + ly0 + 4 * rr, X = X0 + lx;
    if (Y < g.H && X < g.W) vs[(size_t)Y * g.W + X] = acc[rr];
  }
  __shared__ double red[4 * 2];
  double v[2] = {s_abs, s_dw};
  block_sum<2>(v, red);
  const unsigned nb = gridDim.x * gridDim.y;
  const unsigned bid = blockIdx.x + gridDim.x * blockIdx.y;
  if (tid == 0) {
    part[(size_t)bid * 2 + 0] = v[0];
    part[(size_t)bid * 2 + 1] = v[1];
  }
  if (last_block(&sc->counters[kCntTv], nb)) {
    double a[2];
    reduce_parts<2>(part, nb, a, red);
    if (tid == 0) {
      sc->reg_abs = a[0];
      sc->dwS2 = a[1];
      sc->counters[kCntTv] = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// H p = cA * sum_k A_k^T A_k p + (vartheta/2) S^T V^2 S p (sec 5), the NLTV
// part written as the symmetric weighted Laplacian
//   sum_d c_d^2 (m(z)^2 + m(z+d)^2) (p(z) - p(z+d)) 1(z+d in the image),
// which equals S^T V^2 S p because the offset set is symmetric.  With
// with_dot, also <p, Hp> and alpha = pi / <p, Hp> (last block).
__global__ __launch_bounds__(kThreads) void k_hp(Geom g, const float* __restrict__ pv, const float* __restrict__ m,
                                                 const float* __restrict__ adj, float* __restrict__ hp,
                                                 double* __restrict__ part, DevScalars* __restrict__ sc, int gate,
                                                 int with_dot) {
  if (gated(sc, gate)) return;
  extern __shared__ float smem[];
  const int rw = g.rw;
  const int LXd = kTvTileX + 2 * rw, LYd = kTvTileY + 2 * rw;
  float* ps = smem;
  float* m2 = ps + LYd * LXd;
  const int X0 = blockIdx.x * kTvTileX, Y0 = blockIdx.y * kTvTileY;
  const int tid = threadIdx.x;
  if (g.sd > 0) {
    for (int idx = tid; idx < LYd * LXd; idx += kThreads) {
      const int a = idx / LXd, b = idx - a * LXd;
      const int Y = Y0 - rw + a, X = X0 - rw + b;
      const bool in = Y >= 0 && Y < g.H && X >= 0 && X < g.W;
      ps[idx] = in ? pv[(size_t)Y * g.W + X] : 0.f;
      const float mv = in ? m[(size_t)Y * g.W + X] : 0.f;
      m2[idx] = mv * mv;
    }
  }
  __syncthreads();
  const int lx = tid & 63, ly0 = tid >> 6;
  const int half = (g.win * g.win) / 2;
  double s_dot = 0.0;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int ly = ly0 + 4 * rr;
    const int Y = Y0 + ly, X = X0 + lx;
    if (Y >= g.H || X >= g.W) continue;
    const size_t o = (size_t)Y * g.W + X;
    float lap = 0.f;
    if (g.sd > 0) {
      const int sl = (ly + rw) * LXd + (lx + rw);
      const float pz = ps[sl], mz = m2[sl];
      for (int d = 0; d < g.sd; ++d) {
        const int id = d < half ? d : d + 1;
        const int dy = id / g.win - rw, dx = id - (id / g.win) * g.win - rw;
        if (Y + dy < 0 || Y + dy >= g.H || X + dx < 0 || X + dx >= g.W) continue;
        const int sn = sl + dy * LXd + dx;
        lap = fmaf(g.cd2[d] * (mz + m2[sn]), pz - ps[sn], lap);
      }
    }
    const float v = g.cA * adj_merge(g, adj, Y, X) + g.half_theta * lap;
    hp[o] = v;
    if (with_dot) s_dot += (double)pv[o] * (double)v;
  }
  if (!with_dot) return;
  __shared__ double red[4];
  double v[1] = {s_dot};
  block_sum<1>(v, red);
  const unsigned nb = gridDim.x * gridDim.y;
  const unsigned bid = blockIdx.x + gridDim.x * blockIdx.y;
  if (tid == 0) part[bid] = v[0];
  if (last_block(&sc->counters[kCntHp], nb)) {
    double a[1];
    reduce_parts<1>(part, nb, a, red);
    if (tid == 0) {
      const double php = a[0];
      sc->php = php;
      if (php > 0.0) {
        sc->alpha = sc->pi / php;
      } else {
        sc->alpha = 0.0;
        sc->cg_done = 1;
      }
      sc->counters[kCntHp] = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// CG start (Algorithm 2 from delta = 0): v = A^T e + (vartheta/2) S^T f,
// r = -v, p = r, pi = <r, r>.  The last block also closes the wz-step's
// statistics: J(x^(n-1)) and the primal residual.
__global__ __launch_bounds__(kThreads) void k_cginit(Geom g, const float* __restrict__ adj,
                                                     const float* __restrict__ vs, float* __restrict__ r,
                                                     float* __restrict__ pv, double* __restrict__ part,
                                                     DevScalars* __restrict__ sc, double* __restrict__ stats_row) {
  if (sc->admm_done) return;
  double s = 0.0;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < g.p; o += (long long)gridDim.x * kThreads) {
    const int Y = (int)(o / g.W), X = (int)(o - (long long)Y * g.W);
    float v = adj_merge(g, adj, Y, X);
    if (g.sd > 0) v += g.half_theta * vs[o];
    const float rv = -v;
    r[o] = rv;
    pv[o] = rv;
    s += (double)rv * (double)rv;
  }
  __shared__ double red[4];
  double v[1] = {s};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
  if (last_block(&sc->counters[kCntInit], gridDim.x)) {
    double a[1];
    reduce_parts<1>(part, gridDim.x, a, red);
    if (threadIdx.x == 0) {
      const double pi = a[0];
      sc->pi = pi;
      sc->cg_steps = 0;
      sc->cg_done = (!(pi > (double)g.cg_tol) || pi == 0.0) ? 1 : 0;
      const double reg = g.sd > 0 ? sc->reg_abs : 0.0;
      const double dws = g.sd > 0 ? sc->dwS2 : 0.0;
      const double data = (double)g.lambda1 * sc->data_abs + (double)g.lambda2 * sc->data_sq;
      const double res = sqrt(sc->dwD2 + dws);
      stats_row[0] = data + reg;
      stats_row[1] = res;
      stats_row[4] = data;
      stats_row[5] = reg;
      if (!sc->res1_set) {
        sc->res1 = res;
        sc->res1_set = 1;
      }
      if (g.stop_tol > 0.f && res <= (double)g.stop_tol * sc->res1) sc->stop_pending = 1;
      sc->counters[kCntInit] = 0;
    }
  }
}

// x += alpha p (the x-step accumulates straight into x), r -= alpha Hp,
// pi' = <r, r>, beta = pi'/pi; CG stops once pi' <= tau or pi' = 0.
__global__ __launch_bounds__(kThreads) void k_cgupd(Geom g, float* __restrict__ x, float* __restrict__ r,
                                                    const float* __restrict__ pv, const float* __restrict__ hp,
                                                    double* __restrict__ part, DevScalars* __restrict__ sc) {
  if (sc->admm_done || sc->cg_done) return;
  const float alpha = (float)sc->alpha;
  double s = 0.0;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < g.p; o += (long long)gridDim.x * kThreads) {
    x[o] = fmaf(alpha, pv[o], x[o]);
    const float rv = fmaf(-alpha, hp[o], r[o]);
    r[o] = rv;
    s += (double)rv * (double)rv;
  }
  __shared__ double red[4];
  double v[1] = {s};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
  if (last_block(&sc->counters[kCntUpd], gridDim.x)) {
    double a[1];
    reduce_parts<1>(part, gridDim.x, a, red);
    if (threadIdx.x == 0) {
      const double pin = a[0];
      sc->beta = pin / sc->pi;
      sc->pi = pin;
      sc->cg_steps += 1;
      if (!(pin > (double)g.cg_tol) || pin == 0.0) sc->cg_done = 1;
      sc->counters[kCntUpd] = 0;
    }
  }
}

// p = r + beta p
__global__ __launch_bounds__(kThreads) void k_cgp(Geom g, const float* __restrict__ r, float* __restrict__ pv,
                                                  const DevScalars* __restrict__ sc) {
  if (sc->admm_done || sc->cg_done) return;
  const float beta = (float)sc->beta;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < g.p; o += (long long)gridDim.x * kThreads)
    pv[o] = fmaf(beta, pv[o], r[o]);
}

// End of an ADMM iteration: CG statistics, iteration count, dual ping-pong, stop flag.
__global__ void k_iter_end(DevScalars* __restrict__ sc, double* __restrict__ stats_row, int has_tv) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (sc->admm_done) return;
  stats_row[2] = sc->pi;
  stats_row[3] = (double)sc->cg_steps;
  sc->iters_done += 1;
  if (has_tv) sc->wcur ^= 1;
  if (sc->stop_pending) sc->admm_done = 1;
}

// ---------------------------------------------------------------------------
// sec 3.4: m = exp(-|grad x|^2 / sigma_e) * occ, forward differences.
__global__ __launch_bounds__(kThreads) void k_edge(Geom g, const float* __restrict__ x, const float* __restrict__ occ,
                                                   float* __restrict__ m, const DevScalars* __restrict__ sc, int gate) {
  if (gated(sc, gate)) return;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < g.p; o += (long long)gridDim.x * kThreads) {
    const int Y = (int)(o / g.W), X = (int)(o - (long long)Y * g.W);
    float we = 1.f;
    if (g.use_edge) {
      const float xz = x[o];
      const float gx = X + 1 < g.W ? x[o + 1] - xz : 0.f;
      const float gy = Y + 1 < g.H ? x[o + g.W] - xz : 0.f;
      we = expf(-(gx * gx + gy * gy) * g.inv_sigma_e);
    }
    m[o] = occ ? we * occ[o] : we;
  }
}

// Keys cubic convolution, a = -1/2.
__device__ __forceinline__ float keys(float s) {
  s = fabsf(s);
  if (s <= 1.f) return (1.5f * s - 2.5f) * s * s + 1.f;
  if (s < 2.f) return ((-0.5f * s + 2.5f) * s - 4.f) * s + 2.f;
  return 0.f;
}

// sec 5: x0 = bicubic up-sampling of one LR view, LR (i,j) at HR (zeta i, zeta j), clamp-to-edge.
__global__ __launch_bounds__(kThreads) void k_bicubic(Geom g, const float* __restrict__ lrv, float* __restrict__ out) {
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < g.p; o += (long long)gridDim.x * kThreads) {
    const int Y = (int)(o / g.W), X = (int)(o - (long long)Y * g.W);
    const int iy = Y / g.zeta, ix = X / g.zeta;
    const float fy = (float)(Y - iy * g.zeta) / (float)g.zeta;
    const float fx = (float)(X - ix * g.zeta) / (float)g.zeta;
    float wy[4], wx[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      wy[t] = keys(fy - (float)(t - 1));
      wx[t] = keys(fx - (float)(t - 1));
    }
    float acc = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = min(max(iy + a - 1, 0), g.sy - 1);
      float row = 0.f;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int j = min(max(ix + b - 1, 0), g.sx - 1);
        row = fmaf(wx[b], lrv[(size_t)i * g.sx + j], row);
      }
      acc = fmaf(wy[a], row, acc);
    }
    out[o] = acc;
  }
}

// Input check: non-finite LR / disparity / occlusion values (bit 0) and
// |disp| > disp_bound (bit 1).
__global__ __launch_bounds__(kThreads) void k_check(Geom g, const float* __restrict__ y, const float* __restrict__ disp,
                                                    const float* __restrict__ occ, DevScalars* __restrict__ sc) {
  int f = 0;
  const long long ny = (long long)g.sk * g.q;
  const long long n = ny > g.p ? ny : g.p;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < n; o += (long long)gridDim.x * kThreads) {
    if (o < ny && !isfinite(y[o])) f |= 1;
    if (o < g.p) {
      const float d = disp[o];
      if (!isfinite(d)) f |= 1;
      else if (fabsf(d) > g.disp_bound) f |= 2;
      if (occ && !isfinite(occ[o])) f |= 1;
    }
  }
  if (f) atomicOr(&sc->err_flags, f);
}

// Fill n floats with a value (used instead of hipMemsetAsync so that the
// sequence can be captured in a graph).
__global__ __launch_bounds__(kThreads) void k_fill(float* __restrict__ p, long long n, float v) {
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < n; o += (long long)gridDim.x * kThreads) p[o] = v;
}

// Reset the device scalars for a fresh state (iters_done = n_done).
__global__ void k_reset(DevScalars* sc, int n_done) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  sc->pi = sc->alpha = sc->beta = sc->php = 0.0;
  sc->data_abs = sc->data_sq = sc->dwD2 = sc->reg_abs = sc->dwS2 = 0.0;
  sc->res1 = 0.0;
  sc->res1_set = 0;
  sc->cg_done = sc->admm_done = sc->stop_pending = sc->cg_steps = 0;
  sc->iters_done = n_done;
  sc->err_flags = 0;
  sc->wcur = 0;
  for (int i = 0; i < 16; ++i) sc->counters[i] = 0;
}

// Copy the current NLTV dual (selected on the device) out, or a new one in.
__global__ __launch_bounds__(kThreads) void k_copy_ws(const float* __restrict__ ws0, const float* __restrict__ ws1,
                                                      float* __restrict__ out, long long n,
                                                      const DevScalars* __restrict__ sc) {
  const float* s = sc->wcur ? ws1 : ws0;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < n; o += (long long)gridDim.x * kThreads) out[o] = s[o];
}

// ---------------------------------------------------------------------------
// Launch helpers (host side).

static inline unsigned grid1d(long long n) {
  long long b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > kRedBlocks) b = kRedBlocks;
  return (unsigned)b;
}

size_t forward_lds(const Geom& g) {
  const int NY = (g.f_tly - 1) * g.zeta + 1 + 2 * g.rb;
  const int NX = (g.f_tlx - 1) * g.zeta + 1 + 2 * g.rb;
  const int SY = NY + 2 * g.halo, SX = NX + 2 * g.halo;
  return sizeof(float) * ((size_t)SY * SX + 2 * (size_t)NY * NX + (size_t)NY * g.f_tlx);
}

size_t adjoint_lds(const Geom& g) {
  const int ci = (g.rb + g.zeta - 1) / g.zeta;
  const int LY = g.a_tly + 2 * ci, LX = g.a_tlx + 2 * ci;
  return sizeof(float) * (4 * (size_t)g.a_ey * g.a_ex + 2 * (size_t)LY * LX + 2 * (size_t)g.a_th * LX);
}

size_t tv_lds(const Geom& g) {
  return sizeof(float) * 2 * (size_t)(kTvTileX + 2 * g.rw) * (kTvTileY + 2 * g.rw);
}

dim3 forward_grid(const Geom& g) {
  return dim3((g.sx + g.f_tlx - 1) / g.f_tlx, (g.sy + g.f_tly - 1) / g.f_tly, (g.sk + g.f_vpb - 1) / g.f_vpb);
}
dim3 adjoint_grid(const Geom& g) { return dim3(g.a_ntx, g.a_nty, 1); }
dim3 tv_grid(const Geom& g) { return dim3((g.W + kTvTileX - 1) / kTvTileX, (g.H + kTvTileY - 1) / kTvTileY, 1); }
unsigned red_blocks(const Geom& g) { return grid1d(g.p); }

void launch_forward(const Geom& g, const float* src, const float* disp, float* out, hipStream_t s,
                    const Bufs& b, int gate) {
  hipLaunchKernelGGL(k_forward<false>, forward_grid(g), dim3(kThreads), forward_lds(g), s, g, src, disp, out,
                     (const float*)nullptr, (float*)nullptr, b.part, b.sc, gate);
}

void launch_forward_wzd(const Geom& g, const float* src, const float* disp, const float* y, hipStream_t s,
                        const Bufs& b) {
  hipLaunchKernelGGL(k_forward<true>, forward_grid(g), dim3(kThreads), forward_lds(g), s, g, src, disp, b.lr, y,
                     b.wD, b.part, b.sc, 1);
}

void launch_adjoint(const Geom& g, const float* lr, const float* disp, hipStream_t s, const Bufs& b, int gate) {
  hipLaunchKernelGGL(k_adjoint, adjoint_grid(g), dim3(kThreads), adjoint_lds(g), s, g, lr, disp, b.adj,
                     (const DevScalars*)b.sc, gate);
}

void launch_merge(const Geom& g, float* out, hipStream_t s, const Bufs& b) {
  hipLaunchKernelGGL(k_merge, dim3(grid1d(g.p)), dim3(kThreads), 0, s, g, (const float*)b.adj, out);
}

void launch_tv(const Geom& g, hipStream_t s, const Bufs& b) {
  hipLaunchKernelGGL(k_tv, tv_grid(g), dim3(kThreads), tv_lds(g), s, g, (const float*)b.x, (const float*)b.m,
                     b.wS[0], b.wS[1], b.vs, b.part, b.sc);
}

void launch_hp(const Geom& g, const float* pv, const float* m, float* out, hipStream_t s, const Bufs& b, int gate,
               int with_dot) {
  hipLaunchKernelGGL(k_hp, tv_grid(g), dim3(kThreads), tv_lds(g), s, g, pv, m, (const float*)b.adj, out, b.part,
                     b.sc, gate, with_dot);
}

void launch_cginit(const Geom& g, double* stats_row, hipStream_t s, const Bufs& b) {
  hipLaunchKernelGGL(k_cginit, dim3(red_blocks(g)), dim3(kThreads), 0, s, g, (const float*)b.adj,
                     (const float*)b.vs, b.r, b.pv, b.part, b.sc, stats_row);
}

void launch_cgupd(const Geom& g, hipStream_t s, const Bufs& b) {
  hipLaunchKernelGGL(k_cgupd, dim3(red_blocks(g)), dim3(kThreads), 0, s, g, b.x, b.r, (const float*)b.pv,
                     (const float*)b.hp, b.part, b.sc);
}

void launch_cgp(const Geom& g, hipStream_t s, const Bufs& b) {
  hipLaunchKernelGGL(k_cgp, dim3(red_blocks(g)), dim3(kThreads), 0, s, g, (const float*)b.r, b.pv,
                     (const DevScalars*)b.sc);
}

void launch_iter_end(const Geom& g, double* stats_row, hipStream_t s, const Bufs& b) {
  hipLaunchKernelGGL(k_iter_end, dim3(1), dim3(64), 0, s, b.sc, stats_row, g.sd > 0 ? 1 : 0);
}

void launch_edge(const Geom& g, const float* x, const float* occ, float* m, hipStream_t s, const Bufs& b, int gate) {
  hipLaunchKernelGGL(k_edge, dim3(grid1d(g.p)), dim3(kThreads), 0, s, g, x, occ, m, (const DevScalars*)b.sc, gate);
}

void launch_bicubic(const Geom& g, const float* lrv, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_bicubic, dim3(grid1d(g.p)), dim3(kThreads), 0, s, g, lrv, out);
}

void launch_check(const Geom& g, const float* y, const float* disp, const float* occ, hipStream_t s, const Bufs& b) {
  long long n = (long long)g.sk * g.q;
  if (n < g.p) n = g.p;
  hipLaunchKernelGGL(k_check, dim3(grid1d(n)), dim3(kThreads), 0, s, g, y, disp, occ, b.sc);
}

void launch_fill(float* p, long long n, float v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(grid1d(n)), dim3(kThreads), 0, s, p, n, v);
}

void launch_reset(int n_done, hipStream_t s, const Bufs& b) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, b.sc, n_done);
}

void launch_copy_ws(float* out, long long n, hipStream_t s, const Bufs& b) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy_ws, dim3(grid1d(n)), dim3(kThreads), 0, s, (const float*)b.wS[0],
                     (const float*)b.wS[1], out, n, (const DevScalars*)b.sc);
}

}  // namespace lfsr
