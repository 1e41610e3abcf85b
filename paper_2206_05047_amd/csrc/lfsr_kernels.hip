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
//    source tile (plus blur radius and warp halo) is staged in LDS once and
//    reused by every view of the group.  Each thread keeps the disparity and
//    LDS offset of its blur positions in registers; per view it issues all of
//    its bilinear gathers before any LDS store, then the separable blur is
//    evaluated only at the lattice points the decimation keeps.
//  * Adjoint: one block owns an HR tile and all views.  B D^T is a polyphase
//    separable filter from an LDS copy of the LR tile (prefetched one view
//    ahead), and W_k^T the scatter with the bilinear weights of W_k into
//    per-wave LDS accumulators (tile + warp halo).  Each block writes its
//    haloed tile to a partial image; consumers sum the overlapping tiles in a
//    fixed order: deterministic, and no global atomics.
//  * Reductions: per-block FP64 partials.  The consumer kernel re-reduces them
//    in a fixed order in every block (partials are visible across the kernel
//    boundary), so no kernel needs a device-scope fence -- on this part such a
//    fence writes back the whole L2 of the XCD.  Control scalars (CG alpha,
//    beta, pi, stop flags) stay on the device: an ADMM iteration never waits
//    for the host.
#include <type_traits>

#include "lfsr_internal.h"

namespace lfsr {

__device__ __forceinline__ int floordiv(int a, int b) {  // b > 0
  return a >= 0 ? a / b : -((-a + b - 1) / b);
}

// projection onto [-c, c] (c >= 0): the median of (u, -c, c), one v_med3_f32
__device__ __forceinline__ float clipf(float u, float c) { return __builtin_amdgcn_fmed3f(u, -c, c); }

// floor(v) as an integer in one instruction (v_cvt_flr_i32_f32); with
// __builtin_amdgcn_fractf (v_fract_f32: v - floor(v), kept below 1) a warp
// coordinate splits into cell and bilinear weight in two instructions
__device__ __forceinline__ int floor_i(float v) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(v));
  return r;
}
// round to nearest (halves up) as an integer in one instruction (v_cvt_rpi_i32_f32)
__device__ __forceinline__ int round_i(float v) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(v));
  return r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum N doubles over a block of NW waves (fixed order); every thread
// receives the totals.
template <int N, int NW = 4>
__device__ __forceinline__ void block_sum(double (&v)[N]) {
  __shared__ double sh[NW * N];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int n = 0; n < N; ++n) v[n] = wave_sum(v[n]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int n = 0; n < N; ++n) sh[wid * N + n] = v[n];
  }
  __syncthreads();
#pragma unroll
  for (int n = 0; n < N; ++n) {
    double t = sh[n];
#pragma unroll
    for (int w = 1; w < NW; ++w) t += sh[w * N + n];
    v[n] = t;
  }
}

// Fixed-order sum of component c of nb per-block partials (stride N); every
// thread of the block receives the same value.
template <int N, int NT = kThreads>
__device__ __forceinline__ void sum_parts(const double* __restrict__ part, int nb, double (&out)[N]) {
#pragma unroll
  for (int n = 0; n < N; ++n) out[n] = 0.0;
  for (int b = threadIdx.x; b < nb; b += NT) {
#pragma unroll
    for (int n = 0; n < N; ++n) out[n] += part[(size_t)b * N + n];
  }
  block_sum<N, NT / 64>(out);
}

// Tile of a block in a 1-D grid of 8 * ceil(ntx * nty / 8) blocks.  Blocks
// are dispatched to the eight XCDs round-robin, so XCD k (blocks k, k+8, ...)
// gets the contiguous row-major run of tiles k * ceil(n/8) ..: neighbouring
// tiles, which read each other's halo cache lines, then share one L2.  The
// padding blocks (t >= ntx * nty) return false.
__device__ __forceinline__ bool xcd_tile(int ntx, int nty, int& tx, int& ty, int& t) {
  const int nb = ntx * nty, per = (nb + 7) / 8, b = blockIdx.x;
  t = (b & 7) * per + (b >> 3);
  if (t >= nb) return false;
  ty = t / ntx;
  tx = t - ty * ntx;
  return true;
}

// The same XCD-aware order inside a grid of any shape, as a bijection: the
// block's linear index b (x fastest) runs on XCD b % 8, and XCD k takes the
// contiguous run of linear tile indices [k q + min(k, r), ... + count) where
// nb = 8 q + r; the run is decoded back into (x, y, z) of the grid.
__device__ __forceinline__ void xcd_block3(int& bx, int& by, int& bz) {
  const unsigned nx = gridDim.x, nxy = gridDim.x * gridDim.y, nb = nxy * gridDim.z;
  const unsigned b = blockIdx.x + nx * (blockIdx.y + gridDim.y * blockIdx.z);
  const unsigned q = nb >> 3, r = nb & 7u, k = b & 7u;
  const unsigned t = k * q + (k < r ? k : r) + (b >> 3);
  bz = (int)(t / nxy);
  const unsigned rem = t - (unsigned)bz * nxy;
  by = (int)(rem / nx);
  bx = (int)(rem - (unsigned)by * nx);
}

__device__ __forceinline__ bool gated(const DevScalars* sc, const Geom& g, int gate) {
  if ((gate & kGateAdmm) && sc->admm_done) return true;
  if ((gate & kGateCg) && sc->cg_done) return true;
  if ((gate & kGateReweight) && !g.reweight && sc->iters_done != 0) return true;
  return false;
}

__device__ __forceinline__ double* stats_row(const Geom& g, double* stats, const DevScalars* sc) {
  const int r = sc->iters_done < g.n_iter ? sc->iters_done : g.n_iter - 1;
  return stats + (size_t)r * 6;
}

// Raw buffer access to one plane of a storage-typed array: a scalar
// descriptor per plane and a 32-bit byte offset per lane (no 64-bit address
// per access).  Descriptor word 3 is the gfx9-family raw-buffer format.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, 0x7fffffff, 0x00020000);
}
// Largest of the n per-block maxima in pm, this thread's share: four
// independent loads per trip, so their latencies overlap.
__device__ __forceinline__ float max_parts(const float* __restrict__ pm, int n) {
  float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f;
  int i = threadIdx.x;
  for (; i + 3 * kThreads < n; i += 4 * kThreads) {
    m0 = fmaxf(m0, pm[i]);
    m1 = fmaxf(m1, pm[i + kThreads]);
    m2 = fmaxf(m2, pm[i + 2 * kThreads]);
    m3 = fmaxf(m3, pm[i + 3 * kThreads]);
  }
  for (; i < n; i += kThreads) m0 = fmaxf(m0, pm[i]);
  return fmaxf(fmaxf(m0, m1), fmaxf(m2, m3));
}

// The disparity map as a range-checked buffer: a load at a byte offset at or
// past the map's end (negative offsets included, as unsigned) returns 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t map_rsrc(const float* base, long long n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)(n * 4), 0x00020000);
}
// Disparity of a lane's column, rows 0..N-1 from the map row Yt: clamped to
// the bound, 0 outside the image.  `ok` false (the lane's column is outside
// the image or idle) gives every row an offset past the map's end; rows
// above or below the image have offsets before its start or past its end.
template <int N>
__device__ __forceinline__ void load_column(const Geom& g, const float* disp, int Yt, int X, bool ok,
                                            float (&om)[N]) {
  const __amdgpu_buffer_rsrc_t rs = map_rsrc(disp, g.p);
  const int base = ok ? (Yt * g.W + X) * 4 : (int)0x80000000;
#pragma unroll
  for (int r = 0; r < N; ++r) {
    const float v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, base + r * g.W * 4, 0, 0));
    om[r] = __builtin_amdgcn_fmed3f(v, -g.disp_bound, g.disp_bound);
  }
}
template <typename T>
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, unsigned off) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
  } else {
    const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
    return (float)__builtin_bit_cast(T, b);
  }
}
template <typename T>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned off, T v) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)off, 0, 0);
  }
}

// Stage a rows x cols tile, element (r, c) = src[(Y0 + r) * W + X0 + c] (zero
// outside [0,H) x [0,W)), into dst[r * ld + c].  Every thread issues a batch
// of loads (clamped, always in-bounds addresses) before any LDS store, so the
// global-memory latency is paid once per batch rather than once per element.
template <typename TS, int BATCH = 8, int NT = kThreads>
__device__ __forceinline__ void stage_tile(float* __restrict__ dst, int ld, const TS* __restrict__ src, int H, int W,
                                           int Y0, int X0, int rows, int cols) {
  const int n = rows * cols;
  const float inv = 1.f / (float)cols;  // (e + 1/2)/cols in float floors exactly for e < 2^16, cols < 400
  for (int base = threadIdx.x; base < n; base += NT * BATCH) {
    float v[BATCH];
    int off[BATCH];
#pragma unroll
    for (int j = 0; j < BATCH; ++j) {
      const int e = base + j * NT;
      const int r = (int)(((float)e + 0.5f) * inv), c = e - r * cols;
      const int Y = Y0 + r, X = X0 + c;
      const bool ok = e < n && Y >= 0 && Y < H && X >= 0 && X < W;
      const int Yc = min(max(Y, 0), H - 1), Xc = min(max(X, 0), W - 1);
      const float t = (float)src[(size_t)Yc * W + Xc];
      v[j] = ok ? t : 0.f;
      off[j] = e < n ? r * ld + c : -1;
    }
#pragma unroll
    for (int j = 0; j < BATCH; ++j)
      if (off[j] >= 0) dst[off[j]] = v[j];
  }
}

// Sum of the per-tile adjoint partial images that cover HR pixel (Y, X).
__device__ __forceinline__ float adj_merge(const Geom& g, const float* __restrict__ adj, int Y, int X) {
  // (Y + 1/2) / a_th in float: the quotient is at least 1/(2 a_th) away from
  // an integer and the rounding error is far below that for Y < 2^22
  const int ty = (int)(((float)Y + 0.5f) * g.a_inv_th), tx = (int)(((float)X + 0.5f) * g.a_inv_tw);
  const int ly = Y - ty * g.a_th, lx = X - tx * g.a_tw;
  const size_t tile = (size_t)g.a_ey * g.a_ex;
  const size_t grp = (size_t)g.a_nty * g.a_ntx * tile;
  float s = 0.f;
  for (int z = 0; z < g.a_vg; ++z) {
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
        s += adj[z * grp + ((size_t)tty * g.a_ntx + ttx) * tile + (size_t)ey * g.a_ex + ex];
      }
    }
  }
  return s;
}

// ---------------------------------------------------------------------------
// Forward operator t_k = D B W_k src for every view (sec 3.1, 4.1).
// WZD = true fuses the data-block z/w-steps of Algorithm 1: r = t - y,
// w_D' = clip(lambda1 r + w_D, +-1/vartheta) (= u - prox(u)), and the input of
// A^T, e = lambda2 r + (vartheta/2) lambda1 (2 w_D' - w_D), written to `out`;
// per-block partials {sum|r|, sum r^2, sum (w_D'-w_D)^2} go to `part`.
// grid = (ceil(sx/f_tlx), ceil(sy/f_tly), ceil(sk/f_vpb)).
// TS is the element type of `src`, TO that of `out` and `wD` (float, or a
// 16-bit storage type: values are rounded once, at the store; all arithmetic
// is FP32).  `pmax` receives per-block max |out| of the stored values.
template <bool WZD, int KBT, typename TS, typename TO>  // KBT: compile-time blur size (0: runtime g.kb)
__global__ __launch_bounds__(kThreads) void k_forward(Geom g, const TS* __restrict__ src,
                                                      const float* __restrict__ disp, TO* __restrict__ out,
                                                      const float* __restrict__ y, TO* __restrict__ wD,
                                                      double* __restrict__ part, float* __restrict__ pmax,
                                                      const DevScalars* __restrict__ sc, int gate) {
  if (gated(sc, g, gate)) return;
  extern __shared__ float smem[];
  const int zeta = g.zeta, rb = g.rb, h = g.halo;
  const int kb = KBT > 0 ? KBT : g.kb;
  const int tly = g.f_tly, tlx = g.f_tlx;
  const int NY = (tly - 1) * zeta + 1 + 2 * rb;
  const int NX = (tlx - 1) * zeta + 1 + 2 * rb;
  const int SY = NY + 2 * h, SX = NX + 2 * h;
  const int NPOS = NY * NX, NH = NY * tlx;
  float* xs = smem;          // [SY][SX] source tile, zero outside the image
  float* wv = xs + SY * SX;  // [NY][NX] warped values of the current view
  float* hb = wv + NPOS;     // [NY][tlx] horizontal blur at lattice columns
  float* t2 = hb + NH;       // [kb][kb] explicit blur kernel (g.blur2d)
  if (g.blur2d)
    for (int i = threadIdx.x; i < kb * kb; i += kThreads) t2[i] = g.taps2d[i];
  const int i0 = blockIdx.y * tly, j0 = blockIdx.x * tlx;
  const int Yp0 = i0 * zeta - rb, Xp0 = j0 * zeta - rb;
  const int tid = threadIdx.x;

  stage_tile(xs, SX, src, g.H, g.W, Yp0 - h, Xp0 - h, SY, SX);
  // (idx + 1/2) / n in float: exact floor division for idx < 2^22
  const float invNX = 1.f / (float)NX, invTLX = 1.f / (float)tlx;
  // Blur positions of this thread: disparity clamped to +-disp_bound (which
  // keeps every gather inside the tile) and 0 outside the image, where the
  // zero tile makes the sample vanish as the zero padding of B requires.
  float om[kFwdSlots];
  int base[kFwdSlots];
  int rbase[kFwdSlots];   // base + row offset of the current angular row
  float fyv[kFwdSlots];   // vertical bilinear weight of the current angular row
  int pofs[kFwdSlots];    // pixel offset in a map, -1 outside the image
  const bool per_view = g.n_disp > 1;  // view k's own map ([k][H][W]), loaded per view
  {
#pragma unroll
    for (int s = 0; s < kFwdSlots; ++s) {  // all loads first (in-bounds addresses), then the math
      const int idx = tid + s * kThreads;
      const int py = (int)(((float)idx + 0.5f) * invNX), px = idx - py * NX;
      const int Y = Yp0 + py, X = Xp0 + px;
      const bool in = idx < NPOS && Y >= 0 && Y < g.H && X >= 0 && X < g.W;
      pofs[s] = in ? Y * g.W + X : -1;
      om[s] = disp[in ? (size_t)Y * g.W + X : 0];
      base[s] = idx < NPOS ? (py + h) * SX + (px + h) : 0;
    }
#pragma unroll
    for (int s = 0; s < kFwdSlots; ++s)
      om[s] = pofs[s] >= 0 ? fminf(fmaxf(om[s], -g.disp_bound), g.disp_bound) : 0.f;
  }
  int hoff[kFwdHSlots];
#pragma unroll
  for (int s = 0; s < kFwdHSlots; ++s) {
    const int idx = tid + s * kThreads;
    const int py = (int)(((float)idx + 0.5f) * invTLX), j = idx - py * tlx;
    hoff[s] = idx < NH ? py * NX + j * zeta : 0;
  }
  const int li = (int)(((float)tid + 0.5f) * invTLX), lj = tid - li * tlx;
  const int oi = i0 + li, oj = j0 + lj;
  const bool vout = tid < tly * tlx && oi < g.sy && oj < g.sx;
  const int voff = li * zeta * tlx + lj;
  __syncthreads();

  const int k0 = blockIdx.z * g.f_vpb;
  const int k1 = min(g.sk, k0 + g.f_vpb);
  double s_abs = 0.0, s_sq = 0.0, s_dw = 0.0;
  float vmax = 0.f;
  for (int k = k0; k < k1; ++k) {
    const int ka = k / g.V, kc = k - ka * g.V;
    const float rho = (float)(kc - (g.V - 1) / 2);
    if (per_view) {
      const float* dk = disp + (size_t)k * g.p;
#pragma unroll
      for (int s = 0; s < kFwdSlots; ++s) om[s] = dk[pofs[s] >= 0 ? pofs[s] : 0];
#pragma unroll
      for (int s = 0; s < kFwdSlots; ++s)
        om[s] = pofs[s] >= 0 ? fminf(fmaxf(om[s], -g.disp_bound), g.disp_bound) : 0.f;
    }
    if (k == k0 || kc == 0 || per_view) {  // one map: the vertical warp coordinate is shared by an angular row
      const float tau = (float)(ka - (g.U - 1) / 2);
#pragma unroll
      for (int s = 0; s < kFwdSlots; ++s) {
        const float sy = tau * om[s];
        const float fy0 = floorf(sy);
        fyv[s] = sy - fy0;
        rbase[s] = base[s] + (int)fy0 * SX;
      }
    }
    const size_t o = (size_t)k * g.q + (size_t)oi * g.sx + oj;
    float yv = 0.f, w0 = 0.f;
    if (WZD && vout) {  // issued early; consumed after the two LDS passes
      yv = y[o];
      w0 = (float)wD[o];
    }
    // W_k at every blur position of this thread: all gathers, then all stores
    float val[kFwdSlots];
#pragma unroll
    for (int s = 0; s < kFwdSlots; ++s) {
      const float sx = rho * om[s];
      const float fx0 = floorf(sx);
      const float fx = sx - fx0;
      const int off = rbase[s] + (int)fx0;
      const float a = xs[off], b = xs[off + 1], c = xs[off + SX], d = xs[off + SX + 1];
      const float top = fmaf(fx, b - a, a);
      const float bot = fmaf(fx, d - c, c);
      val[s] = fmaf(fyv[s], bot - top, top);
    }
#pragma unroll
    for (int s = 0; s < kFwdSlots; ++s) {
      const int idx = tid + s * kThreads;
      if (idx < NPOS) wv[idx] = val[s];
    }
    __syncthreads();
    float t = 0.f;
    if (g.blur2d) {
      // explicit kernel: the 2-D correlation at the lattice point, from the warped values
      if (vout) {
        const float* wp = wv + li * zeta * NX + lj * zeta;
        for (int a = 0; a < kb; ++a)
          for (int b = 0; b < kb; ++b) t = fmaf(t2[a * kb + b], wp[a * NX + b], t);
      }
      __syncthreads();  // reads of wv precede the next view's stores
    } else {
    // B, horizontal pass, only at the lattice columns D keeps
    float hsum[kFwdHSlots];
#pragma unroll
    for (int s = 0; s < kFwdHSlots; ++s) hsum[s] = 0.f;
#pragma unroll
    for (int b = 0; b < (KBT > 0 ? KBT : kMaxTaps); ++b) {
      if (KBT == 0 && b >= kb) break;
      const float gb = g.g[b];
#pragma unroll
      for (int s = 0; s < kFwdHSlots; ++s) hsum[s] = fmaf(gb, wv[hoff[s] + b], hsum[s]);
    }
#pragma unroll
    for (int s = 0; s < kFwdHSlots; ++s) {
      const int idx = tid + s * kThreads;
      if (idx < NH) hb[idx] = hsum[s];
    }
    __syncthreads();
    // B, vertical pass, only at the lattice rows
    if (vout) {
#pragma unroll
      for (int a = 0; a < (KBT > 0 ? KBT : kMaxTaps); ++a) {
        if (KBT == 0 && a >= kb) break;
        t = fmaf(g.g[a], hb[voff + a * tlx], t);
      }
    }
    }
    // the fused epilogue
    if (vout) {
      if constexpr (!WZD) {
        const TO ts = (TO)t;
        out[o] = ts;
        vmax = fmaxf(vmax, fabsf((float)ts));
      } else {
        const float r = t - yv;
        const float wn = clipf(fmaf(g.lambda1, r, w0), g.clip);
        const float e = g.lambda2 * r + g.half_theta * g.lambda1 * (2.f * wn - w0);
        const TO es = (TO)e;
        out[o] = es;
        vmax = fmaxf(vmax, fabsf((float)es));
        wD[o] = (TO)wn;
        const double rd = (double)r, dw = (double)wn - (double)w0;
        s_abs += fabs(rd);
        s_sq += rd * rd;
        s_dw += dw * dw;
      }
    }
  }
  const unsigned bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, off, 64));
    __shared__ float sm[4];
    if ((tid & 63) == 0) sm[tid >> 6] = vmax;
    __syncthreads();
    if (tid == 0) pmax[bid] = fmaxf(fmaxf(sm[0], sm[1]), fmaxf(sm[2], sm[3]));
  }
  if constexpr (WZD) {
    double v[3] = {s_abs, s_sq, s_dw};
    block_sum<3>(v);
    if (tid == 0) {
      part[(size_t)bid * 3 + 0] = v[0];
      part[(size_t)bid * 3 + 1] = v[1];
      part[(size_t)bid * 3 + 2] = v[2];
    }
  }
}

// ---------------------------------------------------------------------------
// Forward operator, column-per-lane form (same result as k_forward, same
// fused wz-step epilogue).  A block stages the HR source tile of one LR tile
// (TLY x f_tlx lattice points) once; each of its NW waves (eight over quad
// cells, four over the plain tile) then takes whole views (k0 + wave,
// k0 + wave + NW, ...), so the view loop has no block barrier.  Lane px owns column px of the blur positions (NX <= 64): it walks
// the NY positions of its column, warps each one by a bilinear gather from
// the staged tile and feeds it straight into the vertical blur at the lattice
// rows, held in registers; the wave then applies the horizontal blur at the
// lattice columns from a wave-private LDS row buffer.  ZETA, KB and TLY are
// compile-time so that the position walk and the tap selection unroll.
// grid = (ceil(sx/f_tlx), ceil(sy/TLY), ceil(sk/f_vpb)).
// The position walk of k_fwdcol: warp every blur position of the lane's
// column and accumulate the vertical blur at the TLY lattice rows.  The tile
// pitch is the compile-time kColPitch: a tap address is one float FMA (exact
// on these small integers) and one conversion away from the warp's floors,
// and the four taps are two paired LDS reads at immediate offsets.
template <int NY, int TLY, int ZETA, int KB>
__device__ __forceinline__ void fwd_walk(const Geom& g, const float* __restrict__ xs, const float (&om)[NY],
                                         int cbase, float tau, float rho, float (&acc)[TLY]) {
#pragma unroll
  for (int i = 0; i < TLY; ++i) acc[i] = 0.f;
  const float* xc = xs + cbase;
#pragma unroll
  for (int py = 0; py < NY; ++py) {
    const float sy = tau * om[py], sx = rho * om[py];
    const float fy0 = floorf(sy), fx0 = floorf(sx);
    const float fy = sy - fy0, fx = sx - fx0;
    // tile cell of tap (0, 0), relative to (row 0, lane column): exact in float
    const int rel = (int)fmaf(fy0 + (float)py, (float)kColPitch, fx0);
    const float* q = xc + rel;
    const float a = q[0], b = q[1], c = q[kColPitch], d = q[kColPitch + 1];
    const float top = fmaf(fx, b - a, a), bot = fmaf(fx, d - c, c);
    const float val = fmaf(fy, bot - top, top);
    // the lattice rows i this position reaches: 0 <= py - i ZETA < KB
#pragma unroll
    for (int j = 0; j < (KB + ZETA - 1) / ZETA; ++j) {
      const int i = py / ZETA - j;
      const int t = py - i * ZETA;  // compile-time after unrolling
      if (i >= 0 && i < TLY && t < KB) acc[i] = fmaf(g.g[t], val, acc[i]);
    }
  }
}

// The position walk over quad cells: cell (r, c) of the staged tile holds
// (v, v[c+1] - v, v[r+1] - v, v[r+1][c+1] - v[r+1] - v[c+1] + v), so the
// bilinear sample at fraction (fy, fx) is v + fx dh + fy (dv + fx dhv): three
// FMAs after one 16-byte LDS read.  The cell's byte address is one float FMA
// and one conversion (a cell offset, exact on these small integers) and one
// shift-add: from the row base of position py held in registers (RB, rowb),
// else from the tile cell of (row 0, this column) with py added in float.
template <int NY, int TLY, int ZETA, int KB, bool RB>
__device__ __forceinline__ void fwd_walk_q(const Geom& g, const float4* __restrict__ qs, const float (&om)[NY],
                                           const int (&rowb)[RB ? NY : 1], int cb16, float sxf, float tau,
                                           float rho, float (&acc)[TLY]) {
#pragma unroll
  for (int i = 0; i < TLY; ++i) acc[i] = 0.f;
  const char* qb = reinterpret_cast<const char*>(qs);
#pragma unroll
  for (int py = 0; py < NY; ++py) {
    const float sy = tau * om[py], sx = rho * om[py];
    const float fy0 = floorf(sy), fx0 = floorf(sx);
    const float fy = sy - fy0, fx = sx - fx0;
    float4 c;
    if constexpr (RB) {
      const int rel = (int)fmaf(fy0, sxf, fx0);  // cell offset from the row base: exact on these small integers
      c = *reinterpret_cast<const float4*>(qb + (rel * 16 + rowb[RB ? py : 0]));
    } else {
      const int rel = (int)fmaf(fy0 + (float)py, sxf, fx0);  // from (row 0, this column): exact
      c = *reinterpret_cast<const float4*>(qb + (rel * 16 + cb16));
    }
    const float val = fmaf(fy, fmaf(fx, c.w, c.z), fmaf(fx, c.y, c.x));
#pragma unroll
    for (int j = 0; j < (KB + ZETA - 1) / ZETA; ++j) {
      const int i = py / ZETA - j;
      const int t = py - i * ZETA;
      if (i >= 0 && i < TLY && t < KB) acc[i] = fmaf(g.g[t], val, acc[i]);
    }
  }
}

// Mirror orbits of an odd angular grid.  With one disparity map, view
// (tau, rho) samples x at (tau w, rho w) from each position (sec 4.1), so the
// views (+-tau, +-rho) share |tau| w and |rho| w: for s = a - floor(a) > 0,
// floor(-a) = -floor(a) - 1 and -a - floor(-a) = 1 - s, and for an integer a
// the same two values select the cell row below with weight 1, the same
// sample.  An orbit walk computes the floors and fractions once per position
// for all its views.  Kinds: four views (tau, rho > 0), two on the centre
// column (rho = 0), two on the centre row (tau = 0), the centre view.
enum : int { kOrbQuad = 0, kOrbCol = 1, kOrbRow = 2, kOrbCentre = 3 };
__host__ __device__ constexpr int orb_nv(int kind) { return kind == kOrbQuad ? 4 : kind == kOrbCentre ? 1 : 2; }
// member m of an orbit: 1 where its tau (orb_my) or rho (orb_mx) is negated
__host__ __device__ constexpr int orb_my(int kind, int m) { return kind == kOrbQuad ? m >> 1 : kind == kOrbCol ? m : 0; }
__host__ __device__ constexpr int orb_mx(int kind, int m) { return kind == kOrbQuad ? m & 1 : kind == kOrbRow ? m : 0; }

// The position walk of one orbit over quad cells (ta = |tau|, ra = |rho|):
// acc[m] receives the vertical blur of member m's samples, the samples
// fwd_walk_q takes for that view alone (a mirrored member's weights 1 - s and
// its cell sums round differently in the last bit).  Cell addresses are taken
// from (row 0, this column), the row added in float.
template <int NY, int TLY, int ZETA, int KB, int KIND>
__device__ __forceinline__ void fwd_walk_orb(const Geom& g, const float4* __restrict__ qs, const float (&om)[NY],
                                             int cb16, int sx16, float sxf, float ta, float ra,
                                             float (&acc)[orb_nv(KIND)][TLY]) {
  constexpr int NV = orb_nv(KIND);
  constexpr bool HY = KIND == kOrbQuad || KIND == kOrbCol, HX = KIND == kOrbQuad || KIND == kOrbRow;
#pragma unroll
  for (int m = 0; m < NV; ++m)
#pragma unroll
    for (int i = 0; i < TLY; ++i) acc[m][i] = 0.f;
  const char* qb = reinterpret_cast<const char*>(qs);
#pragma unroll
  for (int py = 0; py < NY; ++py) {
    // [0]: the positive member, [1]: the mirrored one; fyr = cell row
    // relative to row 0 of the column, fxc = cell column offset
    float fy[2] = {0.f, 0.f}, fyr[2] = {(float)py, (float)py}, fx[2] = {0.f, 0.f}, fxc[2] = {0.f, 0.f};
    if constexpr (HY) {
      const float s = ta * om[py], f0 = floorf(s), f = s - f0;
      fy[0] = f;
      fyr[0] = f0 + (float)py;
      fy[1] = 1.f - f;
      fyr[1] = (float)(py - 1) - f0;
    }
    if constexpr (HX) {
      const float s = ra * om[py], f0 = floorf(s), f = s - f0;
      fx[0] = f;
      fxc[0] = f0;
      fx[1] = 1.f - f;
      fxc[1] = -1.f - f0;
    }
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const int iy = orb_my(KIND, m), ix = orb_mx(KIND, m);
      // cell offset from (row 0, this column): exact on these small integers
      const int rel = KIND == kOrbCentre ? 0 : HX ? (int)fmaf(fyr[iy], sxf, fxc[ix]) : (int)(fyr[iy] * sxf);
      float4 c = *reinterpret_cast<const float4*>(
          qb + (KIND == kOrbCentre ? cb16 + py * sx16 : rel * 16 + cb16));
      // whole 16-byte cells also where a kind uses part of one: lanes read
      // consecutive cells, so the 16-byte form is free of bank conflicts
      // while one or two words per lane at a 16-byte stride are not
      if constexpr (!(HY && HX)) asm volatile("" : "+v"(c.x), "+v"(c.y), "+v"(c.z), "+v"(c.w));
      float val;
      if constexpr (KIND == kOrbCentre) val = c.x;  // no warp: the cell's own value
      else if constexpr (HY && HX) val = fmaf(fy[iy], fmaf(fx[ix], c.w, c.z), fmaf(fx[ix], c.y, c.x));
      else if constexpr (HY) val = fmaf(fy[iy], c.z, c.x);
      else val = fmaf(fx[ix], c.y, c.x);
#pragma unroll
      for (int j = 0; j < (KB + ZETA - 1) / ZETA; ++j) {
        const int i = py / ZETA - j;
        const int t = py - i * ZETA;
        if (i >= 0 && i < TLY && t < KB) acc[m][i] = fmaf(g.g[t], val, acc[m][i]);
      }
    }
  }
  // keep the accumulation here: the caller reads acc only under a lane
  // condition, and sinking the FMA chains into that branch would hold every
  // position's loaded cells live across the walk
#pragma unroll
  for (int m = 0; m < NV; ++m)
#pragma unroll
    for (int i = 0; i < TLY; ++i) asm volatile("" : "+v"(acc[m][i]));
}

// QUAD: eight waves per block share a tile of quad cells (fwd_walk_q);
// otherwise four waves share a plain tile at pitch kColPitch.  The second
// launch bound is a minimum of waves per SIMD: 4 caps VGPRs at 128 (two
// quad blocks or four plain blocks per CU).  The FP32 quad kernels fit 128
// without the cap (one shape reaches 134 and keeps three waves per SIMD) and
// schedule better without it: with it the wz-step spills in its view loop.
// The 16-bit variants need the cap to stay at 128.
// ORB (CG form over quad cells, one disparity map, odd grid): the waves take
// mirror orbits instead of single views (fwd_walk_orb); the block's range of
// orbit items is its share of the gridDim.z groups.
template <bool WZD, int ZETA, int KB, int TLY, typename TS, typename TO, bool QUAD, bool PV, bool ORB = false>
__global__ __launch_bounds__(QUAD ? 2 * kThreads : kThreads,
                             (QUAD && sizeof(TS) == 4 && sizeof(TO) == 4) ? 2 : 4) void k_fwdcol(Geom g, const TS* __restrict__ src,
                                                     const float* __restrict__ disp, TO* __restrict__ out,
                                                     const float* __restrict__ y, TO* __restrict__ wD,
                                                     double* __restrict__ part, float* __restrict__ pmax,
                                                     const DevScalars* __restrict__ sc, int gate) {
  static_assert(!ORB || (QUAD && !WZD && !PV), "orbit walk: CG form over quad cells with one disparity map");
  if (gated(sc, g, gate)) return;
  constexpr int RB = KB / 2;
  constexpr int NY = (TLY - 1) * ZETA + KB;
  constexpr int NO = (TLY * ((64 - KB) / ZETA + 1) + 63) / 64;  // outputs per lane and view
  constexpr int NW = QUAD ? 8 : 4;                                // waves per block
  extern __shared__ float4 smem_q[];
  float* smem = reinterpret_cast<float*>(smem_q);
  const int h = g.halo, tlx = g.f_tlx;
  const int NX = (tlx - 1) * ZETA + KB;
  const int SY = NY + 2 * h, SX = NX + 2 * h;  // plain tile: SX <= kColPitch
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int TW4 = QUAD ? 4 * SY * SX : SY * kColPitch;  // floats of the source tile
  float* xs = smem;                                      // plain: [SY][kColPitch], zero outside the image
  const float4* qs = smem_q;                             // quad: [SY][SX] cells
  float* vb = smem + TW4 + wave * (TLY * NX);            // wave-private [TLY][NX] vertical-blur rows
  int bx, by, bz;
  xcd_block3(bx, by, bz);
  const int i0 = by * TLY, j0 = bx * tlx;
  const int Yp0 = i0 * ZETA - RB, Xp0 = j0 * ZETA - RB;
  if constexpr (QUAD) {
    // cells from the source (zero outside the image); each cell reads its
    // 2 x 2 neighbourhood, so the tile's last row and column hold cells no
    // sample reaches (the walk's taps stay within rows/columns <= SY-2, SX-2)
    const int n = SY * SX;
    const float inv = 1.f / (float)SX;
    for (int base = tid; base < n; base += NW * 64 * 2) {
      float v[2][4];
      int off[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int e = base + j * NW * 64;
        const int r = (int)(((float)e + 0.5f) * inv), c = e - r * SX;
        const int Y = Yp0 - h + r, X = Xp0 - h + c;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int Yq = Y + (q >> 1), Xq = X + (q & 1);
          const bool ok = e < n && Yq >= 0 && Yq < g.H && Xq >= 0 && Xq < g.W;
          const float t = (float)src[ok ? (size_t)Yq * g.W + Xq : 0];
          v[j][q] = ok ? t : 0.f;
        }
        off[j] = e < n ? e : -1;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j)
        if (off[j] >= 0)
          smem_q[off[j]] = make_float4(v[j][0], v[j][1] - v[j][0], v[j][2] - v[j][0],
                                       (v[j][3] - v[j][2]) - (v[j][1] - v[j][0]));
    }
  } else {
    stage_tile(xs, kColPitch, src, g.H, g.W, Yp0 - h, Xp0 - h, SY, SX);
  }

  // this lane's column of blur positions: clamped disparity, 0 outside the
  // image (the zero tile then makes the sample vanish, as B's zero padding
  // requires); lanes beyond NX address column 0 and discard their results
  const bool colok = lane < NX;
  const int px = colok ? lane : 0;
  const int X = Xp0 + px;
  // PV: one map per view ([k][H][W]), the column reloaded at each view
  const bool colin = colok && X >= 0 && X < g.W;
  float om[NY];
  if constexpr (!PV) load_column<NY>(g, disp, Yp0, X, colin, om);
  const int cbase = h * (QUAD ? SX : kColPitch) + px + h;  // tile cell of (row 0, this column)
  // quad walk: byte row bases of the positions, in registers for the CG form
  // (the wz-step form keeps its registers for the epilogue's loads)
  constexpr bool RBR = QUAD && !WZD && !ORB && NY <= 32;
  const int cb16 = cbase * 16;
  int rowb[RBR ? NY : 1];
  rowb[0] = cb16;
  if constexpr (RBR) {
#pragma unroll
    for (int py = 1; py < NY; ++py) rowb[py] = cb16 + py * SX * 16;
  }
  // outputs of this lane: lattice point (oi, oj) of the tile, slot s
  const float invT = 1.f / (float)tlx;
  int orow[NO], ocol[NO];
  bool oval[NO];
  size_t oofs[NO];
#pragma unroll
  for (int s = 0; s < NO; ++s) {
    const int idx = lane + 64 * s;
    const int a = (int)(((float)idx + 0.5f) * invT), b = idx - a * tlx;
    orow[s] = a;
    ocol[s] = b;
    oval[s] = idx < TLY * tlx && i0 + a < g.sy && j0 + b < g.sx;
    oofs[s] = oval[s] ? (size_t)(i0 + a) * g.sx + (j0 + b) : 0;
  }
  __syncthreads();

  double s_abs = 0.0, s_sq = 0.0, s_dw = 0.0;
  float vmax = 0.f;
  const int k0 = bz * g.f_vpb;
  const int k1 = min(g.sk, k0 + g.f_vpb);
  // horizontal blur at the lattice columns and the epilogue of one view
  auto finish = [&](const float (&acc)[TLY], int k, const float (&yv)[NO], const float (&w0)[NO])
                    __attribute__((always_inline)) {
    const size_t vo = (size_t)k * g.q;
    if (colok) {
#pragma unroll
      for (int i = 0; i < TLY; ++i) vb[i * NX + px] = acc[i];
    }
    __builtin_amdgcn_wave_barrier();  // the wave's LDS writes precede its reads below
    float f_abs = 0.f, f_sq = 0.f, f_dw = 0.f;  // this view's NO outputs in FP32, then the FP64 totals
#pragma unroll
    for (int s = 0; s < NO; ++s) {
      if (!oval[s]) continue;
      const float* rowp = vb + orow[s] * NX + ocol[s] * ZETA;
      float t = 0.f;
#pragma unroll
      for (int b = 0; b < KB; ++b) t = fmaf(g.g[b], rowp[b], t);
      const size_t o = vo + oofs[s];
      if constexpr (!WZD) {
        const TO ts = (TO)t;
        out[o] = ts;
        vmax = fmaxf(vmax, fabsf((float)ts));
      } else {
        const float r = t - yv[s];
        const float wn = clipf(fmaf(g.lambda1, r, w0[s]), g.clip);
        const float e = g.lambda2 * r + g.half_theta * g.lambda1 * (2.f * wn - w0[s]);
        const TO es = (TO)e;
        out[o] = es;
        vmax = fmaxf(vmax, fabsf((float)es));
        wD[o] = (TO)wn;
        const float dw = wn - w0[s];
        f_abs += fabsf(r);
        f_sq = fmaf(r, r, f_sq);
        f_dw = fmaf(dw, dw, f_dw);
      }
    }
    if constexpr (WZD) {
      s_abs += (double)f_abs;
      s_sq += (double)f_sq;
      s_dw += (double)f_dw;
    }
    __builtin_amdgcn_wave_barrier();  // reads of vb complete before it is written again
  };
  auto load_wzd = [&](int k, float (&yv)[NO], float (&w0)[NO]) __attribute__((always_inline)) {
    if constexpr (WZD) {  // issued early; consumed after the position walk
      const size_t vo = (size_t)k * g.q;
#pragma unroll
      for (int s = 0; s < NO; ++s) {
        yv[s] = y[vo + oofs[s]];
        w0[s] = (float)wD[vo + oofs[s]];
      }
    }
  };
  if constexpr (ORB) {
    // orbit items: hy hx quads, hy centre-column pairs, hx centre-row pairs,
    // the centre view; the block takes items [it0, it1) round-robin over its
    // waves (k0, k1 above are unused)
    const int ca = (g.U - 1) / 2, cc = (g.V - 1) / 2, nq = ca * cc, nit = nq + ca + cc + 1;
    const int ipb = (nit + (int)gridDim.z - 1) / (int)gridDim.z;
    const int it1 = min(nit, bz * ipb + ipb);
    const float yd[NO] = {}, wd[NO] = {};  // the CG form has no epilogue inputs
    const int sx16 = SX * 16;
    const float sxf = (float)SX;
    int it = bz * ipb + wave;
    for (; it < it1 && it < nq; it += NW) {
      const int a = it / cc, ta = 1 + a, ra = 1 + it - a * cc;
      float acc[4][TLY];
      fwd_walk_orb<NY, TLY, ZETA, KB, kOrbQuad>(g, qs, om, cb16, sx16, sxf, (float)ta, (float)ra, acc);
      finish(acc[0], (ca + ta) * g.V + (cc + ra), yd, wd);
      finish(acc[1], (ca + ta) * g.V + (cc - ra), yd, wd);
      finish(acc[2], (ca - ta) * g.V + (cc + ra), yd, wd);
      finish(acc[3], (ca - ta) * g.V + (cc - ra), yd, wd);
    }
    for (; it < it1 && it < nq + ca; it += NW) {
      const int ta = 1 + it - nq;
      float acc[2][TLY];
      fwd_walk_orb<NY, TLY, ZETA, KB, kOrbCol>(g, qs, om, cb16, sx16, sxf, (float)ta, 0.f, acc);
      finish(acc[0], (ca + ta) * g.V + cc, yd, wd);
      finish(acc[1], (ca - ta) * g.V + cc, yd, wd);
    }
    for (; it < it1 && it < nq + ca + cc; it += NW) {
      const int ra = 1 + it - nq - ca;
      float acc[2][TLY];
      fwd_walk_orb<NY, TLY, ZETA, KB, kOrbRow>(g, qs, om, cb16, sx16, sxf, 0.f, (float)ra, acc);
      finish(acc[0], ca * g.V + (cc + ra), yd, wd);
      finish(acc[1], ca * g.V + (cc - ra), yd, wd);
    }
    if (it < it1) {
      float acc[1][TLY];
      fwd_walk_orb<NY, TLY, ZETA, KB, kOrbCentre>(g, qs, om, cb16, sx16, sxf, 0.f, 0.f, acc);
      finish(acc[0], ca * g.V + cc, yd, wd);
    }
  } else {
    for (int k = k0 + wave; k < k1; k += NW) {
      if constexpr (PV) load_column<NY>(g, disp + (size_t)k * g.p, Yp0, X, colin, om);
      const int ka = k / g.V, kc = k - ka * g.V;
      float yv[NO], w0[NO];
      load_wzd(k, yv, w0);
      const float tau = (float)(ka - (g.U - 1) / 2), rho = (float)(kc - (g.V - 1) / 2);
      float acc[TLY];
      if constexpr (QUAD) fwd_walk_q<NY, TLY, ZETA, KB, RBR>(g, qs, om, rowb, cb16, (float)SX, tau, rho, acc);
      else fwd_walk<NY, TLY, ZETA, KB>(g, xs, om, cbase, tau, rho, acc);
      finish(acc, k, yv, w0);
    }
  }
  const unsigned bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, off, 64));
    __shared__ float sm[NW];
    if (lane == 0) sm[wave] = vmax;
    __syncthreads();
    if (tid == 0) {
      float m = sm[0];
#pragma unroll
      for (int w = 1; w < NW; ++w) m = fmaxf(m, sm[w]);
      pmax[bid] = m;
    }
  }
  if constexpr (WZD) {
    double v[3] = {s_abs, s_sq, s_dw};
    block_sum<3, NW>(v);
    if (tid == 0) {
      part[(size_t)bid * 3 + 0] = v[0];
      part[(size_t)bid * 3 + 1] = v[1];
      part[(size_t)bid * 3 + 2] = v[2];
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint sum_k A_k^T lr_k = sum_k W_k^T B^T D^T lr_k into per-tile partial
// images [tile][a_ey][a_ex] (HR tile + warp halo).  grid = (a_ntx, a_nty).
//
// Each of the four waves owns a quarter of the tile's HR rows and walks all
// views on its own: it stages the LR rows its rows need in a wave-private LDS
// buffer (prefetched one view ahead), applies B^T D^T as a polyphase
// separable filter, and scatters W_k^T with the bilinear weights of W_k into
// the block's shared accumulator.  No block barrier is needed inside the view
// loop (LDS operations of one wave complete in order).
//
// The accumulator is 64-bit fixed point (ds_add_u64): LDS float atomics run
// ~30x slower than integer ones on this part, and integer addition is
// associative, so the sums are also bitwise reproducible.  Every contribution
// c = u * w has |c| <= M = max |lr| (the polyphase taps and the bilinear
// weights are non-negative and sum to at most 1), so with
// S = 2^(30 - ceil(log2 M)) each c * S truncates to an int32 without
// saturation (resolution 2^-29 M per contribution) and at most
// sk*(2 halo + 1)^2 contributions per cell stay far below 2^63.  M comes from
// the producer's per-block maxima (`pmax`, npmax of them).
// TI is the element type of `lr` (float or a 16-bit storage type).
template <int MMT, typename TI>  // MMT: compile-time taps per polyphase phase, exactly (2 rb)/zeta + 1 (0: runtime)
__global__ __launch_bounds__(kThreads) void k_adjoint(Geom g, const TI* __restrict__ lr,
                                                      const float* __restrict__ disp, float* __restrict__ outp,
                                                      const float* __restrict__ pmax, int npmax,
                                                      const DevScalars* __restrict__ sc, int gate) {
  if (gated(sc, g, gate)) return;
  extern __shared__ long long smem8[];  // 8-byte aligned: the accumulator comes first
  float* smem = reinterpret_cast<float*>(smem8);
  const int zeta = g.zeta, rb = g.rb, h = g.halo, kb = g.kb;
  const int TH = g.a_th, TW = g.a_tw, EY = g.a_ey, EX = g.a_ex;
  const int RH = TH / 4;                           // HR rows per wave
  const int ci = (rb + zeta - 1) / zeta;           // LR rows/cols within blur reach
  const int LX = g.a_tlx + 2 * ci;
  const int RL = RH / zeta + 2 * ci;               // LR rows a wave stages
  const int MM = MMT > 0 ? MMT : (2 * rb) / zeta + 1;  // lattice points within +-rb
  const int PAD = zeta * MM;                       // zero taps below index 0 (indices reach 1 - zeta*MM)
  const int ETS = (RL + MM) * LX, HVS = RH * LX + MM;
  long long* acc = smem8;                          // [EY][EX] fixed-point accumulator
  float* gs = smem + 2 * EY * EX;                  // [PAD + kb] taps, zeros below
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  float* t2 = gs + PAD + kb + 4 * (ETS + HVS);     // [kb][kb] explicit blur kernel (g.blur2d)
  float* e_ = gs + PAD + kb + wave * (ETS + HVS);  // wave-private LR rows (zero-padded)
  if (g.blur2d)
    for (int i = tid; i < kb * kb; i += kThreads) t2[i] = g.taps2d[i];
  float* h_ = e_ + ETS;                            // wave-private vertical pass
  for (int idx = tid; idx < EY * EX; idx += kThreads) acc[idx] = 0;
  for (int idx = tid; idx < PAD + kb; idx += kThreads) gs[idx] = idx < PAD ? 0.f : g.g[idx - PAD];
  for (int idx = lane; idx < ETS + HVS; idx += 64) e_[idx] = 0.f;

  // fixed-point scale from the producer's block maxima (order-free, so exact)
  float mloc = max_parts(pmax, npmax);
  __shared__ float smax[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mloc = fmaxf(mloc, __shfl_xor(mloc, off, 64));
  if (lane == 0) smax[wave] = mloc;
  __syncthreads();
  const float M = fmaxf(fmaxf(smax[0], smax[1]), fmaxf(smax[2], smax[3]));
  int eM = 0;
  if (M > 0.f) (void)frexpf(M, &eM);               // M < 2^eM
  const int sexp = min(max(30 - eM, -120), 120);
  const float S = ldexpf(1.f, sexp), invS = ldexpf(1.f, -sexp);

  const int ty = blockIdx.y, tx = blockIdx.x;
  const int i0 = ty * g.a_tly, j0 = tx * g.a_tlx;
  const int Y0 = i0 * zeta, X0 = j0 * zeta;
  const int ly0 = wave * RH;                       // first HR row of this wave (tile-local)
  const int li0 = i0 + ly0 / zeta - ci;            // first LR row the wave stages
  const float invLX = 1.f / (float)LX, invTW = 1.f / (float)TW;  // (e + 1/2)/n floors exactly here

  // LR values this lane stages per view (offset within a view; -1 = zero)
  int eoff[kAdjESlots];
#pragma unroll
  for (int s = 0; s < kAdjESlots; ++s) {
    const int idx = lane + s * 64;
    const int a = (int)(((float)idx + 0.5f) * invLX), b = idx - a * LX;
    const int i = li0 + a, j = j0 - ci + b;
    eoff[s] = (idx < RL * LX && i >= 0 && i < g.sy && j >= 0 && j < g.sx) ? i * g.sx + j : -1;
  }
  // vertical outputs (wave row r, LR col b): LR rows i = Y div zeta + m for m in [m_lo, m_lo + MM)
  int vbase[kAdjVSlots], vtap[kAdjVSlots];
#pragma unroll
  for (int s = 0; s < kAdjVSlots; ++s) {
    const int idx = lane + s * 64;
    const int r = (int)(((float)idx + 0.5f) * invLX), b = idx - r * LX;
    const int ly = ly0 + r;
    const int ph = ly % zeta;
    const int mlo = floordiv(ph - rb + zeta - 1, zeta);
    // staged row of LR row (Y0 + ly) div zeta + mlo
    vbase[s] = idx < RH * LX ? ((Y0 + ly) / zeta + mlo - li0) * LX + b : 0;
    vtap[s] = PAD + ph - zeta * mlo + rb;
  }
  // scatter pixels (wave row r, col lx): disparity (clamped), horizontal base/tap, accumulator base
  float om[kAdjSlots];
  int hbase[kAdjSlots], htap[kAdjSlots], abase[kAdjSlots], dofs[kAdjSlots], ebase2[kAdjSlots], tapy[kAdjSlots],
      tapx[kAdjSlots];
  bool act[kAdjSlots];
  const bool per_view = g.n_disp > 1;  // view k's own map ([k][H][W]), loaded per view
#pragma unroll
  for (int s = 0; s < kAdjSlots; ++s) {
    const int idx = lane + s * 64;
    const int r = (int)(((float)idx + 0.5f) * invTW), lx = idx - r * TW;
    const int ly = ly0 + r;
    const int Y = Y0 + ly, X = X0 + lx;
    act[s] = idx < RH * TW && Y < g.H && X < g.W;
    dofs[s] = act[s] ? Y * g.W + X : 0;
    om[s] = disp[dofs[s]];  // batched, in bounds
    const int ph = lx % zeta, lq = lx / zeta;
    const int mlo = floordiv(ph - rb + zeta - 1, zeta);
    hbase[s] = act[s] ? r * LX + lq + mlo + ci : 0;
    htap[s] = PAD + ph - zeta * mlo + rb;
    abase[s] = (ly + h) * EX + (lx + h);
    if (g.blur2d) {  // explicit kernel: e_ row / tap row of the first lattice row in reach (the columns as above)
      const int phy = ly % zeta, mloy = floordiv(phy - rb + zeta - 1, zeta);
      ebase2[s] = act[s] ? ((Y0 + ly) / zeta + mloy - li0) * LX + lq + mlo + ci : 0;
      tapy[s] = phy - zeta * mloy + rb;  // kernel row / column of the first lattice point (may be out of range)
      tapx[s] = ph - zeta * mlo + rb;
    }
  }
#pragma unroll
  for (int s = 0; s < kAdjSlots; ++s) om[s] = act[s] ? fminf(fmaxf(om[s], -g.disp_bound), g.disp_bound) : 0.f;
  float ereg[kAdjESlots];
#pragma unroll
  for (int s = 0; s < kAdjESlots; ++s) {
    const float t = (float)lr[eoff[s] >= 0 ? eoff[s] : 0];
    ereg[s] = eoff[s] >= 0 ? t : 0.f;
  }
  __syncthreads();  // accumulator zeroed, taps ready
  // polyphase taps in registers; the horizontal ones carry the fixed-point scale S
  constexpr int RT = MMT > 0 ? MMT : 1;
  float vt[kAdjVSlots][RT], ht[kAdjSlots][RT];
  if constexpr (MMT > 0) {
#pragma unroll
    for (int s = 0; s < kAdjVSlots; ++s)
#pragma unroll
      for (int m = 0; m < MMT; ++m) vt[s][m] = gs[vtap[s] - zeta * m];
#pragma unroll
    for (int s = 0; s < kAdjSlots; ++s)
#pragma unroll
      for (int m = 0; m < MMT; ++m) ht[s][m] = gs[htap[s] - zeta * m] * S;
  }

  unsigned long long* accu = reinterpret_cast<unsigned long long*>(acc);
  // truncation to int32 (|c| <= 2^30 by the choice of S), sign-extended to 64 bits
  auto add_fixed = [&](int cell, float c) { atomicAdd(accu + cell, (unsigned long long)(long long)(int)c); };

  int rowoff[kAdjSlots];
  float wy0[kAdjSlots], wy1[kAdjSlots];
  for (int k = 0; k < g.sk; ++k) {
#pragma unroll
    for (int s = 0; s < kAdjESlots; ++s) {
      const int idx = lane + s * 64;
      if (idx < RL * LX) e_[idx] = ereg[s];
    }
    if (k + 1 < g.sk) {  // prefetch the next view's LR rows
      const TI* ln = lr + (size_t)(k + 1) * g.q;
#pragma unroll
      for (int s = 0; s < kAdjESlots; ++s) {
        const float t = (float)ln[eoff[s] >= 0 ? eoff[s] : 0];
        ereg[s] = eoff[s] >= 0 ? t : 0.f;
      }
    }
    // one map: the vertical warp coordinate is shared by the views of an angular row
    const int ka = k / g.V, kbcol = k - ka * g.V;
    if (per_view) {
      const float* dk = disp + (size_t)k * g.p;
#pragma unroll
      for (int s = 0; s < kAdjSlots; ++s) om[s] = dk[dofs[s]];
#pragma unroll
      for (int s = 0; s < kAdjSlots; ++s) om[s] = act[s] ? fminf(fmaxf(om[s], -g.disp_bound), g.disp_bound) : 0.f;
    }
    if (kbcol == 0 || per_view) {
      const float tau = (float)(ka - (g.U - 1) / 2);
#pragma unroll
      for (int s = 0; s < kAdjSlots; ++s) {
        const float sy = tau * om[s];
        const float fy0 = floorf(sy);
        wy1[s] = sy - fy0;
        wy0[s] = 1.f - wy1[s];
        rowoff[s] = (int)fy0 * EX;
      }
    }
    __builtin_amdgcn_wave_barrier();
    const float rho = (float)(kbcol - (g.V - 1) / 2);
    float uu[kAdjSlots];
    if (g.blur2d) {
      // explicit kernel: B^T D^T as the 2-D correlation with the taps mirrored,
      // over the lattice points within reach (scaled by S)
#pragma unroll
      for (int s = 0; s < kAdjSlots; ++s) {
        float u = 0.f;
        const int ay0 = tapy[s], bx0 = tapx[s];
        for (int my = 0; my < MM; ++my) {
          const int a = ay0 - zeta * my;
          if (a < 0 || a >= kb) continue;
          for (int mx = 0; mx < MM; ++mx) {
            const int b = bx0 - zeta * mx;
            if (b < 0 || b >= kb) continue;
            u = fmaf(t2[a * kb + b], e_[ebase2[s] + my * LX + mx], u);
          }
        }
        uu[s] = u * S;
      }
    } else {
    // B^T D^T, vertical
    float vv[kAdjVSlots];
#pragma unroll
    for (int s = 0; s < kAdjVSlots; ++s) vv[s] = 0.f;
    if constexpr (MMT > 0) {
#pragma unroll
      for (int m = 0; m < MMT; ++m) {
#pragma unroll
        for (int s = 0; s < kAdjVSlots; ++s) vv[s] = fmaf(vt[s][m], e_[vbase[s] + m * LX], vv[s]);
      }
    } else {
      for (int m = 0; m < MM; ++m) {
#pragma unroll
        for (int s = 0; s < kAdjVSlots; ++s) vv[s] = fmaf(gs[vtap[s] - zeta * m], e_[vbase[s] + m * LX], vv[s]);
      }
    }
#pragma unroll
    for (int s = 0; s < kAdjVSlots; ++s) {
      const int idx = lane + s * 64;
      if (idx < RH * LX) h_[idx] = vv[s];
    }
    __builtin_amdgcn_wave_barrier();
    // B^T D^T, horizontal (scaled by S)
#pragma unroll
    for (int s = 0; s < kAdjSlots; ++s) uu[s] = 0.f;
    if constexpr (MMT > 0) {
#pragma unroll
      for (int m = 0; m < MMT; ++m) {
#pragma unroll
        for (int s = 0; s < kAdjSlots; ++s) uu[s] = fmaf(ht[s][m], h_[hbase[s] + m], uu[s]);
      }
    } else {
      for (int m = 0; m < MM; ++m) {
#pragma unroll
        for (int s = 0; s < kAdjSlots; ++s) uu[s] = fmaf(gs[htap[s] - zeta * m] * S, h_[hbase[s] + m], uu[s]);
      }
    }
    }
    // then W_k^T: send u back to the four taps W_k read
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int s = 0; s < kAdjSlots; ++s) {
      if (!act[s]) continue;
      const float u = uu[s];
      const float sx = rho * om[s];
      const float fx0 = floorf(sx);
      const float fx = sx - fx0, gx = 1.f - fx;
      const int cell = abase[s] + rowoff[s] + (int)fx0;
      const float u0 = u * wy0[s], u1 = u * wy1[s];
      add_fixed(cell, u0 * gx);
      add_fixed(cell + 1, u0 * fx);
      add_fixed(cell + EX, u1 * gx);
      add_fixed(cell + EX + 1, u1 * fx);
    }
  }
  __syncthreads();
  float* o = outp + ((size_t)ty * g.a_ntx + tx) * (size_t)(EY * EX);
  for (int idx = tid; idx < EY * EX; idx += kThreads) o[idx] = (float)acc[idx] * invS;
}

// ---------------------------------------------------------------------------
// Adjoint, column-per-lane form (same operator as k_adjoint).  A block owns an
// HR tile of adjcol_th(ZETA) rows x adjcol_tw(ZETA) columns plus the warp
// halo, in a shared 32-bit fixed-point accumulator; its four waves take views
// k0 + wave, k0 + wave + 4, ... of the block's view group.  Fixed point: a
// count pass (k_adjcount, once per disparity map) records the most
// contributions n any cell of the block receives; every contribution is at
// most M = max |lr| in magnitude, so with hd = ceil log2(n + 1) and
// S = 2^(31 - hd - ceil log2 M) each scaled contribution, rounded to
// nearest (no bias), is at most 2^(31 - hd) and the exact integer sum of a
// cell at most (2^hd - 1) 2^(31 - hd) < 2^31: the int32 wrap-around of
// intermediate sums cancels, and integer addition keeps the result bitwise
// reproducible.  Lane x owns tile column x and walks the tile rows: B^T D^T is a
// horizontal polyphase pass per staged LR row (three LDS reads) followed by a
// vertical pass in registers with compile-time taps, so a pixel costs a
// fraction of an LDS read instead of several; then W_k^T sends u to the four
// cells W_k reads.  The per-pixel instruction count is what bounds this
// kernel on gfx950 (a wave64 VALU instruction occupies a 16-lane SIMD for four
// cycles), so the row step is kept to the bare arithmetic.
static constexpr int adjcol_tw(int zeta) { return zeta * (63 / zeta); }
static constexpr int adjcol_th(int zeta) { return zeta * (33 / zeta); }
static constexpr int cdiv_c(int a, int b) { return a >= 0 ? (a + b - 1) / b : -((-a) / b); }

template <int ZETA, int KB, typename TI, bool PV>
__global__ __launch_bounds__(kThreads) void k_adjcol(Geom g, const TI* __restrict__ lr,
                                                     const float* __restrict__ disp, float* __restrict__ outp,
                                                     const float* __restrict__ pmax, int npmax,
                                                     const int* __restrict__ pcnt,
                                                     const DevScalars* __restrict__ sc, int gate) {
  if (gated(sc, g, gate)) return;
  constexpr int RB = KB / 2;
  constexpr int TW = adjcol_tw(ZETA), TH = adjcol_th(ZETA);
  constexpr int CF = RB / ZETA;
  constexpr int RL = (TH - 1 + RB) / ZETA + CF + 1;  // staged LR rows
  constexpr int LX = (TW - 1 + RB) / ZETA + CF + 1;  // staged LR columns
  constexpr int ESL = (RL * LX + 63) / 64;
  constexpr int MM = (2 * RB) / ZETA + 1;            // taps per polyphase phase (at most)
  extern __shared__ uint4 smem_u4[];  // 16-byte aligned: the accumulator is cleared 16 bytes at a time
  float* smem = reinterpret_cast<float*>(smem_u4);
  const int h = g.halo, EY = g.a_ey, EX = g.a_ex;  // EY = TH + 2h, EX = TW + 2h <= kColPitch
  unsigned* acc = reinterpret_cast<unsigned*>(smem);  // [EY][kColPitch]
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  float* e_ = smem + EY * kColPitch + wave * (RL * LX);  // wave-private LR rows
  for (int i = tid; i < EY * (kColPitch / 4); i += kThreads) reinterpret_cast<uint4*>(acc)[i] = make_uint4(0u, 0u, 0u, 0u);

  // fixed-point scale from the producer's block maxima (order-free, so exact)
  float mloc = max_parts(pmax, npmax);
  __shared__ float smax[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mloc = fmaxf(mloc, __shfl_xor(mloc, off, 64));
  if (lane == 0) smax[wave] = mloc;
  __syncthreads();
  const float M = fmaxf(fmaxf(smax[0], smax[1]), fmaxf(smax[2], smax[3]));
  int eM = 0, hd = 0;
  if (M > 0.f) (void)frexpf(M, &eM);  // M < 2^eM
  int bx, by, bz;
  xcd_block3(bx, by, bz);
  const unsigned bid = bx + gridDim.x * (by + gridDim.y * bz);  // the tile's count-pass block
  (void)frexpf((float)pcnt[bid] + 1.f, &hd);  // n + 1 <= 2^hd
  const int sexp = min(max(31 - hd - eM, -120), 120);
  const float S = ldexpf(1.f, sexp), invS = ldexpf(1.f, -sexp);

  const int Y0 = by * TH, X0 = bx * TW;  // tile origin (multiples of ZETA)
  const int i0 = Y0 / ZETA - CF, jb = X0 / ZETA - CF;    // first staged LR row / column
  // staged LR values of this lane: byte offset within a view, or one past
  // the view's end (the range-checked view buffer then reads 0)
  unsigned eoff[ESL];
#pragma unroll
  for (int s = 0; s < ESL; ++s) {
    const int idx = lane + 64 * s;
    const int a = idx / LX, b = idx - a * LX;
    const int i = i0 + a, j = jb + b;
    eoff[s] = (idx < RL * LX && i >= 0 && i < g.sy && j >= 0 && j < g.sx) ? (unsigned)((i * g.sx + j) * sizeof(TI))
                                                                            : 0x80000000u;
  }
  auto fetch = [&](int kv, float (&ev)[ESL]) __attribute__((always_inline)) {
    const __amdgpu_buffer_rsrc_t rv = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<TI*>(lr + (size_t)kv * g.q), (short)0, (int)(g.q * sizeof(TI)), 0x00020000);
#pragma unroll
    for (int s = 0; s < ESL; ++s) ev[s] = buf_load<TI>(rv, eoff[s]);
  };
  // this lane's column: own pixel (x < TW) or idle
  const bool own = lane < TW;
  const int x = own ? lane : 0;
  const int X = X0 + x;
  const bool colin = own && X < g.W;
  // horizontal taps of this column's phase, LR column indices within the staged rows
  float gh[MM];
  int jr[MM];
  {
    const int ph = x % ZETA, q = x / ZETA;
#pragma unroll
    for (int m = 0; m < MM; ++m) {
      gh[m] = 0.f;
      jr[m] = 0;
    }
#pragma unroll
    for (int p = 0; p < ZETA; ++p) {
      if (ph != p) continue;
#pragma unroll
      for (int m = 0; m < MM; ++m) {
        const int lo = cdiv_c(p - RB, ZETA);
        const int t = ZETA * (lo + m) - p + RB;
        gh[m] = t <= 2 * RB ? g.g[t] : 0.f;
        jr[m] = min(q + lo + m + CF, LX - 1);
      }
    }
  }
  // disparity of the column (clamped; 0 outside the image); PV: one map per
  // view ([k][H][W]), the column reloaded at each view
  float om[TH];
  if constexpr (!PV) load_column<TH>(g, disp, Y0, X, colin, om);

  float ereg[ESL];
  const int k0 = bz * g.a_vpb;
  const int k1 = min(g.sk, k0 + g.a_vpb);
  int k = k0 + wave;
  if (k < k1) fetch(k, ereg);
  __syncthreads();  // accumulator zeroed

  unsigned* const accl = acc + (h * kColPitch + x + h);  // accumulator cell of (row 0, this column)
  // PV: the first view's column here, each next one right after the rows of
  // the current view are done with the registers
  if constexpr (PV)
    if (k < k1) load_column<TH>(g, disp + (size_t)k * g.p, Y0, X, colin, om);
  for (; k < k1; k += 4) {
#pragma unroll
    for (int s = 0; s < ESL; ++s)
      if (lane + 64 * s < RL * LX) e_[lane + 64 * s] = ereg[s];
    if (k + 4 < k1) fetch(k + 4, ereg);  // prefetch this wave's next view
    __builtin_amdgcn_wave_barrier();
    // B^T D^T, horizontal: one value per staged LR row, scaled by S
    float hrow[RL];
#pragma unroll
    for (int a = 0; a < RL; ++a) {
      float t = 0.f;
#pragma unroll
      for (int m = 0; m < MM; ++m) t = fmaf(gh[m], e_[a * LX + jr[m]], t);
      hrow[a] = t * S;
    }
    __builtin_amdgcn_wave_barrier();  // reads of e_ precede the next view's staging
    if (!own) continue;  // the idle lanes of the wave (wave-uniform except for them)
    const int ka = k / g.V, kc = k - ka * g.V;
    const float tau = (float)(ka - (g.U - 1) / 2), rho = (float)(kc - (g.V - 1) / 2);
#pragma unroll
    for (int r = 0; r < TH; ++r) {
      // B^T D^T, vertical (compile-time taps of row phase r % ZETA)
      float u = 0.f;
      {
        const int pr = r % ZETA, qr = r / ZETA;
        const int lo = cdiv_c(pr - RB, ZETA);
#pragma unroll
        for (int m = 0; m < MM; ++m) {
          const int t = ZETA * (lo + m) - pr + RB;
          if (t <= 2 * RB) u = fmaf(g.g[t], hrow[qr + lo + m + CF], u);
        }
      }
      // (pixels outside the image have zero disparity, so they only reach
      // accumulator cells outside the image, which the merge never reads)
      const float sy = tau * om[r], sx = rho * om[r];
      const float wy1 = __builtin_amdgcn_fractf(sy), wx1 = __builtin_amdgcn_fractf(sx);
      const float u1 = u * wy1, u0 = u - u1;
      const float br = u1 * wx1, bl = u1 - br, tr = u0 * wx1, tl = u0 - tr;
      // W_k^T: the four cells W_k read (the row, the second tap row and the
      // +1 column are immediate offsets: the pitch is compile-time)
      int cell = floor_i(sy) * kColPitch + floor_i(sx);
      asm("" : "+v"(cell));  // keeps the cell index whole: one shift-add to the lane's byte address
      unsigned* c0 = accl + cell + r * kColPitch;
      unsigned* c1 = c0 + kColPitch;
      atomicAdd(c0, (unsigned)round_i(tl));
      atomicAdd(c0 + 1, (unsigned)round_i(tr));
      atomicAdd(c1, (unsigned)round_i(bl));
      atomicAdd(c1 + 1, (unsigned)round_i(br));
    }
    if constexpr (PV)
      if (k + 4 < k1) load_column<TH>(g, disp + (size_t)(k + 4) * g.p, Y0, X, colin, om);
  }
  __syncthreads();
  const size_t tiles = (size_t)g.a_nty * g.a_ntx;
  float* o = outp + ((size_t)bz * tiles + (size_t)by * g.a_ntx + bx) * (size_t)(EY * EX);
  for (int rr = wave; rr < EY; rr += 4)
    for (int c = lane; c < EX; c += 64) o[rr * EX + c] = (float)(int)acc[rr * kColPitch + c] * invS;
}

// Contribution counts of k_adjcol: the same tiles, view groups and targets,
// each of the four cells of every (view, pixel) counted once; pcnt[block] =
// the largest count of any cell.  Depends on the disparity map only.
template <int ZETA, int KB, bool PV>
__global__ __launch_bounds__(kThreads) void k_adjcount(Geom g, const float* __restrict__ disp, int* __restrict__ pcnt) {
  constexpr int TW = adjcol_tw(ZETA), TH = adjcol_th(ZETA);
  extern __shared__ float smem[];
  const int h = g.halo, EY = g.a_ey, EX = g.a_ex;
  unsigned* cnt = reinterpret_cast<unsigned*>(smem);
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  for (int i = tid; i < EY * EX; i += kThreads) cnt[i] = 0u;
  const int Y0 = blockIdx.y * TH, X0 = blockIdx.x * TW;
  const bool own = lane < TW;
  const int x = own ? lane : 0;
  const int X = X0 + x;
  // the same clamped columns as k_adjcol (PV: one map per view)
  const bool colin = own && X < g.W;
  float om[TH];
  if constexpr (!PV) load_column<TH>(g, disp, Y0, X, colin, om);
  __syncthreads();
  const int k0 = blockIdx.z * g.a_vpb, k1 = min(g.sk, k0 + g.a_vpb);
  const int cb0 = h * EX + x + h;
  if (own) {
    for (int k = k0 + wave; k < k1; k += 4) {
      if constexpr (PV) load_column<TH>(g, disp + (size_t)k * g.p, Y0, X, colin, om);
      const int ka = k / g.V, kc = k - ka * g.V;
      const float tau = (float)(ka - (g.U - 1) / 2), rho = (float)(kc - (g.V - 1) / 2);
#pragma unroll
      for (int r = 0; r < TH; ++r) {
        const float sy = tau * om[r], sx = rho * om[r];
        unsigned* c0 = cnt + (__mul24(floor_i(sy), EX) + floor_i(sx)) + (cb0 + r * EX);
        atomicAdd(c0, 1u);
        atomicAdd(c0 + 1, 1u);
        atomicAdd(c0 + EX, 1u);
        atomicAdd(c0 + EX + 1, 1u);
      }
    }
  }
  __syncthreads();
  unsigned m = 0;
  for (int i = tid; i < EY * EX; i += kThreads) m = max(m, cnt[i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off, 64));
  __shared__ unsigned sm[4];
  if (lane == 0) sm[wave] = m;
  __syncthreads();
  if (tid == 0)
    pcnt[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] =
        (int)max(max(sm[0], sm[1]), max(sm[2], sm[3]));
}

// Per-block max |v| of n floats (scale input of the adjoint entry point).
__global__ __launch_bounds__(kThreads) void k_absmax(const float* __restrict__ v, long long n, float* __restrict__ pmax) {
  float m = 0.f;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < n; o += (long long)gridDim.x * kThreads)
    m = fmaxf(m, fabsf(v[o]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  __shared__ float sm[4];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) pmax[blockIdx.x] = fmaxf(fmaxf(sm[0], sm[1]), fmaxf(sm[2], sm[3]));
}

// out = sum of the adjoint partial images (dense A^T e, read by the CG
// kernels and returned by the operator entry point).
// Same sum when the halo is at most half a tile: a pixel then lies in the
// halo of at most one neighbouring tile row and one neighbouring tile column,
// so each view group contributes at most four values.  All four are loaded
// unconditionally (absent ones from the pixel's own cell, a cache hit) and
// masked afterwards, so the loads of every group are in flight together.
__device__ __forceinline__ float adj_merge_near(const Geom& g, const float* __restrict__ adj, int Y, int X) {
  const int ty = (int)(((float)Y + 0.5f) * g.a_inv_th), tx = (int)(((float)X + 0.5f) * g.a_inv_tw);
  const int ly = Y - ty * g.a_th, lx = X - tx * g.a_tw, h = g.halo;
  const int sy = ly < h ? -1 : (ly >= g.a_th - h ? 1 : 0);
  const int sx = lx < h ? -1 : (lx >= g.a_tw - h ? 1 : 0);
  const bool hy = sy != 0 && ty + sy >= 0 && ty + sy < g.a_nty;
  const bool hx = sx != 0 && tx + sx >= 0 && tx + sx < g.a_ntx;
  const bool hxy = hx && hy;
  const long long tile = (long long)g.a_ey * g.a_ex;
  const long long grp = (long long)g.a_nty * g.a_ntx * tile;
  const long long r0 = (long long)(ly + h) * g.a_ex, r1 = (long long)(ly - sy * g.a_th + h) * g.a_ex;
  const int c0 = lx + h, c1 = lx - sx * g.a_tw + h;
  const long long t00 = ((long long)ty * g.a_ntx + tx) * tile;
  const long long o00 = t00 + r0 + c0;
  const long long o01 = hx ? ((long long)ty * g.a_ntx + tx + sx) * tile + r0 + c1 : o00;
  const long long o10 = hy ? ((long long)(ty + sy) * g.a_ntx + tx) * tile + r1 + c0 : o00;
  const long long o11 = hxy ? ((long long)(ty + sy) * g.a_ntx + tx + sx) * tile + r1 + c1 : o00;
  float v[8][4];
#pragma unroll
  for (int z = 0; z < 8; ++z) {
    if (z >= g.a_vg) break;
    const float* a = adj + z * grp;
    v[z][0] = a[o00];
    v[z][1] = a[o01];
    v[z][2] = a[o10];
    v[z][3] = a[o11];
  }
  float s = 0.f;
#pragma unroll
  for (int z = 0; z < 8; ++z) {
    if (z >= g.a_vg) break;
    s += v[z][0];
    s += hx ? v[z][1] : 0.f;
    s += hy ? v[z][2] : 0.f;
    s += hxy ? v[z][3] : 0.f;
  }
  return s;
}

// The same gather with 32-bit byte offsets through one buffer descriptor over
// all partial images, the view group's plane in the scalar offset, so the four
// candidate offsets are computed once for every group (adj_rs_ok: the partial
// images span less than 2 GiB).
__device__ __forceinline__ bool adj_rs_ok(const Geom& g) {
  return (long long)g.a_vg * g.a_nty * g.a_ntx * g.a_ey * g.a_ex * 4 < 0x7fffffffLL;
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t adj_rsrc(const Geom& g, const float* adj) {
  const long long bytes = (long long)g.a_vg * g.a_nty * g.a_ntx * g.a_ey * g.a_ex * 4;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(adj), (short)0,
                                           (int)(bytes < 0x7fffffffLL ? bytes : 0x7fffffffLL), 0x00020000);
}
__device__ __forceinline__ float adj_merge_near_rs(const Geom& g, __amdgpu_buffer_rsrc_t rs, int Y, int X) {
  const int ty = (int)(((float)Y + 0.5f) * g.a_inv_th), tx = (int)(((float)X + 0.5f) * g.a_inv_tw);
  const int ly = Y - ty * g.a_th, lx = X - tx * g.a_tw, h = g.halo;
  const int sy = ly < h ? -1 : (ly >= g.a_th - h ? 1 : 0);
  const int sx = lx < h ? -1 : (lx >= g.a_tw - h ? 1 : 0);
  const bool hy = sy != 0 && ty + sy >= 0 && ty + sy < g.a_nty;
  const bool hx = sx != 0 && tx + sx >= 0 && tx + sx < g.a_ntx;
  const bool hxy = hx && hy;
  const int tile = g.a_ey * g.a_ex, grpb = g.a_nty * g.a_ntx * tile * 4;
  const int r0 = (ly + h) * g.a_ex, r1 = (ly - sy * g.a_th + h) * g.a_ex;
  const int c0 = lx + h, c1 = lx - sx * g.a_tw + h;
  const int o00 = ((ty * g.a_ntx + tx) * tile + r0 + c0) * 4;
  const int o01 = hx ? ((ty * g.a_ntx + tx + sx) * tile + r0 + c1) * 4 : o00;
  const int o10 = hy ? (((ty + sy) * g.a_ntx + tx) * tile + r1 + c0) * 4 : o00;
  const int o11 = hxy ? (((ty + sy) * g.a_ntx + tx + sx) * tile + r1 + c1) * 4 : o00;
  float v[8][4];
#pragma unroll
  for (int z = 0; z < 8; ++z) {
    if (z >= g.a_vg) break;
    const int so = z * grpb;
    v[z][0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, o00, so, 0));
    v[z][1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, o01, so, 0));
    v[z][2] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, o10, so, 0));
    v[z][3] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, o11, so, 0));
  }
  float s = 0.f;
#pragma unroll
  for (int z = 0; z < 8; ++z) {
    if (z >= g.a_vg) break;
    s += v[z][0];
    s += hx ? v[z][1] : 0.f;
    s += hy ? v[z][2] : 0.f;
    s += hxy ? v[z][3] : 0.f;
  }
  return s;
}

__global__ __launch_bounds__(kThreads) void k_merge(Geom g, const float* __restrict__ adj, float* __restrict__ out,
                                                    const DevScalars* __restrict__ sc, int gate) {
  if (gated(sc, g, gate)) return;
  const bool near = 2 * g.halo <= g.a_th && 2 * g.halo <= g.a_tw && g.a_vg <= 8;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < g.p; o += (long long)gridDim.x * kThreads) {
    const int Y = (int)(o / g.W), X = (int)(o - (long long)Y * g.W);
    out[o] = near ? adj_merge_near(g, adj, Y, X) : adj_merge(g, adj, Y, X);
  }
}

// ---------------------------------------------------------------------------
// NLTV block of the wz-step (sec 3.4, 4.1; Algorithm 1): for every offset d
//   g_d = c_d m (x - S_d x)  (dropped where z+d is outside),
//   w_S' = clip(g_d + w_S, +-1/vartheta),  f_d = 2 w_S' - w_S,
//   vs = S^T f = sum_d [c_d m(z) f_d(z) 1(z+d in) - c_d m(z-d) f_d(z-d) 1(z-d in)].
// The second term is pulled: f_d(z-d) is recomputed from the previous dual,
// which ping-pong buffers keep intact.  Per-block partials {sum|g|,
// sum (w_S'-w_S)^2} go to `part`.  grid = (ceil(W/64), ceil(H/16)).
// Offset d of a (2 rw + 1)^2 NLTV window, row-major with the centre skipped
// (the host builds the weight tables in the same order).
__host__ __device__ constexpr int win_dy(int rw, int d) {
  return (d < ((2 * rw + 1) * (2 * rw + 1)) / 2 ? d : d + 1) / (2 * rw + 1) - rw;
}
__host__ __device__ constexpr int win_dx(int rw, int d) {
  return (d < ((2 * rw + 1) * (2 * rw + 1)) / 2 ? d : d + 1) % (2 * rw + 1) - rw;
}

// RW > 0: compile-time window radius (offsets and tile pitch become
// immediates); RW = 0: the radius and offsets come from g at run time.
template <bool INTERIOR, typename T, int RW, int NT>
__device__ __forceinline__ void tv_tile(const Geom& g, const float* __restrict__ xs, const float* __restrict__ ms,
                                        const T* wo, T* wn_, float* __restrict__ vs, int X0, int Y0,
                                        double& s_abs, double& s_dw) {
  const int rw = RW > 0 ? RW : g.rw;
  const int LXd = kTvTileX + 2 * rw;
  const int SD = RW > 0 ? (2 * RW + 1) * (2 * RW + 1) - 1 : g.sd;
  constexpr int NW = NT / 64, RPT = kTvTileY / NW;  // waves; tile rows per thread (ly0 + NW rr)
  const int lx = threadIdx.x & 63, ly0 = threadIdx.x >> 6;
  const int X = X0 + lx;
  int Y[RPT], sl[RPT];
  bool in[RPT];
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int ly = ly0 + NW * rr;
    Y[rr] = Y0 + ly;
    in[rr] = INTERIOR || (Y[rr] < g.H && X < g.W);
    sl[rr] = (ly + rw) * LXd + (lx + rw);
  }
  float acc[RPT];
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) acc[rr] = 0.f;
  // statistics: FP32 sums over at most 4 RPT terms (one ring step of four
  // offsets x RPT rows, relative error <= 4 RPT u), added to the FP64 totals
  float f_abs = 0.f, f_dw = 0.f;
  auto flush = [&]() __attribute__((always_inline)) {
    s_abs += (double)f_abs;
    s_dw += (double)f_dw;
    f_abs = 0.f;
    f_dw = 0.f;
  };
  // byte offset of pixel (Y[rr], X) within one dual plane (a plane is below
  // 2 GiB), so every dual access is a uniform plane pointer plus this offset
  unsigned boff[RPT];
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) boff[rr] = in[rr] ? (unsigned)(((size_t)Y[rr] * g.W + X) * sizeof(T)) : 0u;
  auto load = [&](int d, float (&w0)[RPT], float (&w2)[RPT]) __attribute__((always_inline)) {
    const int dy = RW > 0 ? win_dy(RW, d) : g.ody[d], dx = RW > 0 ? win_dx(RW, d) : g.odx[d];
    const T* wd = wo + (size_t)d * g.p;
    const __amdgpu_buffer_rsrc_t r0 = plane_rsrc(wd);
    const __amdgpu_buffer_rsrc_t r2 = plane_rsrc(wd - ((ptrdiff_t)dy * g.W + dx));  // plane shifted by -d
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      w0[rr] = in[rr] ? buf_load<T>(r0, boff[rr]) : 0.f;
      const bool bin = INTERIOR || (in[rr] && Y[rr] - dy >= 0 && Y[rr] - dy < g.H && X - dx >= 0 && X - dx < g.W);
      w2[rr] = bin ? buf_load<T>(r2, boff[rr]) : 0.f;
    }
  };
  // offset d with its dual values w0 = w_d(z), w2 = w_d(z - d)
  auto step = [&](int d, const float (&w0)[RPT], const float (&w2)[RPT]) __attribute__((always_inline)) {
    const int dy = RW > 0 ? win_dy(RW, d) : g.ody[d], dx = RW > 0 ? win_dx(RW, d) : g.odx[d];
    const int dd = dy * LXd + dx;
    const float c = g.cd[d];
    const __amdgpu_buffer_rsrc_t rn = plane_rsrc(wn_ + (size_t)d * g.p);
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      if (!in[rr]) continue;
      const float xz = xs[sl[rr]], mz = ms[sl[rr]];
      const bool fin = INTERIOR || (Y[rr] + dy >= 0 && Y[rr] + dy < g.H && X + dx >= 0 && X + dx < g.W);
      const float gv = fin ? c * mz * (xz - xs[sl[rr] + dd]) : 0.f;
      const float wn = clipf(gv + w0[rr], g.clip);
      buf_store<T>(rn, boff[rr], (T)wn);
      if (fin) acc[rr] = fmaf(c * mz, 2.f * wn - w0[rr], acc[rr]);
      const float dw = wn - w0[rr];
      f_abs += fabsf(gv);
      f_dw = fmaf(dw, dw, f_dw);
      const bool bin = INTERIOR || (Y[rr] - dy >= 0 && Y[rr] - dy < g.H && X - dx >= 0 && X - dx < g.W);
      if (bin) {
        const float mm = ms[sl[rr] - dd];
        const float g2 = c * mm * (xs[sl[rr] - dd] - xz);
        const float wn2 = clipf(g2 + w2[rr], g.clip);
        acc[rr] = fmaf(-(c * mm), 2.f * wn2 - w2[rr], acc[rr]);
      }
    }
  };
  if constexpr (RW > 0) {
    // ring of P in-flight offsets: slot j holds offset d0 + j and is refilled
    // with offset d0 + j + P right after its use, so no register is moved and
    // P - 1 offsets of loads stay in flight behind the one being used
    constexpr int P = 4, SDc = (2 * RW + 1) * (2 * RW + 1) - 1;
    static_assert(SDc % P == 0, "the window's offset count is a multiple of 4");
    float b0[P][RPT], b2[P][RPT];
#pragma unroll
    for (int j = 0; j < P; ++j) load(j, b0[j], b2[j]);
#pragma unroll 1
    for (int d0 = 0; d0 < SDc - P; d0 += P) {
#pragma unroll
      for (int j = 0; j < P; ++j) {
        step(d0 + j, b0[j], b2[j]);
        load(d0 + j + P, b0[j], b2[j]);
      }
      flush();
    }
#pragma unroll
    for (int j = 0; j < P; ++j) step(SDc - P + j, b0[j], b2[j]);
    flush();
  } else {
    // software pipeline: the dual values of offsets d+1 and d+2 are in flight while d is used
    float c0[RPT], c2[RPT], n0[RPT], n2[RPT];
    if (SD > 0) load(0, c0, c2);
    if (SD > 1) load(1, n0, n2);
#pragma unroll 1
    for (int d = 0; d < SD; ++d) {
      float w0[RPT], w2[RPT];
#pragma unroll
      for (int rr = 0; rr < RPT; ++rr) {
        w0[rr] = c0[rr];
        w2[rr] = c2[rr];
        c0[rr] = n0[rr];
        c2[rr] = n2[rr];
      }
      if (d + 2 < SD) load(d + 2, n0, n2);
      step(d, w0, w2);
      flush();
    }
  }
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr)
    if (in[rr]) vs[(size_t)Y[rr] * g.W + X] = acc[rr];
}

// Interior tiles with 16-bit duals and an even image width: the same
// per-pixel arithmetic as tv_tile<true>, with the lanes mapped to pixel pairs
// so that every dual access is a dword (2-byte accesses cost as much per
// instruction as 4-byte ones here).  Lane l of wave w (of NW) owns columns
// 2 (l & 31) and 2 (l & 31) + 1 of rows 2 w + (l >> 5) + 2 NW q for its
// row-steps q; slot rr = 2 q + column.  Pair (X, X + 1), X even, is one aligned dword of a
// plane; the pulled term's pair (X - dx, X + 1 - dx) is one aligned dword for
// even dx and the high / low halves of the two dwords around it for odd dx.
template <typename T, int RW, int NT>
__device__ __forceinline__ void tv_tile_pair(const Geom& g, const float* __restrict__ xs, const float* __restrict__ ms,
                                             const T* wo, T* wn_, float* __restrict__ vs, int X0, int Y0,
                                             double& s_abs, double& s_dw) {
  static_assert(sizeof(T) == 2 && RW > 0, "16-bit duals, compile-time radius");
  constexpr int LXd = kTvTileX + 2 * RW, SD = (2 * RW + 1) * (2 * RW + 1) - 1, P = 4;
  static_assert(SD % P == 0, "the window's offset count is a multiple of 4");
  constexpr int NW = NT / 64, NRS = kTvTileY / (2 * NW), NS = 2 * NRS;  // row-steps, slots per thread
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int Y[NS], X[NS], sl[NS];
#pragma unroll
  for (int rr = 0; rr < NS; ++rr) {
    const int lx = 2 * (lane & 31) + (rr & 1), ly = 2 * wave + (lane >> 5) + 2 * NW * (rr >> 1);
    Y[rr] = Y0 + ly;
    X[rr] = X0 + lx;
    sl[rr] = (ly + RW) * LXd + (lx + RW);
  }
  unsigned boff[NRS];  // byte offset of each row's pair (dword aligned)
#pragma unroll
  for (int q = 0; q < NRS; ++q) boff[q] = (unsigned)(((size_t)Y[2 * q] * g.W + X[2 * q]) * 2);
  float acc[NS];
#pragma unroll
  for (int rr = 0; rr < NS; ++rr) acc[rr] = 0.f;
  float f_abs = 0.f, f_dw = 0.f;  // FP32 sums over one ring step (16 terms), then FP64
  auto flush = [&]() __attribute__((always_inline)) {
    s_abs += (double)f_abs;
    s_dw += (double)f_dw;
    f_abs = 0.f;
    f_dw = 0.f;
  };
  auto half = [](unsigned dw, int hi) __attribute__((always_inline)) {
    return (float)__builtin_bit_cast(T, (unsigned short)(hi ? dw >> 16 : dw & 0xffffu));
  };
  // raw dwords of offset d: a0[q] = pair at z, b0[q] / b1[q] = the dword(s) of the pair at z - d
  auto load = [&](int d, unsigned (&a0)[NRS], unsigned (&b0)[NRS], unsigned (&b1)[NRS]) __attribute__((always_inline)) {
    const int dy = win_dy(RW, d), dx = win_dx(RW, d);
    const T* wd = wo + (size_t)d * g.p;
    const __amdgpu_buffer_rsrc_t r0 = plane_rsrc(wd);
    const __amdgpu_buffer_rsrc_t r2 = plane_rsrc(wd - ((ptrdiff_t)dy * g.W + dx));  // plane shifted by -d
    const unsigned od = (unsigned)(dx & 1) * 2u;  // odd dx: the dwords either side (even: the same one twice)
#pragma unroll
    for (int q = 0; q < NRS; ++q) {
      a0[q] = __builtin_amdgcn_raw_buffer_load_b32(r0, (int)boff[q], 0, 0);
      b0[q] = __builtin_amdgcn_raw_buffer_load_b32(r2, (int)(boff[q] - od), 0, 0);
      b1[q] = __builtin_amdgcn_raw_buffer_load_b32(r2, (int)(boff[q] + od), 0, 0);
    }
  };
  auto step = [&](int d, const unsigned (&a0)[NRS], const unsigned (&b0)[NRS], const unsigned (&b1)[NRS])
                  __attribute__((always_inline)) {
    const int dy = win_dy(RW, d), dx = win_dx(RW, d);
    const int dd = dy * LXd + dx;
    const float c = g.cd[d];
    const __amdgpu_buffer_rsrc_t rn = plane_rsrc(wn_ + (size_t)d * g.p);
    unsigned bits[NS];
#pragma unroll
    for (int rr = 0; rr < NS; ++rr) {
      const int q = rr >> 1, h = rr & 1;
      const float w0 = half(a0[q], h);
      // odd dx: the pair straddles two dwords (high half of the first, low half of the second)
      const float w2 = (dx & 1) ? (h ? half(b1[q], 0) : half(b0[q], 1)) : half(b0[q], h);
      const float xz = xs[sl[rr]], mz = ms[sl[rr]];
      const float gv = c * mz * (xz - xs[sl[rr] + dd]);
      const float wn = clipf(gv + w0, g.clip);
      bits[rr] = __builtin_bit_cast(unsigned short, (T)wn);
      acc[rr] = fmaf(c * mz, 2.f * wn - w0, acc[rr]);
      const float dw = wn - w0;
      f_abs += fabsf(gv);
      f_dw = fmaf(dw, dw, f_dw);
      const float mm = ms[sl[rr] - dd];
      const float g2 = c * mm * (xs[sl[rr] - dd] - xz);
      const float wn2 = clipf(g2 + w2, g.clip);
      acc[rr] = fmaf(-(c * mm), 2.f * wn2 - w2, acc[rr]);
    }
#pragma unroll
    for (int q = 0; q < NRS; ++q)
      __builtin_amdgcn_raw_buffer_store_b32(bits[2 * q] | (bits[2 * q + 1] << 16), rn, (int)boff[q], 0, 0);
  };
  unsigned a0[P][NRS], b0[P][NRS], b1[P][NRS];
#pragma unroll
  for (int j = 0; j < P; ++j) load(j, a0[j], b0[j], b1[j]);
#pragma unroll 1
  for (int d0 = 0; d0 < SD - P; d0 += P) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      step(d0 + j, a0[j], b0[j], b1[j]);
      load(d0 + j + P, a0[j], b0[j], b1[j]);
    }
    flush();
  }
#pragma unroll
  for (int j = 0; j < P; ++j) step(SD - P + j, a0[j], b0[j], b1[j]);
  flush();
#pragma unroll
  for (int rr = 0; rr < NS; ++rr) vs[(size_t)Y[rr] * g.W + X[rr]] = acc[rr];
}

// T: storage type of x and of the dual; the dual recomputed for the pulled
// term is the same FP32 value the owning thread stores (rounded) for w_S'.
// Eight waves share a tile (two rows per thread), so twice as many waves
// overlap their arithmetic with the dual streams as with four.
template <typename T, int RW>
__global__ __launch_bounds__(kTvThreads) void k_tv(Geom g, const T* __restrict__ x, const float* __restrict__ m,
                                                 T* ws0, T* ws1, float* __restrict__ vs,
                                                 double* __restrict__ part, const DevScalars* __restrict__ sc) {
  if (sc->admm_done) return;
  int tx, ty, tt;
  if (!xcd_tile((g.W + kTvTileX - 1) / kTvTileX, (g.H + kTvTileY - 1) / kTvTileY, tx, ty, tt)) return;
  extern __shared__ float smem[];
  const int rw = RW > 0 ? RW : g.rw;
  const int LXd = kTvTileX + 2 * rw, LYd = kTvTileY + 2 * rw;
  float* xs = smem;
  float* ms = xs + LYd * LXd;
  const int X0 = tx * kTvTileX, Y0 = ty * kTvTileY;
  stage_tile<T, 8, kTvThreads>(xs, LXd, x, g.H, g.W, Y0 - rw, X0 - rw, LYd, LXd);
  stage_tile<float, 8, kTvThreads>(ms, LXd, m, g.H, g.W, Y0 - rw, X0 - rw, LYd, LXd);
  __syncthreads();
  const T* wo = sc->wcur ? ws1 : ws0;
  T* wn_ = sc->wcur ? ws0 : ws1;
  const bool interior = X0 - rw >= 0 && X0 + kTvTileX + rw <= g.W && Y0 - rw >= 0 && Y0 + kTvTileY + rw <= g.H;
  double s_abs = 0.0, s_dw = 0.0;
  if constexpr (sizeof(T) == 2 && RW > 0) {
    // (odd dx reads the dword past the halo's last column: keep that column inside the row)
    if (interior && (g.W & 1) == 0 && X0 + kTvTileX + RW + 1 <= g.W)
      tv_tile_pair<T, RW, kTvThreads>(g, xs, ms, wo, wn_, vs, X0, Y0, s_abs, s_dw);
    else if (interior) tv_tile<true, T, RW, kTvThreads>(g, xs, ms, wo, wn_, vs, X0, Y0, s_abs, s_dw);
    else tv_tile<false, T, RW, kTvThreads>(g, xs, ms, wo, wn_, vs, X0, Y0, s_abs, s_dw);
  } else {
    if (interior) tv_tile<true, T, RW, kTvThreads>(g, xs, ms, wo, wn_, vs, X0, Y0, s_abs, s_dw);
    else tv_tile<false, T, RW, kTvThreads>(g, xs, ms, wo, wn_, vs, X0, Y0, s_abs, s_dw);
  }
  double v[2] = {s_abs, s_dw};
  block_sum<2, kTvThreads / 64>(v);
  if (threadIdx.x == 0) {
    part[(size_t)tt * 2 + 0] = v[0];
    part[(size_t)tt * 2 + 1] = v[1];
  }
}

// ---------------------------------------------------------------------------
// H p = cA * sum_k A_k^T A_k p + (vartheta/2) S^T V^2 S p (sec 5), the NLTV
// part written as the symmetric weighted Laplacian
//   sum_d c_d^2 (m(z)^2 + m(z+d)^2) (p(z) - p(z+d)) 1(z+d in the image),
// which equals S^T V^2 S p because the offset set is symmetric.  With
// with_dot, per-block partials of <p, Hp> go to `part`.
template <bool INTERIOR, int RW>
__device__ __forceinline__ float tv_laplacian(const Geom& g, const float* __restrict__ ps,
                                              const float* __restrict__ m2, int sl, int Y, int X, int LXd) {
  const float pz = ps[sl], mz = m2[sl];
  float lap = 0.f;
  const int SD = RW > 0 ? (2 * RW + 1) * (2 * RW + 1) - 1 : g.sd;
#pragma unroll(RW > 0 ? 64 : 8)
  for (int d = 0; d < SD; ++d) {
    const int dy = RW > 0 ? win_dy(RW, d) : g.ody[d], dx = RW > 0 ? win_dx(RW, d) : g.odx[d];
    const int sn = sl + dy * LXd + dx;
    float t = g.cd2[d] * (mz + m2[sn]) * (pz - ps[sn]);
    if (!INTERIOR && (Y + dy < 0 || Y + dy >= g.H || X + dx < 0 || X + dx >= g.W)) t = 0.f;
    lap += t;
  }
  return lap;
}

// `hp` holds the merged A^T A p on entry and H p on exit (read, then written,
// by the same thread).
template <int RW>
__global__ __launch_bounds__(kThreads) void k_hp(Geom g, const float* __restrict__ pv, const float* __restrict__ m,
                                                 float* hp,
                                                 double* __restrict__ part, const DevScalars* __restrict__ sc,
                                                 int gate, int with_dot) {
  if (gated(sc, g, gate)) return;
  extern __shared__ float smem[];
  const int rw = RW > 0 ? RW : g.rw;
  const int LXd = kTvTileX + 2 * rw, LYd = kTvTileY + 2 * rw;
  float* ps = smem;
  float* m2 = ps + LYd * LXd;
  const int X0 = blockIdx.x * kTvTileX, Y0 = blockIdx.y * kTvTileY;
  const int tid = threadIdx.x;
  if (g.sd > 0) {
    stage_tile(ps, LXd, pv, g.H, g.W, Y0 - rw, X0 - rw, LYd, LXd);
    stage_tile(m2, LXd, m, g.H, g.W, Y0 - rw, X0 - rw, LYd, LXd);
    __syncthreads();
    for (int idx = tid; idx < LYd * LXd; idx += kThreads) m2[idx] = m2[idx] * m2[idx];
  }
  __syncthreads();
  const bool interior = X0 - rw >= 0 && X0 + kTvTileX + rw <= g.W && Y0 - rw >= 0 && Y0 + kTvTileY + rw <= g.H;
  const int lx = tid & 63, ly0 = tid >> 6;
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
      lap = interior ? tv_laplacian<true, RW>(g, ps, m2, sl, Y, X, LXd)
                     : tv_laplacian<false, RW>(g, ps, m2, sl, Y, X, LXd);
    }
    const float v = g.cA * hp[o] + g.half_theta * lap;
    hp[o] = v;
    if (with_dot) s_dot += (double)pv[o] * (double)v;
  }
  if (!with_dot) return;
  double v[1] = {s_dot};
  block_sum<1>(v);
  if (tid == 0) part[blockIdx.x + gridDim.x * blockIdx.y] = v[0];
}

// k_hp with a compile-time window radius: lane = tile column, wave w = a
// strip of kTvTileY/4 consecutive rows.  p and m^2 are staged interleaved,
// so each window row a strip needs is 2 RW + 1 paired 8-byte LDS reads shared
// by the strip's pixels, and every term of the Laplacian is plain VALU work
// (same terms and weights as tv_laplacian, summed by window row).
template <bool INTERIOR, int RW>
__device__ __forceinline__ void hp_strip(const Geom& g, const float2* __restrict__ pm, int lx, int r0, int Y0, int X,
                                         float (&pz)[kTvTileY / 4], float (&lap)[kTvTileY / 4]) {
  constexpr int HS = kTvTileY / 4, WN = 2 * RW + 1, LXd = kTvTileX + 2 * RW, CTR = (WN * WN - 1) / 2;
  float mz[HS];
  // boundary tiles: bit j of rok = window row j inside the image, bit q of
  // cok = column offset q - RW inside (interior tiles skip the test)
  unsigned rok = 0u, cok = 0u;
  if (!INTERIOR) {
#pragma unroll
    for (int j = 0; j < HS + 2 * RW; ++j) {
      const int Yn = Y0 + r0 + j - RW;
      rok |= (Yn >= 0 && Yn < g.H) ? 1u << j : 0u;
    }
#pragma unroll
    for (int q = 0; q < WN; ++q) {
      const int Xn = X + q - RW;
      cok |= (Xn >= 0 && Xn < g.W) ? 1u << q : 0u;
    }
  }
#pragma unroll
  for (int i = 0; i < HS; ++i) {
    const float2 c = pm[(r0 + i + RW) * LXd + lx + RW];
    pz[i] = c.x;
    mz[i] = c.y;
    lap[i] = 0.f;
  }
#pragma unroll
  for (int j = 0; j < HS + 2 * RW; ++j) {  // window row j: tile row r0 + j - RW
    float2 n[WN];
#pragma unroll
    for (int q = 0; q < WN; ++q) n[q] = pm[(r0 + j) * LXd + lx + q];
#pragma unroll
    for (int i = 0; i < HS; ++i) {
      const int dy = j - RW - i;
      if (dy < -RW || dy > RW) continue;
#pragma unroll
      for (int q = 0; q < WN; ++q) {
        const int dx = q - RW;
        if (dy == 0 && dx == 0) continue;
        const int idx = (dy + RW) * WN + (dx + RW);
        const int d = idx < CTR ? idx : idx - 1;
        float w = g.cd2[d] * (mz[i] + n[q].y);
        if (!INTERIOR) w = ((rok >> j) & (cok >> q) & 1u) ? w : 0.f;
        lap[i] = fmaf(w, pz[i] - n[q].x, lap[i]);
      }
    }
  }
}

template <int RW>
__global__ __launch_bounds__(kThreads, 6) void k_hpstrip(Geom g, const float* __restrict__ pv,
                                                      const float* __restrict__ m, float* hp,
                                                      const float* __restrict__ adj,
                                                      double* __restrict__ part,
                                                      const DevScalars* __restrict__ sc, int gate, int with_dot,
                                                      int fused) {
  static_assert(RW > 0, "compile-time radius");
  if (gated(sc, g, gate)) return;
  constexpr int HS = kTvTileY / 4, LXd = kTvTileX + 2 * RW, LYd = kTvTileY + 2 * RW;
  extern __shared__ float2 smem_f2[];
  float2* pm = smem_f2;  // [LYd][LXd] (p, m^2), zero outside the image
  int bx, by, bz;
  xcd_block3(bx, by, bz);
  const int X0 = bx * kTvTileX, Y0 = by * kTvTileY;
  const int tid = threadIdx.x;
  {
    constexpr int n = LYd * LXd, BATCH = 4;
    for (int base = tid; base < n; base += kThreads * BATCH) {
      float pvv[BATCH], mv[BATCH];
      int off[BATCH];
#pragma unroll
      for (int j = 0; j < BATCH; ++j) {
        const int e = base + j * kThreads;
        const int r = e / LXd, c = e - r * LXd;
        const int Y = Y0 - RW + r, X = X0 - RW + c;
        const bool ok = e < n && Y >= 0 && Y < g.H && X >= 0 && X < g.W;
        const size_t o = ok ? (size_t)Y * g.W + X : 0;
        pvv[j] = ok ? pv[o] : 0.f;
        mv[j] = ok ? m[o] : 0.f;
        off[j] = e < n ? e : -1;
      }
#pragma unroll
      for (int j = 0; j < BATCH; ++j)
        if (off[j] >= 0) pm[off[j]] = make_float2(pvv[j], mv[j] * mv[j]);
    }
  }
  __syncthreads();
  const bool interior = X0 - RW >= 0 && X0 + kTvTileX + RW <= g.W && Y0 - RW >= 0 && Y0 + kTvTileY + RW <= g.H;
  const int lx = tid & 63, r0 = (tid >> 6) * HS;
  const int X = X0 + lx;
  float pz[HS], lap[HS];
  if (interior) hp_strip<true, RW>(g, pm, lx, r0, Y0, X, pz, lap);
  else hp_strip<false, RW>(g, pm, lx, r0, Y0, X, pz, lap);
  double s_dot = 0.0;
  const bool rs_ok = fused && adj_rs_ok(g);
  const __amdgpu_buffer_rsrc_t ars = adj_rsrc(g, adj);
#pragma unroll
  for (int i = 0; i < HS; ++i) {
    const int Y = Y0 + r0 + i;
    if (Y >= g.H || X >= g.W) continue;
    const size_t o = (size_t)Y * g.W + X;
    // fused: A^T A p gathered here from the adjoint's partial images
    const float ata = rs_ok ? adj_merge_near_rs(g, ars, Y, X) : fused ? adj_merge_near(g, adj, Y, X) : hp[o];
    const float v = g.cA * ata + g.half_theta * lap[i];
    hp[o] = v;
    if (with_dot) s_dot += (double)pz[i] * (double)v;
  }
  if (!with_dot) return;
  double v[1] = {s_dot};
  block_sum<1>(v);
  if (tid == 0) part[blockIdx.x + gridDim.x * blockIdx.y] = v[0];
}

// ---------------------------------------------------------------------------
// CG start (Algorithm 2 from delta = 0): v = A^T e + (vartheta/2) S^T f,
// r = -v, p = r, partials of <r, r>.  Block 0 also closes the wz-step's
// statistics: J(x^(n-1)), the primal residual and the stop test.
// `r` holds the merged A^T e on entry.
__global__ __launch_bounds__(kCgThreads) void k_cginit(Geom g, const float* __restrict__ vs, float* r,
                                                     float* __restrict__ pv, double* __restrict__ prr,
                                                     const double* __restrict__ pwzd, int nwzd,
                                                     const double* __restrict__ ptv, int ntv,
                                                     double* __restrict__ stats, DevScalars* __restrict__ sc,
                                                     const float* __restrict__ adj, int fused) {
  if (sc->admm_done) return;
  double s = 0.0;
  const bool rs_ok = fused && adj_rs_ok(g);
  const __amdgpu_buffer_rsrc_t ars = adj_rsrc(g, adj);
  const long long gstride = (long long)gridDim.x * kCgThreads * 4;
  for (long long o0 = blockIdx.x * (long long)kCgThreads * 4 + threadIdx.x; o0 < g.p; o0 += gstride) {
    float v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long o = o0 + j * kCgThreads;
      v[j] = 0.f;
      if (o < g.p) {
        if (fused) {  // A^T e gathered here from the adjoint's partial images
          const unsigned Y = (unsigned)o / (unsigned)g.W, X = (unsigned)o - Y * (unsigned)g.W;
          v[j] = rs_ok ? adj_merge_near_rs(g, ars, (int)Y, (int)X) : adj_merge_near(g, adj, (int)Y, (int)X);
        } else {
          v[j] = r[o];
        }
        if (g.sd > 0) v[j] += g.half_theta * vs[o];
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long o = o0 + j * kCgThreads;
      if (o < g.p) {
        const float rv = -v[j];
        r[o] = rv;
        pv[o] = rv;
        s += (double)rv * (double)rv;
      }
    }
  }
  double v[1] = {s};
  block_sum<1, kCgThreads / 64>(v);
  if (threadIdx.x == 0) prr[blockIdx.x] = v[0];
  if (blockIdx.x != 0) return;
  double a[3], b[2] = {0.0, 0.0};
  sum_parts<3, kCgThreads>(pwzd, nwzd, a);
  if (g.sd > 0) sum_parts<2, kCgThreads>(ptv, ntv, b);
  if (threadIdx.x == 0) {
    double* row = stats_row(g, stats, sc);
    const double data = (double)g.lambda1 * a[0] + (double)g.lambda2 * a[1];
    const double res = sqrt(a[2] + b[1]);
    row[0] = data + b[0];
    row[1] = res;
    row[4] = data;
    row[5] = b[0];
    if (!sc->res1_set) {
      sc->res1 = res;
      sc->res1_set = 1;
    }
    if (g.stop_tol > 0.f && res <= (double)g.stop_tol * sc->res1) sc->stop_pending = 1;
    sc->cg_done = 0;
    sc->cg_steps = 0;
  }
}

// CG step `step` (1-based), part 1: pi = <r,r> from the previous partials,
// alpha = pi / <p, Hp>; x += alpha p (the x-step accumulates straight into the
// FP32 estimate: x itself, or the FP32 remainder of a 16-bit x),
// r -= alpha Hp, partials of the new <r, r>.  CG stops (Algorithm 2) when
// pi <= tau, pi = 0, or <p, Hp> <= 0.
__global__ __launch_bounds__(kCgThreads) void k_cgupd(Geom g, float* __restrict__ x, float* __restrict__ r,
                                                    const float* __restrict__ pv, const float* __restrict__ hp,
                                                    const double* __restrict__ prr_prev, double* __restrict__ prr_new,
                                                    const double* __restrict__ pphp, int nphp, int step,
                                                    DevScalars* __restrict__ sc) {
  if (sc->admm_done || sc->cg_done) return;
  double t[2];
  {
    double a[1], b[1];
    sum_parts<1, kCgThreads>(prr_prev, g.red_blocks, a);
    sum_parts<1, kCgThreads>(pphp, nphp, b);
    t[0] = a[0];
    t[1] = b[0];
  }
  const double pi = t[0], php = t[1];
  if (!(pi > (double)g.cg_tol) || pi == 0.0 || !(php > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->cg_done = 1;
    return;
  }
  const float alpha = (float)(pi / php);
  double s = 0.0;
  const long long gstride = (long long)gridDim.x * kCgThreads * 4;
  for (long long o0 = blockIdx.x * (long long)kCgThreads * 4 + threadIdx.x; o0 < g.p; o0 += gstride) {
    float xv[4], pw[4], hw[4], rw[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long o = o0 + j * kCgThreads;
      const bool in = o < g.p;
      xv[j] = in ? x[o] : 0.f;
      pw[j] = in ? pv[o] : 0.f;
      hw[j] = in ? hp[o] : 0.f;
      rw[j] = in ? r[o] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long o = o0 + j * kCgThreads;
      if (o < g.p) {
        x[o] = fmaf(alpha, pw[j], xv[j]);
        const float rv = fmaf(-alpha, hw[j], rw[j]);
        r[o] = rv;
        s += (double)rv * (double)rv;
      }
    }
  }
  double v[1] = {s};
  block_sum<1, kCgThreads / 64>(v);
  if (threadIdx.x == 0) prr_new[blockIdx.x] = v[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->cg_steps = step;
}

// CG step part 2: beta = pi_new / pi_old, p = r + beta p.
__global__ __launch_bounds__(kCgThreads) void k_cgp(Geom g, const float* __restrict__ r, float* __restrict__ pv,
                                                  const double* __restrict__ prr_old,
                                                  const double* __restrict__ prr_new,
                                                  const DevScalars* __restrict__ sc) {
  if (sc->admm_done || sc->cg_done) return;
  double a[1], b[1];
  sum_parts<1, kCgThreads>(prr_new, g.red_blocks, a);
  sum_parts<1, kCgThreads>(prr_old, g.red_blocks, b);
  const float beta = (float)(a[0] / b[0]);
  const long long gstride = (long long)gridDim.x * kCgThreads * 4;
  for (long long o0 = blockIdx.x * (long long)kCgThreads * 4 + threadIdx.x; o0 < g.p; o0 += gstride) {
    float pw[4], rw[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long o = o0 + j * kCgThreads;
      const bool in = o < g.p;
      pw[j] = in ? pv[o] : 0.f;
      rw[j] = in ? r[o] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long o = o0 + j * kCgThreads;
      if (o < g.p) pv[o] = fmaf(beta, pw[j], rw[j]);
    }
  }
}

// End of an ADMM iteration: final CG pi and step count, iteration count,
// NLTV-dual ping-pong, stop flag.  One block.
__global__ __launch_bounds__(kThreads) void k_iter_end(Geom g, const double* __restrict__ prr0,
                                                       const double* __restrict__ prr1, double* __restrict__ stats,
                                                       DevScalars* __restrict__ sc) {
  if (sc->admm_done) return;
  const int steps = sc->cg_steps;
  double a[1];
  sum_parts<1>((steps & 1) ? prr1 : prr0, g.red_blocks, a);
  if (threadIdx.x != 0) return;
  double* row = stats_row(g, stats, sc);
  row[2] = a[0];
  row[3] = (double)steps;
  sc->pi = a[0];
  sc->iters_done += 1;
  if (g.sd > 0) sc->wcur ^= 1;
  if (sc->stop_pending) sc->admm_done = 1;
}

// ---------------------------------------------------------------------------
// sec 3.4: m = exp(-|grad x|^2 / sigma_e) * occ, forward differences.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_edge(Geom g, const T* __restrict__ x, const float* __restrict__ occ,
                                                   float* __restrict__ m, const DevScalars* __restrict__ sc, int gate) {
  if (gated(sc, g, gate)) return;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < g.p; o += (long long)gridDim.x * kThreads) {
    const int Y = (int)(o / g.W), X = (int)(o - (long long)Y * g.W);
    float we = 1.f;
    if (g.use_edge) {
      const float xz = (float)x[o];
      const float gx = X + 1 < g.W ? (float)x[o + 1] - xz : 0.f;
      const float gy = Y + 1 < g.H ? (float)x[o + g.W] - xz : 0.f;
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

// Gradient-descent baselines (sec 7.1), data part: over t = A x in `lr`,
// r = t - y, q = lambda1 sgn(r) + 2 lambda2 r written back over t, and the
// block's share of lambda1 |r| + lambda2 r^2.
__global__ __launch_bounds__(kThreads) void k_gd_data(Geom g, const float* __restrict__ y, float* __restrict__ lr,
                                                      double* __restrict__ part) {
  const long long n = (long long)g.sk * g.q;
  double acc = 0.0;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < n; o += (long long)gridDim.x * kThreads) {
    const float r = lr[o] - y[o];
    const float sg = (float)((r > 0.f) - (r < 0.f));
    lr[o] = fmaf(2.f * g.lambda2, r, g.lambda1 * sg);
    acc += (double)g.lambda1 * fabs((double)r) + (double)g.lambda2 * (double)r * (double)r;
  }
  double v[1] = {acc};
  block_sum<1, 4>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Regulariser part: at pixel z, the cost share sum_d c_d m(z) |x(z) - x(z+d)|
// and the subgradient S^T sgn(g) = sum_d c_d [m(z) sgn(x(z) - x(z+d))
// - m(z-d) sgn(x(z-d) - x(z))] (pairs leaving the image are dropped;
// sgn(0) = 0).  Plain gathers: a baseline, not a tuned stencil.
__global__ __launch_bounds__(kThreads) void k_gd_tv(Geom g, const float* __restrict__ x, const float* __restrict__ m,
                                                    float* __restrict__ out, double* __restrict__ part) {
  double acc = 0.0;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < g.p; o += (long long)gridDim.x * kThreads) {
    const int Y = (int)(o / g.W), X = (int)(o - (long long)Y * g.W);
    const float xz = x[o], mz = m[o];
    float sub = 0.f, cost = 0.f;
    for (int d = 0; d < g.sd; ++d) {
      const int dy = g.ody[d], dx = g.odx[d];
      const float c = g.cd[d];
      if (Y + dy >= 0 && Y + dy < g.H && X + dx >= 0 && X + dx < g.W) {
        const float df = xz - x[o + (long long)dy * g.W + dx];
        cost = fmaf(c * mz, fabsf(df), cost);
        sub = fmaf(c * mz, (float)((df > 0.f) - (df < 0.f)), sub);
      }
      if (Y - dy >= 0 && Y - dy < g.H && X - dx >= 0 && X - dx < g.W) {
        const long long q = o - (long long)dy * g.W - dx;
        const float df = x[q] - xz;
        sub = fmaf(-c * m[q], (float)((df > 0.f) - (df < 0.f)), sub);
      }
    }
    out[o] = sub;
    acc += (double)cost;
  }
  double v[1] = {acc};
  block_sum<1, 4>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Fixed-order total of one or two partial arrays into a device scalar.
__global__ __launch_bounds__(kThreads) void k_gd_total(const double* __restrict__ p0, int n0,
                                                       const double* __restrict__ p1, int n1,
                                                       double* __restrict__ dst) {
  double a[1], b[1];
  sum_parts<1>(p0, n0, a);
  if (n1 > 0) sum_parts<1>(p1, n1, b);
  else b[0] = 0.0;
  if (threadIdx.x == 0) *dst = a[0] + b[0];
}

// g = a + t and the block's share of |g|^2.
__global__ __launch_bounds__(kThreads) void k_gd_grad(Geom g, const float* __restrict__ a, const float* __restrict__ t,
                                                      float* __restrict__ gout, double* __restrict__ part) {
  double acc = 0.0;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < g.p; o += (long long)gridDim.x * kThreads) {
    const float v = a[o] + t[o];
    gout[o] = v;
    acc += (double)v * (double)v;
  }
  double v[1] = {acc};
  block_sum<1, 4>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// out = x - eta g (out may be x: no restrict on those two)
__global__ __launch_bounds__(kThreads) void k_gd_step(const float* x, const float* __restrict__ gr, float eta,
                                                      float* out, long long n) {
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < n; o += (long long)gridDim.x * kThreads)
    out[o] = fmaf(-eta, gr[o], x[o]);
}

// Occlusion weight (sec 3.4, eq. weight_occ), projection-error part: for one
// view k, acc += (L_ref(z) - L_k(z - theta_k w(z)))^2 at every HR pixel z, with
// L_ref, L_k the bicubic up-sampled views (the x0 operator) and L_k read
// bilinearly at the position clamped to the image.
__global__ __launch_bounds__(kThreads) void k_occ_acc(Geom g, const float* __restrict__ lref,
                                                      const float* __restrict__ lk, const float* __restrict__ disp,
                                                      float tau, float rho, float* __restrict__ acc) {
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < g.p; o += (long long)gridDim.x * kThreads) {
    const int Y = (int)(o / g.W), X = (int)(o - (long long)Y * g.W);
    const float w = disp[o];
    const float py = fminf(fmaxf((float)Y - tau * w, 0.f), (float)(g.H - 1));
    const float px = fminf(fmaxf((float)X - rho * w, 0.f), (float)(g.W - 1));
    const int i0 = (int)floorf(py), j0 = (int)floorf(px);
    const int i1 = min(i0 + 1, g.H - 1), j1 = min(j0 + 1, g.W - 1);
    const float fy = py - (float)i0, fx = px - (float)j0;
    const float* r0 = lk + (size_t)i0 * g.W;
    const float* r1 = lk + (size_t)i1 * g.W;
    const float top = fmaf(fx, r0[j1] - r0[j0], r0[j0]);
    const float bot = fmaf(fx, r1[j1] - r1[j0], r1[j0]);
    const float d = lref[o] - fmaf(fy, bot - top, top);
    acc[o] = fmaf(d, d, acc[o]);
  }
}

// Occlusion weight, final: w_o = exp(-b^2 c1) exp(-(acc / nviews) c2) with b
// the negative part of the forward-difference divergence of the disparity
// map (zero differences at the last row / column); c = 1/(2 sigma^2), 0 for
// a factor that is switched off.
__global__ __launch_bounds__(kThreads) void k_occ_final(Geom g, const float* __restrict__ disp,
                                                        const float* __restrict__ acc, float inv_views, float c1,
                                                        float c2, float* __restrict__ out) {
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < g.p; o += (long long)gridDim.x * kThreads) {
    const int Y = (int)(o / g.W), X = (int)(o - (long long)Y * g.W);
    const float w = disp[o];
    const float gx = X + 1 < g.W ? disp[o + 1] - w : 0.f;
    const float gy = Y + 1 < g.H ? disp[o + g.W] - w : 0.f;
    const float b = fminf(gx + gy, 0.f);
    const float p2 = acc[o] * inv_views;
    out[o] = expf(-b * b * c1) * expf(-p2 * c2);
  }
}

// Input check: non-finite LR / disparity / occlusion values (bit 0) and
// |disp| > disp_bound (bit 1).
__global__ __launch_bounds__(kThreads) void k_check(Geom g, const float* __restrict__ y, const float* __restrict__ disp,
                                                    const float* __restrict__ occ, DevScalars* __restrict__ sc) {
  int f = 0;
  const long long ny = (long long)g.sk * g.q, nd = (long long)g.n_disp * g.p;
  long long n = ny > nd ? ny : nd;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < n; o += (long long)gridDim.x * kThreads) {
    if (o < ny && !isfinite(y[o])) f |= 1;
    if (o < nd) {
      const float d = disp[o];
      if (!isfinite(d)) f |= 1;
      else if (fabsf(d) > g.disp_bound) f |= 2;
    }
    if (o < g.p && occ && !isfinite(occ[o])) f |= 1;
  }
  if (f) atomicOr(&sc->err_flags, f);
}

// Explicit blur kernel, passed by value (so the host copy need not outlive the launch).
struct Taps2D {
  float v[kMax2DTaps * kMax2DTaps];
};
__global__ void k_set_taps(Taps2D t, int n, float* __restrict__ dst) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = t.v[i];
}

// Fill n floats with a value (a kernel rather than hipMemsetAsync, so that
// the sequence stays capturable in a graph).
__global__ __launch_bounds__(kThreads) void k_fill(float* __restrict__ p, long long n, float v) {
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < n; o += (long long)gridDim.x * kThreads) p[o] = v;
}

// Reset the device scalars for a fresh state (iters_done = n_done).
__global__ void k_reset(DevScalars* sc, int n_done) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  sc->pi = 0.0;
  sc->res1 = 0.0;
  sc->res1_set = 0;
  sc->wcur = 0;
  sc->cg_done = 0;
  sc->cg_steps = 0;
  sc->admm_done = 0;
  sc->stop_pending = 0;
  sc->iters_done = n_done;
  sc->err_flags = 0;
}

// Copy the current NLTV dual (selected on the device) out as float.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_copy_ws(const T* __restrict__ ws0, const T* __restrict__ ws1,
                                                      float* __restrict__ out, long long n,
                                                      const DevScalars* __restrict__ sc) {
  const T* s = sc->wcur ? ws1 : ws0;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < n; o += (long long)gridDim.x * kThreads)
    out[o] = (float)s[o];
}

// Element-wise conversion between float and a storage type.
template <typename TI, typename TO>
__global__ __launch_bounds__(kThreads) void k_convert(const TI* __restrict__ in, TO* __restrict__ out, long long n) {
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < n; o += (long long)gridDim.x * kThreads)
    out[o] = (TO)(float)in[o];
}

// Split an FP32 image into a 16-bit part and its FP32 rounding remainder:
// x16 = T(v), dx = v - x16 (exact), so x16 + dx reproduces v bit for bit.
// `src` may alias `dx`.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_split(const float* src, T* __restrict__ x16, float* dx, long long n) {
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < n; o += (long long)gridDim.x * kThreads) {
    const float v = src[o];
    const T t = (T)v;
    x16[o] = t;
    dx[o] = v - (float)t;
  }
}

// End of a 16-bit x-step: fold the FP32 CG accumulation into the stored
// estimate, keeping the new rounding remainder (no stagnation below the
// 16-bit ulp).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fold(Geom g, T* __restrict__ x16, float* __restrict__ dx,
                                                   const DevScalars* __restrict__ sc) {
  if (sc->admm_done) return;
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < g.p; o += (long long)gridDim.x * kThreads) {
    const float v = (float)x16[o] + dx[o];
    const T t = (T)v;
    x16[o] = t;
    dx[o] = v - (float)t;
  }
}

// FP32 estimate x16 + dx of a 16-bit x.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_join(const T* __restrict__ x16, const float* __restrict__ dx,
                                                   float* __restrict__ out, long long n) {
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < n; o += (long long)gridDim.x * kThreads)
    out[o] = (float)x16[o] + dx[o];
}

// Zero n elements of a storage-typed buffer.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_zero(T* __restrict__ p, long long n) {
  for (long long o = blockIdx.x * (long long)kThreads + threadIdx.x; o < n; o += (long long)gridDim.x * kThreads)
    p[o] = (T)0.f;
}

// ---------------------------------------------------------------------------
// Launch helpers (host side).

static inline unsigned grid1d(long long n, long long cap = 4096) {
  long long b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

static inline void fwd_dims(const Geom& g, int& NY, int& NX, int& SY, int& SX) {
  NY = (g.f_tly - 1) * g.zeta + 1 + 2 * g.rb;
  NX = (g.f_tlx - 1) * g.zeta + 1 + 2 * g.rb;
  SY = NY + 2 * g.halo;
  SX = NX + 2 * g.halo;
}

size_t forward_lds(const Geom& g) {
  int NY, NX, SY, SX;
  fwd_dims(g, NY, NX, SY, SX);
  if (g.f_col == 2) return sizeof(float) * (4 * (size_t)SY * SX + 8 * (size_t)g.f_tly * NX);
  if (g.f_col) return sizeof(float) * ((size_t)SY * kColPitch + 4 * (size_t)g.f_tly * NX);
  return sizeof(float) * ((size_t)SY * SX + (size_t)NY * NX + (size_t)NY * g.f_tlx +
                          (g.blur2d ? (size_t)g.kb * g.kb : 0));
}

// (zeta, blur size) pairs with a compiled column-per-lane forward kernel, and
// its lattice rows per tile
static constexpr bool fwdcol_shape(int zeta, int kb) {
  return (zeta == 2 && (kb == 3 || kb == 5 || kb == 7 || kb == 9)) || (zeta == 3 && (kb == 5 || kb == 7 || kb == 9)) ||
         (zeta == 4 && (kb == 7 || kb == 9));
}
static constexpr int fwdcol_tly(int zeta, int kb) { return (void)zeta, (void)kb, 8; }

bool forward_col_setup(Geom& g) {
  // the column kernels hold the lane's disparity column in registers: for
  // one map across all views, for per-view maps (their PV form) reloaded per
  // view; explicit 2-D blur kernels take the tiled kernels
  if (!fwdcol_shape(g.zeta, g.kb) || g.blur2d) return false;
  Geom t = g;
  t.f_col = 1;
  t.f_tly = fwdcol_tly(g.zeta, g.kb);
  const int tmax = (64 - g.kb) / g.zeta + 1;  // NX <= 64
  // the widest tile with the fewest tile columns
  const int ncol = (g.sx + tmax - 1) / tmax;
  t.f_tlx = (g.sx + ncol - 1) / ncol;
  int NY, NX, SY, SX;
  fwd_dims(t, NY, NX, SY, SX);
  // quad cells when two 8-wave blocks fit a CU's LDS and there are views for
  // all eight waves, else the plain 4-wave tile
  Geom q = t;
  q.f_col = 2;
  if (forward_lds(q) <= 80 * 1024 && g.sk >= 8) {
    g = q;
    return true;
  }
  if (SX > kColPitch || forward_lds(t) > 60 * 1024) return false;
  g = t;
  return true;
}

// Orbit walk for the CG form: estimated VALU instructions per lane of a
// block's slowest wave, single views against orbits over the same view groups
// (per blur position: 15 for a view of fwd_walk_q, 47 / 20 / 19 / 5 for an
// orbit of four / a centre-column pair / a centre-row pair / the centre view
// in fwd_walk_orb; per view the horizontal pass, TLY + NO (KB + 3)).  Used
// when the orbits shorten that wave by more than 3 %.
void forward_orbit_setup(Geom& g) {
  g.f_orb = 0;
  if (g.f_col != 2 || g.n_disp != 1 || g.U % 2 == 0 || g.V % 2 == 0 || g.sk < 2) return;
  const int NW = 8, NY = (g.f_tly - 1) * g.zeta + g.kb;
  const int NO = (g.f_tly * ((64 - g.kb) / g.zeta + 1) + 63) / 64;
  const double fin = g.f_tly + NO * (g.kb + 3.0);
  const double c_view = 15.0 * NY + fin;
  const int groups = (g.sk + g.f_vpb - 1) / g.f_vpb;
  const double plain = ((std::min(g.sk, g.f_vpb) + NW - 1) / NW) * c_view;
  const int ca = (g.U - 1) / 2, cc = (g.V - 1) / 2, nq = ca * cc, nit = nq + ca + cc + 1;
  auto cost = [&](int it) {
    if (it < nq) return 47.0 * NY + 4 * fin;
    if (it < nq + ca) return 20.0 * NY + 2 * fin;
    if (it < nq + ca + cc) return 19.0 * NY + 2 * fin;
    return 5.0 * NY + fin;
  };
  const int ipb = (nit + groups - 1) / groups;
  double orb = 0.0;
  for (int z = 0; z < groups; ++z)
    for (int w = 0; w < NW; ++w) {
      double t = 0.0;
      for (int it = z * ipb + w; it < std::min(nit, z * ipb + ipb); it += NW) t += cost(it);
      orb = std::max(orb, t);
    }
  if (orb < 0.97 * plain) g.f_orb = 1;
}

bool forward_tile_ok(const Geom& g) {
  int NY, NX, SY, SX;
  fwd_dims(g, NY, NX, SY, SX);
  return NY * NX <= kThreads * kFwdSlots && NY * g.f_tlx <= kThreads * kFwdHSlots &&
         g.f_tly * g.f_tlx <= kThreads && forward_lds(g) <= 60 * 1024;
}

static inline void adj_dims(const Geom& g, int& ci, int& LY, int& LX, int& MM, int& PAD) {
  ci = (g.rb + g.zeta - 1) / g.zeta;
  LY = g.a_tly + 2 * ci;
  LX = g.a_tlx + 2 * ci;
  MM = (2 * g.rb) / g.zeta + 1;
  PAD = g.zeta * MM;
}

size_t adjoint_lds(const Geom& g) {
  if (g.a_col) {
    const int z = g.zeta, CF = g.rb / z;
    const int RL = (g.a_th - 1 + g.rb) / z + CF + 1, LXc = (g.a_tw - 1 + g.rb) / z + CF + 1;
    return 4 * (size_t)g.a_ey * kColPitch + sizeof(float) * 4 * (size_t)RL * LXc;
  }
  int ci, LY, LX, MM, PAD;
  adj_dims(g, ci, LY, LX, MM, PAD);
  const int RH = g.a_th / 4, RL = RH / g.zeta + 2 * ci;
  const size_t ets = (size_t)(RL + MM) * LX, hvs = (size_t)RH * LX + MM;
  return sizeof(float) * (2 * (size_t)g.a_ey * g.a_ex + PAD + g.kb + 4 * (ets + hvs) +
                          (g.blur2d ? (size_t)g.kb * g.kb : 0));
}

bool adjoint_tile_ok(const Geom& g) {
  int ci, LY, LX, MM, PAD;
  adj_dims(g, ci, LY, LX, MM, PAD);
  if (g.a_tly % 4 != 0) return false;  // each wave owns a whole number of LR rows
  const int RH = g.a_th / 4, RL = RH / g.zeta + 2 * ci;
  return g.a_th >= g.halo && g.a_tw >= g.halo && RH * g.a_tw <= 64 * kAdjSlots && RH * LX <= 64 * kAdjVSlots &&
         RL * LX <= 64 * kAdjESlots && adjoint_lds(g) <= 60 * 1024;
}

size_t tv_lds(const Geom& g) {
  return sizeof(float) * 2 * (size_t)(kTvTileX + 2 * g.rw) * (kTvTileY + 2 * g.rw);
}

dim3 forward_grid(const Geom& g) {
  return dim3((g.sx + g.f_tlx - 1) / g.f_tlx, (g.sy + g.f_tly - 1) / g.f_tly, (g.sk + g.f_vpb - 1) / g.f_vpb);
}
dim3 adjoint_grid(const Geom& g) { return dim3(g.a_ntx, g.a_nty, g.a_vg); }

static constexpr bool adjcol_shape(int zeta, int kb) { return fwdcol_shape(zeta, kb); }

bool adjoint_col_setup(Geom& g) {
  if (!adjcol_shape(g.zeta, g.kb) || g.blur2d) return false;
  Geom t = g;
  t.a_col = 1;
  t.a_th = adjcol_th(g.zeta);
  t.a_tw = adjcol_tw(g.zeta);
  if (g.halo > t.a_th || g.halo > t.a_tw) return false;  // partial images may overlap only neighbouring tiles
  t.a_tly = t.a_th / g.zeta;
  t.a_tlx = t.a_tw / g.zeta;
  t.a_ey = t.a_th + 2 * g.halo;
  t.a_ex = t.a_tw + 2 * g.halo;
  if (t.a_ex > kColPitch) return false;
  const size_t lds = adjoint_lds(t);
  if (lds > 64 * 1024) return false;
  t.a_nty = (g.H + t.a_th - 1) / t.a_th;
  t.a_ntx = (g.W + t.a_tw - 1) / t.a_tw;
  t.a_inv_th = (float)(1.0 / t.a_th);
  t.a_inv_tw = (float)(1.0 / t.a_tw);
  // view groups: a block's time grows with its view passes (its four waves
  // take views in parallel, so ceil(views / 4) passes), a launch takes
  // ceil(blocks / resident slots) rounds, and every extra group adds a set of
  // partial images to merge; pick the group count with the lowest estimate
  long long per_cu = (long long)((160 * 1024) / lds);
  if (per_cu > 4) per_cu = 4;  // ~100 VGPRs: four waves per SIMD
  if (g.n_disp > 1 && per_cu > 3) per_cu = 3;  // per-view maps: ~150 VGPRs, three
  if (per_cu < 1) per_cu = 1;
  const long long slots = 256 * per_cu, tiles = (long long)t.a_nty * t.a_ntx;
  int best_g = 1;
  double best = 1e30;
  const double passes1 = (double)((g.sk + 3) / 4);
  for (int G = 1; G <= 8 && G <= g.sk; ++G) {
    const double rounds = (double)((tiles * G + slots - 1) / slots);
    const double passes = (double)(((g.sk + G - 1) / G + 3) / 4);
    const double cost = rounds * passes / passes1 + 0.05 * G;
    if (cost < best - 1e-12) {
      best = cost;
      best_g = G;
    }
  }
  t.a_vpb = (g.sk + best_g - 1) / best_g;
  t.a_vg = (g.sk + t.a_vpb - 1) / t.a_vpb;
  g = t;
  return true;
}
dim3 tv_grid(const Geom& g) { return dim3((g.W + kTvTileX - 1) / kTvTileX, (g.H + kTvTileY - 1) / kTvTileY, 1); }

static inline int nblocks(dim3 d) { return (int)(d.x * d.y * d.z); }

// Calls f with a null pointer of the storage element type `st`.
template <class F>
static void by_storage(int st, F&& f) {
  switch (st) {
    case kStF16: f((_Float16*)nullptr); break;
    case kStBF16: f((__bf16*)nullptr); break;
    default: f((float*)nullptr); break;
  }
}
#define LFSR_ELEM(tag) std::remove_pointer_t<decltype(tag)>

template <bool WZD, typename TS, typename TO>
static void launch_fwd_kb(const Geom& g, const TS* src, const float* disp, TO* out, const float* y, TO* wD,
                          double* part, float* pmax, const DevScalars* sc, int gate, hipStream_t s) {
  const dim3 grid = forward_grid(g), blk(kThreads);
  const size_t lds = forward_lds(g);
  if (g.f_col) {
#define LFSR_FWC_PV(Z, K, PV)                                                                                     \
  do {                                                                                                            \
    constexpr int TL = fwdcol_tly(Z, K);                                                                          \
    if constexpr (!WZD && !PV)                                                                                    \
      if (g.f_orb) {                                                                                              \
        hipLaunchKernelGGL((k_fwdcol<WZD, Z, K, TL, TS, TO, true, false, true>), grid, dim3(2 * kThreads), lds,   \
                           s, g, src, disp, out, y, wD, part, pmax, sc, gate);                                    \
        break;                                                                                                    \
      }                                                                                                           \
    if (g.f_col == 2)                                                                                             \
      hipLaunchKernelGGL((k_fwdcol<WZD, Z, K, TL, TS, TO, true, PV>), grid, dim3(2 * kThreads), lds, s, g, src,   \
                         disp, out, y, wD, part, pmax, sc, gate);                                                 \
    else                                                                                                          \
      hipLaunchKernelGGL((k_fwdcol<WZD, Z, K, TL, TS, TO, false, PV>), grid, blk, lds, s, g, src, disp, out, y,   \
                         wD, part, pmax, sc, gate);                                                               \
  } while (0)
#define LFSR_FWC(Z, K)                                    \
  if (g.zeta == Z && g.kb == K) {                         \
    if (g.n_disp > 1) LFSR_FWC_PV(Z, K, true);            \
    else LFSR_FWC_PV(Z, K, false);                        \
    return;                                                \
  }
    LFSR_FWC(2, 3) LFSR_FWC(2, 5) LFSR_FWC(2, 7) LFSR_FWC(2, 9) LFSR_FWC(3, 5) LFSR_FWC(3, 7) LFSR_FWC(3, 9)
    LFSR_FWC(4, 7) LFSR_FWC(4, 9)
#undef LFSR_FWC
#undef LFSR_FWC_PV
    return;  // unreachable: forward_col_setup admits only the shapes above
  }
#define LFSR_FWD(KB) \
  hipLaunchKernelGGL((k_forward<WZD, KB, TS, TO>), grid, blk, lds, s, g, src, disp, out, y, wD, part, pmax, sc, gate)
  switch (g.kb) {
    case 1: LFSR_FWD(1); break;
    case 3: LFSR_FWD(3); break;
    case 5: LFSR_FWD(5); break;
    case 7: LFSR_FWD(7); break;
    case 9: LFSR_FWD(9); break;
    case 11: LFSR_FWD(11); break;
    case 13: LFSR_FWD(13); break;
    default: LFSR_FWD(0); break;
  }
#undef LFSR_FWD
}

void launch_forward(const Geom& g, const float* src, const float* disp, float* out, hipStream_t s,
                    const Bufs& b, int gate) {
  launch_fwd_kb<false>(g, src, disp, out, (const float*)nullptr, (float*)nullptr, nullptr, b.p_max, b.sc, gate, s);
}

void launch_forward_cg(const Geom& g, const float* src, const float* disp, hipStream_t s, const Bufs& b, int gate) {
  by_storage(b.st, [&](auto* tag) {
    using T = LFSR_ELEM(tag);
    launch_fwd_kb<false>(g, src, disp, (T*)b.lr, (const float*)nullptr, (T*)nullptr, nullptr, b.p_max, b.sc, gate, s);
  });
}

void launch_forward_wzd(const Geom& g, const float* disp, const float* y, hipStream_t s, const Bufs& b) {
  by_storage(b.st, [&](auto* tag) {
    using T = LFSR_ELEM(tag);
    launch_fwd_kb<true>(g, (const T*)b.x, disp, (T*)b.lr, y, (T*)b.wD, b.p_wzd, b.p_max, b.sc, (int)kGateAdmm, s);
  });
}

void launch_adjoint(const Geom& g, const void* lr, int lr_st, const float* disp, hipStream_t s, const Bufs& b,
                    int gate, int npmax) {
  const int MM = (2 * g.rb) / g.zeta + 1;
  const dim3 grid = adjoint_grid(g), blk(kThreads);
  const size_t lds = adjoint_lds(g);
  const float* pm = b.p_max;
  const DevScalars* sc = b.sc;
  by_storage(lr_st, [&](auto* tag) {
    using T = LFSR_ELEM(tag);
    const T* in = (const T*)lr;
    if (g.a_col) {
#define LFSR_ADC(Z, K)                                                                                          \
  if (g.zeta == Z && g.kb == K) {                                                                               \
    if (g.n_disp > 1)                                                                                           \
      hipLaunchKernelGGL((k_adjcol<Z, K, T, true>), grid, blk, lds, s, g, in, disp, b.adj, pm, npmax, b.p_cnt,  \
                         sc, gate);                                                                             \
    else                                                                                                        \
      hipLaunchKernelGGL((k_adjcol<Z, K, T, false>), grid, blk, lds, s, g, in, disp, b.adj, pm, npmax, b.p_cnt, \
                         sc, gate);                                                                             \
    return;                                                                                                     \
  }
      LFSR_ADC(2, 3) LFSR_ADC(2, 5) LFSR_ADC(2, 7) LFSR_ADC(2, 9) LFSR_ADC(3, 5) LFSR_ADC(3, 7) LFSR_ADC(3, 9)
      LFSR_ADC(4, 7) LFSR_ADC(4, 9)
#undef LFSR_ADC
      return;  // unreachable: adjoint_col_setup admits only the shapes above
    }
#define LFSR_ADJ(M) hipLaunchKernelGGL((k_adjoint<M, T>), grid, blk, lds, s, g, in, disp, b.adj, pm, npmax, sc, gate)
    switch (MM) {
      case 1: LFSR_ADJ(1); break;
      case 2: LFSR_ADJ(2); break;
      case 3: LFSR_ADJ(3); break;
      case 4: LFSR_ADJ(4); break;
      case 5: LFSR_ADJ(5); break;
      case 6: LFSR_ADJ(6); break;
      case 7: LFSR_ADJ(7); break;
      default: LFSR_ADJ(0); break;
    }
#undef LFSR_ADJ
  });
}

int launch_absmax(const Geom& g, const float* v, long long n, hipStream_t s, const Bufs& b) {
  const unsigned nb = grid1d(n, kRedBlocks);
  hipLaunchKernelGGL(k_absmax, dim3(nb), dim3(kThreads), 0, s, v, n, b.p_max);
  return (int)nb;
}

int forward_blocks(const Geom& g) { return nblocks(forward_grid(g)); }

void launch_adjcount(const Geom& g, const float* disp, hipStream_t s, const Bufs& b) {
  if (!g.a_col) return;
  const dim3 grid = adjoint_grid(g), blk(kThreads);
  const size_t lds = 4 * (size_t)g.a_ey * g.a_ex;
#define LFSR_CNT(Z, K)                                                                   \
  if (g.zeta == Z && g.kb == K) {                                                        \
    if (g.n_disp > 1)                                                                    \
      hipLaunchKernelGGL((k_adjcount<Z, K, true>), grid, blk, lds, s, g, disp, b.p_cnt); \
    else                                                                                 \
      hipLaunchKernelGGL((k_adjcount<Z, K, false>), grid, blk, lds, s, g, disp, b.p_cnt); \
    return;                                                                              \
  }
  LFSR_CNT(2, 3) LFSR_CNT(2, 5) LFSR_CNT(2, 7) LFSR_CNT(2, 9) LFSR_CNT(3, 5) LFSR_CNT(3, 7) LFSR_CNT(3, 9)
  LFSR_CNT(4, 7) LFSR_CNT(4, 9)
#undef LFSR_CNT
}

void launch_merge(const Geom& g, float* out, hipStream_t s, const Bufs& b, int gate) {
  hipLaunchKernelGGL(k_merge, dim3(grid1d(g.p)), dim3(kThreads), 0, s, g, (const float*)b.adj, out,
                     (const DevScalars*)b.sc, gate);
}

void launch_tv(const Geom& g, hipStream_t s, const Bufs& b) {
  by_storage(b.st, [&](auto* tag) {
    using T = LFSR_ELEM(tag);
#define LFSR_TV(R)                                                                                                 \
  hipLaunchKernelGGL((k_tv<T, R>), dim3(8 * ((nblocks(tv_grid(g)) + 7) / 8)), dim3(kTvThreads), tv_lds(g), s, g, (const T*)b.x, (const float*)b.m, \
                     (T*)b.wS[0], (T*)b.wS[1], b.vs, b.p_tv, (const DevScalars*)b.sc)
    switch (g.rw) {
      case 1: LFSR_TV(1); break;
      case 2: LFSR_TV(2); break;
      case 3: LFSR_TV(3); break;
      default: LFSR_TV(0); break;
    }
#undef LFSR_TV
  });
}

bool merge_fusable(const Geom& g) {
  return g.a_col && g.rw >= 1 && g.rw <= 3 && 2 * g.halo <= g.a_th && 2 * g.halo <= g.a_tw && g.a_vg <= 8;
}

void launch_hp(const Geom& g, const float* pv, const float* m, float* out, hipStream_t s, const Bufs& b, int gate,
               int with_dot, int fused) {
#define LFSR_HPS(R)                                                                                        \
  hipLaunchKernelGGL(k_hpstrip<R>, tv_grid(g), dim3(kThreads), tv_lds(g), s, g, pv, m, out, (const float*)b.adj, \
                     b.p_php, (const DevScalars*)b.sc, gate, with_dot, fused)
  switch (g.rw) {
    case 1: LFSR_HPS(1); break;
    case 2: LFSR_HPS(2); break;
    case 3: LFSR_HPS(3); break;
    default:
      hipLaunchKernelGGL(k_hp<0>, tv_grid(g), dim3(kThreads), tv_lds(g), s, g, pv, m, out, b.p_php,
                         (const DevScalars*)b.sc, gate, with_dot);
      break;
  }
#undef LFSR_HPS
}

void launch_cginit(const Geom& g, hipStream_t s, const Bufs& b, int fused) {
  hipLaunchKernelGGL(k_cginit, dim3(g.red_blocks), dim3(kCgThreads), 0, s, g, (const float*)b.vs, b.r, b.pv,
                     b.p_rr[0], (const double*)b.p_wzd, nblocks(forward_grid(g)),
                     (const double*)b.p_tv, nblocks(tv_grid(g)), b.stats, b.sc, (const float*)b.adj, fused);
}

void launch_cgupd(const Geom& g, int step, hipStream_t s, const Bufs& b) {
  float* xacc = b.st == kStF32 ? (float*)b.x : b.dx;
  hipLaunchKernelGGL(k_cgupd, dim3(g.red_blocks), dim3(kCgThreads), 0, s, g, xacc, b.r, (const float*)b.pv,
                     (const float*)b.hp, (const double*)b.p_rr[(step - 1) & 1], b.p_rr[step & 1],
                     (const double*)b.p_php, nblocks(tv_grid(g)), step, b.sc);
}

void launch_cgp(const Geom& g, int step, hipStream_t s, const Bufs& b) {
  hipLaunchKernelGGL(k_cgp, dim3(g.red_blocks), dim3(kCgThreads), 0, s, g, (const float*)b.r, b.pv,
                     (const double*)b.p_rr[(step - 1) & 1], (const double*)b.p_rr[step & 1],
                     (const DevScalars*)b.sc);
}

void launch_iter_end(const Geom& g, hipStream_t s, const Bufs& b) {
  hipLaunchKernelGGL(k_iter_end, dim3(1), dim3(kThreads), 0, s, g, (const double*)b.p_rr[0],
                     (const double*)b.p_rr[1], b.stats, b.sc);
}

void launch_edge(const Geom& g, const void* x, int x_st, const float* occ, float* m, hipStream_t s, const Bufs& b,
                 int gate) {
  by_storage(x_st, [&](auto* tag) {
    using T = LFSR_ELEM(tag);
    hipLaunchKernelGGL(k_edge<T>, dim3(grid1d(g.p)), dim3(kThreads), 0, s, g, (const T*)x, occ, m,
                       (const DevScalars*)b.sc, gate);
  });
}

void launch_fold(const Geom& g, hipStream_t s, const Bufs& b) {
  if (b.st == kStF32) return;
  by_storage(b.st, [&](auto* tag) {
    using T = LFSR_ELEM(tag);
    hipLaunchKernelGGL(k_fold<T>, dim3(grid1d(g.p)), dim3(kThreads), 0, s, g, (T*)b.x, b.dx, (const DevScalars*)b.sc);
  });
}

void launch_split(const Geom& g, const float* src, hipStream_t s, const Bufs& b) {
  by_storage(b.st, [&](auto* tag) {
    using T = LFSR_ELEM(tag);
    hipLaunchKernelGGL(k_split<T>, dim3(grid1d(g.p)), dim3(kThreads), 0, s, src, (T*)b.x, b.dx, (long long)g.p);
  });
}

void launch_join(const Geom& g, float* out, hipStream_t s, const Bufs& b) {
  by_storage(b.st, [&](auto* tag) {
    using T = LFSR_ELEM(tag);
    hipLaunchKernelGGL(k_join<T>, dim3(grid1d(g.p)), dim3(kThreads), 0, s, (const T*)b.x, (const float*)b.dx, out,
                       (long long)g.p);
  });
}

void launch_to_float(const void* in, int st, float* out, long long n, hipStream_t s) {
  if (n <= 0) return;
  by_storage(st, [&](auto* tag) {
    using T = LFSR_ELEM(tag);
    hipLaunchKernelGGL((k_convert<T, float>), dim3(grid1d(n)), dim3(kThreads), 0, s, (const T*)in, out, n);
  });
}

void launch_from_float(const float* in, void* out, int st, long long n, hipStream_t s) {
  if (n <= 0) return;
  by_storage(st, [&](auto* tag) {
    using T = LFSR_ELEM(tag);
    hipLaunchKernelGGL((k_convert<float, T>), dim3(grid1d(n)), dim3(kThreads), 0, s, in, (T*)out, n);
  });
}

void launch_zero(void* p, int st, long long n, hipStream_t s) {
  if (n <= 0) return;
  by_storage(st, [&](auto* tag) {
    using T = LFSR_ELEM(tag);
    hipLaunchKernelGGL(k_zero<T>, dim3(grid1d(n)), dim3(kThreads), 0, s, (T*)p, n);
  });
}

void launch_bicubic(const Geom& g, const float* lrv, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_bicubic, dim3(grid1d(g.p)), dim3(kThreads), 0, s, g, lrv, out);
}

void launch_gd_cost(const Geom& g, const float* xp, const float* disp, const float* y, hipStream_t s, const Bufs& b) {
  float* lr = (float*)b.lr;
  launch_forward(g, xp, disp, lr, s, b, 0);
  const unsigned nb = (unsigned)g.red_blocks;
  hipLaunchKernelGGL(k_gd_data, dim3(nb), dim3(kThreads), 0, s, g, y, lr, b.p_rr[0]);
  if (g.sd > 0)
    hipLaunchKernelGGL(k_gd_tv, dim3(nb), dim3(kThreads), 0, s, g, xp, (const float*)b.m, b.hp, b.p_rr[1]);
  else
    launch_fill(b.hp, g.p, 0.f, s);
  hipLaunchKernelGGL(k_gd_total, dim3(1), dim3(kThreads), 0, s, (const double*)b.p_rr[0], (int)nb,
                     (const double*)b.p_rr[1], g.sd > 0 ? (int)nb : 0, &b.sc->gd_cost);
}

void launch_gd_grad(const Geom& g, const float* disp, hipStream_t s, const Bufs& b) {
  const float* q = (const float*)b.lr;
  const int npmax = launch_absmax(g, q, (long long)g.sk * g.q, s, b);
  launch_adjoint(g, q, kStF32, disp, s, b, 0, npmax);
  launch_merge(g, b.r, s, b, 0);
  const unsigned nb = (unsigned)g.red_blocks;
  hipLaunchKernelGGL(k_gd_grad, dim3(nb), dim3(kThreads), 0, s, g, (const float*)b.r, (const float*)b.hp, b.pv,
                     b.p_rr[0]);
  hipLaunchKernelGGL(k_gd_total, dim3(1), dim3(kThreads), 0, s, (const double*)b.p_rr[0], (int)nb,
                     (const double*)nullptr, 0, &b.sc->gd_gnorm);
}

void launch_gd_step(const Geom& g, const float* x, float eta, float* out, hipStream_t s, const Bufs& b) {
  (void)b;
  hipLaunchKernelGGL(k_gd_step, dim3(grid1d(g.p)), dim3(kThreads), 0, s, x, (const float*)b.pv, eta, out,
                     (long long)g.p);
}

void launch_occ_acc(const Geom& g, const float* lref, const float* lk, const float* disp, int k, float* acc,
                    hipStream_t s) {
  const int a = k / g.V, c = k - a * g.V;
  const float tau = (float)(a - (g.U - 1) / 2), rho = (float)(c - (g.V - 1) / 2);
  hipLaunchKernelGGL(k_occ_acc, dim3(grid1d(g.p)), dim3(kThreads), 0, s, g, lref, lk, disp, tau, rho, acc);
}

void launch_occ_final(const Geom& g, const float* disp, const float* acc, float inv_views, float c1, float c2,
                      float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_occ_final, dim3(grid1d(g.p)), dim3(kThreads), 0, s, g, disp, acc, inv_views, c1, c2, out);
}

void launch_check(const Geom& g, const float* y, const float* disp, const float* occ, hipStream_t s, const Bufs& b) {
  long long n = (long long)g.sk * g.q;
  if (n < (long long)g.n_disp * g.p) n = (long long)g.n_disp * g.p;
  hipLaunchKernelGGL(k_check, dim3(grid1d(n)), dim3(kThreads), 0, s, g, y, disp, occ, b.sc);
}

void launch_fill(float* p, long long n, float v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(grid1d(n)), dim3(kThreads), 0, s, p, n, v);
}

void launch_set_taps(const Geom& g, const float* host_taps, hipStream_t s) {
  Taps2D t{};
  const int n = g.kb * g.kb;
  for (int i = 0; i < n; ++i) t.v[i] = host_taps[i];
  hipLaunchKernelGGL(k_set_taps, dim3(1), dim3(256), 0, s, t, n, const_cast<float*>(g.taps2d));
}

void launch_reset(int n_done, hipStream_t s, const Bufs& b) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, b.sc, n_done);
}

void launch_copy_ws(float* out, long long n, hipStream_t s, const Bufs& b) {
  if (n <= 0) return;
  by_storage(b.st, [&](auto* tag) {
    using T = LFSR_ELEM(tag);
    hipLaunchKernelGGL(k_copy_ws<T>, dim3(grid1d(n)), dim3(kThreads), 0, s, (const T*)b.wS[0], (const T*)b.wS[1],
                       out, n, (const DevScalars*)b.sc);
  });
}
#undef LFSR_ELEM

}  // namespace lfsr
