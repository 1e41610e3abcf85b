/*
 * lfsr_oracle.c -- FP64 CPU oracle for the ADMM light-field super-resolution
 * method of "GPU-accelerated light-field super-resolution" (arXiv 2206.05047).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
 * reference that the HIP path is checked against.  Only the test-suite, the
 * smoke entry and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or helper with the HIP library.
 *
 * Everything is double precision, plain loops, no tiling and no fusion beyond
 * evaluating a composition only where the next operator reads it (D keeps only
 * the lattice samples of B(.), so B is evaluated there only).  OpenMP is used
 * over independent views / rows; every reduction is serial and in a fixed
 * order, so results are reproducible for a fixed thread count.
 *
 * Conventions (the readings of the paper this oracle takes):
 *   - HR image x is [H][W] row-major, H = zeta*sy, W = zeta*sx.
 *   - Views k = a*V + b over the U x V angular grid (U, V odd); the angular
 *     offset of view k from the centre (reference) view is
 *     tau_k = a - (U-1)/2 (rows), rho_k = b - (V-1)/2 (columns)      (sec 3.1).
 *   - W_k x(Y,X) = bilinear sample of x at (Y + tau_k*w, X + rho_k*w) with
 *     w = disparity map of view k (n_disp == sk) or of the reference view
 *     (n_disp == 1); taps outside the image contribute zero         (sec 4.1).
 *   - W_k^T is the exact transpose of W_k (a scatter with the same weights).
 *   - B: zero-padded 'same' correlation with a normalised kb x kb Gaussian,
 *     B^T its transpose                                              (sec 4.1).
 *   - D picks the top-left pixel of each zeta x zeta block, D^T puts it back
 *                                                                      (sec 4.1).
 *   - NLTV offsets d = (dy,dx) run row-major over the win x win window minus
 *     the centre; g_d(z) = V_d(z)(x(z) - x(z+d)) if z+d lies in the image,
 *     else 0; V_d(z) = c_d m(z), c_d = exp(-|d|^2/sigma_s),
 *     m = w_e * w_o, w_e(z) = exp(-|grad x(z)|^2/sigma_e) with forward
 *     differences (zero at the last row/column)                       (sec 3.4, 4.1).
 *   - The occlusion weight w_o (eq. weight_occ) is computed from the LR views
 *     and the reference view's disparity map by orc_occlusion_weight (below). 
 *   - The ADMM loop is the reordered one of sec 5, Algorithm 1, in the
 *     unscaled per-block form (valid for lambda2 = 0 as well), with the x-step
 *     solved by the conjugate-gradient loop of Algorithm 2 on the normal
 *     equations (sec 5).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int32_t U, V;          /* angular grid rows, cols */
  int32_t sy, sx, zeta;  /* LR size and scale factor */
  int32_t n_disp;        /* 1: one map (reference view) for all views; U*V: one per view */
  int32_t kb;            /* blur size (odd) */
  double sigma_b;        /* blur std-dev */
  double lambda1, lambda2;
  int32_t win;           /* NLTV window (odd); 1 = no regulariser */
  double sigma_s, sigma_e;  /* sigma_e <= 0 or inf: no edge weight */
  int32_t reweight;      /* 1: edge weight recomputed every ADMM iteration */
  double theta;          /* ADMM penalty (vartheta) */
  int32_t cg_iter;       /* K */
  double cg_tol;         /* tau */
  int32_t weight_kind;   /* spatial weight: 0 exp(-|d|^2/sigma_s); 1 BTV sigma_s^(|dy|+|dx|) */
  const double* blur_taps;  /* NULL: the Gaussian below; else the kb x kb correlation kernel, row-major */
} orc_params;

/* ------------------------------------------------------------------ sizes */

static int64_t hr_h(const orc_params* p) { return (int64_t)p->zeta * p->sy; }
static int64_t hr_w(const orc_params* p) { return (int64_t)p->zeta * p->sx; }
static int64_t n_hr(const orc_params* p) { return hr_h(p) * hr_w(p); }
static int64_t n_lr(const orc_params* p) { return (int64_t)p->sy * p->sx; }
static int n_views(const orc_params* p) { return p->U * p->V; }
static int n_offsets(const orc_params* p) { return p->win * p->win - 1; }

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Angular offset of view k from the reference view (sec 3.1: the SAIs are a
 * 1-D set of s_k observations taken from the 2-D angular grid).  The
 * reference is the centre view of an odd grid; an even grid (the multi-image
 * workload: 2 x 2 images) takes offsets 0 .. U-1 - (U-1)/2 from view
 * ((U-1)/2, (V-1)/2). */
void orc_view_offset(const orc_params* p, int k, int* tau, int* rho) {
  *tau = k / p->V - (p->U - 1) / 2;
  *rho = k % p->V - (p->V - 1) / 2;
}

/* The reference view: the one with angular offset (0, 0). */
int orc_ref_view(const orc_params* p) { return ((p->U - 1) / 2) * p->V + (p->V - 1) / 2; }

static const double* disp_of(const orc_params* p, const double* disp, int k) {
  return p->n_disp == 1 ? disp : disp + (int64_t)k * n_hr(p);
}

/* ------------------------------------------------------------ blur kernel */

/* sec 4.1: B is a Gaussian kernel; we take the 2-D kernel
 * h(a,b) ~ exp(-(a^2+b^2)/(2 sigma^2)) on the kb x kb grid, normalised to 1.
 * sec 7.1 models motion blur by another convolution kernel for B: given
 * explicitly (blur_taps), it is used as is, with no symmetry assumed. */
void orc_blur_kernel(const orc_params* p, double* h) {
  if (p->blur_taps) {
    memcpy(h, p->blur_taps, sizeof(double) * p->kb * p->kb);
    return;
  }
  int r = p->kb / 2;
  double s = 0.0;
  for (int a = -r; a <= r; ++a)
    for (int b = -r; b <= r; ++b) {
      double v = exp(-(double)(a * a + b * b) / (2.0 * p->sigma_b * p->sigma_b));
      h[(a + r) * p->kb + (b + r)] = v;
      s += v;
    }
  for (int i = 0; i < p->kb * p->kb; ++i) h[i] /= s;
}

/* ------------------------------------------------------------ warp W_k */

/* sec 4.1: the forward warp takes the reference-view image to view k:
 * W_k x(z) = x(z + theta_k * w(z)), sampled bilinearly. */
void orc_warp(const orc_params* p, const double* x, const double* disp, int k, double* out) {
  int64_t H = hr_h(p), W = hr_w(p);
  int tau, rho;
  orc_view_offset(p, k, &tau, &rho);
  const double* w = disp_of(p, disp, k);
#pragma omp parallel for schedule(static)
  for (int64_t Y = 0; Y < H; ++Y)
    for (int64_t X = 0; X < W; ++X) {
      double om = w[Y * W + X];
      double sy = (double)Y + tau * om, sx = (double)X + rho * om;
      double fy0 = floor(sy), fx0 = floor(sx);
      int64_t i0 = (int64_t)fy0, j0 = (int64_t)fx0;
      double fy = sy - fy0, fx = sx - fx0;
      double acc = 0.0;
      for (int di = 0; di < 2; ++di)
        for (int dj = 0; dj < 2; ++dj) {
          int64_t i = i0 + di, j = j0 + dj;
          if (i < 0 || i >= H || j < 0 || j >= W) continue;
          double wt = (di ? fy : 1.0 - fy) * (dj ? fx : 1.0 - fx);
          acc += wt * x[i * W + j];
        }
      out[Y * W + X] = acc;
    }
}

/* Exact transpose of orc_warp: every source pixel (Y,X) of the view-k image
 * sends u(Y,X) times each bilinear weight back to the tap it was read from.
 * Accumulates into out (serial: taps of different pixels may coincide). */
void orc_warp_t_acc(const orc_params* p, const double* u, const double* disp, int k, double* out) {
  int64_t H = hr_h(p), W = hr_w(p);
  int tau, rho;
  orc_view_offset(p, k, &tau, &rho);
  const double* w = disp_of(p, disp, k);
  for (int64_t Y = 0; Y < H; ++Y)
    for (int64_t X = 0; X < W; ++X) {
      double om = w[Y * W + X];
      double sy = (double)Y + tau * om, sx = (double)X + rho * om;
      double fy0 = floor(sy), fx0 = floor(sx);
      int64_t i0 = (int64_t)fy0, j0 = (int64_t)fx0;
      double fy = sy - fy0, fx = sx - fx0;
      double val = u[Y * W + X];
      for (int di = 0; di < 2; ++di)
        for (int dj = 0; dj < 2; ++dj) {
          int64_t i = i0 + di, j = j0 + dj;
          if (i < 0 || i >= H || j < 0 || j >= W) continue;
          double wt = (di ? fy : 1.0 - fy) * (dj ? fx : 1.0 - fx);
          out[i * W + j] += wt * val;
        }
    }
}

/* ------------------------------------------------------------ blur B, B^T */

/* B u (Y,X) = sum_{a,b} h(a,b) u(Y+a, X+b), a,b in [-r, r], zero outside. */
void orc_blur(const orc_params* p, const double* u, double* out) {
  int64_t H = hr_h(p), W = hr_w(p);
  int r = p->kb / 2;
  double* h = malloc(sizeof(double) * p->kb * p->kb);
  orc_blur_kernel(p, h);
#pragma omp parallel for schedule(static)
  for (int64_t Y = 0; Y < H; ++Y)
    for (int64_t X = 0; X < W; ++X) {
      double acc = 0.0;
      for (int a = -r; a <= r; ++a)
        for (int b = -r; b <= r; ++b) {
          int64_t i = Y + a, j = X + b;
          if (i < 0 || i >= H || j < 0 || j >= W) continue;
          acc += h[(a + r) * p->kb + (b + r)] * u[i * W + j];
        }
      out[Y * W + X] = acc;
    }
  free(h);
}

/* B^T: the transpose of orc_blur, written as the scatter it is. */
void orc_blur_t(const orc_params* p, const double* u, double* out) {
  int64_t H = hr_h(p), W = hr_w(p);
  int r = p->kb / 2;
  double* h = malloc(sizeof(double) * p->kb * p->kb);
  orc_blur_kernel(p, h);
  memset(out, 0, sizeof(double) * H * W);
  for (int64_t Y = 0; Y < H; ++Y)
    for (int64_t X = 0; X < W; ++X)
      for (int a = -r; a <= r; ++a)
        for (int b = -r; b <= r; ++b) {
          int64_t i = Y + a, j = X + b;
          if (i < 0 || i >= H || j < 0 || j >= W) continue;
          out[i * W + j] += h[(a + r) * p->kb + (b + r)] * u[Y * W + X];
        }
  free(h);
}

/* ------------------------------------------------------------ D, D^T */

/* sec 4.1: D keeps the top-left pixel of every zeta x zeta block. */
void orc_down(const orc_params* p, const double* u, double* out) {
  int64_t W = hr_w(p);
  for (int64_t i = 0; i < p->sy; ++i)
    for (int64_t j = 0; j < p->sx; ++j) out[i * p->sx + j] = u[(i * p->zeta) * W + j * p->zeta];
}

/* D^T puts each LR sample back at its block's top-left pixel, zeros elsewhere. */
void orc_up(const orc_params* p, const double* lr, double* out) {
  int64_t W = hr_w(p);
  memset(out, 0, sizeof(double) * n_hr(p));
  for (int64_t i = 0; i < p->sy; ++i)
    for (int64_t j = 0; j < p->sx; ++j) out[(i * p->zeta) * W + j * p->zeta] = lr[i * p->sx + j];
}

/* ------------------------------------------------------------ A_k, A^T */

/* sec 3.1: A_k = D B W_k for every view.  out is [sk][sy][sx].  B is
 * evaluated only at the lattice points D keeps. */
void orc_forward(const orc_params* p, const double* x, const double* disp, double* out) {
  int64_t H = hr_h(p), W = hr_w(p), q = n_lr(p);
  int r = p->kb / 2, sk = n_views(p);
  double* h = malloc(sizeof(double) * p->kb * p->kb);
  orc_blur_kernel(p, h);
  double* wx = malloc(sizeof(double) * H * W);
  for (int k = 0; k < sk; ++k) {
    orc_warp(p, x, disp, k, wx);
    double* o = out + (int64_t)k * q;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < p->sy; ++i)
      for (int64_t j = 0; j < p->sx; ++j) {
        int64_t Y = i * p->zeta, X = j * p->zeta;
        double acc = 0.0;
        for (int a = -r; a <= r; ++a)
          for (int b = -r; b <= r; ++b) {
            int64_t ii = Y + a, jj = X + b;
            if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
            acc += h[(a + r) * p->kb + (b + r)] * wx[ii * W + jj];
          }
        o[i * p->sx + j] = acc;
      }
  }
  free(wx);
  free(h);
}

/* A^T e = sum_k W_k^T B^T D^T e_k (the adjoint of orc_forward). */
void orc_adjoint(const orc_params* p, const double* e, const double* disp, double* out) {
  int64_t H = hr_h(p), W = hr_w(p), q = n_lr(p), n = H * W;
  int r = p->kb / 2, sk = n_views(p);
  double* h = malloc(sizeof(double) * p->kb * p->kb);
  orc_blur_kernel(p, h);
  int nt = orc_num_threads();
  double* acc = calloc((size_t)nt * n, sizeof(double));
  double* tmp = malloc(sizeof(double) * (size_t)nt * n);
#pragma omp parallel
  {
#ifdef _OPENMP
    int t = omp_get_thread_num();
#else
    int t = 0;
#endif
    double* u = tmp + (int64_t)t * n;
    double* a_t = acc + (int64_t)t * n;
#pragma omp for schedule(static)
    for (int k = 0; k < sk; ++k) {
      const double* ek = e + (int64_t)k * q;
      memset(u, 0, sizeof(double) * n);
      /* B^T D^T e_k: each lattice sample spreads through the blur taps */
      for (int64_t i = 0; i < p->sy; ++i)
        for (int64_t j = 0; j < p->sx; ++j) {
          int64_t Y = i * p->zeta, X = j * p->zeta;
          double v = ek[i * p->sx + j];
          for (int a = -r; a <= r; ++a)
            for (int b = -r; b <= r; ++b) {
              int64_t ii = Y + a, jj = X + b;
              if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
              u[ii * W + jj] += h[(a + r) * p->kb + (b + r)] * v;
            }
        }
      orc_warp_t_acc(p, u, disp, k, a_t);
    }
  }
  memset(out, 0, sizeof(double) * n);
  for (int t = 0; t < nt; ++t)
    for (int64_t z = 0; z < n; ++z) out[z] += acc[(int64_t)t * n + z];
  free(tmp);
  free(acc);
  free(h);
}

/* ------------------------------------------------------------ weights */

/* sec 3.4: spatial weight of offset d (read with a decreasing exponent); or,
 * for the BTV regulariser the paper matches in its multi-image experiment
 * (sec 7.3), alpha^(|dy|+|dx|) with alpha = sigma_s in (0, 1]. */
double orc_spatial_weight(const orc_params* p, int dy, int dx) {
  if (p->weight_kind == 1) return pow(p->sigma_s, (double)(abs(dy) + abs(dx)));
  return exp(-(double)(dy * dy + dx * dx) / p->sigma_s);
}

/* sec 3.4: m = w_e * w_o with the edge weight w_e = exp(-|grad x|^2/sigma_e)
 * (forward differences, zero at the last row/column); occ may be NULL (=1). */
void orc_edge_weight(const orc_params* p, const double* x, const double* occ, double* m) {
  int64_t H = hr_h(p), W = hr_w(p);
  int use_edge = p->sigma_e > 0.0 && isfinite(p->sigma_e);
  for (int64_t Y = 0; Y < H; ++Y)
    for (int64_t X = 0; X < W; ++X) {
      double we = 1.0;
      if (use_edge) {
        double gx = X + 1 < W ? x[Y * W + X + 1] - x[Y * W + X] : 0.0;
        double gy = Y + 1 < H ? x[(Y + 1) * W + X] - x[Y * W + X] : 0.0;
        we = exp(-(gx * gx + gy * gy) / p->sigma_e);
      }
      m[Y * W + X] = we * (occ ? occ[Y * W + X] : 1.0);
    }
}

/* NLTV offset number d (row-major over the window, centre skipped). */
void orc_offset(const orc_params* p, int d, int* dy, int* dx) {
  int r = p->win / 2;
  int idx = d < (p->win * p->win) / 2 ? d : d + 1;
  *dy = idx / p->win - r;
  *dx = idx % p->win - r;
}

/* ------------------------------------------------------------ S, S^T */

/* sec 4.1: weighted directional gradient,
 * g_d(z) = V_d(z) (x(z) - x(z+d)), V_d = c_d m, dropped where z+d is outside. */
void orc_nltv_grad(const orc_params* p, const double* x, const double* m, double* g) {
  int64_t H = hr_h(p), W = hr_w(p), n = H * W;
  int sd = n_offsets(p);
#pragma omp parallel for schedule(static)
  for (int d = 0; d < sd; ++d) {
    int dy, dx;
    orc_offset(p, d, &dy, &dx);
    double c = orc_spatial_weight(p, dy, dx);
    double* gd = g + (int64_t)d * n;
    for (int64_t Y = 0; Y < H; ++Y)
      for (int64_t X = 0; X < W; ++X) {
        int64_t Y2 = Y + dy, X2 = X + dx;
        double v = 0.0;
        if (Y2 >= 0 && Y2 < H && X2 >= 0 && X2 < W)
          v = c * m[Y * W + X] * (x[Y * W + X] - x[Y2 * W + X2]);
        gd[Y * W + X] = v;
      }
  }
}

/* sec 4.1: weighted directional divergence = S^T g, the exact adjoint of
 * orc_nltv_grad:  out(z) = sum_d [V_d(z) g_d(z) 1(z+d in image)
 *                                  - V_d(z-d) g_d(z-d) 1(z-d in image)]. */
void orc_nltv_div(const orc_params* p, const double* g, const double* m, double* out) {
  int64_t H = hr_h(p), W = hr_w(p), n = H * W;
  int sd = n_offsets(p);
  double* cd = malloc(sizeof(double) * (sd > 0 ? sd : 1));
  int* oy = malloc(sizeof(int) * (sd > 0 ? sd : 1));
  int* ox = malloc(sizeof(int) * (sd > 0 ? sd : 1));
  for (int d = 0; d < sd; ++d) {
    orc_offset(p, d, &oy[d], &ox[d]);
    cd[d] = orc_spatial_weight(p, oy[d], ox[d]);
  }
#pragma omp parallel for schedule(static)
  for (int64_t Y = 0; Y < H; ++Y)
    for (int64_t X = 0; X < W; ++X) {
      double acc = 0.0;
      for (int d = 0; d < sd; ++d) {
        const double* gd = g + (int64_t)d * n;
        int64_t Yp = Y + oy[d], Xp = X + ox[d];
        if (Yp >= 0 && Yp < H && Xp >= 0 && Xp < W) acc += cd[d] * m[Y * W + X] * gd[Y * W + X];
        int64_t Ym = Y - oy[d], Xm = X - ox[d];
        if (Ym >= 0 && Ym < H && Xm >= 0 && Xm < W) acc -= cd[d] * m[Ym * W + Xm] * gd[Ym * W + Xm];
      }
      out[Y * W + X] = acc;
    }
  free(cd);
  free(oy);
  free(ox);
}

/* ------------------------------------------------------------ x0 */

/* Keys cubic-convolution kernel with a = -1/2. */
static double keys(double s) {
  const double a = -0.5;
  s = fabs(s);
  if (s <= 1.0) return (a + 2.0) * s * s * s - (a + 3.0) * s * s + 1.0;
  if (s < 2.0) return a * s * s * s - 5.0 * a * s * s + 8.0 * a * s - 4.0 * a;
  return 0.0;
}

/* sec 5: x is initialised with a bicubic up-sampling of the low-resolution
 * image; we take the reference (centre) view, LR sample (i,j) sitting at
 * HR (zeta*i, zeta*j) (the pixel D keeps), clamp-to-edge. */
void orc_bicubic(const orc_params* p, const double* lr, double* out) {
  int64_t H = hr_h(p), W = hr_w(p);
  for (int64_t Y = 0; Y < H; ++Y)
    for (int64_t X = 0; X < W; ++X) {
      double py = (double)Y / p->zeta, px = (double)X / p->zeta;
      int64_t iy = (int64_t)floor(py), ix = (int64_t)floor(px);
      double fy = py - iy, fx = px - ix;
      double acc = 0.0;
      for (int mm = -1; mm <= 2; ++mm)
        for (int nn = -1; nn <= 2; ++nn) {
          int64_t i = iy + mm, j = ix + nn;
          if (i < 0) i = 0;
          if (i >= p->sy) i = p->sy - 1;
          if (j < 0) j = 0;
          if (j >= p->sx) j = p->sx - 1;
          acc += keys(fy - mm) * keys(fx - nn) * lr[i * p->sx + j];
        }
      out[Y * W + X] = acc;
    }
}

/* ------------------------------------------------------------ occlusion weight */

/* sec 3.4, eq. (weight_occ): w_o(z) = exp(-b(z)^2 / (2 s1^2)) exp(-p(z)^2 / (2 s2^2)).
 *   b: one-sided divergence of the reference view's disparity map w: the sum
 *      of its two forward differences (zero at the last column / row), kept
 *      where it is negative (occluding boundaries) and 0 elsewhere.
 *   p: projection error between the reference view and the other views
 *      brought back to it.  L_i is the bicubic up-sampling of y_i (the x0
 *      operator above); view i's sample of reference pixel z sits at
 *      z - theta_i w(z) (the inverse of the forward warp, which reads the
 *      reference at z + theta_i w(z)), read bilinearly with the position
 *      clamped to the image; p(z)^2 is the mean of (L_ref(z) - L_i(.))^2 over
 *      the views i other than the reference (0 with a single view).
 * s1 or s2 infinite: that factor is 1. */
void orc_occlusion_weight(const orc_params* p, const double* y, const double* disp, double s1, double s2,
                          double* out) {
  const int64_t H = hr_h(p), W = hr_w(p), n = n_hr(p), q = n_lr(p);
  const int sk = n_views(p), kref = orc_ref_view(p);
  const double* w = disp_of(p, disp, kref);
  double* l0 = (double*)malloc(sizeof(double) * n);
  double* li = (double*)malloc(sizeof(double) * n);
  double* acc = (double*)calloc((size_t)n, sizeof(double));
  orc_bicubic(p, y + (int64_t)kref * q, l0);
  for (int k = 0; k < sk; ++k) {
    if (k == kref) continue;
    int tau, rho;
    orc_view_offset(p, k, &tau, &rho);
    orc_bicubic(p, y + (int64_t)k * q, li);
    for (int64_t Y = 0; Y < H; ++Y)
      for (int64_t X = 0; X < W; ++X) {
        double py = (double)Y - tau * w[Y * W + X], px = (double)X - rho * w[Y * W + X];
        if (py < 0.0) py = 0.0;
        if (py > (double)(H - 1)) py = (double)(H - 1);
        if (px < 0.0) px = 0.0;
        if (px > (double)(W - 1)) px = (double)(W - 1);
        const int64_t i0 = (int64_t)floor(py), j0 = (int64_t)floor(px);
        const int64_t i1 = i0 + 1 < H ? i0 + 1 : H - 1, j1 = j0 + 1 < W ? j0 + 1 : W - 1;
        const double fy = py - i0, fx = px - j0;
        const double v = (1.0 - fy) * ((1.0 - fx) * li[i0 * W + j0] + fx * li[i0 * W + j1]) +
                         fy * ((1.0 - fx) * li[i1 * W + j0] + fx * li[i1 * W + j1]);
        const double d = l0[Y * W + X] - v;
        acc[Y * W + X] += d * d;
      }
  }
  for (int64_t Y = 0; Y < H; ++Y)
    for (int64_t X = 0; X < W; ++X) {
      const double gx = X + 1 < W ? w[Y * W + X + 1] - w[Y * W + X] : 0.0;
      const double gy = Y + 1 < H ? w[(Y + 1) * W + X] - w[Y * W + X] : 0.0;
      const double b = gx + gy < 0.0 ? gx + gy : 0.0;
      const double p2 = sk > 1 ? acc[Y * W + X] / (sk - 1) : 0.0;
      const double f1 = isinf(s1) ? 1.0 : exp(-b * b / (2.0 * s1 * s1));
      const double f2 = isinf(s2) ? 1.0 : exp(-p2 / (2.0 * s2 * s2));
      out[Y * W + X] = f1 * f2;
    }
  free(l0);
  free(li);
  free(acc);
}

/* ------------------------------------------------------------ reductions */

static double dot(const double* a, const double* b, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* ------------------------------------------------------------ x-step */

/* sec 5: G^T G = (lambda2 + vartheta lambda1^2 / 2) A^T A + (vartheta/2) S^T S
 * (the paper's expression in the unscaled per-block form). */
void orc_normal_apply(const orc_params* p, const double* disp, const double* m, const double* x,
                      double* out) {
  int64_t n = n_hr(p), q = n_lr(p);
  int sk = n_views(p), sd = n_offsets(p);
  double cA = p->lambda2 + 0.5 * p->theta * p->lambda1 * p->lambda1;
  double* t = malloc(sizeof(double) * sk * q);
  double* ata = malloc(sizeof(double) * n);
  orc_forward(p, x, disp, t);
  orc_adjoint(p, t, disp, ata);
  for (int64_t z = 0; z < n; ++z) out[z] = cA * ata[z];
  if (sd > 0) {
    double* g = malloc(sizeof(double) * sd * n);
    double* sts = malloc(sizeof(double) * n);
    orc_nltv_grad(p, x, m, g);
    orc_nltv_div(p, g, m, sts);
    for (int64_t z = 0; z < n; ++z) out[z] += 0.5 * p->theta * sts[z];
    free(sts);
    free(g);
  }
  free(ata);
  free(t);
}

/* sec 5, Algorithm 2: conjugate gradients on the normal equations
 * H delta = -v from delta = 0, at most K steps, continuing while pi > tau
 * (and pi > 0).  Returns the number of steps taken; *pi_out = final pi. */
int orc_cg(const orc_params* p, const double* disp, const double* m, const double* v, double* delta,
           double* pi_out) {
  int64_t n = n_hr(p);
  double* r = malloc(sizeof(double) * n);
  double* pv = malloc(sizeof(double) * n);
  double* hp = malloc(sizeof(double) * n);
  for (int64_t z = 0; z < n; ++z) {
    delta[z] = 0.0;
    r[z] = -v[z];
    pv[z] = r[z];
  }
  double pi = dot(r, r, n);
  int steps = 0;
  for (int k = 0; k < p->cg_iter; ++k) {
    if (!(pi > p->cg_tol) || pi == 0.0) break;
    orc_normal_apply(p, disp, m, pv, hp);
    double php = dot(pv, hp, n);
    if (!(php > 0.0)) break;
    double alpha = pi / php;
    for (int64_t z = 0; z < n; ++z) {
      delta[z] += alpha * pv[z];
      r[z] -= alpha * hp[z];
    }
    double pi_new = dot(r, r, n);
    double beta = pi_new / pi;
    for (int64_t z = 0; z < n; ++z) pv[z] = r[z] + beta * pv[z];
    pi = pi_new;
    ++steps;
  }
  *pi_out = pi;
  free(hp);
  free(pv);
  free(r);
  return steps;
}

/* ------------------------------------------------------------ ADMM */

/* sec 4, closed-form prox of (1/vartheta)|.|_1 and the w-step that follows it:
 * w' = u - soft(u, 1/vartheta), i.e. u clipped to [-1/vartheta, 1/vartheta]. */
static double soft(double u, double t) {
  double a = fabs(u) - t;
  if (a <= 0.0) return 0.0;
  return u > 0.0 ? a : -a;
}

double orc_soft_threshold(double u, double t) { return soft(u, t); }

/* Per-iteration statistics, 6 doubles each:
 *   [0] J(x^(n-1))  (the cost function of sec 4)
 *   [1] primal residual |w^(n) - w^(n-1)|_2 over both blocks
 *   [2] final CG pi
 *   [3] CG steps taken
 *   [4] data part lambda1 sum|r| + lambda2 sum r^2
 *   [5] regulariser part sum|g|                                              */
#define ORC_NSTAT 6

/* sec 5, Algorithm 1: run `count` ADMM iterations from the state (x, wD, wS, m),
 * the iteration number of the first being n_first (1-based; it decides whether
 * the edge weight is computed when reweighting is off).  State is updated in
 * place.  y: [sk][sy][sx]; wD: [sk][sy][sx]; wS: [sd][H][W]; m: [H][W]. */
void orc_admm_iterate(const orc_params* p, const double* y, const double* disp, const double* occ,
                      double* x, double* wD, double* wS, double* m, int n_first, int count,
                      double* stats) {
  int64_t n = n_hr(p), q = n_lr(p);
  int sk = n_views(p), sd = n_offsets(p);
  int64_t nd = (int64_t)sk * q, ns = (int64_t)sd * n;
  double lim = 1.0 / p->theta;
  double* r = malloc(sizeof(double) * nd);
  double* e = malloc(sizeof(double) * nd);
  double* g = malloc(sizeof(double) * (ns > 0 ? ns : 1));
  double* f = malloc(sizeof(double) * (ns > 0 ? ns : 1));
  double* v = malloc(sizeof(double) * n);
  double* vs = malloc(sizeof(double) * n);
  double* delta = malloc(sizeof(double) * n);
  for (int it = 0; it < count; ++it) {
    int nn = n_first + it;
    if (p->reweight || nn == 1) orc_edge_weight(p, x, occ, m);
    /* a = A x - b and F x - b' (unscaled blocks): r_k = A_k x - y_k, g = S x */
    orc_forward(p, x, disp, r);
    for (int64_t i = 0; i < nd; ++i) r[i] -= y[i];
    if (sd > 0) orc_nltv_grad(p, x, m, g);
    double s1 = 0.0, s2 = 0.0, sg = 0.0, res2 = 0.0;
    for (int64_t i = 0; i < nd; ++i) {
      s1 += fabs(r[i]);
      s2 += r[i] * r[i];
    }
    for (int64_t i = 0; i < ns; ++i) sg += fabs(g[i]);
    /* z-step (prox) and w-step on the data block; f = 2w' - w */
    for (int64_t i = 0; i < nd; ++i) {
      double u = p->lambda1 * r[i] + wD[i];
      double z = soft(u, lim);
      double wn = u - z;
      double fD = 2.0 * wn - wD[i];
      res2 += (wn - wD[i]) * (wn - wD[i]);
      wD[i] = wn;
      /* the data-block input of A^T: lambda2 r + (vartheta/2) lambda1 f_D */
      e[i] = p->lambda2 * r[i] + 0.5 * p->theta * p->lambda1 * fD;
    }
    for (int64_t i = 0; i < ns; ++i) {
      double u = g[i] + wS[i];
      double z = soft(u, lim);
      double wn = u - z;
      f[i] = 2.0 * wn - wS[i];
      res2 += (wn - wS[i]) * (wn - wS[i]);
      wS[i] = wn;
    }
    /* v = A^T a + (vartheta/2) F^T f */
    orc_adjoint(p, e, disp, v);
    if (sd > 0) {
      orc_nltv_div(p, f, m, vs);
      for (int64_t z = 0; z < n; ++z) v[z] += 0.5 * p->theta * vs[z];
    }
    double pi_fin = 0.0;
    int steps = orc_cg(p, disp, m, v, delta, &pi_fin);
    for (int64_t z = 0; z < n; ++z) x[z] += delta[z];
    if (stats) {
      double* st = stats + (int64_t)it * ORC_NSTAT;
      st[0] = p->lambda1 * s1 + p->lambda2 * s2 + sg;
      st[1] = sqrt(res2);
      st[2] = pi_fin;
      st[3] = steps;
      st[4] = p->lambda1 * s1 + p->lambda2 * s2;
      st[5] = sg;
    }
  }
  free(delta);
  free(vs);
  free(v);
  free(f);
  free(g);
  free(e);
  free(r);
}

/* The cost function of sec 4 at x (with weight map m). */
double orc_objective(const orc_params* p, const double* y, const double* disp, const double* m,
                     const double* x) {
  int64_t n = n_hr(p), q = n_lr(p);
  int sk = n_views(p), sd = n_offsets(p);
  int64_t nd = (int64_t)sk * q, ns = (int64_t)sd * n;
  double* r = malloc(sizeof(double) * nd);
  double* g = malloc(sizeof(double) * (ns > 0 ? ns : 1));
  orc_forward(p, x, disp, r);
  double s1 = 0.0, s2 = 0.0, sg = 0.0;
  for (int64_t i = 0; i < nd; ++i) {
    double ri = r[i] - y[i];
    s1 += fabs(ri);
    s2 += ri * ri;
  }
  if (sd > 0) {
    orc_nltv_grad(p, x, m, g);
    for (int64_t i = 0; i < ns; ++i) sg += fabs(g[i]);
  }
  free(g);
  free(r);
  return p->lambda1 * s1 + p->lambda2 * s2 + sg;
}
