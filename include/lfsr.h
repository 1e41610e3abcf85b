/*
 * lfsr.h -- C ABI of the MI355X (gfx950) light-field super-resolution solver.
 *
 * The solver minimises, over the high-resolution (HR) reference view x,
 *
 *   J(x) = lambda1 sum_k |A_k x - y_k|_1 + lambda2 sum_k |A_k x - y_k|_2^2
 *          + sum_d | V_d (x - S_d x) |_1                                   (paper sec 4, cost J)
 *
 * with the per-view forward model A_k = D B W_k (sec 3.1): a disparity warp
 * W_k of x to angular view k, a Gaussian blur B and a decimation D that keeps
 * the top-left pixel of every scale x scale block (sec 4.1).  The regulariser
 * is weighted non-local TV over the offsets d of an NLTV window with weights
 * V_d(z) = exp(-|d|^2/sigma_s) * exp(-|grad x(z)|^2/sigma_e) * occ(z)
 * (sec 3.4).  The minimiser is the ADMM iteration of sec 5, Algorithm 1 (z-
 * and w-steps before the x-step, the penalty absorbed into the dual) with the
 * x-step solved by the conjugate-gradient loop of Algorithm 2.
 *
 * Layouts (all row-major, no padding, float32 unless stated):
 *   LR views   y     [s_k][lr_h][lr_w], s_k = ang_rows*ang_cols, view k at
 *                    angular row k / ang_cols and column k % ang_cols, angular
 *                    offset tau_k = k / ang_cols - (ang_rows-1)/2 rows and
 *                    rho_k = k % ang_cols - (ang_cols-1)/2 columns; the
 *                    reference is the view with offset (0, 0).
 *   disparity  disp  [n_disp][H][W], H = scale*lr_h, W = scale*lr_w: HR
 *                    pixels of shift per unit angular step.  With n_disp = 1
 *                    one map, defined on the reference view, serves every
 *                    view; with n_disp = s_k map k belongs to view k (sec 4.1
 *                    gives each perspective its own map).  View k (angular
 *                    offset tau_k rows, rho_k columns from the centre) samples
 *                    x bilinearly at (Y + tau_k*w(Y,X), X + rho_k*w(Y,X)),
 *                    w its map; samples outside the image read zero (sec 4.1).
 *   HR image   x     [H][W].
 *   data dual  w_D   [s_k][lr_h][lr_w]; NLTV dual w_S [s_d][H][W] with the
 *                    s_d = nltv_window^2 - 1 offsets d = (dy,dx) row-major
 *                    over the window, centre skipped.
 *
 * Ownership: every pointer is owned by the caller.  Pointers named d_* are
 * device (HBM) pointers, h_* host pointers.  The library allocates no device
 * memory: the caller provides one workspace of lfsr_workspace_bytes() bytes
 * (256-byte aligned) that must outlive the handle.  Input buffers bound by
 * lfsr_init() must stay alive and unchanged until the last lfsr_iterate().
 *
 * Streams: every call that takes a hip_stream (a hipStream_t; NULL = the
 * default stream) only enqueues work on it and returns, unless documented as
 * synchronising.  One handle must not be used from two streams at once.
 *
 * Errors: return codes only; no exception crosses this interface.  Parameter
 * errors are caught by lfsr_create() (LFSR_EINVAL).  Input-data errors found
 * on the device (non-finite values, disparity beyond disp_bound) are recorded
 * on the device and reported by the next synchronising call
 * (lfsr_get_stats, or lfsr_solve with h_stats != NULL).  A failed HIP call
 * makes the handle unusable (LFSR_EDEVICE now, LFSR_ESTATE afterwards).
 * lfsr_last_error() returns a description of the last failure.
 */
#ifndef LFSR_H
#define LFSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lfsr_handle lfsr_handle;

typedef enum {
  LFSR_OK = 0,
  LFSR_EINVAL = -1,     /* bad parameter, size, pointer or input data */
  LFSR_ENOMEM = -2,     /* workspace missing or too small */
  LFSR_EDEVICE = -3,    /* a HIP runtime call failed */
  LFSR_ESTATE = -4,     /* call out of order, or handle broken by an earlier device error */
  LFSR_ENONFINITE = -5, /* NaN/Inf in the inputs */
  LFSR_EBUSY = -6       /* reserved */
} lfsr_status;

/* Storage type of the solver state: the HR estimate x, the dual fields w_D
 * and w_S, and the LR work stack (e in the wz-step, t = A p in CG).  With
 * LFSR_F16 / LFSR_BF16 these are stored in 16 bits (rounded to nearest even
 * at each store) and all stencil arithmetic stays FP32; x is kept as the
 * 16-bit value the stencils read plus an FP32 remainder into which CG
 * accumulates, so x is exact to FP32 and lfsr_read_state / lfsr_solve return
 * that FP32 value.  The CG vectors r, p, Hp, the weight map and every
 * reduction (FP64) are unchanged.  Inputs and outputs are always float. */
typedef enum { LFSR_F32 = 0, LFSR_F16 = 1, LFSR_BF16 = 2 } lfsr_storage;

typedef struct {
  int32_t ang_rows, ang_cols; /* U, V: angular grid; the reference is view ((U-1)/2, (V-1)/2), the
                                 centre of an odd grid (an even grid, e.g. the 2 x 2 images of the
                                 multi-image workload, has offsets 0 .. U/2 from it) */
  int32_t lr_h, lr_w;         /* s_y, s_x: LR view size */
  int32_t scale;              /* zeta in 1..8: HR = scale * LR (sec 4.1); HR at most 32768 per side and 2^28 pixels */
  int32_t n_disp;             /* 1: one disparity map on the reference view, used by every view;
                                 ang_rows*ang_cols: one map per view (sec 4.1: w_k per perspective) */
  int32_t blur_size;          /* odd, 1..31; <= 0 with blur_sigma <= 0: paper default (see below) */
  float blur_sigma;           /* Gaussian std-dev in HR px; <= 0: sqrt(scale^2-1)/4 (sec 4.1), size 2*ceil(3 sigma)+1 */
  float lambda1, lambda2;     /* l1 and l2 fidelity weights (sec 3.3), >= 0, not both 0 */
  int32_t nltv_window;        /* odd, 1..15; 1 switches the regulariser off */
  float sigma_s;              /* spatial weight scale (sec 3.4), > 0 */
  float sigma_e;              /* edge weight scale (sec 3.4), > 0; +INF: no edge weight */
  int32_t reweight;           /* 1: edge weight recomputed from x at every ADMM iteration (sec 7.1); 0: from x0 only */
  float admm_penalty;         /* vartheta > 0 (sec 4) */
  int32_t admm_iters;         /* N >= 1 (Algorithm 1) */
  int32_t cg_iters;           /* K >= 0 (Algorithm 2) */
  float cg_tol;               /* tau >= 0: CG continues while |r|^2 > tau (0: exactly K steps unless r = 0) */
  float stop_tol;             /* >= 0: stop after iteration n once res_n <= stop_tol * res_1 (0: run N) */
  float disp_bound;           /* > 0: the caller's bound on |disp| (sizes the warp halo; larger values are an input error) */
  int32_t storage;            /* lfsr_storage of the solver state (see below) */
  int32_t spatial_weight;     /* NLTV spatial weight of offset d: 0 = exp(-|d|^2 / sigma_s) (sec 3.4);
                                 1 = BTV, sigma_s^(|dy|+|dx|) with 0 < sigma_s <= 1 (sec 7.3) */
  const float* blur_taps;     /* NULL: the Gaussian of blur_size / blur_sigma; else host memory holding an
                                 explicit [blur_size][blur_size] correlation kernel, row-major, blur_size odd
                                 <= 15, read by lfsr_create / lfsr_workspace_bytes only (sec 7.1 models motion
                                 blur this way; no symmetry is assumed: B^T is its transpose) */
} lfsr_params;

#define LFSR_NSTAT 6
typedef struct {
  int32_t iters_run;    /* ADMM iterations completed since lfsr_init */
  int32_t cg_steps;     /* CG steps taken in the last iteration */
  double objective;     /* J(x^(n-1)) of the last iteration n (FP64 reduction) */
  double primal_res;    /* |w^(n) - w^(n-1)|_2 over both dual blocks */
  double cg_pi;         /* final |r|^2 of the last x-step */
  double* h_hist;       /* NULL, or caller memory for [admm_iters][LFSR_NSTAT] doubles:
                           {J, primal residual, final pi, CG steps, data part, regulariser part} */
} lfsr_stats;

/* Bytes of device workspace a handle with these parameters needs; 0 if the
 * parameters are invalid (lfsr_last_error(NULL) says why). Host-only.
 * The workspace holds the state of the ADMM iteration of sec 5, Algorithm 1
 * (x, the dual fields w_D and w_S, the weight map, the CG vectors of
 * Algorithm 2) for the problem of sec 3.1 / sec 4 that the parameters
 * describe; with 16-bit storage its dominant fields take half the bytes. */
size_t lfsr_workspace_bytes(const lfsr_params* p);

/* Validate p and build a handle over the caller's workspace (d_workspace, at
 * least lfsr_workspace_bytes(p) bytes, 256-byte aligned).  Host-only: touches
 * no device memory.  The handle fixes one instance of the problem of sec 3.1
 * and sec 4 (angular grid, LR size, scale, blur, fidelity weights, NLTV
 * window and weights) and the solver settings of sec 5 (penalty vartheta,
 * N ADMM iterations, K CG steps, CG tolerance tau).  Errors: LFSR_EINVAL
 * (bad parameter or alignment, *out = NULL), LFSR_ENOMEM (workspace NULL or
 * too small). */
lfsr_status lfsr_create(const lfsr_params* p, void* d_workspace, size_t bytes, lfsr_handle** out);

/* Release the handle of a problem instance (sec 3.1 / sec 4) created by
 * lfsr_create (NULL-safe).  Does not free the workspace and waits for
 * nothing: work already enqueued on a stream keeps using the workspace, so
 * the caller frees it only after that work has completed. */
void lfsr_destroy(lfsr_handle* h);

/* Text of the last error on h, or of the calling thread's last handle-less
 * error when h is NULL.  Never NULL.  Parameter errors name the field of the
 * problem statement (sec 3.1, sec 4, sec 5) that is out of range. */
const char* lfsr_last_error(const lfsr_handle* h);

/* Complete solve (Algorithm 1): lfsr_init + lfsr_iterate(admm_iters) + copy
 * of x into d_hr_out [H][W].  Asynchronous on hip_stream unless h_stats is
 * non-NULL, in which case it synchronises and fills *h_stats. */
lfsr_status lfsr_solve(lfsr_handle* h, const float* d_lr, const float* d_disp, const float* d_occ,
                       const float* d_x0, float* d_hr_out, lfsr_stats* h_stats, void* hip_stream);

/* Variant of lfsr_solve for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): it takes the parameters instead of a handle and runs the same
 * kernels over a workspace held in a static device array of
 * LFSR_NOALLOC_MAX_BYTES bytes, one per GPU, resident until the process ends.
 * It calls no hipMalloc / hipFree and allocates no device memory; the caller
 * still provides the inputs (layouts as for lfsr_init) and d_hr_out [H][W].
 * Problems whose lfsr_workspace_bytes exceed LFSR_NOALLOC_MAX_BYTES are
 * rejected with LFSR_ENOMEM before any work is enqueued; invalid parameters
 * give LFSR_EINVAL.  Errors are reported through lfsr_last_error(NULL).
 * Every call on one GPU uses that GPU's one array and leaves its state there
 * (each call starts from x0 and w = 0 of its own): calls that overlap on one
 * GPU (two streams, two threads, or a second call before the first one's work
 * has completed on another stream) race and give wrong results; calls on one
 * stream are ordered and safe.  Asynchronous on hip_stream unless h_stats is
 * non-NULL (then it synchronises and fills *h_stats, as lfsr_solve does). */
#define LFSR_NOALLOC_MAX_BYTES ((size_t)64 << 20)
lfsr_status lfsr_solve_noalloc(const lfsr_params* p, const float* d_lr, const float* d_disp, const float* d_occ,
                               const float* d_x0, float* d_hr_out, lfsr_stats* h_stats, void* hip_stream);

/* Bind the inputs (d_lr [s_k][lr_h][lr_w], d_disp [n_disp][H][W], d_occ [H][W]
 * occlusion weight or NULL = 1) and set the state to x = d_x0 (or, if NULL,
 * the bicubic up-sampling of the centre view: Keys a = -1/2, LR sample (i,j)
 * at HR (scale*i, scale*j), clamp-to-edge; sec 5), w_D = w_S = 0, n = 0.
 * Enqueues an input check (non-finite values; |disp| > disp_bound). */
lfsr_status lfsr_init(lfsr_handle* h, const float* d_lr, const float* d_disp, const float* d_occ,
                      const float* d_x0, void* hip_stream);

/* Run `count` more ADMM iterations (sec 5, Algorithm 1) on the bound inputs. */
lfsr_status lfsr_iterate(lfsr_handle* h, int32_t count, void* hip_stream);

/* Copy the state out as float32: x [H][W], w_D [s_k][lr_h][lr_w],
 * w_S [s_d][H][W], the weight map m = w_e * occ [H][W].  Any pointer may be NULL. */
lfsr_status lfsr_read_state(lfsr_handle* h, float* d_x, float* d_wd, float* d_ws, float* d_m,
                            void* hip_stream);

/* Replace the state (checkpoint resume): same layouts as lfsr_read_state;
 * n_done = iterations already run (decides whether the edge weight is
 * recomputed on the next iteration when reweight = 0).  All pointers
 * required except d_m when reweight = 1.  With 16-bit storage the duals are
 * rounded to the storage type (exact for values lfsr_read_state returned)
 * and x is split exactly, so read -> write -> iterate resumes bit for bit. */
lfsr_status lfsr_write_state(lfsr_handle* h, const float* d_x, const float* d_wd, const float* d_ws,
                             const float* d_m, int32_t n_done, void* hip_stream);

/* Synchronise hip_stream and report statistics (see lfsr_stats).  Returns
 * LFSR_ENONFINITE / LFSR_EINVAL if the input check of lfsr_init failed. */
lfsr_status lfsr_get_stats(lfsr_handle* h, lfsr_stats* out, void* hip_stream);

/* Operators of the forward model on the handle's geometry (sec 3.1, 4.1):
 *   lfsr_forward: d_lr_out[k] = A_k d_x = D B W_k d_x for every view k.
 *   lfsr_adjoint: d_hr_out = sum_k A_k^T d_lr[k] (exact transpose; W_k^T is
 *                 the scatter with the bilinear weights of W_k).
 *   lfsr_normal:  d_out = (lambda2 + vartheta*lambda1^2/2) A^T A d_p
 *                         + (vartheta/2) S^T S d_p with the weights of d_m
 *                 (the x-step normal operator G^T G of sec 5); the
 *                 intermediate A d_p is stored in the handle's storage type,
 *                 exactly as in the solver's CG steps.
 *                 d_out must not alias d_p or d_m (LFSR_EINVAL).
 * lfsr_forward / lfsr_adjoint are FP32 throughout whatever the storage type.
 * They use the handle's work buffers, so they must not overlap an iteration. */
lfsr_status lfsr_forward(lfsr_handle* h, const float* d_x, const float* d_disp, float* d_lr_out,
                         void* hip_stream);
lfsr_status lfsr_adjoint(lfsr_handle* h, const float* d_lr, const float* d_disp, float* d_hr_out,
                         void* hip_stream);
lfsr_status lfsr_normal(lfsr_handle* h, const float* d_p, const float* d_disp, const float* d_m,
                        float* d_out, void* hip_stream);

/* sec 3.4: d_m_out = exp(-|grad x|^2 / sigma_e) * occ (forward differences,
 * zero at the last row/column; occ NULL = 1). */
lfsr_status lfsr_edge_weight(lfsr_handle* h, const float* d_x, const float* d_occ, float* d_m_out,
                             void* hip_stream);

/* sec 3.4, eq. (weight_occ): the occlusion weight
 *   d_occ_out = exp(-b^2 / (2 sigma_o1^2)) * exp(-p^2 / (2 sigma_o2^2))   [H][W]
 * from the LR views d_lr [s_k][lr_h][lr_w] and the reference view's disparity
 * map (d_disp [n_disp][H][W]; with one map per view, map kref), ready to pass as
 * d_occ to lfsr_init / lfsr_solve.
 *   b: the one-sided divergence of the disparity map, the sum of its two
 *      forward differences (zero at the last column / row), where negative
 *      (occluding boundaries), else 0;
 *   p: the projection error, p^2 = mean over the views k other than the
 *      reference of (L_ref(z) - L_k(z - theta_k disp(z)))^2, L the bicubic
 *      up-sampling of a view (as for x0), read bilinearly at the position
 *      clamped to the image (z - theta_k disp(z) is where view k shows the
 *      reference pixel z under the forward warp).
 * sigma_o1, sigma_o2 > 0; +INF switches that factor off.  Uses the handle's
 * work buffers (must not overlap an iteration); FP32. */
lfsr_status lfsr_occlusion_weight(lfsr_handle* h, const float* d_lr, const float* d_disp, float sigma_o1,
                                  float sigma_o2, float* d_occ_out, void* hip_stream);

/* The gradient-descent baselines the paper compares ADMM with (sec 7.1: gd
 * and gd-ls): subgradient descent on the cost J of sec 4 with the weights
 * fixed at the starting point (m = w_e(x) * occ), from the state lfsr_init
 * (or lfsr_write_state) left, updating the handle's x in place (read it with
 * lfsr_read_state).  The subgradient is
 *   sum_k A_k^T (lambda1 sgn(r_k) + 2 lambda2 r_k) + S^T sgn(V (I - S) x),
 * r_k = A_k x - y_k, sgn(0) = 0.  line_search = 0: x <- x - step g, each step
 * two computation units (CU: one is A with S for a cost, one A^T with S^T
 * for a gradient).  line_search = 1: backtracking from twice the last
 * accepted step (the first from `step`), halving until
 * J(x - eta g) <= J(x) - 1e-4 eta |g|^2 (one CU per trial, at most 30; a step
 * with no accepted trial leaves x unchanged), then one CU for the gradient
 * at the new point.  h_hist (NULL or [iters + 1][3] doubles) receives
 * (J(x_n), CU spent after step n, eta) for n = 0 .. iters.  FP32 storage
 * only (LFSR_EINVAL otherwise).  Synchronises the stream after every cost
 * evaluation; uses the handle's work buffers. */
lfsr_status lfsr_gd(lfsr_handle* h, int32_t iters, float step, int32_t line_search, double* h_hist,
                    void* hip_stream);

/* sec 5: bicubic up-sampling of one LR view d_lr_view [lr_h][lr_w] to [H][W]
 * (the x0 of lfsr_init). */
lfsr_status lfsr_bicubic(lfsr_handle* h, const float* d_lr_view, float* d_hr_out, void* hip_stream);

/* Kernel timing (tracing aid).  While a profile is open, every launch of a
 * selected kernel kind issued by this handle is bracketed by two HIP events
 * recorded on the stream it is launched on; lfsr_profile_end synchronises on
 * them and returns, per kind, the summed event-measured duration and the
 * number of timed launches.  capacity bounds the number of timed launches
 * (the rest run untimed); the events are created by lfsr_profile_begin and
 * destroyed by lfsr_profile_end.  Opening a second profile is LFSR_ESTATE. */
typedef enum {
  LFSR_K_FORWARD = 0, /* A_k x for all views (wz-step and CG variants) */
  LFSR_K_ADJOINT = 1, /* sum_k A_k^T e_k */
  LFSR_K_NLTV = 2,    /* NLTV z/w-step and divergence */
  LFSR_K_NORMAL = 3,  /* normal-operator assembly G^T G p and <p, Hp> */
  LFSR_K_CG = 4,      /* CG start / update kernels */
  LFSR_K_OTHER = 5,   /* edge weight, merge of the adjoint's partial images, iteration bookkeeping */
  LFSR_K_COUNT = 6
} lfsr_kernel_kind;

lfsr_status lfsr_profile_begin(lfsr_handle* h, uint32_t kind_mask, int32_t capacity);
lfsr_status lfsr_profile_end(lfsr_handle* h, double* h_total_ms, int32_t* h_launches);

/* ------------------------------------------------------------------------
 * Serving pool: many independent super-resolution jobs (any mix of angular
 * sizes, spatial sizes and scales) solved concurrently on one GPU, each one
 * the ADMM iteration of sec 5 (Algorithms 1 and 2) exactly as lfsr_solve
 * runs it, so a job's result is bit-identical to its solo lfsr_solve.
 *
 * The caller gives the pool one device arena; a job is admitted when a slot
 * is free and its workspace (lfsr_workspace_bytes of its parameters) fits in
 * the arena's free space (first fit, 256-byte aligned), and its ADMM state
 * stays resident there until it is harvested.  lfsr_pool_tick advances every
 * active job by one ADMM iteration with a single launch of a HIP graph that
 * holds one branch per job; the graph is captured again only when the set of
 * active jobs has changed.  A job that has run its admm_iters iterations has
 * its result copied to its d_hr_out on the pool's stream and is retired; a
 * later lfsr_pool_poll reports it once the copy has completed and frees its
 * arena space.  Jobs whose stop test fires idle (their iterations become
 * no-ops on the device) until they reach admm_iters ticks.
 *
 * All input buffers of a job and its d_hr_out must stay valid until the job
 * is reported by lfsr_pool_poll.  The pool's calls are not thread-safe.  A
 * pool's work runs on an internal stream ordered after the caller's stream
 * at each call (submit, tick) and before it at the end of each tick.
 * ------------------------------------------------------------------------ */
typedef struct lfsr_pool lfsr_pool;

/* d_arena: device memory of `bytes` bytes (256-byte aligned, caller-owned,
 * not freed by the pool); max_slots: 1..256 concurrent jobs. */
lfsr_status lfsr_pool_create(void* d_arena, size_t bytes, int32_t max_slots, lfsr_pool** out);

/* Waits for the pool's outstanding work, destroys every job and the pool.
 * NULL-safe. */
void lfsr_pool_destroy(lfsr_pool* pool);

/* Text of the last error of this pool (thread-local text if pool is NULL). */
const char* lfsr_pool_last_error(const lfsr_pool* pool);

/* Admit a job: inputs as for lfsr_solve.  Returns LFSR_EBUSY (nothing done)
 * when no slot is free or its workspace does not fit in the free arena space
 * now; LFSR_ENOMEM when it can never fit (larger than the arena); LFSR_EINVAL
 * for invalid parameters or NULL pointers.  On success *job_id receives the
 * job's id (> 0) and the job's setup (input check, x0, w = 0) is enqueued,
 * ordered after the work already on hip_stream.  Input errors of the job
 * (non-finite values, |disp| > disp_bound) do not fail the call: the job
 * runs and lfsr_pool_poll reports its status. */
lfsr_status lfsr_pool_submit(lfsr_pool* pool, const lfsr_params* params, const float* d_lr, const float* d_disp,
                             const float* d_occ, const float* d_x0, float* d_hr_out, void* hip_stream,
                             int64_t* job_id);

/* One ADMM iteration of every active job (one graph launch), then the
 * retirement of the jobs that have finished.  hip_stream is ordered before
 * and after the pool's work.  *h_active (may be NULL) receives the number of
 * jobs advanced. */
lfsr_status lfsr_pool_tick(lfsr_pool* pool, void* hip_stream, int32_t* h_active);

/* Non-blocking harvest: up to `cap` ids of retired jobs whose result is
 * complete in their d_hr_out, with their status (LFSR_OK, or the input error
 * of lfsr_get_stats) and the number of ADMM iterations they ran. */
lfsr_status lfsr_pool_poll(lfsr_pool* pool, int64_t* h_ids, int32_t* h_status, int32_t* h_iters, int32_t cap,
                           int32_t* h_count);

/* Occupancy: active and retiring jobs, free arena bytes, largest free block. */
lfsr_status lfsr_pool_info(const lfsr_pool* pool, int32_t* h_active, int32_t* h_retiring, size_t* h_free,
                           size_t* h_largest_free);

#ifdef __cplusplus
}
#endif

#endif /* LFSR_H */
