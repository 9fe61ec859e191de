/*
 * cryosplat.h -- C-ABI of the MI355X (gfx950) differentiable splat renderer.
 *
 * The library renders a 3-D anisotropic Gaussian mixture into CTF-modulated
 * 2-D projection images and back-propagates a squared-error image loss to
 * the Gaussians (cryoSplat, arXiv 2508.04929):
 *
 *   image formation     Y = H * int V(W^T r + t) dr_z            Sec. 3.2, Eq. 1
 *   mixture             V(r) = sum_n A_n G_n(r), G normalised    Sec. 3.3.1, Eq. 2, 4
 *   covariance          Sigma = R S S^T R^T, S = diag(s)          Eq. 5
 *   viewing transform   mu' = W mu (+ t), Sigma' = W Sigma W^T    Sec. 3.3.2, Eq. 6
 *   projection          drop z; G~ = exp(-d^T S~^-1 d/2)/(2 pi |S~|^1/2)
 *                                                                 Sec. 3.3.3, Eq. 7-8, 12
 *   splat sum           Q = sum_n A_n G~_n  (additive, no alpha)  Eq. 9
 *   FFT-aligned raster  Q_ij = Q((j-c)p, -(i-c)p), c = floor(D/2) Sec. 3.3.4, Eq. 13
 *   CTF                 X = F^-1(H^ . F(Q))                       App. A.2, Eq. 14
 *   loss                L = scale * sum ||X - Y||^2               Sec. 3.3.5
 *   gradients           Eq. 15-21 (App. A.2)
 *
 * Conventions fixed by this library (readings of the paper):
 *   - quaternions are scalar-first (w, x, y, z) and are normalised inside;
 *     a quaternion of norm below 1e-12 is treated as norm 1e-12;
 *   - scales are s = exp(log_scale) (scale_act = CS_ACT_EXP) or
 *     softplus(log_scale) (CS_ACT_SOFTPLUS, the paper's choice); amplitudes
 *     are used as given (CS_ACT_IDENTITY) or through softplus;
 *   - rot[b] is the 3x3 row-major world-to-view rotation W; the projected
 *     mean is P mu + t with P the first two rows of W and t = shift[b] an
 *     in-plane shift in Angstrom (the sign of the phase factor of Eq. 11);
 *   - the splat is point-sampled at pixel centres, clipped to the D x D
 *     image; terms with squared Mahalanobis distance above q_cut are
 *     dropped (default 2 ln 1e6, a relative truncation of about 1e-6);
 *   - the CTF is the weak-phase CTF with amplitude contrast w:
 *       CTF(s) = -(sqrt(1-w^2) sin chi + w cos chi) exp(-B s^2/4),
 *       chi = pi lam df(a) s^2 - pi/2 Cs lam^3 s^4 - phase,
 *       df(a) = (df_u+df_v)/2 + (df_u-df_v)/2 cos 2(a - astig),
 *     on the unshifted DFT grid (row frequencies carry the y-flip), made
 *     exactly even at the Nyquist row/column by averaging the two mirror
 *     values; the convolution is circular and unpadded.
 *
 * Memory: every array argument is DEVICE memory on the context's device,
 * FP32, C-contiguous, row-major, owned by the caller; the library never
 * frees or retains it.  The context owns a grow-on-demand workspace (freed
 * by cs_destroy).  All work is enqueued asynchronously on the given HIP
 * stream (NULL = the null stream); argument errors are returned before
 * anything is enqueued; device faults surface at the caller's next
 * synchronisation.  Gradient outputs are overwritten, never accumulated.
 *
 * Errors: every entry point returns CS_OK (0) or a negative cs_status; the
 * message of the last failure on a context is cs_last_error().  Calls on
 * one context are not thread-safe.
 */
#ifndef CRYOSPLAT_H
#define CRYOSPLAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cs_ctx cs_ctx;

typedef enum {
  CS_OK = 0,
  CS_ERR_INVALID_ARG = -1, /* null pointer, N < 0, B < 1, D < 1, pixel <= 0, ... */
  CS_ERR_UNSUPPORTED = -2, /* D not even with prime factors {2,3} when a CTF is used, D > 512 */
  CS_ERR_OOM = -3,         /* workspace allocation failed or exceeds CS_WORKSPACE_MAX bytes */
  CS_ERR_HIP = -4          /* a HIP runtime call failed */
} cs_status;

typedef enum { CS_SUM = 0, CS_MEAN = 1 } cs_reduction;

typedef enum { CS_ACT_EXP = 0, CS_ACT_SOFTPLUS = 1 } cs_scale_act;
typedef enum { CS_ACT_IDENTITY = 0, CS_ACT_SOFTPLUS_AMP = 1 } cs_amp_act;

/* Gaussian mixture (Sec. 3.3.1): 11 parameters per Gaussian. */
typedef struct {
  const float *means;      /* [N][3] world-frame means, Angstrom */
  const float *log_scales; /* [N][3] pre-activation scales */
  const float *quats;      /* [N][4] (w, x, y, z), any nonzero norm */
  const float *amps;       /* [N]    pre-activation amplitudes */
  int64_t n;               /* N >= 0; N = 0 renders zero images */
  int32_t scale_act;       /* cs_scale_act */
  int32_t amp_act;         /* cs_amp_act */
} cs_gaussians;

/* Images to render: poses (Eq. 1, 6) and raster geometry (Eq. 13). */
typedef struct {
  const float *rot;   /* [B][3][3] world-to-view rotations W, row-major */
  const float *shift; /* [B][2] in-plane shifts t in Angstrom, or NULL for 0 */
  int64_t b;          /* B >= 1 images */
  int32_t d;          /* image side D, 1 <= D <= 512 */
  float pixel;        /* pixel size p in Angstrom, > 0 */
} cs_views;

/* Per-image CTF parameters (App. A.2, Eq. 14); pass NULL for no CTF (X = Q). */
typedef struct {
  const float *defocus_u; /* [B] Angstrom */
  const float *defocus_v; /* [B] Angstrom */
  const float *astig;     /* [B] astigmatism angle, rad (or NULL = 0) */
  const float *phase;     /* [B] extra phase shift, rad (or NULL = 0) */
  double voltage_kv;      /* accelerating voltage, kV (> 0) */
  double cs_mm;           /* spherical aberration, mm */
  double amp_contrast;    /* amplitude contrast w in [0, 1) */
  double bfactor;         /* B-factor, Angstrom^2 (0 = no envelope) */
} cs_ctf;

/* Gradient outputs, same shapes as the cs_gaussians arrays (overwritten).
 * Any member may be NULL to skip that output. */
typedef struct {
  float *means;
  float *log_scales;
  float *quats;
  float *amps;
} cs_grads;

/* Launch options; pass NULL for defaults.  Results do not depend on tile,
 * halo or budget beyond floating-point summation order (for fixed options
 * every result is bitwise reproducible). */
typedef struct {
  float q_cut;    /* squared-Mahalanobis truncation; <= 0 selects 2 ln 1e6 */
  int32_t tile;   /* owner-tile side in pixels (16..128); 0 = automatic */
  int32_t halo;   /* canvas halo in pixels (0..tile); 0 = automatic */
  int32_t budget; /* Gaussians per work item (>= 64); 0 = automatic */
  int32_t graph;  /* cs_loss_and_grad: 1 = capture the launch sequence once per
                     argument signature (shapes, pointers, scalars) as a HIP
                     graph and replay it; the first call with a signature
                     must not itself be inside a caller's stream capture */
} cs_options;

/* Create a context on HIP device `device`.  *out receives the handle. */
int cs_create(int device, cs_ctx **out);

/* Release the context and its workspace (synchronises the device). */
void cs_destroy(cs_ctx *ctx);

/* Message of the last failure on ctx (empty string if none; never NULL). */
const char *cs_last_error(const cs_ctx *ctx);

/* Forward render (Alg. 2 Rasterize followed by ApplyCTF, Alg. 1):
 * images[B][D][D] = X (with ctf) or Q (ctf == NULL). */
int cs_render(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v,
              const cs_ctf *ctf, const cs_options *opt, float *images,
              void *stream);

/* Adjoint of cs_render (App. A.2, Eq. 15-21): given d_images = dL/dimages
 * [B][D][D], writes dL/d{means, log_scales, quats, amps}. */
int cs_render_backward(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v,
                       const cs_ctf *ctf, const cs_options *opt,
                       const float *d_images, cs_grads *grads, void *stream);

/* Fused forward + loss + adjoint (Sec. 3.3.5, App. A.2):
 *   loss[b] = scale * ||X_b - observed_b||^2 for b < B, loss[B] = sum_b loss[b]
 *   scale = 1 (CS_SUM) or 1/(B D^2) (CS_MEAN).
 * loss: device [B+1]; grads may be NULL (loss only); images_out [B][D][D]
 * receives X when not NULL. */
int cs_loss_and_grad(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v,
                     const cs_ctf *ctf, const cs_options *opt,
                     const float *observed, int32_t reduction, float *loss,
                     cs_grads *grads, float *images_out, void *stream);

/* One independent rendering problem of a batched call: a mixture, its
 * images (each problem has its own D and pixel size), CTF (NULL = none),
 * launch options (zeros = defaults), observed images and outputs.  Loss and
 * gradient semantics are those of cs_loss_and_grad; a problem whose four
 * gradient pointers are all NULL is evaluated without its adjoint. */
typedef struct {
  cs_gaussians g;
  cs_views v;
  const cs_ctf *ctf;
  cs_options opt;
  const float *observed; /* [B][D][D] */
  int32_t reduction;     /* CS_SUM or CS_MEAN */
  float *loss;           /* device [B+1] */
  cs_grads grads;
  float *images_out;     /* [B][D][D] or NULL */
} cs_problem;

/* Batched forward + loss + adjoint over `count` independent problems
 * (uneven mixture sizes and image sides).  The per-problem setup kernels
 * run back to back; the forward and the adjoint splat are each ONE
 * persistent launch whose blocks drain the work queues of all problems in
 * order, so small problems do not leave the GPU idle.  With use_graph = 1
 * the whole sequence is captured once per argument signature into a HIP
 * graph and replayed with a single hipGraphLaunch on `stream`.
 * 1 <= count; every problem is validated as in cs_loss_and_grad. */
int cs_loss_and_grad_multi(cs_ctx *ctx, const cs_problem *problems, int32_t count,
                           int32_t use_graph, void *stream);

/* Launch-option autotuner: for every problem, times cs_loss_and_grad over
 * candidate (tile, halo, budget) settings (`reps` timed calls each, median)
 * and writes the fastest into problems[i].opt (q_cut and graph are kept).
 * Choices are cached per context by (D, N, B, pixel, CTF, q_cut) and, when
 * the environment variable CS_AUTOTUNE_CACHE names a file, persisted there
 * (a missing or malformed file means "no cached entries").  The problems'
 * output buffers are overwritten while tuning.  Synchronises `stream`. */
int cs_autotune(cs_ctx *ctx, cs_problem *problems, int32_t count, int32_t reps, void *stream);

/* Adam step (Alg. 1, Sec. 4.1) over `count` FP32 parameters in place:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps),  step >= 1. */
int cs_adam_step(cs_ctx *ctx, float *params, const float *grads, float *m,
                 float *v, int64_t count, int64_t step, float lr, float b1,
                 float b2, float eps, void *stream);

/* Number of (Gaussian, pixel) pairs with squared Mahalanobis distance at
 * most q_cut inside each image (the splat's algorithmic work), computed
 * in FP32 with the same projection as the renderer.
 * counts: device int64 [B]. */
int cs_pair_count(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v,
                  const cs_options *opt, int64_t *counts, void *stream);

/* Stage timing for measurement.  While enabled (enable != 0), every kernel
 * the library launches on ctx is bracketed by HIP events recorded on the
 * call's stream; enabling clears the accumulated totals.  Kernel names are
 * the library's stage names (e.g. "k_splat_fwd", "k_splat_bwd"). */
int cs_set_timing(cs_ctx *ctx, int enable);

/* Total milliseconds and launch count of stage `name` since timing was last
 * enabled (synchronises the recorded events).  Unknown names give 0. */
int cs_stage_time(cs_ctx *ctx, const char *name, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* CRYOSPLAT_H */
