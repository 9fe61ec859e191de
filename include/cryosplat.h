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
  CS_ERR_HIP = -4,         /* a HIP runtime call failed */
  CS_ERR_NONFINITE = -5    /* debug checks only: NaN or infinity in an input or output */
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
  int64_t b;          /* B images, 1 <= B <= 65535 */
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
  float pixel_a;          /* pixel size in Angstrom of the CTF's frequency grid
                             (index k -> k / (D pixel_a)); 0 = the geometry's own
                             pixel.  Lets the geometry use other length units,
                             e.g. the box-normalised [-1/2, 1/2] domain of
                             Sec. 4.1 (pixel 1/D), while the CTF stays physical. */
} cs_ctf;

/* Gradient outputs, same shapes as the cs_gaussians arrays (overwritten).
 * Any member may be NULL to skip that output.  rot [B][3][3] and shift
 * [B][2] are the gradients w.r.t. the views' rotation matrices (entry-wise,
 * the matrices taken as given, not constrained to SO(3); the third row does
 * not enter the image and gets 0) and shifts: the pose gradients that a
 * joint optimisation of poses and Gaussians needs (Sec. 5, limitation and future work),
 * from the same adjoint (App. A.2, Eq. 18 and 21):
 *   dL/dt = sum_n dL/dmu~_n,  dL/dP = sum_n (dL/dmu~_n mu_n^T + 2 dL/dSigma~_n P Sigma_n)
 * with P the first two rows of the rotation. */
typedef struct {
  float *means;
  float *log_scales;
  float *quats;
  float *amps;
  float *rot;
  float *shift;
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
  int32_t lane_order; /* 0 = each work item's Gaussians go to lanes in list
                         order; 1 = dealt so that the lanes of a wave start on
                         distinct LDS banks (pays for wide footprints);
                         2 = sorted by footprint shape (row count, then
                         widest span) so that the lanes of a wave walk
                         similar footprints (pays where sizes spread).  The
                         results are identical in every order. */
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

/* Size in bytes of the library's static device scratch (64 MiB), the
 * largest workspace cs_loss_and_grad_noalloc can use. */
#define CS_NOALLOC_SCRATCH_BYTES (64u << 20)

/* cs_loss_and_grad without any device allocation, for callers that cannot
 * allocate: code under HIP stream capture, tight serving or training loops,
 * harnesses that forbid hipMalloc.  Same arguments, results and errors as
 * cs_loss_and_grad, except:
 *   - the workspace is a static device array of CS_NOALLOC_SCRATCH_BYTES
 *     that the library holds on every device it runs on until the process
 *     ends (its address is looked up once per device by cs_create); a call
 *     whose workspace (about 32 B per Gaussian-image pair plus the canvases,
 *     spectra and moments of its B images) does not fit returns CS_ERR_OOM
 *     before anything is enqueued;
 *   - opt->graph is ignored (the call never captures or instantiates a
 *     graph itself; a caller may capture it into its own), stage timing is
 *     off and debug checks are not run;
 *   - every call on a device shares that device's scratch and leaves its
 *     contents behind; the kernels clear what must start at zero, so calls
 *     in sequence are independent, but calls that overlap in time on one
 *     device (two streams, two threads, two contexts) race and give
 *     undefined results.
 * On success the call makes no device allocation: no hipMalloc or hipFree,
 * no events, streams or graphs. */
int cs_loss_and_grad_noalloc(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v,
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

/* Debug checks (also enabled at cs_create by CS_DEBUG_CHECKS=1 in the
 * environment): after cs_render, cs_render_backward, cs_loss_and_grad and
 * cs_loss_and_grad_multi have enqueued their work, every input and output
 * array of the call is scanned on the device for NaN and infinity, the call
 * synchronises its stream and returns CS_ERR_NONFINITE (inputs are reported
 * before outputs) instead of CS_OK.  The outputs are still written.  Off by
 * default: the scan and the synchronisation cost time on every call. */
int cs_set_debug_checks(cs_ctx *ctx, int enable);

/* Total milliseconds and launch count of stage `name` since timing was last
 * enabled (synchronises the recorded events).  Unknown names give 0. */
int cs_stage_time(cs_ctx *ctx, const char *name, double *total_ms, int64_t *launches);


/* ======================================================================
 * Learned pose proposal.  The paper assumes known poses and names pose
 * estimation as future work (Sec. 3.3, Sec. 5); this part proposes a pose
 * per particle image with a small CNN trained on images this renderer
 * produces, and scores pose grids with the renderer's own image model.
 *
 * Network (cs_cnn): input a D x D image (D a multiple of 64, at most 512),
 * standardised per image (zero mean, unit variance); six 3x3 stride-2
 * pad-1 convolutions with 1 -> 32 -> 64 -> 128 -> 256 -> 256 -> 256
 * channels, each followed by ReLU; flatten (NHWC order) to
 * (D/64)^2 * 256 features; linear -> 256 + ReLU; linear -> 8 outputs:
 * a 6-D rotation representation (a1, a2) and a 2-D shift.  The rotation
 * is the Gram-Schmidt frame R = [b1 b2 b3] (columns), b1 = a1/|a1|,
 * b2 = normalise(a2 - (b1.a2) b1), b3 = b1 x b2.  Weights and activations
 * are BF16 (round to nearest even), accumulation is FP32 on MFMA, master
 * weights and Adam moments are FP32.  Parameters form one flat FP32
 * vector, per layer weight then bias; conv weights [Cout][3][3][Cin],
 * linear weights [Out][In].
 *
 * Training loss over a batch of B (mean over the batch):
 *   L = (1/B) sum_b ( ||R_b - R*_b||_F^2 + lambda ||t_b - t*_b||^2 ).
 * ====================================================================== */
typedef struct cs_cnn cs_cnn;

/* Allocate a network for D x D inputs and batches up to max_batch;
 * He-uniform initial weights from a SplitMix64 stream seeded by `seed`,
 * zero biases.  Synchronous.  Errors: CS_ERR_UNSUPPORTED for D outside
 * {64, 128, ..., 512}; CS_ERR_OOM. */
int cs_cnn_create(cs_ctx *ctx, int32_t D, int32_t max_batch, uint64_t seed, cs_cnn **out);
void cs_cnn_destroy(cs_cnn *net);
/* Number of FP32 parameters (weights and biases of all layers). */
int64_t cs_cnn_param_count(const cs_cnn *net);
/* Copy the FP32 parameters out of / into the network (device buffers of
 * cs_cnn_param_count floats); setting also refreshes the BF16 weights. */
int cs_cnn_get_params(cs_cnn *net, float *dst, void *stream);
int cs_cnn_set_params(cs_cnn *net, const float *src, void *stream);

/* Inference on B <= max_batch images [B][D][D] (FP32): rot [B][3][3]
 * row-major (the Gram-Schmidt frame), shift [B][2] (may be NULL), raw
 * [B][8] FP32 network outputs (may be NULL). */
int cs_cnn_forward(cs_cnn *net, const float *images, int32_t B, float *rot, float *shift,
                   float *raw, void *stream);

/* Inference from an input already standardised per image, bfloat16 [B][D][D]
 * (as cs_pose_batch_load writes it): cs_cnn_forward without its
 * standardisation step; the input stays the caller's (cs_cnn_tensor index 0
 * is not stored). */
int cs_cnn_forward_std(cs_cnn *net, const uint16_t *x, int32_t B, float *rot, float *shift,
                       float *raw, void *stream);

/* One training step: forward, loss (written to loss[0], device), backward
 * through every layer, then (apply_update != 0) one Adam step with
 * (beta1, beta2, eps) = (0.9, 0.999, 1e-8) and learning rate lr on all
 * parameters.  grads_out (device, cs_cnn_param_count floats, may be NULL)
 * receives the FP32 parameter gradient of this batch. */
int cs_cnn_train_step(cs_cnn *net, const float *images, const float *rot_target,
                      const float *shift_target, int32_t B, float lambda, float lr, float *loss,
                      float *grads_out, int32_t apply_update, void *stream);

/* Copy of a bfloat16 tensor the last forward / training step stored, for
 * inspection: grad = 0: index 0 = standardised input [B][D][D], index l (1..7)
 * = output of layer l-1 after ReLU (conv outputs NHWC, then the hidden
 * vector); grad = 1: the gradient w.r.t. the pre-activation of layer
 * index-1 (masked by its ReLU), index 8 = dL/d(outputs) [B][8] as stored.
 * B is that of the last call; capacity in elements.  cs_cnn_forward runs
 * the first two convolutions as one kernel and does not store index 1 (an
 * error after it); its other tensors equal those of a training step. */
int cs_cnn_tensor(cs_cnn *net, int32_t index, int32_t grad, uint16_t *dst, int64_t capacity,
                  void *stream);

/* Single layers of the network (BF16 tensors passed as raw uint16 bits).
 * conv: in NHWC [B][H][W][Cin], out [B][H/2][W/2][Cout], w [Cout][3][3][Cin],
 * bias [Cout] FP32 (may be NULL), padding 1, stride 2; H, W even; Cout a
 * multiple of 8; Cin a multiple of 8, or Cin = 1 (H = W, Cout <= 256) for
 * the first layer.  out_f32 (may be NULL) receives the FP32 values before rounding.
 * dgrad: din = conv^T(dout) with wt = w transposed to [Cin][3][3][Cout],
 * zeroed where act_in <= 0 (act_in may be NULL: no mask); Cin % 8 == 0.
 * wgrad: dw [Cout][3][3][Cin] FP32 = sum over batch and pixels (Cin = 1
 * needs Cout <= 32). */
int cs_bf16_conv3x3s2_forward(cs_ctx *ctx, const uint16_t *in, const uint16_t *w, const float *bias,
                              int32_t B, int32_t H, int32_t W, int32_t Cin, int32_t Cout,
                              int32_t relu, uint16_t *out, float *out_f32, void *stream);
int cs_bf16_conv3x3s2_dgrad(cs_ctx *ctx, const uint16_t *dout, const uint16_t *wt,
                            const uint16_t *act_in, int32_t B, int32_t H, int32_t W, int32_t Cin,
                            int32_t Cout, uint16_t *din, float *din_f32, void *stream);
int cs_bf16_conv3x3s2_wgrad(cs_ctx *ctx, const uint16_t *dout, const uint16_t *in, int32_t B,
                            int32_t H, int32_t W, int32_t Cin, int32_t Cout, float *dw,
                            void *stream);
/* linear: y [B][Out] = x [B][In] w^T + bias, w [Out][In]; In, Out multiples
 * of 8.  dgrad: dx [B][In] = dy wt^T with wt = w^T [In][Out], masked by
 * x_act > 0 (may be NULL).  wgrad: dw [Out][In] FP32 = dy^T x. */
int cs_bf16_linear_forward(cs_ctx *ctx, const uint16_t *x, const uint16_t *w, const float *bias,
                           int32_t B, int32_t In, int32_t Out, int32_t relu, uint16_t *y,
                           float *y_f32, void *stream);
int cs_bf16_linear_dgrad(cs_ctx *ctx, const uint16_t *dy, const uint16_t *wt, const uint16_t *x_act,
                         int32_t B, int32_t In, int32_t Out, uint16_t *dx, float *dx_f32,
                         void *stream);
int cs_bf16_linear_wgrad(cs_ctx *ctx, const uint16_t *dy, const uint16_t *x, int32_t B, int32_t In,
                         int32_t Out, float *dw, void *stream);
/* Pose head on raw outputs [B][8]: rot [B][3][3] and shift [B][2] (rot may
 * be NULL to skip); with rot_target, shift_target, loss and d_raw all set,
 * also the batch loss (loss[0]) and d_raw [B][8] = dL/draw (FP32). */
int cs_pose_head(cs_ctx *ctx, const float *raw, int32_t B, float *rot, float *shift,
                 const float *rot_target, const float *shift_target, float lambda, float *loss,
                 float *d_raw, void *stream);


/* ----------------------------------------------------------------------
 * Pose scoring with the renderer's image model (Sec. 3.2, Eq. 1; App. A.2,
 * Eq. 14; Sec. 3.3.5).  The score of rotation W and in-plane shift t for a
 * particle image Y with CTF H is the squared error ||H (P_W V + t) - Y||^2
 * of the splatted projection (Eq. 9, 13) shifted by t.  Shifts are whole
 * pixels (dx, dy) in [-r, r]^2, t = (dx, dy) * pixel in Angstrom in the
 * convention of the renderer (projected mean P mu + t), shift index
 * s = (dy + r)(2r + 1) + (dx + r); a shift moves the projection circularly,
 * which equals the rendered shift while the mixture stays r pixels away
 * from the image border.
 *
 * A bank holds, per rotation, the projection (no CTF) and its power
 * spectrum as bfloat16, rendered once by this library; searches score
 * particles against the bank with FP32 accumulation on MFMA:
 *   score = ||Y||^2 + ||H Q_W||^2 - 2 < shift_t(Q_W), H Y >.
 * ---------------------------------------------------------------------- */
typedef struct cs_pose_bank cs_pose_bank;

/* Rotation grid on the host: HEALPix (ring scheme, Gorski et al. 2005)
 * viewing directions with nside, times n_psi in-plane angles psi_m =
 * 2 pi m / n_psi.  Rotation (d, m) has index d * n_psi + m and is
 * W = Rz(psi_m) Ry(-theta_d) Rz(-phi_d) (row-major, world to view; its third
 * row is the viewing direction).  *count = 12 nside^2 n_psi; rot (HOST
 * memory, [count][9]) may be NULL to query the count. */
int cs_pose_grid(int32_t nside, int32_t n_psi, float *rot, int64_t *count);

/* Render the bank: rot device [K][9] (copied); n_psi > 0 declares that the
 * rotations form a (direction, psi) grid with psi the fastest index, as
 * cs_pose_grid builds (needed for proposal-driven refinement), 0 = no
 * structure.  D a multiple of 16 with prime factors 2 and 3, at most 512.
 * Memory: K (D^2 + D (D/2 + 1) rounded up to 128) * 2 bytes. */
int cs_pose_bank_create(cs_ctx *ctx, const cs_gaussians *g, const float *rot, int64_t K,
                        int32_t n_psi, int32_t D, float pixel, const cs_options *opt,
                        cs_pose_bank **out, void *stream);
void cs_pose_bank_destroy(cs_pose_bank *bank);
int64_t cs_pose_bank_size(const cs_pose_bank *bank);
/* Copy of the bank's rotations (device [K][9]). */
int cs_pose_bank_rotations(const cs_pose_bank *bank, float *rot, void *stream);

/* Exhaustive search: for each of P images [P][D][D] (device FP32, CTF
 * parameters per image as in cs_ctf, or ctf NULL for none) the minimum
 * score over all bank rotations and all (2r+1)^2 shifts, 0 <= r <= 4.
 * Outputs (device, [P]): best_rot (bank index), best_shift (shift index,
 * may be NULL), best_score (may be NULL); scores (may be NULL) receives
 * every score [P][K][(2r+1)^2].  Ties go to the smaller rot * S + s. */
int cs_pose_grid_search(cs_pose_bank *bank, const float *images, const cs_ctf *ctf, int32_t P,
                        int32_t shift_radius, int32_t *best_rot, int32_t *best_shift,
                        float *best_score, float *scores, void *stream);

/* Local refinement: the same score over L = n_dir * n_psi_c candidate
 * rotations per particle.  With a proposal (device [P][3][3] world-to-view
 * rotations) the candidates are the n_dir bank directions nearest the
 * proposal's viewing direction (largest dot product, ties to the smaller
 * direction index; n_dir <= 64), and for each the n_psi_c consecutive psi
 * indices around psi* = atan2(M01 - M10, M00 + M11), M = A_d W^T, which
 * maximises trace(W^T Rz(psi) A_d) (A_d = the bank rotation of direction d
 * at psi = 0); they are written to cand [P][L] when cand is not NULL.
 * Without a proposal, cand [P][L] (L = n_dir * n_psi_c) is the input list
 * of bank indices; entries outside [0, K) are skipped.  Outputs as for the
 * grid search (scores [P][L][(2r+1)^2]). */
int cs_pose_refine(cs_pose_bank *bank, const float *images, const cs_ctf *ctf, int32_t P,
                   const float *proposal, int32_t n_dir, int32_t n_psi_c, int32_t shift_radius,
                   int32_t *cand, int32_t *best_rot, int32_t *best_shift, float *best_score,
                   float *scores, void *stream);


/* Particle side of pose scoring, computed once per batch of particles and
 * shared by every search and refinement stage on any bank of the same D:
 * Z = H Y (the image filtered by its own CTF, the matched filter of the
 * image model), the (2r+1)^2 circularly shifted copies of -2 Z (bfloat16),
 * the energy weights w_f |H^|^2 / D^2 (bfloat16) and ||Y||^2.
 * create: capacity particles of side D (multiple of 16, prime factors 2
 * and 3, <= 512), shift radius 0 <= r <= 4; device memory about
 * capacity * D^2 * (2 (2r+1)^2 + 18) bytes.  load: P <= capacity images
 * [P][D][D] with per-particle CTF parameters (ctf NULL = no CTF); filtered
 * (may be NULL) receives Z [P][D][D] FP32; standardized (may be NULL)
 * receives Z standardised per image, (Z - mean) / std as bfloat16 [P][D][D],
 * the input of cs_cnn_forward_std (at D = 128 the mean and variance come
 * from the spectrum by Parseval's identity, so they can differ from a
 * two-pass computation in the last bits).  A batch is reused by later
 * loads; searches use the last load. */
typedef struct cs_pose_batch cs_pose_batch;
int cs_pose_batch_create(cs_ctx *ctx, int32_t D, float pixel, int32_t capacity,
                         int32_t shift_radius, cs_pose_batch **out);
void cs_pose_batch_destroy(cs_pose_batch *batch);
int cs_pose_batch_load(cs_pose_batch *batch, const float *images, const cs_ctf *ctf, int32_t P,
                       float *filtered, uint16_t *standardized, void *stream);
/* cs_pose_grid_search / cs_pose_refine on a loaded batch (same outputs;
 * the batch's shift radius applies).  best_rotation (may be NULL) receives
 * the winning rotation matrices [P][3][3] from the bank's table (NaN where
 * no candidate was scored), ready to serve as the next stage's proposal. */
int cs_pose_batch_search(cs_pose_bank *bank, cs_pose_batch *batch, int32_t *best_rot,
                         int32_t *best_shift, float *best_score, float *scores,
                         float *best_rotation, void *stream);
int cs_pose_batch_refine(cs_pose_bank *bank, cs_pose_batch *batch, const float *proposal,
                         int32_t n_dir, int32_t n_psi_c, int32_t *cand, int32_t *best_rot,
                         int32_t *best_shift, float *best_score, float *scores,
                         float *best_rotation, void *stream);

/* Fit of each loaded particle's winning pose (outputs of a search or
 * refinement on this batch): z[p] = (||Y||^2 - best_score[p]) / ||H Q_k||^2
 * with k = best_rot[p], which equals 2 a - 1 for a = <S_t Q_k, H Y> /
 * ||H Q_k||^2, the least-squares amplitude of the winning template in the
 * particle (Sec. 3.3.5 squared error expanded as for the scores).  Near 1
 * when the template at the winning pose explains the particle, lower when
 * it does not; a learned proposal uses it to send particles back to the
 * exhaustive search.  sigmas (may be NULL) receives the shortfall from a
 * perfect fit in units of the noise spread of z at the true pose of a
 * noise-dominated particle: s = (1 - z) ||H Q_k|| D / (2 ||Y||) (the spread
 * of z is 2 sigma / ||H Q_k|| with sigma^2 about ||Y||^2 / D^2).  NaN where
 * best_rot is outside the bank.  Device arrays [P] (P = the batch's last
 * load). */
int cs_pose_batch_confidence(cs_pose_bank *bank, cs_pose_batch *batch, const int32_t *best_rot,
                             const float *best_score, float *z, float *sigmas, void *stream);

/* The mixture read out as a volume (the voxelisation of the reconstruction
 * in the overview of Sec. 3): vol [D][D][D] (index [iz][iy][ix]) receives
 * sum_n A_n (2 pi)^-3/2 det(Sigma_n)^-1/2 exp(-q_n / 2) at (x, y, z) =
 * ((ix - D/2) p, (iy - D/2) p, (iz - D/2) p), over the Gaussians with
 * q_n = (x - mu_n)^T Sigma_n^-1 (x - mu_n) <= q_cut (q_cut <= 0: the
 * renderer's default 2 ln 1e6); the integral along z is the identity-pose
 * image (Eq. 8) up to the raster's row flip.  D a multiple of 8, at most
 * 512.  Every term is truncated to a common fixed-point grid (2^-61 of the
 * sum of |weights|) and the terms are summed exactly, so the result is the
 * same bit for bit whatever the order of the Gaussians.
 * Reads the (brick, Gaussian) pair count back from the device, so the call
 * waits for the stream and cannot be captured in a graph. */
int cs_voxelize(cs_ctx *ctx, const cs_gaussians *g, int32_t D, float pixel, float q_cut,
                float *vol, void *stream);

/* Fourier shell correlation of two volumes (Sec. 4, Eq. 10): fsc
 * [D/2 + 1] receives, for shells k = round(|(kx, ky, kz)|) = 0 .. D/2 of the
 * integer frequency grid, sum Re(Va^ conj Vb^) / sqrt(sum |Va^|^2 sum
 * |Vb^|^2) over the full spectrum (0 for a shell without energy); the
 * resolution is the first shell where it drops below 0.143.  D even with
 * prime factors 2 and 3, at most 512.  Shell sums are exact fixed-point sums
 * (reproducible). */
int cs_fsc(cs_ctx *ctx, const float *vol_a, const float *vol_b, int32_t D, float *fsc,
           void *stream);

/* Resolution read-out of an FSC curve (Sec. 4: the resolution at which the
 * FSC of Eq. 10 falls below 0.143): fsc [D/2 + 1] (device, as cs_fsc writes
 * it); shell [1] (device int32, may be NULL) receives the first shell
 * k >= 1 with fsc[k] < threshold, or D/2 when there is none; resolution [1]
 * (device float, may be NULL) receives D pixel / k in Angstrom.  At least
 * one output must be given; D even, at most 512; pixel > 0. */
int cs_fsc_resolution(cs_ctx *ctx, const float *fsc, int32_t D, float pixel, float threshold,
                      int32_t *shell, float *resolution, void *stream);

/* ApplyCTF of Alg. 1 for arbitrary images (App. A.2, Eq. 14):
 * out = F^-1(H^ . F images) [B][D][D], per-image CTF (NULL = identity);
 * D even with prime factors 2 and 3, at most 512; out may alias images. */
int cs_ctf_filter(cs_ctx *ctx, const float *images, const cs_ctf *ctf, int32_t B, int32_t D,
                  float pixel, float *out, void *stream);

/* Synthetic data: add white Gaussian noise to B images [B][D][D] in place
 * at a per-image SNR of snr_db (noise variance = image variance /
 * 10^(snr_db/10)), the noise model of the paper's synthetic study
 * (App. D.3).  Normals: Philox4x32-10 (Salmon et al. 2011) with key = seed
 * and counter (b + offset, pixel / 4), Box-Muller transform; identical
 * (seed, offset) give identical noise. */
int cs_add_noise(cs_ctx *ctx, float *images, int32_t B, int32_t D, float snr_db, uint64_t seed,
                 int64_t offset, void *stream);

/* ----------------------------------------------------------------------
 * Training loop of Alg. 1 with the settings of Sec. 4.1 (batch size 1,
 * one learning rate, box-normalised units)
 * ---------------------------------------------------------------------- */

/* FourierShift (Alg. 1, centre alignment; Sec. 4.1 applies the published
 * particle translations to the observed images by a phase shift in Fourier
 * space).  Translates every image of images [B][D][D] by direction * t_b,
 * t_b = shift[b] = (t_x, t_y) in the units of `pixel`, band-limited and
 * circular: the content at image-plane position r moves to r + direction *
 * t_b, i.e. a_c = direction t_x / p columns and a_r = -direction t_y / p
 * rows on the raster of Eq. 13; out = Re F^-1(F(Y) exp(-2 pi i (k_c a_c +
 * k_r a_r) / D)) with signed frequency indices, which on the Nyquist lines
 * of even D is the factor cos(pi a) (cos(pi (a_c + a_r)) at the corner).
 * direction = -1 centres images observed with translations t.  D even with
 * prime factors 2 and 3, at most 512; out may alias images.  Errors:
 * CS_ERR_INVALID_ARG (null pointer, B < 1, pixel <= 0, direction not +-1),
 * CS_ERR_UNSUPPORTED (D). */
int cs_fourier_shift(cs_ctx *ctx, const float *images, const float *shift, int64_t B, int32_t D,
                     float pixel, float direction, float *out, void *stream);

/* InitAttributes (Alg. 1) with the values of Sec. 4.1 in box units (domain
 * [-1/2, 1/2]^3): from normal draws z [N][3] (device) writes the flat
 * pre-activation parameters params [11 N] = means [N][3] | log_scales [N][3]
 * | quats [N][4] | amps [N]: means 0.075 z, every scale pre-activation
 * softplus^-1(0.0075), quaternion (1, 0, 0, 0), amplitude pre-activation
 * softplus^-1(1 / (2 N)); to be rendered with the softplus activations
 * (Sec. 3.3.1).  N >= 1. */
int cs_init_attributes(cs_ctx *ctx, const float *z, int64_t n, float *params, void *stream);

/* A training set for the batch-1 loop (device arrays; images already
 * centred, e.g. by cs_fourier_shift with direction -1). */
typedef struct {
  const float *images; /* [M][D][D] observed images */
  const float *rot;    /* [M][3][3] their world-to-view rotations W */
  int64_t m;           /* M >= 1 */
  int32_t d;           /* D, as for cs_loss_and_grad */
  float pixel;         /* geometry pixel, e.g. 1/D in box units */
} cs_dataset;

/* The inner loop of Alg. 1 at batch size 1 (Sec. 4.1): for k = 0 .. count-1
 * and image i = order[k] (host array, 0 <= i < M): Rasterize at rot[i],
 * ApplyCTF with image i's CTF (ctf: per-image arrays of length M, with
 * pixel_a for box units; NULL = none), Loss against images[i] (reduction,
 * Sec. 3.3.5), gradients (App. A.2), then one Adam step of every parameter
 * (step number step0 + k + 1; lr, b1, b2, eps) on the flat parameters
 * params [11 N] (layout of cs_init_attributes, activations scale_act /
 * amp_act) with moments adam_m, adam_v [11 N] (zero before the first step).
 * loss (device [count], or NULL) receives each step's loss before its
 * update.  With opt->graph = 1 the image, rotation and CTF values of a
 * step are first copied into fixed buffers, so that the loss path is one
 * replayed HIP graph per step; otherwise they are read in place.  Enqueued
 * on `stream`; identical inputs give identical bits, with or without the
 * graph. */
int cs_train_sequential(cs_ctx *ctx, float *params, float *adam_m, float *adam_v, int64_t n,
                        int32_t scale_act, int32_t amp_act, const cs_dataset *data,
                        const cs_ctf *ctf, const cs_options *opt, int32_t reduction,
                        const int64_t *order, int64_t count, int64_t step0, float lr, float b1,
                        float b2, float eps, float *loss, void *stream);

/* Densification (Alg. 1: IsDoubleGaussians / SplitGaussian; App. C.1 gives
 * no split rule).  Splits every Gaussian of the flat parameters params
 * [11 N] (layout of cs_init_attributes, activations scale_act / amp_act)
 * into two, written to out_params [22 N] (2N Gaussians, same layout): with
 * k the axis of the largest scale (compared on the stored pre-activations,
 * lowest index among equals), s_k its activated scale and u = R(q) e_k,
 * the children sit at mu + (s_k / 2) u (index i) and mu - (s_k / 2) u
 * (index N + i), with s_k' = s_k sqrt(3) / 2, amplitude A / 2 and the other
 * scales and the quaternion unchanged, so each pair keeps the parent's
 * mass, mean and covariance.  With adam_m, adam_v [11 N] and out_m, out_v
 * [22 N] (all four, or none) both children inherit the parent's moments.
 * Outputs must not overlap inputs or each other.  FP64 arithmetic, FP32
 * results. */
int cs_split_gaussians(cs_ctx *ctx, const float *params, const float *adam_m, const float *adam_v,
                       int64_t n, int32_t scale_act, int32_t amp_act, float *out_params,
                       float *out_m, float *out_v, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CRYOSPLAT_H */
