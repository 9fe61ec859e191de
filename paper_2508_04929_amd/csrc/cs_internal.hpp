// Internal declarations shared by the HIP translation units of libcryosplat.
//
// Data flow of one loss_and_grad call (all on the caller's stream):
//   k_build        per Gaussian: activations, Sigma = R diag(s)^2 R^T (Eq. 5)
//   k_bin_count    per (image, Gaussian): projection (Eq. 6, 8, 12, 13), cull,
//                  owner tile, per-block bin counts
//   k_bin_blockscan per bin: scan of the block counts, bin totals
//   k_scan         exclusive scans -> list offsets, work items (tile chunks)
//   k_bin_scatter  per (image, Gaussian): 32-byte splat record into its
//                  owner tile's segment of the list (stable: by index)
//   k_splat_fwd    per work item: additive splat (Eq. 9) into an LDS canvas
//                  covering the owner tile plus a halo -> partial canvases
//   k_canvas_reduce per tile: sum of the overlapping partial canvases -> Q
//   k_big_*        Gaussians wider than the halo: 64-bit fixed-point sums
//                  per image (order-free), then added to Q
//   FFT kernels    X = F^-1(H^ . F Q), residual, loss, G_Q = F^-1(H^ . F G_X)
//                  (Eq. 14, Sec. 3.3.5; H^ real and even -> self-adjoint)
//   k_splat_bwd    per work item: per-(image, Gaussian) pixel moments of
//                  G_Q against the splat (Eq. 16-20 need only these)
//   k_big_bwd      the same for wide Gaussians
//   k_chain        per Gaussian: moments -> screen gradients -> world frame,
//                  summed over images, then s, q, A chain rule (Eq. 18-21)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cs {

constexpr int kBlock = 256;                  // threads per block of every splat kernel
constexpr float kHalfLog2e = 0.72134752044448170368f;  // 0.5 * log2(e)
constexpr int kImgPerBinBlock = 8;           // images per block in the binning kernels

// Geometry of one rendering call, passed by value to the kernels.
struct Geom {
  int B;          // images
  int N;          // Gaussians
  int D;          // image side
  int c0;         // floor(D/2): the FFT-grid origin (Eq. 13)
  float pixel;    // Angstrom per pixel
  float qk;       // q_cut * 0.5 * log2(e): truncation in exp2 units
  int T;          // owner-tile side
  int halo;       // canvas halo
  int C;          // canvas side = T + 2 halo
  int S;          // LDS row stride of a canvas = C + 4 (padding for unrolled walks)
  int ntx;        // tiles per row
  int ntiles;     // tiles per image
  int K;          // bins per image = ntiles + 1 (last bin: wide Gaussians)
  int budget;     // Gaussians per work item
  int scale_act;  // 0 exp, 1 softplus
  int amp_act;    // 0 identity, 1 softplus
  int deal;       // 1: splat lanes take records in bank-dealt order
};

// One problem (mixture + its images) as seen by the persistent splat
// kernels, which drain the work queues of several problems in one launch.
struct ProbDev {
  Geom G;
  const float4 *list;   // splat records
  const int4 *items;    // work items
  const int *n_items;   // [0] item count, [1] wide-record count
  const float *wabs;    // |w| of every record, in list order
  int *queue;           // [0] forward, [1] backward work-queue counter
  float *partials;      // forward partial canvases
  const float *GQ;      // dL/dQ (backward)
  float *mom;           // pixel moments (backward)
};

constexpr int kMaxProblems = 16;

struct MultiProb {
  int count;
  ProbDev p[kMaxProblems];
};

// Per-image CTF description for the Fourier-space kernels.
struct CtfDev {
  const float *defocus_u, *defocus_v, *astig, *phase;  // [B] (astig/phase may be null)
  double lam;            // electron wavelength, Angstrom
  double cs;             // spherical aberration, Angstrom
  double w;              // amplitude contrast
  double bfactor;        // Angstrom^2
  int enabled;
};

// Mixed-radix (4, 2, 3) Stockham plan for one transform length.
struct FftPlan {
  int L;
  int nst;
  int radix[12];
};

// ----------------------------------------------------------------------------
// Device helpers
// ----------------------------------------------------------------------------

// Work index of block k of a grid of `total` blocks such that each XCD runs
// one contiguous run of work indices: the dispatcher deals workgroups to the
// eight XCDs in turn (block k to XCD k mod 8), so XCD x takes indices
// [start_x, start_x + count_x) in order, count_x = the number of k < total
// with k mod 8 = x.  Neighbouring work (sharing cache lines) then meets in
// one XCD's L2.  A bijection of [0, total) for any total.
__device__ __forceinline__ int xcd_work(int k, int total) {
  const int per = (total + 7) / 8, r = total % 8 == 0 ? 8 : total % 8;
  const int x = k % 8;
  return x * (per - 1) + min(x, r) + k / 8;
}

__device__ __forceinline__ float softplusf(float x) {
  return x > 20.f ? x : log1pf(__expf(x));
}
__device__ __forceinline__ float sigmoidf_(float x) { return 1.f / (1.f + __expf(-x)); }

// Projection of one Gaussian into one image.  Inputs: world mean and
// covariance (g0 = mu.xyz, A; g1 = Sxx Sxy Sxz Syy; g2 = Syz Szz), the first
// two rows p0, p1 of W and the shift.  Outputs in pixel units.
struct Proj {
  float u, v;            // centre: column and row coordinate (Eq. 13)
  float sxx, sxy, syy;   // projected covariance, Angstrom^2 (Eq. 12)
  float det;             // its determinant (floored at 1e-20)
  float al, be, ga;      // 0.5 log2(e) * pixel-unit conic: q = (a dj^2 + 2 b dj di + c di^2)
  float w;               // view-dependent weight A / (2 pi sqrt(det)) (Eq. 8), signed
  float hx, hy;          // half extents of the q_cut ellipse, pixels
};

__device__ __forceinline__ void project_one(const float4 g0, const float4 g1, const float2 g2,
                                            const float p0[3], const float p1[3], float tx,
                                            float ty, const Geom &G, Proj &P) {
  const float mx = p0[0] * g0.x + p0[1] * g0.y + p0[2] * g0.z + tx;
  const float my = p1[0] * g0.x + p1[1] * g0.y + p1[2] * g0.z + ty;
  // Sigma p0 and Sigma p1
  const float a0 = g1.x * p0[0] + g1.y * p0[1] + g1.z * p0[2];
  const float a1 = g1.y * p0[0] + g1.w * p0[1] + g2.x * p0[2];
  const float a2 = g1.z * p0[0] + g2.x * p0[1] + g2.y * p0[2];
  const float b0 = g1.x * p1[0] + g1.y * p1[1] + g1.z * p1[2];
  const float b1 = g1.y * p1[0] + g1.w * p1[1] + g2.x * p1[2];
  const float b2 = g1.z * p1[0] + g2.x * p1[1] + g2.y * p1[2];
  P.sxx = p0[0] * a0 + p0[1] * a1 + p0[2] * a2;
  P.sxy = p1[0] * a0 + p1[1] * a1 + p1[2] * a2;
  P.syy = p1[0] * b0 + p1[1] * b1 + p1[2] * b2;
  P.det = fmaxf(P.sxx * P.syy - P.sxy * P.sxy, 1e-20f);
  const float inv_det = 1.f / P.det;
  const float p2 = G.pixel * G.pixel;
  const float ip = 1.f / G.pixel;
  P.u = mx * ip + (float)G.c0;
  P.v = (float)G.c0 - my * ip;
  // pixel-unit conic: a = p^2 Cxx, b = -p^2 Cxy, c = p^2 Cyy with C = Sigma~^-1
  P.al = kHalfLog2e * p2 * P.syy * inv_det;
  P.be = kHalfLog2e * p2 * P.sxy * inv_det;
  P.ga = kHalfLog2e * p2 * P.sxx * inv_det;
  P.w = g0.w * rsqrtf(P.det) * 0.15915494309189535f;  // A / (2 pi sqrt(det))
  const float qc = G.qk * (1.f / kHalfLog2e);
  P.hx = sqrtf(qc * P.sxx) * ip;
  P.hy = sqrtf(qc * P.syy) * ip;
}

// Clamp a float pixel coordinate before int conversion (guards NaN/huge).
__device__ __forceinline__ int clamp_px(float x, int lo, int hi) {
  x = fminf(fmaxf(x, (float)lo), (float)hi);
  return (int)x;
}

// ----------------------------------------------------------------------------
// Kernels (definitions in k_geom.hip, k_splat.hip, k_fft.hip)
// ----------------------------------------------------------------------------

__global__ void k_build(const float *means, const float *log_scales, const float *quats,
                        const float *amps, Geom G, float4 *gc, int *zero_buf, int zero_count);

__global__ void k_bin_count(const float4 *gc, const float *rot, const float *shift, Geom G,
                            int *key, int *blk, int nbx);

__global__ void k_bin_blockscan(int *blk, int nbx, int *count);

__global__ void k_scan(int *count, Geom G, int *off, int4 *items, int *item_off,
                       int *n_items, int *queues, int *blk, int nbx);

__global__ void k_bin_scatter(const float4 *gc, const float *rot, const float *shift, Geom G,
                              const int *key, const int *off, const int *blk, int nbx,
                              float4 *list, float *wabs);

__global__ void k_splat_fwd(MultiProb MP);

__global__ void k_canvas_reduce(const float *partials, const int *item_off, const int4 *items,
                                Geom G, float *Q);

__global__ void k_big_prep(const int *off, const int *count, const float *wabs, Geom G,
                           double *wscale, long long *wq);

__global__ void k_big_fwd(const float4 *list, const int *off, const int *count,
                          const int *n_wide, Geom G, const double *wscale, long long *wq);

__global__ void k_big_add(const int *count, Geom G, const double *wscale, const long long *wq,
                          float *Q);

__global__ void k_splat_bwd(MultiProb MP);

__global__ void k_big_bwd(const float4 *list, const int *off, const int *count,
                          const int *n_wide, Geom G, const float *GQ, float *mom);

__global__ void k_chain(const float4 *gc, const float *log_scales, const float *quats,
                        const float *amps, const float *rot, const float *shift, Geom G,
                        const int *key, const float *mom, float *g_means, float *g_log_scales,
                        float *g_quats, float *g_amps);

constexpr int kPoseImg = 8;    // images per block of k_pose_grad_part
constexpr int kPoseGauss = 4;  // Gaussians per thread of k_pose_grad_part
__global__ void k_pose_grad_part(const float4 *gc, const float *rot, const float *shift, Geom G,
                                 const int *key, const float *mom, float *part);
__global__ void k_pose_grad_sum(const float *part, int B, int nblk, float *g_rot, float *g_shift);

__global__ void k_pair_count(const float4 *gc, const float *rot, const float *shift, Geom G,
                             unsigned long long *counts);

__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                       float b1, float b2, float eps, float bc1, float bc2);

__global__ void k_fill(float *p, int64_t n, float value);

__global__ void k_check_finite(const float *p, int64_t n, int bit, int *flag);

__global__ void k_twiddles(int L, float2 *tw);

__global__ void k_fft_rows_fwd(const float *src, FftPlan P, const float2 *tw, int B, float2 *spec);

__global__ void k_ctf_table(int L, float pixel, CtfDev ctf, int B, float *table);

__global__ void k_fft_cols_ctf(float2 *spec, FftPlan P, const float2 *tw, int B, int cpw,
                               const float *table);

__global__ void k_fft_cols_shift(float2 *spec, FftPlan P, const float2 *tw, int cpw,
                                 const float *shift, float inv_pixel, float sign);
__global__ void k_fft_rows_inv(const float2 *spec, FftPlan P, const float2 *tw, int B,
                               float *dst);

__global__ void k_fft_rows_inv_loss(float2 *spec, FftPlan P, const float2 *tw, int B,
                                    const float *obs, float *images_out, float grad_scale,
                                    float *loss_part);

__global__ void k_fft_axis(float2 *data, FftPlan P, const float2 *tw, int inner, int cpw);

__global__ void k_fft_cols_power(const float2 *spec, FftPlan P, const float2 *tw, int B, int cpw,
                                 unsigned short *out, size_t ld);
__global__ void k_loss_reduce(const float *loss_part, int B, int parts, float scale, float *loss);

__global__ void k_loss_total(float *loss, int B);

__global__ void k_residual(float *Q, const float *obs, float *images_out, int B, int D,
                           float grad_scale, float *loss_part);

}  // namespace cs
