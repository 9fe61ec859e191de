// Kernels of the batch-1 training loop (Alg. 1; Sec. 4.1).
#include "cs_internal.hpp"
#include "cs_train.hpp"

namespace cs {

// Initial pre-activation parameters in the flat layout
// means | log_scales | quats | amps: means = 0.075 z (box units), every
// log-scale and amplitude the given pre-activation constant, quaternion
// (1, 0, 0, 0).
__global__ void __launch_bounds__(256)
k_init_attributes(const float *z, int64_t n, float scale_pre, float amp_pre, float *params) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float *means = params, *ls = params + 3 * n, *q = params + 6 * n, *a = params + 10 * n;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    means[3 * i + k] = 0.075f * z[3 * i + k];
    ls[3 * i + k] = scale_pre;
  }
  q[4 * i] = 1.f;
  q[4 * i + 1] = 0.f;
  q[4 * i + 2] = 0.f;
  q[4 * i + 3] = 0.f;
  a[i] = amp_pre;
}

// Copy image `idx` of the data set (pixels, rotation, CTF values) into the
// fixed staging buffers the step reads, and record the previous step's loss.
__global__ void __launch_bounds__(256)
k_train_gather(const float *images, const float *rot, TrainCtfSrc src, int64_t idx, int npix,
               TrainStage stage, const float *rec_src, float *rec_dst) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const float *img = images + idx * (int64_t)npix;
  for (int k = i; k < npix; k += gridDim.x * 256) stage.image[k] = img[k];
  if (i < 9) stage.rot[i] = rot[9 * idx + i];
  if (i == 0) {
    if (src.defocus_u) {
      stage.ctf[0] = src.defocus_u[idx];
      stage.ctf[1] = src.defocus_v[idx];
      stage.ctf[2] = src.astig ? src.astig[idx] : 0.f;
      stage.ctf[3] = src.phase ? src.phase[idx] : 0.f;
    }
    if (rec_dst) *rec_dst = *rec_src;
  }
}

// SplitGaussian (Alg. 1 densification), moment-preserving: the largest axis k
// (compared on the stored pre-activations, lowest index among equals), its
// scale s_k and direction u = R(q) e_k; children at mu +- (s_k / 2) u with
// s_k' = s_k sqrt(3) / 2 and amplitude A / 2 (other scales and the
// quaternion kept), so each pair keeps its parent's mass, mean and
// covariance.  Output index i (+ side) and N + i (- side); the Adam
// moments (if given) are copied to both children.  FP64 arithmetic.
__device__ __forceinline__ double softplus_d(double x) { return x > 30.0 ? x : log1p(exp(x)); }

__global__ void __launch_bounds__(256)
k_split_gaussians(const float *__restrict__ p, const float *__restrict__ m,
                  const float *__restrict__ v, int64_t n, int scale_act, int amp_act,
                  float *__restrict__ q, float *__restrict__ qm, float *__restrict__ qv) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t n2 = 2 * n;
  // every input value of this Gaussian is read before anything is written
  // (the outputs never overlap the inputs: restrict), so the loads are in
  // flight together
  float mu[3], ls[3], qt[4], mv[2][11];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    mu[c] = p[3 * i + c];
    ls[c] = p[3 * n + 3 * i + c];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) qt[c] = p[6 * n + 4 * i + c];
  const float a = p[10 * n + i];
  if (qm) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const float *src = t ? v : m;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        mv[t][c] = src[3 * i + c];
        mv[t][3 + c] = src[3 * n + 3 * i + c];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) mv[t][6 + c] = src[6 * n + 4 * i + c];
      mv[t][10] = src[10 * n + i];
    }
  }
  int k = 0;
  float lk = ls[0];
  if (ls[1] > lk) { k = 1; lk = ls[1]; }
  if (ls[2] > lk) { k = 2; lk = ls[2]; }
  const double sk = scale_act ? softplus_d((double)lk) : exp((double)lk);
  double w = qt[0], x = qt[1], y = qt[2], z = qt[3];
  const double nq = fmax(sqrt(w * w + x * x + y * y + z * z), 1e-12);
  w /= nq; x /= nq; y /= nq; z /= nq;
  double u0, u1, u2;  // column k of R(q)
  if (k == 0) {
    u0 = w * w + x * x - y * y - z * z; u1 = 2.0 * (x * y + w * z); u2 = 2.0 * (x * z - w * y);
  } else if (k == 1) {
    u0 = 2.0 * (x * y - w * z); u1 = w * w - x * x + y * y - z * z; u2 = 2.0 * (y * z + w * x);
  } else {
    u0 = 2.0 * (x * z + w * y); u1 = 2.0 * (y * z - w * x); u2 = w * w - x * x - y * y + z * z;
  }
  const double h = 0.5 * sk;
  const double d[3] = {h * u0, h * u1, h * u2};
  const double shrunk = 0.86602540378443865 * sk;  // sqrt(3) / 2
  const float lk_new = (float)(scale_act ? log(expm1(shrunk)) : log(shrunk));
  const double A = amp_act ? softplus_d((double)a) : (double)a;
  const float a_new = (float)(amp_act ? log(expm1(0.5 * A)) : 0.5 * A);
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int64_t j = i + side * n;
    const double sg = side ? -1.0 : 1.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      q[3 * j + c] = (float)((double)mu[c] + sg * d[c]);
      q[3 * n2 + 3 * j + c] = c == k ? lk_new : ls[c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) q[6 * n2 + 4 * j + c] = qt[c];
    q[10 * n2 + j] = a_new;
    if (qm) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        float *dst = t ? qv : qm;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          dst[3 * j + c] = mv[t][c];
          dst[3 * n2 + 3 * j + c] = mv[t][3 + c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) dst[6 * n2 + 4 * j + c] = mv[t][6 + c];
        dst[10 * n2 + j] = mv[t][10];
      }
    }
  }
}

__global__ void k_train_record(const float *src, float *dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

}  // namespace cs
