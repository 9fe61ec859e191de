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

__global__ void k_train_record(const float *src, float *dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

}  // namespace cs
