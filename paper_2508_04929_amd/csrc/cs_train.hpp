// Training-loop kernels (Alg. 1; Sec. 4.1).
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace cs {

// Per-image CTF arrays of the data set (NULL defocus_u: no CTF).
struct TrainCtfSrc {
  const float *defocus_u, *defocus_v, *astig, *phase;
};

// Fixed buffers one training step reads: image [D][D], rotation [9], CTF
// values (defocus_u, defocus_v, astig, phase).
struct TrainStage {
  float *image, *rot, *ctf;
};

__global__ void k_init_attributes(const float *z, int64_t n, float scale_pre, float amp_pre,
                                  float *params);
__global__ void k_train_gather(const float *images, const float *rot, TrainCtfSrc src, int64_t idx,
                               int npix, TrainStage stage, const float *rec_src, float *rec_dst);
__global__ void k_train_record(const float *src, float *dst);
__global__ void k_split_gaussians(const float *__restrict__ p, const float *__restrict__ m,
                                  const float *__restrict__ v, int64_t n, int scale_act, int amp_act,
                                  float *__restrict__ q, float *__restrict__ qm,
                                  float *__restrict__ qv);

}  // namespace cs
