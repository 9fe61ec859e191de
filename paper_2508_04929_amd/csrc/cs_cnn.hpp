// Launchers of the pose-proposal network kernels (k_cnn.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace cs {

typedef unsigned short bf16;  // raw bfloat16 bits

// 3x3 stride-2 pad-1 convolutions, NHWC activations, weights [Cout][3][3][Cin]
// (dgrad takes the transpose [Cin][3][3][Cout]).  Cin = 1 uses a VALU kernel
// (forward and weight gradient only); otherwise Cin, Cout are multiples of 8.
hipError_t conv_fwd(const bf16 *in, const bf16 *w, const float *bias, int B, int Hi, int Wi,
                    int Cin, int Cout, int relu, bf16 *out, float *out32, hipStream_t st);
// Inference: the first (1 -> 32) and second (32 -> 64) convolutions fused,
// ReLU after both; in0 [B][H0][H0] (H0 % 64 == 0) -> out [B][H0/4][H0/4][64].
hipError_t conv12_fwd(const bf16 *in0, const bf16 *w1, const float *b1, const bf16 *w2,
                      const float *b2, int B, int H0, bf16 *out, hipStream_t st);
hipError_t conv_dgrad(const bf16 *dout, const bf16 *wt, const bf16 *act_in, int B, int Hi, int Wi,
                      int Cin, int Cout, bf16 *din, float *din32, hipStream_t st);
hipError_t conv_wgrad(const bf16 *dout, const bf16 *in, int B, int Hi, int Wi, int Cin, int Cout,
                      float *part, size_t part_cap, float *dw, hipStream_t st);
// Linear layers, weights [Out][In] (dgrad takes [In][Out]); In, Out multiples of 8.
hipError_t lin_fwd(const bf16 *x, const bf16 *w, const float *bias, int B, int In, int Out,
                   int relu, bf16 *y, float *y32, hipStream_t st);
hipError_t lin_dgrad(const bf16 *dy, const bf16 *wt, const bf16 *x_act, int B, int In, int Out,
                     bf16 *dx, float *dx32, hipStream_t st);
hipError_t lin_wgrad(const bf16 *dy, const bf16 *x, int B, int In, int Out, float *part,
                     size_t part_cap, float *dw, hipStream_t st);
hipError_t colsum(const bf16 *g, int M, int N, float *part, size_t part_cap, float *out,
                  hipStream_t st);
hipError_t standardize(const float *img, int B, int npx, bf16 *out, hipStream_t st);
hipError_t head(const float *out8, int B, float *rot, float *shift, hipStream_t st);
hipError_t head_loss(const float *out8, const float *rot_t, const float *shift_t, int B,
                     float lambda, float *loss_part, bf16 *dout8, float *dout32, hipStream_t st);
hipError_t to_bf16(const float *w, int Cout, int taps, int Cin, bf16 *wb, bf16 *wt, hipStream_t st);
hipError_t f32_to_bf16(const float *x, int64_t n, bf16 *y, hipStream_t st);
hipError_t bf16_to_f32(const bf16 *x, int64_t n, float *y, hipStream_t st);
hipError_t sum_into(const float *part, int n, float *out, hipStream_t st);

}  // namespace cs
