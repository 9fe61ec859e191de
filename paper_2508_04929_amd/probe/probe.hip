// Chip-rate probes for the benchmark's roofline: how fast this MI355X
// issues FP32 VALU instructions, v_exp_f32, LDS reads, BF16 MFMA and HBM
// copies, and at what shader clock.  Measurement only: nothing in the
// renderer calls these.  Every kernel runs a bounded loop over registers or
// its own LDS and writes one value per thread, so the work cannot be
// removed by the compiler; the host wrappers time one launch with HIP
// events on the null stream and synchronise.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kThreads = 256;

// Per block: shader-clock and constant-clock stamps at start and end (lane 0
// of wave 0), so the host can state the clock the loop ran at.
__device__ __forceinline__ void stamp(unsigned long long *clk, int slot) {
  if (threadIdx.x == 0) {
    clk[4 * blockIdx.x + slot] = clock64();
    clk[4 * blockIdx.x + 2 + slot] = wall_clock64();
  }
}

// Eight independent FMA chains, unrolled by four: 32 v_fma_f32 per pass.
__global__ void __launch_bounds__(kThreads) k_fma(float *out, unsigned long long *clk, int iters) {
  stamp(clk, 0);
  float a0 = threadIdx.x * 1e-3f, a1 = a0 + 1.f, a2 = a0 + 2.f, a3 = a0 + 3.f;
  float a4 = a0 + 4.f, a5 = a0 + 5.f, a6 = a0 + 6.f, a7 = a0 + 7.f;
  const float x = 0.9999999f, y = 1e-7f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a0 = fmaf(a0, x, y); a1 = fmaf(a1, x, y); a2 = fmaf(a2, x, y); a3 = fmaf(a3, x, y);
      a4 = fmaf(a4, x, y); a5 = fmaf(a5, x, y); a6 = fmaf(a6, x, y); a7 = fmaf(a7, x, y);
    }
  }
  stamp(clk, 1);
  out[blockIdx.x * kThreads + threadIdx.x] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7;
}

// Eight independent v_exp_f32 chains (the argument stays in [-1, 0]),
// unrolled by four: 32 transcendentals per pass.
__global__ void __launch_bounds__(kThreads) k_exp(float *out, unsigned long long *clk, int iters) {
  stamp(clk, 0);
  float a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = -0.1f * (float)(k + 1) - threadIdx.x * 1e-5f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] = -__builtin_amdgcn_exp2f(a[k]);
  }
  stamp(clk, 1);
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// LDS reads: every lane reads 16 bytes per instruction from a 32 KiB array,
// consecutive lanes from consecutive slots (no bank conflict), 32 reads of
// distinct slots per pass at constant offsets from one address.
__global__ void __launch_bounds__(kThreads) k_lds(float *out, unsigned long long *clk, int iters) {
  __shared__ float4 buf[2048];
  for (int i = threadIdx.x; i < 2048; i += kThreads) buf[i] = make_float4(i, i + 1, i + 2, i + 3);
  __syncthreads();
  stamp(clk, 0);
  float4 acc = make_float4(0, 0, 0, 0);
  int base = threadIdx.x;  // in [0, 1024): base + 32 u stays below 2048
  for (int i = 0; i < iters; ++i) {
    const float4 *p = buf + base;
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const float4 v = p[32 * u];
      acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
    }
    base = (base + 64) & 1023;
  }
  stamp(clk, 1);
  out[blockIdx.x * kThreads + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

// BF16 MFMA: four independent v_mfma_f32_16x16x32_bf16 accumulators per
// wave, unrolled by four: 16 MFMA per pass.
__global__ void __launch_bounds__(kThreads) k_mfma(float *out, unsigned long long *clk, int iters) {
  stamp(clk, 0);
  bf16x8 a, b;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    a[k] = (short)(0x3f80 + ((threadIdx.x + k) & 7));  // bfloat16 values near 1
    b[k] = (short)(0x3c00 + ((threadIdx.x * 3 + k) & 7));
  }
  f32x4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c3, 0, 0, 0);
    }
  }
  stamp(clk, 1);
  out[blockIdx.x * kThreads + threadIdx.x] = c0[0] + c1[1] + c2[2] + c3[3];
}

// Copy: each block copies one contiguous range of float4 (the fastest of the
// copy patterns measured here), four 16-byte loads in flight per lane
// before their stores.
__global__ void __launch_bounds__(kThreads) k_copy(const float4 *src, float4 *dst, int64_t n4,
                                                   int64_t per_block) {
  const int64_t b0 = (int64_t)blockIdx.x * per_block;
  const int64_t b1 = b0 + per_block < n4 ? b0 + per_block : n4;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 4 * kThreads) {
    float4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = i + u * kThreads;
      v[u] = k < b1 ? src[k] : make_float4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = i + u * kThreads;
      if (k < b1) dst[k] = v[u];
    }
  }
}

template <class F>
double timed(F launch) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0;
  }
  (void)hipEventRecord(e0, nullptr);
  launch();
  (void)hipEventRecord(e1, nullptr);
  float ms = -1.f;
  const bool ok = hipGetLastError() == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                  hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ok ? (double)ms : -1.0;
}

}  // namespace

extern "C" {

// Each probe: blocks of 256 threads, `iters` passes of its loop; `out` holds
// blocks * 256 floats and `clk` blocks * 4 stamps (device memory, caller
// owned).  Returns the launch time in milliseconds, or a negative value on a
// HIP error.  Per pass and wave: 32 FP32 FMA (k_fma), 32 v_exp_f32 (k_exp),
// 32 16-byte LDS reads (k_lds), 16 BF16 MFMA 16x16x32 (k_mfma).
double csp_fma(float *out, unsigned long long *clk, int blocks, int iters) {
  return timed([&] { hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(kThreads), 0, nullptr, out, clk, iters); });
}
double csp_exp(float *out, unsigned long long *clk, int blocks, int iters) {
  return timed([&] { hipLaunchKernelGGL(k_exp, dim3(blocks), dim3(kThreads), 0, nullptr, out, clk, iters); });
}
double csp_lds(float *out, unsigned long long *clk, int blocks, int iters) {
  return timed([&] { hipLaunchKernelGGL(k_lds, dim3(blocks), dim3(kThreads), 0, nullptr, out, clk, iters); });
}
double csp_mfma(float *out, unsigned long long *clk, int blocks, int iters) {
  return timed([&] { hipLaunchKernelGGL(k_mfma, dim3(blocks), dim3(kThreads), 0, nullptr, out, clk, iters); });
}
// Copy n4 float4 from src to dst (device memory, non-overlapping).
double csp_copy(const void *src, void *dst, int64_t n4, int blocks) {
  if (blocks < 1) return -1.0;
  const int64_t per = (n4 + blocks - 1) / blocks;
  return timed([&] {
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(kThreads), 0, nullptr, (const float4 *)src,
                       (float4 *)dst, n4, per);
  });
}
// The constant clock's rate in kHz (the reference for the stamps).
int csp_wall_clock_khz(int device) {
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess) return -1;
  return khz;
}

}  // extern "C"
