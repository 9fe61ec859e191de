// Host-side context shared by the C-ABI translation units.
#pragma once

#include <cstdarg>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/cryosplat.h"
#include "cs_internal.hpp"

struct cs_ctx {
  int device = 0;
  std::string err;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  size_t ws_max = 0;  // 0 = unlimited
  int n_cu = 256;
  std::map<int, float2 *> twiddles;
  // stage timing
  bool timing = false;
  struct Pending { const char *name; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::map<std::string, std::pair<double, int64_t>> stage_ms;
  // graph capture
  bool capturing = false;
  hipStream_t cap_stream = nullptr;
  std::map<std::string, hipGraphExec_t> graphs;
  // autotuner cache: signature -> (tile, halo, budget)
  std::map<std::string, std::vector<int>> tuned;
  std::string tune_file;
  // scratch of the standalone network-layer entry points
  void *aux = nullptr;
  size_t aux_bytes = 0;
  // scratch of the voxelisation and FSC entry points
  void *vol = nullptr;
  size_t vol_bytes = 0;
  // scratch of the training loop (gradients, staged image) and FourierShift
  void *train = nullptr;
  size_t train_bytes = 0;
  // debug checks (CS_ERR_NONFINITE): device flag, enabled by cs_set_debug_checks
  // or CS_DEBUG_CHECKS=1 in the environment at cs_create
  bool debug_checks = false;
  int *check_flag = nullptr;
  // device address of the library's static scratch array on this context's
  // device (cs_loss_and_grad_noalloc); null if the lookup at cs_create failed
  char *scratch = nullptr;
  std::string scratch_err;
};

namespace cs {

inline int fail(cs_ctx *c, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

// Shared host helpers (api.hip).
bool fft_plan(int L, FftPlan &P);                          // radix (4, 2, 3) plan, L <= 512
double electron_wavelength_A(double kv);                  // relativistic, Angstrom
int get_twiddles(cs_ctx *ctx, int L, const float2 **out);  // cached device table
int fft_cols_per_block(int D, int64_t B);                   // columns per block of the column pass
CtfDev make_ctf(const cs_ctf *ctf);                        // disabled when ctf is null
float ctf_pixel(const cs_ctf *ctf, float geometry_pixel);  // pixel of the CTF's frequency grid
// one loss-and-gradient problem, eager or through the context's graph cache
int run_loss(cs_ctx *ctx, const cs_problem &pr, bool use_graph, hipStream_t st);

}  // namespace cs

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) return cs::fail(ctx, CS_ERR_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCHCHK(name)                                                              \
  do {                                                                               \
    hipError_t e_ = hipGetLastError();                                               \
    if (e_ != hipSuccess) return cs::fail(ctx, CS_ERR_HIP, "launch %s: %s", name, hipGetErrorString(e_)); \
  } while (0)

// Launch with optional event bracketing (stage timing; off during capture).
#define TLAUNCH(kernel, grid, block, lds, st, ...)                                   \
  do {                                                                               \
    hipEvent_t ea_ = nullptr, eb_ = nullptr;                                         \
    const bool tm_ = ctx->timing && !ctx->capturing;                                 \
    if (tm_) {                                                                       \
      (void)hipEventCreate(&ea_);                                                    \
      (void)hipEventCreate(&eb_);                                                    \
      (void)hipEventRecord(ea_, st);                                                 \
    }                                                                                \
    hipLaunchKernelGGL(kernel, grid, block, lds, st, __VA_ARGS__);                   \
    LAUNCHCHK(#kernel);                                                              \
    if (tm_) {                                                                       \
      (void)hipEventRecord(eb_, st);                                                 \
      ctx->pending.push_back({#kernel, ea_, eb_});                                   \
    }                                                                                \
  } while (0)

namespace cs {

// Grow-only device buffer (synchronises the device before a reallocation).
inline int grow(cs_ctx *ctx, void **p, size_t *cap, size_t bytes) {
  if (bytes <= *cap) return CS_OK;
  HIPCHK(hipDeviceSynchronize());
  if (*p) HIPCHK(hipFree(*p));
  *p = nullptr;
  *cap = 0;
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, CS_ERR_OOM, "allocation of %zu bytes", bytes);
  }
  *cap = bytes;
  return CS_OK;
}

}  // namespace cs
