// Host side of libcryosplat: argument validation, workspace, launch order.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/cryosplat.h"
#include "cs_internal.hpp"

using namespace cs;

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
};

namespace {

constexpr float kDefaultQCut = 27.631021115928547f;  // 2 ln 1e6
constexpr int kDefaultTile = 64;
constexpr int kDefaultHalo = 16;
constexpr int kDefaultBudget = 2048;
constexpr int kMaxD = 512;

int fail(cs_ctx *c, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) return fail(ctx, CS_ERR_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

// Launch with optional event bracketing (stage timing).
#define TLAUNCH(kernel, grid, block, lds, st, ...)                                    \
  do {                                                                               \
    hipEvent_t ea_ = nullptr, eb_ = nullptr;                                         \
    if (ctx->timing) {                                                               \
      (void)hipEventCreate(&ea_);                                                    \
      (void)hipEventCreate(&eb_);                                                    \
      (void)hipEventRecord(ea_, st);                                                 \
    }                                                                                \
    hipLaunchKernelGGL(kernel, grid, block, lds, st, __VA_ARGS__);        \
    LAUNCHCHK(#kernel);                                                              \
    if (ctx->timing) {                                                               \
      (void)hipEventRecord(eb_, st);                                                 \
      ctx->pending.push_back({#kernel, ea_, eb_});                                   \
    }                                                                                \
  } while (0)

#define LAUNCHCHK(name)                                                              \
  do {                                                                               \
    hipError_t e_ = hipGetLastError();                                               \
    if (e_ != hipSuccess) return fail(ctx, CS_ERR_HIP, "launch %s: %s", name, hipGetErrorString(e_)); \
  } while (0)

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

bool fft_plan(int L, FftPlan &P) {
  if (L < 2 || L > kMaxD) return false;
  P.L = L;
  P.nst = 0;
  int r = L;
  while (r % 4 == 0) { P.radix[P.nst++] = 4; r /= 4; }
  while (r % 2 == 0) { P.radix[P.nst++] = 2; r /= 2; }
  while (r % 3 == 0) { P.radix[P.nst++] = 3; r /= 3; }
  return r == 1 && P.nst <= 12;
}

double electron_wavelength_A(double kv) {
  const double h = 6.62607015e-34, m0 = 9.1093837015e-31, e = 1.602176634e-19, c = 299792458.0;
  const double eV = e * kv * 1e3;
  return h / std::sqrt(2.0 * m0 * eV * (1.0 + eV / (2.0 * m0 * c * c))) * 1e10;
}

// Workspace carve-up for one call.
struct Layout {
  size_t gc = 0, key = 0, count = 0, off = 0, blk = 0, item_off = 0, n_items = 0, queues = 0,
         items = 0, list = 0, partials = 0, Q = 0, spec = 0, ctf = 0, mom = 0, loss_part = 0;
  size_t total = 0;
  int max_items = 0;
  int nbx = 0;  // Gaussian blocks of the binning kernels
};

Layout make_layout(const Geom &G, bool need_partials, bool need_mom, bool need_fft) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align_up(bytes); return at; };
  const size_t BN = (size_t)G.B * G.N;
  const size_t BK = (size_t)G.B * G.K;
  L.max_items = (int)((size_t)G.B * G.ntiles + (BN + G.budget - 1) / G.budget);
  L.gc = take((size_t)G.N * 48 + 16);
  L.key = take(BN * 4 + 4);
  L.count = take(BK * 4);
  L.off = take(BK * 4);
  L.nbx = (int)((G.N + kBlock - 1) / kBlock);
  L.blk = take(BK * (size_t)std::max(L.nbx, 1) * 4);
  L.item_off = take((BK + 1) * 4);
  L.n_items = take(16);
  L.queues = take(16);
  L.items = take((size_t)L.max_items * 16 + 16);
  L.list = take(BN * 32 + 32);
  if (need_partials) L.partials = take((size_t)L.max_items * G.C * G.C * 4);
  L.Q = take((size_t)G.B * G.D * G.D * 4);
  if (need_fft) {
    L.spec = take((size_t)G.B * G.D * (G.D / 2 + 1) * 8);
    L.ctf = take((size_t)G.B * G.D * (G.D / 2 + 1) * 4);
  }
  if (need_mom) L.mom = take(BN * 24 + 32);
  L.loss_part = take((size_t)G.B * G.D * 4);
  L.total = o;
  return L;
}

int ensure_ws(cs_ctx *ctx, size_t need, hipStream_t stream) {
  if (need <= ctx->ws_bytes) return CS_OK;
  if (ctx->ws_max && need > ctx->ws_max)
    return fail(ctx, CS_ERR_OOM, "workspace of %zu bytes exceeds CS_WORKSPACE_MAX=%zu", need,
                ctx->ws_max);
  if (ctx->ws) {
    HIPCHK(hipStreamSynchronize(stream));
    HIPCHK(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  size_t want = need + need / 4;
  if (ctx->ws_max && want > ctx->ws_max) want = need;
  if (hipMalloc(&ctx->ws, want) != hipSuccess) {
    (void)hipGetLastError();
    ctx->ws = nullptr;
    return fail(ctx, CS_ERR_OOM, "hipMalloc(%zu) failed", want);
  }
  ctx->ws_bytes = want;
  return CS_OK;
}

int get_twiddles(cs_ctx *ctx, int L, const float2 **out) {
  auto it = ctx->twiddles.find(L);
  if (it != ctx->twiddles.end()) { *out = it->second; return CS_OK; }
  std::vector<float2> h(L);
  for (int k = 0; k < L; ++k) {
    const double a = 2.0 * M_PI * (double)k / (double)L;
    h[k] = make_float2((float)std::cos(a), (float)-std::sin(a));
  }
  float2 *d = nullptr;
  HIPCHK(hipMalloc(&d, sizeof(float2) * L));
  HIPCHK(hipMemcpy(d, h.data(), sizeof(float2) * L, hipMemcpyHostToDevice));
  ctx->twiddles[L] = d;
  *out = d;
  return CS_OK;
}

int validate(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v, const cs_ctf *ctf,
             const cs_options *opt) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!g || !v) return fail(ctx, CS_ERR_INVALID_ARG, "null gaussians or views");
  if (g->n < 0) return fail(ctx, CS_ERR_INVALID_ARG, "negative Gaussian count");
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->amps))
    return fail(ctx, CS_ERR_INVALID_ARG, "null Gaussian parameter array");
  if (g->scale_act != 0 && g->scale_act != 1) return fail(ctx, CS_ERR_INVALID_ARG, "bad scale_act");
  if (g->amp_act != 0 && g->amp_act != 1) return fail(ctx, CS_ERR_INVALID_ARG, "bad amp_act");
  if (!v->rot) return fail(ctx, CS_ERR_INVALID_ARG, "null rotations");
  if (v->b < 1) return fail(ctx, CS_ERR_INVALID_ARG, "image count must be >= 1");
  if (v->d < 1) return fail(ctx, CS_ERR_INVALID_ARG, "image side must be >= 1");
  if (v->d > kMaxD) return fail(ctx, CS_ERR_UNSUPPORTED, "image side %d > %d", v->d, kMaxD);
  if (!(v->pixel > 0.f) || !std::isfinite(v->pixel))
    return fail(ctx, CS_ERR_INVALID_ARG, "pixel size must be positive");
  if ((int64_t)v->b * (int64_t)std::max<int64_t>(g->n, 1) >= (int64_t)1 << 31)
    return fail(ctx, CS_ERR_UNSUPPORTED, "B*N must be below 2^31");
  if (ctf) {
    FftPlan P;
    if (v->d % 2 != 0 || !fft_plan(v->d, P))
      return fail(ctx, CS_ERR_UNSUPPORTED, "CTF needs an even D with prime factors 2 and 3 (got %d)", v->d);
    if (!ctf->defocus_u || !ctf->defocus_v) return fail(ctx, CS_ERR_INVALID_ARG, "null defocus");
    if (!(ctf->voltage_kv > 0.0)) return fail(ctx, CS_ERR_INVALID_ARG, "voltage must be positive");
    if (!(ctf->amp_contrast >= 0.0 && ctf->amp_contrast < 1.0))
      return fail(ctx, CS_ERR_INVALID_ARG, "amplitude contrast must be in [0, 1)");
  }
  if (opt) {
    if (opt->tile != 0 && (opt->tile < 16 || opt->tile > 128))
      return fail(ctx, CS_ERR_INVALID_ARG, "tile must be 0 or in [16, 128]");
    const int T = opt->tile ? opt->tile : kDefaultTile;
    if (opt->halo < 0 || opt->halo > T) return fail(ctx, CS_ERR_INVALID_ARG, "halo must be in [0, tile]");
    if (opt->budget != 0 && opt->budget < 64) return fail(ctx, CS_ERR_INVALID_ARG, "budget must be 0 or >= 64");
    if (!std::isfinite(opt->q_cut)) return fail(ctx, CS_ERR_INVALID_ARG, "q_cut must be finite");
  }
  return CS_OK;
}

Geom make_geom(const cs_gaussians *g, const cs_views *v, const cs_options *opt) {
  Geom G;
  G.B = (int)v->b;
  G.N = (int)g->n;
  G.D = v->d;
  G.c0 = v->d / 2;
  G.pixel = v->pixel;
  const float qc = (opt && opt->q_cut > 0.f) ? opt->q_cut : kDefaultQCut;
  G.qk = qc * kHalfLog2e;
  G.T = (opt && opt->tile) ? opt->tile : kDefaultTile;
  G.halo = (opt && opt->halo) ? opt->halo : std::min(kDefaultHalo, G.T);
  G.C = G.T + 2 * G.halo;
  G.S = G.C + 4;  // padding columns: unrolled row walks stay inside a row
  G.ntx = (G.D + G.T - 1) / G.T;
  G.ntiles = G.ntx * G.ntx;
  G.K = G.ntiles + 1;
  G.budget = (opt && opt->budget) ? opt->budget : kDefaultBudget;
  G.scale_act = g->scale_act;
  G.amp_act = g->amp_act;
  return G;
}

unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

// k_build + binning (count, scan, scatter).
int launch_binning(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v, const Geom &G,
                   const Layout &L, char *ws, hipStream_t st) {
  float4 *gc = (float4 *)(ws + L.gc);
  int *count = (int *)(ws + L.count);
  const size_t BK = (size_t)G.B * G.K;
  const size_t nb = std::max<size_t>((size_t)G.N, BK);
  TLAUNCH(k_build, dim3(cdiv(nb, kBlock)), dim3(kBlock), 0, st, g->means, g->log_scales,
          g->quats, g->amps, G, gc, count, (int)BK);
  const dim3 bgrid(cdiv(G.N, kBlock), cdiv(G.B, kImgPerBinBlock));
  const size_t hist_bytes = (size_t)kImgPerBinBlock * G.K * 4;
  TLAUNCH(k_bin_count, bgrid, dim3(kBlock), hist_bytes, st, gc, v->rot, v->shift, G,
          (int *)(ws + L.key), (int *)(ws + L.blk), L.nbx);
  TLAUNCH(k_bin_blockscan, dim3((unsigned)BK), dim3(kBlock), 0, st, (int *)(ws + L.blk), L.nbx,
          count);
  TLAUNCH(k_scan, dim3(1), dim3(1024), 0, st, count, G, (int *)(ws + L.off),
          (int4 *)(ws + L.items), (int *)(ws + L.item_off), (int *)(ws + L.n_items),
          (int *)(ws + L.queues));
  TLAUNCH(k_bin_scatter, bgrid, dim3(kBlock), (size_t)(kBlock / 64) * G.K * 4, st, gc, v->rot,
          v->shift, G, (const int *)(ws + L.key), (const int *)(ws + L.off),
          (const int *)(ws + L.blk), L.nbx, (float4 *)(ws + L.list));
  return CS_OK;
}

int persistent_grid(cs_ctx *ctx, const void *kernel, size_t lds, int *grid) {
  int nb = 0;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, lds));
  if (nb < 1) nb = 1;
  *grid = nb * ctx->n_cu;
  return CS_OK;
}

// Splat forward into Q (ws or caller buffer).
int launch_forward(cs_ctx *ctx, const Geom &G, const Layout &L, char *ws, float *Q, hipStream_t st) {
  const size_t lds = (size_t)G.C * G.S * 4;
  int grid = 0;
  int rc = persistent_grid(ctx, (const void *)k_splat_fwd, lds, &grid);
  if (rc) return rc;
  TLAUNCH(k_splat_fwd, dim3(grid), dim3(kBlock), lds, st, (const float4 *)(ws + L.list),
                     (const int4 *)(ws + L.items), (const int *)(ws + L.n_items),
                     (int *)(ws + L.queues), G, (float *)(ws + L.partials));
  TLAUNCH(k_canvas_reduce, dim3(G.ntiles, G.B), dim3(kBlock), 0, st,
                     (const float *)(ws + L.partials), (const int *)(ws + L.item_off),
                     (const int4 *)(ws + L.items), G, Q);
  TLAUNCH(k_big_fwd, dim3(256), dim3(kBlock), 0, st, (const float4 *)(ws + L.list),
          (const int *)(ws + L.off), (const int *)(ws + L.count), (const int *)(ws + L.n_items) + 1,
          G, Q);
  return CS_OK;
}

int launch_backward(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v, const Geom &G,
                    const Layout &L, char *ws, const float *GQ, cs_grads *grads, hipStream_t st) {
  const size_t lds = (size_t)G.C * G.S * 4;
  int grid = 0;
  int rc = persistent_grid(ctx, (const void *)k_splat_bwd, lds, &grid);
  if (rc) return rc;
  float *mom = (float *)(ws + L.mom);
  TLAUNCH(k_splat_bwd, dim3(grid), dim3(kBlock), lds, st, (const float4 *)(ws + L.list),
                     (const int4 *)(ws + L.items), (const int *)(ws + L.n_items),
                     (int *)(ws + L.queues) + 1, G, GQ, mom);
  TLAUNCH(k_big_bwd, dim3(256), dim3(kBlock), 0, st, (const float4 *)(ws + L.list),
          (const int *)(ws + L.off), (const int *)(ws + L.count), (const int *)(ws + L.n_items) + 1,
          G, GQ, mom);
  TLAUNCH(k_chain, dim3(cdiv(G.N, kBlock)), dim3(kBlock), 0, st, (const float4 *)(ws + L.gc),
                     g->log_scales, g->quats, g->amps, v->rot, v->shift, G,
                     (const int *)(ws + L.key), mom, grads->means, grads->log_scales,
                     grads->quats, grads->amps);
  return CS_OK;
}

int zero_grads(cs_ctx *ctx, const cs_gaussians *g, cs_grads *grads, hipStream_t st) {
  const int64_t n = g->n;
  struct { float *p; int64_t k; } outs[4] = {
      {grads->means, 3 * n}, {grads->log_scales, 3 * n}, {grads->quats, 4 * n}, {grads->amps, n}};
  for (auto &o : outs) {
    if (!o.p || o.k == 0) continue;
    TLAUNCH(k_fill, dim3(cdiv(o.k, kBlock)), dim3(kBlock), 0, st, o.p, o.k, 0.f);
  }
  return CS_OK;
}

CtfDev make_ctf(const cs_ctf *ctf) {
  CtfDev c{};
  if (!ctf) return c;
  c.enabled = 1;
  c.defocus_u = ctf->defocus_u;
  c.defocus_v = ctf->defocus_v;
  c.astig = ctf->astig;
  c.phase = ctf->phase;
  c.lam = electron_wavelength_A(ctf->voltage_kv);
  c.cs = ctf->cs_mm * 1e7;
  c.w = ctf->amp_contrast;
  c.bfactor = ctf->bfactor;
  return c;
}

// Launch shapes of the FFT kernels for one image side.
struct FftLaunch {
  FftPlan P;
  const float2 *tw = nullptr;
  dim3 rgrid, cgrid;
  size_t rlds = 0, clds = 0;
  int cpw = 16;
};

int fft_setup(cs_ctx *ctx, const Geom &G, FftLaunch &F) {
  fft_plan(G.D, F.P);
  int rc = get_twiddles(ctx, G.D, &F.tw);
  if (rc) return rc;
  F.rgrid = dim3(cdiv(G.D / 2, 4), G.B);
  F.rlds = (size_t)(4 * 2 + 1) * G.D * 8;  // four row pairs (ping-pong) + twiddles
  F.cpw = G.D > 256 ? 8 : 16;
  F.cgrid = dim3(cdiv(G.D / 2 + 1, F.cpw), G.B);
  F.clds = (size_t)(F.cpw * 2 + 1) * G.D * 8;
  return CS_OK;
}

int launch_ctf_table(cs_ctx *ctx, const Geom &G, const cs_ctf *ctf, float *table, hipStream_t st) {
  const size_t n = (size_t)G.B * G.D * (G.D / 2 + 1);
  TLAUNCH(k_ctf_table, dim3(cdiv(n, 256)), dim3(256), 0, st, G.D, G.pixel, make_ctf(ctf), G.B, table);
  return CS_OK;
}

// src (real [B][D][D]) -> spec -> H^ -> dst (real), i.e. dst = F^-1(H^ F src).
int launch_ctf_roundtrip(cs_ctx *ctx, const Geom &G, const cs_ctf *ctf, const float *src,
                         float2 *spec, float *table, float *dst, hipStream_t st) {
  FftLaunch F;
  int rc = fft_setup(ctx, G, F);
  if (rc) return rc;
  rc = launch_ctf_table(ctx, G, ctf, table, st);
  if (rc) return rc;
  TLAUNCH(k_fft_rows_fwd, F.rgrid, dim3(256), F.rlds, st, src, F.P, F.tw, G.B, spec);
  TLAUNCH(k_fft_cols_ctf, F.cgrid, dim3(256), F.clds, st, spec, F.P, F.tw, G.B, F.cpw,
          (const float *)table);
  TLAUNCH(k_fft_rows_inv, F.rgrid, dim3(256), F.rlds, st, (const float2 *)spec, F.P, F.tw, G.B, dst);
  return CS_OK;
}

}  // namespace

// No-CTF residual: loss partials per row, optional X output, G_Q in place.
namespace cs {
__global__ void __launch_bounds__(256)
k_residual(float *Q, const float *obs, float *images_out, int B, int D, float grad_scale,
           float *loss_part) {
  const int row = blockIdx.x, b = blockIdx.y;
  const size_t o = ((size_t)b * D + row) * D;
  float acc = 0.f;
  for (int j = threadIdx.x; j < D; j += 256) {
    const float x = Q[o + j];
    if (images_out) images_out[o + j] = x;
    const float r = x - obs[o + j];
    acc += r * r;
    Q[o + j] = grad_scale * r;
  }
  __shared__ float red[4];
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) acc += __shfl_xor(acc, s, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) loss_part[(size_t)b * D + row] = red[0] + red[1] + red[2] + red[3];
}
}  // namespace cs

extern "C" {

int cs_create(int device, cs_ctx **out) {
  if (!out) return CS_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return CS_ERR_INVALID_ARG;
  }
  cs_ctx *c = new cs_ctx();
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) { delete c; return CS_ERR_HIP; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->n_cu = prop.multiProcessorCount;
  const char *cap = std::getenv("CS_WORKSPACE_MAX");
  if (cap) c->ws_max = (size_t)std::strtoull(cap, nullptr, 10);
  // allow canvases above 64 KiB of LDS
  (void)hipFuncSetAttribute((const void *)k_splat_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipFuncSetAttribute((const void *)k_splat_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipGetLastError();
  *out = c;
  return CS_OK;
}

void cs_destroy(cs_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->ws) (void)hipFree(ctx->ws);
  for (auto &kv : ctx->twiddles) (void)hipFree(kv.second);
  delete ctx;
}

const char *cs_last_error(const cs_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int cs_render(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v, const cs_ctf *ctf,
              const cs_options *opt, float *images, void *stream) {
  int rc = validate(ctx, g, v, ctf, opt);
  if (rc) return rc;
  if (!images) return fail(ctx, CS_ERR_INVALID_ARG, "null images");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const Geom G = make_geom(g, v, opt);
  const Layout L = make_layout(G, true, false, ctf != nullptr);
  rc = ensure_ws(ctx, L.total, st);
  if (rc) return rc;
  char *ws = (char *)ctx->ws;
  float *Q = ctf ? (float *)(ws + L.Q) : images;
  const size_t npx = (size_t)G.B * G.D * G.D;
  if (G.N == 0) {
    TLAUNCH(k_fill, dim3(cdiv(npx, kBlock)), dim3(kBlock), 0, st, images, (int64_t)npx, 0.f);
    return CS_OK;
  }
  rc = launch_binning(ctx, g, v, G, L, ws, st);
  if (rc) return rc;
  rc = launch_forward(ctx, G, L, ws, Q, st);
  if (rc) return rc;
  if (ctf)
    return launch_ctf_roundtrip(ctx, G, ctf, Q, (float2 *)(ws + L.spec), (float *)(ws + L.ctf),
                                images, st);
  return CS_OK;
}

int cs_render_backward(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v, const cs_ctf *ctf,
                       const cs_options *opt, const float *d_images, cs_grads *grads,
                       void *stream) {
  int rc = validate(ctx, g, v, ctf, opt);
  if (rc) return rc;
  if (!d_images || !grads) return fail(ctx, CS_ERR_INVALID_ARG, "null d_images or grads");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  if (g->n == 0) return CS_OK;
  const Geom G = make_geom(g, v, opt);
  const Layout L = make_layout(G, false, true, ctf != nullptr);
  rc = ensure_ws(ctx, L.total, st);
  if (rc) return rc;
  char *ws = (char *)ctx->ws;
  const float *GQ = d_images;
  if (ctf) {
    rc = launch_ctf_roundtrip(ctx, G, ctf, d_images, (float2 *)(ws + L.spec), (float *)(ws + L.ctf),
                              (float *)(ws + L.Q), st);
    if (rc) return rc;
    GQ = (const float *)(ws + L.Q);
  }
  rc = launch_binning(ctx, g, v, G, L, ws, st);
  if (rc) return rc;
  return launch_backward(ctx, g, v, G, L, ws, GQ, grads, st);
}

int cs_loss_and_grad(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v, const cs_ctf *ctf,
                     const cs_options *opt, const float *observed, int32_t reduction,
                     float *loss, cs_grads *grads, float *images_out, void *stream) {
  int rc = validate(ctx, g, v, ctf, opt);
  if (rc) return rc;
  if (!observed || !loss) return fail(ctx, CS_ERR_INVALID_ARG, "null observed or loss");
  if (reduction != CS_SUM && reduction != CS_MEAN) return fail(ctx, CS_ERR_INVALID_ARG, "bad reduction");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const Geom G = make_geom(g, v, opt);
  const bool want_grads = grads && G.N > 0;
  const Layout L = make_layout(G, true, want_grads, ctf != nullptr);
  rc = ensure_ws(ctx, L.total, st);
  if (rc) return rc;
  char *ws = (char *)ctx->ws;
  float *Q = (float *)(ws + L.Q);
  const size_t npx = (size_t)G.B * G.D * G.D;
  if (G.N == 0) {
    TLAUNCH(k_fill, dim3(cdiv(npx, kBlock)), dim3(kBlock), 0, st, Q, (int64_t)npx, 0.f);
  } else {
    rc = launch_binning(ctx, g, v, G, L, ws, st);
    if (rc) return rc;
    rc = launch_forward(ctx, G, L, ws, Q, st);
    if (rc) return rc;
  }
  const double scale = reduction == CS_MEAN ? 1.0 / ((double)G.B * G.D * G.D) : 1.0;
  const float gscale = (float)(2.0 * scale);
  float *loss_part = (float *)(ws + L.loss_part);
  int parts;
  if (ctf) {
    FftLaunch F;
    rc = fft_setup(ctx, G, F);
    if (rc) return rc;
    float2 *spec = (float2 *)(ws + L.spec);
    float *table = (float *)(ws + L.ctf);
    rc = launch_ctf_table(ctx, G, ctf, table, st);
    if (rc) return rc;
    TLAUNCH(k_fft_rows_fwd, F.rgrid, dim3(256), F.rlds, st, Q, F.P, F.tw, G.B, spec);
    TLAUNCH(k_fft_cols_ctf, F.cgrid, dim3(256), F.clds, st, spec, F.P, F.tw, G.B, F.cpw,
            (const float *)table);
    TLAUNCH(k_fft_rows_inv_loss, F.rgrid, dim3(256), F.rlds, st, spec, F.P, F.tw, G.B, observed,
            images_out, gscale, loss_part);
    parts = G.D / 2;
    if (want_grads) {
      TLAUNCH(k_fft_cols_ctf, F.cgrid, dim3(256), F.clds, st, spec, F.P, F.tw, G.B, F.cpw,
              (const float *)table);
      TLAUNCH(k_fft_rows_inv, F.rgrid, dim3(256), F.rlds, st, (const float2 *)spec, F.P, F.tw,
              G.B, Q);
    }
  } else {
    TLAUNCH(k_residual, dim3(G.D, G.B), dim3(256), 0, st, Q, observed, images_out, G.B,
                       G.D, gscale, loss_part);
    parts = G.D;
  }
  TLAUNCH(k_loss_reduce, dim3(G.B), dim3(256), 0, st, (const float *)loss_part, G.B, parts,
          (float)scale, loss);
  TLAUNCH(k_loss_total, dim3(1), dim3(256), 0, st, loss, G.B);
  if (!grads) return CS_OK;
  if (G.N == 0) return zero_grads(ctx, g, grads, st);
  return launch_backward(ctx, g, v, G, L, ws, Q, grads, st);
}

int cs_adam_step(cs_ctx *ctx, float *params, const float *grads, float *m, float *v, int64_t count,
                 int64_t step, float lr, float b1, float b2, float eps, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (count < 0 || step < 1) return fail(ctx, CS_ERR_INVALID_ARG, "count >= 0 and step >= 1 required");
  if (count == 0) return CS_OK;
  if (!params || !grads || !m || !v) return fail(ctx, CS_ERR_INVALID_ARG, "null Adam array");
  if (!(b1 >= 0.f && b1 < 1.f && b2 >= 0.f && b2 < 1.f))
    return fail(ctx, CS_ERR_INVALID_ARG, "betas must be in [0, 1)");
  HIPCHK(hipSetDevice(ctx->device));
  const float bc1 = (float)(1.0 - std::pow((double)b1, (double)step));
  const float bc2 = (float)(1.0 - std::pow((double)b2, (double)step));
  TLAUNCH(k_adam, dim3(cdiv(count, kBlock)), dim3(kBlock), 0, (hipStream_t)stream, params,
                     grads, m, v, count, lr, b1, b2, eps, bc1, bc2);
  return CS_OK;
}

int cs_pair_count(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v, const cs_options *opt,
                  int64_t *counts, void *stream) {
  int rc = validate(ctx, g, v, nullptr, opt);
  if (rc) return rc;
  if (!counts) return fail(ctx, CS_ERR_INVALID_ARG, "null counts");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const Geom G = make_geom(g, v, opt);
  TLAUNCH(k_fill, dim3(cdiv(2 * (size_t)G.B, kBlock)), dim3(kBlock), 0, st, (float *)counts,
                     (int64_t)(2 * G.B), 0.f);  // all-zero bits
  if (G.N == 0) return CS_OK;
  const Layout L = make_layout(G, false, false, false);
  rc = ensure_ws(ctx, L.total, st);
  if (rc) return rc;
  char *ws = (char *)ctx->ws;
  float4 *gc = (float4 *)(ws + L.gc);
  TLAUNCH(k_build, dim3(cdiv(G.N, kBlock)), dim3(kBlock), 0, st, g->means, g->log_scales,
          g->quats, g->amps, G, gc, (int *)nullptr, 0);
  TLAUNCH(k_pair_count, dim3(cdiv(G.N, kBlock), G.B), dim3(kBlock), 0, st, gc, v->rot,
                     v->shift, G, (unsigned long long *)counts);
  return CS_OK;
}

int cs_set_timing(cs_ctx *ctx, int enable) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  for (auto &p : ctx->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  ctx->pending.clear();
  ctx->stage_ms.clear();
  ctx->timing = enable != 0;
  return CS_OK;
}

int cs_stage_time(cs_ctx *ctx, const char *name, double *total_ms, int64_t *launches) {
  if (!ctx || !name || !total_ms || !launches) return CS_ERR_INVALID_ARG;
  for (auto &p : ctx->pending) {
    HIPCHK(hipEventSynchronize(p.b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
    auto &acc = ctx->stage_ms[p.name];
    acc.first += ms;
    acc.second += 1;
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  ctx->pending.clear();
  auto it = ctx->stage_ms.find(name);
  *total_ms = it == ctx->stage_ms.end() ? 0.0 : it->second.first;
  *launches = it == ctx->stage_ms.end() ? 0 : it->second.second;
  return CS_OK;
}

}  // extern "C"
