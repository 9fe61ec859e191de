// Host side of libcryosplat: argument validation, workspace, launch order,
// batching of several problems, HIP-graph capture and the autotuner.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/cryosplat.h"
#include "cs_host.hpp"
#include "cs_internal.hpp"

using namespace cs;

namespace {

constexpr float kDefaultQCut = 27.631021115928547f;  // 2 ln 1e6
constexpr int kDefaultTile = 64;
constexpr int kDefaultHalo = 16;
constexpr int kDefaultBudget = 2048;
constexpr int kMinAutoBudget = 256;

// Automatic work-item size: the default budget while N B Gaussian-image
// pairs fill about a thousand work items, smaller (down to 256) for calls
// with few images, which otherwise leave most of the chip idle (batch-1
// training puts a whole mixture into a few tiles of one image).
int auto_budget(int64_t N, int64_t B) {
  int b = kDefaultBudget;
  while (b > kMinAutoBudget && N * B < (int64_t)b * 1024) b >>= 1;
  return b;
}
constexpr int kMaxD = 512;
constexpr int kMaxImages = 65535;  // launches put the image index in grid y

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }
unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of cs_loss_and_grad_noalloc: device memory that exists for
// as long as the library is loaded, so that entry point needs no allocation.
// In host code `scratch` is only a stand-in for the symbol; the device
// address comes from hipGetSymbolAddress, once per device (every device
// holds its own copy of the array).
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = (size_t)CS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_rc[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// The device address of `scratch` on `device`, which must be current.
hipError_t scratch_address(int device, char **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) (void)hipGetLastError();
    g_scratch_rc[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? (char *)p : nullptr;
    g_scratch_done[device] = true;
  }
  *out = g_scratch_ptr[device];
  return g_scratch_rc[device];
}

}  // namespace

namespace cs {

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

}  // namespace cs

namespace {

}  // namespace

namespace cs {

double electron_wavelength_A(double kv) {
  const double h = 6.62607015e-34, m0 = 9.1093837015e-31, e = 1.602176634e-19, c = 299792458.0;
  const double eV = e * kv * 1e3;
  return h / std::sqrt(2.0 * m0 * eV * (1.0 + eV / (2.0 * m0 * c * c))) * 1e10;
}

}  // namespace cs

namespace {

// ---------------------------------------------------------------------------
// Per-problem plan
// ---------------------------------------------------------------------------
enum Mode { RENDER, BACKWARD, LOSS };

struct Layout {
  size_t gc = 0, key = 0, count = 0, off = 0, blk = 0, item_off = 0, n_items = 0, queues = 0,
         items = 0, list = 0, partials = 0, Q = 0, spec = 0, ctf = 0, mom = 0, loss_part = 0,
         pose_part = 0, wabs = 0, wscale = 0, wideq = 0;
  size_t total = 0;
  int max_items = 0;
  int nbx = 0;  // Gaussian blocks of the binning kernels
};

struct Plan {
  Mode mode = LOSS;
  cs_gaussians g{};
  cs_views v{};
  const cs_ctf *ctf = nullptr;
  Geom G{};
  Layout L;
  char *ws = nullptr;  // this problem's workspace region
  const float2 *tw = nullptr;  // FFT twiddles; null = the context's cached table
  bool fwd = false;    // runs the forward splat
  bool bwd = false;    // runs the adjoint
  // RENDER
  float *images = nullptr;
  // BACKWARD
  const float *d_images = nullptr;
  // LOSS
  const float *observed = nullptr;
  int reduction = CS_SUM;
  float *loss = nullptr;
  float *images_out = nullptr;
  cs_grads grads{};
  float *Q() const { return (float *)(ws + L.Q); }
  const float *GQ() const {
    if (mode == BACKWARD && !ctf) return d_images;
    return (const float *)(ws + L.Q);
  }
};

Layout make_layout(const Geom &G, bool need_partials, bool need_mom, bool need_fft) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align_up(bytes); return at; };
  const size_t BN = (size_t)G.B * G.N;
  const size_t BK = (size_t)G.B * G.K;
  L.max_items = (int)((size_t)G.B * G.ntiles + (BN + G.budget - 1) / G.budget);
  L.nbx = (int)((G.N + kBlock - 1) / kBlock);
  L.gc = take((size_t)G.N * 48 + 16);
  L.key = take(BN * 4 + 4);
  L.count = take(BK * 4);
  L.off = take(BK * 4);
  L.blk = take(BK * (size_t)std::max(L.nbx, 1) * 4);
  L.item_off = take((BK + 1) * 4);
  L.n_items = take(16);
  L.queues = take(16);
  L.items = take((size_t)L.max_items * 16 + 16);
  L.list = take(BN * 32 + 32);
  L.wabs = take(BN * 4 + 16);
  if (need_partials) {
    L.partials = take((size_t)L.max_items * G.C * G.C * 4);
    L.wscale = take((size_t)G.B * 8);
    L.wideq = take((size_t)G.B * G.D * G.D * 8);
  }
  L.Q = take((size_t)G.B * G.D * G.D * 4);
  if (need_fft) {
    L.spec = take((size_t)G.B * G.D * (G.D / 2 + 1) * 8);
    L.ctf = take((size_t)G.B * G.D * (G.D / 2 + 1) * 4);
  }
  if (need_mom) {
    L.mom = take(BN * 24 + 32);
    L.pose_part = take((size_t)G.B * std::max(L.nbx, 1) * 32);
  }
  L.loss_part = take((size_t)G.B * G.D * 4);
  L.total = o;
  return L;
}

int ensure_ws(cs_ctx *ctx, size_t need, hipStream_t stream) {
  if (need <= ctx->ws_bytes) return CS_OK;
  if (ctx->capturing) return fail(ctx, CS_ERR_HIP, "workspace growth during graph capture");
  if (ctx->ws_max && need > ctx->ws_max)
    return fail(ctx, CS_ERR_OOM, "workspace of %zu bytes exceeds CS_WORKSPACE_MAX=%zu", need,
                ctx->ws_max);
  if (ctx->ws) {
    HIPCHK(hipStreamSynchronize(stream));
    HIPCHK(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    // graphs captured against the old workspace are stale
    for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
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

}  // namespace

namespace cs {

int fft_cols_per_block(int D, int64_t B) {
  // four columns per block (18 KB of LDS at D = 256: eight blocks per CU
  // hide the latency of the strided column loads), two when a small batch
  // would leave the pass with fewer than a few hundred blocks; each column's
  // transform is the same whatever the blocking
  int c = 4;
  while (c > 2 && (int64_t)((D / 2 + c) / c) * B < 512) c >>= 1;
  return c;
}

int get_twiddles(cs_ctx *ctx, int L, const float2 **out) {
  auto it = ctx->twiddles.find(L);
  if (it != ctx->twiddles.end()) { *out = it->second; return CS_OK; }
  if (ctx->capturing) return fail(ctx, CS_ERR_HIP, "twiddle upload during graph capture");
  float2 *d = nullptr;
  HIPCHK(hipMalloc(&d, sizeof(float2) * L));
  // the same table kernel serves the static-scratch entry point, so both
  // paths transform with identical twiddles
  hipLaunchKernelGGL(k_twiddles, dim3(cdiv(L, 256)), dim3(256), 0, nullptr, L, d);
  LAUNCHCHK("k_twiddles");
  HIPCHK(hipStreamSynchronize(nullptr));
  ctx->twiddles[L] = d;
  *out = d;
  return CS_OK;
}

}  // namespace cs

namespace {

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
  if (v->b > kMaxImages)
    return fail(ctx, CS_ERR_UNSUPPORTED, "image count %lld > %d (one grid row per image)",
                (long long)v->b, kMaxImages);
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
    if (!(ctf->pixel_a >= 0.0f) || !std::isfinite(ctf->pixel_a))
      return fail(ctx, CS_ERR_INVALID_ARG, "CTF pixel size must be >= 0");
  }
  if (opt) {
    if (opt->tile != 0 && (opt->tile < 16 || opt->tile > 128))
      return fail(ctx, CS_ERR_INVALID_ARG, "tile must be 0 or in [16, 128]");
    const int T = opt->tile ? opt->tile : kDefaultTile;
    if (opt->halo < 0 || opt->halo > T) return fail(ctx, CS_ERR_INVALID_ARG, "halo must be in [0, tile]");
    if (opt->budget != 0 && opt->budget < 64) return fail(ctx, CS_ERR_INVALID_ARG, "budget must be 0 or >= 64");
    if (!std::isfinite(opt->q_cut)) return fail(ctx, CS_ERR_INVALID_ARG, "q_cut must be finite");
    if (opt->lane_order < 0 || opt->lane_order > 2)
      return fail(ctx, CS_ERR_INVALID_ARG, "lane_order must be 0, 1 or 2");
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
  G.S = G.C + 4;  // padding columns keep unrolled row walks inside a row
  G.ntx = (G.D + G.T - 1) / G.T;
  G.ntiles = G.ntx * G.ntx;
  G.K = G.ntiles + 1;
  G.budget = (opt && opt->budget) ? opt->budget : auto_budget(G.N, G.B);
  G.scale_act = g->scale_act;
  G.amp_act = g->amp_act;
  G.deal = opt ? opt->lane_order : 0;
  return G;
}

}  // namespace

namespace cs {

float ctf_pixel(const cs_ctf *ctf, float geometry_pixel) {
  return (ctf && ctf->pixel_a > 0.f) ? ctf->pixel_a : geometry_pixel;
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

}  // namespace cs

namespace {

bool has_grads(const cs_grads &g) {
  return g.means || g.log_scales || g.quats || g.amps || g.rot || g.shift;
}

// ---------------------------------------------------------------------------
// Enqueue helpers
// ---------------------------------------------------------------------------
int launch_binning(cs_ctx *ctx, const Plan &P, hipStream_t st) {
  const Geom &G = P.G;
  const Layout &L = P.L;
  char *ws = P.ws;
  float4 *gc = (float4 *)(ws + L.gc);
  int *count = (int *)(ws + L.count);
  const size_t BK = (size_t)G.B * G.K;
  const size_t nb = std::max<size_t>((size_t)G.N, BK);
  TLAUNCH(k_build, dim3(cdiv(nb, kBlock)), dim3(kBlock), 0, st, P.g.means, P.g.log_scales,
          P.g.quats, P.g.amps, G, gc, count, (int)BK);
  const dim3 bgrid(cdiv(G.N, kBlock), cdiv(G.B, kImgPerBinBlock));
  const size_t hist_bytes = (size_t)kImgPerBinBlock * G.K * 4;
  TLAUNCH(k_bin_count, bgrid, dim3(kBlock), hist_bytes, st, gc, P.v.rot, P.v.shift, G,
          (int *)(ws + L.key), (int *)(ws + L.blk), L.nbx);
  // small problems scan their per-block counts inside k_scan
  const bool fuse = BK <= 64;
  if (!fuse)
    TLAUNCH(k_bin_blockscan, dim3((unsigned)BK), dim3(kBlock), 0, st, (int *)(ws + L.blk), L.nbx,
            count);
  TLAUNCH(k_scan, dim3(1), dim3(1024), 0, st, count, G, (int *)(ws + L.off),
          (int4 *)(ws + L.items), (int *)(ws + L.item_off), (int *)(ws + L.n_items),
          (int *)(ws + L.queues), fuse ? (int *)(ws + L.blk) : (int *)nullptr, L.nbx);
  TLAUNCH(k_bin_scatter, bgrid, dim3(kBlock), (size_t)(kBlock / 64) * G.K * 8, st, gc, P.v.rot,
          P.v.shift, G, (const int *)(ws + L.key), (const int *)(ws + L.off),
          (const int *)(ws + L.blk), L.nbx, (float4 *)(ws + L.list), (float *)(ws + L.wabs));
  return CS_OK;
}

int persistent_grid(cs_ctx *ctx, const void *kernel, size_t lds, int *grid) {
  int nb = 0;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, lds));
  if (nb < 1) nb = 1;
  *grid = nb * ctx->n_cu;
  return CS_OK;
}

ProbDev prob_dev(const Plan &P) {
  ProbDev d;
  d.G = P.G;
  d.list = (const float4 *)(P.ws + P.L.list);
  d.items = (const int4 *)(P.ws + P.L.items);
  d.n_items = (const int *)(P.ws + P.L.n_items);
  d.wabs = (const float *)(P.ws + P.L.wabs);
  d.queue = (int *)(P.ws + P.L.queues);
  d.partials = (float *)(P.ws + P.L.partials);
  d.GQ = P.GQ();
  d.mom = (float *)(P.ws + P.L.mom);
  return d;
}

// Persistent launches of the forward or adjoint splat over the given
// problems: problems with the same canvas size share one launch (up to
// kMaxProblems each), so that no problem runs at the occupancy of a larger
// canvas; groups keep the problems' order.  Allocates nothing.
int launch_one_persistent(cs_ctx *ctx, bool forward, const MultiProb &MP, size_t lds,
                          hipStream_t st) {
  int grid = 0;
  int rc = persistent_grid(ctx, forward ? (const void *)k_splat_fwd : (const void *)k_splat_bwd,
                           lds, &grid);
  if (rc) return rc;
  if (forward) {
    TLAUNCH(k_splat_fwd, dim3(grid), dim3(kBlock), lds, st, MP);
  } else {
    TLAUNCH(k_splat_bwd, dim3(grid), dim3(kBlock), lds, st, MP);
  }
  return CS_OK;
}

int launch_persistent(cs_ctx *ctx, bool forward, const Plan *const *all, int n, hipStream_t st) {
  auto canvas = [&](int i) { return all[i]->G.C * all[i]->G.S; };
  for (int i = 0; i < n; ++i) {
    bool seen = false;  // canvas size already launched with an earlier group
    for (int j = 0; j < i && !seen; ++j) seen = canvas(j) == canvas(i);
    if (seen) continue;
    MultiProb MP{};
    size_t lds = 0;
    for (int k = i; k < n; ++k) {
      if (canvas(k) != canvas(i)) continue;
      MP.p[MP.count++] = prob_dev(*all[k]);
      lds = std::max(lds, (size_t)canvas(k) * 4);
      if (MP.count == kMaxProblems) {
        int rc = launch_one_persistent(ctx, forward, MP, lds, st);
        if (rc) return rc;
        MP = MultiProb{};
        lds = 0;
      }
    }
    if (MP.count) {
      int rc = launch_one_persistent(ctx, forward, MP, lds, st);
      if (rc) return rc;
    }
  }
  return CS_OK;
}

// After the forward splat: Q of one problem (reduce + wide Gaussians).
// Blocks per image of the wide-record kernels (grid rows are images): about
// 512 blocks in all, at least 4 per image.
int big_blocks(int B) { return std::max(4, (512 + B - 1) / B); }

int launch_forward_finish(cs_ctx *ctx, const Plan &P, float *Q, hipStream_t st) {
  const Geom &G = P.G;
  char *ws = P.ws;
  // split each tile's pixels over up to 4 blocks when there are few tiles
  // (one image): the per-pixel sums are unchanged
  const int per_tile = (G.T * G.T / 4 + kBlock - 1) / kBlock;
  const int zsplit = std::max(1, std::min(per_tile, (int)((512 + (int64_t)G.ntiles * G.B - 1) /
                                                          ((int64_t)G.ntiles * G.B))));
  TLAUNCH(k_canvas_reduce, dim3(G.ntiles, G.B, zsplit), dim3(kBlock), 0, st,
          (const float *)(ws + P.L.partials), (const int *)(ws + P.L.item_off),
          (const int4 *)(ws + P.L.items), G, Q);
  double *wscale = (double *)(ws + P.L.wscale);
  long long *wq = (long long *)(ws + P.L.wideq);
  TLAUNCH(k_big_prep, dim3(G.B), dim3(kBlock), 0, st, (const int *)(ws + P.L.off),
          (const int *)(ws + P.L.count), (const float *)(ws + P.L.wabs), G, wscale, wq);
  TLAUNCH(k_big_fwd, dim3(big_blocks(G.B), G.B), dim3(kBlock), 0, st, (const float4 *)(ws + P.L.list),
          (const int *)(ws + P.L.off), (const int *)(ws + P.L.count),
          (const int *)(ws + P.L.n_items) + 1, G, (const double *)wscale, wq);
  TLAUNCH(k_big_add, dim3(cdiv((size_t)G.D * G.D, 4 * kBlock), G.B), dim3(kBlock), 0, st,
          (const int *)(ws + P.L.count), G, (const double *)wscale, (const long long *)wq, Q);
  return CS_OK;
}

int launch_backward_finish(cs_ctx *ctx, const Plan &P, hipStream_t st) {
  const Geom &G = P.G;
  char *ws = P.ws;
  float *mom = (float *)(ws + P.L.mom);
  TLAUNCH(k_big_bwd, dim3(big_blocks(G.B), G.B), dim3(kBlock), 0, st, (const float4 *)(ws + P.L.list),
          (const int *)(ws + P.L.off), (const int *)(ws + P.L.count),
          (const int *)(ws + P.L.n_items) + 1, G, P.GQ(), mom);
  TLAUNCH(k_chain, dim3(cdiv(G.N, 64)), dim3(kBlock), 0, st, (const float4 *)(ws + P.L.gc),
          P.g.log_scales, P.g.quats, P.g.amps, P.v.rot, P.v.shift, G, (const int *)(ws + P.L.key),
          mom, P.grads.means, P.grads.log_scales, P.grads.quats, P.grads.amps);
  if (P.grads.rot || P.grads.shift) {
    const int nblk = cdiv(G.N, kBlock * kPoseGauss);
    float *part = (float *)(ws + P.L.pose_part);
    TLAUNCH(k_pose_grad_part, dim3(nblk, cdiv(G.B, kPoseImg)), dim3(kBlock), 0, st,
            (const float4 *)(ws + P.L.gc), P.v.rot, P.v.shift, G, (const int *)(ws + P.L.key), mom,
            part);
    TLAUNCH(k_pose_grad_sum, dim3(G.B), dim3(kBlock), 0, st, (const float *)part, G.B, nblk,
            P.grads.rot, P.grads.shift);
  }
  return CS_OK;
}

// Launch shapes of the FFT kernels for one image side.
struct FftLaunch {
  FftPlan P;
  const float2 *tw = nullptr;
  dim3 rgrid, cgrid, rblock;
  size_t rlds = 0, clds = 0;
  int cpw = 16;
};

int fft_setup(cs_ctx *ctx, const Geom &G, const float2 *tw, FftLaunch &F) {
  fft_plan(G.D, F.P);
  F.tw = tw;
  if (!F.tw) {
    int rc = get_twiddles(ctx, G.D, &F.tw);
    if (rc) return rc;
  }
  F.rgrid = dim3(cdiv(G.D / 2, 4), G.B);
  F.rlds = (size_t)(4 * 2 + 1) * G.D * 8;  // four row pairs (ping-pong) + twiddles
  F.rblock = dim3(256);
  if ((int64_t)F.rgrid.x * G.B < 512) {    // small batches: one row pair per block
    F.rgrid = dim3(G.D / 2, G.B);
    F.rlds = (size_t)(1 * 2 + 1) * G.D * 8;
    F.rblock = dim3(64);
  }
  F.cpw = fft_cols_per_block(G.D, G.B);
  F.cgrid = dim3(cdiv(G.D / 2 + 1, F.cpw), G.B);
  F.clds = (size_t)(F.cpw * 2 + 1) * G.D * 8;
  return CS_OK;
}

int launch_ctf_table(cs_ctx *ctx, const Plan &P, hipStream_t st) {
  const Geom &G = P.G;
  // one grid row per image; a few entries per thread where there are
  // enough images to fill the chip
  const size_t per = (size_t)G.D * (G.D / 2 + 1);
  const size_t ept = G.B >= 16 ? 8 : 1;
  TLAUNCH(k_ctf_table, dim3(cdiv(per, 256 * ept), G.B), dim3(256), 0, st, G.D, ctf_pixel(P.ctf, G.pixel),
          make_ctf(P.ctf), G.B,
          (float *)(P.ws + P.L.ctf));
  return CS_OK;
}

// dst = F^-1(H^ F src) for one problem (CTF table already built).
int launch_ctf_roundtrip(cs_ctx *ctx, const Plan &P, const float *src, float *dst, hipStream_t st) {
  const Geom &G = P.G;
  FftLaunch F;
  int rc = fft_setup(ctx, G, P.tw, F);
  if (rc) return rc;
  float2 *spec = (float2 *)(P.ws + P.L.spec);
  TLAUNCH(k_fft_rows_fwd, F.rgrid, F.rblock, F.rlds, st, src, F.P, F.tw, G.B, spec);
  TLAUNCH(k_fft_cols_ctf, F.cgrid, dim3(256), F.clds, st, spec, F.P, F.tw, G.B, F.cpw,
          (const float *)(P.ws + P.L.ctf));
  TLAUNCH(k_fft_rows_inv, F.rgrid, F.rblock, F.rlds, st, (const float2 *)spec, F.P, F.tw, G.B, dst);
  return CS_OK;
}

// Loss of one problem from Q; leaves G_Q in Q when the adjoint follows.
int launch_loss(cs_ctx *ctx, const Plan &P, hipStream_t st) {
  const Geom &G = P.G;
  float *Q = P.Q();
  float *loss_part = (float *)(P.ws + P.L.loss_part);
  const double scale = P.reduction == CS_MEAN ? 1.0 / ((double)G.B * G.D * G.D) : 1.0;
  const float gscale = (float)(2.0 * scale);
  int parts;
  if (P.ctf) {
    FftLaunch F;
    int rc = fft_setup(ctx, G, P.tw, F);
    if (rc) return rc;
    float2 *spec = (float2 *)(P.ws + P.L.spec);
    const float *table = (const float *)(P.ws + P.L.ctf);
    TLAUNCH(k_fft_rows_fwd, F.rgrid, F.rblock, F.rlds, st, Q, F.P, F.tw, G.B, spec);
    TLAUNCH(k_fft_cols_ctf, F.cgrid, dim3(256), F.clds, st, spec, F.P, F.tw, G.B, F.cpw, table);
    TLAUNCH(k_fft_rows_inv_loss, F.rgrid, F.rblock, F.rlds, st, spec, F.P, F.tw, G.B, P.observed,
            P.images_out, gscale, loss_part);
    parts = G.D / 2;
    if (P.bwd) {
      TLAUNCH(k_fft_cols_ctf, F.cgrid, dim3(256), F.clds, st, spec, F.P, F.tw, G.B, F.cpw, table);
      TLAUNCH(k_fft_rows_inv, F.rgrid, F.rblock, F.rlds, st, (const float2 *)spec, F.P, F.tw, G.B, Q);
    }
  } else {
    TLAUNCH(k_residual, dim3(G.D, G.B), dim3(256), 0, st, Q, P.observed, P.images_out, G.B, G.D,
            gscale, loss_part);
    parts = G.D;
  }
  TLAUNCH(k_loss_reduce, dim3(G.B), dim3(256), 0, st, (const float *)loss_part, G.B, parts,
          (float)scale, P.loss);
  if (G.B > 1) TLAUNCH(k_loss_total, dim3(1), dim3(256), 0, st, P.loss, G.B);
  return CS_OK;
}

int fill(cs_ctx *ctx, float *p, size_t n, hipStream_t st) {
  if (!p || n == 0) return CS_OK;
  TLAUNCH(k_fill, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, p, (int64_t)n, 0.f);
  return CS_OK;
}

// ---------------------------------------------------------------------------
// Debug checks (CS_ERR_NONFINITE): after a call's work, every input and
// output array is scanned for NaN / infinity; the call then synchronises its
// stream and reports the first class found (inputs before outputs).
// ---------------------------------------------------------------------------
struct CheckList {
  std::vector<std::pair<const float *, int64_t>> in, out;
  void input(const float *p, int64_t n) { if (p && n > 0) in.push_back({p, n}); }
  void output(const float *p, int64_t n) { if (p && n > 0) out.push_back({p, n}); }
  void gaussians(const cs_gaussians &g) {
    input(g.means, 3 * g.n); input(g.log_scales, 3 * g.n); input(g.quats, 4 * g.n); input(g.amps, g.n);
  }
  void views(const cs_views &v) { input(v.rot, 9 * v.b); input(v.shift, 2 * v.b); }
  void grads(const cs_grads &gr, int64_t n, int64_t b) {
    output(gr.means, 3 * n); output(gr.log_scales, 3 * n); output(gr.quats, 4 * n);
    output(gr.amps, n); output(gr.rot, 9 * b); output(gr.shift, 2 * b);
  }
};

int run_debug_checks(cs_ctx *ctx, const CheckList &L, hipStream_t st) {
  if (!ctx->debug_checks) return CS_OK;
  if (!ctx->check_flag) HIPCHK(hipMalloc((void **)&ctx->check_flag, 256));
  // 0.f has the bit pattern of integer 0: the fill kernel clears the flag
  TLAUNCH(k_fill, dim3(1), dim3(kBlock), 0, st, (float *)ctx->check_flag, (int64_t)1, 0.f);
  for (int cls = 0; cls < 2; ++cls)
    for (const auto &a : cls ? L.out : L.in)
      TLAUNCH(k_check_finite, dim3((unsigned)std::min<int64_t>(1024, cdiv(a.second, kBlock))),
              dim3(kBlock), 0, st, a.first, a.second, 1 << cls, ctx->check_flag);
  int h = 0;
  HIPCHK(hipMemcpyAsync(&h, ctx->check_flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (h & 1) return fail(ctx, CS_ERR_NONFINITE, "debug checks: NaN or infinity in an input array");
  if (h & 2) return fail(ctx, CS_ERR_NONFINITE, "debug checks: NaN or infinity in an output array");
  return CS_OK;
}

CheckList loss_checks(const cs_problem &p) {
  CheckList L;
  L.gaussians(p.g);
  L.views(p.v);
  L.input(p.observed, p.v.b * (int64_t)p.v.d * p.v.d);
  L.output(p.loss, p.v.b + 1);
  L.grads(p.grads, p.g.n, p.v.b);
  L.output(p.images_out, p.v.b * (int64_t)p.v.d * p.v.d);
  return L;
}

// The whole launch sequence of a set of plans, in stage order.  `sel`
// is caller storage for `count` plan pointers (the forward and adjoint
// subsets); nothing is allocated here.
int enqueue(cs_ctx *ctx, Plan *plans, int count, const Plan **sel, hipStream_t st) {
  int rc;
  for (int i = 0; i < count; ++i) {
    Plan &P = plans[i];
    if (P.ctf) {
      rc = launch_ctf_table(ctx, P, st);
      if (rc) return rc;
    }
    if (P.mode == BACKWARD && P.ctf) {
      rc = launch_ctf_roundtrip(ctx, P, P.d_images, P.Q(), st);
      if (rc) return rc;
    }
    if (P.fwd || P.bwd) {
      rc = launch_binning(ctx, P, st);
      if (rc) return rc;
    }
  }
  int nsel = 0;
  for (int i = 0; i < count; ++i)
    if (plans[i].fwd) sel[nsel++] = &plans[i];
  if (nsel) {
    rc = launch_persistent(ctx, true, sel, nsel, st);
    if (rc) return rc;
  }
  for (int i = 0; i < count; ++i) {
    Plan &P = plans[i];
    if (P.mode == BACKWARD) continue;
    // pre-CTF image: the caller's buffer for a CTF-free render, else workspace
    float *Q = (P.mode == RENDER && !P.ctf) ? P.images : P.Q();
    if (P.fwd) {
      rc = launch_forward_finish(ctx, P, Q, st);
    } else {
      rc = fill(ctx, Q, (size_t)P.G.B * P.G.D * P.G.D, st);
    }
    if (rc) return rc;
    if (P.mode == RENDER) {
      if (P.ctf) rc = launch_ctf_roundtrip(ctx, P, Q, P.images, st);
    } else {
      rc = launch_loss(ctx, P, st);
    }
    if (rc) return rc;
  }
  nsel = 0;
  for (int i = 0; i < count; ++i)
    if (plans[i].bwd) sel[nsel++] = &plans[i];
  if (nsel) {
    rc = launch_persistent(ctx, false, sel, nsel, st);
    if (rc) return rc;
    for (int i = 0; i < nsel; ++i) {
      rc = launch_backward_finish(ctx, *sel[i], st);
      if (rc) return rc;
    }
  }
  return CS_OK;
}

int enqueue(cs_ctx *ctx, std::vector<Plan> &plans, hipStream_t st) {
  std::vector<const Plan *> sel(plans.size());
  return enqueue(ctx, plans.data(), (int)plans.size(), sel.data(), st);
}

// Workspace for all plans; assigns every plan its region and creates the
// host-side resources the launches need (before any capture).
int place(cs_ctx *ctx, std::vector<Plan> &plans, hipStream_t st) {
  size_t total = 0;
  std::vector<size_t> offs;
  for (auto &P : plans) {
    offs.push_back(total);
    total += align_up(P.L.total);
  }
  int rc = ensure_ws(ctx, total, st);
  if (rc) return rc;
  for (size_t i = 0; i < plans.size(); ++i) plans[i].ws = (char *)ctx->ws + offs[i];
  for (auto &P : plans) {
    if (P.ctf) {
      const float2 *tw;
      rc = get_twiddles(ctx, P.G.D, &tw);
      if (rc) return rc;
    }
  }
  return CS_OK;
}

int make_loss_plan(cs_ctx *ctx, const cs_problem &pr, Plan &P) {
  int rc = validate(ctx, &pr.g, &pr.v, pr.ctf, &pr.opt);
  if (rc) return rc;
  if (!pr.observed || !pr.loss) return fail(ctx, CS_ERR_INVALID_ARG, "null observed or loss");
  if (pr.reduction != CS_SUM && pr.reduction != CS_MEAN) return fail(ctx, CS_ERR_INVALID_ARG, "bad reduction");
  P.mode = LOSS;
  P.g = pr.g;
  P.v = pr.v;
  P.ctf = pr.ctf;
  P.G = make_geom(&pr.g, &pr.v, &pr.opt);
  P.observed = pr.observed;
  P.reduction = pr.reduction;
  P.loss = pr.loss;
  P.images_out = pr.images_out;
  P.grads = pr.grads;
  P.fwd = P.G.N > 0;
  P.bwd = P.G.N > 0 && has_grads(pr.grads);
  P.L = make_layout(P.G, P.fwd, P.bwd, P.ctf != nullptr);
  return CS_OK;
}

// Signature of a batched call for the graph cache: every byte the captured
// launches depend on (shapes, pointers, scalars, options, workspace).
std::string signature(cs_ctx *ctx, const cs_problem *problems, int count) {
  std::string s;
  auto add = [&](const void *p, size_t n) { s.append((const char *)p, n); };
  add(&ctx->ws, sizeof(void *));
  add(&ctx->ws_bytes, sizeof(size_t));
  for (int i = 0; i < count; ++i) {
    const cs_problem &p = problems[i];
    add(&p.g, sizeof(p.g));
    add(&p.v, sizeof(p.v));
    const int has_ctf = p.ctf != nullptr;
    add(&has_ctf, sizeof(int));
    if (p.ctf) add(p.ctf, sizeof(cs_ctf));
    add(&p.opt, sizeof(p.opt));
    add(&p.observed, sizeof(void *));
    add(&p.reduction, sizeof(int32_t));
    add(&p.loss, sizeof(void *));
    add(&p.grads, sizeof(p.grads));
    add(&p.images_out, sizeof(void *));
  }
  return s;
}

int run_loss_problems(cs_ctx *ctx, const cs_problem *problems, int count, bool use_graph,
                      hipStream_t st) {
  std::vector<Plan> plans(count);
  for (int i = 0; i < count; ++i) {
    int rc = make_loss_plan(ctx, problems[i], plans[i]);
    if (rc) return rc;
  }
  int rc = place(ctx, plans, st);
  if (rc) return rc;
  if (!use_graph) {
    rc = enqueue(ctx, plans, st);
    for (int i = 0; i < count && rc == CS_OK; ++i) rc = run_debug_checks(ctx, loss_checks(problems[i]), st);
    return rc;
  }
  const std::string key = signature(ctx, problems, count);
  auto it = ctx->graphs.find(key);
  if (it == ctx->graphs.end()) {
    if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    ctx->capturing = true;
    rc = enqueue(ctx, plans, ctx->cap_stream);
    ctx->capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(ctx, CS_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(ctx, CS_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
    it = ctx->graphs.emplace(key, exec).first;
  }
  HIPCHK(hipGraphLaunch(it->second, st));
  for (int i = 0; i < count && rc == CS_OK; ++i) rc = run_debug_checks(ctx, loss_checks(problems[i]), st);
  return rc;
}

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------
std::string tune_key(const cs_problem &p) {
  char buf[256];
  const float qc = p.opt.q_cut > 0.f ? p.opt.q_cut : kDefaultQCut;
  snprintf(buf, sizeof(buf), "D%d_N%lld_B%lld_p%.4f_ctf%d_q%.4f_act%d%d", p.v.d, (long long)p.g.n,
           (long long)p.v.b, p.v.pixel, p.ctf ? 1 : 0, qc, p.g.scale_act, p.g.amp_act);
  return buf;
}

void load_tune_file(cs_ctx *ctx) {
  if (ctx->tune_file.empty()) return;
  std::ifstream f(ctx->tune_file);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string key;
    int t, h, b, d = 0;
    if (is >> key >> t >> h >> b && t >= 16 && t <= 128 && h >= 0 && h <= t && b >= 64) {
      if (!(is >> d) || d < 0 || d > 2) d = 0;  // lane order: optional fourth field
      ctx->tuned[key] = {t, h, b, d};
    }
  }
}

void save_tune_file(cs_ctx *ctx) {
  if (ctx->tune_file.empty()) return;
  std::ofstream f(ctx->tune_file, std::ios::trunc);
  for (auto &kv : ctx->tuned)
    f << kv.first << " " << kv.second[0] << " " << kv.second[1] << " " << kv.second[2] << " "
      << kv.second[3] << "\n";
}

int time_problem(cs_ctx *ctx, const cs_problem &pr, int reps, hipStream_t st, double *ms_out) {
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  std::vector<double> ts;
  int rc = run_loss_problems(ctx, &pr, 1, false, st);  // warm-up (also sizes the workspace)
  for (int r = 0; r < reps && rc == CS_OK; ++r) {
    (void)hipEventRecord(a, st);
    rc = run_loss_problems(ctx, &pr, 1, false, st);
    (void)hipEventRecord(b, st);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    ts.push_back(ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc) return rc;
  std::sort(ts.begin(), ts.end());
  *ms_out = ts.empty() ? 0.0 : ts[ts.size() / 2];
  return CS_OK;
}

}  // namespace

namespace cs {

int run_loss(cs_ctx *ctx, const cs_problem &pr, bool use_graph, hipStream_t st) {
  return run_loss_problems(ctx, &pr, 1, use_graph, st);
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
  const char *dc = std::getenv("CS_DEBUG_CHECKS");
  c->debug_checks = dc && std::strcmp(dc, "0") != 0 && dc[0] != 0;
  const char *tf = std::getenv("CS_AUTOTUNE_CACHE");
  if (tf) c->tune_file = tf;
  load_tune_file(c);
  // the static scratch's address on this device (cs_loss_and_grad_noalloc)
  const hipError_t se = scratch_address(device, &c->scratch);
  if (se != hipSuccess) c->scratch_err = hipGetErrorString(se);
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
  for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (auto &p : ctx->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->check_flag) (void)hipFree(ctx->check_flag);
  if (ctx->aux) (void)hipFree(ctx->aux);
  if (ctx->vol) (void)hipFree(ctx->vol);
  if (ctx->train) (void)hipFree(ctx->train);
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
  std::vector<Plan> plans(1);
  Plan &P = plans[0];
  P.mode = RENDER;
  P.g = *g;
  P.v = *v;
  P.ctf = ctf;
  P.G = make_geom(g, v, opt);
  P.images = images;
  P.fwd = P.G.N > 0;
  P.L = make_layout(P.G, P.fwd, false, ctf != nullptr);
  rc = place(ctx, plans, st);
  if (rc) return rc;
  rc = enqueue(ctx, plans, st);
  if (rc) return rc;
  CheckList L;
  L.gaussians(*g);
  L.views(*v);
  L.output(images, v->b * (int64_t)v->d * v->d);
  return run_debug_checks(ctx, L, st);
}

int cs_render_backward(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v, const cs_ctf *ctf,
                       const cs_options *opt, const float *d_images, cs_grads *grads,
                       void *stream) {
  int rc = validate(ctx, g, v, ctf, opt);
  if (rc) return rc;
  if (!d_images || !grads) return fail(ctx, CS_ERR_INVALID_ARG, "null d_images or grads");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  if (g->n == 0 || !has_grads(*grads)) return CS_OK;
  std::vector<Plan> plans(1);
  Plan &P = plans[0];
  P.mode = BACKWARD;
  P.g = *g;
  P.v = *v;
  P.ctf = ctf;
  P.G = make_geom(g, v, opt);
  P.d_images = d_images;
  P.grads = *grads;
  P.bwd = true;
  P.L = make_layout(P.G, false, true, ctf != nullptr);
  rc = place(ctx, plans, st);
  if (rc) return rc;
  rc = enqueue(ctx, plans, st);
  if (rc) return rc;
  CheckList L;
  L.gaussians(*g);
  L.views(*v);
  L.input(d_images, v->b * (int64_t)v->d * v->d);
  L.grads(*grads, g->n, v->b);
  return run_debug_checks(ctx, L, st);
}

int cs_loss_and_grad(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v, const cs_ctf *ctf,
                     const cs_options *opt, const float *observed, int32_t reduction,
                     float *loss, cs_grads *grads, float *images_out, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!g || !v) return fail(ctx, CS_ERR_INVALID_ARG, "null gaussians or views");
  HIPCHK(hipSetDevice(ctx->device));
  cs_problem pr{};
  pr.g = *g;
  pr.v = *v;
  pr.ctf = ctf;
  if (opt) pr.opt = *opt;
  pr.observed = observed;
  pr.reduction = reduction;
  pr.loss = loss;
  if (grads) pr.grads = *grads;
  pr.images_out = images_out;
  return run_loss_problems(ctx, &pr, 1, opt && opt->graph, (hipStream_t)stream);
}

int cs_loss_and_grad_noalloc(cs_ctx *ctx, const cs_gaussians *g, const cs_views *v,
                             const cs_ctf *ctf, const cs_options *opt, const float *observed,
                             int32_t reduction, float *loss, cs_grads *grads, float *images_out,
                             void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!g || !v) return fail(ctx, CS_ERR_INVALID_ARG, "null gaussians or views");
  cs_problem pr{};
  pr.g = *g;
  pr.v = *v;
  pr.ctf = ctf;
  if (opt) pr.opt = *opt;
  pr.opt.graph = 0;
  pr.observed = observed;
  pr.reduction = reduction;
  pr.loss = loss;
  if (grads) pr.grads = *grads;
  pr.images_out = images_out;
  Plan P;
  int rc = make_loss_plan(ctx, pr, P);
  if (rc) return rc;
  // scratch layout: [twiddle table][this call's workspace]
  const size_t tw_bytes = ctf ? align_up(sizeof(float2) * (size_t)P.G.D) : 0;
  const size_t need = tw_bytes + align_up(P.L.total);
  if (need > kScratchBytes)
    return fail(ctx, CS_ERR_OOM,
                "cs_loss_and_grad_noalloc: this call needs %zu bytes of scratch; the static "
                "scratch holds %zu (use cs_loss_and_grad)", need, kScratchBytes);
  HIPCHK(hipSetDevice(ctx->device));
  if (!ctx->scratch)
    return fail(ctx, CS_ERR_HIP, "static scratch unavailable on device %d: %s", ctx->device,
                ctx->scratch_err.c_str());
  hipStream_t st = (hipStream_t)stream;
  P.ws = ctx->scratch + tw_bytes;
  if (ctf) {
    float2 *tw = (float2 *)ctx->scratch;
    hipLaunchKernelGGL(k_twiddles, dim3(cdiv(P.G.D, 256)), dim3(256), 0, st, P.G.D, tw);
    LAUNCHCHK("k_twiddles");
    P.tw = tw;
  }
  // no stage timing here: its events would be allocations
  const bool timing = ctx->timing;
  ctx->timing = false;
  const Plan *sel[1];
  rc = enqueue(ctx, &P, 1, sel, st);
  ctx->timing = timing;
  return rc;
}

int cs_loss_and_grad_multi(cs_ctx *ctx, const cs_problem *problems, int32_t count,
                           int32_t use_graph, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!problems || count < 1) return fail(ctx, CS_ERR_INVALID_ARG, "need at least one problem");
  HIPCHK(hipSetDevice(ctx->device));
  return run_loss_problems(ctx, problems, count, use_graph != 0, (hipStream_t)stream);
}

int cs_autotune(cs_ctx *ctx, cs_problem *problems, int32_t count, int32_t reps, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!problems || count < 1 || reps < 1) return fail(ctx, CS_ERR_INVALID_ARG, "bad autotune arguments");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const bool was_timing = ctx->timing;
  ctx->timing = false;
  int rc = CS_OK;
  for (int i = 0; i < count && rc == CS_OK; ++i) {
    cs_problem pr = problems[i];
    pr.opt.graph = 0;
    const std::string key = tune_key(pr);
    auto hit = ctx->tuned.find(key);
    if (hit == ctx->tuned.end()) {
      // stage 1: tile x halo at the default budget in list order.  Timings
      // within kTuneSlack of the fastest count as ties, resolved by the fixed
      // candidate order (the smaller canvas first, then the default budget),
      // so that near-equal candidates do not flip between runs.
      constexpr double kTuneSlack = 1.02;
      std::vector<int> best = {kDefaultTile, kDefaultHalo, kDefaultBudget, 0};
      const int tiles[] = {32, 40, 48, 56, 64, 96, 128};
      const int halos[] = {8, 10, 12, 14, 16, 24};
      std::vector<std::pair<double, std::vector<int>>> cand;
      for (int T : tiles) {
        if (T > std::max(32, pr.v.d)) continue;
        for (int h : halos) {
          if (h > T) continue;
          pr.opt.tile = T;
          pr.opt.halo = h;
          pr.opt.budget = kDefaultBudget;
          pr.opt.lane_order = 0;
          double ms = 0;
          rc = time_problem(ctx, pr, reps, st, &ms);
          if (rc) break;
          cand.push_back({ms, {T, h, kDefaultBudget, 0}});
        }
        if (rc) break;
      }
      if (rc) break;
      // stage 2: the dealt and the size-sorted lane orders for the four
      // fastest tile x halo candidates (they shift the balance towards
      // larger canvases)
      {
        std::vector<std::pair<double, std::vector<int>>> fast = cand;
        std::stable_sort(fast.begin(), fast.end(),
                         [](const auto &a, const auto &b) { return a.first < b.first; });
        for (size_t k = 0; k < fast.size() && k < 4 && rc == CS_OK; ++k) {
          for (int lo = 1; lo <= 2 && rc == CS_OK; ++lo) {
            pr.opt.tile = fast[k].second[0];
            pr.opt.halo = fast[k].second[1];
            pr.opt.budget = kDefaultBudget;
            pr.opt.lane_order = lo;
            double ms = 0;
            rc = time_problem(ctx, pr, reps, st, &ms);
            cand.push_back({ms, {pr.opt.tile, pr.opt.halo, kDefaultBudget, lo}});
          }
        }
      }
      if (rc) break;
      // ties: smaller canvas (T + 2h) first, then the smaller tile, list order first
      std::stable_sort(cand.begin(), cand.end(), [](const auto &a, const auto &b) {
        const int ca = a.second[0] + 2 * a.second[1], cb = b.second[0] + 2 * b.second[1];
        if (ca != cb) return ca < cb;
        if (a.second[0] != b.second[0]) return a.second[0] < b.second[0];
        return a.second[3] < b.second[3];
      });
      double best_ms = 1e30;
      for (const auto &c : cand) best_ms = std::min(best_ms, c.first);
      for (const auto &c : cand)
        if (c.first <= kTuneSlack * best_ms) { best = c.second; best_ms = c.first; break; }
      // stage 3: budget for the chosen tile, halo and lane order
      const int budgets[] = {256, 512, 1024, 4096, 8192};
      double bud_ms = best_ms;
      for (int bgt : budgets) {
        if (rc) break;
        pr.opt.tile = best[0];
        pr.opt.halo = best[1];
        pr.opt.budget = bgt;
        pr.opt.lane_order = best[3];
        double ms = 0;
        rc = time_problem(ctx, pr, reps, st, &ms);
        if (rc) break;
        if (ms * kTuneSlack < bud_ms) { bud_ms = ms; best[2] = bgt; }
      }
      if (rc) break;
      hit = ctx->tuned.emplace(key, best).first;
      save_tune_file(ctx);
    }
    problems[i].opt.tile = hit->second[0];
    problems[i].opt.halo = hit->second[1];
    problems[i].opt.budget = hit->second[2];
    problems[i].opt.lane_order = hit->second.size() > 3 ? hit->second[3] : 0;
  }
  ctx->timing = was_timing;
  if (rc == CS_OK) HIPCHK(hipStreamSynchronize(st));
  return rc;
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
  hipStream_t st = (hipStream_t)stream;
  TLAUNCH(k_adam, dim3(cdiv(count, kBlock)), dim3(kBlock), 0, st, params, grads, m, v, count, lr,
          b1, b2, eps, bc1, bc2);
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
  rc = fill(ctx, (float *)counts, 2 * (size_t)G.B, st);  // all-zero bits
  if (rc) return rc;
  if (G.N == 0) return CS_OK;
  const Layout L = make_layout(G, false, false, false);
  rc = ensure_ws(ctx, L.total, st);
  if (rc) return rc;
  char *ws = (char *)ctx->ws;
  float4 *gc = (float4 *)(ws + L.gc);
  TLAUNCH(k_build, dim3(cdiv(G.N, kBlock)), dim3(kBlock), 0, st, g->means, g->log_scales,
          g->quats, g->amps, G, gc, (int *)nullptr, 0);
  TLAUNCH(k_pair_count, dim3(cdiv(G.N, kBlock), G.B), dim3(kBlock), 0, st, gc, v->rot, v->shift,
          G, (unsigned long long *)counts);
  return CS_OK;
}

int cs_set_debug_checks(cs_ctx *ctx, int enable) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  ctx->debug_checks = enable != 0;
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
