// Host side of the training-loop entry points: cs_fourier_shift,
// cs_init_attributes, cs_train_sequential (Alg. 1; Sec. 4.1).
#include <algorithm>
#include <cmath>

#include "../../include/cryosplat.h"
#include "cs_host.hpp"
#include "cs_internal.hpp"
#include "cs_train.hpp"

using namespace cs;

namespace {

constexpr int kRowTeamsShift = 4;                     // row pairs per block of the row passes
constexpr size_t kShiftChunkBytes = (size_t)256 << 20;  // spectrum staged per chunk of images

size_t al256t(size_t x) { return (x + 255) & ~size_t(255); }
unsigned cdivt(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

extern "C" {

int cs_fourier_shift(cs_ctx *ctx, const float *images, const float *shift, int64_t B, int32_t D,
                     float pixel, float direction, float *out, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!images || !shift || !out) return fail(ctx, CS_ERR_INVALID_ARG, "null images, shifts or output");
  if (B < 1) return fail(ctx, CS_ERR_INVALID_ARG, "B must be >= 1");
  if (!(pixel > 0.f) || !std::isfinite(pixel)) return fail(ctx, CS_ERR_INVALID_ARG, "pixel size must be positive");
  if (direction != 1.f && direction != -1.f) return fail(ctx, CS_ERR_INVALID_ARG, "direction must be +1 or -1");
  FftPlan P;
  if (D < 2 || D % 2 != 0 || D > 512 || !fft_plan(D, P))
    return fail(ctx, CS_ERR_UNSUPPORTED, "D must be even with prime factors 2 and 3 (<= 512)");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const float2 *tw = nullptr;
  int rc = get_twiddles(ctx, D, &tw);
  if (rc) return rc;
  const int Dh = D / 2 + 1;
  const size_t per = (size_t)D * Dh * 8;
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>({B, 65535, (int64_t)(kShiftChunkBytes / per)}));
  rc = grow(ctx, &ctx->aux, &ctx->aux_bytes, al256t((size_t)chunk * per));
  if (rc) return rc;
  float2 *spec = (float2 *)ctx->aux;
  const size_t rlds = (size_t)(kRowTeamsShift * 2 + 1) * D * 8;
  const size_t npix = (size_t)D * D;
  for (int64_t b0 = 0; b0 < B; b0 += chunk) {
    const int nb = (int)std::min<int64_t>(chunk, B - b0);
    const int cpw = fft_cols_per_block(D, nb);
    const size_t clds = (size_t)(cpw * 2 + 1) * D * 8;
    const dim3 rgrid(cdivt(D / 2, kRowTeamsShift), nb);
    TLAUNCH(k_fft_rows_fwd, rgrid, dim3(256), rlds, st, images + b0 * npix, P, tw, nb, spec);
    TLAUNCH(k_fft_cols_shift, dim3(cdivt(Dh, cpw), nb), dim3(256), clds, st, spec, P, tw, cpw,
            shift + 2 * b0, 1.f / pixel, direction);
    TLAUNCH(k_fft_rows_inv, rgrid, dim3(256), rlds, st, (const float2 *)spec, P, tw, nb,
            out + b0 * npix);
  }
  return CS_OK;
}

int cs_init_attributes(cs_ctx *ctx, const float *z, int64_t n, float *params, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!z || !params) return fail(ctx, CS_ERR_INVALID_ARG, "null draws or parameters");
  if (n < 1) return fail(ctx, CS_ERR_INVALID_ARG, "N must be >= 1");
  HIPCHK(hipSetDevice(ctx->device));
  // softplus^-1(y) = log(expm1(y))
  const float scale_pre = (float)std::log(std::expm1(0.0075));
  const float amp_pre = (float)std::log(std::expm1(1.0 / (2.0 * (double)n)));
  hipStream_t st = (hipStream_t)stream;
  TLAUNCH(k_init_attributes, dim3(cdivt(n, 256)), dim3(256), 0, st, z, n, scale_pre, amp_pre, params);
  return CS_OK;
}

int cs_train_sequential(cs_ctx *ctx, float *params, float *adam_m, float *adam_v, int64_t n,
                        int32_t scale_act, int32_t amp_act, const cs_dataset *data,
                        const cs_ctf *ctf, const cs_options *opt, int32_t reduction,
                        const int64_t *order, int64_t count, int64_t step0, float lr, float b1,
                        float b2, float eps, float *loss, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!params || !adam_m || !adam_v) return fail(ctx, CS_ERR_INVALID_ARG, "null parameters or moments");
  if (n < 1) return fail(ctx, CS_ERR_INVALID_ARG, "N must be >= 1");
  if (!data || !data->images || !data->rot) return fail(ctx, CS_ERR_INVALID_ARG, "null data set");
  if (data->m < 1) return fail(ctx, CS_ERR_INVALID_ARG, "empty data set");
  if (data->d < 1 || data->d > 512) return fail(ctx, CS_ERR_INVALID_ARG, "bad image side");
  if (count < 0 || (count > 0 && !order)) return fail(ctx, CS_ERR_INVALID_ARG, "bad order");
  if (step0 < 0) return fail(ctx, CS_ERR_INVALID_ARG, "step0 must be >= 0");
  if (!(b1 >= 0.f && b1 < 1.f && b2 >= 0.f && b2 < 1.f))
    return fail(ctx, CS_ERR_INVALID_ARG, "betas must be in [0, 1)");
  if (ctf && (!ctf->defocus_u || !ctf->defocus_v)) return fail(ctx, CS_ERR_INVALID_ARG, "null defocus");
  for (int64_t k = 0; k < count; ++k)
    if (order[k] < 0 || order[k] >= data->m)
      return fail(ctx, CS_ERR_INVALID_ARG, "order[%lld] = %lld outside [0, %lld)", (long long)k,
                  (long long)order[k], (long long)data->m);
  if (count == 0) return CS_OK;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int D = data->d;
  const size_t npix = (size_t)D * D, np = (size_t)11 * n;
  // scratch: gradients [11 N] | image [D][D] | rotation [9] | CTF [4] | loss [2]
  const size_t o_g = 0, o_img = al256t(np * 4), o_rot = o_img + al256t(npix * 4);
  const size_t o_ctf = o_rot + 256, o_loss = o_ctf + 256;
  int rc = grow(ctx, &ctx->train, &ctx->train_bytes, o_loss + 256);
  if (rc) return rc;
  char *w = (char *)ctx->train;
  float *g = (float *)(w + o_g), *lossbuf = (float *)(w + o_loss);
  TrainStage stage{(float *)(w + o_img), (float *)(w + o_rot), (float *)(w + o_ctf)};
  TrainCtfSrc src{nullptr, nullptr, nullptr, nullptr};
  cs_ctf sctf{};
  if (ctf) {
    src = TrainCtfSrc{ctf->defocus_u, ctf->defocus_v, ctf->astig, ctf->phase};
    sctf = *ctf;
    sctf.defocus_u = stage.ctf;
    sctf.defocus_v = stage.ctf + 1;
    sctf.astig = stage.ctf + 2;
    sctf.phase = stage.ctf + 3;
  }
  cs_problem pr{};
  pr.g = cs_gaussians{params, params + 3 * n, params + 6 * n, params + 10 * n, n, scale_act, amp_act};
  pr.v = cs_views{stage.rot, nullptr, 1, D, data->pixel};
  pr.ctf = ctf ? &sctf : nullptr;
  if (opt) pr.opt = *opt;
  const bool graph = opt && opt->graph;
  pr.opt.graph = 0;
  pr.observed = stage.image;
  pr.reduction = reduction;
  pr.loss = lossbuf;
  pr.grads = cs_grads{g, g + 3 * n, g + 6 * n, g + 10 * n, nullptr, nullptr};
  pr.images_out = nullptr;
  const unsigned gblocks = std::min<unsigned>(cdivt((int64_t)npix, 256), 256);
  for (int64_t k = 0; k < count; ++k) {
    const int64_t i = order[k];
    if (graph) {
      // fixed pointers for the replayed graph: stage image i, record the
      // previous step's loss
      float *rec = (loss && k > 0) ? loss + (k - 1) : nullptr;
      TLAUNCH(k_train_gather, dim3(gblocks), dim3(256), 0, st, data->images, data->rot, src, i,
              (int)npix, stage, (const float *)lossbuf, rec);
    } else {
      // eager: read image i in place; the loss pair [image, total] goes to
      // loss + k (the next step overwrites the total), the last step's to the
      // scratch pair
      pr.v.rot = data->rot + 9 * i;
      pr.observed = data->images + i * (int64_t)npix;
      if (ctf) {
        sctf.defocus_u = ctf->defocus_u + i;
        sctf.defocus_v = ctf->defocus_v + i;
        sctf.astig = ctf->astig ? ctf->astig + i : nullptr;
        sctf.phase = ctf->phase ? ctf->phase + i : nullptr;
      }
      pr.loss = (loss && k + 1 < count) ? loss + k : lossbuf;
    }
    rc = run_loss(ctx, pr, graph, st);
    if (rc) return rc;
    const int64_t step = step0 + k + 1;
    const float bc1 = (float)(1.0 - std::pow((double)b1, (double)step));
    const float bc2 = (float)(1.0 - std::pow((double)b2, (double)step));
    TLAUNCH(k_adam, dim3(cdivt((int64_t)np, kBlock)), dim3(kBlock), 0, st, params, (const float *)g,
            adam_m, adam_v, (int64_t)np, lr, b1, b2, eps, bc1, bc2);
  }
  if (loss) TLAUNCH(k_train_record, dim3(1), dim3(64), 0, st, (const float *)lossbuf, loss + count - 1);
  return CS_OK;
}

int cs_split_gaussians(cs_ctx *ctx, const float *params, const float *adam_m, const float *adam_v,
                       int64_t n, int32_t scale_act, int32_t amp_act, float *out_params,
                       float *out_m, float *out_v, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!params || !out_params) return fail(ctx, CS_ERR_INVALID_ARG, "null parameters");
  if (n < 1) return fail(ctx, CS_ERR_INVALID_ARG, "N must be >= 1");
  if (n > ((int64_t)1 << 40)) return fail(ctx, CS_ERR_UNSUPPORTED, "N too large");
  const bool mom = adam_m || adam_v || out_m || out_v;
  if (mom && !(adam_m && adam_v && out_m && out_v))
    return fail(ctx, CS_ERR_INVALID_ARG, "Adam moments: give all four arrays or none");
  if (scale_act != 0 && scale_act != 1) return fail(ctx, CS_ERR_INVALID_ARG, "bad scale_act");
  if (amp_act != 0 && amp_act != 1) return fail(ctx, CS_ERR_INVALID_ARG, "bad amp_act");
  const size_t in_b = (size_t)11 * n * 4, out_b = 2 * in_b;
  auto overlap = [](const void *a, size_t na, const void *b, size_t nb) {
    const char *x = (const char *)a, *y = (const char *)b;
    return a && b && x < y + nb && y < x + na;
  };
  // no output may overlap an input or another output (the kernel reads its
  // inputs through restrict pointers)
  const void *ins[3] = {params, adam_m, adam_v};
  const void *outs[3] = {out_params, out_m, out_v};
  bool bad = false;
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b) bad = bad || overlap(ins[a], in_b, outs[b], out_b);
    for (int b = a + 1; b < 3; ++b) bad = bad || overlap(outs[a], out_b, outs[b], out_b);
  }
  if (bad) return fail(ctx, CS_ERR_INVALID_ARG, "outputs must not overlap the inputs or each other");
  HIPCHK(hipSetDevice(ctx->device));
  TLAUNCH(k_split_gaussians, dim3(cdivt(n, 256)), dim3(256), 0, (hipStream_t)stream, params,
          adam_m, adam_v, n, scale_act, amp_act, out_params, mom ? out_m : nullptr,
          mom ? out_v : nullptr);
  return CS_OK;
}

}  // extern "C"
