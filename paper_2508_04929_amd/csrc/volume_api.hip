// Host side of the voxelisation and FSC entry points (cs_voxelize, cs_fsc).
#include <algorithm>

#include "../../include/cryosplat.h"
#include "cs_host.hpp"
#include "cs_volume.hpp"

using namespace cs;

namespace {

constexpr float kDefaultQCutVol = 27.631021115928547f;  // 2 ln 1e6, as the renderer
constexpr int kRowTeamsVol = 4;                          // row pairs per block of k_fft_rows_fwd

size_t al256v(size_t x) { return (x + 255) & ~size_t(255); }
unsigned cdivv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

extern "C" {

int cs_voxelize(cs_ctx *ctx, const cs_gaussians *g, int32_t D, float pixel, float q_cut,
                float *vol, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!g || !vol) return fail(ctx, CS_ERR_INVALID_ARG, "null gaussians or volume");
  if (g->n < 0) return fail(ctx, CS_ERR_INVALID_ARG, "negative Gaussian count");
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->amps))
    return fail(ctx, CS_ERR_INVALID_ARG, "null Gaussian parameter array");
  if (g->scale_act != 0 && g->scale_act != 1) return fail(ctx, CS_ERR_INVALID_ARG, "bad scale_act");
  if (g->amp_act != 0 && g->amp_act != 1) return fail(ctx, CS_ERR_INVALID_ARG, "bad amp_act");
  if (D < 8 || D % 8 != 0 || D > 512) return fail(ctx, CS_ERR_UNSUPPORTED, "D must be a multiple of 8 in [8, 512]");
  if (!(pixel > 0.f)) return fail(ctx, CS_ERR_INVALID_ARG, "voxel size must be positive");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int N = (int)g->n, nb = D / 8, nbr = nb * nb * nb;
  VoxGeom V{N, D, D / 2, nb, pixel, q_cut > 0.f ? q_cut : kDefaultQCutVol};
  const size_t o_gc = 0, o_rec = o_gc + al256v((size_t)N * 48 + 16);
  const size_t o_box = o_rec + al256v((size_t)N * 48 + 16);
  const size_t o_cnt = o_box + al256v((size_t)N * 16 + 16);
  const size_t o_off = o_cnt + al256v((size_t)nbr * 4);
  const size_t o_cur = o_off + al256v((size_t)(nbr + 1) * 4);
  const size_t o_scale = o_cur + al256v((size_t)nbr * 4);
  const int nwp = (int)cdivv(N, 256);  // blocks of k_vox_prep: partial sums of |w|
  const size_t o_wp = o_scale + 256;
  const size_t o_list = o_wp + al256v((size_t)nwp * 8 + 8);
  int rc = grow(ctx, &ctx->vol, &ctx->vol_bytes, o_list + 256);
  if (rc) return rc;
  // per-Gaussian records, brick counts and offsets, fixed-point scale
  auto prepare = [&]() -> int {
    char *w = (char *)ctx->vol;
    float4 *gc = (float4 *)(w + o_gc), *rec = (float4 *)(w + o_rec);
    int *cnt = (int *)(w + o_cnt), *cur = (int *)(w + o_cur);
    TLAUNCH(k_fill_i32z, dim3(cdivv(nbr, 256)), dim3(256), 0, st, cnt, nbr);
    TLAUNCH(k_fill_i32z, dim3(cdivv(nbr, 256)), dim3(256), 0, st, cur, nbr);
    if (N > 0) {
      Geom G{};
      G.N = N;
      G.scale_act = g->scale_act;
      G.amp_act = g->amp_act;
      TLAUNCH(k_build, dim3(cdivv(N, kBlock)), dim3(kBlock), 0, st, g->means, g->log_scales,
              g->quats, g->amps, G, gc, (int *)nullptr, 0);
      TLAUNCH(k_vox_prep, dim3(nwp), dim3(256), 0, st, (const float4 *)gc, V, rec,
              (int4 *)(w + o_box), (double *)(w + o_wp));
      TLAUNCH(k_vox_count, dim3(cdivv(N, 4)), dim3(256), 0, st, (const int4 *)(w + o_box), V, cnt);
    }
    TLAUNCH(k_vox_scan, dim3(1), dim3(1024), 0, st, (const int *)cnt, nbr,
            (const double *)(w + o_wp), N > 0 ? nwp : 0, (int *)(w + o_off),
            (double *)(w + o_scale));
    return CS_OK;
  };
  rc = prepare();
  if (rc) return rc;
  // the list length is known only now: read it back (this call synchronises)
  int total = 0;
  HIPCHK(hipMemcpyAsync(&total, (char *)ctx->vol + o_off + (size_t)nbr * 4, sizeof(int),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (total < 0) return fail(ctx, CS_ERR_UNSUPPORTED, "too many (brick, Gaussian) pairs");
  const size_t need = o_list + al256v((size_t)total * 4 + 4);
  if (need > ctx->vol_bytes) {
    // a larger scratch does not keep its contents: prepare again (same values)
    rc = grow(ctx, &ctx->vol, &ctx->vol_bytes, need);
    if (rc) return rc;
    rc = prepare();
    if (rc) return rc;
  }
  char *w = (char *)ctx->vol;
  const float4 *rec = (const float4 *)(w + o_rec);
  const int *off = (const int *)(w + o_off);
  const double *scale = (const double *)(w + o_scale);
  int *list = (int *)(w + o_list);
  if (N > 0 && total > 0)
    TLAUNCH(k_vox_fill, dim3(cdivv(N, 4)), dim3(256), 0, st, (const int4 *)(w + o_box), V, off,
            (int *)(w + o_cur), list);
  // one 64-lane workgroup per 4^3 sub-cube, eight per brick (XCD-aware order)
  TLAUNCH(k_vox_eval, dim3(cdivv(nbr, 8) * 64), dim3(64), 0, st, rec, (const int *)list, off, V,
          scale, vol);
  return CS_OK;
}

int cs_fsc(cs_ctx *ctx, const float *vol_a, const float *vol_b, int32_t D, float *fsc,
           void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!vol_a || !vol_b || !fsc) return fail(ctx, CS_ERR_INVALID_ARG, "null volume or output");
  FftPlan P;
  if (D < 2 || D % 2 != 0 || D > 512 || !fft_plan(D, P))
    return fail(ctx, CS_ERR_UNSUPPORTED, "D must be even with prime factors 2 and 3 (<= 512)");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const float2 *tw = nullptr;
  int rc = get_twiddles(ctx, D, &tw);
  if (rc) return rc;
  const int Dh = D / 2 + 1, ns = D / 2 + 1;
  const size_t spec = (size_t)D * D * Dh * 8;
  const size_t o_a = 0, o_b = al256v(spec), o_scale = o_b + al256v(spec), o_sums = o_scale + 256;
  const size_t o_part = o_sums + al256v((size_t)3 * ns * 8);
  rc = grow(ctx, &ctx->vol, &ctx->vol_bytes, o_part + (size_t)2 * kEnergyBlocks * 8);
  if (rc) return rc;
  char *w = (char *)ctx->vol;
  float2 *fa = (float2 *)(w + o_a), *fb = (float2 *)(w + o_b);
  double *scale = (double *)(w + o_scale);
  unsigned long long *sums = (unsigned long long *)(w + o_sums);
  double *part = (double *)(w + o_part);
  TLAUNCH(k_fsc_energy_part, dim3(kEnergyBlocks), dim3(256), 0, st, vol_a, vol_b,
          (int64_t)D * D * D, part);
  TLAUNCH(k_fsc_energy_scale, dim3(1), dim3(kEnergyBlocks), 0, st, (const double *)part, D, scale);
  const dim3 rgrid(cdivv(D / 2, kRowTeamsVol), D);
  const size_t rlds = (size_t)(kRowTeamsVol * 2 + 1) * D * 8;
  const int cpw = fft_cols_per_block(D, D);
  const size_t alds = (size_t)(cpw * 2 + 1) * D * 8;
  for (int v = 0; v < 2; ++v) {
    const float *src = v ? vol_b : vol_a;
    float2 *F = v ? fb : fa;
    TLAUNCH(k_fft_rows_fwd, rgrid, dim3(256), rlds, st, src, P, tw, D, F);   // x (real rows)
    TLAUNCH(k_fft_axis, dim3(cdivv(Dh, cpw), D), dim3(256), alds, st, F, P, tw, Dh, cpw);  // y
    TLAUNCH(k_fft_axis, dim3(cdivv((int64_t)D * Dh, cpw), 1), dim3(256), alds, st, F, P, tw,
            D * Dh, cpw);                                                        // z
  }
  TLAUNCH(k_fill_u64z, dim3(cdivv(3 * ns, 256)), dim3(256), 0, st, sums, 3 * ns);
  const unsigned blocks = std::min<unsigned>(2048, cdivv((int64_t)D * D * Dh, 256));
  TLAUNCH(k_fsc_shells, dim3(blocks), dim3(256), (size_t)3 * ns * 8, st, (const float2 *)fa,
          (const float2 *)fb, D, (const double *)scale, sums);
  TLAUNCH(k_fsc_final, dim3(cdivv(ns, 256)), dim3(256), 0, st, (const unsigned long long *)sums, ns,
          (const double *)scale, fsc);
  return CS_OK;
}

int cs_fsc_resolution(cs_ctx *ctx, const float *fsc, int32_t D, float pixel, float threshold,
                      int32_t *shell, float *resolution, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!fsc || (!shell && !resolution)) return fail(ctx, CS_ERR_INVALID_ARG, "null curve or outputs");
  if (D < 2 || D % 2 != 0 || D > 512) return fail(ctx, CS_ERR_UNSUPPORTED, "D must be even, at most 512");
  if (!(pixel > 0.f)) return fail(ctx, CS_ERR_INVALID_ARG, "voxel size must be positive");
  if (!(threshold == threshold)) return fail(ctx, CS_ERR_INVALID_ARG, "threshold is NaN");
  HIPCHK(hipSetDevice(ctx->device));
  TLAUNCH(k_fsc_resolution, dim3(1), dim3(64), 0, (hipStream_t)stream, fsc, D / 2 + 1, D, pixel,
          threshold, (int *)shell, resolution);
  return CS_OK;
}

}  // extern "C"
