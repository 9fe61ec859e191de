// C-ABI of pose scoring: pose grids, template banks rendered by the
// splatter, exhaustive grid search and gathered local refinement.
//
// The image model is the paper's (Sec. 3.2, Eq. 1; CTF in Fourier space,
// App. A.2, Eq. 14) and the score is its squared error (Sec. 3.3.5); the
// paper takes poses as given, so the search itself is this library's.
#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/cryosplat.h"
#include "cs_cnn.hpp"
#include "cs_host.hpp"
#include "cs_internal.hpp"
#include "cs_pose.hpp"

using namespace cs;

struct cs_pose_batch {
  cs_ctx *ctx = nullptr;
  int D = 0, npx = 0, F = 0, F8 = 0, r = 0, S = 0, cap = 0, P = 0;
  float pixel = 0.f;
  void *mem = nullptr;              // fixed buffers below, sized for cap particles
  float *table = nullptr, *Z = nullptr, *yy = nullptr;
  float2 *spec = nullptr;
  unsigned short *zs = nullptr, *w = nullptr, *zb = nullptr;
  bool zs_valid = false;            // shifted copies are built on first use after a load
  unsigned long long *best = nullptr;
  void *E = nullptr;                // energy matrix [P][K] of a grid search (grown on demand)
  size_t E_bytes = 0;
  void *cand = nullptr;             // candidate lists when the caller passes none
  size_t cand_bytes = 0;
};

struct cs_pose_bank {
  cs_ctx *ctx = nullptr;
  int D = 0, npx = 0, F = 0, F8 = 0, n_psi = 0, ndir = 0;
  float pixel = 0.f;
  int64_t K = 0, Kext = 0;
  float *rot = nullptr;             // [K][9]
  unsigned short *data = nullptr;   // [K][Kext] bfloat16: projection, then |FFT|^2
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  cs_pose_batch *tmp = nullptr;     // batch of the raw-image convenience calls
};

namespace {

constexpr int kRowTeamsHost = 4;  // row pairs per block of the row FFT kernels
constexpr int kBankChunk = 1024;  // rotations rendered per call
constexpr int kParticleChunk = 1024;

unsigned cdivu(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }
size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// HEALPix ring-scheme pixel centre (Gorski et al. 2005), phi ascending from
// 0 within a ring.
void healpix_ring(int nside, int64_t pix, double &theta, double &phi) {
  const int64_t ns = nside, npix = 12 * ns * ns, ncap = 2 * ns * (ns - 1);
  double z;
  if (pix < ncap) {
    int64_t i = (int64_t)(0.5 * (1.0 + std::sqrt(1.0 + 2.0 * (double)pix)));
    while (2 * i * (i - 1) > pix) --i;
    while (2 * (i + 1) * i <= pix) ++i;
    const int64_t j = pix + 1 - 2 * i * (i - 1);
    z = 1.0 - (double)(i * i) / (3.0 * (double)(ns * ns));
    phi = ((double)j - 0.5) * (0.5 * M_PI) / (double)i;
  } else if (pix < npix - ncap) {
    const int64_t ip = pix - ncap;
    const int64_t i = ip / (4 * ns) + ns;
    const int64_t j = ip % (4 * ns) + 1;
    const double fodd = ((i + ns) & 1) ? 1.0 : 0.5;
    z = (double)(2 * ns - i) * 2.0 / (3.0 * (double)ns);
    phi = ((double)j - fodd) * M_PI / (2.0 * (double)ns);
  } else {
    const int64_t ip = npix - pix;
    int64_t i = (int64_t)(0.5 * (1.0 + std::sqrt(2.0 * (double)ip - 1.0)));
    while (i > 1 && 2 * i * (i - 1) >= ip) --i;
    while (2 * i * (i + 1) < ip) ++i;
    const int64_t j = 4 * i + 1 - (ip - 2 * i * (i - 1));
    z = -1.0 + (double)(i * i) / (3.0 * (double)(ns * ns));
    phi = ((double)j - 0.5) * (0.5 * M_PI) / (double)i;
  }
  theta = std::acos(std::max(-1.0, std::min(1.0, z)));
}

// W = Rz(psi) Ry(-theta) Rz(-phi): third row is the viewing direction
// (sin t cos f, sin t sin f, cos t); psi turns the image plane.
void view_rotation(double theta, double phi, double psi, float *W) {
  const double ct = std::cos(theta), st = std::sin(theta), cf = std::cos(phi), sf = std::sin(phi);
  const double cp = std::cos(psi), sp = std::sin(psi);
  // A = Ry(-theta) Rz(-phi)
  const double A[3][3] = {{ct * cf, ct * sf, -st}, {-sf, cf, 0.0}, {st * cf, st * sf, ct}};
  const double Rz[3][3] = {{cp, -sp, 0.0}, {sp, cp, 0.0}, {0.0, 0.0, 1.0}};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += Rz[i][k] * A[k][j];
      W[3 * i + j] = (float)s;
    }
}

int ensure_scratch(cs_pose_bank *b, size_t bytes) {
  cs_ctx *ctx = b->ctx;
  if (bytes <= b->scratch_bytes) return CS_OK;
  HIPCHK(hipDeviceSynchronize());
  if (b->scratch) HIPCHK(hipFree(b->scratch));
  b->scratch = nullptr;
  b->scratch_bytes = 0;
  if (hipMalloc(&b->scratch, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, CS_ERR_OOM, "pose scratch of %zu bytes", bytes);
  }
  b->scratch_bytes = bytes;
  return CS_OK;
}

// Z = F^-1(H^ F Y) for P particles, plus the CTF table H^ / D^2.
int ctf_filter_into(cs_ctx *ctx, int D, float pixel, const float *Y, const cs_ctf *ctf, int P,
                    float *table, float2 *spec, float *Z, hipStream_t st) {
  const int Dh = D / 2 + 1;
  FftPlan P_;
  fft_plan(D, P_);
  const float2 *tw = nullptr;
  int rc = get_twiddles(ctx, D, &tw);
  if (rc) return rc;
  // one grid row per particle (the kernel strides rows beyond 65535), a few
  // entries per thread where there are enough particles to fill the chip
  const size_t per = (size_t)D * Dh;
  const size_t ept = P >= 16 ? 8 : 1;
  const unsigned rows = (unsigned)(P < 65535 ? P : 65535);
  hipLaunchKernelGGL(k_ctf_table, dim3(cdivu(per, 256 * ept), rows), dim3(256), 0, st, D, ctf_pixel(ctf, pixel),
                     make_ctf(ctf), P,
                     table);
  LAUNCHCHK("k_ctf_table");
  const dim3 rgrid(cdivu(D / 2, kRowTeamsHost), P);
  const size_t rlds = (size_t)(kRowTeamsHost * 2 + 1) * D * 8;
  const int cpw = fft_cols_per_block(D, P);
  const dim3 cgrid(cdivu(Dh, cpw), P);
  const size_t clds = (size_t)(cpw * 2 + 1) * D * 8;
  hipLaunchKernelGGL(k_fft_rows_fwd, rgrid, dim3(256), rlds, st, Y, P_, tw, P, spec);
  LAUNCHCHK("k_fft_rows_fwd");
  hipLaunchKernelGGL(k_fft_cols_ctf, cgrid, dim3(256), clds, st, spec, P_, tw, P, cpw,
                     (const float *)table);
  LAUNCHCHK("k_fft_cols_ctf");
  hipLaunchKernelGGL(k_fft_rows_inv, rgrid, dim3(256), rlds, st, (const float2 *)spec, P_, tw, P, Z);
  LAUNCHCHK("k_fft_rows_inv");
  return CS_OK;
}

cs_ctf ctf_offset(const cs_ctf *ctf, int p0) {
  cs_ctf c = *ctf;
  c.defocus_u += p0;
  c.defocus_v += p0;
  if (c.astig) c.astig += p0;
  if (c.phase) c.phase += p0;
  return c;
}

int check_batch(cs_ctx *ctx, const cs_pose_bank *b, const cs_pose_batch *q) {
  if (!b || !q) return fail(ctx, CS_ERR_INVALID_ARG, "null bank or batch");
  if (b->D != q->D) return fail(ctx, CS_ERR_INVALID_ARG, "bank side %d != batch side %d", b->D, q->D);
  if (q->P < 1) return fail(ctx, CS_ERR_INVALID_ARG, "batch holds no particles (load it first)");
  return CS_OK;
}

}  // namespace

extern "C" {

int cs_pose_grid(int32_t nside, int32_t n_psi, float *rot, int64_t *count) {
  if (nside < 1 || nside > 1024 || n_psi < 1 || n_psi > 4096 || !count) return CS_ERR_INVALID_ARG;
  const int64_t ndir = 12 * (int64_t)nside * nside;
  *count = ndir * n_psi;
  if (!rot) return CS_OK;
  for (int64_t d = 0; d < ndir; ++d) {
    double th, ph;
    healpix_ring(nside, d, th, ph);
    for (int m = 0; m < n_psi; ++m)
      view_rotation(th, ph, 2.0 * M_PI * (double)m / (double)n_psi, rot + 9 * (d * n_psi + m));
  }
  return CS_OK;
}

int cs_pose_bank_create(cs_ctx *ctx, const cs_gaussians *g, const float *rot, int64_t K,
                        int32_t n_psi, int32_t D, float pixel, const cs_options *opt,
                        cs_pose_bank **out, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!g || !rot || !out) return fail(ctx, CS_ERR_INVALID_ARG, "null bank argument");
  *out = nullptr;
  FftPlan P;
  if (D < 16 || D % 16 != 0 || D > 512 || !fft_plan(D, P))
    return fail(ctx, CS_ERR_UNSUPPORTED, "bank side must be a multiple of 16 with prime factors 2, 3 (<= 512)");
  if (K < 1 || K > (1 << 24)) return fail(ctx, CS_ERR_INVALID_ARG, "rotation count must be in [1, 2^24]");
  if (n_psi < 0 || (n_psi > 0 && K % n_psi != 0))
    return fail(ctx, CS_ERR_INVALID_ARG, "n_psi must be 0 or divide the rotation count");
  if (!(pixel > 0.f)) return fail(ctx, CS_ERR_INVALID_ARG, "pixel size must be positive");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  cs_pose_bank *b = new cs_pose_bank();
  b->ctx = ctx;
  b->D = D;
  b->npx = D * D;
  b->F = D * (D / 2 + 1);
  b->F8 = (b->F + 127) / 128 * 128;  // K steps of the GEMMs never straddle the two segments
  b->Kext = b->npx + b->F8;
  b->K = K;
  b->n_psi = n_psi;
  b->ndir = n_psi > 0 ? (int)(K / n_psi) : 0;
  b->pixel = pixel;
  auto bail = [&](int rc) {
    if (b->rot) (void)hipFree(b->rot);
    if (b->data) (void)hipFree(b->data);
    if (b->scratch) (void)hipFree(b->scratch);
    delete b;
    return rc;
  };
  if (hipMalloc(&b->rot, (size_t)K * 9 * 4) != hipSuccess ||
      hipMalloc(&b->data, (size_t)K * b->Kext * 2) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(ctx, CS_ERR_OOM, "bank of %lld rotations", (long long)K));
  }
  if (hipMemcpyAsync(b->rot, rot, (size_t)K * 9 * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return bail(fail(ctx, CS_ERR_HIP, "copy of bank rotations failed"));
  if (fill_u16(b->data, K * b->Kext, st) != hipSuccess)
    return bail(fail(ctx, CS_ERR_HIP, "bank clear failed"));
  // render chunks of projections (no CTF), then their power spectra
  const int chunk = (int)std::min<int64_t>(K, kBankChunk);
  const int Dh = D / 2 + 1;
  const size_t qbytes = al256((size_t)chunk * b->npx * 4);
  const size_t sbytes = al256((size_t)chunk * D * Dh * 8);
  int rc = ensure_scratch(b, qbytes + sbytes);
  if (rc) return bail(rc);
  float *Q = (float *)b->scratch;
  float2 *spec = (float2 *)((char *)b->scratch + qbytes);
  const float2 *tw = nullptr;
  rc = get_twiddles(ctx, D, &tw);
  if (rc) return bail(rc);
  for (int64_t k0 = 0; k0 < K; k0 += chunk) {
    const int kc = (int)std::min<int64_t>(chunk, K - k0);
    const int cpw = fft_cols_per_block(D, kc);
    cs_views v{};
    v.rot = rot + 9 * k0;
    v.shift = nullptr;
    v.b = kc;
    v.d = D;
    v.pixel = pixel;
    rc = cs_render(ctx, g, &v, nullptr, opt, Q, stream);
    if (rc) return bail(rc);
    if (rows_to_bf16(Q, kc, b->npx, b->data + k0 * b->Kext, b->Kext, st) != hipSuccess)
      return bail(fail(ctx, CS_ERR_HIP, "bank conversion failed"));
    hipLaunchKernelGGL(k_fft_rows_fwd, dim3(cdivu(D / 2, kRowTeamsHost), kc), dim3(256),
                       (size_t)(kRowTeamsHost * 2 + 1) * D * 8, st, Q, P, tw, kc, spec);
    hipLaunchKernelGGL(k_fft_cols_power, dim3(cdivu(Dh, cpw), kc), dim3(256),
                       (size_t)(cpw * 2 + 1) * D * 8, st, (const float2 *)spec, P, tw, kc, cpw,
                       b->data + k0 * b->Kext + b->npx, (size_t)b->Kext);
    if (hipGetLastError() != hipSuccess) return bail(fail(ctx, CS_ERR_HIP, "bank spectra failed"));
  }
  *out = b;
  return CS_OK;
}

void cs_pose_bank_destroy(cs_pose_bank *b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  if (b->tmp) cs_pose_batch_destroy(b->tmp);
  if (b->rot) (void)hipFree(b->rot);
  if (b->data) (void)hipFree(b->data);
  if (b->scratch) (void)hipFree(b->scratch);
  delete b;
}

int64_t cs_pose_bank_size(const cs_pose_bank *b) { return b ? b->K : -1; }


int cs_pose_batch_create(cs_ctx *ctx, int32_t D, float pixel, int32_t capacity,
                         int32_t shift_radius, cs_pose_batch **out) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!out) return fail(ctx, CS_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  FftPlan P;
  if (D < 16 || D % 16 != 0 || D > 512 || !fft_plan(D, P))
    return fail(ctx, CS_ERR_UNSUPPORTED, "batch side must be a multiple of 16 with prime factors 2, 3 (<= 512)");
  if (capacity < 1 || capacity > (1 << 20)) return fail(ctx, CS_ERR_INVALID_ARG, "capacity must be in [1, 2^20]");
  if (shift_radius < 0 || shift_radius > 4) return fail(ctx, CS_ERR_INVALID_ARG, "shift radius must be in [0, 4]");
  if (!(pixel > 0.f)) return fail(ctx, CS_ERR_INVALID_ARG, "pixel size must be positive");
  HIPCHK(hipSetDevice(ctx->device));
  cs_pose_batch *q = new cs_pose_batch();
  q->ctx = ctx;
  q->D = D;
  q->npx = D * D;
  q->F = D * (D / 2 + 1);
  q->F8 = (q->F + 127) / 128 * 128;
  q->r = shift_radius;
  q->S = (2 * shift_radius + 1) * (2 * shift_radius + 1);
  q->cap = capacity;
  q->pixel = pixel;
  const size_t C = capacity, Dh = D / 2 + 1;
  size_t o = 0;
  // the one-pass preparation at D = 128 needs no spectrum, table or Z buffers
  const size_t CF = (D == kPrepD) ? 0 : C;
  const size_t o_table = o; o += al256(CF * q->F * 4);
  const size_t o_spec = o;  o += al256(CF * D * Dh * 8);
  const size_t o_Z = o;     o += al256(CF * q->npx * 4);
  const size_t o_zs = o;    o += al256(C * q->S * q->npx * 2);
  const size_t o_zb = o;    o += al256(C * D * (D + 16) * 2);
  const size_t o_w = o;     o += al256(C * q->F8 * 2);
  const size_t o_yy = o;    o += al256(C * 4);
  const size_t o_best = o;  o += al256(C * 8);
  if (hipMalloc(&q->mem, o) != hipSuccess) {
    (void)hipGetLastError();
    delete q;
    return fail(ctx, CS_ERR_OOM, "pose batch of %zu bytes", o);
  }
  char *m = (char *)q->mem;
  q->table = (float *)(m + o_table);
  q->spec = (float2 *)(m + o_spec);
  q->Z = (float *)(m + o_Z);
  q->zs = (unsigned short *)(m + o_zs);
  q->zb = (unsigned short *)(m + o_zb);
  q->w = (unsigned short *)(m + o_w);
  q->yy = (float *)(m + o_yy);
  q->best = (unsigned long long *)(m + o_best);
  *out = q;
  return CS_OK;
}

void cs_pose_batch_destroy(cs_pose_batch *q) {
  if (!q) return;
  (void)hipDeviceSynchronize();
  if (q->mem) (void)hipFree(q->mem);
  if (q->E) (void)hipFree(q->E);
  if (q->cand) (void)hipFree(q->cand);
  delete q;
}

int cs_pose_batch_load(cs_pose_batch *q, const float *images, const cs_ctf *ctf, int32_t P,
                       float *filtered, uint16_t *standardized, void *stream) {
  if (!q) return CS_ERR_INVALID_ARG;
  cs_ctx *ctx = q->ctx;
  if (!images) return fail(ctx, CS_ERR_INVALID_ARG, "null images");
  if (P < 1 || P > q->cap) return fail(ctx, CS_ERR_INVALID_ARG, "particle count must be in [1, capacity]");
  if (ctf && (!ctf->defocus_u || !ctf->defocus_v)) return fail(ctx, CS_ERR_INVALID_ARG, "null defocus");
  if (ctf && (!(ctf->pixel_a >= 0.f) || !std::isfinite(ctf->pixel_a)))
    return fail(ctx, CS_ERR_INVALID_ARG, "CTF pixel size must be >= 0");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  if (q->D == kPrepD) {
    const float2 *tw = nullptr;
    int rc = get_twiddles(ctx, q->D, &tw);
    if (rc) return rc;
    HIPCHK(pose_prep128(images, tw, ctf_pixel(ctf, q->pixel), make_ctf(ctf), P, q->F8, filtered, standardized,
                        q->zb, q->w, q->yy, st));
  } else {
    int rc = ctf_filter_into(ctx, q->D, q->pixel, images, ctf, P, q->table, q->spec, q->Z, st);
    if (rc) return rc;
    HIPCHK(pose_prep(images, q->Z, q->table, P, q->D, q->F8, q->zb, q->w, q->yy, st));
    if (filtered)
      HIPCHK(hipMemcpyAsync(filtered, q->Z, (size_t)P * q->npx * 4, hipMemcpyDeviceToDevice, st));
    if (standardized) HIPCHK(standardize(q->Z, P, q->npx, standardized, st));
  }
  q->zs_valid = false;
  q->P = P;
  return CS_OK;
}

int cs_pose_batch_search(cs_pose_bank *b, cs_pose_batch *q, int32_t *best_rot, int32_t *best_shift,
                         float *best_score, float *scores, float *best_rotation, void *stream) {
  if (!q) return CS_ERR_INVALID_ARG;
  cs_ctx *ctx = q->ctx;
  int rc = check_batch(ctx, b, q);
  if (rc) return rc;
  if (!best_rot) return fail(ctx, CS_ERR_INVALID_ARG, "null best_rot");
  if ((int64_t)q->P * q->S >= ((int64_t)1 << 31) || b->K * q->S >= ((int64_t)1 << 31))
    return fail(ctx, CS_ERR_UNSUPPORTED, "search too large for 32-bit indices");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  rc = grow(ctx, &q->E, &q->E_bytes, (size_t)q->P * b->K * 4);
  if (rc) return rc;
  float *E = (float *)q->E;
  if (!q->zs_valid) {
    HIPCHK(pose_shifts(q->zb, q->P, q->D, q->r, q->zs, st));
    q->zs_valid = true;
  }
  PoseGemmArgs e;
  e.A = q->w; e.lda = q->F8;
  e.B = b->data; e.ldb = b->Kext; e.boff = b->npx;
  e.M = q->P; e.N = (int)b->K; e.K = q->F8;
  e.C = E; e.ldc = b->K;
  HIPCHK(pose_gemm_store(e, st));
  HIPCHK(fill_u64(q->best, q->P, ~0ull, st));
  PoseGemmArgs a;
  a.A = q->zs; a.lda = q->npx;
  a.B = b->data; a.ldb = b->Kext; a.boff = 0;
  a.M = q->P * q->S; a.N = (int)b->K; a.K = q->npx; a.S = q->S;
  a.E = E; a.lde = b->K; a.yy = q->yy; a.best = q->best;
  a.scores = scores;
  HIPCHK(pose_gemm_score(a, st));
  HIPCHK(pose_decode(q->best, q->P, q->S, best_rot, best_shift, best_score, b->rot, best_rotation, st));
  return CS_OK;
}

int cs_pose_batch_refine(cs_pose_bank *b, cs_pose_batch *q, const float *proposal, int32_t n_dir,
                         int32_t n_psi_c, int32_t *cand, int32_t *best_rot, int32_t *best_shift,
                         float *best_score, float *scores, float *best_rotation, void *stream) {
  if (!q) return CS_ERR_INVALID_ARG;
  cs_ctx *ctx = q->ctx;
  int rc = check_batch(ctx, b, q);
  if (rc) return rc;
  if (!best_rot) return fail(ctx, CS_ERR_INVALID_ARG, "null best_rot");
  if (n_dir < 1 || n_psi_c < 1) return fail(ctx, CS_ERR_INVALID_ARG, "n_dir and n_psi_c must be >= 1");
  const int L = n_dir * n_psi_c;
  if (L > 4096) return fail(ctx, CS_ERR_INVALID_ARG, "at most 4096 candidates per particle");
  if (proposal) {
    if (b->n_psi < 1) return fail(ctx, CS_ERR_UNSUPPORTED, "bank has no (direction, psi) grid structure");
    if (n_dir > b->ndir || n_dir > 64) return fail(ctx, CS_ERR_INVALID_ARG, "n_dir must be <= min(64, bank directions)");
    if (n_psi_c > b->n_psi) return fail(ctx, CS_ERR_INVALID_ARG, "n_psi_c exceeds the bank's psi count");
  } else if (!cand) {
    return fail(ctx, CS_ERR_INVALID_ARG, "need a proposal or candidate lists");
  }
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  int *cl = cand;
  if (!cl) {
    rc = grow(ctx, &q->cand, &q->cand_bytes, (size_t)q->P * L * 4);
    if (rc) return rc;
    cl = (int *)q->cand;
  }
  if (proposal)
    HIPCHK(pose_candidates(proposal, q->P, b->rot, b->ndir, b->n_psi, n_dir, n_psi_c, cl, st));
  HIPCHK(fill_u64(q->best, q->P, ~0ull, st));
  if (pose_refine_z_lds(q->D, q->F8) <= 65536) {
    PoseRefineArgs z;
    z.zb = q->zb; z.w = q->w; z.bank = b->data; z.ldb = b->Kext;
    z.cand = cl; z.L = L; z.nrows = b->K;
    z.D = q->D; z.r = q->r; z.S = q->S; z.F8 = q->F8; z.npx = q->npx;
    z.yy = q->yy; z.best = q->best; z.scores = scores;
    HIPCHK(pose_refine_z(z, q->P, st));
    HIPCHK(pose_decode(q->best, q->P, q->S, best_rot, best_shift, best_score, b->rot, best_rotation, st));
    return CS_OK;
  }
  if (!q->zs_valid) {  // particles too large for LDS: gathered GEMM over the shifted copies
    HIPCHK(pose_shifts(q->zb, q->P, q->D, q->r, q->zs, st));
    q->zs_valid = true;
  }
  PoseGemmArgs a;
  a.A = q->zs; a.lda = q->npx;
  a.A2 = q->w; a.lda2 = q->F8; a.ka_split = q->npx;
  a.B = b->data; a.ldb = b->Kext; a.boff = 0;
  a.cand = cl; a.L = L; a.nrows = b->K;
  a.M = q->S; a.N = L; a.K = (int)b->Kext; a.S = q->S;
  a.yy = q->yy; a.best = q->best;
  a.scores = scores;
  HIPCHK(pose_gemm_refine(a, q->P, st));
  HIPCHK(pose_decode(q->best, q->P, q->S, best_rot, best_shift, best_score, b->rot, best_rotation, st));
  return CS_OK;
}

int cs_pose_batch_confidence(cs_pose_bank *b, cs_pose_batch *q, const int32_t *best_rot,
                             const float *best_score, float *z, float *sigmas, void *stream) {
  if (!q) return CS_ERR_INVALID_ARG;
  cs_ctx *ctx = q->ctx;
  int rc = check_batch(ctx, b, q);
  if (rc) return rc;
  if (!best_rot || !best_score || !z) return fail(ctx, CS_ERR_INVALID_ARG, "null argument");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(pose_confidence(b->data, b->Kext, b->npx, b->K, q->w, q->F8, q->D, q->yy, best_rot,
                         best_score, q->P, z, sigmas, (hipStream_t)stream));
  return CS_OK;
}

// Convenience forms on raw images: chunks through a batch owned by the bank.
static int bank_batch(cs_pose_bank *b, int r, cs_pose_batch **q) {
  cs_ctx *ctx = b->ctx;
  if (b->tmp && b->tmp->r != r) {
    cs_pose_batch_destroy(b->tmp);
    b->tmp = nullptr;
  }
  if (!b->tmp) {
    int rc = cs_pose_batch_create(ctx, b->D, b->pixel, kParticleChunk, r, &b->tmp);
    if (rc) return rc;
  }
  *q = b->tmp;
  return CS_OK;
}

int cs_pose_grid_search(cs_pose_bank *b, const float *images, const cs_ctf *ctf, int32_t P,
                        int32_t shift_radius, int32_t *best_rot, int32_t *best_shift,
                        float *best_score, float *scores, void *stream) {
  if (!b) return CS_ERR_INVALID_ARG;
  cs_ctx *ctx = b->ctx;
  if (P < 1 || !images) return fail(ctx, CS_ERR_INVALID_ARG, "need images and P >= 1");
  cs_pose_batch *q = nullptr;
  int rc = bank_batch(b, shift_radius, &q);
  if (rc) return rc;
  for (int p0 = 0; p0 < P; p0 += kParticleChunk) {
    const int Pc = std::min(kParticleChunk, P - p0);
    cs_ctf c{};
    if (ctf) c = ctf_offset(ctf, p0);
    rc = cs_pose_batch_load(q, images + (size_t)p0 * b->npx, ctf ? &c : nullptr, Pc, nullptr, nullptr,
                            stream);
    if (rc) return rc;
    rc = cs_pose_batch_search(b, q, best_rot + p0, best_shift ? best_shift + p0 : nullptr,
                              best_score ? best_score + p0 : nullptr,
                              scores ? scores + (size_t)p0 * b->K * q->S : nullptr, nullptr,
                              stream);
    if (rc) return rc;
  }
  return CS_OK;
}

int cs_pose_refine(cs_pose_bank *b, const float *images, const cs_ctf *ctf, int32_t P,
                   const float *proposal, int32_t n_dir, int32_t n_psi_c, int32_t shift_radius,
                   int32_t *cand, int32_t *best_rot, int32_t *best_shift, float *best_score,
                   float *scores, void *stream) {
  if (!b) return CS_ERR_INVALID_ARG;
  cs_ctx *ctx = b->ctx;
  if (P < 1 || !images) return fail(ctx, CS_ERR_INVALID_ARG, "need images and P >= 1");
  cs_pose_batch *q = nullptr;
  int rc = bank_batch(b, shift_radius, &q);
  if (rc) return rc;
  const int L = n_dir * n_psi_c;
  for (int p0 = 0; p0 < P; p0 += kParticleChunk) {
    const int Pc = std::min(kParticleChunk, P - p0);
    cs_ctf c{};
    if (ctf) c = ctf_offset(ctf, p0);
    rc = cs_pose_batch_load(q, images + (size_t)p0 * b->npx, ctf ? &c : nullptr, Pc, nullptr, nullptr,
                            stream);
    if (rc) return rc;
    rc = cs_pose_batch_refine(b, q, proposal ? proposal + 9 * (size_t)p0 : nullptr, n_dir, n_psi_c,
                              cand ? cand + (size_t)p0 * L : nullptr, best_rot + p0,
                              best_shift ? best_shift + p0 : nullptr,
                              best_score ? best_score + p0 : nullptr,
                              scores ? scores + (size_t)p0 * L * q->S : nullptr, nullptr,
                              stream);
    if (rc) return rc;
  }
  return CS_OK;
}

int cs_ctf_filter(cs_ctx *ctx, const float *images, const cs_ctf *ctf, int32_t B, int32_t D,
                  float pixel, float *out, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!images || !out || B < 1) return fail(ctx, CS_ERR_INVALID_ARG, "bad filter arguments");
  FftPlan P;
  if (D < 2 || D % 2 != 0 || D > 512 || !fft_plan(D, P))
    return fail(ctx, CS_ERR_UNSUPPORTED, "D must be even with prime factors 2, 3 (<= 512)");
  if (!(pixel > 0.f)) return fail(ctx, CS_ERR_INVALID_ARG, "pixel size must be positive");
  if (ctf && (!ctf->defocus_u || !ctf->defocus_v)) return fail(ctx, CS_ERR_INVALID_ARG, "null defocus");
  if (ctf && (!(ctf->pixel_a >= 0.f) || !std::isfinite(ctf->pixel_a)))
    return fail(ctx, CS_ERR_INVALID_ARG, "CTF pixel size must be >= 0");
  HIPCHK(hipSetDevice(ctx->device));
  const size_t Dh = D / 2 + 1;
  const size_t tb = al256((size_t)B * D * Dh * 4), sb = al256((size_t)B * D * Dh * 8);
  int rc = grow(ctx, &ctx->aux, &ctx->aux_bytes, tb + sb);
  if (rc) return rc;
  return ctf_filter_into(ctx, D, pixel, images, ctf, B, (float *)ctx->aux,
                         (float2 *)((char *)ctx->aux + tb), out, (hipStream_t)stream);
}

int cs_add_noise(cs_ctx *ctx, float *images, int32_t B, int32_t D, float snr_db, uint64_t seed,
                 int64_t offset, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!images || B < 1 || D < 1) return fail(ctx, CS_ERR_INVALID_ARG, "bad noise arguments");
  if (!std::isfinite(snr_db)) return fail(ctx, CS_ERR_INVALID_ARG, "snr_db must be finite");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(add_noise(images, B, D * D, snr_db, seed, offset, (hipStream_t)stream));
  return CS_OK;
}

int cs_pose_bank_rotations(const cs_pose_bank *b, float *rot, void *stream) {
  if (!b || !rot) return CS_ERR_INVALID_ARG;
  cs_ctx *ctx = b->ctx;
  HIPCHK(hipMemcpyAsync(rot, b->rot, (size_t)b->K * 9 * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return CS_OK;
}

}  // extern "C"
