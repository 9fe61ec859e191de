// Launchers of the pose-scoring kernels (k_pose.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cs_internal.hpp"

namespace cs {

enum { kPoseStore = 0, kPoseScore = 1, kPoseRefine = 2 };

// Operands of the pose GEMMs (bfloat16 as raw uint16, K contiguous).
struct PoseGemmArgs {
  const unsigned short *A = nullptr;   // rows of length >= K (lda elements apart)
  int64_t lda = 0;
  const unsigned short *A2 = nullptr;  // refine: second A segment (per particle), k >= ka_split
  int64_t lda2 = 0;
  int ka_split = 0;
  const unsigned short *B = nullptr;   // row n (or cand[p][n]) at B + row * ldb + boff
  int64_t ldb = 0, boff = 0;
  const int *cand = nullptr;           // refine: [P][L] bank rows (out of [0, nrows): skipped)
  int L = 0;
  int64_t nrows = 0;                   // refine: rows of B
  int M = 0, N = 0, K = 0;             // K a multiple of the kernel's K step (32 / 128)
  int S = 1;                           // shifts per particle
  float *C = nullptr;                  // store: [M][ldc]
  int64_t ldc = 0;
  const float *E = nullptr;            // score: energy [P][lde]
  int64_t lde = 0;
  const float *yy = nullptr;           // [P]
  unsigned long long *best = nullptr;  // [P] packed (score, index) minima
  float *scores = nullptr;             // optional [P][N][S]
};

// Gathered refinement with the particle in LDS (k_pose_refine_z).
struct PoseRefineArgs {
  const unsigned short *zb = nullptr;    // [P][D][D+16] bfloat16 -2 Z, wrap-padded rows
  const unsigned short *w = nullptr;     // [P][F8] energy weights
  const unsigned short *bank = nullptr;  // rows of ldb elements: D^2 pixels, then F8 spectrum
  int64_t ldb = 0;
  const int *cand = nullptr;             // [P][L] bank rows (out of [0, nrows): skipped)
  int L = 0;
  int64_t nrows = 0;
  int D = 0, r = 0, S = 1, F8 = 0, npx = 0;
  const float *yy = nullptr;
  unsigned long long *best = nullptr;
  float *scores = nullptr;               // optional [P][L][S]
};

// One-pass preparation at D = kPrepD (k_pose_prep.hip): Z = H Y (written
// when Z is not null), Z standardised per image as bfloat16 (when zs is not
// null), the padded -2 Z rows, the energy weights and ||Y||^2.
constexpr int kPrepD = 128;
hipError_t pose_prep128(const float *Y, const float2 *tw, float pixel, const CtfDev &ctf, int P,
                        int F8, float *Z, unsigned short *zs, unsigned short *zb,
                        unsigned short *w, float *yy, hipStream_t st);
hipError_t pose_prep(const float *Y, const float *Z, const float *table, int P, int D, int F8,
                     unsigned short *zb, unsigned short *w, float *yy, hipStream_t st);
hipError_t pose_shifts(const unsigned short *zb, int P, int D, int r, unsigned short *zs,
                       hipStream_t st);
hipError_t pose_refine_z(const PoseRefineArgs &a, int P, hipStream_t st);
size_t pose_refine_z_lds(int D, int F8);
hipError_t rows_to_bf16(const float *src, int64_t rows, int len, unsigned short *dst, int64_t ld,
                        hipStream_t st);
hipError_t fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t st);
hipError_t fill_u16(unsigned short *p, int64_t n, hipStream_t st);
hipError_t pose_decode(const unsigned long long *best, int P, int S, int *rot_idx, int *shift_idx,
                       float *score, const float *bank_rot, float *rot_out, hipStream_t st);
hipError_t pose_confidence(const unsigned short *bank, int64_t ldb, int64_t boff, int64_t K,
                           const unsigned short *w, int F8, int D, const float *yy,
                           const int *rot_idx, const float *score, int P, float *z, float *sig,
                           hipStream_t st);
hipError_t pose_gemm_store(const PoseGemmArgs &a, hipStream_t st);
hipError_t pose_gemm_score(const PoseGemmArgs &a, hipStream_t st);
hipError_t pose_gemm_refine(const PoseGemmArgs &a, int P, hipStream_t st);
hipError_t pose_candidates(const float *prop, int P, const float *bank_rot, int ndir, int n_psi,
                           int n_dir, int n_psi_c, int *cand, hipStream_t st);

hipError_t add_noise(float *img, int B, int npx, float snr_db, unsigned long long seed,
                     long long offset, hipStream_t st);

}  // namespace cs
