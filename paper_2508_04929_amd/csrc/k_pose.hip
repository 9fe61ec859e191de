// Pose scoring kernels: the squared error between a particle image and the
// CTF-modulated projection of the mixture at every (rotation, shift) of a
// pose bank, without rendering per particle.
//
// With H the particle's CTF (a real, even Fourier filter, hence a symmetric
// circulant operator), Q_k the projection at rotation k and S_t a circular
// shift by t whole pixels,
//   || H S_t Q_k - Y ||^2 = ||Y||^2 + ||H Q_k||^2 - 2 < S_t Q_k, H Y >,
// and by Parseval ||H Q_k||^2 = sum_f w_f |H^(f)|^2 |Q^_k(f)|^2 / D^2 over
// the half spectrum (w_f = 1 on the kx = 0 and Nyquist columns, 2 elsewhere).
// Both sums are dense contractions over pixels / frequencies between
// per-particle rows and per-rotation rows, done here as BF16 MFMA GEMMs with
// FP32 accumulation; the energy term is a GEMM of its own for the full
// grid and is fused into the K dimension for gathered candidate lists.
#include <algorithm>

#include "cs_pose.hpp"

namespace cs {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

__device__ __forceinline__ float pbf2f(unsigned short v) { return __uint_as_float((unsigned)v << 16); }

__device__ __forceinline__ unsigned short pf2bf(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// Monotone map of a float to uint32 (total order of non-NaN values).
__device__ __forceinline__ unsigned ord_bits(float v) {
  const unsigned u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord_float(unsigned o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

// ---------------------------------------------------------------------------
// Particle preparation.
//   k_pose_zpad    (block = particle): -2 Z as bfloat16 rows with wrap padding
//   k_pose_shifts  (block = (particle, shift s)), from the padded rows:
//     zs[p][s][i][j] = -2 Z[p][(i - dy) mod D][(j + dx) mod D]   (bfloat16)
//     shift s = (dy + r)(2r + 1) + (dx + r); 8 outputs (16 bytes) per lane
//   k_pose_weights (block = particle):
//     w[p][f] = w_f * table[p][f]^2 * D^2 = w_f |H^(f)|^2 / D^2, zero pad to F8
//     yy[p]   = sum Y^2
// where Z = H Y and table = H^ / D^2 (the CTF table of the FFT kernels).
// ---------------------------------------------------------------------------
// 8 consecutive bfloat16 starting at element c of a dword-aligned row.
// Branch-free: five dword reads and a funnel shift by 0 or 16 bits (the row
// holds at least c / 2 + 5 dwords).
__device__ __forceinline__ uint4 load8_at(const unsigned *row, int c) {
  const int d = c >> 1;
  const unsigned sh = (unsigned)(c & 1) << 4;
  const unsigned w0 = row[d], w1 = row[d + 1], w2 = row[d + 2], w3 = row[d + 3], w4 = row[d + 4];
  return make_uint4(__builtin_amdgcn_alignbit(w1, w0, sh), __builtin_amdgcn_alignbit(w2, w1, sh),
                    __builtin_amdgcn_alignbit(w3, w2, sh), __builtin_amdgcn_alignbit(w4, w3, sh));
}

// zb[p][i][t] = bfloat16(-2 Z[p][i][(t - 8) mod D]), rows of D + 16 (8 columns
// of wrap-around on each side), so that a shift |dx| <= 4 is a plain offset.
__global__ void __launch_bounds__(256)
k_pose_zpad(const float *Z, int D, unsigned short *zb) {
  const int p = blockIdx.x, RS = D + 16;
  const float *z = Z + (size_t)p * D * D;
  unsigned short *o = zb + (size_t)p * D * RS;
  for (int e = threadIdx.x; e < D * RS; e += 256) {
    const int i = e / RS, t = e - i * RS;
    int c = t - 8;
    c += (c < 0) ? D : 0;
    c -= (c >= D) ? D : 0;
    o[e] = pf2bf(-2.f * z[(size_t)i * D + c]);
  }
}

// zs[p][s][i][j] = zb[p][(i - dy) mod D][j + dx + 8]  (block = (particle, shift))
__global__ void __launch_bounds__(256)
k_pose_shifts(const unsigned short *zb, int D, int r, unsigned short *zs) {
  const int p = blockIdx.x, s = blockIdx.y;
  const int side = 2 * r + 1, S = side * side, npx = D * D, RS = D + 16;
  const int dy = s / side - r, dx = s % side - r;
  const unsigned short *zp = zb + (size_t)p * D * RS;
  uint4 *o = (uint4 *)(zs + ((size_t)p * S + s) * npx);
  const int per_row = D / 8;
  for (int v = threadIdx.x; v < npx / 8; v += 256) {
    const int i = v / per_row, j0 = (v - i * per_row) * 8;
    int si = i - dy;
    si += (si < 0) ? D : 0;
    si -= (si >= D) ? D : 0;
    o[v] = load8_at((const unsigned *)(zp + (size_t)si * RS), j0 + dx + 8);
  }
}

__global__ void __launch_bounds__(256)
k_pose_weights(const float *Y, const float *table, int D, int F8, unsigned short *w, float *yy) {
  const int p = blockIdx.x;
  const int npx = D * D, Dh = D / 2 + 1, F = D * Dh;
  const float4 *y = (const float4 *)(Y + (size_t)p * npx);
  double acc = 0.0;
  for (int i = threadIdx.x; i < npx / 4; i += 256) {
    const float4 v = y[i];
    acc += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
  }
  const float *tb = table + (size_t)p * F;
  const float d2 = (float)D * (float)D;
  for (int f = threadIdx.x; f < F8; f += 256) {
    float v = 0.f;
    if (f < F) {
      const int kx = f % Dh;
      const float wf = (kx == 0 || kx == D / 2) ? 1.f : 2.f;
      const float h = tb[f];
      v = wf * h * h * d2;
    }
    w[(size_t)p * F8 + f] = pf2bf(v);
  }
  __shared__ double red[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) yy[p] = (float)(red[0] + red[1] + red[2] + red[3]);
}

// FP32 rows -> bfloat16 rows of a wider matrix: dst[r * ld + c] (c < len).
__global__ void __launch_bounds__(256)
k_rows_to_bf16(const float *src, int64_t rows, int len, unsigned short *dst, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= rows * len) return;
  const int64_t rr = i / len;
  const int c = (int)(i - rr * len);
  dst[rr * ld + c] = pf2bf(src[i]);
}

__global__ void __launch_bounds__(256) k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256) k_fill_u16(unsigned short *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}

// best key -> (rotation index, shift index, score) and optionally the
// rotation matrix itself, bank_rot[rotation index] (NaN when nothing won)
__global__ void __launch_bounds__(256)
k_pose_decode(const unsigned long long *best, int P, int S, int *rot_idx, int *shift_idx,
              float *score, const float *bank_rot, float *rot_out) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const unsigned long long k = best[p];
  const unsigned idx = (unsigned)(k & 0xffffffffu);
  const bool none = k == ~0ull;
  if (rot_idx) rot_idx[p] = none ? -1 : (int)(idx / S);
  if (shift_idx) shift_idx[p] = none ? -1 : (int)(idx % S);
  if (score) score[p] = none ? __int_as_float(0x7fc00000) : ord_float((unsigned)(k >> 32));
  if (rot_out) {
    const float *A = bank_rot + 9 * (size_t)(idx / S);
#pragma unroll
    for (int e = 0; e < 9; ++e) rot_out[9 * (size_t)p + e] = none ? __int_as_float(0x7fc00000) : A[e];
  }
}

// Fit statistic of each particle's winning pose (block = particle):
//   E = ||H Q_k||^2 = sum_f w[p][f] |Q^_k(f)|^2   (same bfloat16 operands
//       and Parseval weights as the scores), k = rot_idx[p]
//   z = (||Y||^2 - score) / E = 2 <S_t Q_k, H Y> / ||H Q_k||^2 - 1,
// i.e. 2 a - 1 with a the least-squares amplitude of the winning template
// in the particle; and (optional) its shortfall from a perfect fit in units
// of the noise spread of z at the true pose of a noise-dominated particle,
//   s = (1 - z) sqrt(E) D / (2 ||Y||)     (std of z = 2 sigma / ||H Q_k||,
//                                           sigma^2 ~ ||Y||^2 / D^2).
// NaN where no rotation won or E is not positive.
__global__ void __launch_bounds__(256)
k_pose_confidence(const unsigned short *bank, int64_t ldb, int64_t boff, int64_t K,
                  const unsigned short *w, int F8, int D, const float *yy, const int *rot_idx,
                  const float *score, float *z, float *sig) {
  const int p = blockIdx.x;
  const int k = rot_idx[p];
  __shared__ float red[4];
  float acc = 0.f;
  if (k >= 0 && k < K) {
    const unsigned short *q = bank + (size_t)k * ldb + boff;
    const unsigned short *wp = w + (size_t)p * F8;
    for (int f = threadIdx.x; f < F8; f += 256) acc += pbf2f(wp[f]) * pbf2f(q[f]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float E = (red[0] + red[1]) + (red[2] + red[3]);
    const bool ok = k >= 0 && k < K && E > 0.f;
    const float zp = ok ? (yy[p] - score[p]) / E : __int_as_float(0x7fc00000);
    z[p] = zp;
    if (sig) sig[p] = ok && yy[p] > 0.f ? (1.f - zp) * sqrtf(E) * (float)D / (2.f * sqrtf(yy[p]))
                                       : __int_as_float(0x7fc00000);
  }
}

// ---------------------------------------------------------------------------
// TN GEMM on MFMA: C[m][n] = sum_k A[m][k] B[n][k], bfloat16 operands with
// K contiguous, FP32 accumulation (v_mfma_f32_16x16x32_bf16), K a multiple
// of 32.  256 threads = 4 waves in a WGM x (4 / WGM) arrangement; tiles of
// BM x BN, K steps of 32 double-buffered through LDS (rows padded to 80 B so
// that the 16-byte operand reads of 16 lanes hit 64 distinct banks).
//
//   MODE kStore:  C (FP32) = A B^T                        (energy matrix)
//   MODE kScore:  rows m = p S + s, value = acc + E[p][n] + yy[p];
//                 per-particle minimum of (value, n S + s) by 64-bit atomicMin
//   MODE kRefine: block x = particle p, rows s < S, B rows gathered through
//                 cand[p][n]; A switches at k = ka_split from the shifted
//                 particle rows to the particle's energy weights (energy fused
//                 into the contraction); value = acc + yy[p]
// ---------------------------------------------------------------------------
template <int BM, int BN, int WGM, int MODE, int kBK>
__global__ void __launch_bounds__(256) k_pose_gemm(PoseGemmArgs a) {
  constexpr int kLDK = kBK + 8;   // padded row: 16-lane operand reads hit distinct banks
  constexpr int KQ = kBK / 8;     // 16-byte loads per row and K step
  constexpr int WGN = 4 / WGM;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int TI = WTM / 16, TJ = WTN / 16;
  constexpr int LA = BM * kBK / 8, LB = BN * kBK / 8;  // 16-byte loads per K step
  constexpr int NA = (LA + 255) / 256, NB = (LB + 255) / 256;
  static_assert(TI >= 1 && TJ >= 1 && LA % 64 == 0 && LB % 64 == 0, "tile shape");
  __shared__ unsigned short sA[2][BM][kLDK];
  __shared__ unsigned short sB[2][BN][kLDK];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = (wv / WGN) * WTM, wn = (wv % WGN) * WTN;

  int mt, nt, p = 0;
  if (MODE == kPoseRefine) {
    p = blockIdx.x;
    mt = 0;
    nt = blockIdx.y;
  } else {
    // XCD-aware order: consecutive block ids land on different XCDs, so give
    // each XCD a contiguous range of tiles, grouped 8 row tiles at a time.
    const int Mt = (a.M + BM - 1) / BM, Nt = (a.N + BN - 1) / BN;
    const int T = Mt * Nt;
    int t = blockIdx.x;
    if ((T & 7) == 0) t = (t & 7) * (T >> 3) + (t >> 3);
    const int G = 8;
    const int grp = t / (G * Nt);
    const int first = grp * G;
    const int gs = min(Mt - first, G);
    const int within = t - grp * G * Nt;
    mt = first + within % gs;
    nt = within / gs;
  }
  const int m0 = mt * BM, n0 = nt * BN;

  // global -> register staging of one K step
  uint4 ra[NA], rb[NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int idx = tid + 256 * i, row = idx / KQ, kq = (idx % KQ) * 8;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (idx >= LA) {
      } else if (MODE == kPoseRefine) {
        if (row < a.S) {
          const int k = k0 + kq;
          v = (k < a.ka_split)
                  ? *(const uint4 *)(a.A + ((int64_t)p * a.S + row) * a.lda + k)
                  : *(const uint4 *)(a.A2 + (int64_t)p * a.lda2 + (k - a.ka_split));
        }
      } else {
        const int m = m0 + row;
        if (m < a.M) v = *(const uint4 *)(a.A + (int64_t)m * a.lda + k0 + kq);
      }
      ra[i] = v;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int idx = tid + 256 * i, row = idx / KQ, kq = (idx % KQ) * 8;
      uint4 v = make_uint4(0, 0, 0, 0);
      const int n = n0 + row;
      if (idx < LB && n < a.N) {
        const int64_t brow = (MODE == kPoseRefine) ? (int64_t)a.cand[(int64_t)p * a.L + n] : n;
        if (MODE != kPoseRefine || (brow >= 0 && brow < a.nrows))
          v = *(const uint4 *)(a.B + brow * a.ldb + a.boff + k0 + kq);
      }
      rb[i] = v;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int idx = tid + 256 * i;
      if (idx < LA) *(uint4 *)&sA[buf][idx / KQ][(idx % KQ) * 8] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int idx = tid + 256 * i;
      if (idx < LB) *(uint4 *)&sB[buf][idx / KQ][(idx % KQ) * 8] = rb[i];
    }
  };

  f32x4_t acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  const int nk = a.K / kBK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * kBK);
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 32) {
      bf16x8_t af[TI], bv[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i)
        af[i] = *(const bf16x8_t *)&sA[cur][wm + i * 16 + (lane & 15)][kk + (lane >> 4) * 8];
#pragma unroll
      for (int j = 0; j < TJ; ++j)
        bv[j] = *(const bf16x8_t *)&sB[cur][wn + j * 16 + (lane & 15)][kk + (lane >> 4) * 8];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }

  // ---- epilogue (acc[i][j][r] is C[wm + 16 i + 4 (lane / 16) + r][wn + 16 j + lane % 16])
  if (MODE == kPoseStore) {
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
          const int n = n0 + wn + j * 16 + (lane & 15);
          if (m < a.M && n < a.N) a.C[(int64_t)m * a.ldc + n] = acc[i][j][r];
        }
    return;
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ml = wm + i * 16 + (lane >> 4) * 4 + r;
      int pp, s;
      bool valid;
      if (MODE == kPoseRefine) {
        pp = p;
        s = ml;
        valid = s < a.S;
      } else {
        const int m = m0 + ml;
        valid = m < a.M;
        pp = valid ? m / a.S : 0;
        s = valid ? m - pp * a.S : 0;
      }
      unsigned long long key = ~0ull;
      if (valid) {
        const float base = a.yy[pp];
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          const int n = n0 + wn + j * 16 + (lane & 15);
          if (n < a.N) {
            float v = acc[i][j][r] + base;
            int rot;
            if (MODE == kPoseRefine) {
              rot = a.cand[(int64_t)pp * a.L + n];
              if (rot < 0 || rot >= a.nrows) continue;
            } else {
              v += a.E[(int64_t)pp * a.lde + n];
              rot = n;
            }
            if (a.scores) a.scores[((int64_t)pp * a.N + n) * a.S + s] = v;
            const unsigned long long k2 =
                ((unsigned long long)ord_bits(v) << 32) | (unsigned)(rot * a.S + s);
            key = k2 < key ? k2 : key;
          }
        }
      }
      // minimum over the 16 lanes that hold the same row
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        const unsigned lo = __shfl_xor((unsigned)(key & 0xffffffffu), o, 64);
        const unsigned hi = __shfl_xor((unsigned)(key >> 32), o, 64);
        const unsigned long long k2 = ((unsigned long long)hi << 32) | lo;
        key = k2 < key ? k2 : key;
      }
      if ((lane & 15) == 0 && key != ~0ull) atomicMin(a.best + pp, key);
    }
}

// ---------------------------------------------------------------------------
// Gathered refinement with the particle resident in LDS (block = particle x
// 64 candidates, one wave per 16 candidates).  K runs over the bank row:
// D^2 pixels, then the power spectrum.  MFMA A rows are the shifts s; their
// pixel fragments are assembled from the padded -2 Z rows in LDS (a shift is
// a row / column offset), their spectrum fragments are the particle's energy
// weights (equal for every shift).  B fragments are 16 bytes per lane straight
// from the gathered bank row into registers, PF slices ahead; waves never
// synchronise after the LDS fill.  Value = acc + ||Y||^2; 64-bit atomicMin of
// (score, bank row x S + s) per particle.
// ---------------------------------------------------------------------------
template <int PF, int KSPLIT, bool A32>
__global__ void __launch_bounds__(256) k_pose_refine_z(PoseRefineArgs a) {
  extern __shared__ unsigned lz[];
  constexpr int NG = 4 / KSPLIT;  // candidate groups of 16 per block
  // the wave index is uniform across the wave: in a scalar register, so that
  // the K-range bounds below and the branches on them are scalar
  const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cg = wv / KSPLIT, kp = wv % KSPLIT;
  const int D = a.D, RS = D + 16;
  const int zdw = D * RS / 2, wdw = a.F8 / 2;
  const uint4 *gz = (const uint4 *)(a.zb + (size_t)p * D * RS);
  for (int q = tid; q < zdw / 4; q += 256) ((uint4 *)lz)[q] = gz[q];
  const uint4 *gw = (const uint4 *)(a.w + (size_t)p * a.F8);
  for (int q = tid; q < wdw / 4; q += 256) ((uint4 *)(lz + zdw))[q] = gw[q];
  __syncthreads();

  const int n = blockIdx.y * (16 * NG) + cg * 16 + (lane & 15);
  int64_t brow = -1;
  if (n < a.L) {
    brow = a.cand[(int64_t)p * a.L + n];
    if (brow < 0 || brow >= a.nrows) brow = -1;
  }
  const int kq = (lane >> 4) * 8;
  // a skipped candidate reads bank row 0 (its sums are never used), which
  // keeps the loads free of divergent branches
  const unsigned short *bp = a.bank + (brow < 0 ? 0 : brow * a.ldb) + kq;
  const int side = 2 * a.r + 1;
  // lanes of shift rows s >= S read the unshifted particle; their sums are
  // never used
  int dx[2], dy[2];
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    const int s = f * 16 + (lane & 15);
    dy[f] = s < a.S ? s / side - a.r : 0;
    dx[f] = s < a.S ? s % side - a.r : 0;
  }
  const int nsl_all = (a.npx + a.F8) / 32, npsl = a.npx / 32;
  // this wave's part of the K slices
  const int ks0 = (int)((int64_t)nsl_all * kp / KSPLIT), ks1 = (int)((int64_t)nsl_all * (kp + 1) / KSPLIT);
  const uint4 zero = make_uint4(0, 0, 0, 0);
  uint4 q[PF];
#pragma unroll
  for (int u = 0; u < PF; ++u)
    q[u] = (ks0 + u < ks1) ? *(const uint4 *)(bp + (size_t)(ks0 + u) * 32) : zero;
  f32x4_t acc[2] = {f32x4_t{0.f, 0.f, 0.f, 0.f}, f32x4_t{0.f, 0.f, 0.f, 0.f}};
  // A operand of a pixel slice: 8 pixels of image row i, columns j .. j + 7,
  // shifted by (dy, dx) = dword address ad[f] into the padded rows and a
  // funnel shift sh[f] (the column parity never changes: j moves by 32 or by
  // -D, both even); the addresses move along with j instead of being
  // recomputed.  With D a multiple of 32 every lane changes row at the same
  // slice (a scalar countdown); otherwise each lane checks its own column.
  const int e0 = min(ks0, npsl) * 32 + kq;
  int j = e0 % D;
  int cs = (D - (e0 - kq) % D) / 32;  // slices left in the current row (A32)
  int ad[2], si[2];
  unsigned sh[2];
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    si[f] = (e0 / D - dy[f] + D) % D;
    const int c = j + dx[f] + 8;
    sh[f] = (unsigned)(c & 1) << 4;
    ad[f] = si[f] * (RS / 2) + (c >> 1);
  }
  const unsigned *lw = lz + zdw;
  auto next_row = [&](int f) {
    ad[f] += RS / 2 - D / 2;
    if (++si[f] == D) {
      si[f] = 0;
      ad[f] -= D * (RS / 2);
    }
  };
  auto step = [&](int ks, const uint4 &b) {
    uint4 av[2];
    if (ks < npsl) {
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const unsigned *r = lz + ad[f];
        const unsigned w0 = r[0], w1 = r[1], w2 = r[2], w3 = r[3], w4 = r[4];
        av[f] = make_uint4(__builtin_amdgcn_alignbit(w1, w0, sh[f]), __builtin_amdgcn_alignbit(w2, w1, sh[f]),
                           __builtin_amdgcn_alignbit(w3, w2, sh[f]), __builtin_amdgcn_alignbit(w4, w3, sh[f]));
        ad[f] += 16;
      }
      if (A32) {
        if (--cs == 0) {
          cs = D / 32;
#pragma unroll
          for (int f = 0; f < 2; ++f) next_row(f);
        }
      } else {
        // D >= 16: at most two row changes per slice
        j += 32;
#pragma unroll
        for (int t = 0; t < 2; ++t)
          if (j >= D) {
            j -= D;
#pragma unroll
            for (int f = 0; f < 2; ++f) next_row(f);
          }
      }
    } else {
      av[0] = av[1] = ((const uint4 *)lw)[((ks - npsl) * 32 + kq) >> 3];
    }
    bf16x8_t bb, a0, a1;
    __builtin_memcpy(&bb, &b, 16);
    __builtin_memcpy(&a0, &av[0], 16);
    __builtin_memcpy(&a1, &av[1], 16);
    acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bb, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bb, acc[1], 0, 0, 0);
  };
  // full groups of PF slices: no bounds checks; then the tail
  int k0 = ks0;
  for (; k0 + PF <= ks1; k0 += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int ks = k0 + u;
      const uint4 b = q[u];
      if (ks + PF < ks1) q[u] = *(const uint4 *)(bp + (size_t)(ks + PF) * 32);
      step(ks, b);
    }
  }
#pragma unroll
  for (int u = 0; u < PF; ++u)
    if (k0 + u < ks1) step(k0 + u, q[u]);
  if (KSPLIT > 1) {
    // partial sums of the K parts, added in part order (deterministic); the
    // particle's LDS rows are no longer read after this barrier
    __syncthreads();
    float *red = (float *)lz;
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[((wv * 2 + f) * 4 + r) * 64 + lane] = acc[f][r];
    __syncthreads();
    if (kp != 0) return;
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = 0.f;
        for (int t = 0; t < KSPLIT; ++t) v += red[(((cg * KSPLIT + t) * 2 + f) * 4 + r) * 64 + lane];
        acc[f][r] = v;
      }
  }
  // acc[f][r] = C[shift f*16 + 4*(lane/16) + r][candidate lane % 16]
  unsigned long long key = ~0ull;
  if (brow >= 0) {
    const float base = a.yy[p];
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = f * 16 + (lane >> 4) * 4 + r;
        if (s < a.S) {
          const float v = acc[f][r] + base;
          if (a.scores) a.scores[((int64_t)p * a.L + n) * a.S + s] = v;
          const unsigned long long k2 =
              ((unsigned long long)ord_bits(v) << 32) | (unsigned)(brow * a.S + s);
          key = k2 < key ? k2 : key;
        }
      }
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned lo = __shfl_xor((unsigned)(key & 0xffffffffu), o, 64);
    const unsigned hi = __shfl_xor((unsigned)(key >> 32), o, 64);
    const unsigned long long k2 = ((unsigned long long)hi << 32) | lo;
    key = k2 < key ? k2 : key;
  }
  if (lane == 0 && key != ~0ull) atomicMin(a.best + p, key);
}

size_t pose_refine_z_lds(int D, int F8) {
  // particle rows + energy weights; the K-split reduction (8 KiB) reuses them
  return std::max<size_t>((size_t)D * (D + 16) * 2 + (size_t)F8 * 2, 8192);
}

// ---------------------------------------------------------------------------
// Refinement candidates (one wave per particle): the n_dir bank directions
// nearest the proposal's viewing direction (third row of the proposal W),
// and for each the n_psi_c in-plane indices around the angle psi* that
// maximises trace(W^T Rz(psi) A_d) = cos psi (M00 + M11) + sin psi (M01 - M10)
// + M22 with M = A_d W^T, A_d the bank rotation of direction d at psi = 0.
// Bank rotation index = d * n_psi + m, psi_m = 2 pi m / n_psi.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_pose_candidates(const float *prop, int P, const float *bank_rot, int ndir, int n_psi, int n_dir,
                  int n_psi_c, int *cand) {
  // viewing directions (third rows at psi = 0) of the bank, staged once per
  // block of four particles
  extern __shared__ float vd[];
  for (int d = threadIdx.x; d < ndir; d += 256) {
    const float *A = bank_rot + 9 * ((size_t)d * n_psi);
    vd[3 * d] = A[6];
    vd[3 * d + 1] = A[7];
    vd[3 * d + 2] = A[8];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= P) return;  // whole wave exits together
  const float *W = prop + 9 * (size_t)p;
  const float v0 = W[6], v1 = W[7], v2 = W[8];
  const int L = n_dir * n_psi_c;
  unsigned long long prev = ~0ull;
  for (int q = 0; q < n_dir; ++q) {
    unsigned long long best = 0ull;
    for (int d = lane; d < ndir; d += 64) {
      const float dot = vd[3 * d] * v0 + vd[3 * d + 1] * v1 + vd[3 * d + 2] * v2;
      const unsigned long long k = ((unsigned long long)ord_bits(dot) << 32) | (0xffffffffu - (unsigned)d);
      if (k < prev && k > best) best = k;
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned lo = __shfl_xor((unsigned)(best & 0xffffffffu), o, 64);
      const unsigned hi = __shfl_xor((unsigned)(best >> 32), o, 64);
      const unsigned long long k2 = ((unsigned long long)hi << 32) | lo;
      best = k2 > best ? k2 : best;
    }
    prev = best;
    int d = (int)(0xffffffffu - (unsigned)(best & 0xffffffffu));
    d = (d >= 0 && d < ndir) ? d : 0;
    if (lane == 0) {
      const float *A = bank_rot + 9 * ((size_t)d * n_psi);
      float M[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          M[i][j] = A[3 * i] * W[3 * j] + A[3 * i + 1] * W[3 * j + 1] + A[3 * i + 2] * W[3 * j + 2];
      const float psi = atan2f(M[0][1] - M[1][0], M[0][0] + M[1][1]);
      const float step = 6.283185307179586f / (float)n_psi;
      const int base = (int)floorf(psi / step - 0.5f * (float)(n_psi_c - 1) + 0.5f);
      for (int c = 0; c < n_psi_c; ++c) {
        int m = (base + c) % n_psi;
        m += (m < 0) ? n_psi : 0;
        cand[(size_t)p * L + q * n_psi_c + c] = d * n_psi + m;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static unsigned pcdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

hipError_t pose_prep(const float *Y, const float *Z, const float *table, int P, int D, int F8,
                     unsigned short *zb, unsigned short *w, float *yy, hipStream_t st) {
  hipLaunchKernelGGL(k_pose_zpad, dim3(P), dim3(256), 0, st, Z, D, zb);
  hipLaunchKernelGGL(k_pose_weights, dim3(P), dim3(256), 0, st, Y, table, D, F8, w, yy);
  return hipGetLastError();
}

hipError_t pose_shifts(const unsigned short *zb, int P, int D, int r, unsigned short *zs,
                       hipStream_t st) {
  const int S = (2 * r + 1) * (2 * r + 1);
  hipLaunchKernelGGL(k_pose_shifts, dim3(P, S), dim3(256), 0, st, zb, D, r, zs);
  return hipGetLastError();
}

hipError_t pose_refine_z(const PoseRefineArgs &a, int P, hipStream_t st) {
  // one block per particle and 16 candidates, its four waves splitting the K
  // range: the gathered rows are the traffic, and four independent streams
  // per block keep more of them in flight
  const size_t lds = pose_refine_z_lds(a.D, a.F8);
  if (a.D % 32 == 0)
    hipLaunchKernelGGL((k_pose_refine_z<16, 4, true>), dim3(P, pcdiv(a.L, 16)), dim3(256), lds, st, a);
  else
    hipLaunchKernelGGL((k_pose_refine_z<16, 4, false>), dim3(P, pcdiv(a.L, 16)), dim3(256), lds, st, a);
  return hipGetLastError();
}

hipError_t rows_to_bf16(const float *src, int64_t rows, int len, unsigned short *dst, int64_t ld,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_rows_to_bf16, dim3(pcdiv(rows * len, 256)), dim3(256), 0, st, src, rows,
                     len, dst, ld);
  return hipGetLastError();
}

hipError_t fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u64, dim3(pcdiv(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t fill_u16(unsigned short *p, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u16, dim3(pcdiv(n, 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t pose_decode(const unsigned long long *best, int P, int S, int *rot_idx, int *shift_idx,
                       float *score, const float *bank_rot, float *rot_out, hipStream_t st) {
  hipLaunchKernelGGL(k_pose_decode, dim3(pcdiv(P, 256)), dim3(256), 0, st, best, P, S, rot_idx,
                     shift_idx, score, bank_rot, rot_out);
  return hipGetLastError();
}

hipError_t pose_confidence(const unsigned short *bank, int64_t ldb, int64_t boff, int64_t K,
                           const unsigned short *w, int F8, int D, const float *yy,
                           const int *rot_idx, const float *score, int P, float *z, float *sig,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_pose_confidence, dim3(P), dim3(256), 0, st, bank, ldb, boff, K, w, F8, D, yy,
                     rot_idx, score, z, sig);
  return hipGetLastError();
}

hipError_t pose_gemm_store(const PoseGemmArgs &a, hipStream_t st) {
  const unsigned tiles = pcdiv(a.M, 128) * pcdiv(a.N, 128);
  hipLaunchKernelGGL((k_pose_gemm<128, 128, 2, kPoseStore, 32>), dim3(tiles), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t pose_gemm_score(const PoseGemmArgs &a, hipStream_t st) {
  const unsigned tiles = pcdiv(a.M, 128) * pcdiv(a.N, 128);
  hipLaunchKernelGGL((k_pose_gemm<128, 128, 2, kPoseScore, 32>), dim3(tiles), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t pose_gemm_refine(const PoseGemmArgs &a, int P, hipStream_t st) {
  hipLaunchKernelGGL((k_pose_gemm<32, 64, 1, kPoseRefine, 128>), dim3(P, pcdiv(a.N, 64)), dim3(256), 0,
                     st, a);
  return hipGetLastError();
}

hipError_t pose_candidates(const float *prop, int P, const float *bank_rot, int ndir, int n_psi,
                           int n_dir, int n_psi_c, int *cand, hipStream_t st) {
  hipLaunchKernelGGL(k_pose_candidates, dim3(pcdiv(P, 4)), dim3(256), (size_t)ndir * 12, st, prop,
                     P, bank_rot, ndir, n_psi, n_dir, n_psi_c, cand);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Synthetic particle noise: images[b] += sigma_b * N(0, 1) with
// sigma_b^2 = var(images[b]) / 10^(snr_db / 10) (white Gaussian noise at the
// given per-image SNR).  Normals come from Philox4x32-10 (Salmon et al.,
// SC'11) keyed by `seed`, counter (image index + offset, pixel / 4, 0, 0),
// turned into normals by the Box-Muller transform.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const unsigned lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const unsigned lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

__global__ void __launch_bounds__(256)
k_add_noise(float *img, int npx, float snr_db, unsigned long long seed, long long offset) {
  const int b = blockIdx.x;
  float *x = img + (size_t)b * npx;
  double s = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < npx; i += 256) {
    const double v = x[i];
    s += v;
    s2 += v * v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_xor(s, o, 64);
    s2 += __shfl_xor(s2, o, 64);
  }
  __shared__ double red[2][4];
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s;
    red[1][threadIdx.x >> 6] = s2;
  }
  __syncthreads();
  const double m = (red[0][0] + red[0][1] + red[0][2] + red[0][3]) / npx;
  const double var = (red[1][0] + red[1][1] + red[1][2] + red[1][3]) / npx - m * m;
  const float sigma = (float)sqrt(fmax(var, 0.0) / pow(10.0, 0.1 * (double)snr_db));
  const unsigned long long img_id = (unsigned long long)((long long)b + offset);
  const uint2 key = make_uint2((unsigned)seed, (unsigned)(seed >> 32));
  for (int q = threadIdx.x; q * 4 < npx; q += 256) {
    const uint4 r = philox4x32_10(make_uint4((unsigned)img_id, (unsigned)(img_id >> 32), (unsigned)q, 0u), key);
    const float u1 = ((float)r.x + 1.0f) * 2.3283064365386963e-10f;  // (0, 1]
    const float u2 = (float)r.y * 2.3283064365386963e-10f;
    const float u3 = ((float)r.z + 1.0f) * 2.3283064365386963e-10f;
    const float u4 = (float)r.w * 2.3283064365386963e-10f;
    const float ra = sqrtf(-2.f * logf(fminf(u1, 1.f))), rb = sqrtf(-2.f * logf(fminf(u3, 1.f)));
    float sa, ca, sb, cb;
    sincosf(6.283185307179586f * u2, &sa, &ca);
    sincosf(6.283185307179586f * u4, &sb, &cb);
    const float z[4] = {ra * ca, ra * sa, rb * cb, rb * sb};
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (q * 4 + e < npx) x[q * 4 + e] += sigma * z[e];
  }
}

hipError_t add_noise(float *img, int B, int npx, float snr_db, unsigned long long seed,
                     long long offset, hipStream_t st) {
  hipLaunchKernelGGL(k_add_noise, dim3(B), dim3(256), 0, st, img, npx, snr_db, seed, offset);
  return hipGetLastError();
}

}  // namespace cs
