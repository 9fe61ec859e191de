// Particle preparation for pose scoring at D = 128, one particle per block,
// in one pass over HBM: the CTF matched filter Z = F^-1(H^ . F(Y))
// (App. A.2, Eq. 14), -2 Z as bfloat16 rows with 8 wrapped columns on each
// side, the energy weights w_f H^2 / D^2 of the Parseval sum (bfloat16) and
// ||Y||^2 (the terms of the squared error of Sec. 3.3.5 that do not depend
// on the pose), and optionally the pose network's input: Z standardised per
// image, its mean and variance taken from the spectrum (Parseval).
//
// The half spectrum (128 rows x 64 complex, row stride 65 so that column
// accesses spread over the LDS banks) stays in LDS for the whole 2-D
// transform, CTF multiply and inverse transform.  Every 128-point transform
// belongs to 8 lanes of one wave, 16 complex values per lane, as
// 128 = 16 x 8 Cooley-Tukey: a 16-point DFT in registers over stride-8
// elements, a twiddle w128^(n2 k1), an exchange through the transform's own
// 128 LDS slots, and two 8-point DFTs per lane; the inverse runs the same
// steps backwards.  An exchange needs a wave-level fence only: a wave's LDS
// operations complete in order, and no other wave touches those slots.
//   rows:    rows (2j, 2j+1) as one complex transform, split into the two
//            half spectra; the real kx = 0 and kx = 64 values of a row share
//            column 0 of the spectrum as (re, im) = (X[0], X[64])
//   columns: 63 ordinary columns, plus column 0 carrying the kx = 0 and
//            kx = 64 columns as one complex transform, separated by the
//            Hermitian split before the CTF multiply and packed again after
//   rows:    inverse, two rows per transform
// The CTF values (H^ / D^2, FP64 phase) are computed where they are used;
// no table goes through HBM.
#include "cs_ctf_dev.hpp"
#include "cs_pose.hpp"

namespace cs {
namespace {

constexpr int kN = 128;   // transform length (the particle side)
constexpr int kRS = 65;   // spectrum row stride in complex values
constexpr int kZW = kN + 16;  // padded row of -2 Z

__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 c_mulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// times exp(-i pi/2) = -i (forward) or exp(+i pi/2) = i (inverse)
template <bool INV>
__device__ __forceinline__ float2 c_rot(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// exp(-+ 2 pi i m / 16) for a compile-time m (folded after unrolling)
__device__ __forceinline__ constexpr float cos16(int m) {
  constexpr float c1 = 0.92387953251128674f, c2 = 0.70710678118654752f, c3 = 0.38268343236508978f;
  switch (m & 15) {
    case 0: return 1.f;   case 1: return c1;   case 2: return c2;   case 3: return c3;
    case 4: return 0.f;   case 5: return -c3;  case 6: return -c2;  case 7: return -c1;
    case 8: return -1.f;  case 9: return -c1;  case 10: return -c2; case 11: return -c3;
    case 12: return 0.f;  case 13: return c3;  case 14: return c2;  default: return c1;
  }
}
__device__ __forceinline__ constexpr float sin16(int m) { return cos16(m - 4); }
template <bool INV>
__device__ __forceinline__ float2 w16(int m) {
  return make_float2(cos16(m), INV ? sin16(m) : -sin16(m));
}

template <bool INV>
__device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3) {
  const float2 s02 = c_add(a0, a2), d02 = c_sub(a0, a2);
  const float2 s13 = c_add(a1, a3), d13 = c_rot<INV>(c_sub(a1, a3));
  a0 = c_add(s02, s13);
  a2 = c_sub(s02, s13);
  a1 = c_add(d02, d13);
  a3 = c_sub(d02, d13);
}

// In-place 16-point DFT, natural order in and out (16 = 4 x 4).
template <bool INV>
__device__ __forceinline__ void dft16(float2 (&v)[16]) {
#pragma unroll
  for (int b = 0; b < 4; ++b) dft4<INV>(v[b], v[4 + b], v[8 + b], v[12 + b]);
#pragma unroll
  for (int b = 1; b < 4; ++b)
#pragma unroll
    for (int c = 1; c < 4; ++c) v[4 * c + b] = c_mul(v[4 * c + b], w16<INV>(b * c));
#pragma unroll
  for (int c = 0; c < 4; ++c) dft4<INV>(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
  float2 t[16];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int d = 0; d < 4; ++d) t[c + 4 * d] = v[4 * c + d];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = t[k];
}

// In-place 8-point DFT, natural order in and out (8 = 2 x 4).
template <bool INV>
__device__ __forceinline__ void dft8(float2 (&v)[8]) {
  dft4<INV>(v[0], v[2], v[4], v[6]);
  dft4<INV>(v[1], v[3], v[5], v[7]);
#pragma unroll
  for (int c = 1; c < 4; ++c) v[2 * c + 1] = c_mul(v[2 * c + 1], w16<INV>(2 * c));
  float2 t[8];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    t[c] = c_add(v[2 * c], v[2 * c + 1]);
    t[c + 4] = c_sub(v[2 * c], v[2 * c + 1]);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = t[k];
}

// Orders the LDS accesses of one wave (no other wave shares the slots).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The 128 slots of one transform: a row pair (two spectrum rows) or a column.
// operator[] is the exchange layout: slot s is stored at s ^ ((s >> 4) & 7),
// so that the lanes of an exchange (16 slots apart) hit different banks;
// nat() is the spectrum's own order.
struct Slots {
  float2 *base;
  bool column;
  __device__ __forceinline__ float2 &nat(int s) const {
    return column ? base[s * kRS] : base[(s >> 6) * kRS + (s & 63)];
  }
  __device__ __forceinline__ float2 &operator[](int s) const { return nat(s ^ ((s >> 4) & 7)); }
};

// Forward transform.  In: lane q holds v[n1] = x[8 n1 + q].  Out: u[e][k2] =
// X[k1 + 16 k2] with k1 = 2 q + e.
__device__ __forceinline__ void fwd128(float2 (&v)[16], float2 (&u)[2][8], const Slots &sl,
                                       const float2 *twl, int q) {
  dft16<false>(v);
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) v[k1] = c_mul(v[k1], twl[q * k1]);
  wave_sync();
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) sl[k1 * 8 + q] = v[k1];
  wave_sync();
#pragma unroll
  for (int e = 0; e < 2; ++e)
#pragma unroll
    for (int n2 = 0; n2 < 8; ++n2) u[e][n2] = sl[(2 * q + e) * 8 + n2];
  wave_sync();
  dft8<false>(u[0]);
  dft8<false>(u[1]);
}

// Inverse transform (no 1/N).  In: u[e][k2] = X[k1 + 16 k2], k1 = 2 q + e.
// Out: v[n1] = x[8 n1 + q].
__device__ __forceinline__ void inv128(float2 (&u)[2][8], float2 (&v)[16], const Slots &sl,
                                       const float2 *twl, int q) {
  dft8<true>(u[0]);
  dft8<true>(u[1]);
#pragma unroll
  for (int e = 0; e < 2; ++e)
#pragma unroll
    for (int n2 = 1; n2 < 8; ++n2) u[e][n2] = c_mulc(u[e][n2], twl[n2 * (2 * q + e)]);
  wave_sync();
#pragma unroll
  for (int e = 0; e < 2; ++e)
#pragma unroll
    for (int n2 = 0; n2 < 8; ++n2) sl[(2 * q + e) * 8 + n2] = u[e][n2];
  wave_sync();
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) v[k1] = sl[k1 * 8 + q];
  wave_sync();
  dft16<true>(v);
}

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// H^ / D^2 on the DFT grid, the renderer's CTF (Eq. 13 with the grid and
// Nyquist conventions of its Fourier pass) with the phase written as a
// polynomial in (sx, sy): chi / 2pi = a s^2 + bc (sx^2 - sy^2) + bs sx sy
// - c4 s^4 - ph / 2pi, which is df(angle) s^2 without the division by s^2.
// FP64 phase, reduced to one turn in FP64, then one FP32 sincos.
struct PrepCtf {
  int enabled;
  double a, bc, bs, c4, ph, amp_s, amp_c, bq, inv;

  __device__ void init(const CtfDev &c, int p, float pixel) {
    enabled = c.enabled;
    inv = 1.0 / ((double)kN * (double)pixel);
    if (!enabled) return;
    const CtfParticle q = ctf_particle(c, p);
    a = 0.25 * c.lam * (q.du + q.dv);
    bc = 0.25 * c.lam * (q.du - q.dv) * q.c2a;
    bs = 0.5 * c.lam * (q.du - q.dv) * q.s2a;
    c4 = 0.25 * c.cs * c.lam * c.lam * c.lam;
    ph = q.ph * (0.5 / M_PI);
    amp_s = sqrt(1.0 - c.w * c.w);
    amp_c = c.w;
    bq = -0.25 * c.bfactor;
  }
  __device__ __forceinline__ double at(double sx, double sy) const {
    const double x2 = sx * sx, y2 = sy * sy, s2 = x2 + y2;
    const double t = a * s2 + bc * (x2 - y2) + bs * (sx * sy) - c4 * s2 * s2 - ph;
    const float red = (float)((t - rint(t)) * (2.0 * M_PI));
    float sn, cs;
    sincosf(red, &sn, &cs);
    double h = -(amp_s * (double)sn + amp_c * (double)cs);
    if (bq != 0.0) h *= exp(bq * s2);
    return h;
  }
  __device__ float h(int ky, int kx) const {
    const float norm = 1.f / ((float)kN * (float)kN);
    if (!enabled) return norm;
    const int fkx = (kx < kN / 2) ? kx : kx - kN;
    const int fky = (ky < kN / 2) ? ky : ky - kN;
    const double sx = fkx * inv, sy = -fky * inv;
    double v = at(sx, sy);
    if (kx == kN / 2 || ky == kN / 2)
      v = 0.5 * (v + at((kx == kN / 2) ? -sx : sx, (ky == kN / 2) ? -sy : sy));
    return (float)v * norm;
  }
};

__device__ __forceinline__ unsigned short energy_weight(float h, int kx) {
  const float wf = (kx == 0 || kx == kN / 2) ? 1.f : 2.f;
  return bf16_rne(wf * h * h * ((float)kN * (float)kN));
}

}  // namespace

__global__ void __launch_bounds__(256)
k_pose_prep128(const float *Y, const float2 *tw, float pixel, CtfDev ctf, int F8, float *Z,
               unsigned short *zs, unsigned short *zb, unsigned short *w, float *yy) {
  __shared__ float2 sp[kN * kRS];
  __shared__ float2 twl[kN];
  __shared__ double red[4], pred[4], dcs;
  const int p = blockIdx.x, tid = threadIdx.x;
  const int wv = tid >> 6, g = (tid >> 3) & 7, q = tid & 7;
  if (tid < kN) twl[tid] = tw[tid];

  // image -> LDS rows (stride 2 kRS floats), ||Y||^2 in FP64
  const float4 *y4 = (const float4 *)(Y + (size_t)p * kN * kN);
  float *spf = (float *)sp;
  double acc = 0.0;
#pragma unroll 4
  for (int i = tid; i < kN * kN / 4; i += 256) {
    const float4 v = y4[i];
    acc += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
    float2 *d = (float2 *)(spf + (i >> 5) * (2 * kRS) + (i & 31) * 4);
    d[0] = make_float2(v.x, v.y);
    d[1] = make_float2(v.z, v.w);
  }
  __syncthreads();

  // forward rows, two real rows per complex transform
  for (int rnd = 0; rnd < 2; ++rnd) {
    const int j = rnd * 32 + wv * 8 + g;
    float2 *reg = sp + 2 * j * kRS;
    const Slots sl{reg, false};
    const float *r0 = (const float *)reg, *r1 = (const float *)(reg + kRS);
    float2 v[16], u[2][8];
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) v[n1] = make_float2(r0[8 * n1 + q], r1[8 * n1 + q]);
    fwd128(v, u, sl, twl, q);
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) sl[2 * q + e + 16 * k2] = u[e][k2];
    wave_sync();
    // split: A = (X[k] + conj X[-k]) / 2 (row 2j), B = (X[k] - conj X[-k]) / 2i
    float2 A[8], Bv[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int k = 8 * q + m;
      const float2 X = sl[k], Xm = sl[(kN - k) & (kN - 1)];
      A[m] = make_float2(0.5f * (X.x + Xm.x), 0.5f * (X.y - Xm.y));
      Bv[m] = make_float2(0.5f * (X.y + Xm.y), -0.5f * (X.x - Xm.x));
    }
    if (q == 0) {
      const float2 X0 = sl[0], X64 = sl[kN / 2];
      A[0] = make_float2(X0.x, X64.x);
      Bv[0] = make_float2(X0.y, X64.y);
    }
    wave_sync();
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      reg[8 * q + m] = A[m];
      reg[kRS + 8 * q + m] = Bv[m];
    }
  }
  __syncthreads();

  // columns: forward, CTF multiply (energy weights on the way), inverse
  // sum over the full spectrum of |Z^|^2 (half spectrum, kx = 1..63 twice)
  // and the DC value: the mean and variance of Z by Parseval
  double pw = 0.0;
  PrepCtf H;
  H.init(ctf, p, pixel);
  unsigned short *wp = w + (size_t)p * F8;
  for (int rnd = 0; rnd < 2; ++rnd) {
    const int kx = 8 * g + wv + 4 * rnd;
    const Slots sl{sp + kx, true};
    float2 v[16], u[2][8];
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) v[n1] = sl.nat(8 * n1 + q);
    fwd128(v, u, sl, twl, q);
    // spectrum column in natural order into its slots; each lane then
    // filters slots that no other lane touches (the CTF code stays rolled)
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) sl[2 * q + e + 16 * k2] = u[e][k2];
    wave_sync();
    if (kx != 0) {
#pragma unroll 1
      for (int i = 0; i < 16; ++i) {
        const int ky = q + 8 * i;
        const float h = H.h(ky, kx);
        const float2 X = sl[ky];
        const float2 Xh = make_float2(X.x * h, X.y * h);
        sl[ky] = Xh;
        pw += 2.0 * ((double)Xh.x * Xh.x + (double)Xh.y * Xh.y);
        wp[ky * (kN / 2 + 1) + kx] = energy_weight(h, kx);
      }
    } else {
      // column 0 = (kx = 0) + i (kx = 64): split, filter each, pack again;
      // a lane owns the pair (ky, -ky)
#pragma unroll 1
      for (int i = 0; i < 9; ++i) {
        const int ky = (i < 8) ? q + 8 * i : kN / 2;
        if (i == 8 && q != 0) break;
        const int km = (kN - ky) & (kN - 1);
        const float2 X = sl[ky], Xm = sl[km];
        const float h0 = H.h(ky, 0), h64 = H.h(ky, kN / 2);
        // A = (X[k] + conj X[-k]) / 2, B = (X[k] - conj X[-k]) / 2i at k = ky;
        // at -ky they are the conjugates (H^ is even in ky)
        const float2 A = make_float2(0.5f * (X.x + Xm.x) * h0, 0.5f * (X.y - Xm.y) * h0);
        const float2 Bv = make_float2(0.5f * (X.y + Xm.y) * h64, -0.5f * (X.x - Xm.x) * h64);
        sl[ky] = make_float2(A.x - Bv.y, A.y + Bv.x);
        sl[km] = make_float2(A.x + Bv.y, -A.y + Bv.x);
        pw += (km != ky ? 2.0 : 1.0) *
              ((double)A.x * A.x + (double)A.y * A.y + (double)Bv.x * Bv.x + (double)Bv.y * Bv.y);
        if (ky == 0) dcs = A.x;
        wp[ky * (kN / 2 + 1)] = energy_weight(h0, 0);
        wp[ky * (kN / 2 + 1) + kN / 2] = energy_weight(h64, kN / 2);
        if (km != ky) {
          wp[km * (kN / 2 + 1)] = energy_weight(h0, 0);
          wp[km * (kN / 2 + 1) + kN / 2] = energy_weight(h64, kN / 2);
        }
      }
    }
    wave_sync();
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) u[e][k2] = sl[2 * q + e + 16 * k2];
    wave_sync();
    inv128(u, v, sl, twl, q);
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) sl.nat(8 * n1 + q) = v[n1];
  }
  for (int f = kN * (kN / 2 + 1) + tid; f < F8; f += 256) wp[f] = 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) pw += __shfl_xor(pw, o, 64);
  if ((tid & 63) == 0) pred[wv] = pw;
  __syncthreads();
  // standardisation of Z (as the network's input step): mean = Z^(0, 0),
  // variance = sum |Z^|^2 - mean^2
  const double zm = dcs, zv = (pred[0] + pred[1] + pred[2] + pred[3]) - zm * zm;
  const float zmf = (float)zm, zinv = zv > 0.0 ? (float)(1.0 / sqrt(zv)) : 1.f;
  unsigned short *sp0 = zs ? zs + (size_t)p * kN * kN : nullptr;

  // inverse rows: C[k] = A[k] + i B[k] from the spectrum rows (2j, 2j+1)
  float *zp = Z ? Z + (size_t)p * kN * kN : nullptr;
  unsigned short *bp = zb + (size_t)p * kN * kZW;
  for (int rnd = 0; rnd < 2; ++rnd) {
    const int j = rnd * 32 + wv * 8 + g;
    float2 *reg = sp + 2 * j * kRS;
    const Slots sl{reg, false};
    float2 v[16], u[2][8];
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) {
        const int k = 2 * q + e + 16 * k2;
        float2 A, Bv;
        if (k == 0) {
          A = make_float2(reg[0].x, 0.f);
          Bv = make_float2(reg[kRS].x, 0.f);
        } else if (k == kN / 2) {
          A = make_float2(reg[0].y, 0.f);
          Bv = make_float2(reg[kRS].y, 0.f);
        } else if (k < kN / 2) {
          A = reg[k];
          Bv = reg[kRS + k];
        } else {
          A = reg[kN - k];
          Bv = reg[kRS + kN - k];
          A.y = -A.y;
          Bv.y = -Bv.y;
        }
        u[e][k2] = make_float2(A.x - Bv.y, A.y + Bv.x);
      }
    wave_sync();
    inv128(u, v, sl, twl, q);
    unsigned short *o0 = bp + (size_t)(2 * j) * kZW, *o1 = o0 + kZW;
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) {
      const int n = 8 * n1 + q;
      const float2 z = v[n1];
      if (zp) {
        zp[(2 * j) * kN + n] = z.x;
        zp[(2 * j + 1) * kN + n] = z.y;
      }
      if (sp0) {
        sp0[(2 * j) * kN + n] = bf16_rne((z.x - zmf) * zinv);
        sp0[(2 * j + 1) * kN + n] = bf16_rne((z.y - zmf) * zinv);
      }
      const unsigned short b0 = bf16_rne(-2.f * z.x), b1 = bf16_rne(-2.f * z.y);
      o0[n + 8] = b0;
      o1[n + 8] = b1;
      if (n1 == 15) { o0[n - 120] = b0; o1[n - 120] = b1; }
      if (n1 == 0) { o0[n + 136] = b0; o1[n + 136] = b1; }
    }
  }

#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((tid & 63) == 0) red[wv] = acc;
  __syncthreads();
  if (tid == 0) yy[p] = (float)(red[0] + red[1] + red[2] + red[3]);
}

hipError_t pose_prep128(const float *Y, const float2 *tw, float pixel, const CtfDev &ctf, int P,
                        int F8, float *Z, unsigned short *zs, unsigned short *zb, unsigned short *w,
                        float *yy, hipStream_t st) {
  hipLaunchKernelGGL(k_pose_prep128, dim3(P), dim3(256), 0, st, Y, tw, pixel, ctf, F8, Z, zs, zb,
                     w, yy);
  return hipGetLastError();
}

}  // namespace cs
