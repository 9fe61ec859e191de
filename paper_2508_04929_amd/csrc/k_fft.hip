// Fourier-space CTF application, loss and adjoint (App. A.2, Eq. 14; Sec. 3.3.5).
//
// X = F^-1(H^ . F(Q)) is computed as
//   rows:     real FFT of every row (two rows packed as one complex FFT)
//   columns:  for each of the D/2+1 half-spectrum columns: FFT over rows,
//             multiply by H^ (real, evaluated on the fly with an FP64 phase)
//             and the 1/D^2 normalisation, inverse FFT over rows
//   rows:     inverse real FFT of every row (two rows packed again)
// Every transform is a mixed-radix (4, 2, 3) Stockham FFT in LDS with
// twiddles from an FP64-accurate table (k_twiddles).  Because H^ is real and
// even, the same column pass is its own adjoint, so the loss gradient
// G_Q = F^-1(H^ . F(G_X)) reuses the three passes; the row pass between the
// two applications fuses the inverse rows of X, the residual X - Y, the
// squared-error partial sums and the forward rows of G_X.
#include "cs_ctf_dev.hpp"

namespace cs {

// Twiddle table of one transform length: tw[k] = exp(-2 pi i k / L),
// evaluated in FP64 and rounded once to FP32.
__global__ void __launch_bounds__(256) k_twiddles(int L, float2 *tw) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= L) return;
  double sn, cn;
  sincospi(2.0 * (double)k / (double)L, &sn, &cn);
  tw[k] = make_float2((float)cn, (float)-sn);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One Stockham transform of length P.L by a team of `ts` threads (thread
// index t within the team).  x holds the input, y is scratch; returns the
// buffer that holds the result.  Every thread of the block must call it
// (it synchronises the block after every stage).
__device__ float2 *fft_team(float2 *x, float2 *y, const FftPlan &P, const float2 *tw, int t,
                            int ts, bool inverse) {
  const int L = P.L;
  int Ns = 1;
  const float sg = inverse ? 1.f : -1.f;  // sign of the exponent
  for (int st = 0; st < P.nst; ++st) {
    const int R = P.radix[st];
    const int LR = L / R;
    const int tws = L / (Ns * R);
    for (int j = t; j < LR; j += ts) {
      const int k = j % Ns;
      const int base = (j / Ns) * Ns * R + k;
      if (R == 4) {
        float2 v0 = x[j], v1 = x[j + LR], v2 = x[j + 2 * LR], v3 = x[j + 3 * LR];
        if (k) {
          float2 w1 = tw[k * tws], w2 = tw[2 * k * tws], w3 = tw[3 * k * tws];
          if (inverse) { w1.y = -w1.y; w2.y = -w2.y; w3.y = -w3.y; }
          v1 = cmul(v1, w1); v2 = cmul(v2, w2); v3 = cmul(v3, w3);
        }
        const float2 a0 = make_float2(v0.x + v2.x, v0.y + v2.y);
        const float2 a1 = make_float2(v0.x - v2.x, v0.y - v2.y);
        const float2 a2 = make_float2(v1.x + v3.x, v1.y + v3.y);
        const float2 a3 = make_float2(v1.x - v3.x, v1.y - v3.y);
        // y1 = a1 + sg*i*a3, y3 = a1 - sg*i*a3
        y[base] = make_float2(a0.x + a2.x, a0.y + a2.y);
        y[base + Ns] = make_float2(a1.x - sg * a3.y, a1.y + sg * a3.x);
        y[base + 2 * Ns] = make_float2(a0.x - a2.x, a0.y - a2.y);
        y[base + 3 * Ns] = make_float2(a1.x + sg * a3.y, a1.y - sg * a3.x);
      } else if (R == 2) {
        float2 v0 = x[j], v1 = x[j + LR];
        if (k) {
          float2 w1 = tw[k * tws];
          if (inverse) w1.y = -w1.y;
          v1 = cmul(v1, w1);
        }
        y[base] = make_float2(v0.x + v1.x, v0.y + v1.y);
        y[base + Ns] = make_float2(v0.x - v1.x, v0.y - v1.y);
      } else {  // R == 3
        float2 v0 = x[j], v1 = x[j + LR], v2 = x[j + 2 * LR];
        if (k) {
          float2 w1 = tw[k * tws], w2 = tw[2 * k * tws];
          if (inverse) { w1.y = -w1.y; w2.y = -w2.y; }
          v1 = cmul(v1, w1); v2 = cmul(v2, w2);
        }
        const float c3 = 0.86602540378443864676f;  // sqrt(3)/2
        const float2 t1 = make_float2(v1.x + v2.x, v1.y + v2.y);
        const float2 t2 = make_float2(v1.x - v2.x, v1.y - v2.y);
        const float2 m = make_float2(v0.x - 0.5f * t1.x, v0.y - 0.5f * t1.y);
        // y1 = m + sg*i*c3*t2, y2 = m - sg*i*c3*t2
        y[base] = make_float2(v0.x + t1.x, v0.y + t1.y);
        y[base + Ns] = make_float2(m.x - sg * c3 * t2.y, m.y + sg * c3 * t2.x);
        y[base + 2 * Ns] = make_float2(m.x + sg * c3 * t2.y, m.y - sg * c3 * t2.x);
      }
    }
    __syncthreads();
    float2 *tmp = x; x = y; y = tmp;
    Ns *= R;
  }
  return x;
}

// Row kernels: one team of 64 threads per row pair, blockDim.x / 64 teams
// per block (the host picks fewer for small batches; each pair's transform
// is the same either way).

// ---------------------------------------------------------------------------
// Forward row pass: spec[b][r][0..D/2] = rFFT(src[b][r][:]) for every row.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void split_store(const float2 *res, int L, int t, float2 *spec_a,
                                            float2 *spec_b, bool valid) {
  for (int k = t; k <= L / 2; k += 64) {
    const float2 Z = res[k];
    const float2 Zm = res[(L - k) % L];
    // A = (Z + conj(Zm)) / 2,  B = (Z - conj(Zm)) / (2i)
    const float dx = Z.x - Zm.x, dy = Z.y + Zm.y;
    if (valid) {
      spec_a[k] = make_float2(0.5f * (Z.x + Zm.x), 0.5f * (Z.y - Zm.y));
      spec_b[k] = make_float2(0.5f * dy, -0.5f * dx);
    }
  }
}

__global__ void __launch_bounds__(256)
k_fft_rows_fwd(const float *src, FftPlan P, const float2 *tw, int B, float2 *spec) {
  extern __shared__ float2 lds[];
  const int L = P.L, Dh = L / 2 + 1;
  const int teams = blockDim.x >> 6, team = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int pr = blockIdx.x * teams + team;  // row pair
  const int b = blockIdx.y;
  const bool valid = pr < L / 2;
  float2 *x = lds + team * 2 * L, *y = x + L;
  float2 *twl = lds + teams * 2 * L;
  for (int k = threadIdx.x; k < L; k += blockDim.x) twl[k] = tw[k];
  const float *ra = src + ((size_t)b * L + 2 * pr) * L;
  for (int j = t; j < L; j += 64) x[j] = valid ? make_float2(ra[j], ra[L + j]) : make_float2(0.f, 0.f);
  __syncthreads();
  const float2 *res = fft_team(x, y, P, twl, t, 64, false);
  float2 *sa = spec + ((size_t)b * L + 2 * pr) * Dh;
  split_store(res, L, t, sa, sa + Dh, valid);
}

// H^ / D^2 on the half-spectrum grid [B][D][D/2+1], once per call.
__global__ void __launch_bounds__(256)
k_ctf_table(int L, float pixel, CtfDev ctf, int B, float *table) {
  // grid rows walk the images (b = blockIdx.y, blockIdx.y + gridDim.y, ...);
  // a thread fills entries blockIdx.x * 256 + threadIdx.x + k * gridDim.x *
  // 256 of an image with its constants (defocus, astigmatism angle, phase,
  // frequency step) evaluated once
  const int Dh = L / 2 + 1;
  const int per = L * Dh;
  const float norm = 1.f / ((float)L * (float)L);
  const CtfGrid g = ctf_grid(L, pixel, ctf);
  for (int b = blockIdx.y; b < B; b += gridDim.y) {
    float *row = table + (size_t)b * per;
    if (!ctf.enabled) {
      for (int r = blockIdx.x * 256 + threadIdx.x; r < per; r += gridDim.x * 256) row[r] = norm;
      continue;
    }
    const CtfParticle q = ctf_particle(ctf, b);
    for (int r = blockIdx.x * 256 + threadIdx.x; r < per; r += gridDim.x * 256) {
      const int ky = r / Dh, kx = r % Dh;
      row[r] = ctf_value(ky, kx, L, g, ctf, q) * norm;
    }
  }
}

// ---------------------------------------------------------------------------
// Column pass: for cpw adjacent half-spectrum columns per block, FFT over
// rows, times a multiplier mul(ky, kx, z) of image blockIdx.y, inverse FFT
// over rows, in place.
// ---------------------------------------------------------------------------
// Image and column group of this block: the grid is (column groups, images)
// and the XCD-aware order keeps an image's adjacent column groups (whose
// rows share cache lines) on one XCD.
__device__ __forceinline__ void cols_block(int &b, int &group) {
  const int j = xcd_work(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  b = j / gridDim.x;
  group = j % gridDim.x;
}

template <class Mul>
__device__ __forceinline__ void fft_cols_apply(float2 *spec, const FftPlan &P, const float2 *tw,
                                               int cpw, int b, int group, const Mul &mul) {
  extern __shared__ float2 lds[];
  const int L = P.L, Dh = L / 2 + 1;
  const int kx0 = group * cpw;
  const int ts = 256 / cpw;
  const int team = threadIdx.x / ts, t = threadIdx.x % ts;
  float2 *img = spec + (size_t)b * L * Dh;
  float2 *twl = lds + (size_t)cpw * 2 * L;
  for (int k = threadIdx.x; k < L; k += 256) twl[k] = tw[k];
  // coalesced load: consecutive threads take consecutive columns of a row
  for (int q = threadIdx.x; q < cpw * L; q += 256) {
    const int c = q % cpw, r = q / cpw;
    const int kx = kx0 + c;
    lds[c * 2 * L + r] = (kx < Dh) ? img[(size_t)r * Dh + kx] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  float2 *x = lds + team * 2 * L, *y = x + L;
  float2 *res = fft_team(x, y, P, twl, t, ts, false);
  const int kx = kx0 + team;
  for (int ky = t; ky < L; ky += ts) res[ky] = (kx < Dh) ? mul(ky, kx, res[ky]) : make_float2(0.f, 0.f);
  __syncthreads();
  float2 *other = (res == x) ? y : x;
  float2 *out = fft_team(res, other, P, twl, t, ts, true);
  // every team's result sits in the same half of its buffer pair
  const int oofs = (int)(out - (lds + team * 2 * L));
  for (int q = threadIdx.x; q < cpw * L; q += 256) {
    const int c = q % cpw, r = q / cpw;
    const int kc = kx0 + c;
    if (kc < Dh) img[(size_t)r * Dh + kc] = lds[c * 2 * L + oofs + r];
  }
}

// times the table H^ / D^2 (Eq. 14)
__global__ void __launch_bounds__(256)
k_fft_cols_ctf(float2 *spec, FftPlan P, const float2 *tw, int B, int cpw, const float *table) {
  const int L = P.L, Dh = L / 2 + 1;
  int b, group;
  cols_block(b, group);
  const float *hcol = table + (size_t)b * L * Dh;
  fft_cols_apply(spec, P, tw, cpw, b, group, [&](int ky, int kx, float2 z) {
    const float h = hcol[(size_t)ky * Dh + kx];
    return make_float2(z.x * h, z.y * h);
  });
}

// Translation of image b by (a_c, a_r) = (sign t_x / p, -sign t_y / p)
// columns / rows (the row axis is y-flipped, Eq. 13): times
// exp(-2 pi i (kx a_c + ky a_r) / L) / L^2 with signed frequency indices,
// made Hermitian on the Nyquist lines of even L (the real part of the
// complex inverse transform): cos(pi a) there in place of the exponential,
// cos(pi (a_c + a_r)) at the corner.  Turns in FP64, one FP32 sincos.
__global__ void __launch_bounds__(256)
k_fft_cols_shift(float2 *spec, FftPlan P, const float2 *tw, int cpw, const float *shift,
                 float inv_pixel, float sign) {
  const int L = P.L;
  int b, group;
  cols_block(b, group);
  const double ac = (double)(sign * shift[2 * b] * inv_pixel);
  const double ar = -(double)(sign * shift[2 * b + 1] * inv_pixel);
  const bool even = (L % 2) == 0;
  const int half = L / 2;
  const float norm = 1.f / ((float)L * (float)L);
  fft_cols_apply(spec, P, tw, cpw, b, group, [&](int ky, int kx, float2 z) {
    const bool nx = even && kx == half, ny = even && ky == half;
    const int fy = ky < (L + 1) / 2 ? ky : ky - L;
    double turns;
    double amp = 1.0;
    if (nx && ny) {
      turns = 0.0;
      amp = cos(M_PI * (ac + ar));
    } else if (nx) {
      turns = -(double)fy * ar / L;
      amp = cos(M_PI * ac);
    } else if (ny) {
      turns = -(double)kx * ac / L;
      amp = cos(M_PI * ar);
    } else {
      turns = -((double)kx * ac + (double)fy * ar) / L;
    }
    const float red = (float)((turns - rint(turns)) * (2.0 * M_PI));
    float sn, cs;
    sincosf(red, &sn, &cs);
    const float m = (float)amp * norm;
    const float re = cs * m, im = sn * m;
    return make_float2(z.x * re - z.y * im, z.x * im + z.y * re);
  });
}

// Hermitian-packed inverse of two half-spectrum rows into one complex row.
__device__ __forceinline__ void pack_inverse(const float2 *sa, const float2 *sb, int L, int t,
                                             float2 *x, bool valid) {
  const int half = L / 2;
  for (int k = t; k < L; k += 64) {
    float2 A, Bv;
    if (!valid) {
      A = Bv = make_float2(0.f, 0.f);
    } else if (k <= half) {
      A = sa[k];
      Bv = sb[k];
      if (k == 0 || (k == half && (L % 2 == 0))) { A.y = 0.f; Bv.y = 0.f; }
    } else {
      A = sa[L - k];
      Bv = sb[L - k];
      A.y = -A.y;
      Bv.y = -Bv.y;
    }
    x[k] = make_float2(A.x - Bv.y, A.y + Bv.x);  // A + i B
  }
}

__global__ void __launch_bounds__(256)
k_fft_rows_inv(const float2 *spec, FftPlan P, const float2 *tw, int B, float *dst) {
  extern __shared__ float2 lds[];
  const int L = P.L, Dh = L / 2 + 1;
  const int teams = blockDim.x >> 6, team = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int pr = blockIdx.x * teams + team;
  const int b = blockIdx.y;
  const bool valid = pr < L / 2;
  float2 *x = lds + team * 2 * L, *y = x + L;
  float2 *twl = lds + teams * 2 * L;
  for (int k = threadIdx.x; k < L; k += blockDim.x) twl[k] = tw[k];
  const float2 *sa = spec + ((size_t)b * L + 2 * pr) * Dh;
  pack_inverse(sa, sa + Dh, L, t, x, valid);
  __syncthreads();
  const float2 *res = fft_team(x, y, P, twl, t, 64, true);
  if (valid) {
    float *ra = dst + ((size_t)b * L + 2 * pr) * L;
    for (int j = t; j < L; j += 64) {
      const float2 z = res[j];
      ra[j] = z.x;
      ra[L + j] = z.y;
    }
  }
}

// ---------------------------------------------------------------------------
// Fused: inverse rows of X, optional X output, residual R = X - Y, partial
// sums of R^2 per row pair, G_X = grad_scale * R and the forward rows of
// G_X written back into spec.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_fft_rows_inv_loss(float2 *spec, FftPlan P, const float2 *tw, int B, const float *obs,
                    float *images_out, float grad_scale, float *loss_part) {
  extern __shared__ float2 lds[];
  const int L = P.L, Dh = L / 2 + 1;
  const int teams = blockDim.x >> 6, team = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int pr = blockIdx.x * teams + team;
  const int b = blockIdx.y;
  const bool valid = pr < L / 2;
  float2 *x = lds + team * 2 * L, *y = x + L;
  float2 *twl = lds + teams * 2 * L;
  for (int k = threadIdx.x; k < L; k += blockDim.x) twl[k] = tw[k];
  float2 *sa = spec + ((size_t)b * L + 2 * pr) * Dh;
  pack_inverse(sa, sa + Dh, L, t, x, valid);
  __syncthreads();
  float2 *res = fft_team(x, y, P, twl, t, 64, true);
  float2 *other = (res == x) ? y : x;
  float acc = 0.f;
  const size_t row0 = ((size_t)b * L + 2 * pr) * L;
  for (int j = t; j < L; j += 64) {
    float2 g = make_float2(0.f, 0.f);
    if (valid) {
      const float2 z = res[j];
      if (images_out) {
        images_out[row0 + j] = z.x;
        images_out[row0 + L + j] = z.y;
      }
      const float ra = z.x - obs[row0 + j], rb = z.y - obs[row0 + L + j];
      acc += ra * ra + rb * rb;
      g = make_float2(grad_scale * ra, grad_scale * rb);
    }
    other[j] = g;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (t == 0 && valid) loss_part[(size_t)b * (L / 2) + pr] = acc;
  __syncthreads();
  const float2 *r2 = fft_team(other, res, P, twl, t, 64, false);
  split_store(r2, L, t, sa, sa + Dh, valid);
}

// loss[b] = scale * sum of the row-pair partials of image b (one block per
// image, FP64 sums), then loss[B] = the total in image order.
__global__ void __launch_bounds__(256)
k_loss_reduce(const float *loss_part, int B, int parts, float scale, float *loss) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int k = threadIdx.x; k < parts; k += 256) s += (double)loss_part[(size_t)b * parts + k];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float v = (float)(scale * (red[0] + red[1] + red[2] + red[3]));
    loss[b] = v;
    if (B == 1) loss[1] = v;  // the total of one image (k_loss_total is skipped)
  }
}

__global__ void __launch_bounds__(256) k_loss_total(float *loss, int B) {
  __shared__ double red[4];
  double s = 0.0;
  for (int b = threadIdx.x; b < B; b += 256) s += (double)loss[b];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) loss[B] = (float)(red[0] + red[1] + red[2] + red[3]);
}

// No-CTF residual (X = Q): loss partials per row, optional X output and
// G_Q = grad_scale (X - Y) written in place over Q.
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


// ---------------------------------------------------------------------------
// Forward transform along the middle axis of data[outer][L][inner]
// (complex, in place): cpw adjacent inner columns per block, outer index =
// blockIdx.y.  The y and z passes of the 3-D transform of a volume.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_fft_axis(float2 *data, FftPlan P, const float2 *tw, int inner, int cpw) {
  extern __shared__ float2 lds[];
  const int L = P.L;
  const int i0 = blockIdx.x * cpw;
  const int ts = 256 / cpw;
  const int team = threadIdx.x / ts, t = threadIdx.x % ts;
  float2 *base = data + (size_t)blockIdx.y * L * inner;
  float2 *twl = lds + (size_t)cpw * 2 * L;
  for (int k = threadIdx.x; k < L; k += 256) twl[k] = tw[k];
  for (int q = threadIdx.x; q < cpw * L; q += 256) {
    const int c = q % cpw, r = q / cpw;
    const int i = i0 + c;
    lds[c * 2 * L + r] = (i < inner) ? base[(size_t)r * inner + i] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  float2 *x = lds + team * 2 * L, *y = x + L;
  float2 *res = fft_team(x, y, P, twl, t, ts, false);
  const int oofs = (int)(res - (lds + team * 2 * L));
  __syncthreads();
  for (int q = threadIdx.x; q < cpw * L; q += 256) {
    const int c = q % cpw, r = q / cpw;
    const int i = i0 + c;
    if (i < inner) base[(size_t)r * inner + i] = lds[c * 2 * L + oofs + r];
  }
}

// ---------------------------------------------------------------------------
// Column pass for power spectra: for cpw adjacent half-spectrum columns per
// block, forward FFT over rows and |.|^2 stored as bfloat16 (nearest even)
// at out[b * ld + ky * (D/2+1) + kx].
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned short f2bf_rne(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__global__ void __launch_bounds__(256)
k_fft_cols_power(const float2 *spec, FftPlan P, const float2 *tw, int B, int cpw,
                 unsigned short *out, size_t ld) {
  extern __shared__ float2 lds[];
  const int L = P.L, Dh = L / 2 + 1;
  const int b = blockIdx.y;
  const int kx0 = blockIdx.x * cpw;
  const int ts = 256 / cpw;
  const int team = threadIdx.x / ts, t = threadIdx.x % ts;
  const float2 *img = spec + (size_t)b * L * Dh;
  float2 *twl = lds + (size_t)cpw * 2 * L;
  for (int k = threadIdx.x; k < L; k += 256) twl[k] = tw[k];
  for (int q = threadIdx.x; q < cpw * L; q += 256) {
    const int c = q % cpw, r = q / cpw;
    const int kx = kx0 + c;
    lds[c * 2 * L + r] = (kx < Dh) ? img[(size_t)r * Dh + kx] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  float2 *x = lds + team * 2 * L, *y = x + L;
  const float2 *res = fft_team(x, y, P, twl, t, ts, false);
  const int kx = kx0 + team;
  if (kx < Dh) {
    unsigned short *o = out + (size_t)b * ld + kx;
    for (int ky = t; ky < L; ky += ts) {
      const float2 z = res[ky];
      o[(size_t)ky * Dh] = f2bf_rne(z.x * z.x + z.y * z.y);
    }
  }
}

}  // namespace cs
