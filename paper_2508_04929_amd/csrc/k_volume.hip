// Voxelisation of the mixture and Fourier shell correlation.
//
// The reconstruction is a Gaussian mixture; the overview of Sec. 3 reads
// the final volume out by voxelising it, and Sec. 4 compares volumes by the
// Fourier shell correlation of Eq. 10 with the 0.143 threshold.
//
// Voxelisation: voxel (iz, iy, ix) sits at ((ix - c0) p, (iy - c0) p,
// (iz - c0) p) and holds sum_n A_n (2 pi)^-3/2 det(Sigma_n)^-1/2
// exp(-q_n / 2) over the Gaussians with q_n <= q_cut.  Bricks of 8^3 voxels:
// every Gaussian is listed under the bricks its q <= q_cut box touches
// (counting sort); a block evaluates one brick against its list, one wave
// per 4^3 sub-cube, each Gaussian only where a conservative bound of its
// form over the sub-cube is within the cut.  Each voxel's sum is kept as a 64-bit fixed-point integer
// (scale 2^e with the bound sum_n |w_n| < 2^61 / scale), so the result does
// not depend on the order of the list: it is reproducible bit for bit.
//
// FSC: the 3-D real DFT is the renderer's row pass (real rows along x, two
// per complex transform) over the D slices, then the same Stockham
// transform along y and along z (k_fft_axis); shell sums of
// Re(Fa conj Fb), |Fa|^2, |Fb|^2 (weight 2 off the kx = 0 and Nyquist
// planes) are again exact 64-bit fixed-point sums, scaled by Parseval's
// bound D^3 max(sum Va^2, sum Vb^2) on every shell sum.
#include "cs_volume.hpp"

namespace cs {

constexpr int kBrick = 8;

__device__ __forceinline__ int clampi(float x, int lo, int hi) {
  x = fminf(fmaxf(x, (float)lo), (float)hi);
  return (int)x;
}

// Per Gaussian: mean and weight, inverse covariance (FP64 adjugate) and the
// brick range of its q <= q_cut box; per block the sum of |w| (fixed-order
// tree, FP64) for the fixed-point scale.
__global__ void __launch_bounds__(256)
k_vox_prep(const float4 *gc, VoxGeom V, float4 *rec, int4 *box, double *wpart) {
  __shared__ double red[256];
  const int n = blockIdx.x * 256 + threadIdx.x;
  double aw = 0.0;
  if (n < V.N) {
    const float4 g0 = gc[3 * n], g1 = gc[3 * n + 1], g2 = gc[3 * n + 2];
    const double sxx = g1.x, sxy = g1.y, sxz = g1.z, syy = g1.w, syz = g2.x, szz = g2.y;
    const double cxx = syy * szz - syz * syz, cxy = sxz * syz - sxy * szz, cxz = sxy * syz - sxz * syy;
    const double cyy = sxx * szz - sxz * sxz, cyz = sxy * sxz - sxx * syz, czz = sxx * syy - sxy * sxy;
    const double det = fmax(sxx * cxx + sxy * cxy + sxz * cxz, 1e-30);
    const float w = (float)((double)g0.w * 0.063493635934240969 / sqrt(det));  // (2 pi)^-3/2
    aw = fabs((double)w);
    // quadratic form scaled by log2(e) / 2, cross terms doubled, so that
    // exp(-q / 2) = 2^-(x^T B x) with B = (log2(e) / 2) Sigma^-1
    const double f = 0.72134752044448170 / det;  // log2(e) / 2 / det
    rec[3 * n] = make_float4(g0.x, g0.y, g0.z, w);
    rec[3 * n + 1] = make_float4((float)(cxx * f), (float)(2.0 * cxy * f), (float)(2.0 * cxz * f),
                                 (float)(cyy * f));
    rec[3 * n + 2] = make_float4((float)(2.0 * cyz * f), (float)(czz * f), 0.f, 0.f);
    // axis-aligned box of the ellipsoid q <= q_cut: half extents sqrt(q_cut S_ii)
    const float mu[3] = {g0.x, g0.y, g0.z};
    const float hh[3] = {sqrtf(V.q_cut * g1.x), sqrtf(V.q_cut * g1.w), sqrtf(V.q_cut * g2.y)};
    const float ip = 1.f / V.pixel;
    int lo[3], hi[3];
    bool empty = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float a = ceilf((mu[k] - hh[k]) * ip + (float)V.c0);
      const float b = floorf((mu[k] + hh[k]) * ip + (float)V.c0);
      empty |= !(a <= b) || b < 0.f || a > (float)(V.D - 1);
      lo[k] = clampi(a, 0, V.D - 1) / kBrick;
      hi[k] = clampi(b, 0, V.D - 1) / kBrick;
    }
    box[n] = empty ? make_int4(0, 0, 0, 0)
                   : make_int4(lo[0] | (hi[0] << 16), lo[1] | (hi[1] << 16), lo[2] | (hi[2] << 16), 1);
  }
  red[threadIdx.x] = aw;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) wpart[blockIdx.x] = red[0];
}

// Brick index of entry l of a Gaussian's brick box (x fastest).
__device__ __forceinline__ int box_brick(int4 b, int l, int nb) {
  const int x0 = b.x & 0xffff, nx = (b.x >> 16) - x0 + 1;
  const int y0 = b.y & 0xffff, ny = (b.y >> 16) - y0 + 1;
  const int z0 = b.z & 0xffff;
  const int bx = x0 + l % nx, by = y0 + (l / nx) % ny, bz = z0 + l / (nx * ny);
  return (bz * nb + by) * nb + bx;
}

__device__ __forceinline__ int box_size(int4 b) {
  if (!b.w) return 0;
  return ((b.x >> 16) - (b.x & 0xffff) + 1) * ((b.y >> 16) - (b.y & 0xffff) + 1) *
         ((b.z >> 16) - (b.z & 0xffff) + 1);
}

// Brick counts: one wave per Gaussian, its lanes over the bricks of its box
// (a large box is no longer one thread's serial chain of atomics).
__global__ void __launch_bounds__(256)
k_vox_count(const int4 *box, VoxGeom V, int *count) {
  const int n = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (n >= V.N) return;
  const int4 b = box[n];
  const int m = box_size(b);
  for (int l = lane; l < m; l += 64) atomicAdd(&count[box_brick(b, l, V.nb)], 1);
}

// Exclusive scan of the brick counts (one block) and the fixed-point scale
// of the voxel sums from the bound sum_n |w_n| (k_vox_prep's per-block
// partials added in a fixed order, FP64).
__global__ void __launch_bounds__(1024)
k_vox_scan(const int *count, int nbr, const double *wpart, int nwp, int *off, double *scale) {
  __shared__ int part[1024];
  __shared__ double wsum[1024];
  const int t = threadIdx.x;
  const int per = (nbr + 1023) / 1024;
  const int a = t * per, b = min(nbr, a + per);
  int s = 0;
  for (int i = a; i < b; ++i) s += count[i];
  part[t] = s;
  double ws = 0.0;
  for (int i = t; i < nwp; i += 1024) ws += wpart[i];
  wsum[t] = ws;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive Hillis-Steele scan of the chunk sums
    const int v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  for (int h = 512; h > 0; h >>= 1) {
    if (t < h) wsum[t] += wsum[t + h];
    __syncthreads();
  }
  int run = t ? part[t - 1] : 0;
  for (int i = a; i < b; ++i) {
    off[i] = run;
    run += count[i];
  }
  if (t == 0) {
    off[nbr] = part[1023];
    const double total = wsum[0] > 0.0 ? wsum[0] : 1.0;
    int e;
    frexp(total, &e);  // total < 2^e
    *scale = ldexp(1.0, 61 - e);
  }
}

// Brick lists, one wave per Gaussian as in k_vox_count.
__global__ void __launch_bounds__(256)
k_vox_fill(const int4 *box, VoxGeom V, const int *off, int *cursor, int *list) {
  const int n = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (n >= V.N) return;
  const int4 b = box[n];
  const int m = box_size(b);
  for (int l = lane; l < m; l += 64) {
    const int k = box_brick(b, l, V.nb);
    list[off[k] + atomicAdd(&cursor[k], 1)] = n;
  }
}

// w 2^k as a 64-bit integer, truncated toward zero (|w| 2^k < 2^61); zero
// and subnormal w give 0.  Branch-free: y = |w| 2^k is exact (ldexp), its
// part above 2^32 is trunc(y 2^-32) and the rest, y - hi 2^32, is exact too
// (the bits of y below 2^32), so both convert exactly.  A function of w
// alone, so the voxel sums do not depend on the order of their terms.
__device__ __forceinline__ long long fixed_point(float w, int k) {
  const unsigned u = __float_as_uint(w);
  const float y = ldexpf(fabsf(w), k);
  const float hi = truncf(y * 0x1p-32f);
  const float lo = fmaf(hi, -0x1p32f, y);
  unsigned long long mag = ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo;
  mag = (u & 0x7f800000u) ? mag : 0ull;
  const long long sgn = (long long)((int)u >> 31);  // 0 or -1
  return ((long long)mag ^ sgn) - sgn;
}

// Lower bound of the scaled form over the voxel centres of a 4^3 sub-cube,
// minus a rounding margin: with c the centre of the sub-cube, h = 1.5 p the
// largest offset of a voxel centre from it along each axis and P the
// (positive semi-definite) form, q(c + d) = q(c) + 2 d.P(c - mu) + d.P d
// >= q(c) - h sum_k |2 (P(c - mu))_k|.  The margin T / 1024, with
// T = sum_ij |P_ij| (|c_i - mu_i| + h)(|c_j - mu_j| + h) bounding every term
// of q over the sub-cube, exceeds by far the rounding of both this bound and
// the per-voxel evaluation (positions included), so a sub-cube whose bound
// exceeds the cut holds no voxel that the per-voxel test would keep.
__device__ __forceinline__ float subcube_bound(float4 a, float4 B, float4 C, float cx, float cy,
                                               float cz, float h) {
  const float dx = cx - a.x, dy = cy - a.y, dz = cz - a.z;
  const float q = fmaf(dz, fmaf(C.y, dz, fmaf(B.z, dx, C.x * dy)),
                       fmaf(fmaf(B.x, dx, B.y * dy), dx, B.w * dy * dy));
  const float gx = fmaf(2.f * B.x, dx, fmaf(B.y, dy, B.z * dz));
  const float gy = fmaf(B.y, dx, fmaf(2.f * B.w, dy, C.x * dz));
  const float gz = fmaf(B.z, dx, fmaf(C.x, dy, 2.f * C.y * dz));
  const float ax = fabsf(dx) + h, ay = fabsf(dy) + h, az = fabsf(dz) + h;
  const float T = fabsf(B.x) * ax * ax + fabsf(B.w) * ay * ay + fabsf(C.y) * az * az +
                  ax * (fabsf(B.y) * ay + fabsf(B.z) * az) + fabsf(C.x) * ay * az;
  return q - h * (fabsf(gx) + fabsf(gy) + fabsf(gz)) - T * (1.f / 1024.f);
}

// One Gaussian's term at one voxel: the scaled form (mean, weight in a;
// form in B, C), the cut and the fixed-point value of w 2^-q.
__device__ __forceinline__ long long vox_term(float4 a, float4 B, float4 C, float px, float py,
                                              float pz, float qc, int k) {
  const float dx = px - a.x, dy = py - a.y;
  const float cxy = fmaf(fmaf(B.x, dx, B.y * dy), dx, B.w * dy * dy);
  const float fz = fmaf(B.z, dx, C.x * dy);
  const float dz = pz - a.z;
  const float q = fmaf(dz, fmaf(C.y, dz, fz), cxy);
  const long long v = fixed_point(a.w * __builtin_amdgcn_exp2f(-q), k);
  return q <= qc ? v : 0ll;
}

// One 4^3 sub-cube of a brick per wave (a workgroup of 64), one voxel per
// lane.  The eight sub-cubes of brick k are the workgroups
// 64 (k / 8) + 8 s + k % 8, s = 0 .. 7: workgroups are dealt to the eight
// XCDs in turn, so all eight land on the XCD of k % 8 and share its L2 for
// the brick's list and records.  The wave takes the list 64 Gaussians at a
// time: each lane loads one record and tests it against the sub-cube, the
// kept ones are staged in LDS, and the wave evaluates them one ballot bit
// at a time (two per pass).  The per-voxel arithmetic (form, cut, exp2,
// fixed point) is the same for every kept Gaussian whatever the order, and
// the sums are integers, so the result is that of evaluating every listed
// Gaussian at every voxel of the brick.
__global__ void __launch_bounds__(64)
k_vox_eval(const float4 *rec, const int *list, const int *off, VoxGeom V, const double *scale,
           float *vol) {
  __shared__ float4 sr[3][64];
  const int b = blockIdx.x;
  const int k = (b >> 6) * 8 + (b & 7), s = (b >> 3) & 7;
  if (k >= V.nb * V.nb * V.nb) return;
  const int bx = k % V.nb, by = (k / V.nb) % V.nb, bz = k / (V.nb * V.nb);
  const int lane = threadIdx.x;
  const int sx = bx * kBrick + 4 * (s & 1), sy = by * kBrick + 4 * ((s >> 1) & 1),
            sz = bz * kBrick + 4 * (s >> 2);
  const int ix = sx + (lane & 3), iy = sy + ((lane >> 2) & 3), iz = sz + (lane >> 4);
  const float px = (float)(ix - V.c0) * V.pixel, py = (float)(iy - V.c0) * V.pixel;
  const float pz = (float)(iz - V.c0) * V.pixel;
  const float h = 1.5f * V.pixel;
  const float cx = ((float)(sx - V.c0) + 1.5f) * V.pixel, cy = ((float)(sy - V.c0) + 1.5f) * V.pixel,
              cz = ((float)(sz - V.c0) + 1.5f) * V.pixel;
  const double S = *scale;
  int k2;
  frexp(S, &k2);
  const int kk = k2 - 1;                    // S = 2^(k2 - 1)
  const float qc = V.q_cut * 0.72134752f;   // the cut in the scaled form
  long long acc0 = 0, acc1 = 0;
  const int b0 = off[k], cnt = off[k + 1] - b0;
  for (int c = 0; c < cnt; c += 64) {
    bool keep = false;
    if (c + lane < cnt) {
      const int n = list[b0 + c + lane];
      const float4 a = rec[3 * n], B = rec[3 * n + 1], C = rec[3 * n + 2];
      keep = subcube_bound(a, B, C, cx, cy, cz, h) <= qc;
      sr[0][lane] = a;
      sr[1][lane] = B;
      sr[2][lane] = C;
    }
    __syncthreads();
    unsigned long long bits = __ballot(keep);
    while (bits) {  // two kept Gaussians per pass: independent chains
      const int j0 = __builtin_ctzll(bits);
      bits &= bits - 1ull;
      const bool two = bits != 0ull;
      const int j1 = two ? __builtin_ctzll(bits) : j0;
      bits &= bits - 1ull;
      const long long t0 = vox_term(sr[0][j0], sr[1][j0], sr[2][j0], px, py, pz, qc, kk);
      const long long t1 = vox_term(sr[0][j1], sr[1][j1], sr[2][j1], px, py, pz, qc, kk);
      acc0 += t0;
      acc1 += two ? t1 : 0ll;
    }
    __syncthreads();
  }
  vol[((int64_t)iz * V.D + iy) * V.D + ix] = (float)((double)(acc0 + acc1) / S);
}

// ---------------------------------------------------------------------------
// FSC
// ---------------------------------------------------------------------------

// Sum of squares of each volume in FP64: a fixed grid of kEnergyBlocks
// blocks, each over a fixed strided subset, so the summation order (and the
// scale below) does not depend on the device or on timing.
__global__ void __launch_bounds__(256)
k_fsc_energy_part(const float *va, const float *vb, int64_t n, double *part) {
  __shared__ double r[2][256];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0;
  const int64_t stride = (int64_t)kEnergyBlocks * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + t;
  for (; i + 3 * stride < n; i += 4 * stride) {  // four independent loads in flight
    const float a0 = va[i], a1 = va[i + stride], a2 = va[i + 2 * stride], a3 = va[i + 3 * stride];
    const float b0 = vb[i], b1 = vb[i + stride], b2 = vb[i + 2 * stride], b3 = vb[i + 3 * stride];
    a += (double)a0 * a0 + (double)a1 * a1 + (double)a2 * a2 + (double)a3 * a3;
    b += (double)b0 * b0 + (double)b1 * b1 + (double)b2 * b2 + (double)b3 * b3;
  }
  for (; i < n; i += stride) {
    a += (double)va[i] * va[i];
    b += (double)vb[i] * vb[i];
  }
  r[0][t] = a;
  r[1][t] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      r[0][t] += r[0][t + h];
      r[1][t] += r[1][t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[blockIdx.x] = r[0][0];
    part[kEnergyBlocks + blockIdx.x] = r[1][0];
  }
}

// Total of the block sums (fixed tree) and the shell scale from it.
__global__ void __launch_bounds__(kEnergyBlocks)
k_fsc_energy_scale(const double *part, int D, double *scale) {
  __shared__ double r[2][kEnergyBlocks];
  const int t = threadIdx.x;
  r[0][t] = part[t];
  r[1][t] = part[kEnergyBlocks + t];
  __syncthreads();
  for (int h = kEnergyBlocks / 2; h > 0; h >>= 1) {
    if (t < h) {
      r[0][t] += r[0][t + h];
      r[1][t] += r[1][t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    // every shell sum is at most D^3 max(sum Va^2, sum Vb^2) (Parseval)
    double bound = (double)D * D * D * fmax(r[0][0], r[1][0]);
    if (!(bound > 0.0)) bound = 1.0;
    int e;
    frexp(bound, &e);
    *scale = ldexp(1.0, 61 - e);
  }
}

// Shell sums over the half spectrum [kz][ky][kx] (kx = 0 .. D/2).
__global__ void __launch_bounds__(256)
k_fsc_shells(const float2 *fa, const float2 *fb, int D, const double *scale,
             unsigned long long *sums) {
  extern __shared__ unsigned long long ls[];  // [3][ns]
  const int ns = D / 2 + 1, Dh = D / 2 + 1;
  for (int i = threadIdx.x; i < 3 * ns; i += 256) ls[i] = 0ull;
  __syncthreads();
  const double S = *scale;
  const int64_t total = (int64_t)D * D * Dh;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int kx = (int)(i % Dh);
    const int64_t r = i / Dh;
    const int ky = (int)(r % D), kz = (int)(r / D);
    const int fy = ky < (D + 1) / 2 ? ky : ky - D, fz = kz < (D + 1) / 2 ? kz : kz - D;
    const int s = (int)rint(sqrt((double)(kx * kx + fy * fy + fz * fz)));
    if (s > D / 2) continue;
    const double w = (kx == 0 || kx == D / 2) ? 1.0 : 2.0;
    const float2 a = fa[i], b = fb[i];
    const double num = w * ((double)a.x * b.x + (double)a.y * b.y);
    const double da = w * ((double)a.x * a.x + (double)a.y * a.y);
    const double db = w * ((double)b.x * b.x + (double)b.y * b.y);
    atomicAdd(&ls[s], (unsigned long long)__double2ll_rn(num * S));
    atomicAdd(&ls[ns + s], (unsigned long long)__double2ll_rn(da * S));
    atomicAdd(&ls[2 * ns + s], (unsigned long long)__double2ll_rn(db * S));
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * ns; i += 256)
    if (ls[i]) atomicAdd(&sums[i], ls[i]);
}

__global__ void __launch_bounds__(256)
k_fsc_final(const unsigned long long *sums, int ns, const double *scale, float *fsc) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= ns) return;
  const double S = *scale;
  const double num = (double)(long long)sums[s] / S;
  const double da = (double)(long long)sums[ns + s] / S, db = (double)(long long)sums[2 * ns + s] / S;
  const double den = sqrt(da * db);
  fsc[s] = den > 0.0 ? (float)(num / den) : 0.f;
}

// Resolution read-out of an FSC curve: the first shell k >= 1 whose
// correlation is below the threshold (the last shell, D/2, when none is),
// and D p / k in Angstrom.  One wave: a ballot over the shells in order.
__global__ void __launch_bounds__(64)
k_fsc_resolution(const float *fsc, int ns, int D, float pixel, float threshold, int *shell,
                 float *resolution) {
  int first = ns - 1;
  for (int base = 1; base < ns; base += 64) {
    const int k = base + (int)threadIdx.x;
    const unsigned long long below = __ballot(k < ns && fsc[k] < threshold);
    if (below) {
      first = base + __ffsll((long long)below) - 1;
      break;
    }
  }
  if (threadIdx.x == 0) {
    if (shell) *shell = first;
    if (resolution) *resolution = (float)((double)D * (double)pixel / (double)first);
  }
}

__global__ void __launch_bounds__(256) k_fill_u64z(unsigned long long *p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void __launch_bounds__(256) k_fill_i32z(int *p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace cs
