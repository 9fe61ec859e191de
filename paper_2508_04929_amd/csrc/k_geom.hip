// Per-Gaussian and per-(image, Gaussian) kernels: covariance construction,
// projection, owner-tile binning, the per-Gaussian gradient chain, the pair
// counter and Adam.
#include "cs_internal.hpp"

namespace cs {

// ---------------------------------------------------------------------------
// Eq. 5 with the Sec. 3.3.1 activations: s = exp(l) or softplus(l),
// A = a or softplus(a), q normalised, Sigma = R diag(s)^2 R^T.
// Also clears `zero_count` ints of zero_buf (the binning counters).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_build(const float *means, const float *log_scales, const float *quats, const float *amps,
        Geom G, float4 *gc, int *zero_buf, int zero_count) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n < zero_count) zero_buf[n] = 0;
  if (n >= G.N) return;
  float s[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float l = log_scales[3 * n + k];
    s[k] = G.scale_act ? softplusf(l) : __expf(l);
  }
  const float a = amps[n];
  const float A = G.amp_act ? softplusf(a) : a;
  float w = quats[4 * n + 0], x = quats[4 * n + 1], y = quats[4 * n + 2], z = quats[4 * n + 3];
  const float inv = 1.f / fmaxf(sqrtf(w * w + x * x + y * y + z * z), 1e-12f);
  w *= inv; x *= inv; y *= inv; z *= inv;
  const float R[3][3] = {
      {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y)},
      {2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x)},
      {2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)}};
  float M[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[r][k] = R[r][k] * s[k];
  auto sig = [&](int i, int j) { return M[i][0] * M[j][0] + M[i][1] * M[j][1] + M[i][2] * M[j][2]; };
  gc[3 * n + 0] = make_float4(means[3 * n + 0], means[3 * n + 1], means[3 * n + 2], A);
  gc[3 * n + 1] = make_float4(sig(0, 0), sig(0, 1), sig(0, 2), sig(1, 1));
  gc[3 * n + 2] = make_float4(sig(1, 2), sig(2, 2), 0.f, 0.f);
}

__device__ __forceinline__ void load_pose(const float *rot, const float *shift, int b,
                                          float p0[3], float p1[3], float &tx, float &ty) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    p0[k] = rot[9 * b + k];
    p1[k] = rot[9 * b + 3 + k];
  }
  tx = shift ? shift[2 * b] : 0.f;
  ty = shift ? shift[2 * b + 1] : 0.f;
}

// Owner-tile key of a projected Gaussian: -1 when it touches no pixel of
// the image, the owner tile when its pixel box lies inside that tile's
// canvas (tile plus halo), G.ntiles ("wide") otherwise.
__device__ __forceinline__ int tile_key(const Proj &P, const Geom &G) {
  if (!(isfinite(P.u) && isfinite(P.v) && isfinite(P.hx) && isfinite(P.hy))) return -1;
  const float fj0 = fmaxf(ceilf(P.u - P.hx), 0.f);
  const float fj1 = fminf(floorf(P.u + P.hx), (float)(G.D - 1));
  const float fi0 = fmaxf(ceilf(P.v - P.hy), 0.f);
  const float fi1 = fminf(floorf(P.v + P.hy), (float)(G.D - 1));
  if (!(fj0 <= fj1 && fi0 <= fi1)) return -1;
  const int tx = (int)fminf(fmaxf(floorf(P.u / (float)G.T), 0.f), (float)(G.ntx - 1));
  const int ty = (int)fminf(fmaxf(floorf(P.v / (float)G.T), 0.f), (float)(G.ntx - 1));
  const int j0 = (int)fj0, j1 = (int)fj1, i0 = (int)fi0, i1 = (int)fi1;
  const bool fast = j0 >= tx * G.T - G.halo && j1 <= tx * G.T + G.T - 1 + G.halo &&
                    i0 >= ty * G.T - G.halo && i1 <= ty * G.T + G.T - 1 + G.halo;
  return fast ? ty * G.ntx + tx : G.ntiles;
}

// ---------------------------------------------------------------------------
// Binning pass 1: key per (image, Gaussian) and per-block bin counts.
// Block (x, y): Gaussians [256 x, 256 x + 256) of images [8 y, 8 y + 8);
// blk[(b K + k) nbx + x] receives the block's count of bin k of image b
// (every bin, zeros included), so that a scan over x orders the bin's
// entries by Gaussian index.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_bin_count(const float4 *gc, const float *rot, const float *shift, Geom G, int *key,
            int *blk, int nbx) {
  extern __shared__ int hist[];  // [kImgPerBinBlock][K]
  const int n = blockIdx.x * kBlock + threadIdx.x;
  const int b0 = blockIdx.y * kImgPerBinBlock;
  for (int i = threadIdx.x; i < kImgPerBinBlock * G.K; i += kBlock) hist[i] = 0;
  __syncthreads();
  float4 g0 = make_float4(0, 0, 0, 0), g1 = g0, g2 = g0;
  if (n < G.N) {
    g0 = gc[3 * n];
    g1 = gc[3 * n + 1];
    g2 = gc[3 * n + 2];
  }
  for (int bi = 0; bi < kImgPerBinBlock; ++bi) {
    const int b = b0 + bi;
    if (b >= G.B) break;
    if (n < G.N) {
      float p0[3], p1[3], tx, ty;
      load_pose(rot, shift, b, p0, p1, tx, ty);
      Proj P;
      project_one(g0, g1, make_float2(g2.x, g2.y), p0, p1, tx, ty, G, P);
      const int k = tile_key(P, G);
      key[(size_t)b * G.N + n] = k;
      if (k >= 0) atomicAdd(&hist[bi * G.K + k], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kImgPerBinBlock * G.K; i += kBlock) {
    const int b = b0 + i / G.K;
    if (b < G.B) blk[((size_t)b * G.K + i % G.K) * nbx + blockIdx.x] = hist[i];
  }
}

// Per bin: exclusive scan of the per-block counts over blocks (in place)
// and the bin total.  One block of 256 threads per bin.
__global__ void __launch_bounds__(kBlock)
k_bin_blockscan(int *blk, int nbx, int *count) {
  __shared__ int wsum[kBlock / 64];
  int *row = blk + (size_t)blockIdx.x * nbx;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int carry = 0;
  for (int base = 0; base < nbx; base += kBlock) {
    const int x = base + threadIdx.x;
    const int val = x < nbx ? row[x] : 0;
    int inc = val;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(inc, o, 64);
      if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int wpre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      wpre += (w < wid) ? wsum[w] : 0;
      tot += wsum[w];
    }
    if (x < nbx) row[x] = carry + wpre + inc - val;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) count[blockIdx.x] = carry;
}

// Exclusive scan across one block of 1024 threads (16 waves of 64).
__device__ int block_scan_1024(int val, int *sh, int &total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = val;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  if (wid == 0) {
    int s = lane < 16 ? sh[lane] : 0;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const int y = __shfl_up(s, o, 64);
      if (lane >= o) s += y;
    }
    if (lane < 16) sh[lane] = s;
  }
  __syncthreads();
  const int prefix = wid > 0 ? sh[wid - 1] : 0;
  total = sh[15];
  __syncthreads();
  return prefix + x - val;
}

// ---------------------------------------------------------------------------
// Binning pass 2 (one block of 1024 threads): list offsets per bin and the
// work items.  A work item is a chunk of at most G.budget Gaussians of one
// owner tile.  Also resets the work-queue counters.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024)
k_scan(int *count, Geom G, int *off, int4 *items, int *item_off, int *n_items,
       int *queues, int *blk, int nbx) {
  __shared__ int sh[16];
  const int total = G.B * G.K;
  if (blk) {
    // few (image, tile) entries: the per-entry scans of k_bin_blockscan, one
    // wave per entry (the same integers, one launch fewer)
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int e = wid; e < total; e += 16) {
      int *row = blk + (size_t)e * nbx;
      int carry = 0;
      for (int base = 0; base < nbx; base += 64) {
        const int x = base + lane;
        const int v = x < nbx ? row[x] : 0;
        int inc = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(inc, o, 64);
          if (lane >= o) inc += y;
        }
        if (x < nbx) row[x] = carry + inc - v;
        carry += __shfl(inc, 63, 64);
      }
      if (lane == 0) count[e] = carry;
    }
    __syncthreads();
  }
  const int seg = (total + 1023) / 1024;
  const int e0 = min(threadIdx.x * seg, total), e1 = min(e0 + seg, total);
  int s = 0, si = 0, sw = 0;
  for (int e = e0; e < e1; ++e) {
    const int c = count[e];
    s += c;
    if (e % G.K < G.ntiles) si += (c + G.budget - 1) / G.budget;
    else sw += c;
  }
  int tot, itot, wtot;
  int pre = block_scan_1024(s, sh, tot);
  int ipre = block_scan_1024(si, sh, itot);
  block_scan_1024(sw, sh, wtot);
  for (int e = e0; e < e1; ++e) {
    const int c = count[e];
    off[e] = pre;
    item_off[e] = ipre;
    const int t = e % G.K;
    if (t < G.ntiles) {
      const int nc = (c + G.budget - 1) / G.budget;
      for (int k = 0; k < nc; ++k)
        items[ipre + k] = make_int4(e / G.K, t, pre + k * G.budget, min(G.budget, c - k * G.budget));
      ipre += nc;
    }
    pre += c;
  }
  if (threadIdx.x == 0) {
    item_off[total] = itot;
    n_items[0] = itot;
    n_items[1] = wtot;  // wide (beyond-halo) records
    queues[0] = 0;
    queues[1] = 0;
  }
}

// ---------------------------------------------------------------------------
// Binning pass 3: write the 32-byte splat record of every visible
// (image, Gaussian) into its bin's segment of the list:
//   rec0 = (u, v, al, be), rec1 = (ga, w, n, i0 | i1 << 16)
// with (al, be, ga) the exp2-scaled pixel conic and [i0, i1] the clipped
// row range of the q_cut ellipse.  The position is the bin offset plus the
// block's scanned offset plus the stable rank inside the block, so every
// bin lists its Gaussians in increasing index (a deterministic counting
// sort; the rank inside the block comes from per-wave LDS bitmasks of the
// lanes holding each bin, and no device-memory atomics are used).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_bin_scatter(const float4 *gc, const float *rot, const float *shift, Geom G, const int *key,
              const int *off, const int *blk, int nbx, float4 *list, float *wabs) {
  // [kBlock/64][K]: per wave and bin, the lanes holding that bin
  extern __shared__ unsigned long long wmask[];
  const int n = blockIdx.x * kBlock + threadIdx.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int b0 = blockIdx.y * kImgPerBinBlock;
  float4 g0 = make_float4(0, 0, 0, 0), g1 = g0, g2 = g0;
  if (n < G.N) {
    g0 = gc[3 * n];
    g1 = gc[3 * n + 1];
    g2 = gc[3 * n + 2];
  }
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // the bins of all the block's images, then their list bases (segment
  // offset plus this block's count of earlier records), requested before
  // the per-image loop so the loads overlap instead of costing two
  // round trips per image
  int kk[kImgPerBinBlock], base[kImgPerBinBlock];
#pragma unroll
  for (int bi = 0; bi < kImgPerBinBlock; ++bi) {
    const int b = b0 + bi;
    kk[bi] = (n < G.N && b < G.B) ? key[(size_t)b * G.N + n] : -1;
  }
#pragma unroll
  for (int bi = 0; bi < kImgPerBinBlock; ++bi) {
    // every load is issued (index 0 for an absent record), so none waits
    // behind a branch
    const int e = kk[bi] >= 0 ? (b0 + bi) * G.K + kk[bi] : 0;
    const int o = off[e], c = blk[(size_t)e * nbx + blockIdx.x];
    base[bi] = o + c;
  }
#pragma unroll
  for (int bi = 0; bi < kImgPerBinBlock; ++bi) {
    const int b = b0 + bi;
    if (b >= G.B) break;
    for (int i = threadIdx.x; i < (kBlock / 64) * G.K; i += kBlock) wmask[i] = 0ull;
    __syncthreads();
    const int k = kk[bi];
    if (k >= 0) atomicOr(&wmask[wid * G.K + k], 1ull << lane);
    __syncthreads();
    if (k >= 0) {
      // stable rank: same-bin lanes below this one in its wave, then the
      // same-bin lanes of the earlier waves
      int rank = __popcll(wmask[wid * G.K + k] & below);
      for (int w = 0; w < wid; ++w) rank += __popcll(wmask[w * G.K + k]);
      const int pos = base[bi] + rank;
      float p0[3], p1[3], tx, ty;
      load_pose(rot, shift, b, p0, p1, tx, ty);
      Proj P;
      project_one(g0, g1, make_float2(g2.x, g2.y), p0, p1, tx, ty, G, P);
      const int i0 = clamp_px(ceilf(P.v - P.hy), 0, G.D - 1);
      const int i1 = clamp_px(floorf(P.v + P.hy), 0, G.D - 1);
      list[2 * (size_t)pos] = make_float4(P.u, P.v, P.al, P.be);
      list[2 * (size_t)pos + 1] =
          make_float4(P.ga, P.w, __int_as_float(n), __int_as_float(i0 | (i1 << 16)));
      // |w| beside the record, in list order: the forward splat sums it per
      // work item for its fixed-point scale without reading the records twice
      wabs[pos] = fabsf(P.w);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Per-Gaussian gradient chain.  For every image where the Gaussian is
// visible, the six pixel moments written by the backward splat,
//   m = sum_pixels G_Q e * (1, dj, di, dj^2, dj di, di^2),  e = exp(-q/2),
// give (pixel units, a b c the pixel conic, w the weight):
//   dL/dw = m0,  dL/du = w (a m1 + b m2),  dL/dv = w (b m1 + c m2),
//   dL/da = -w m3 / 2,  dL/db = -w m4,  dL/dc = -w m5 / 2.
// These map to the screen mean and conic C = Sigma~^-1 (Eq. 18, 20), then
//   dL/dSigma~ = -C G_C C - (w dL/dw / 2) C     (Eq. 20 with |C|^1/2 in w)
// and to the world frame: dmu += P^T dmu~, dSigma += P^T dSigma~ P (Eq. 21).
// Finally Sigma = M M^T with M = R diag(s): dM = 2 dSigma M, ds_k =
// sum_r dM_rk R_rk, dR = dM diag(s), then the unit-quaternion and
// activation derivatives (the 3DGS chain the paper defers to, App. A.2).
// ---------------------------------------------------------------------------
// Screen-frame gradients of one (image, Gaussian) pair from its six pixel
// moments m: dL/dmu~ (Angstrom, x right / y up) and the symmetric dL/dSigma~
// (Eq. 18, 20, with the |C|^1/2 of the weight folded in).
struct ScreenGrad {
  float dmx, dmy, Sxx, Sxy, Syy;
};

__device__ __forceinline__ ScreenGrad screen_grad(const Proj &P, const float *m, float pixel) {
  const float p2 = pixel * pixel, ip = 1.f / pixel;
  const float m0 = m[0], m1 = m[1], m2 = m[2], m3 = m[3], m4 = m[4], m5 = m[5];
  const float inv_det = 1.f / P.det;
  const float Cxx = P.syy * inv_det, Cxy = -P.sxy * inv_det, Cyy = P.sxx * inv_det;
  const float a = p2 * Cxx, bb = -p2 * Cxy, c = p2 * Cyy;
  const float w = P.w;
  const float dLdu = w * (a * m1 + bb * m2);
  const float dLdv = w * (bb * m1 + c * m2);
  ScreenGrad r;
  r.dmx = dLdu * ip;
  r.dmy = -dLdv * ip;
  // symmetric gradient w.r.t. C (entries), from d/da, d/db, d/dc
  const float Gxx = -0.5f * w * m3 * p2;
  const float Gxy = 0.5f * w * m4 * p2;
  const float Gyy = -0.5f * w * m5 * p2;
  // -C G C - (w m0 / 2) C
  const float t_xx = Cxx * Gxx + Cxy * Gxy, t_xy = Cxx * Gxy + Cxy * Gyy;
  const float t_yx = Cxy * Gxx + Cyy * Gxy, t_yy = Cxy * Gxy + Cyy * Gyy;
  const float hw = 0.5f * w * m0;
  r.Sxx = -(t_xx * Cxx + t_xy * Cxy) - hw * Cxx;
  r.Sxy = -(t_xx * Cxy + t_xy * Cyy) - hw * Cxy;
  r.Syy = -(t_yx * Cxy + t_yy * Cyy) - hw * Cyy;
  return r;
}

__global__ void __launch_bounds__(kBlock)
k_chain(const float4 *gc, const float *log_scales, const float *quats, const float *amps,
        const float *rot, const float *shift, Geom G, const int *key, const float *mom,
        float *g_means, float *g_log_scales, float *g_quats, float *g_amps) {
  // 64 Gaussians per block; wave w of the four sums the images b = w mod 4
  // (coalesced 64-Gaussian rows of every image, four times the waves of one
  // thread per Gaussian), the partial sums meet in LDS in a fixed order
  __shared__ float red[4][10][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + lane;
  const bool live = n < G.N;
  float4 g0 = make_float4(0, 0, 0, 0), g1 = g0, g2 = g0;
  if (live) {
    g0 = gc[3 * n];
    g1 = gc[3 * n + 1];
    g2 = gc[3 * n + 2];
  }
  float dmu[3] = {0, 0, 0};
  float dS[6] = {0, 0, 0, 0, 0, 0};  // xx xy xz yy yz zz
  float dw_sum = 0.f;                // sum_b dL/dw * w / A  (= dL/dA)
  // the image index is uniform across the wave: its pose comes through
  // scalar loads
  for (int b = __builtin_amdgcn_readfirstlane(wv); live && b < G.B; b += 4) {
    // the pose, the key and the moment row are read together (the row
    // exists for every (image, Gaussian); it holds moments only where the
    // key is a bin), so an image costs one round trip to memory, not three
    float p0[3], p1[3], tx, ty;
    load_pose(rot, shift, b, p0, p1, tx, ty);
    const size_t row = (size_t)b * G.N + n;
    const int kb = key[row];
    const float2 *m2 = (const float2 *)(mom + row * 6);
    const float2 ma = m2[0], mb = m2[1], mc = m2[2];
    // keeps the row's loads ahead of the branch (the compiler would sink
    // them into it, after the key's round trip)
    asm volatile("" ::"v"(ma), "v"(mb), "v"(mc));
    if (kb < 0) continue;
    const float m[6] = {ma.x, ma.y, mb.x, mb.y, mc.x, mc.y};
    Proj P;
    project_one(g0, g1, make_float2(g2.x, g2.y), p0, p1, tx, ty, G, P);
    const ScreenGrad sg = screen_grad(P, m, G.pixel);
    const float dmx = sg.dmx, dmy = sg.dmy, Sxx = sg.Sxx, Sxy = sg.Sxy, Syy = sg.Syy;
    const float m0 = m[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) dmu[k] += p0[k] * dmx + p1[k] * dmy;
    const int ii[6] = {0, 0, 0, 1, 1, 2}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int i = ii[e], j = jj[e];
      dS[e] += Sxx * p0[i] * p0[j] + Sxy * (p0[i] * p1[j] + p1[i] * p0[j]) + Syy * p1[i] * p1[j];
    }
    dw_sum += m0 * rsqrtf(P.det) * 0.15915494309189535f;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) red[wv][k][lane] = dmu[k];
#pragma unroll
  for (int e = 0; e < 6; ++e) red[wv][3 + e][lane] = dS[e];
  red[wv][9][lane] = dw_sum;
  __syncthreads();
  if (wv != 0 || !live) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) dmu[k] = red[0][k][lane] + red[1][k][lane] + red[2][k][lane] + red[3][k][lane];
#pragma unroll
  for (int e = 0; e < 6; ++e)
    dS[e] = red[0][3 + e][lane] + red[1][3 + e][lane] + red[2][3 + e][lane] + red[3][3 + e][lane];
  dw_sum = red[0][9][lane] + red[1][9][lane] + red[2][9][lane] + red[3][9][lane];
  // Sigma = M M^T, M = R diag(s)
  float s[3], dsdl[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float l = log_scales[3 * n + k];
    if (G.scale_act) {
      s[k] = softplusf(l);
      dsdl[k] = sigmoidf_(l);
    } else {
      s[k] = __expf(l);
      dsdl[k] = s[k];
    }
  }
  float qw = quats[4 * n + 0], qx = quats[4 * n + 1], qy = quats[4 * n + 2], qz = quats[4 * n + 3];
  const float qn = fmaxf(sqrtf(qw * qw + qx * qx + qy * qy + qz * qz), 1e-12f);
  const float iq = 1.f / qn;
  qw *= iq; qx *= iq; qy *= iq; qz *= iq;
  const float R[3][3] = {
      {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy)},
      {2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx)},
      {2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)}};
  const float Sg[3][3] = {{dS[0], dS[1], dS[2]}, {dS[1], dS[3], dS[4]}, {dS[2], dS[4], dS[5]}};
  float dM[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      dM[r][k] = 2.f * (Sg[r][0] * R[0][k] * s[k] + Sg[r][1] * R[1][k] * s[k] + Sg[r][2] * R[2][k] * s[k]);
  float dR[3][3];
  float ds[3] = {0, 0, 0};
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ds[k] += dM[r][k] * R[r][k];
      dR[r][k] = dM[r][k] * s[k];
    }
  // dR/dq for the unit-quaternion form of R
  const float dqw = 2.f * (-qz * dR[0][1] + qy * dR[0][2] + qz * dR[1][0] - qx * dR[1][2] -
                           qy * dR[2][0] + qx * dR[2][1]);
  const float dqx = 2.f * (qy * dR[0][1] + qz * dR[0][2] + qy * dR[1][0] - 2.f * qx * dR[1][1] -
                           qw * dR[1][2] + qz * dR[2][0] + qw * dR[2][1] - 2.f * qx * dR[2][2]);
  const float dqy = 2.f * (-2.f * qy * dR[0][0] + qx * dR[0][1] + qw * dR[0][2] + qx * dR[1][0] +
                           qz * dR[1][2] - qw * dR[2][0] + qz * dR[2][1] - 2.f * qy * dR[2][2]);
  const float dqz = 2.f * (-2.f * qz * dR[0][0] - qw * dR[0][1] + qx * dR[0][2] + qw * dR[1][0] -
                           2.f * qz * dR[1][1] + qy * dR[1][2] + qx * dR[2][0] + qy * dR[2][1]);
  const float dot = qw * dqw + qx * dqx + qy * dqy + qz * dqz;
  if (g_means) {
#pragma unroll
    for (int k = 0; k < 3; ++k) g_means[3 * n + k] = dmu[k];
  }
  if (g_log_scales) {
#pragma unroll
    for (int k = 0; k < 3; ++k) g_log_scales[3 * n + k] = ds[k] * dsdl[k];
  }
  if (g_quats) {
    g_quats[4 * n + 0] = (dqw - qw * dot) * iq;
    g_quats[4 * n + 1] = (dqx - qx * dot) * iq;
    g_quats[4 * n + 2] = (dqy - qy * dot) * iq;
    g_quats[4 * n + 3] = (dqz - qz * dot) * iq;
  }
  if (g_amps) {
    const float a = amps[n];
    g_amps[n] = dw_sum * (G.amp_act ? sigmoidf_(a) : 1.f);
  }
}

// ---------------------------------------------------------------------------
// Pose gradients (the joint pose optimisation the paper names as future work,
// Sec. 5, from the same adjoint, App. A.2 Eq. 18 and 21).  With the
// projection P = the first two rows of the view rotation W, mu~ = P mu + t
// and Sigma~ = P Sigma P^T:
//   dL/dt = sum_n dL/dmu~_n,
//   dL/dP = sum_n ( dL/dmu~_n mu_n^T + 2 dL/dSigma~_n P Sigma_n ),
// the third row of W does not enter the image (its gradient is zero).
// Partials per (image, block of Gaussians) in a fixed order, then a
// fixed-order sum over blocks: deterministic.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_pose_grad_part(const float4 *gc, const float *rot, const float *shift, Geom G, const int *key,
                 const float *mom, float *part) {
  __shared__ float red[kBlock / 64][8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nbase = blockIdx.x * kBlock * kPoseGauss + threadIdx.x;
  // kPoseGauss Gaussians per thread (strided by the block size, so every load
  // stays coalesced), their records read once for kPoseImg images
  float4 g0[kPoseGauss], g1[kPoseGauss], g2[kPoseGauss];
#pragma unroll
  for (int j = 0; j < kPoseGauss; ++j) {
    const int n = nbase + j * kBlock;
    g0[j] = g1[j] = g2[j] = make_float4(0, 0, 0, 0);
    if (n < G.N) {
      g0[j] = gc[3 * n];
      g1[j] = gc[3 * n + 1];
      g2[j] = gc[3 * n + 2];
    }
  }
  const int b1 = min(G.B, (int)(blockIdx.y + 1) * kPoseImg);
  for (int b = blockIdx.y * kPoseImg; b < b1; ++b) {
    float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // t_x, t_y, P_0 (3), P_1 (3)
    float p0[3], p1[3], tx, ty;
    load_pose(rot, shift, b, p0, p1, tx, ty);
    // the keys and moment rows of the thread's Gaussians, all requested
    // before the first branch (indices past N read row 0 and are dropped)
    int kb[kPoseGauss];
    float2 mv[kPoseGauss][3];
#pragma unroll
    for (int j = 0; j < kPoseGauss; ++j) {
      const int n = nbase + j * kBlock;
      const size_t row = (size_t)b * G.N + (n < G.N ? n : 0);
      kb[j] = key[row];
      const float2 *m2 = (const float2 *)(mom + row * 6);
      mv[j][0] = m2[0];
      mv[j][1] = m2[1];
      mv[j][2] = m2[2];
    }
    bool use[kPoseGauss];
    float mrow[kPoseGauss][6];
#pragma unroll
    for (int j = 0; j < kPoseGauss; ++j) {
      // keeps the loads ahead of the branches below (the compiler would
      // sink each into its branch, one round trip per Gaussian)
      asm volatile("" ::"v"(mv[j][0]), "v"(mv[j][1]), "v"(mv[j][2]));
      use[j] = nbase + j * kBlock < G.N && kb[j] >= 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        mrow[j][2 * c] = mv[j][c].x;
        mrow[j][2 * c + 1] = mv[j][c].y;
      }
    }
#pragma unroll
    for (int j = 0; j < kPoseGauss; ++j) {
      if (use[j]) {
        Proj P;
        project_one(g0[j], g1[j], make_float2(g2[j].x, g2[j].y), p0, p1, tx, ty, G, P);
        const ScreenGrad sg = screen_grad(P, mrow[j], G.pixel);
        // Sigma p0, Sigma p1 (Sigma symmetric: the rows of P Sigma)
        const float4 a = g1[j], c = g2[j];
        const float sp0[3] = {a.x * p0[0] + a.y * p0[1] + a.z * p0[2],
                              a.y * p0[0] + a.w * p0[1] + c.x * p0[2],
                              a.z * p0[0] + c.x * p0[1] + c.y * p0[2]};
        const float sp1[3] = {a.x * p1[0] + a.y * p1[1] + a.z * p1[2],
                              a.y * p1[0] + a.w * p1[1] + c.x * p1[2],
                              a.z * p1[0] + c.x * p1[1] + c.y * p1[2]};
        const float mu[3] = {g0[j].x, g0[j].y, g0[j].z};
        v[0] += sg.dmx;
        v[1] += sg.dmy;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          v[2 + k] += sg.dmx * mu[k] + 2.f * (sg.Sxx * sp0[k] + sg.Sxy * sp1[k]);
          v[5 + k] += sg.dmy * mu[k] + 2.f * (sg.Sxy * sp0[k] + sg.Syy * sp1[k]);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float x = v[e];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
      if (lane == 0) red[wv][e] = x;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
      float x = 0.f;
      for (int w = 0; w < kBlock / 64; ++w) x += red[w][threadIdx.x];
      part[((size_t)b * gridDim.x + blockIdx.x) * 8 + threadIdx.x] = x;
    }
    __syncthreads();
  }
}

// g_rot [B][3][3] (third row zero), g_shift [B][2]; either may be null.  One
// block per image: each thread sums a strided subset of the block partials,
// then a fixed tree over the threads.
__global__ void __launch_bounds__(kBlock)
k_pose_grad_sum(const float *part, int B, int nblk, float *g_rot, float *g_shift) {
  __shared__ float red[kBlock][8];
  const int b = blockIdx.x, t = threadIdx.x;
  float x[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = t; k < nblk; k += kBlock)
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] += part[((size_t)b * nblk + k) * 8 + e];
#pragma unroll
  for (int e = 0; e < 8; ++e) red[t][e] = x[e];
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (t < h)
#pragma unroll
      for (int e = 0; e < 8; ++e) red[t][e] += red[t + h][e];
    __syncthreads();
  }
  if (t < 8) {
    const float v = red[0][t];
    if (t < 2) {
      if (g_shift) g_shift[2 * b + t] = v;
    } else if (g_rot) {
      g_rot[9 * b + (t - 2)] = v;  // rows 0 and 1: entries 0..5
      if (t < 5) g_rot[9 * b + 6 + (t - 2)] = 0.f;
    }
  }
}

// ---------------------------------------------------------------------------
// Exact-footprint pair count per image: pixels of the image with squared
// Mahalanobis distance <= q_cut, summed over Gaussians (the splat's
// algorithmic work), using the renderer's per-row spans.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_pair_count(const float4 *gc, const float *rot, const float *shift, Geom G,
             unsigned long long *counts) {
  __shared__ unsigned long long part[kBlock / 64];
  const int n = blockIdx.x * kBlock + threadIdx.x;
  const int b = blockIdx.y;
  unsigned long long cnt = 0;
  if (n < G.N) {
    const float4 g0 = gc[3 * n], g1 = gc[3 * n + 1], g2 = gc[3 * n + 2];
    float p0[3], p1[3], tx, ty;
    load_pose(rot, shift, b, p0, p1, tx, ty);
    Proj P;
    project_one(g0, g1, make_float2(g2.x, g2.y), p0, p1, tx, ty, G, P);
    if (isfinite(P.u) && isfinite(P.v) && isfinite(P.hy)) {
      const int i0 = clamp_px(ceilf(P.v - P.hy), 0, G.D);
      const int i1 = clamp_px(floorf(P.v + P.hy), -1, G.D - 1);
      const float det_s = P.al * P.ga - P.be * P.be;
      const float ia = 1.f / P.al;
      for (int i = i0; i <= i1; ++i) {
        const float di = (float)i - P.v;
        const float disc = P.al * G.qk - det_s * di * di;
        if (disc < 0.f) continue;
        const float h = sqrtf(disc) * ia;
        const float cen = P.u - P.be * di * ia;
        const int j0 = clamp_px(ceilf(cen - h), 0, G.D);
        const int j1 = clamp_px(floorf(cen + h), -1, G.D - 1);
        if (j1 >= j0) cnt += (unsigned long long)(j1 - j0 + 1);
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int k = 0; k < kBlock / 64; ++k) t += part[k];
    if (t) atomicAdd(&counts[b], t);
  }
}

// Adam (Alg. 1 "Adam(grad L)"), bias corrections precomputed on the host.
__global__ void __launch_bounds__(kBlock)
k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
       float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void __launch_bounds__(kBlock) k_fill(float *p, int64_t n, float value) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = value;
}

// Debug checks: flag[0] |= bit when any of the n values is NaN or infinite.
__global__ void __launch_bounds__(kBlock)
k_check_finite(const float *p, int64_t n, int bit, int *flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    bad |= !isfinite(p[i]);
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, bit);
}

}  // namespace cs
