// Forward and adjoint splat kernels (Alg. 2 SumSplats and its backward).
//
// Work decomposition: every visible (image, Gaussian) record belongs to one
// owner tile (T x T pixels); its whole truncated footprint lies inside the
// tile's canvas, the tile plus a halo on every side.  A work item is a chunk
// of at most `budget` records of one owner tile.  Inside an item each lane
// owns one Gaussian and walks its exact footprint row by row: the row span
// comes from the q_cut ellipse, and along a row the Gaussian obeys the
// two-multiply recurrence
//     e(j+1) = e(j) r(j),   r(j+1) = r(j) K,   K = exp(-a)
// (a is the pixel-unit conic's xx entry), so no transcendental is evaluated
// per pixel.  The forward accumulates into an LDS canvas in 32-bit fixed
// point with integer LDS atomics (LDS float atomics are ~30x slower on
// gfx950; integer addition also makes the sum order-independent, matching
// the order-free additive splat of Sec. 3.3.4).  The fixed-point scale of
// an item is the largest power of two with scale * sum|w| <= 2^30, so no
// pixel can overflow.  The backward reads G_Q from an LDS copy of the
// canvas region and accumulates the six pixel moments per Gaussian in
// registers, so no per-pixel state is stored between the passes.
#include "cs_internal.hpp"

namespace cs {

// Hardware exp2/sqrt (v_exp_f32 / v_sqrt_f32, about 1 ulp; results below
// 2^-126 flush to zero, far under the 1e-6 truncation of every term).
__device__ __forceinline__ float hexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Exact column span of the row at vertical offset di = i - v for the
// ellipse q <= q_cut, clipped to [clo, chi]: first column j0 and length L
// (false for an empty row).  aqk = al * qk.  The span ends are converted to
// integers before clamping (finite here: al > 0 and the record fits its
// canvas).
__device__ __forceinline__ bool row_span(float u, float di, float al, float be, float det_s,
                                         float inv_al, float aqk, int clo, int chi, int &j0,
                                         int &L) {
  const float disc = aqk - det_s * di * di;
  if (!(disc >= 0.f)) return false;
  const float h = hsqrt(disc) * inv_al;
  const float cen = u - be * di * inv_al;
  j0 = max((int)ceilf(cen - h), clo);
  L = min((int)floorf(cen + h), chi) - j0 + 1;
  return L > 0;
}

// Row of flat index x in rows of length n: x / n through a float reciprocal
// (exact while x < 2^20 and n <= 1024: the quotient (x + 1/2) / n stays at
// least 1 / (2 n) away from an integer, far above the rounding error).
__device__ __forceinline__ int row_of(int x, float inv_n) {
  return (int)(((float)x + 0.5f) * inv_n);
}

__device__ __forceinline__ int next_item(int *queue, int *slot) {
  if (threadIdx.x == 0) *slot = atomicAdd(queue, 1);
  __syncthreads();
  return *slot;
}

// ---------------------------------------------------------------------------
// Dealing records to lanes.  Every lane walks its own Gaussian, so at a step
// the lanes of a wave touch canvas words around their own centres; words of
// equal address mod 64 fall into one LDS bank and serialise.  With rows of
// S words, a lane's word at row i, column j sits in bank (S i + j) mod 64;
// as all lanes step rows and columns together, the bank of lane l is
// key_l + w_l + (a common offset), where key_l = (S i0_l + floor(u_l)) mod 64
// (its first row and centre column) and w_l in {0, 1} the rounding of its
// span start.  A chunk of kDealChunk records is therefore put in an order in
// which every 64 consecutive records carry distinct keys, the first 32 even
// keys and the last 32 odd keys: records are grouped by key, and round r
// takes the r-th record of every group in the order 0, 2, ..., 62, 1, 3,
// ..., 63 (a record's place is the size of the earlier rounds plus the
// non-empty groups before its own in its round).  Within a half-wave the keys
// then differ by at least 2, so the span-start rounding cannot make two lanes
// meet.  The order only changes which lane takes which record: every result
// is the same.  Groups of more than kDealRounds records keep the list order.
// Dealing costs a pass over the chunk's records and pays where footprints
// are wide (many steps per record); it is the launch option lane_order = 1,
// chosen per problem by the autotuner.
// ---------------------------------------------------------------------------
constexpr int kDealChunk = 512;
constexpr int kDealRounds = 32;

struct DealLds {
  unsigned long long M[kDealRounds];  // round r: groups with more than r records
  int R[kDealRounds];                 // records in rounds before r
  int cnt[64];
  unsigned short perm[kDealChunk];    // place -> record (within the chunk)
  int ok;
};

__device__ __forceinline__ void deal(const float4 *list, size_t base, int n, int S, int R0, int C0,
                                     DealLds &d) {
  const int t = threadIdx.x;
  if (t < 64) d.cnt[t] = 0;
  __syncthreads();
  constexpr int kPer = kDealChunk / kBlock;
  int key[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int g = t + j * kBlock;
    key[j] = -1;
    if (g < n) {
      const float4 r0 = list[2 * (base + g)];
      const int rows = __float_as_int(list[2 * (base + g) + 1].w);
      const int k = (S * ((rows & 0xffff) - R0) + (int)floorf(r0.x) - C0) & 63;
      const int grp = (k >> 1) | ((k & 1) << 5);  // even keys first, then odd
      key[j] = (atomicAdd(&d.cnt[grp], 1) << 6) | grp;
    }
  }
  __syncthreads();
  if (t < 64) {  // one wave lays out the rounds
    const int c = d.cnt[t];
    int mx = c;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
    const bool ok = mx <= kDealRounds;
    if (ok) {
      int run = 0;
      for (int r = 0; r < mx; ++r) {
        const unsigned long long m = __ballot(c > r);
        if (t == 0) {
          d.M[r] = m;
          d.R[r] = run;
        }
        run += __popcll(m);
      }
    }
    if (t == 0) d.ok = ok;
  }
  __syncthreads();
  const bool ok = d.ok;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    if (key[j] < 0) continue;
    const int g = t + j * kBlock;
    int pos = g;
    if (ok) {
      const int r = key[j] >> 6, grp = key[j] & 63;
      pos = d.R[r] + __popcll(d.M[r] & ((1ull << grp) - 1ull));
    }
    d.perm[pos] = (unsigned short)g;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Sorting records by footprint shape.  A wave steps as many rows as its
// tallest footprint and, per row, as many pixel groups as its widest active
// span, so where footprint sizes spread (anisotropic Gaussians with
// log-normal scales) most lanes idle for most steps.  Launch option
// lane_order = 2 orders each chunk of kSortChunk records by (row count,
// width class) with a counting sort in LDS: the row count is the record's
// row range clipped to the canvas (capped at 31), the width class the
// widest span, 2 sqrt(qk / a) at the centre row, in steps of four pixels
// (capped at 7).  The order among equal keys follows the LDS atomics and
// is not fixed, which is harmless: as with the dealt order, only the lane
// that walks a record changes, never its arithmetic, and the forward sums
// are order-free integers, so every result is the same.
// ---------------------------------------------------------------------------
constexpr int kSortChunk = 1024;
constexpr int kSortKeys = 256;  // 32 row counts x 8 width classes
static_assert(kSortKeys == kBlock, "one key counter per thread");

struct SortLds {
  int start[kSortKeys];
  int wsum[kBlock / 64];
  unsigned short perm[kSortChunk];  // place -> record (within the chunk)
};

union OrderLds {
  DealLds deal;
  SortLds sort;
};

__device__ __forceinline__ void size_sort(const float4 *list, size_t base, int n, int rlo, int rhi,
                                          float qk, SortLds &d) {
  const int t = threadIdx.x;
  d.start[t] = 0;
  __syncthreads();
  constexpr int kPer = kSortChunk / kBlock;
  int key[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int g = t + j * kBlock;
    key[j] = -1;
    if (g < n) {
      const float al = list[2 * (base + g)].z;
      const int rows = __float_as_int(list[2 * (base + g) + 1].w);
      const int nr = min(rows >> 16, rhi) - max(rows & 0xffff, rlo) + 1;
      const int wc = (int)fminf(2.f * hsqrt(qk / al), 64.f) >> 2;
      const int k = min(max(nr, 0), 31) * 8 + min(wc, 7);
      key[j] = (atomicAdd(&d.start[k], 1) << 8) | k;
    }
  }
  __syncthreads();
  // exclusive scan of the key counts: wave scans, then the wave totals
  const int c = d.start[t];
  int x = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if ((t & 63) >= o) x += y;
  }
  if ((t & 63) == 63) d.wsum[t >> 6] = x;
  __syncthreads();
  int off = x - c;
  for (int w = 0; w < (t >> 6); ++w) off += d.wsum[w];
  d.start[t] = off;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kPer; ++j)
    if (key[j] >= 0) d.perm[d.start[key[j] & 255] + (key[j] >> 8)] = (unsigned short)(t + j * kBlock);
  __syncthreads();
}

// Records per ordered chunk for an item of w records, by lane_order.
__device__ __forceinline__ int chunk_len(const Geom &G, int w) {
  return G.deal == 1 ? kDealChunk : G.deal == 2 ? kSortChunk : w;
}

// Orders one chunk of records as the launch option lane_order asks and
// returns the place -> record map (null: list order).  Block-wide: every
// thread of the block calls it.
__device__ __forceinline__ const unsigned short *order_records(const float4 *list, size_t base,
                                                               int n, const Geom &G, int R0, int C0,
                                                               int rlo, int rhi, OrderLds &o) {
  if (G.deal == 1) {
    deal(list, base, n, G.S, R0, C0, o.deal);
    return o.deal.perm;
  }
  if (G.deal == 2) {
    size_sort(list, base, n, rlo, rhi, G.qk, o.sort);
    return o.sort.perm;
  }
  return nullptr;
}

// ---------------------------------------------------------------------------
// Forward: partial canvas of one work item.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_splat_fwd(MultiProb MP) {
  extern __shared__ int4 smem4[];     // 16-byte aligned dynamic LDS
  int *icanvas = (int *)smem4;        // C rows of stride S (fixed point)
  __shared__ int slot;
  __shared__ float wsum[kBlock / 64];
  __shared__ OrderLds ol;
  // drain the problems' queues in order: blocks that find one exhausted move on
  for (int p = 0; p < MP.count; ++p) {
  const Geom G = MP.p[p].G;
  const float4 *list = MP.p[p].list;
  const int4 *items = MP.p[p].items;
  float *partials = MP.p[p].partials;
  int *queue = MP.p[p].queue;
  const int nitems = *MP.p[p].n_items;
  const int CS = G.C * G.S;
  for (;;) {
    const int it = next_item(queue, &slot);
    if (it >= nitems) break;
    for (int i = threadIdx.x; i < CS / 4; i += kBlock) smem4[i] = make_int4(0, 0, 0, 0);
    for (int i = (CS & ~3) + threadIdx.x; i < CS; i += kBlock) icanvas[i] = 0;
    const int4 itm = items[it];
    // fixed-point scale: 2^e with 2^e * sum|w| <= 2^30 (the item's |w| are
    // contiguous beside the list, summed in a fixed order)
    const float *wa = MP.p[p].wabs + itm.z;
    float aw = 0.f;
    // four loads in flight per thread, added in the same order as one at a time
    int g = threadIdx.x;
    for (; g + 3 * kBlock < itm.w; g += 4 * kBlock) {
      const float a0 = wa[g], a1 = wa[g + kBlock], a2 = wa[g + 2 * kBlock], a3 = wa[g + 3 * kBlock];
      aw += a0;
      aw += a1;
      aw += a2;
      aw += a3;
    }
    for (; g < itm.w; g += kBlock) aw += wa[g];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) aw += __shfl_xor(aw, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = aw;
    __syncthreads();
    const float tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    int ex = 0;
    if (tot > 0.f && isfinite(tot)) {
      frexpf(tot, &ex);          // tot in [2^(ex-1), 2^ex)
      ex = min(max(30 - ex, -126), 126);  // 2^ex * tot < 2^30 (unless clamped)
    }
    const float scale = ldexpf(1.f, ex), inv_scale = ldexpf(1.f, -ex);
    const int ty = itm.y / G.ntx, tx = itm.y % G.ntx;
    const int R0 = ty * G.T - G.halo, C0 = tx * G.T - G.halo;
    const int rlo = max(R0, 0), rhi = min(R0 + G.C - 1, G.D - 1);
    const int clo = max(C0, 0), chi = min(C0 + G.C - 1, G.D - 1);
    __syncthreads();  // canvas cleared
    const int chunk = chunk_len(G, itm.w);
    for (int c0 = 0; c0 < itm.w; c0 += chunk) {
    const int nc = min(chunk, itm.w - c0);
    const unsigned short *perm =
        order_records(list, (size_t)itm.z + c0, nc, G, R0, C0, rlo, rhi, ol);
    for (int s = threadIdx.x; s < nc; s += kBlock) {
      const size_t rec = 2 * ((size_t)itm.z + c0 + (perm ? perm[s] : s));
      const float4 r0 = list[rec], r1 = list[rec + 1];
      const float u = r0.x, v = r0.y, al = r0.z, be = r0.w, ga = r1.x, w = r1.y * scale;
      const int rows = __float_as_int(r1.w);
      const int i0 = max(rows & 0xffff, rlo), i1 = min(rows >> 16, rhi);
      const float det_s = al * ga - be * be;
      const float inv_al = 1.f / al;
      const float aqk = al * G.qk;
      const float K = hexp2(-2.f * al);
      float fi = (float)i0;
      int rowo = (i0 - R0) * G.S - C0;  // canvas offset of (row i, column 0)
      for (int i = i0; i <= i1; ++i, fi += 1.f, rowo += G.S) {
        const float di = fi - v;
        int j0, L;
        if (!row_span(u, di, al, be, det_s, inv_al, aqk, clo, chi, j0, L)) continue;
        const float dj = (float)j0 - u;
        float e = w * hexp2(-(al * dj * dj + 2.f * be * dj * di + ga * di * di));
        float r = hexp2(-(al * (2.f * dj + 1.f) + 2.f * be * di));
        int *px = icanvas + rowo + j0;
        const int L4 = L & ~3;
        for (int k = 0; k < L4; k += 4) {
          const int v0 = __float2int_rn(e); e *= r; r *= K;
          const int v1 = __float2int_rn(e); e *= r; r *= K;
          const int v2 = __float2int_rn(e); e *= r; r *= K;
          const int v3 = __float2int_rn(e); e *= r; r *= K;
          atomicAdd(px + k, v0);
          atomicAdd(px + k + 1, v1);
          atomicAdd(px + k + 2, v2);
          atomicAdd(px + k + 3, v3);
        }
        if (L4 < L) {  // 1 to 3 trailing pixels
          const int v0 = __float2int_rn(e); e *= r; r *= K;
          const int v1 = __float2int_rn(e); e *= r;
          const int v2 = __float2int_rn(e);
          atomicAdd(px + L4, v0);
          if (L4 + 1 < L) atomicAdd(px + L4 + 1, v1);
          if (L4 + 2 < L) atomicAdd(px + L4 + 2, v2);
        }
      }
    }
    __syncthreads();  // the next chunk rewrites the order
    }
    float *out = partials + (size_t)it * G.C * G.C;
    const float inv_c = 1.f / (float)G.C;
    for (int i = threadIdx.x; i < G.C * G.C; i += kBlock) {
      const int r = row_of(i, inv_c), c = i - r * G.C;
      out[i] = (float)icanvas[r * G.S + c] * inv_scale;
    }
    __syncthreads();
  }
  }
}

// ---------------------------------------------------------------------------
// Q for one (image, tile): every pixel sums, in a fixed order, the partial
// canvases of the owner tiles whose canvas covers it (its own tile and the
// neighbours whose halo reaches it).  When tile, halo and D are multiples
// of 4, a thread takes four adjacent pixels of a row (16-byte loads) and
// keeps four items in flight.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float4 f4add(float4 a, float4 b) {
  return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}

__global__ void __launch_bounds__(kBlock)
k_canvas_reduce(const float *partials, const int *item_off, const int4 *items, Geom G,
                float *Q) {
  // XCD-aware order: a work index runs over the z-split parts of a tile,
  // then the tiles of an image, so the blocks that read one canvas (its own
  // and its neighbours' halos) meet in one XCD's L2
  const int zsplit = gridDim.z;
  const int j = xcd_work(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                         gridDim.x * gridDim.y * zsplit);
  const int zz = j % zsplit, t = (j / zsplit) % gridDim.x, b = j / (zsplit * gridDim.x);
  const int ty = t / G.ntx, tx = t % G.ntx;
  // item ranges of the 3 x 3 owner tiles around this one (empty outside the
  // image), read once per block rather than per pixel and neighbour
  __shared__ int2 range[9];
  if (threadIdx.x < 9) {
    const int sy = ty + threadIdx.x / 3 - 1, sx = tx + threadIdx.x % 3 - 1;
    int2 r = make_int2(0, 0);
    if (sy >= 0 && sy < G.ntx && sx >= 0 && sx < G.ntx) {
      const int e = b * G.K + sy * G.ntx + sx;
      r = make_int2(item_off[e], item_off[e + 1]);
    }
    range[threadIdx.x] = r;
  }
  __syncthreads();
  const int r_lo = ty * G.T, r_hi = min(r_lo + G.T, G.D);
  const int c_lo = tx * G.T, c_hi = min(c_lo + G.T, G.D);
  const int wdt = c_hi - c_lo;
  float *img = Q + (size_t)b * G.D * G.D;
  const size_t CC = (size_t)G.C * G.C;
  const bool vec = (G.T % 4 == 0) && (G.halo % 4 == 0) && (G.D % 4 == 0);
  const int px_per = vec ? 4 : 1;
  const int wq = wdt / px_per;
  const int nq = (r_hi - r_lo) * wq;
  for (int q = threadIdx.x + zz * kBlock; q < nq; q += kBlock * zsplit) {
    const int i = r_lo + q / wq, j = c_lo + px_per * (q % wq);
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int dy = -1; dy <= 1; ++dy) {
      const int sy = ty + dy;
      if (sy < 0 || sy >= G.ntx) continue;
      const int ri = i - (sy * G.T - G.halo);
      if (ri < 0 || ri >= G.C) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int sx = tx + dx;
        if (sx < 0 || sx >= G.ntx) continue;
        const int cj = j - (sx * G.T - G.halo);
        if (cj < 0 || cj >= G.C) continue;
        const int2 r = range[3 * (dy + 1) + dx + 1];
        const int it0 = r.x, it1 = r.y;
        const float *base = partials + (size_t)ri * G.C + cj;
        if (vec) {
          int it = it0;
          for (; it + 4 <= it1; it += 4) {
            const float4 a0 = *(const float4 *)(base + (size_t)it * CC);
            const float4 a1 = *(const float4 *)(base + (size_t)(it + 1) * CC);
            const float4 a2 = *(const float4 *)(base + (size_t)(it + 2) * CC);
            const float4 a3 = *(const float4 *)(base + (size_t)(it + 3) * CC);
            acc = f4add(acc, f4add(f4add(a0, a1), f4add(a2, a3)));
          }
          for (; it < it1; ++it) acc = f4add(acc, *(const float4 *)(base + (size_t)it * CC));
        } else {
          for (int it = it0; it < it1; ++it) acc.x += base[(size_t)it * CC];
        }
      }
    }
    float *o = img + (size_t)i * G.D + j;
    if (vec) {
      *(float4 *)o = acc;
    } else {
      o[0] = acc.x;
    }
  }
}

// ---------------------------------------------------------------------------
// Wide Gaussians (footprint larger than the canvas): one block per record,
// threads over the pixel box, exp per pixel, device atomics into Q.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wide_box(const float4 r0, const float4 r1, const Geom &G,
                                         int &i0, int &i1, int &j0, int &j1) {
  const int rows = __float_as_int(r1.w);
  i0 = rows & 0xffff;
  i1 = rows >> 16;
  const float det_s = r0.z * r1.x - r0.w * r0.w;
  const float hx = sqrtf(G.qk * r1.x / det_s);
  j0 = clamp_px(ceilf(r0.x - hx), 0, G.D);
  j1 = clamp_px(floorf(r0.x + hx), -1, G.D - 1);
}

// Wide records are summed in 64-bit fixed point so that the result does not
// depend on the order of the device atomics: per image, the scale is the
// power of two 2^e with 2^e * sum|w| < 2^61 over the image's wide records
// (their |w| summed in a fixed order), every term is rounded to an integer
// and the integer image is added to Q once all terms are in.
// k_big_prep: one block per image: the scale, and the integer image cleared.
__global__ void __launch_bounds__(kBlock)
k_big_prep(const int *off, const int *count, const float *wabs, Geom G, double *wscale,
           long long *wq) {
  const int b = blockIdx.x;
  const int e = b * G.K + G.ntiles;
  const int cnt = count[e], start = off[e];
  if (cnt == 0) return;
  __shared__ double red[kBlock / 64];
  double a = 0.0;
  for (int k = threadIdx.x; k < cnt; k += kBlock) a += (double)wabs[start + k];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  long long *img = wq + (size_t)b * G.D * G.D;
  for (int i = threadIdx.x; i < G.D * G.D; i += kBlock) img[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double tot = (red[0] + red[1]) + (red[2] + red[3]);
    int ex = 0;
    if (tot > 0.0) frexp(tot, &ex);  // tot < 2^ex
    wscale[b] = ldexp(1.0, 61 - ex);
  }
}

// k_big_fwd: grid row b takes image b's wide records, one block per record
// at a time, threads over its pixel box, exp per pixel, 64-bit integer
// atomics into the image's integer sum.
__global__ void __launch_bounds__(kBlock)
k_big_fwd(const float4 *list, const int *off, const int *count, const int *n_wide, Geom G,
          const double *wscale, long long *wq) {
  if (*n_wide == 0) return;
  const int b = blockIdx.y;
  const int e = b * G.K + G.ntiles;
  const int cnt = count[e], start = off[e];
  if (cnt == 0) return;
  const double S = wscale[b];
  unsigned long long *img = (unsigned long long *)(wq + (size_t)b * G.D * G.D);
  for (int k = blockIdx.x; k < cnt; k += gridDim.x) {
    const float4 r0 = list[2 * (size_t)(start + k)], r1 = list[2 * (size_t)(start + k) + 1];
    int i0, i1, j0, j1;
    wide_box(r0, r1, G, i0, i1, j0, j1);
    if (i1 < i0 || j1 < j0) continue;
    const int wdt = j1 - j0 + 1;
    const long npx = (long)(i1 - i0 + 1) * wdt;
    for (long q = threadIdx.x; q < npx; q += kBlock) {
      const int i = i0 + (int)(q / wdt), j = j0 + (int)(q % wdt);
      const float dj = (float)j - r0.x, di = (float)i - r0.y;
      const float qq = r0.z * dj * dj + 2.f * r0.w * dj * di + r1.x * di * di;
      if (qq <= G.qk) {
        const long long v = __double2ll_rn((double)(r1.y * exp2f(-qq)) * S);
        atomicAdd(&img[(size_t)i * G.D + j], (unsigned long long)v);
      }
    }
  }
}

// k_big_add: Q += integer sum / scale for images with wide records.
__global__ void __launch_bounds__(kBlock)
k_big_add(const int *count, Geom G, const double *wscale, const long long *wq, float *Q) {
  const int b = blockIdx.y;
  if (count[b * G.K + G.ntiles] == 0) return;
  const double inv = 1.0 / wscale[b];
  const size_t n = (size_t)G.D * G.D;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    const long long v = wq[(size_t)b * n + i];
    if (v) Q[(size_t)b * n + i] += (float)((double)v * inv);
  }
}

// ---------------------------------------------------------------------------
// Backward: six pixel moments per (image, Gaussian) of one work item,
//   m = sum G_Q e (1, dj, di, dj^2, dj di, di^2),  e = exp(-q/2),
// with dj = j - u, di = i - v (pixels).  Written to mom[(b N + n) 6 + k].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_splat_bwd(MultiProb MP) {
  extern __shared__ float gq[];  // C rows of stride S
  __shared__ int slot;
  __shared__ OrderLds ol;
  for (int p = 0; p < MP.count; ++p) {
  const Geom G = MP.p[p].G;
  const float4 *list = MP.p[p].list;
  const int4 *items = MP.p[p].items;
  const float *GQ = MP.p[p].GQ;
  float *mom = MP.p[p].mom;
  int *queue = MP.p[p].queue + 1;
  const int nitems = *MP.p[p].n_items;
  for (;;) {
    const int it = next_item(queue, &slot);
    if (it >= nitems) break;
    const int4 itm = items[it];
    const int b = itm.x;
    const int ty = itm.y / G.ntx, tx = itm.y % G.ntx;
    const int R0 = ty * G.T - G.halo, C0 = tx * G.T - G.halo;
    const int rlo = max(R0, 0), rhi = min(R0 + G.C - 1, G.D - 1);
    const int clo = max(C0, 0), chi = min(C0 + G.C - 1, G.D - 1);
    const float *src = GQ + (size_t)b * G.D * G.D;
    const float inv_s = 1.f / (float)G.S;
    // G_Q of the canvas region into LDS (zero outside the image and in the
    // row padding): four unconditional loads in flight per thread (outside
    // the image they read the image's first value, then dropped)
    const int CS = G.C * G.S;
    for (int q0 = threadIdx.x; q0 < CS; q0 += 4 * kBlock) {
      float v[4];
      bool ok[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + u * kBlock;
        const int r = row_of(q, inv_s), c = q - r * G.S;
        const int i = R0 + r, j = C0 + c;
        ok[u] = q < CS && c < G.C && i >= 0 && i < G.D && j >= 0 && j < G.D;
        v[u] = src[ok[u] ? (size_t)i * G.D + j : 0];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + u * kBlock;
        if (q < CS) gq[q] = ok[u] ? v[u] : 0.f;
      }
    }
    __syncthreads();
    const int chunk = chunk_len(G, itm.w);
    for (int c0 = 0; c0 < itm.w; c0 += chunk) {
    const int nc = min(chunk, itm.w - c0);
    const unsigned short *perm =
        order_records(list, (size_t)itm.z + c0, nc, G, R0, C0, rlo, rhi, ol);
    for (int s = threadIdx.x; s < nc; s += kBlock) {
      const size_t rec = 2 * ((size_t)itm.z + c0 + (perm ? perm[s] : s));
      const float4 r0 = list[rec], r1 = list[rec + 1];
      const float u = r0.x, v = r0.y, al = r0.z, be = r0.w, ga = r1.x;
      const int n = __float_as_int(r1.z);
      const int rows = __float_as_int(r1.w);
      const int i0 = max(rows & 0xffff, rlo), i1 = min(rows >> 16, rhi);
      const float det_s = al * ga - be * be;
      const float inv_al = 1.f / al;
      const float aqk = al * G.qk;
      const float K = hexp2(-2.f * al);
      float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f, m5 = 0.f;
      float fi = (float)i0;
      int rowo = (i0 - R0) * G.S - C0;  // canvas offset of (row i, column 0)
      for (int i = i0; i <= i1; ++i, fi += 1.f, rowo += G.S) {
        const float di = fi - v;
        int j0, L;
        if (!row_span(u, di, al, be, det_s, inv_al, aqk, clo, chi, j0, L)) continue;
        const float dj = (float)j0 - u;
        float e = hexp2(-(al * dj * dj + 2.f * be * dj * di + ga * di * di));
        float r = hexp2(-(al * (2.f * dj + 1.f) + 2.f * be * di));
        const float *px = gq + rowo + j0;
        // Prefix-sum moments over t_k = G_Q e, k = 0 .. M-1 (M steps, t_k = 0
        // for k >= L):
        //   a0 = sum t_k, a1 = sum t_k (M-k), a2 = sum t_k (M-k)(M-k+1)/2
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
        const int L4 = L & ~3;
        for (int k = 0; k < L4; k += 4) {
          const float g0 = px[k], g1 = px[k + 1], g2 = px[k + 2], g3 = px[k + 3];
          float t = g0 * e; e *= r; r *= K;
          a0 += t; a1 += a0; a2 += a1;
          t = g1 * e; e *= r; r *= K;
          a0 += t; a1 += a0; a2 += a1;
          t = g2 * e; e *= r; r *= K;
          a0 += t; a1 += a0; a2 += a1;
          t = g3 * e; e *= r; r *= K;
          a0 += t; a1 += a0; a2 += a1;
        }
        int M = L4;
        if (L4 < L) {
          // 1 to 3 trailing pixels as three steps with G_Q = 0 past the span.
          // The three reads are unconditional: the span ends at column C - 1
          // at most, so they reach column C + 1 at most, inside the row of
          // stride C + 4.
          const float g0 = px[L4], h1 = px[L4 + 1], h2 = px[L4 + 2];
          const float g1 = L4 + 1 < L ? h1 : 0.f;
          const float g2 = L4 + 2 < L ? h2 : 0.f;
          float t = g0 * e; e *= r; r *= K;
          a0 += t; a1 += a0; a2 += a1;
          t = g1 * e; e *= r;
          a0 += t; a1 += a0; a2 += a1;
          t = g2 * e;
          a0 += t; a1 += a0; a2 += a1;
          M = L4 + 3;
        }
        // sum t dj = c a0 - a1, sum t dj^2 = c^2 a0 - 2 c a1 + 2 a2 - a1, c = dj0 + M
        const float c = dj + (float)M;
        const float sdj = c * a0 - a1;
        const float sdj2 = c * (c * a0 - 2.f * a1) + 2.f * a2 - a1;
        m0 += a0;
        m1 += sdj;
        m2 += a0 * di;
        m3 += sdj2;
        m4 += sdj * di;
        m5 += a0 * di * di;
      }
      float *o = mom + ((size_t)b * G.N + n) * 6;
      o[0] = m0; o[1] = m1; o[2] = m2; o[3] = m3; o[4] = m4; o[5] = m5;
    }
    __syncthreads();  // the next chunk rewrites the order
    }
  }
  }
}

// Grid row b takes image b's wide records, one block per record at a time:
// per-thread moments over the pixel box, then a fixed-order block sum.
__global__ void __launch_bounds__(kBlock)
k_big_bwd(const float4 *list, const int *off, const int *count, const int *n_wide, Geom G,
          const float *GQ, float *mom) {
  __shared__ float red[6][kBlock / 64];
  if (*n_wide == 0) return;
  const int b = blockIdx.y;
  const int e = b * G.K + G.ntiles;
  const int cnt = count[e], start = off[e];
  for (int k = blockIdx.x; k < cnt; k += gridDim.x) {
    const float4 r0 = list[2 * (size_t)(start + k)], r1 = list[2 * (size_t)(start + k) + 1];
    int i0, i1, j0, j1;
    wide_box(r0, r1, G, i0, i1, j0, j1);
    float m[6] = {0, 0, 0, 0, 0, 0};
    if (i1 >= i0 && j1 >= j0) {
      const int wdt = j1 - j0 + 1;
      const long npx = (long)(i1 - i0 + 1) * wdt;
      for (long q = threadIdx.x; q < npx; q += kBlock) {
        const int i = i0 + (int)(q / wdt), j = j0 + (int)(q % wdt);
        const float dj = (float)j - r0.x, di = (float)i - r0.y;
        const float qq = r0.z * dj * dj + 2.f * r0.w * dj * di + r1.x * di * di;
        if (qq <= G.qk) {
          const float t = GQ[((size_t)b * G.D + i) * G.D + j] * exp2f(-qq);
          m[0] += t; m[1] += t * dj; m[2] += t * di;
          m[3] += t * dj * dj; m[4] += t * dj * di; m[5] += t * di * di;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      float x = m[c];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
      if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = x;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
      float x = 0.f;
      for (int wv = 0; wv < kBlock / 64; ++wv) x += red[threadIdx.x][wv];
      const int n = __float_as_int(r1.z);
      mom[((size_t)b * G.N + n) * 6 + threadIdx.x] = x;
    }
    __syncthreads();
  }
}

}  // namespace cs
