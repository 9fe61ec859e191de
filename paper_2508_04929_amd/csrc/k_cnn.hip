// Pose-proposal network kernels: BF16 MFMA GEMMs for 3x3 stride-2 convs
// (forward, data gradient, weight gradient) and linear layers, a
// 16x16x16 MFMA kernel for the single-channel first conv (its 9 taps padded
// to K = 16), the 6-D -> SO(3) head and its loss.
//
// Activations are NHWC BF16 ([B][H][W][C]); weights are [Cout][ky][kx][Cin]
// BF16 with FP32 masters.  Every GEMM accumulates in FP32 with
// v_mfma_f32_16x16x32_bf16 (gfx950): a 64x64 block tile, four waves of
// 32x32, K steps of 32 staged through LDS.  Operand tiles are gathered
// straight from the activations (implicit im2col), 16 bytes per thread.
#include "cs_cnn.hpp"

namespace cs {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ float bf2f(bf16 v) { return __uint_as_float((unsigned)v << 16); }

// 1.0 in bfloat16: what an absent ReLU mask reads
__device__ const bf16 kBf16One = 0x3f80;

// Round to nearest even (the hardware conversion, v_cvt_pk_bf16_f32).
__device__ __forceinline__ bf16 f2bf(float x) { return __builtin_bit_cast(bf16, (__bf16)x); }

// MK: K of one MFMA (and the granularity of split-K ranges); BK: K staged
// per LDS step; LDS rows padded to 80 bytes (conflict-free 16-byte reads)
constexpr int MK = 32, BK = 32, LDK = BK + 8;

union Vec8 {
  uint4 u;
  bf16 h[8];
};

// ---------------------------------------------------------------------------
// Generic split-K GEMM: C[m][n] = sum_k A[m][k] B[n][k] over k in this
// block's K range.  Op supplies the gathers and the epilogue:
//   Op::kATrans / kBTrans: false = 8 consecutive k of one row per 16-byte
//   load (ptr_a / ptr_b); true = 8 consecutive rows of one k (ptr_aT / ptr_bT).
// A gather returns the address of its 16 bytes and whether they are real
// operand values; outside the operand (image padding, past M, N or the K
// range) it returns an address that is still valid to read (the tensor's
// first element) with ok = false, and the value read is replaced by zeros
// when it is staged into LDS.  Every load is thus unconditional, so the
// compiler can count the loads in flight exactly and wait only for the one
// step being staged, keeping the prefetched steps in flight.
// ---------------------------------------------------------------------------
// One K step of an operand tile: each thread fetches 16 bytes into a
// register (prefetched while the previous step computes), then stores them
// into the LDS tile (non-transposed: 8 consecutive k of one row; transposed:
// 8 consecutive rows of one k, scattered into 8 rows).  A non-transposed
// operand keeps the same rows for the whole K loop, so each thread decodes
// its rows once (Op::row_a / row_b) and gathers with the step's base k
// (uniform across the block) plus its own offset (Op::ptr_a / ptr_b).
template <class Op, bool IS_A>
struct Gather {
  typedef typename Op::Row Row;
  __device__ static Row row(const Op &op, int r) { return IS_A ? op.row_a(r) : op.row_b(r); }
  __device__ static const uint4 *ptr(const Op &op, const Row &w, int k0, int koff, bool &ok) {
    return IS_A ? op.ptr_a(w, k0, koff, ok) : op.ptr_b(w, k0, koff, ok);
  }
};

template <class Op, int TB>
__device__ __forceinline__ uint4 fetch_trans(const Op &op, bool isA, int idx, int r0, int k0, int R,
                                             int Kend, bool &ok) {
  const int r = r0 + (idx % (TB / 8)) * 8, k = k0 + idx / (TB / 8);
  const bool in = r < R && k < Kend;
  bool okp;
  const uint4 *p = isA ? op.ptr_aT(in ? r : 0, in ? k : 0, okp) : op.ptr_bT(in ? r : 0, in ? k : 0, okp);
  ok = in && okp;
  return *p;
}

template <class Op, int TB>
__device__ __forceinline__ void put_tile(bool isA, bf16 (*tile)[LDK], int idx, uint4 v) {
  const bool trans = isA ? Op::kATrans : Op::kBTrans;
  if (!trans) {
    *(uint4 *)&tile[idx / (BK / 8)][(idx % (BK / 8)) * 8] = v;
  } else {
    Vec8 u;
    u.u = v;
    const int kk = idx / (TB / 8), rq = (idx % (TB / 8)) * 8;
#pragma unroll
    for (int i = 0; i < 8; ++i) tile[rq + i][kk] = u.h[i];
  }
}

// Per-thread operand fetch state of one side of the GEMM.
template <class Op, int TB, int NQ, bool IS_A>
struct Side {
  static constexpr bool kTrans = IS_A ? Op::kATrans : Op::kBTrans;
  typename Op::Row row[NQ];
  bool ok[NQ];
  int koff[NQ];
  __device__ void init(const Op &op, int tid, int r0, int R) {
    if constexpr (!kTrans) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int idx = tid + 256 * q, r = r0 + idx / (BK / 8);
        ok[q] = r < R;
        koff[q] = (idx % (BK / 8)) * 8;
        row[q] = Gather<Op, IS_A>::row(op, ok[q] ? r : r0);
      }
    }
  }
  // the 16 bytes of gather q at step base k0 (always read) and whether
  // they are operand values (false: to be replaced by zeros)
  __device__ uint4 fetch(const Op &op, int q, int tid, int r0, int k0, int R, int Kend,
                         bool &valid) const {
    if constexpr (kTrans) {
      return fetch_trans<Op, TB>(op, IS_A, tid + 256 * q, r0, k0, R, Kend, valid);
    } else {
      // beyond the K range the read goes to the range's last 8 columns
      // (Kend is a multiple of 8): an in-bounds address from the step base,
      // which stays uniform across the block
      const bool in = ok[q] && k0 + koff[q] < Kend;
      const int kc = k0 < Kend ? k0 : Kend - 8;
      bool okp;
      const uint4 *p = Gather<Op, IS_A>::ptr(op, row[q], kc, in ? koff[q] : 0, okp);
      valid = in && okp;
      return *p;
    }
  }
};

__device__ __forceinline__ uint4 keep_if(bool valid, uint4 v) {
  return valid ? v : make_uint4(0, 0, 0, 0);
}

// Keeps loaded values ahead of the branches that use them: without it the
// compiler sinks each load into its branch, one round trip per element.
template <int TI>
__device__ __forceinline__ void pin_loads(const float (&v)[TI][4]) {
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) asm volatile("" ::"v"(v[i][r]));
}

// TBM x TBN block tile, four waves in 2 x 2, each wave (TBM/2) x (TBN/2) as
// 16 x 16 MFMA tiles; K steps of 32 double-buffered through LDS (operands
// prefetched into registers while the current step computes).  The tile
// shape changes only the partition: every output accumulates its K steps in
// the same order, so results do not depend on it.
template <class Op, int TBM, int TBN>
__global__ void __launch_bounds__(256, 3) k_gemm(Op op, int M, int N, int K, int kchunk) {
  constexpr int TI = TBM / 32, TJ = TBN / 32;
  constexpr int NA = TBM * BK / 8 / 256, NB = TBN * BK / 8 / 256;
  static_assert(NA >= 1 && NB >= 1, "tile");
  // operand tiles; after the K loop the same memory stages the output tile
  constexpr int LDC = TBN + 8;
  constexpr int kOps = 2 * (TBM + TBN) * LDK, kOut = TBM * LDC;
  __shared__ __attribute__((aligned(16))) bf16 smem[kOps > kOut ? kOps : kOut];
  bf16 (*sA)[TBM][LDK] = (bf16 (*)[TBM][LDK])smem;
  bf16 (*sB)[TBN][LDK] = (bf16 (*)[TBN][LDK])(smem + 2 * TBM * LDK);
  const int m0 = blockIdx.x * TBM, n0 = blockIdx.y * TBN;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * (TBM / 2), wn = (w & 1) * (TBN / 2);
  f32x4 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  Side<Op, TBM, NA, true> sa;
  Side<Op, TBN, NB, false> sb;
  sa.init(op, tid, m0, M);
  sb.init(op, tid, n0, N);
  // operand registers of S consecutive K steps: a step's global loads are
  // issued S - 1 steps before it is staged into LDS, so their latency hides
  // behind that many steps of MFMA work (va / vb: validity of each gather)
  constexpr int S = 3;
  uint4 ra[S][NA], rb[S][NB];
  bool va[S][NA], vb[S][NB];
  const int nsteps = (ke - kb + BK - 1) / BK;
#pragma unroll
  for (int u = 0; u < S; ++u) {
#pragma unroll
    for (int q = 0; q < NA; ++q) ra[u][q] = sa.fetch(op, q, tid, m0, kb + u * BK, M, ke, va[u][q]);
#pragma unroll
    for (int q = 0; q < NB; ++q) rb[u][q] = sb.fetch(op, q, tid, n0, kb + u * BK, N, ke, vb[u][q]);
  }
#pragma unroll
  for (int q = 0; q < NA; ++q) put_tile<Op, TBM>(true, sA[0], tid + 256 * q, keep_if(va[0][q], ra[0][q]));
#pragma unroll
  for (int q = 0; q < NB; ++q) put_tile<Op, TBN>(false, sB[0], tid + 256 * q, keep_if(vb[0][q], rb[0][q]));
  __syncthreads();
  for (int t0 = 0; t0 < nsteps; t0 += S) {
#pragma unroll
    for (int u = 0; u < S; ++u) {
      const int t = t0 + u;
      const int cur = t & 1, k0 = kb + t * BK;
      // register slot u held step t (already in LDS): refill it with t + S,
      // past the last step too (those gathers come back invalid), so that
      // the loads issued per step never depend on a branch
#pragma unroll
      for (int q = 0; q < NA; ++q) ra[u][q] = sa.fetch(op, q, tid, m0, k0 + S * BK, M, ke, va[u][q]);
#pragma unroll
      for (int q = 0; q < NB; ++q) rb[u][q] = sb.fetch(op, q, tid, n0, k0 + S * BK, N, ke, vb[u][q]);
      if (t < nsteps) {
#pragma unroll
        for (int ks = 0; ks < BK / MK; ++ks) {
          if (k0 + ks * MK >= ke) break;  // past the end of this K range: nothing to add
          bf16x8 af[TI], bv[TJ];
#pragma unroll
          for (int i = 0; i < TI; ++i)
            af[i] = *(const bf16x8 *)&sA[cur][wm + i * 16 + (lane & 15)][ks * MK + (lane >> 4) * 8];
#pragma unroll
          for (int j = 0; j < TJ; ++j)
            bv[j] = *(const bf16x8 *)&sB[cur][wn + j * 16 + (lane & 15)][ks * MK + (lane >> 4) * 8];
#pragma unroll
          for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bv[j], acc[i][j], 0, 0, 0);
        }
        if (t + 1 < nsteps) {
          const int un = (u + 1) % S;  // a constant once the loop is unrolled
#pragma unroll
          for (int q = 0; q < NA; ++q)
            put_tile<Op, TBM>(true, sA[cur ^ 1], tid + 256 * q, keep_if(va[un][q], ra[un][q]));
#pragma unroll
          for (int q = 0; q < NB; ++q)
            put_tile<Op, TBN>(false, sB[cur ^ 1], tid + 256 * q, keep_if(vb[un][q], rb[un][q]));
        }
      }
      __syncthreads();
    }
  }
  if constexpr (Op::kStaged) {
    // epilogue through LDS: values (bias / ReLU / mask applied per element)
    // rounded to bfloat16 into an output tile, then written as 16-byte rows
    // (N is a multiple of 8); the optional FP32 copy is stored per element
    bf16 (*sC)[LDC] = (bf16 (*)[LDC])smem;
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int nl = wn + j * 16 + (lane & 15), n = n0 + nl;
      const float cv = n < N ? op.col(n) : 0.f;
      // the column's per-element epilogue inputs, requested together (at
      // clamped indices, so no load waits behind a branch)
      float ein[TI][4];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
          ein[i][r] = op.epi_in(min(m, M - 1), min(n, N - 1));
        }
      pin_loads(ein);
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ml = wm + i * 16 + (lane >> 4) * 4 + r, m = m0 + ml;
          float v = 0.f;
          if (m < M && n < N) {
            v = op.epi(acc[i][j][r], cv, ein[i][r]);
            if (op.f32_out()) op.f32_out()[(size_t)m * op.ldo() + n] = v;
          }
          sC[ml][nl] = f2bf(v);
        }
    }
    __syncthreads();
    bf16 *out = op.bf16_out();
    const int64_t ldo = op.ldo();
    for (int e = tid; e < TBM * TBN / 8; e += 256) {
      const int ml = e / (TBN / 8), nl = (e % (TBN / 8)) * 8;
      const int m = m0 + ml, n = n0 + nl;
      if (m < M && n < N) *(uint4 *)&out[(size_t)m * ldo + n] = *(const uint4 *)&sC[ml][nl];
    }
  } else {
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int n = n0 + wn + j * 16 + (lane & 15);
      float ein[TI][4];  // as in the staged epilogue
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
          ein[i][r] = op.epi_in(min(m, M - 1), min(n, N - 1));
        }
      pin_loads(ein);
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
          if (m < M && n < N) op.store(m, n, acc[i][j][r], blockIdx.z, ein[i][r]);
        }
    }
  }
}


// ---------------------------------------------------------------------------
// 3x3 stride-2 pad-1 convolution as GEMMs (NHWC, Cin and Cout multiples of 8)
// ---------------------------------------------------------------------------
struct ConvGeom {
  int B, Hi, Wi, Cin, Ho, Wo, Cout;
};

// forward: M = B Ho Wo, N = Cout, K = 9 Cin (k = tap * Cin + ci)
struct ConvFwdOp {
  static constexpr bool kATrans = false, kBTrans = false;
  ConvGeom g;
  int tap_uniform;  // Cin % BK == 0: a K step stays within one tap
  const bf16 *in, *w;
  const float *bias;
  bf16 *out;
  float *out32;
  int relu;
  struct Row {
    int64_t off;
    int y, x;
  };
  // output pixel m = (b, oy, ox): the top-left input corner of its window
  __device__ Row row_a(int m) const {
    const int ox = m % g.Wo, t = m / g.Wo, oy = t % g.Ho, b = t / g.Ho;
    Row r;
    r.y = 2 * oy - 1;
    r.x = 2 * ox - 1;
    r.off = (((int64_t)b * g.Hi + r.y) * g.Wi + r.x) * g.Cin;
    return r;
  }
  __device__ const uint4 *ptr_a(const Row &r, int k0, int koff, bool &ok) const {
    int tap, ci;
    if (tap_uniform) {
      tap = k0 / g.Cin;
      ci = k0 - tap * g.Cin + koff;
    } else {
      const int k = k0 + koff;
      tap = k / g.Cin;
      ci = k - tap * g.Cin;
    }
    const int dy = tap / 3, dx = tap - 3 * dy;
    const int iy = r.y + dy, ix = r.x + dx;
    ok = (unsigned)iy < (unsigned)g.Hi && (unsigned)ix < (unsigned)g.Wi;
    return (const uint4 *)(ok ? &in[r.off + ((int64_t)dy * g.Wi + dx) * g.Cin + ci] : in);
  }
  __device__ Row row_b(int n) const { return Row{(int64_t)n * 9 * g.Cin, 0, 0}; }
  __device__ const uint4 *ptr_b(const Row &r, int k0, int koff, bool &ok) const {
    ok = true;
    return (const uint4 *)&w[r.off + k0 + koff];
  }
  static constexpr bool kStaged = true;
  __device__ float col(int n) const { return bias ? bias[n] : 0.f; }
  __device__ float epi_in(int, int) const { return 0.f; }
  __device__ float epi(float v, float cv, float) const {
    v += cv;
    return relu ? fmaxf(v, 0.f) : v;
  }
  __device__ bf16 *bf16_out() const { return out; }
  __device__ float *f32_out() const { return out32; }
  __device__ int64_t ldo() const { return g.Cout; }
};

// data gradient: M = B Hi Wi, N = Cin, K = 9 Cout (k = tap * Cout + co);
// wt is the weight transposed to [Cin][tap][Cout]; the epilogue applies
// the ReLU mask of the layer's input activation (act_in > 0).
struct ConvDgradOp {
  static constexpr bool kATrans = false, kBTrans = false;
  ConvGeom g;
  int tap_uniform;  // Cout % BK == 0
  const bf16 *dout, *wt, *act_in;
  bf16 *din;
  float *din32;
  struct Row {
    int64_t off;
    int y, x;
  };
  // input pixel m = (b, iy, ix)
  __device__ Row row_a(int m) const {
    const int ix = m % g.Wi, t = m / g.Wi, iy = t % g.Hi, b = t / g.Hi;
    return Row{(int64_t)b * g.Ho * g.Wo * g.Cout, iy, ix};
  }
  __device__ const uint4 *ptr_a(const Row &r, int k0, int koff, bool &ok) const {
    int tap, co;
    if (tap_uniform) {
      tap = k0 / g.Cout;
      co = k0 - tap * g.Cout + koff;
    } else {
      const int k = k0 + koff;
      tap = k / g.Cout;
      co = k - tap * g.Cout;
    }
    const int dy = tap / 3, dx = tap - 3 * dy;
    const int oy2 = r.y + 1 - dy, ox2 = r.x + 1 - dx;
    const int oy = oy2 >> 1, ox = ox2 >> 1;
    ok = oy2 >= 0 && ox2 >= 0 && !(oy2 & 1) && !(ox2 & 1) && oy < g.Ho && ox < g.Wo;
    return (const uint4 *)(ok ? &dout[r.off + ((int64_t)oy * g.Wo + ox) * g.Cout + co] : dout);
  }
  __device__ Row row_b(int n) const { return Row{(int64_t)n * 9 * g.Cout, 0, 0}; }
  __device__ const uint4 *ptr_b(const Row &r, int k0, int koff, bool &ok) const {
    ok = true;
    return (const uint4 *)&wt[r.off + k0 + koff];
  }
  static constexpr bool kStaged = true;
  __device__ float col(int) const { return 0.f; }
  // the input activation (1 without a mask): the gradient passes where it
  // is > 0; a pointer select, not a branch, so the loads need no branch
  __device__ float epi_in(int m, int n) const {
    return bf2f(*(act_in ? act_in + (size_t)m * g.Cin + n : &kBf16One));
  }
  __device__ float epi(float v, float, float a) const { return a > 0.f ? v : 0.f; }
  __device__ bf16 *bf16_out() const { return din; }
  __device__ float *f32_out() const { return din32; }
  __device__ int64_t ldo() const { return g.Cin; }
};

// weight gradient: M = Cout, N = 9 Cin (n = tap * Cin + ci), K = B Ho Wo
// pixels; split-K partials part[z][M][N] (FP32).
struct ConvWgradOp {
  static constexpr bool kATrans = true, kBTrans = true;
  ConvGeom g;
  const bf16 *dout, *in;
  float *part;
  struct Row {};
  // 8 consecutive output channels of pixel p
  __device__ const uint4 *ptr_aT(int m, int p, bool &ok) const {
    ok = true;
    return (const uint4 *)&dout[(size_t)p * g.Cout + m];
  }
  // 8 consecutive (tap, ci) columns of the im2col row of pixel p
  __device__ const uint4 *ptr_bT(int n, int p, bool &ok) const {
    const int ox = p % g.Wo, t = p / g.Wo, oy = t % g.Ho, b = t / g.Ho;
    const int tap = n / g.Cin, ci = n - tap * g.Cin;
    const int iy = 2 * oy + tap / 3 - 1, ix = 2 * ox + tap % 3 - 1;
    ok = iy >= 0 && iy < g.Hi && ix >= 0 && ix < g.Wi;
    return (const uint4 *)(ok ? &in[(((size_t)b * g.Hi + iy) * g.Wi + ix) * g.Cin + ci] : in);
  }
  static constexpr bool kStaged = false;
  __device__ float epi_in(int, int) const { return 0.f; }
  __device__ void store(int m, int n, float v, int z, float) const {
    part[((size_t)z * g.Cout + m) * 9 * g.Cin + n] = v;
  }
};

// ---------------------------------------------------------------------------
// Linear layers: y[b][o] = sum_i W[o][i] x[b][i] + bias[o]
// ---------------------------------------------------------------------------
struct LinGeom {
  int B, In, Out;
};

struct LinRow {
  int64_t off;
};

struct LinFwdOp {  // M = B, N = Out, K = In
  static constexpr bool kATrans = false, kBTrans = false;
  LinGeom g;
  const bf16 *x, *w;
  const float *bias;
  bf16 *y;
  float *y32;
  int relu;
  typedef LinRow Row;
  __device__ Row row_a(int m) const { return Row{(int64_t)m * g.In}; }
  __device__ Row row_b(int n) const { return Row{(int64_t)n * g.In}; }
  __device__ const uint4 *ptr_a(const Row &r, int k0, int koff, bool &ok) const {
    ok = true;
    return (const uint4 *)&x[r.off + k0 + koff];
  }
  __device__ const uint4 *ptr_b(const Row &r, int k0, int koff, bool &ok) const {
    ok = true;
    return (const uint4 *)&w[r.off + k0 + koff];
  }
  static constexpr bool kStaged = false;
  __device__ float epi_in(int, int) const { return 0.f; }
  __device__ void store(int m, int n, float v, int, float) const {
    v += bias ? bias[n] : 0.f;
    if (relu) v = fmaxf(v, 0.f);
    const size_t o = (size_t)m * g.Out + n;
    if (y32) y32[o] = v;
    if (y) y[o] = f2bf(v);
  }
};

struct LinDgradOp {  // M = B, N = In, K = Out; wt = W^T [In][Out]
  static constexpr bool kATrans = false, kBTrans = false;
  LinGeom g;
  const bf16 *dy, *wt, *x_act;
  bf16 *dx;
  float *dx32;
  typedef LinRow Row;
  __device__ Row row_a(int m) const { return Row{(int64_t)m * g.Out}; }
  __device__ Row row_b(int n) const { return Row{(int64_t)n * g.Out}; }
  __device__ const uint4 *ptr_a(const Row &r, int k0, int koff, bool &ok) const {
    ok = true;
    return (const uint4 *)&dy[r.off + k0 + koff];
  }
  __device__ const uint4 *ptr_b(const Row &r, int k0, int koff, bool &ok) const {
    ok = true;
    return (const uint4 *)&wt[r.off + k0 + koff];
  }
  static constexpr bool kStaged = false;
  // the layer's input activation (1 without a mask): the gradient passes
  // where it is > 0 (a pointer select, as in ConvDgradOp)
  __device__ float epi_in(int m, int n) const {
    return bf2f(*(x_act ? x_act + (size_t)m * g.In + n : &kBf16One));
  }
  __device__ void store(int m, int n, float v, int, float a) const {
    const size_t o = (size_t)m * g.In + n;
    if (!(a > 0.f)) v = 0.f;
    if (dx32) dx32[o] = v;
    dx[o] = f2bf(v);
  }
};

struct LinWgradOp {  // M = Out, N = In, K = B; split-K partials
  static constexpr bool kATrans = true, kBTrans = true;
  LinGeom g;
  const bf16 *dy, *x;
  float *part;
  struct Row {};
  __device__ const uint4 *ptr_aT(int m, int b, bool &ok) const {
    ok = true;
    return (const uint4 *)&dy[(size_t)b * g.Out + m];
  }
  __device__ const uint4 *ptr_bT(int n, int b, bool &ok) const {
    ok = true;
    return (const uint4 *)&x[(size_t)b * g.In + n];
  }
  static constexpr bool kStaged = false;
  __device__ float epi_in(int, int) const { return 0.f; }
  __device__ void store(int m, int n, float v, int z, float) const {
    part[((size_t)z * g.Out + m) * g.In + n] = v;
  }
};

// Sum of split-K partials in a fixed order: out[i] = sum_z part[z][i].
__global__ void __launch_bounds__(256)
k_splitk_reduce(const float *part, int splits, int64_t n, float *out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  // loads issued 8 ahead, added in split order
  float s = 0.f;
  int z = 0;
  for (; z + 8 <= splits; z += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(z + u) * n + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; z < splits; ++z) s += part[(size_t)z * n + i];
  out[i] = s;
}

// Column sums of an [M][N] BF16 gradient (bias gradients): partials over
// row chunks part[chunk][N], then a fixed-order reduce.
__global__ void __launch_bounds__(256)
k_colsum(const bf16 *g, int M, int N, int rows_per_chunk, float *part) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const int r0 = blockIdx.y * rows_per_chunk, r1 = min(M, r0 + rows_per_chunk);
  float s = 0.f;
  int m = r0;
  for (; m + 8 <= r1; m += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = bf2f(g[(size_t)(m + u) * N + n]);
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; m < r1; ++m) s += bf2f(g[(size_t)m * N + n]);
  part[(size_t)blockIdx.y * N + n] = s;
}

// out[0] = sum of n partials (fixed order).
__global__ void k_sum_into(const float *part, int n, float *out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    out[0] = (float)s;
  }
}

// ---------------------------------------------------------------------------
// First conv (Cin = 1) on MFMA (v_mfma_f32_16x16x16_bf16): output rows = 16
// channels, columns = 16 output pixels, K = the 9 taps padded with zeros to
// 16.  Lane l holds taps 4 (l >> 4) .. 4 (l >> 4) + 3 of channel (A) or
// pixel (B) l & 15; its result rows are the four consecutive channels
// 4 (l >> 4) .. + 3 of pixel l & 15.  The accumulator starts at the bias.
// The inference kernel below computes the first layer with these same
// fragments, so both produce the same bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bf16x4 conv1_wfrag(const bf16 *w, int Cout, int c0, int lane) {
  const int c = c0 + (lane & 15), kq = 4 * (lane >> 4);
  bf16x4 f;
#pragma unroll
  for (int e = 0; e < 4; ++e) f[e] = (c < Cout && kq + e < 9) ? (short)w[c * 9 + kq + e] : (short)0;
  return f;
}

__device__ __forceinline__ f32x4 conv1_bias(const float *bias, int Cout, int c0, int lane) {
  f32x4 b;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int c = c0 + 4 * (lane >> 4) + r;
    b[r] = (bias && c < Cout) ? bias[c] : 0.f;
  }
  return b;
}

// One wave per 16 output pixels, all channel tiles; Cout a multiple of 8.
__global__ void __launch_bounds__(256)
k_conv1_fwd(const bf16 *in, const bf16 *w, const float *bias, int B, int Hi, int Wi, int Cout,
            int relu, bf16 *out, float *out32) {
  const int lane = threadIdx.x & 63;
  const int Ho = Hi / 2, Wo = Wi / 2;
  const int64_t np = (int64_t)B * Ho * Wo;
  const int64_t p = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 + (lane & 15);
  const bool live = p < np;
  const int kq = 4 * (lane >> 4);
  bf16x4 x;
  {
    const int64_t pc = live ? p : 0;
    const int ox = (int)(pc % Wo), t = (int)(pc / Wo), oy = t % Ho, b = t / Ho;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int tap = kq + e;
      const int iy = 2 * oy + tap / 3 - 1, ix = 2 * ox + tap % 3 - 1;
      x[e] = (tap < 9 && iy >= 0 && iy < Hi && ix >= 0 && ix < Wi)
                 ? (short)in[((size_t)b * Hi + iy) * Wi + ix] : (short)0;
    }
  }
  for (int c0 = 0; c0 < Cout; c0 += 16) {
    f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(conv1_wfrag(w, Cout, c0, lane), x,
                                                          conv1_bias(bias, Cout, c0, lane), 0, 0, 0);
    const int c = c0 + kq;  // four consecutive channels of pixel p
    if (!live || c >= Cout) continue;
    bf16x4 o;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float v = relu ? fmaxf(acc[r], 0.f) : acc[r];
      if (out32) out32[p * Cout + c + r] = v;
      o[r] = (short)f2bf(v);
    }
    *(bf16x4 *)&out[p * Cout + c] = o;
  }
}

// First-conv weight gradient partials: part[blk][co][tap] over a chunk of
// pix_per_block (<= 256) output pixels.  The chunk's 3x3 input patches and
// gradient rows are staged in LDS once; each (co, tap) then sums over the
// chunk's pixels in pixel order.
__global__ void __launch_bounds__(256)
k_conv1_wgrad(const bf16 *in, const bf16 *dpre, int B, int Hi, int Wi, int Cout,
              int pix_per_block, float *part) {
  __shared__ float xs[256][9];
  __shared__ float gs[256 * 32];  // Cout <= 32 gradient values per pixel
  const int Ho = Hi / 2, Wo = Wi / 2;
  const int64_t npix = (int64_t)B * Ho * Wo;
  const int64_t p0 = (int64_t)blockIdx.x * pix_per_block;
  const int np = (int)min((int64_t)pix_per_block, npix - p0);
  for (int q = threadIdx.x; q < np * 9; q += 256) {
    const int pl = q / 9, tap = q - pl * 9;
    const int64_t p = p0 + pl;
    const int ox = (int)(p % Wo), t = (int)(p / Wo), oy = t % Ho, b = t / Ho;
    const int iy = 2 * oy + tap / 3 - 1, ix = 2 * ox + tap % 3 - 1;
    xs[pl][tap] = (iy >= 0 && iy < Hi && ix >= 0 && ix < Wi) ? bf2f(in[((size_t)b * Hi + iy) * Wi + ix]) : 0.f;
  }
  for (int q = threadIdx.x; q < np * Cout; q += 256) gs[q] = bf2f(dpre[p0 * Cout + q]);
  __syncthreads();
  for (int ct = threadIdx.x; ct < Cout * 9; ct += 256) {
    const int co = ct / 9, tap = ct % 9;
    float s = 0.f;
    for (int pl = 0; pl < np; ++pl) s += gs[pl * Cout + co] * xs[pl][tap];
    part[(size_t)blockIdx.x * Cout * 9 + ct] = s;
  }
}

// ---------------------------------------------------------------------------
// Inference: the first two convolutions fused (C1 = 32 first-layer channels,
// C2 = 64 second-layer channels).  A block owns 8 x 16 second-layer output
// pixels of one image: it stages the 35 x 67 input patch, computes the
// 17 x 33 x 32 first-layer patch once into LDS (the MFMA fragments of
// k_conv1_fwd, so the values are identical), then runs the second
// layer on MFMA with A fragments read from the LDS patch (im2col addressing,
// one tap per K slice of 32 channels) and B fragments (weights) loaded from
// global memory straight into registers.  The first layer's activation never
// goes to HBM.
// ---------------------------------------------------------------------------
constexpr int C12_PY = 17, C12_PX = 33, C12_IY = 35, C12_IX = 67, C12_PS = 36;

__global__ void __launch_bounds__(256)
k_conv12_fwd(const bf16 *in0, const bf16 *w1, const float *b1, const bf16 *w2, const float *b2,
             int H0, bf16 *out) {
  __shared__ float xin[C12_IY * C12_IX];
  // first-layer outputs [y][x][c], pixels C12_PS bf16 apart: 8 consecutive
  // lanes read pixels 2 apart, which then fall on different banks
  __shared__ __attribute__((aligned(16))) bf16 a1[C12_PY * C12_PX * C12_PS];
  const int H1 = H0 / 2, H2 = H1 / 2;
  const int tiles_x = H2 / 16;
  const int b = blockIdx.y;
  const int oy0 = (blockIdx.x / tiles_x) * 8, ox0 = (blockIdx.x % tiles_x) * 16;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int cq = (lane >> 4) * 8;
  // wave wv computes output channels [16 wv, 16 wv + 16) for all 128 pixels;
  // its weight fragments for the 9 taps are requested now and arrive while
  // the first layer is computed
  bf16x8 bw[9];
#pragma unroll
  for (int t = 0; t < 9; ++t)
    bw[t] = *(const bf16x8 *)&w2[(size_t)(wv * 16 + (lane & 15)) * 288 + t * 32 + cq];
  // first-layer weight fragments and biases of the two channel tiles
  const bf16x4 wf0 = conv1_wfrag(w1, 32, 0, lane), wf1 = conv1_wfrag(w1, 32, 16, lane);
  const f32x4 bf0 = conv1_bias(b1, 32, 0, lane), bf1 = conv1_bias(b1, 32, 16, lane);
  // input patch rows 4 oy0 - 3 .., columns 4 ox0 - 3 .. 4 ox0 + 63: 16-byte
  // loads of the aligned columns 4 ox0 - 8 .. 4 ox0 + 63 (9 per row)
  // (both loads of a thread are issued before either is used: outside the
  // image they read the tensor's first 16 bytes, replaced by zeros)
  const int iy0 = 4 * oy0 - 3, cx0 = 4 * ox0 - 8;
  static_assert(C12_IY * 9 <= 2 * 256, "two patch loads per thread");
  uint4 pv[2];
  bool pok[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int q = tid + 256 * h;
    const int ry = q / 9, t = q - ry * 9;
    const int yy = iy0 + ry, xx = cx0 + 8 * t;
    pok[h] = q < C12_IY * 9 && yy >= 0 && yy < H0 && xx >= 0 && xx < H0;
    pv[h] = *(const uint4 *)(pok[h] ? &in0[((size_t)b * H0 + yy) * H0 + xx] : in0);
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int q = tid + 256 * h;
    if (q >= C12_IY * 9) continue;
    const int ry = q / 9, t = q - ry * 9;
    Vec8 v;
    v.u = pok[h] ? pv[h] : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = 8 * t + e - 5;  // patch column of input column xx + e
      if (c >= 0 && c < C12_IX) xin[ry * C12_IX + c] = bf2f(v.h[e]);
    }
  }
  __syncthreads();
  // first layer at patch positions (y, x) = first-layer rows 2 oy0 - 1 + y,
  // columns 2 ox0 - 1 + x: 16 positions per MFMA column tile, wave wv takes
  // tiles wv, wv + 4, ...; positions outside the first-layer image are 0
  {
    const int kq = 4 * (lane >> 4);
    for (int tile = wv; tile * 16 < C12_PY * C12_PX; tile += 4) {
      const int pos = tile * 16 + (lane & 15);
      const int pc = min(pos, C12_PY * C12_PX - 1);
      const int y = pc / C12_PX, x = pc - y * C12_PX;
      bf16x4 xf;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int tap = kq + e;
        xf[e] = tap < 9 ? (short)f2bf(xin[(2 * y + tap / 3) * C12_IX + 2 * x + tap % 3]) : (short)0;
      }
      const f32x4 r0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wf0, xf, bf0, 0, 0, 0);
      const f32x4 r1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wf1, xf, bf1, 0, 0, 0);
      if (pos < C12_PY * C12_PX) {
        const int y1 = 2 * oy0 - 1 + y, x1 = 2 * ox0 - 1 + x;
        const bool in_img = y1 >= 0 && y1 < H1 && x1 >= 0 && x1 < H1;
        bf16x4 o0, o1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          o0[r] = in_img ? (short)f2bf(fmaxf(r0[r], 0.f)) : (short)0;
          o1[r] = in_img ? (short)f2bf(fmaxf(r1[r], 0.f)) : (short)0;
        }
        *(bf16x4 *)&a1[pos * C12_PS + kq] = o0;
        *(bf16x4 *)&a1[pos * C12_PS + 16 + kq] = o1;
      }
    }
  }
  __syncthreads();  // the whole first-layer patch is in LDS (every wave reads all of it)
  // second layer: MFMA row tiles i = pixels [16 i, 16 i + 16) of the 8 x 16
  // tile (one output row each), columns = this wave's 16 channels
  f32x4 acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int ky = tap / 3, kx = tap % 3;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int y = 2 * i + ky, x = 2 * (lane & 15) + kx;
      const uint2 *src = (const uint2 *)&a1[(y * C12_PX + x) * C12_PS + cq];
      Vec8 a;
      const uint2 lo = src[0], hi = src[1];
      a.u = make_uint4(lo.x, lo.y, hi.x, hi.y);
      bf16x8 af;
      __builtin_memcpy(&af, &a, 16);
      acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bw[tap], acc[i], 0, 0, 0);
    }
  }
  // output tile [128 pixels][64 channels] staged in the first-layer buffer,
  // then written as 16-byte chunks (each output row of 16 pixels is 2 KiB
  // of contiguous NHWC memory)
  const int n = wv * 16 + (lane & 15);
  const float bn = b2 ? b2[n] : 0.f;
  __syncthreads();
  bf16 *sc = a1;  // [128][72]
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) sc[(i * 16 + (lane >> 4) * 4 + r) * 72 + n] = f2bf(fmaxf(acc[i][r] + bn, 0.f));
  __syncthreads();
  for (int e = tid; e < 128 * 8; e += 256) {
    const int m = e >> 3, c8 = (e & 7) * 8;
    const int oy = oy0 + (m >> 4), ox = ox0 + (m & 15);
    *(uint4 *)&out[(((size_t)b * H2 + oy) * H2 + ox) * 64 + c8] = *(const uint4 *)&sc[m * 72 + c8];
  }
}

// ---------------------------------------------------------------------------
// Input standardisation: x = (img - mean) / std per image, to BF16.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_standardize(const float *img, int npx, bf16 *out) {
  __shared__ double red[2][4];
  const int b = blockIdx.x;
  const float *x = img + (size_t)b * npx;
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
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s;
    red[1][threadIdx.x >> 6] = s2;
  }
  __syncthreads();
  const double m = (red[0][0] + red[0][1] + red[0][2] + red[0][3]) / npx;
  const double var = (red[1][0] + red[1][1] + red[1][2] + red[1][3]) / npx - m * m;
  const float inv = var > 0.0 ? (float)(1.0 / sqrt(var)) : 1.f;
  for (int i = threadIdx.x; i < npx; i += 256) out[(size_t)b * npx + i] = f2bf((x[i] - (float)m) * inv);
}

// ---------------------------------------------------------------------------
// Head: 6-D representation -> rotation by Gram-Schmidt (columns b1, b2,
// b1 x b2), 2-D shift; loss ||R^ - R||_F^2 + lambda ||t^ - t||^2 averaged
// over the batch, and its gradient w.r.t. the 8 network outputs.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cross3(const float a[3], const float b[3], float c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ float dot3(const float a[3], const float b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ void gram_schmidt(const float *o, float b1[3], float b2[3], float b3[3], float &n1,
                             float &n2, float u2[3]) {
  const float a1[3] = {o[0], o[1], o[2]}, a2[3] = {o[3], o[4], o[5]};
  n1 = fmaxf(sqrtf(dot3(a1, a1)), 1e-12f);
  for (int k = 0; k < 3; ++k) b1[k] = a1[k] / n1;
  const float d = dot3(b1, a2);
  for (int k = 0; k < 3; ++k) u2[k] = a2[k] - d * b1[k];
  n2 = fmaxf(sqrtf(dot3(u2, u2)), 1e-12f);
  for (int k = 0; k < 3; ++k) b2[k] = u2[k] / n2;
  cross3(b1, b2, b3);
}

__global__ void __launch_bounds__(256)
k_head(const float *out8, int B, float *rot, float *shift) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  float b1[3], b2[3], b3[3], u2[3], n1, n2;
  gram_schmidt(out8 + 8 * b, b1, b2, b3, n1, n2, u2);
  for (int r = 0; r < 3; ++r) {
    rot[9 * b + 3 * r + 0] = b1[r];
    rot[9 * b + 3 * r + 1] = b2[r];
    rot[9 * b + 3 * r + 2] = b3[r];
  }
  if (shift) {
    shift[2 * b] = out8[8 * b + 6];
    shift[2 * b + 1] = out8[8 * b + 7];
  }
}

__global__ void __launch_bounds__(256)
k_head_loss(const float *out8, const float *rot_t, const float *shift_t, int B, float lambda,
            float *loss_part, bf16 *dout8, float *dout32) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  float l = 0.f;
  if (b < B) {
    const float *o = out8 + 8 * b;
    float b1[3], b2[3], b3[3], u2[3], n1, n2;
    gram_schmidt(o, b1, b2, b3, n1, n2, u2);
    const float *R = rot_t + 9 * b;
    const float inv_b = 1.f / (float)B;
    float g1[3], g2[3], g3[3];
    for (int r = 0; r < 3; ++r) {
      const float e1 = b1[r] - R[3 * r], e2 = b2[r] - R[3 * r + 1], e3 = b3[r] - R[3 * r + 2];
      l += e1 * e1 + e2 * e2 + e3 * e3;
      g1[r] = 2.f * e1 * inv_b;
      g2[r] = 2.f * e2 * inv_b;
      g3[r] = 2.f * e3 * inv_b;
    }
    // b3 = b1 x b2
    float t[3];
    cross3(b2, g3, t);
    for (int k = 0; k < 3; ++k) g1[k] += t[k];
    cross3(g3, b1, t);
    for (int k = 0; k < 3; ++k) g2[k] += t[k];
    // b2 = u2 / |u2|
    float gu[3];
    const float p2 = dot3(b2, g2);
    for (int k = 0; k < 3; ++k) gu[k] = (g2[k] - b2[k] * p2) / n2;
    // u2 = a2 - (b1 . a2) b1
    const float a2[3] = {o[3], o[4], o[5]};
    const float bu = dot3(b1, gu), ba = dot3(b1, a2);
    float ga2[3];
    for (int k = 0; k < 3; ++k) {
      ga2[k] = gu[k] - b1[k] * bu;
      g1[k] -= ba * gu[k] + bu * a2[k];
    }
    // b1 = a1 / |a1|
    float ga1[3];
    const float p1 = dot3(b1, g1);
    for (int k = 0; k < 3; ++k) ga1[k] = (g1[k] - b1[k] * p1) / n1;
    float d[8];
    for (int k = 0; k < 3; ++k) {
      d[k] = ga1[k];
      d[3 + k] = ga2[k];
    }
    for (int k = 0; k < 2; ++k) {
      const float e = o[6 + k] - shift_t[2 * b + k];
      l += lambda * e * e;
      d[6 + k] = 2.f * lambda * e * inv_b;
    }
    for (int k = 0; k < 8; ++k) {
      dout8[8 * b + k] = f2bf(d[k]);
      if (dout32) dout32[8 * b + k] = d[k];
    }
  }
  // per-block partial of the batch loss (fixed order)
  __shared__ float red[4];
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) l += __shfl_xor(l, s, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) loss_part[blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) / (float)B;
}

// FP32 master weights -> BF16 weights and, optionally, the BF16 transpose
// [Cin][tap][Cout] (from [Cout][tap][Cin]; taps = 1 for linear layers).
__global__ void __launch_bounds__(256)
k_to_bf16(const float *w, int Cout, int taps, int Cin, bf16 *wb, bf16 *wt) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = (int64_t)Cout * taps * Cin;
  if (i >= n) return;
  const bf16 v = f2bf(w[i]);
  wb[i] = v;
  if (wt) {
    const int ci = (int)(i % Cin), tap = (int)((i / Cin) % taps), co = (int)(i / ((int64_t)Cin * taps));
    wt[((size_t)ci * taps + tap) * Cout + co] = v;
  }
}

__global__ void __launch_bounds__(256) k_f32_to_bf16(const float *x, int64_t n, bf16 *y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

__global__ void __launch_bounds__(256) k_bf16_to_f32(const bf16 *x, int64_t n, float *y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = bf2f(x[i]);
}

// ---------------------------------------------------------------------------
// Host-side launchers (declared in cs_cnn.hpp)
// ---------------------------------------------------------------------------
static unsigned cdiv_(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <class Op>
static hipError_t launch_gemm(const Op &op, int M, int N, int K, int splits, hipStream_t st) {
  int kchunk = K;
  if (splits > 1) {
    kchunk = (int)(((int64_t)K + splits - 1) / splits);
    kchunk = (kchunk + MK - 1) / MK * MK;
    splits = (K + kchunk - 1) / kchunk;
  }
  // larger tiles where there are enough of them to fill the chip
  if (splits == 1 && M >= 16384 && N >= 128) {
    hipLaunchKernelGGL((k_gemm<Op, 128, 128>), dim3(cdiv_(M, 128), cdiv_(N, 128), 1), dim3(256), 0,
                       st, op, M, N, K, kchunk);
  } else if (splits == 1 && M >= 16384 && N >= 64) {
    hipLaunchKernelGGL((k_gemm<Op, 128, 64>), dim3(cdiv_(M, 128), cdiv_(N, 64), 1), dim3(256), 0,
                       st, op, M, N, K, kchunk);
  } else {
    hipLaunchKernelGGL((k_gemm<Op, 64, 64>), dim3(cdiv_(M, 64), cdiv_(N, 64), splits), dim3(256), 0,
                       st, op, M, N, K, kchunk);
  }
  return hipGetLastError();
}

int wgrad_splits(int M, int N, int K) {
  const int tiles = (int)(cdiv_(M, 64) * cdiv_(N, 64));
  int s = (512 + tiles - 1) / tiles;
  s = std::max(1, std::min(s, K / MK));
  return s;
}

hipError_t conv_fwd(const bf16 *in, const bf16 *w, const float *bias, int B, int Hi, int Wi,
                    int Cin, int Cout, int relu, bf16 *out, float *out32, hipStream_t st) {
  if (Cin == 1) {
    const int64_t np = (int64_t)B * (Hi / 2) * (Wi / 2);
    hipLaunchKernelGGL(k_conv1_fwd, dim3(cdiv_(np, 64)), dim3(256), 0, st, in, w, bias, B, Hi, Wi,
                       Cout, relu, out, out32);
    return hipGetLastError();
  }
  ConvFwdOp op;
  op.g = {B, Hi, Wi, Cin, Hi / 2, Wi / 2, Cout};
  op.tap_uniform = Cin % BK == 0;
  op.in = in; op.w = w; op.bias = bias; op.out = out; op.out32 = out32; op.relu = relu;
  return launch_gemm(op, B * (Hi / 2) * (Wi / 2), Cout, 9 * Cin, 1, st);
}

hipError_t conv12_fwd(const bf16 *in0, const bf16 *w1, const float *b1, const bf16 *w2,
                      const float *b2, int B, int H0, bf16 *out, hipStream_t st) {
  if (H0 % 64 != 0) return hipErrorInvalidValue;
  const int H2 = H0 / 4;
  hipLaunchKernelGGL(k_conv12_fwd, dim3((H2 / 8) * (H2 / 16), B), dim3(256), 0, st, in0, w1, b1, w2,
                     b2, H0, out);
  return hipGetLastError();
}

hipError_t conv_dgrad(const bf16 *dout, const bf16 *wt, const bf16 *act_in, int B, int Hi, int Wi,
                      int Cin, int Cout, bf16 *din, float *din32, hipStream_t st) {
  ConvDgradOp op;
  op.g = {B, Hi, Wi, Cin, Hi / 2, Wi / 2, Cout};
  op.tap_uniform = Cout % BK == 0;
  op.dout = dout; op.wt = wt; op.act_in = act_in; op.din = din; op.din32 = din32;
  return launch_gemm(op, B * Hi * Wi, Cin, 9 * Cout, 1, st);
}

hipError_t conv_wgrad(const bf16 *dout, const bf16 *in, int B, int Hi, int Wi, int Cin, int Cout,
                      float *part, size_t part_cap, float *dw, hipStream_t st) {
  const int64_t npix = (int64_t)B * (Hi / 2) * (Wi / 2);
  if (Cin == 1) {
    const int ppb = 256;
    const unsigned blocks = cdiv_(npix, ppb);
    if (Cout > 32 || (size_t)blocks * Cout * 9 > part_cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_conv1_wgrad, dim3(blocks), dim3(256), 0, st, in, dout, B, Hi, Wi, Cout,
                       ppb, part);
    hipLaunchKernelGGL(k_splitk_reduce, dim3(cdiv_(Cout * 9, 256)), dim3(256), 0, st, part,
                       (int)blocks, (int64_t)Cout * 9, dw);
    return hipGetLastError();
  }
  ConvWgradOp op;
  op.g = {B, Hi, Wi, Cin, Hi / 2, Wi / 2, Cout};
  op.dout = dout; op.in = in; op.part = part;
  const int M = Cout, N = 9 * Cin, K = (int)npix;
  int s = wgrad_splits(M, N, K);
  while ((size_t)s * M * N > part_cap && s > 1) --s;
  if ((size_t)s * M * N > part_cap) return hipErrorInvalidValue;
  int kchunk = (K + s - 1) / s;
  kchunk = (kchunk + MK - 1) / MK * MK;
  s = (K + kchunk - 1) / kchunk;
  hipError_t e = launch_gemm(op, M, N, K, s, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_splitk_reduce, dim3(cdiv_((int64_t)M * N, 256)), dim3(256), 0, st, part, s,
                     (int64_t)M * N, dw);
  return hipGetLastError();
}

hipError_t lin_fwd(const bf16 *x, const bf16 *w, const float *bias, int B, int In, int Out,
                   int relu, bf16 *y, float *y32, hipStream_t st) {
  LinFwdOp op;
  op.g = {B, In, Out};
  op.x = x; op.w = w; op.bias = bias; op.y = y; op.y32 = y32; op.relu = relu;
  return launch_gemm(op, B, Out, In, 1, st);
}

hipError_t lin_dgrad(const bf16 *dy, const bf16 *wt, const bf16 *x_act, int B, int In, int Out,
                     bf16 *dx, float *dx32, hipStream_t st) {
  LinDgradOp op;
  op.g = {B, In, Out};
  op.dy = dy; op.wt = wt; op.x_act = x_act; op.dx = dx; op.dx32 = dx32;
  return launch_gemm(op, B, In, Out, 1, st);
}

hipError_t lin_wgrad(const bf16 *dy, const bf16 *x, int B, int In, int Out, float *part,
                     size_t part_cap, float *dw, hipStream_t st) {
  LinWgradOp op;
  op.g = {B, In, Out};
  op.dy = dy; op.x = x; op.part = part;
  const int M = Out, N = In, K = B;
  int s = wgrad_splits(M, N, K);
  while ((size_t)s * M * N > part_cap && s > 1) --s;
  if ((size_t)s * M * N > part_cap) return hipErrorInvalidValue;
  int kchunk = (K + s - 1) / s;
  kchunk = (kchunk + MK - 1) / MK * MK;
  s = (K + kchunk - 1) / kchunk;
  hipError_t e = launch_gemm(op, M, N, K, s, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_splitk_reduce, dim3(cdiv_((int64_t)M * N, 256)), dim3(256), 0, st, part, s,
                     (int64_t)M * N, dw);
  return hipGetLastError();
}

hipError_t colsum(const bf16 *g, int M, int N, float *part, size_t part_cap, float *out,
                  hipStream_t st) {
  int chunks = std::max(1, std::min(1024, M / 256));
  while ((size_t)chunks * N > part_cap && chunks > 1) chunks /= 2;
  if ((size_t)chunks * N > part_cap) return hipErrorInvalidValue;
  const int rpc = (M + chunks - 1) / chunks;
  hipLaunchKernelGGL(k_colsum, dim3(cdiv_(N, 256), chunks), dim3(256), 0, st, g, M, N, rpc, part);
  hipLaunchKernelGGL(k_splitk_reduce, dim3(cdiv_(N, 256)), dim3(256), 0, st, part, chunks,
                     (int64_t)N, out);
  return hipGetLastError();
}

hipError_t sum_into(const float *part, int n, float *out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(64), 0, st, part, n, out);
  return hipGetLastError();
}

hipError_t standardize(const float *img, int B, int npx, bf16 *out, hipStream_t st) {
  hipLaunchKernelGGL(k_standardize, dim3(B), dim3(256), 0, st, img, npx, out);
  return hipGetLastError();
}

hipError_t head(const float *out8, int B, float *rot, float *shift, hipStream_t st) {
  hipLaunchKernelGGL(k_head, dim3(cdiv_(B, 256)), dim3(256), 0, st, out8, B, rot, shift);
  return hipGetLastError();
}

hipError_t head_loss(const float *out8, const float *rot_t, const float *shift_t, int B,
                     float lambda, float *loss_part, bf16 *dout8, float *dout32, hipStream_t st) {
  hipLaunchKernelGGL(k_head_loss, dim3(cdiv_(B, 256)), dim3(256), 0, st, out8, rot_t, shift_t, B,
                     lambda, loss_part, dout8, dout32);
  return hipGetLastError();
}

hipError_t to_bf16(const float *w, int Cout, int taps, int Cin, bf16 *wb, bf16 *wt, hipStream_t st) {
  const int64_t n = (int64_t)Cout * taps * Cin;
  hipLaunchKernelGGL(k_to_bf16, dim3(cdiv_(n, 256)), dim3(256), 0, st, w, Cout, taps, Cin, wb, wt);
  return hipGetLastError();
}

hipError_t f32_to_bf16(const float *x, int64_t n, bf16 *y, hipStream_t st) {
  hipLaunchKernelGGL(k_f32_to_bf16, dim3(cdiv_(n, 256)), dim3(256), 0, st, x, n, y);
  return hipGetLastError();
}

hipError_t bf16_to_f32(const bf16 *x, int64_t n, float *y, hipStream_t st) {
  hipLaunchKernelGGL(k_bf16_to_f32, dim3(cdiv_(n, 256)), dim3(256), 0, st, x, n, y);
  return hipGetLastError();
}

}  // namespace cs
