// C-ABI of the pose-proposal network: six 3x3 stride-2 convolutions
// (1 -> 32 -> 64 -> 128 -> 256 -> 256 -> 256 channels, ReLU) and two linear
// layers (flatten -> 256 ReLU -> 8) mapping a particle image to a 6-D
// rotation representation and a 2-D shift; BF16 weights and activations,
// FP32 accumulation and FP32 master weights trained with Adam.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/cryosplat.h"
#include "cs_cnn.hpp"
#include "cs_host.hpp"
#include "cs_internal.hpp"

using namespace cs;

namespace {

struct Layer {
  bool conv;
  int Cin, Cout, Hi;  // input channels, output channels, input side (convs)
  int In, Out;        // linear sizes
  int taps;           // 9 for convs, 1 for linear
  size_t w_off, b_off;        // offsets in the flat FP32 parameter array (floats)
  size_t wb_off, wt_off;      // offsets in the BF16 weight buffer (elements)
  int64_t wcount() const { return (int64_t)Cout * taps * Cin; }
};

inline size_t al(size_t x) { return (x + 63) & ~size_t(63); }

}  // namespace

struct cs_cnn {
  cs_ctx *ctx = nullptr;
  int D = 0, max_batch = 0;
  std::vector<Layer> layers;  // 6 convs + 2 linear
  int64_t nparam = 0;
  float *param = nullptr, *grad = nullptr, *adam_m = nullptr, *adam_v = nullptr;
  bf16 *wbuf = nullptr;
  std::vector<bf16 *> act;   // act[0] input, act[l + 1] output of layer l
  std::vector<bf16 *> dact;  // dact[l + 1] gradient of the pre-activation of layer l
  float *out8 = nullptr;
  float *part = nullptr;
  size_t part_cap = 0;
  float *loss_part = nullptr;
  int64_t step = 0;
  int last_B = 0;
  bool act1_valid = false;  // the first layer's activation is stored by training steps only
  bool act0_valid = false;  // the standardised input is stored unless it came from the caller
  std::vector<size_t> elems;  // per-image elements of act[i] / dact[i]
  std::vector<void *> allocs;
};

namespace {

int ensure_aux(cs_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->aux_bytes) return CS_OK;
  HIPCHK(hipDeviceSynchronize());
  if (ctx->aux) HIPCHK(hipFree(ctx->aux));
  ctx->aux = nullptr;
  ctx->aux_bytes = 0;
  if (hipMalloc(&ctx->aux, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, CS_ERR_OOM, "hipMalloc(%zu) failed", bytes);
  }
  ctx->aux_bytes = bytes;
  return CS_OK;
}

// Deterministic uniform numbers for the initial weights (SplitMix64).
struct SplitMix {
  uint64_t s;
  double next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  }
};

int refresh_bf16(cs_cnn *net, hipStream_t st) {
  cs_ctx *ctx = net->ctx;
  for (auto &L : net->layers) {
    HIPCHK(to_bf16(net->param + L.w_off, L.Cout, L.taps, L.Cin, net->wbuf + L.wb_off,
                   net->wbuf + L.wt_off, st));
  }
  return CS_OK;
}

// fused: inference, the first two convolutions in one kernel (the first
// layer's activation is not stored; training steps need it and run unfused)
// x0: an already standardised bfloat16 input (fused inference only), used in
// place of the standardisation step.
int forward_layers(cs_cnn *net, const float *images, int B, hipStream_t st, bool fused = false,
                   const bf16 *x0 = nullptr) {
  cs_ctx *ctx = net->ctx;
  if (!x0) HIPCHK(standardize(images, B, net->D * net->D, net->act[0], st));
  net->act0_valid = x0 == nullptr;
  size_t l0 = 0;
  if (fused) {
    const Layer &L1 = net->layers[0], &L2 = net->layers[1];
    HIPCHK(conv12_fwd(x0 ? x0 : net->act[0], net->wbuf + L1.wb_off, net->param + L1.b_off,
                      net->wbuf + L2.wb_off, net->param + L2.b_off, B, net->D, net->act[2], st));
    l0 = 2;
  }
  for (size_t l = l0; l < net->layers.size(); ++l) {
    const Layer &L = net->layers[l];
    const bf16 *w = net->wbuf + L.wb_off;
    const float *b = net->param + L.b_off;
    const bool last = l + 1 == net->layers.size();
    if (L.conv) {
      HIPCHK(conv_fwd(net->act[l], w, b, B, L.Hi, L.Hi, L.Cin, L.Cout, 1, net->act[l + 1], nullptr, st));
    } else {
      HIPCHK(lin_fwd(net->act[l], w, b, B, L.In, L.Out, last ? 0 : 1, last ? nullptr : net->act[l + 1],
                     last ? net->out8 : nullptr, st));
    }
  }
  return CS_OK;
}

}  // namespace

extern "C" {

int cs_cnn_create(cs_ctx *ctx, int32_t D, int32_t max_batch, uint64_t seed, cs_cnn **out) {
  if (!ctx || !out) return CS_ERR_INVALID_ARG;
  *out = nullptr;
  if (D < 64 || D % 64 != 0 || D > 512) return fail(ctx, CS_ERR_UNSUPPORTED, "network input side must be a multiple of 64 in [64, 512]");
  if (max_batch < 1) return fail(ctx, CS_ERR_INVALID_ARG, "max_batch must be >= 1");
  HIPCHK(hipSetDevice(ctx->device));
  cs_cnn *net = new cs_cnn();
  net->ctx = ctx;
  net->D = D;
  net->max_batch = max_batch;
  const int chans[7] = {1, 32, 64, 128, 256, 256, 256};
  size_t po = 0, wo = 0;
  int side = D;
  for (int l = 0; l < 6; ++l) {
    Layer L{};
    L.conv = true;
    L.Cin = chans[l];
    L.Cout = chans[l + 1];
    L.Hi = side;
    L.taps = 9;
    L.w_off = po;
    po += L.wcount();
    L.b_off = po;
    po += L.Cout;
    L.wb_off = wo;
    wo += al(L.wcount());
    L.wt_off = wo;
    wo += al(L.wcount());
    net->layers.push_back(L);
    side /= 2;
  }
  const int flat = side * side * 256;
  const int lin[3] = {flat, 256, 8};
  for (int l = 0; l < 2; ++l) {
    Layer L{};
    L.conv = false;
    L.Cin = L.In = lin[l];
    L.Cout = L.Out = lin[l + 1];
    L.taps = 1;
    L.w_off = po;
    po += L.wcount();
    L.b_off = po;
    po += L.Cout;
    L.wb_off = wo;
    wo += al(L.wcount());
    L.wt_off = wo;
    wo += al(L.wcount());
    net->layers.push_back(L);
  }
  net->nparam = (int64_t)po;
  auto alloc = [&](size_t bytes, void **p) -> int {
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return CS_ERR_OOM;
    }
    net->allocs.push_back(*p);
    return CS_OK;
  };
  int rc = CS_OK;
  rc |= alloc(po * 4, (void **)&net->param);
  rc |= alloc(po * 4, (void **)&net->grad);
  rc |= alloc(po * 4, (void **)&net->adam_m);
  rc |= alloc(po * 4, (void **)&net->adam_v);
  rc |= alloc(wo * 2, (void **)&net->wbuf);
  // activations: act[0] = input (1 channel), act[l+1] = layer l output
  std::vector<size_t> act_elems;
  act_elems.push_back((size_t)D * D);
  for (auto &L : net->layers) act_elems.push_back(L.conv ? (size_t)(L.Hi / 2) * (L.Hi / 2) * L.Cout : (size_t)L.Out);
  net->elems = act_elems;
  for (size_t i = 0; i < act_elems.size(); ++i) {
    bf16 *a = nullptr, *d = nullptr;
    rc |= alloc(al(act_elems[i] * max_batch) * 2, (void **)&a);
    rc |= alloc(al(act_elems[i] * max_batch) * 2, (void **)&d);
    net->act.push_back(a);
    net->dact.push_back(d);
  }
  rc |= alloc((size_t)max_batch * 8 * 4, (void **)&net->out8);
  net->part_cap = (size_t)1 << 23;
  rc |= alloc(net->part_cap * 4, (void **)&net->part);
  rc |= alloc(((size_t)max_batch / 256 + 2) * 4, (void **)&net->loss_part);
  if (rc) {
    for (void *p : net->allocs) (void)hipFree(p);
    delete net;
    return fail(ctx, CS_ERR_OOM, "network allocation failed");
  }
  // He-uniform initial weights, zero biases
  std::vector<float> h(po, 0.f);
  SplitMix rng{seed};
  for (auto &L : net->layers) {
    const double a = std::sqrt(6.0 / (double)(L.Cin * L.taps));
    for (int64_t i = 0; i < L.wcount(); ++i) h[L.w_off + i] = (float)((2.0 * rng.next() - 1.0) * a);
  }
  HIPCHK(hipMemcpy(net->param, h.data(), po * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemset(net->adam_m, 0, po * 4));
  HIPCHK(hipMemset(net->adam_v, 0, po * 4));
  rc = refresh_bf16(net, nullptr);
  HIPCHK(hipDeviceSynchronize());
  if (rc) {
    for (void *p : net->allocs) (void)hipFree(p);
    delete net;
    return rc;
  }
  *out = net;
  return CS_OK;
}

void cs_cnn_destroy(cs_cnn *net) {
  if (!net) return;
  (void)hipDeviceSynchronize();
  for (void *p : net->allocs) (void)hipFree(p);
  delete net;
}

int64_t cs_cnn_param_count(const cs_cnn *net) { return net ? net->nparam : -1; }

int cs_cnn_get_params(cs_cnn *net, float *dst, void *stream) {
  if (!net || !dst) return CS_ERR_INVALID_ARG;
  cs_ctx *ctx = net->ctx;
  HIPCHK(hipMemcpyAsync(dst, net->param, net->nparam * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return CS_OK;
}

int cs_cnn_set_params(cs_cnn *net, const float *src, void *stream) {
  if (!net || !src) return CS_ERR_INVALID_ARG;
  cs_ctx *ctx = net->ctx;
  HIPCHK(hipMemcpyAsync(net->param, src, net->nparam * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return refresh_bf16(net, (hipStream_t)stream);
}

int cs_cnn_forward(cs_cnn *net, const float *images, int32_t B, float *rot, float *shift,
                   float *raw, void *stream) {
  if (!net) return CS_ERR_INVALID_ARG;
  cs_ctx *ctx = net->ctx;
  if (!images || !rot) return fail(ctx, CS_ERR_INVALID_ARG, "null images or rot");
  if (B < 1 || B > net->max_batch) return fail(ctx, CS_ERR_INVALID_ARG, "batch must be in [1, max_batch]");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  int rc = forward_layers(net, images, B, st, true);
  if (rc) return rc;
  net->last_B = B;
  net->act1_valid = false;
  HIPCHK(head(net->out8, B, rot, shift, st));
  if (raw) HIPCHK(hipMemcpyAsync(raw, net->out8, (size_t)B * 8 * 4, hipMemcpyDeviceToDevice, st));
  return CS_OK;
}

int cs_cnn_forward_std(cs_cnn *net, const uint16_t *x, int32_t B, float *rot, float *shift,
                       float *raw, void *stream) {
  if (!net) return CS_ERR_INVALID_ARG;
  cs_ctx *ctx = net->ctx;
  if (!x || !rot) return fail(ctx, CS_ERR_INVALID_ARG, "null input or rot");
  if (B < 1 || B > net->max_batch) return fail(ctx, CS_ERR_INVALID_ARG, "batch must be in [1, max_batch]");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  int rc = forward_layers(net, nullptr, B, st, true, x);
  if (rc) return rc;
  net->last_B = B;
  net->act1_valid = false;
  HIPCHK(head(net->out8, B, rot, shift, st));
  if (raw) HIPCHK(hipMemcpyAsync(raw, net->out8, (size_t)B * 8 * 4, hipMemcpyDeviceToDevice, st));
  return CS_OK;
}

int cs_cnn_train_step(cs_cnn *net, const float *images, const float *rot_target,
                      const float *shift_target, int32_t B, float lambda, float lr, float *loss,
                      float *grads_out, int32_t apply_update, void *stream) {
  if (!net) return CS_ERR_INVALID_ARG;
  cs_ctx *ctx = net->ctx;
  if (!images || !rot_target || !shift_target || !loss)
    return fail(ctx, CS_ERR_INVALID_ARG, "null training argument");
  if (B < 1 || B > net->max_batch) return fail(ctx, CS_ERR_INVALID_ARG, "batch must be in [1, max_batch]");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  int rc = forward_layers(net, images, B, st);
  if (rc) return rc;
  net->last_B = B;
  net->act1_valid = true;
  const int nl = (int)net->layers.size();
  // head: loss and d(out8)
  HIPCHK(head_loss(net->out8, rot_target, shift_target, B, lambda, net->loss_part,
                   net->dact[nl], nullptr, st));
  HIPCHK(sum_into(net->loss_part, (B + 255) / 256, loss, st));
  // backward, last layer first
  for (int l = nl - 1; l >= 0; --l) {
    const Layer &L = net->layers[l];
    bf16 *dy = net->dact[l + 1];
    float *gw = net->grad + L.w_off, *gb = net->grad + L.b_off;
    if (L.conv) {
      const int Ho = L.Hi / 2;
      HIPCHK(conv_wgrad(dy, net->act[l], B, L.Hi, L.Hi, L.Cin, L.Cout, net->part, net->part_cap, gw, st));
      HIPCHK(colsum(dy, B * Ho * Ho, L.Cout, net->part, net->part_cap, gb, st));
      if (l > 0)
        HIPCHK(conv_dgrad(dy, net->wbuf + L.wt_off, net->act[l], B, L.Hi, L.Hi, L.Cin, L.Cout,
                          net->dact[l], nullptr, st));
    } else {
      HIPCHK(lin_wgrad(dy, net->act[l], B, L.In, L.Out, net->part, net->part_cap, gw, st));
      HIPCHK(colsum(dy, B, L.Out, net->part, net->part_cap, gb, st));
      HIPCHK(lin_dgrad(dy, net->wbuf + L.wt_off, net->act[l], B, L.In, L.Out, net->dact[l], nullptr, st));
    }
  }
  if (grads_out)
    HIPCHK(hipMemcpyAsync(grads_out, net->grad, net->nparam * 4, hipMemcpyDeviceToDevice, st));
  if (apply_update) {
    net->step += 1;
    rc = cs_adam_step(ctx, net->param, net->grad, net->adam_m, net->adam_v, net->nparam, net->step,
                      lr, 0.9f, 0.999f, 1e-8f, st);
    if (rc) return rc;
    rc = refresh_bf16(net, st);
    if (rc) return rc;
  }
  return CS_OK;
}

int cs_cnn_tensor(cs_cnn *net, int32_t index, int32_t grad, uint16_t *dst, int64_t capacity,
                  void *stream) {
  if (!net) return CS_ERR_INVALID_ARG;
  cs_ctx *ctx = net->ctx;
  if (!dst || index < 0 || index >= (int)net->act.size() || (!grad && index == (int)net->act.size() - 1))
    return fail(ctx, CS_ERR_INVALID_ARG, "bad tensor index");
  const int64_t n = (int64_t)net->last_B * (int64_t)net->elems[index];
  if (n == 0) return fail(ctx, CS_ERR_INVALID_ARG, "no forward pass yet");
  if (index == 1 && !grad && !net->act1_valid)
    return fail(ctx, CS_ERR_INVALID_ARG, "inference does not store the first layer's activation");
  if (index == 0 && !grad && !net->act0_valid)
    return fail(ctx, CS_ERR_INVALID_ARG, "the last forward took its standardised input from the caller");
  if (capacity < n) return fail(ctx, CS_ERR_INVALID_ARG, "capacity %lld < %lld", (long long)capacity, (long long)n);
  HIPCHK(hipMemcpyAsync(dst, grad ? net->dact[index] : net->act[index], n * 2, hipMemcpyDeviceToDevice,
                        (hipStream_t)stream));
  return CS_OK;
}

// ---- single layers through the C-ABI (BF16 as raw uint16) ----------------

int cs_bf16_conv3x3s2_forward(cs_ctx *ctx, const uint16_t *in, const uint16_t *w, const float *bias,
                              int32_t B, int32_t H, int32_t W, int32_t Cin, int32_t Cout,
                              int32_t relu, uint16_t *out, float *out_f32, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!in || !w || !out || B < 1 || H < 2 || W < 2 || H % 2 || W % 2 || Cout % 8 ||
      (Cin != 1 && Cin % 8))
    return fail(ctx, CS_ERR_INVALID_ARG, "bad conv forward arguments");
  if (Cin == 1 && (H != W || Cout > 256))
    return fail(ctx, CS_ERR_INVALID_ARG, "first-layer conv needs H == W and Cout <= 256");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(conv_fwd((const bf16 *)in, (const bf16 *)w, bias, B, H, W, Cin, Cout, relu, (bf16 *)out,
                  out_f32, (hipStream_t)stream));
  return CS_OK;
}

int cs_bf16_conv3x3s2_dgrad(cs_ctx *ctx, const uint16_t *dout, const uint16_t *wt,
                            const uint16_t *act_in, int32_t B, int32_t H, int32_t W, int32_t Cin,
                            int32_t Cout, uint16_t *din, float *din_f32, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!dout || !wt || !din || B < 1 || H < 2 || W < 2 || H % 2 || W % 2 || Cin % 8 || Cout % 8)
    return fail(ctx, CS_ERR_INVALID_ARG, "bad conv dgrad arguments");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(conv_dgrad((const bf16 *)dout, (const bf16 *)wt, (const bf16 *)act_in, B, H, W, Cin, Cout,
                    (bf16 *)din, din_f32, (hipStream_t)stream));
  return CS_OK;
}

int cs_bf16_conv3x3s2_wgrad(cs_ctx *ctx, const uint16_t *dout, const uint16_t *in, int32_t B,
                            int32_t H, int32_t W, int32_t Cin, int32_t Cout, float *dw,
                            void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!dout || !in || !dw || B < 1 || H < 2 || W < 2 || H % 2 || W % 2 || Cout % 8 ||
      (Cin != 1 && Cin % 8) || (Cin == 1 && Cout > 32))
    return fail(ctx, CS_ERR_INVALID_ARG, "bad conv wgrad arguments");
  HIPCHK(hipSetDevice(ctx->device));
  const size_t cap = (size_t)1 << 23;
  int rc = ensure_aux(ctx, cap * 4);
  if (rc) return rc;
  HIPCHK(conv_wgrad((const bf16 *)dout, (const bf16 *)in, B, H, W, Cin, Cout, (float *)ctx->aux, cap,
                    dw, (hipStream_t)stream));
  return CS_OK;
}

int cs_bf16_linear_forward(cs_ctx *ctx, const uint16_t *x, const uint16_t *w, const float *bias,
                           int32_t B, int32_t In, int32_t Out, int32_t relu, uint16_t *y,
                           float *y_f32, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!x || !w || (!y && !y_f32) || B < 1 || In % 8 || Out % 8 || In < 8 || Out < 8)
    return fail(ctx, CS_ERR_INVALID_ARG, "bad linear forward arguments");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(lin_fwd((const bf16 *)x, (const bf16 *)w, bias, B, In, Out, relu, (bf16 *)y, y_f32,
                 (hipStream_t)stream));
  return CS_OK;
}

int cs_bf16_linear_dgrad(cs_ctx *ctx, const uint16_t *dy, const uint16_t *wt, const uint16_t *x_act,
                         int32_t B, int32_t In, int32_t Out, uint16_t *dx, float *dx_f32,
                         void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!dy || !wt || !dx || B < 1 || In % 8 || Out % 8 || In < 8 || Out < 8)
    return fail(ctx, CS_ERR_INVALID_ARG, "bad linear dgrad arguments");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(lin_dgrad((const bf16 *)dy, (const bf16 *)wt, (const bf16 *)x_act, B, In, Out, (bf16 *)dx,
                   dx_f32, (hipStream_t)stream));
  return CS_OK;
}

int cs_bf16_linear_wgrad(cs_ctx *ctx, const uint16_t *dy, const uint16_t *x, int32_t B, int32_t In,
                         int32_t Out, float *dw, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!dy || !x || !dw || B < 1 || In % 8 || Out % 8 || In < 8 || Out < 8)
    return fail(ctx, CS_ERR_INVALID_ARG, "bad linear wgrad arguments");
  HIPCHK(hipSetDevice(ctx->device));
  const size_t cap = (size_t)1 << 23;
  int rc = ensure_aux(ctx, cap * 4);
  if (rc) return rc;
  HIPCHK(lin_wgrad((const bf16 *)dy, (const bf16 *)x, B, In, Out, (float *)ctx->aux, cap, dw,
                   (hipStream_t)stream));
  return CS_OK;
}

int cs_pose_head(cs_ctx *ctx, const float *raw, int32_t B, float *rot, float *shift,
                 const float *rot_target, const float *shift_target, float lambda, float *loss,
                 float *d_raw, void *stream) {
  if (!ctx) return CS_ERR_INVALID_ARG;
  if (!raw || B < 1) return fail(ctx, CS_ERR_INVALID_ARG, "bad head arguments");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  if (rot) HIPCHK(head(raw, B, rot, shift, st));
  if (rot_target && shift_target && loss && d_raw) {
    const size_t nb = (size_t)(B + 255) / 256;
    int rc = ensure_aux(ctx, (nb + (size_t)B * 8) * 4 + 256);
    if (rc) return rc;
    float *lp = (float *)ctx->aux;
    bf16 *tmp = (bf16 *)(lp + nb + 16);
    HIPCHK(head_loss(raw, rot_target, shift_target, B, lambda, lp, tmp, d_raw, st));
    HIPCHK(sum_into(lp, (int)nb, loss, st));
  }
  return CS_OK;
}

}  // extern "C"
