"""FP64 reference of the pose-proposal network (test infrastructure only).

Nothing in the library imports this module; tests, the smoke check and the
CPU-baseline leg of the benchmark use it to check the HIP kernels.

The paper treats poses as known and leaves their estimation to future work
(Sec. 3.3 assumes W and t given; Sec. 5).  The network below is this
project's pose proposer, defined by its plain mathematics:

  * per-image standardisation x = (y - mean(y)) / std(y) (population std);
  * six 3x3 convolutions, stride 2, zero padding 1, each + bias + ReLU:
      out[b, oy, ox, co] = bias[co]
          + sum_{ky, kx, ci} w[co, ky, kx, ci] x[b, 2 oy + ky - 1, 2 ox + kx - 1, ci];
  * flatten (NHWC order), linear + ReLU to 256, linear to 8 outputs;
  * head: 6-D rotation representation (a1, a2) -> R = [b1 b2 b3] (columns)
    by Gram-Schmidt, b1 = a1/|a1|, b2 = normalise(a2 - (b1.a2) b1),
    b3 = b1 x b2; shift t = outputs 6, 7;
  * loss L = (1/B) sum_b ||R_b - R*_b||_F^2 + lambda ||t_b - t*_b||^2.

Backward passes are the hand-written adjoints of these definitions.  With
``bf16=True`` the same functions round to bfloat16 (nearest even) at the
points where the GPU stores bfloat16 tensors (standardised input, weights,
post-ReLU activations, masked activation gradients, head gradient), so that
the comparison isolates the FP32-accumulation order; ``bf16=False`` is the
pure FP64 network, used by the finite-difference pins.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (1, 32, 64, 128, 256, 256, 256)
HIDDEN = 256
OUTPUTS = 8


def round_bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    The value is first rounded to float32 (the precision the GPU holds it
    in before storing bfloat16)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(a.shape)


def _q(x, bf16):
    return round_bf16(x) if bf16 else np.asarray(x, dtype=np.float64)


# ---------------------------------------------------------------- layout

def layer_shapes(D):
    """[(kind, weight shape, bias length)] in parameter order."""
    out = []
    for l in range(6):
        out.append(("conv", (CHANNELS[l + 1], 3, 3, CHANNELS[l]), CHANNELS[l + 1]))
    flat = (D // 64) ** 2 * CHANNELS[-1]
    out.append(("linear", (HIDDEN, flat), HIDDEN))
    out.append(("linear", (OUTPUTS, HIDDEN), OUTPUTS))
    return out


def unflatten(theta, D):
    """Split the flat parameter vector into [(w, b)] per layer."""
    theta = np.asarray(theta, dtype=np.float64)
    layers, o = [], 0
    for _, ws, nb in layer_shapes(D):
        nw = int(np.prod(ws))
        layers.append((theta[o:o + nw].reshape(ws), theta[o + nw:o + nw + nb]))
        o += nw + nb
    assert o == theta.size, (o, theta.size)
    return layers


def flatten(layers):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in layers])


# ---------------------------------------------------------------- layers

def standardize(images):
    y = np.asarray(images, dtype=np.float64)
    m = y.mean(axis=(1, 2), keepdims=True)
    v = ((y - m) ** 2).mean(axis=(1, 2), keepdims=True)
    s = np.where(v > 0, np.sqrt(v), 1.0)
    return ((y - m) / s)[..., None]  # NHWC with one channel


def conv3x3s2(x, w, b=None):
    """x [B][H][W][Cin], w [Cout][3][3][Cin] -> [B][H/2][W/2][Cout]."""
    B, H, W, Cin = x.shape
    Ho, Wo = H // 2, W // 2
    xp = np.zeros((B, H + 2, W + 2, Cin))
    xp[:, 1:H + 1, 1:W + 1] = x
    out = np.zeros((B, Ho, Wo, w.shape[0]))
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :]  # x[2oy+ky-1, 2ox+kx-1]
            out += patch @ w[:, ky, kx, :].T
    if b is not None:
        out += b
    return out


def conv3x3s2_dgrad(dy, w, H, W):
    """Adjoint of conv3x3s2 in its input: dy [B][H/2][W/2][Cout] -> [B][H][W][Cin]."""
    B, Ho, Wo, _ = dy.shape
    Cin = w.shape[3]
    dxp = np.zeros((B, H + 2, W + 2, Cin))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :] += dy @ w[:, ky, kx, :]
    return dxp[:, 1:H + 1, 1:W + 1]


def conv3x3s2_wgrad(dy, x):
    """Adjoint of conv3x3s2 in its weights: sum over batch and pixels."""
    B, H, W, Cin = x.shape
    Ho, Wo = H // 2, W // 2
    xp = np.zeros((B, H + 2, W + 2, Cin))
    xp[:, 1:H + 1, 1:W + 1] = x
    dw = np.zeros((dy.shape[3], 3, 3, Cin))
    g = dy.reshape(-1, dy.shape[3])
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :].reshape(-1, Cin)
            dw[:, ky, kx, :] = g.T @ patch
    return dw


def gram_schmidt(a):
    """a [B][6] -> R [B][3][3] with columns b1, b2, b3 (and the intermediates)."""
    a1, a2 = a[:, 0:3], a[:, 3:6]
    n1 = np.maximum(np.linalg.norm(a1, axis=1, keepdims=True), 1e-12)
    b1 = a1 / n1
    u2 = a2 - np.sum(b1 * a2, axis=1, keepdims=True) * b1
    n2 = np.maximum(np.linalg.norm(u2, axis=1, keepdims=True), 1e-12)
    b2 = u2 / n2
    b3 = np.cross(b1, b2)
    R = np.stack([b1, b2, b3], axis=2)
    return R, (a1, a2, n1, b1, u2, n2, b2, b3)


def head_loss(out8, rot_t, shift_t, lam):
    """Loss and dL/d(out8) of the pose head (batch mean)."""
    out8 = np.asarray(out8, dtype=np.float64)
    B = out8.shape[0]
    R, (a1, a2, n1, b1, u2, n2, b2, b3) = gram_schmidt(out8[:, :6])
    E = R - rot_t
    dt = out8[:, 6:8] - shift_t
    loss = (np.sum(E ** 2) + lam * np.sum(dt ** 2)) / B
    G = 2.0 * E / B
    g1, g2, g3 = G[:, :, 0].copy(), G[:, :, 1].copy(), G[:, :, 2].copy()
    # b3 = b1 x b2:  d<g3, b1 x b2> = <b2 x g3, db1> + <g3 x b1, db2>
    g1 += np.cross(b2, g3)
    g2 += np.cross(g3, b1)
    # b2 = u2 / n2
    gu = (g2 - b2 * np.sum(b2 * g2, axis=1, keepdims=True)) / n2
    # u2 = a2 - (b1.a2) b1
    bu = np.sum(b1 * gu, axis=1, keepdims=True)
    ba = np.sum(b1 * a2, axis=1, keepdims=True)
    ga2 = gu - b1 * bu
    g1 = g1 - ba * gu - bu * a2
    # b1 = a1 / n1
    ga1 = (g1 - b1 * np.sum(b1 * g1, axis=1, keepdims=True)) / n1
    d = np.concatenate([ga1, ga2, 2.0 * lam * dt / B], axis=1)
    return loss, d


# ---------------------------------------------------------------- network

def forward(layers, images, bf16=False):
    """Activations [x0, a1, ..., a7] and the FP outputs [B][8]."""
    acts = [_q(standardize(images), bf16)]
    x = acts[0]
    for l in range(6):
        w, b = layers[l]
        x = _q(np.maximum(conv3x3s2(x, _q(w, bf16), b), 0.0), bf16)
        acts.append(x)
    B = x.shape[0]
    h = x.reshape(B, -1)
    w, b = layers[6]
    h = _q(np.maximum(h @ _q(w, bf16).T + b, 0.0), bf16)
    acts.append(h)
    w, b = layers[7]
    out = h @ _q(w, bf16).T + b
    return acts, out


def loss_and_grad(layers, images, rot_t, shift_t, lam=1.0, bf16=False):
    """Batch loss and the gradient of every layer's (w, b)."""
    acts, out = forward(layers, images, bf16)
    loss, d = head_loss(out, rot_t, shift_t, lam)
    dy = _q(d, bf16)
    grads = [None] * 8
    # fc2, fc1
    B = dy.shape[0]
    for l in (7, 6):
        w, _ = layers[l]
        x = acts[l].reshape(B, -1)
        grads[l] = (dy.T @ x, dy.sum(axis=0))
        dy = _q((dy @ _q(w, bf16)) * (x > 0), bf16)
    dy = dy.reshape(acts[6].shape)
    for l in range(5, -1, -1):
        w, _ = layers[l]
        x = acts[l]
        grads[l] = (conv3x3s2_wgrad(dy, x), dy.sum(axis=(0, 1, 2)))
        if l > 0:
            dy = _q(conv3x3s2_dgrad(dy, _q(w, bf16), x.shape[1], x.shape[2]) * (x > 0), bf16)
    return loss, grads, out


def predict(layers, images, bf16=False):
    _, out = forward(layers, images, bf16)
    R, _ = gram_schmidt(out[:, :6])
    return R, out[:, 6:8], out


def he_uniform(D, rng):
    """Independent He-uniform initialisation (for oracle-only pins)."""
    layers = []
    for _, ws, nb in layer_shapes(D):
        fan_in = int(np.prod(ws[1:]))
        a = np.sqrt(6.0 / fan_in)
        layers.append((rng.uniform(-a, a, ws), np.zeros(nb)))
    return layers
