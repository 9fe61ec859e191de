"""Pins of the FP64 pose-network oracle (CPU).

The network is this project's own (the paper leaves pose estimation to
future work), so the pins fix it against plain mathematics: scipy's 2-D
correlation for the strided convolution, torch's bfloat16 rounding, the
adjoint (dot-product) identities of every backward operator, orthonormality
and recovery properties of the Gram-Schmidt head, and finite differences of
the whole network.
"""
import numpy as np
import pytest
import torch
from scipy import signal
from scipy.spatial.transform import Rotation

from oracle import cnn


def test_round_bf16_matches_torch_nearest_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        # exact ties: 1 + 2^-8 (-> 1), 1 + 3 * 2^-8 (-> 1 + 2^-6)
                        [1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 0.0, -0.0]])
    got = cnn.round_bf16(x)
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(got, ref)
    assert got[-5] == 1.0 and got[-4] == 1 + 2.0 ** -6


def test_conv_matches_scipy_correlate_then_stride():
    rng = np.random.default_rng(1)
    B, H, W, Cin, Cout = 2, 10, 14, 3, 4
    x = rng.standard_normal((B, H, W, Cin))
    w = rng.standard_normal((Cout, 3, 3, Cin))
    bias = rng.standard_normal(Cout)
    got = cnn.conv3x3s2(x, w, bias)
    ref = np.zeros_like(got)
    for b in range(B):
        for co in range(Cout):
            acc = np.zeros((H, W))
            for ci in range(Cin):
                acc += signal.correlate2d(x[b, :, :, ci], w[co, :, :, ci], mode="same",
                                          boundary="fill")
            ref[b, :, :, co] = acc[::2, ::2] + bias[co]
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_conv_centre_delta_is_subsampling():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 8, 8, 5))
    w = np.zeros((5, 3, 3, 5))
    for c in range(5):
        w[c, 1, 1, c] = 1.0
    np.testing.assert_array_equal(cnn.conv3x3s2(x, w), x[:, ::2, ::2, :])


def test_conv_adjoints_dot_product():
    rng = np.random.default_rng(3)
    B, H, W, Cin, Cout = 2, 12, 8, 3, 5
    x = rng.standard_normal((B, H, W, Cin))
    w = rng.standard_normal((Cout, 3, 3, Cin))
    y = rng.standard_normal((B, H // 2, W // 2, Cout))
    lhs = np.sum(cnn.conv3x3s2(x, w) * y)
    np.testing.assert_allclose(np.sum(x * cnn.conv3x3s2_dgrad(y, w, H, W)), lhs, rtol=1e-12)
    np.testing.assert_allclose(np.sum(w * cnn.conv3x3s2_wgrad(y, x)), lhs, rtol=1e-12)


def test_standardize_is_affine_invariant():
    rng = np.random.default_rng(4)
    y = rng.standard_normal((3, 16, 16)) * 4 + 2
    s = cnn.standardize(y)
    np.testing.assert_allclose(s.mean(axis=(1, 2, 3)), 0, atol=1e-12)
    np.testing.assert_allclose(s.std(axis=(1, 2, 3)), 1, atol=1e-12)
    np.testing.assert_allclose(cnn.standardize(7.5 * y - 3.0), s, atol=1e-12)


def test_gram_schmidt_is_a_rotation_and_recovers_frames():
    rng = np.random.default_rng(5)
    a = rng.standard_normal((100, 6))
    R, _ = cnn.gram_schmidt(a)
    np.testing.assert_allclose(np.einsum("bji,bjk->bik", R, R), np.broadcast_to(np.eye(3), R.shape),
                               atol=1e-13)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-13)
    # columns of a known rotation, rescaled and with a2 tilted along b1
    Rt = Rotation.random(50, random_state=6).as_matrix()
    a = np.concatenate([3.0 * Rt[:, :, 0], 0.5 * Rt[:, :, 1] + 2.0 * Rt[:, :, 0]], axis=1)
    R, _ = cnn.gram_schmidt(a)
    np.testing.assert_allclose(R, Rt, atol=1e-13)


def test_head_loss_gradient_finite_differences():
    rng = np.random.default_rng(7)
    B = 5
    out = rng.standard_normal((B, 8))
    Rt = Rotation.random(B, random_state=8).as_matrix()
    tt = rng.standard_normal((B, 2))
    loss, d = cnn.head_loss(out, Rt, tt, 0.7)
    h = 1e-6
    fd = np.zeros_like(out)
    for i in range(B):
        for k in range(8):
            p, m = out.copy(), out.copy()
            p[i, k] += h
            m[i, k] -= h
            fd[i, k] = (cnn.head_loss(p, Rt, tt, 0.7)[0] - cnn.head_loss(m, Rt, tt, 0.7)[0]) / (2 * h)
    np.testing.assert_allclose(d, fd, rtol=1e-6, atol=1e-9)
    # zero loss and gradient at the target
    a = np.concatenate([Rt[:, :, 0], Rt[:, :, 1], tt], axis=1)
    l0, d0 = cnn.head_loss(a, Rt, tt, 0.7)
    assert l0 < 1e-25 and np.abs(d0).max() < 1e-12


def test_network_gradient_finite_differences():
    """Whole network (FP64, D=64): sampled parameters of every layer."""
    rng = np.random.default_rng(9)
    D, B = 64, 3
    layers = cnn.he_uniform(D, rng)
    layers = [(w, 0.05 * rng.standard_normal(b.shape)) for w, b in layers]
    img = rng.standard_normal((B, D, D))
    Rt = Rotation.random(B, random_state=10).as_matrix()
    tt = rng.standard_normal((B, 2))
    loss, grads, _ = cnn.loss_and_grad(layers, img, Rt, tt, lam=0.5)
    theta = cnn.flatten(layers)
    g_flat = cnn.flatten(grads)
    h = 1e-6
    offs = np.cumsum([0] + [w.size + b.size for w, b in layers])
    for l in range(8):
        idx = rng.integers(offs[l], offs[l + 1], 4)
        for i in idx:
            tp, tm = theta.copy(), theta.copy()
            tp[i] += h
            tm[i] -= h
            lp = cnn.loss_and_grad(cnn.unflatten(tp, D), img, Rt, tt, lam=0.5)[0]
            lm = cnn.loss_and_grad(cnn.unflatten(tm, D), img, Rt, tt, lam=0.5)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g_flat[i]) <= 1e-5 * max(1e-3, abs(fd)), (l, i, fd, g_flat[i])


def test_bf16_network_stays_close_to_fp64():
    rng = np.random.default_rng(11)
    D, B = 64, 2
    layers = cnn.he_uniform(D, rng)
    img = rng.standard_normal((B, D, D))
    _, o64 = cnn.forward(layers, img, bf16=False)
    _, o16 = cnn.forward(layers, img, bf16=True)
    assert np.linalg.norm(o16 - o64) <= 0.05 * np.linalg.norm(o64)
