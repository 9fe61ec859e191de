"""Pose-proposal network kernels vs the FP64 network oracle (GPU).

Layer tests feed the same bfloat16 operands to both sides (the oracle widens
them to FP64), so the FP32 outputs differ only by accumulation order:
normwise <= 1e-5.  Stored bfloat16 outputs must equal the oracle's FP64
value rounded to bfloat16 except where the FP32 accumulator and the FP64
value straddle a rounding boundary (a one-ulp difference on a tiny
fraction of elements).  Shapes are ragged against the 64 x 64 x 32 tiles.

A whole training step is checked layer by layer from the GPU's own stored
bfloat16 inputs (teacher forcing), at the same per-layer tolerances: a free
running comparison of the whole bfloat16 network is chaotic at the 1e-2
level, because one-ulp rounding flips upstream move a few pre-activations
across the ReLU kink and switch whole gradient rows.  The oracle itself is
pinned by finite differences.
"""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import adam as o_adam
from oracle import cnn
from gpu_util import announce, dev, host, normwise
from paper_2508_04929_amd import binding

pytestmark = pytest.mark.gpu


def bf(x):
    """FP64 array (already bfloat16-representable or not) -> device bfloat16."""
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda().to(torch.bfloat16)


def hb(t):
    return t.float().cpu().numpy().astype(np.float64)


def check_bf16_rounding(got_bf16, ref64, max_frac=1e-3):
    """Stored bfloat16 values vs the FP64 value rounded to bfloat16.

    Every mismatch must be by at most one bfloat16 ulp plus the FP32
    accumulation error (1e-5 of the tensor's largest magnitude, the normwise
    bar of the FP32 outputs): near-zero results of cancelling sums carry that
    absolute error, however small their own ulp.  A mismatch whose FP64
    value lies within that error (or 1e-5 of itself) of the rounding boundary
    between the two bfloat16 neighbours is a rounding decided by the FP32
    error and always allowed; the others may be at most a max_frac fraction
    of the elements."""
    ref64 = np.asarray(ref64, dtype=np.float64)
    ref = cnn.round_bf16(ref64)
    got = hb(got_bf16)
    diff = got != ref
    if diff.any():
        ulp = np.abs(ref[diff]) * 2.0 ** -7
        acc = 1e-5 * np.abs(ref64).max()
        assert np.all(np.abs(got[diff] - ref64[diff]) <= 1.01 * ulp + acc)
        mid = 0.5 * (got[diff] + ref[diff])
        tie = np.abs(ref64[diff] - mid) <= acc + 1e-5 * np.abs(ref64[diff])
        assert (~tie).sum() <= max_frac * diff.size, ((~tie).sum(), diff.size)


@pytest.mark.parametrize("B,H,W,Cin,Cout", [(3, 34, 34, 40, 72), (2, 66, 66, 1, 32),
                                            (5, 8, 6, 256, 256),
                                            # M >= 16384: 128 x 128 and 128 x 64 tiles, ragged
                                            (20, 64, 64, 32, 128), (17, 66, 66, 8, 64)])
def test_conv_forward(gpu_lib, B, H, W, Cin, Cout):
    announce(f"conv forward B={B} H={H} W={W} Cin={Cin} Cout={Cout}")
    rng = np.random.default_rng(100 + Cin)
    x = cnn.round_bf16(rng.standard_normal((B, H, W, Cin)))
    w = cnn.round_bf16(rng.standard_normal((Cout, 3, 3, Cin)) / np.sqrt(9 * Cin))
    b = rng.standard_normal(Cout).astype(np.float32).astype(np.float64)
    y, y32 = gpu_lib.conv_forward(bf(x), bf(w), dev(b), relu=True, want_f32=True)
    ref = np.maximum(cnn.conv3x3s2(x, w, b), 0.0)
    assert normwise(host(y32), ref) <= 1e-5
    check_bf16_rounding(y, ref)


@pytest.mark.parametrize("B,H,W,Cin,Cout", [(3, 34, 34, 40, 72), (4, 16, 16, 256, 256),
                                            (5, 64, 64, 64, 128), (4, 66, 66, 128, 64)])
def test_conv_dgrad(gpu_lib, B, H, W, Cin, Cout):
    announce(f"conv dgrad B={B} H={H} W={W} Cin={Cin} Cout={Cout}")
    rng = np.random.default_rng(200 + Cin)
    dy = cnn.round_bf16(rng.standard_normal((B, H // 2, W // 2, Cout)))
    w = cnn.round_bf16(rng.standard_normal((Cout, 3, 3, Cin)) / np.sqrt(9 * Cout))
    act = cnn.round_bf16(np.maximum(rng.standard_normal((B, H, W, Cin)), 0.0))
    wt = np.ascontiguousarray(w.transpose(3, 1, 2, 0))
    dx, dx32 = gpu_lib.conv_dgrad(bf(dy), bf(wt), bf(act), want_f32=True)
    ref = cnn.conv3x3s2_dgrad(dy, w, H, W) * (act > 0)
    assert normwise(host(dx32), ref) <= 1e-5
    check_bf16_rounding(dx, ref)


@pytest.mark.parametrize("B,H,W,Cin,Cout", [(3, 34, 34, 40, 72), (2, 66, 66, 1, 32),
                                            (6, 8, 8, 256, 256)])
def test_conv_wgrad(gpu_lib, B, H, W, Cin, Cout):
    announce(f"conv wgrad B={B} H={H} W={W} Cin={Cin} Cout={Cout}")
    rng = np.random.default_rng(300 + Cin)
    dy = cnn.round_bf16(rng.standard_normal((B, H // 2, W // 2, Cout)))
    x = cnn.round_bf16(rng.standard_normal((B, H, W, Cin)))
    dw = gpu_lib.conv_wgrad(bf(dy), bf(x))
    assert normwise(host(dw), cnn.conv3x3s2_wgrad(dy, x)) <= 1e-5


def test_linear_layers(gpu_lib):
    announce("linear forward / dgrad / wgrad")
    rng = np.random.default_rng(400)
    B, In, Out = 37, 264, 72
    x = cnn.round_bf16(np.maximum(rng.standard_normal((B, In)), 0.0))
    w = cnn.round_bf16(rng.standard_normal((Out, In)) / np.sqrt(In))
    b = rng.standard_normal(Out).astype(np.float32).astype(np.float64)
    y, y32 = gpu_lib.linear_forward(bf(x), bf(w), dev(b), relu=True)
    ref = np.maximum(x @ w.T + b, 0.0)
    assert normwise(host(y32), ref) <= 1e-5
    check_bf16_rounding(y, ref)
    dy = cnn.round_bf16(rng.standard_normal((B, Out)))
    dx, dx32 = gpu_lib.linear_dgrad(bf(dy), bf(np.ascontiguousarray(w.T)), bf(x), want_f32=True)
    ref = (dy @ w) * (x > 0)
    assert normwise(host(dx32), ref) <= 1e-5
    check_bf16_rounding(dx, ref)
    dw = gpu_lib.linear_wgrad(bf(dy), bf(x))
    assert normwise(host(dw), dy.T @ x) <= 1e-5


def test_pose_head_and_loss(gpu_lib):
    announce("pose head")
    rng = np.random.default_rng(500)
    B = 300
    raw = rng.standard_normal((B, 8)).astype(np.float32).astype(np.float64)
    Rt = Rotation.random(B, random_state=501).as_matrix()
    tt = rng.standard_normal((B, 2))
    out = gpu_lib.pose_head(dev(raw), dev(Rt), dev(tt), lam=0.3)
    R, _ = cnn.gram_schmidt(raw[:, :6])
    np.testing.assert_allclose(host(out["rot"]), R, atol=2e-6)
    np.testing.assert_allclose(host(out["shift"]), raw[:, 6:8], atol=0)
    loss, d = cnn.head_loss(raw, Rt, tt.astype(np.float32).astype(np.float64), 0.3)
    np.testing.assert_allclose(host(out["loss"])[0], loss, rtol=1e-5)
    assert normwise(host(out["d_raw"]), d) <= 1e-5


def _net_and_batch(gpu_lib, D, B, seed):
    net = gpu_lib.network(D, max_batch=B, seed=seed)
    rng = np.random.default_rng(seed)
    theta = host(net.get_params())
    layers = cnn.unflatten(theta, D)
    # non-zero biases so that their gradients and the ReLU masks are exercised
    layers = [(w, (0.05 * rng.standard_normal(bb.shape)).astype(np.float32).astype(np.float64))
              for w, bb in layers]
    theta = cnn.flatten(layers)
    net.set_params(dev(theta))
    img = (rng.standard_normal((B, D, D)) + 0.5).astype(np.float32).astype(np.float64)
    Rt = Rotation.random(B, random_state=seed + 1).as_matrix().astype(np.float32).astype(np.float64)
    tt = rng.standard_normal((B, 2)).astype(np.float32).astype(np.float64)
    return net, layers, theta, img, Rt, tt


def test_network_params_round_trip(gpu_lib):
    net = gpu_lib.network(64, max_batch=4, seed=7)
    p = net.get_params()
    assert p.numel() == sum(int(np.prod(ws)) + nb for _, ws, nb in cnn.layer_shapes(64))
    q = torch.randn_like(p)
    net.set_params(q)
    assert torch.equal(net.get_params(), q)
    net.close()


def _act_shapes(D, B):
    shapes = [(B, D, D, 1)]
    side = D
    for c in cnn.CHANNELS[1:]:
        side //= 2
        shapes.append((B, side, side, c))
    shapes.append((B, cnn.HIDDEN))
    shapes.append((B, cnn.OUTPUTS))
    return shapes  # index i: act[i] (0..7), dact[i] (1..8)


@pytest.mark.parametrize("D,B", [(64, 5), (128, 3)])
def test_network_layers_teacher_forced(gpu_lib, D, B):
    """Every layer of a full training step, checked from the GPU's own stored
    inputs: forward activations, head gradient, masked activation gradients
    and parameter gradients, each at the per-layer tolerances."""
    announce(f"network step teacher-forced D={D} B={B}")
    net, layers, theta, img, Rt, tt = _net_and_batch(gpu_lib, D, B, seed=600 + D)
    _, _, raw = net.forward(dev(img))
    loss, grads = net.train_step(dev(img), dev(Rt), dev(tt), lam=0.5, update=False,
                                 want_grads=True)
    torch.cuda.synchronize()
    shapes = _act_shapes(D, B)
    A = [hb(net.tensor(i, False, shapes[i])) for i in range(8)]
    G = [None] + [hb(net.tensor(i, True, shapes[i])) for i in range(1, 9)]
    wq = [(cnn.round_bf16(w), b) for w, b in layers]
    g = cnn.unflatten(host(grads), D)
    raw = host(raw)
    # input and forward
    check_bf16_rounding(net.tensor(0, False, shapes[0]), cnn.standardize(img))
    for l in range(6):
        ref = np.maximum(cnn.conv3x3s2(A[l], wq[l][0], wq[l][1]), 0.0)
        check_bf16_rounding(net.tensor(l + 1, False, shapes[l + 1]), ref)
    ref = np.maximum(A[6].reshape(B, -1) @ wq[6][0].T + wq[6][1], 0.0)
    check_bf16_rounding(net.tensor(7, False, shapes[7]), ref)
    assert normwise(raw, A[7] @ wq[7][0].T + wq[7][1]) <= 1e-5
    # head
    l_ref, d = cnn.head_loss(raw, Rt, tt, 0.5)
    np.testing.assert_allclose(host(loss)[0], l_ref, rtol=1e-5)
    check_bf16_rounding(net.tensor(8, True, shapes[8]), d)
    # backward: linear layers, then convs
    for l in (7, 6):
        x = A[l].reshape(B, -1)
        assert normwise(g[l][0], G[l + 1].T @ x) <= 1e-5, ("w", l)
        assert normwise(g[l][1], G[l + 1].sum(axis=0)) <= 1e-5, ("b", l)
        ref = ((G[l + 1] @ wq[l][0]) * (x > 0)).reshape(shapes[l])
        check_bf16_rounding(net.tensor(l, True, shapes[l]), ref)
    for l in range(5, -1, -1):
        assert normwise(g[l][0], cnn.conv3x3s2_wgrad(G[l + 1], A[l])) <= 1e-5, ("w", l)
        assert normwise(g[l][1], G[l + 1].sum(axis=(0, 1, 2))) <= 1e-5, ("b", l)
        if l > 0:
            ref = cnn.conv3x3s2_dgrad(G[l + 1], wq[l][0], A[l].shape[1], A[l].shape[2]) * (A[l] > 0)
            check_bf16_rounding(net.tensor(l, True, shapes[l]), ref)
    # inference (first two layers fused) stores the same activations, bitwise
    net.forward(dev(img))
    for i in (0, 2, 3, 4, 5, 6, 7):
        assert torch.equal(net.tensor(i, False, shapes[i]), bf(A[i]).to(torch.bfloat16)), i
    # free-running: the loss of the whole bfloat16 network agrees with the
    # oracle's (per-layer rounding flips move it by far less than 1e-3)
    l16, _, _ = cnn.loss_and_grad(layers, img, Rt, tt, lam=0.5, bf16=True)
    assert abs(host(loss)[0] - l16) <= 1e-3 * abs(l16)
    # no update was applied
    assert torch.equal(net.get_params(), dev(theta))
    net.close()


def test_inference_equals_training_forward_large_batch(gpu_lib):
    """B=20 at D=128 puts the later convolutions on 128 x 128 tiles."""
    announce("inference vs training forward, D=128 B=20")
    D, B = 128, 20
    net, layers, theta, img, Rt, tt = _net_and_batch(gpu_lib, D, B, seed=650)
    net.train_step(dev(img), dev(Rt), dev(tt), update=False)
    shapes = _act_shapes(D, B)
    ref = [net.tensor(i, False, shapes[i]).clone() for i in range(8)]
    _, _, raw = net.forward(dev(img))
    for i in (0, 2, 3, 4, 5, 6, 7):
        assert torch.equal(net.tensor(i, False, shapes[i]), ref[i]), i
    with pytest.raises(binding.CryoSplatError):
        net.tensor(1, False, shapes[1])
    wq = cnn.round_bf16(layers[7][0])
    assert normwise(host(raw), hb(ref[7]) @ wq.T + layers[7][1]) <= 1e-5
    net.close()


def test_network_adam_update(gpu_lib):
    announce("network Adam step")
    D, B = 64, 4
    net, layers, theta, img, Rt, tt = _net_and_batch(gpu_lib, D, B, seed=700)
    _, grads = net.train_step(dev(img), dev(Rt), dev(tt), lam=1.0, lr=1e-3, update=True,
                              want_grads=True)
    g = host(grads)
    p_ref, _, _ = o_adam.adam_step(theta, g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    got = host(net.get_params())
    assert normwise(got - theta, p_ref - theta) <= 1e-4
    net.close()


def test_training_overfits_a_fixed_batch(gpu_lib):
    announce("network overfit")
    D, B = 64, 16
    net, layers, theta, img, Rt, tt = _net_and_batch(gpu_lib, D, B, seed=800)
    imgs, R, t = dev(img), dev(Rt), dev(tt)
    first = None
    for it in range(150):
        loss, _ = net.train_step(imgs, R, t, lam=1.0, lr=1e-3)
        if first is None:
            first = float(loss.item())
    last = float(loss.item())
    assert last < 0.2 * first, (first, last)
    net.close()
