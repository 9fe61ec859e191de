"""GPU (HIP) renderer against the FP64 oracle, element by element.

Bars: images (pre- and post-CTF) within 1e-4 normwise per image, gradients
within 1e-3 normwise per parameter group, integer pair counts exact up to
pixels whose FP32 and FP64 distances straddle the cut.  All calls go through
the C-ABI via the ctypes binding.
"""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import adam as o_adam
from oracle import ctf as o_ctf
from oracle import model as o_model
from oracle import objective as o_obj
from paper_2508_04929_amd import binding, inputs

from gpu_util import (announce, ctf_arg, dev, host, mixture_args, normwise,
                      per_image_normwise, view_args)

pytestmark = pytest.mark.gpu

Q_MATCHED = 2.0 * np.log(1e6)
IMG_TOL = 1e-4
GRAD_TOL = 1e-3
GROUPS = ("means", "log_scales", "quats", "amps")


def _oracle_Q(g, v, q_cut=Q_MATCHED, **kw):
    return o_model.render_pre_ctf(g.means, g.log_scales, g.quats, g.amps, v.rot, v.shift,
                                  v.D, v.pixel, q_cut, **kw)


def _observed(rng, X, snr_db=-20.0):
    return inputs.add_noise(rng, 0.7 * X, snr_db)


# ------------------------------------------------------------------ forward

def test_forward_c1_pre_ctf(gpu_lib):
    g, v, _ = inputs.c1(b=16)
    announce("c1 forward pre-CTF N=1000 B=16 D=64")
    Q = host(gpu_lib.render(**mixture_args(g), **view_args(v)))
    ref = _oracle_Q(g, v)
    ref_exact = _oracle_Q(g, v, q_cut=None)
    assert per_image_normwise(Q, ref) <= IMG_TOL
    assert per_image_normwise(Q, ref_exact) <= IMG_TOL


def test_forward_c1_with_ctf_and_loss(gpu_lib):
    g, v, gt = inputs.c1(b=16)
    announce("c1 forward with CTF + loss")
    X = host(gpu_lib.render(**mixture_args(g), **view_args(v), ctf=ctf_arg(v)))
    H = o_ctf.ctf_grid_for(v)
    Xr = o_ctf.apply_ctf(_oracle_Q(g, v, q_cut=None), H)
    assert per_image_normwise(X, Xr) <= IMG_TOL
    # observed images: an independent mixture rendered by the oracle, no noise
    Y = o_ctf.apply_ctf(_oracle_Q(gt, v, q_cut=None), H).astype(np.float32)
    for red in ("sum", "mean"):
        loss, _, Xg = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y),
                                            ctf=ctf_arg(v), reduction=red, want_grads=False,
                                            want_images=True)
        per, _ = o_obj.loss_from_images(Xr, Y, red)
        lg = host(loss)
        np.testing.assert_allclose(lg[:-1], per, rtol=1e-4)
        np.testing.assert_allclose(lg[-1], per.sum(), rtol=1e-4)
        assert per_image_normwise(host(Xg), Xr) <= IMG_TOL


@pytest.mark.parametrize("D", [48, 96, 192])
def test_forward_radix3_sizes(gpu_lib, D):
    rng = np.random.default_rng(D)
    g = inputs.mixture_anisotropic(rng, 3000, 0.3 * D * 1.2)
    v = inputs.views(rng, 3, D, 1.2, shift_px_sd=2.0)
    announce(f"radix-3 forward D={D}")
    X = host(gpu_lib.render(**mixture_args(g), **view_args(v), ctf=ctf_arg(v)))
    Xr = o_ctf.apply_ctf(_oracle_Q(g, v), o_ctf.ctf_grid_for(v))
    assert per_image_normwise(X, Xr) <= IMG_TOL


def test_forward_astigmatic_ctf(gpu_lib):
    rng = np.random.default_rng(5)
    g = inputs.mixture_anisotropic(rng, 2000, 30.0)
    v = inputs.views(rng, 4, 64, 1.5)
    v.defocus_v = (v.defocus_u * rng.uniform(0.6, 1.4, 4)).astype(np.float32)
    v.astig = rng.uniform(-3, 3, 4).astype(np.float32)
    v.phase = rng.uniform(0, 0.5, 4).astype(np.float32)
    v.bfactor = 50.0
    announce("astigmatic CTF with phase and B-factor")
    X = host(gpu_lib.render(**mixture_args(g), **view_args(v), ctf=ctf_arg(v)))
    Xr = o_ctf.apply_ctf(_oracle_Q(g, v), o_ctf.ctf_grid_for(v))
    assert per_image_normwise(X, Xr) <= IMG_TOL


def test_forward_odd_size_without_ctf(gpu_lib):
    rng = np.random.default_rng(6)
    g = inputs.mixture_anisotropic(rng, 500, 20.0)
    v = inputs.views(rng, 2, 63, 1.0, shift_px_sd=3.0)
    announce("odd D=63 without CTF")
    Q = host(gpu_lib.render(**mixture_args(g), **view_args(v)))
    assert per_image_normwise(Q, _oracle_Q(g, v)) <= IMG_TOL


def test_gaussians_across_and_outside_the_edge(gpu_lib):
    rng = np.random.default_rng(7)
    D, p = 64, 1.0
    g = inputs.mixture_anisotropic(rng, 400, 10.0)
    g.means[:, :2] = rng.uniform(-40, 40, size=(400, 2)).astype(np.float32)  # many off-image
    v = inputs.views(rng, 2, D, p)
    v.rot = np.repeat(np.eye(3, dtype=np.float32)[None], 2, 0)
    announce("Gaussians across and outside the image edge")
    Q = host(gpu_lib.render(**mixture_args(g), **view_args(v)))
    assert per_image_normwise(Q, _oracle_Q(g, v)) <= IMG_TOL


def test_empty_mixture(gpu_lib):
    rng = np.random.default_rng(8)
    g = inputs.mixture_anisotropic(rng, 0, 10.0)
    v = inputs.views(rng, 2, 32, 1.0)
    Y = rng.standard_normal((2, 32, 32)).astype(np.float32)
    announce("N = 0")
    X = host(gpu_lib.render(**mixture_args(g), **view_args(v), ctf=ctf_arg(v)))
    assert np.all(X == 0)
    loss, grads, _ = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y),
                                           ctf=ctf_arg(v))
    np.testing.assert_allclose(host(loss)[:-1], (Y.astype(np.float64) ** 2).sum((1, 2)), rtol=1e-5)
    assert all(t.numel() == 0 for t in grads.values())


# ------------------------------------------------------------------ gradients

def _check_grads(got, ref, tol=GRAD_TOL):
    for k in GROUPS:
        err = normwise(host(got[k]), ref[k])
        assert err <= tol, (k, err)


def test_loss_and_grad_c2_subset(gpu_lib):
    g, v, gt, rn = inputs.c2(b=256)
    v = v.subset(np.arange(4))
    announce("c2 loss_and_grad N=20000 B=4 D=128 vs oracle")
    H = o_ctf.ctf_grid_for(v)
    Xgt = o_ctf.apply_ctf(_oracle_Q(gt, v), H)
    Y = inputs.add_noise(rn, Xgt, -20.0)
    ref = o_obj.loss_and_grad(g, v, Y, q_cut=Q_MATCHED)
    loss, grads, X = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y),
                                           ctf=ctf_arg(v), want_images=True)
    assert per_image_normwise(host(X), ref["X"]) <= IMG_TOL
    np.testing.assert_allclose(host(loss)[:-1], ref["loss_per_image"], rtol=1e-4)
    _check_grads(grads, ref["grads"])


@pytest.mark.parametrize("acts", [("exp", "identity"), ("softplus", "softplus")])
def test_render_backward_matches_oracle(gpu_lib, acts):
    rng = np.random.default_rng(11)
    g = inputs.mixture_anisotropic(rng, 3000, 25.0)
    if acts[1] == "softplus":
        g.amps = rng.standard_normal(g.n).astype(np.float32)
    v = inputs.views(rng, 3, 96, 1.3, shift_px_sd=2.0)
    dX = rng.standard_normal((3, 96, 96)).astype(np.float32)
    announce(f"render_backward with activations {acts}")
    got = gpu_lib.render_backward(**mixture_args(g), **view_args(v), d_images=dev(dX),
                                  ctf=ctf_arg(v), scale_act=acts[0], amp_act=acts[1])
    GQ = o_ctf.apply_ctf(dX, o_ctf.ctf_grid_for(v))
    ref = o_obj.backward_from_image_grad(g, v, GQ, q_cut=Q_MATCHED, scale_act=acts[0],
                                         amp_act=acts[1])
    _check_grads(got, ref)


def test_gradients_vs_finite_differences(gpu_lib):
    """GPU gradients against FP64 central differences of the oracle loss."""
    rng = np.random.default_rng(12)
    g = inputs.mixture_anisotropic(rng, 40, 8.0)
    v = inputs.views(rng, 3, 32, 1.0, shift_px_sd=1.0)
    Y = (0.01 * rng.standard_normal((3, 32, 32))).astype(np.float32)
    announce("gradients vs FP64 finite differences")
    _, grads, _ = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y),
                                        ctf=ctf_arg(v))
    for field in GROUPS:
        arr = getattr(g, field)
        ent = [tuple(e) for e in np.ndindex(arr.shape)]
        ent = [ent[i] for i in rng.choice(len(ent), size=min(64, len(ent)), replace=False)]
        fd = o_obj.finite_difference(g, v, Y, field, ent, q_cut=None)
        got = host(grads[field])
        gv = np.array([got[e] for e in ent])
        assert np.abs(gv - fd).max() <= GRAD_TOL * np.abs(got).max(), field


def test_mean_reduction_scales_gradients(gpu_lib):
    rng = np.random.default_rng(13)
    g = inputs.mixture_anisotropic(rng, 1000, 20.0)
    v = inputs.views(rng, 2, 64, 1.0)
    Y = rng.standard_normal((2, 64, 64)).astype(np.float32)
    a = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y), ctf=ctf_arg(v))
    b = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y), ctf=ctf_arg(v),
                              reduction="mean")
    s = 1.0 / (2 * 64 * 64)
    np.testing.assert_allclose(host(b[0]), host(a[0]) * s, rtol=1e-5)
    for k in GROUPS:
        assert normwise(host(b[1][k]), host(a[1][k]) * s) <= 1e-5


# ------------------------------------------------------------- invariances

@pytest.mark.parametrize("tile,halo,budget,lane_order", [(16, 8, 64, 0), (32, 16, 256, 0),
                                                         (64, 8, 4096, 0), (128, 24, 512, 0),
                                                         (16, 1, 100, 0), (40, 12, 1024, 1),
                                                         (64, 16, 2048, 1), (32, 24, 3000, 2),
                                                         (16, 8, 64, 2)])
def test_results_independent_of_launch_options(gpu_lib, tile, halo, budget, lane_order):
    rng = np.random.default_rng(14)
    g = inputs.mixture_anisotropic(rng, 6000, 40.0)
    v = inputs.views(rng, 3, 128, 1.5, shift_px_sd=2.0)
    Y = rng.standard_normal((3, 128, 128)).astype(np.float32) * 1e-3
    announce(f"options tile={tile} halo={halo} budget={budget}")
    base = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y),
                                 ctf=ctf_arg(v), want_images=True)
    opt = binding.Options(tile=tile, halo=halo, budget=budget, lane_order=lane_order)
    alt = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y),
                                ctf=ctf_arg(v), want_images=True, options=opt)
    if lane_order:
        # the lane order changes no arithmetic: identical bits to list order
        ref = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y),
                                    ctf=ctf_arg(v), want_images=True,
                                    options=binding.Options(tile=tile, halo=halo, budget=budget))
        assert torch.equal(ref[2], alt[2]) and torch.equal(ref[0], alt[0])
        for k in GROUPS:
            assert torch.equal(ref[1][k], alt[1][k]), k
    assert per_image_normwise(host(alt[2]), host(base[2])) <= 1e-5
    for k in GROUPS:
        assert normwise(host(alt[1][k]), host(base[1][k])) <= 1e-4, k


def test_wide_gaussian_path_matches_oracle(gpu_lib):
    """A halo of one pixel sends nearly every Gaussian down the wide path."""
    rng = np.random.default_rng(15)
    g = inputs.mixture_anisotropic(rng, 800, 25.0, scale_mu=np.log(3.0))
    v = inputs.views(rng, 2, 64, 1.0)
    dX = rng.standard_normal((2, 64, 64)).astype(np.float32)
    opt = binding.Options(tile=16, halo=1)
    announce("wide-Gaussian path")
    Q = host(gpu_lib.render(**mixture_args(g), **view_args(v), options=opt))
    assert per_image_normwise(Q, _oracle_Q(g, v)) <= IMG_TOL
    got = gpu_lib.render_backward(**mixture_args(g), **view_args(v), d_images=dev(dX), options=opt)
    ref = o_obj.backward_from_image_grad(g, v, dX, q_cut=Q_MATCHED)
    _check_grads(got, ref)


def test_pair_count_matches_oracle(gpu_lib):
    g, v, _, _ = inputs.c2(b=4, n=5000)
    announce("pair count")
    got = host(gpu_lib.pair_count(**mixture_args(g), **view_args(v)))
    ref = o_model.pair_count(g.means, g.log_scales, g.quats, v.rot, v.shift, v.D, v.pixel, Q_MATCHED)
    # FP32 and FP64 may disagree on pixels sitting on the cut
    assert np.all(np.abs(got - ref) <= 1e-5 * ref + 2)


def test_adam_matches_oracle(gpu_lib):
    rng = np.random.default_rng(16)
    p = rng.standard_normal(10007).astype(np.float32)
    m = np.zeros_like(p)
    vv = np.zeros_like(p)
    pt, mt, vt = dev(p), dev(m), dev(vv)
    pr, mr, vr = p.astype(np.float64), m.astype(np.float64), vv.astype(np.float64)
    for step in range(1, 4):
        gr = rng.standard_normal(p.size).astype(np.float32)
        gpu_lib.adam_step(pt, dev(gr), mt, vt, step, lr=1e-3)
        pr, mr, vr = o_adam.adam_step(pr, gr, mr, vr, step, lr=1e-3)
    np.testing.assert_allclose(host(pt), pr, rtol=0, atol=1e-6)
    np.testing.assert_allclose(host(mt), mr, rtol=1e-5, atol=1e-7)


def test_batch_additivity(gpu_lib):
    """Gradients of a batch equal the sum over sub-batches (any batch size)."""
    g, v, _, _ = inputs.c2(b=32, n=8000)
    rng = np.random.default_rng(17)
    Y = rng.standard_normal((32, 128, 128)).astype(np.float32) * 1e-3
    full = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y), ctf=ctf_arg(v))
    acc = {k: 0.0 for k in GROUPS}
    for s in range(0, 32, 8):
        vs = v.subset(np.arange(s, s + 8))
        part = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(vs), observed=dev(Y[s:s + 8]),
                                     ctf=ctf_arg(vs))
        for k in GROUPS:
            acc[k] = acc[k] + host(part[1][k])
    for k in GROUPS:
        assert normwise(host(full[1][k]), acc[k]) <= 1e-4, k


def test_forward_is_bitwise_deterministic(gpu_lib):
    g, v, _, _ = inputs.c2(b=8, n=20000)
    a = host(gpu_lib.render(**mixture_args(g), **view_args(v), ctf=ctf_arg(v)))
    b = host(gpu_lib.render(**mixture_args(g), **view_args(v), ctf=ctf_arg(v)))
    assert np.array_equal(a, b)
    Y = np.zeros((8, 128, 128), np.float32)
    ga = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y), ctf=ctf_arg(v))[1]
    gb = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y), ctf=ctf_arg(v))[1]
    for k in GROUPS:
        assert np.array_equal(host(ga[k]), host(gb[k])), k


def test_wide_path_is_bitwise_deterministic_and_matches_oracle(gpu_lib):
    """A two-pixel halo sends most records down the wide path, whose
    footprints overlap heavily: repeated renders and adjoints must agree bit
    for bit (64-bit fixed-point sums per image), and match the oracle."""
    rng = np.random.default_rng(19)
    g = inputs.mixture_anisotropic(rng, 2500, 20.0, scale_mu=np.log(2.5))
    v = inputs.views(rng, 3, 96, 1.0, shift_px_sd=2.0)
    opt = binding.Options(tile=16, halo=2)
    announce("wide path: bitwise repeatability")
    a = host(gpu_lib.render(**mixture_args(g), **view_args(v), ctf=ctf_arg(v), options=opt))
    for _ in range(3):
        b = host(gpu_lib.render(**mixture_args(g), **view_args(v), ctf=ctf_arg(v), options=opt))
        assert np.array_equal(a, b)
    Q = host(gpu_lib.render(**mixture_args(g), **view_args(v), options=opt))
    assert per_image_normwise(Q, _oracle_Q(g, v)) <= IMG_TOL
    dX = dev(rng.standard_normal((3, 96, 96)).astype(np.float32))
    ga = gpu_lib.render_backward(**mixture_args(g), **view_args(v), d_images=dX, options=opt)
    gb = gpu_lib.render_backward(**mixture_args(g), **view_args(v), d_images=dX, options=opt)
    for k in GROUPS:
        assert np.array_equal(host(ga[k]), host(gb[k])), k


def test_fixed_point_with_extreme_weight_spread(gpu_lib):
    """Very narrow and very wide Gaussians share tiles: fixed-point scale stress."""
    rng = np.random.default_rng(18)
    n = 3000
    g = inputs.mixture_anisotropic(rng, n, 30.0)
    ls = np.where(rng.random((n, 1)) < 0.1, np.log(0.35), np.log(2.5))
    g.log_scales = (ls + 0.05 * rng.standard_normal((n, 3))).astype(np.float32)
    g.amps = np.exp(2.0 * rng.standard_normal(n)).astype(np.float32)
    v = inputs.views(rng, 3, 96, 1.0)
    announce("fixed-point stress: weights spanning many decades")
    Q = host(gpu_lib.render(**mixture_args(g), **view_args(v)))
    assert per_image_normwise(Q, _oracle_Q(g, v)) <= IMG_TOL


def test_negative_amplitudes(gpu_lib):
    rng = np.random.default_rng(19)
    g = inputs.mixture_anisotropic(rng, 2000, 25.0)
    g.amps = rng.standard_normal(g.n).astype(np.float32)
    v = inputs.views(rng, 2, 64, 1.2)
    Q = host(gpu_lib.render(**mixture_args(g), **view_args(v)))
    assert per_image_normwise(Q, _oracle_Q(g, v)) <= IMG_TOL
