"""Parity at the workloads' real shapes and launch configurations (GPU).

- The headline training step (N = 200,000, B = 64, D = 256, 1.1 A, CTF,
  launch options from the autotuner, as the bench times it): the adjoint of the full
  64-image call with dL/dimages non-zero on four images and zero elsewhere,
  element by element against the FP64 oracle's gradient of those four
  images (App. A.2, Eq. 15-21).
- Forward + backward at B = 256, D = 128, N = 20,000 (the anisotropic
  mixture with shifts): images of an 8-image subset of the full call, and
  the adjoint of the full call with dL/dimages on those 8 images.
- Uneven batching: the eight real mixtures (N = 5k ... 150k, 128 images
  each, D in {128, 192, 256}) with autotuned launch options in one batched
  graph launch; images and losses of two images per mixture against the
  oracle, the batched results equal to separate calls bitwise, and each
  mixture's adjoint (same options, all 128 images) with dL/dimages on two
  images against the oracle.

Observed images and dL/dimages are seeded normal draws; no oracle input
comes from the library.
"""
import numpy as np
import pytest
import torch

from oracle import ctf as o_ctf
from oracle import objective as o_obj
from paper_2508_04929_amd import inputs

from gpu_util import (announce, ctf_arg, dev, headline_options, host, mixture_args, normwise,
                      view_args)

pytestmark = pytest.mark.gpu
GROUPS = ("means", "log_scales", "quats", "amps")
Q_MATCHED = 2.0 * np.log(1e6)


def _sparse_image_grad(seed, B, D, idx):
    G = np.zeros((B, D, D), np.float32)
    G[list(idx)] = np.random.default_rng(seed).standard_normal((len(idx), D, D)).astype(np.float32)
    return G


def _check_adjoint(lib, g, v, idx, seed, options=None):
    """Adjoint of the full call with dL/dimages on `idx` only, vs the oracle
    on those images."""
    dG = _sparse_image_grad(seed, v.b, v.D, idx)
    got = lib.render_backward(**mixture_args(g), **view_args(v), d_images=dev(dG), ctf=ctf_arg(v),
                              options=options)
    torch.cuda.synchronize()
    vs = v.subset(list(idx))
    GQ = o_ctf.apply_ctf(dG[list(idx)].astype(np.float64), o_ctf.ctf_grid_for(vs))
    ref = o_obj.backward_from_image_grad(g, vs, GQ, q_cut=Q_MATCHED)
    errs = {k: normwise(host(got[k]), ref[k]) for k in GROUPS}
    scale_ref = np.abs(ref["log_scales"]).max()
    if np.abs(ref["quats"]).max() <= 1e-12 * scale_ref:
        # isotropic mixture: dL/dq is exactly zero (a symmetric dSigma has no
        # rotational part), so the FP32 result is rounding residue, bounded
        # against the log-scale gradient of the same Gaussians
        errs["quats"] = np.abs(host(got["quats"])).max() / scale_ref
    announce(f"  adjoint errors {', '.join(f'{k} {e:.2e}' for k, e in errs.items())}")
    for k, e in errs.items():
        assert e <= 1e-3, (k, e)


def _check_images(X, loss, g, v, Y, idx, reduction_scale):
    Xh, lo = host(X), host(loss)
    for b in idx:
        ref = o_obj.forward(g, v.subset([b]), Y[b:b + 1], q_cut=Q_MATCHED, reduction="sum")
        e = normwise(Xh[b], ref["X"][0])
        assert e <= 1e-4, (b, e)
        assert lo[b] == pytest.approx(ref["loss"] * reduction_scale, rel=1e-4)


def test_headline_step_adjoint_elementwise(gpu_lib):
    g, v, _gt, _rn = inputs.c4()
    announce("headline step N=200000 B=64 D=256: adjoint on images 3, 17, 40, 63 vs oracle")
    Y = (2e-6 * np.random.default_rng(129).standard_normal((v.b, v.D, v.D))).astype(np.float32)
    opt = headline_options(gpu_lib, mixture_args(g), dev(v.rot), dev(v.shift), v.D, v.pixel,
                           dev(Y), ctf_arg(v))
    announce(f"  autotuned options tile={opt.tile} halo={opt.halo} budget={opt.budget}")
    _check_adjoint(gpu_lib, g, v, (3, 17, 40, 63), seed=130, options=opt)


def test_b256_forward_and_adjoint_subset(gpu_lib):
    g, v, _gt, _rn = inputs.c2()
    B, D = v.b, v.D
    idx = (0, 31, 64, 100, 128, 170, 222, 255)
    Y = (1e-3 * np.random.default_rng(131).standard_normal((B, D, D))).astype(np.float32)
    announce("N=20000 B=256 D=128: images of 8 of 256 vs oracle")
    loss, _, X = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y),
                                       ctf=ctf_arg(v), reduction="mean", want_grads=False,
                                       want_images=True)
    torch.cuda.synchronize()
    _check_images(X, loss, g, v, Y, idx, 1.0 / (B * D * D))
    announce("N=20000 B=256 D=128: adjoint with dL/dimages on 8 images vs oracle")
    _check_adjoint(gpu_lib, g, v, idx, seed=132)


def test_uneven_batch_real_mixtures(gpu_lib):
    mixtures = inputs.c3()
    probs, host_side = [], []
    for k, (g, v, _gt, _rn) in enumerate(mixtures):
        Y = (1e-3 * np.random.default_rng(140 + k).standard_normal((v.b, v.D, v.D))).astype(np.float32)
        probs.append(gpu_lib.make_problem(**mixture_args(g), **view_args(v), observed=dev(Y),
                                          ctf=ctf_arg(v), reduction="mean", want_images=True))
        host_side.append((g, v, Y))
    announce("eight mixtures N=5k..150k x 128 images: autotune")
    gpu_lib.autotune(probs, reps=1)
    announce(f"  options {[(p.options.tile, p.options.halo, p.options.budget) for p in probs]}")
    gpu_lib.loss_and_grad_multi(probs, use_graph=True)
    torch.cuda.synchronize()
    for k, (pr, (g, v, Y)) in enumerate(zip(probs, host_side)):
        announce(f"  mixture {k} (N={g.n}, D={v.D}): images 0 and 127 vs oracle")
        _check_images(pr.images_out, pr.loss, g, v, Y, (0, v.b - 1), 1.0 / (v.b * v.D * v.D))
    announce("  batched launch vs separate calls (bitwise)")
    for pr in probs:
        loss, grads, X = gpu_lib.loss_and_grad(pr.means, pr.log_scales, pr.quats, pr.amps, pr.rot,
                                               pr.shift, pr.D, pr.pixel, pr.observed, ctf=pr.ctf,
                                               options=pr.options, reduction="mean",
                                               want_images=True)
        torch.cuda.synchronize()
        assert torch.equal(loss, pr.loss)
        assert torch.equal(X, pr.images_out)
        for key in GROUPS:
            assert torch.equal(grads[key], pr.grads[key]), key
    for k, (pr, (g, v, Y)) in enumerate(zip(probs, host_side)):
        announce(f"  mixture {k}: adjoint (autotuned options) on images 5 and 90 vs oracle")
        _check_adjoint(gpu_lib, g, v, (5, 90), seed=150 + k, options=pr.options)


def test_headline_pair_count_vs_oracle(gpu_lib):
    """The pair count that prices the headline roofline (N = 200,000, 64
    images of 256^2): cs_pair_count over all 64 images, images 0 and 63
    against the oracle's exact count (Eq. 8 splat with q <= q_cut; FP32 and
    FP64 may place pixels sitting on the cut on different sides)."""
    from oracle import model as o_model
    g, v, _gt, _rn = inputs.c4()
    announce("headline pair count, images 0 and 63 vs oracle")
    got = host(gpu_lib.pair_count(**mixture_args(g), **view_args(v)))
    assert got.shape == (64,)
    for b in (0, 63):
        ref = o_model.pair_count(g.means, g.log_scales, g.quats, v.rot[b:b + 1], v.shift[b:b + 1],
                                 v.D, v.pixel, Q_MATCHED)[0]
        announce(f"  image {b}: {int(got[b])} vs {int(ref)}")
        assert abs(got[b] - ref) <= 1e-5 * ref + 2
