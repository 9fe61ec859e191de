"""The training step at its full size (N = 200,000 Gaussians, 64 images of
256^2, 1.1 A, CTF, mean reduction), in the launch configuration the bench
times (options from the library's autotuner on the same problem): two sampled images and their losses against the
FP64 oracle, computed image by image, and the full-batch gradient through
the directional derivative of the loss (a central difference of the
library's own loss along the gradient, a property that holds at any size).
The observed images are seeded normal draws, so no oracle input comes from
the library."""
import numpy as np
import pytest
import torch

from oracle import objective
from paper_2508_04929_amd import inputs

from gpu_util import announce, ctf_arg, dev, headline_options, host, mixture_args, normwise

pytestmark = pytest.mark.gpu

Q_MATCHED = 2.0 * np.log(1e6)


def _one(v, i):
    return inputs.Views(rot=v.rot[i:i + 1], shift=v.shift[i:i + 1], defocus_u=v.defocus_u[i:i + 1],
                        defocus_v=v.defocus_v[i:i + 1], astig=v.astig[i:i + 1],
                        phase=v.phase[i:i + 1], D=v.D, pixel=v.pixel)


def test_training_step_full_size(gpu_lib):
    g, v, _gt, _rn = inputs.c4()
    B, D = v.rot.shape[0], v.D
    # observed images at the scale of the rendered ones (RMS about 2e-6), so the
    # loss depends on X as much as on Y
    Y = (2e-6 * np.random.default_rng(120).standard_normal((B, D, D))).astype(np.float32)
    m = mixture_args(g)
    rot, shift, ctf, Yd = dev(v.rot), dev(v.shift), ctf_arg(v), dev(Y)
    announce("full-size training step N=200000 B=64 D=256 (autotuned launch options, as the bench)")
    opt = headline_options(gpu_lib, m, rot, shift, D, v.pixel, Yd, ctf)
    announce(f"  options tile={opt.tile} halo={opt.halo} budget={opt.budget}")
    loss, grads, X = gpu_lib.loss_and_grad(m["means"], m["log_scales"], m["quats"], m["amps"], rot,
                                           shift, D, v.pixel, Yd, ctf=ctf, reduction="mean",
                                           want_images=True, options=opt)
    torch.cuda.synchronize()
    lo, Xh = host(loss), host(X)
    for b in (0, 41):
        announce(f"  oracle image {b}")
        ref = objective.forward(g, _one(v, b), Y[b:b + 1], q_cut=Q_MATCHED, reduction="sum")
        assert normwise(Xh[b], ref["X"][0]) <= 1e-4
        assert lo[b] == pytest.approx(ref["loss"] / (B * D * D), rel=1e-4)
    assert lo[-1] == pytest.approx(lo[:-1].sum(), rel=1e-5)
    # directional derivative along the gradient: (L(p + h d) - L(p - h d)) / 2h = |g|
    keys = ("means", "log_scales", "quats", "amps")
    gnorm = float(np.sqrt(sum(float((grads[k].double() ** 2).sum()) for k in keys)))
    h = 1e-3 * float(lo[-1]) / gnorm
    vals = []
    for sgn in (1.0, -1.0):
        p = {k: (m[k] + sgn * h * grads[k] / gnorm).contiguous() for k in keys}
        l2, _, _ = gpu_lib.loss_and_grad(p["means"], p["log_scales"], p["quats"], p["amps"], rot,
                                         shift, D, v.pixel, Yd, ctf=ctf, reduction="mean",
                                         want_grads=False, options=opt)
        vals.append(float(l2[-1]))
    fd = (vals[0] - vals[1]) / (2 * h)
    announce(f"  directional derivative {fd:.6e} vs |g| {gnorm:.6e}")
    assert fd == pytest.approx(gnorm, rel=1e-2)
