"""cs_loss_and_grad_noalloc: the training-step entry point that runs in the
library's static device scratch instead of an allocated workspace (GPU).

Each call goes through the C-ABI twice, once through cs_loss_and_grad and
once through cs_loss_and_grad_noalloc, on the same seeded inputs; the two
must agree to the parity bar (images 1e-4 per image, gradients 1e-3 per
group, normwise) and in fact bitwise, since both run the same kernels in
the same order.  Two calls in a row, the second smaller, show that what the
first leaves in the shared scratch does not leak into the second.
"""
import numpy as np
import pytest
import torch

from paper_2508_04929_amd import binding, inputs

from gpu_util import announce, ctf_arg, dev, host, mixture_args, normwise, per_image_normwise, view_args

pytestmark = pytest.mark.gpu
GROUPS = ("means", "log_scales", "quats", "amps")


def _case(seed, n, b, D, pixel):
    rng = np.random.default_rng(seed)
    g = inputs.mixture_anisotropic(rng, n, 0.3 * D * pixel)
    v = inputs.views(rng, b, D, pixel, shift_px_sd=2.0)
    Y = (1e-3 * rng.standard_normal((b, D, D))).astype(np.float32)
    return g, v, Y


def _outputs(n, b, D, pose):
    z = lambda *s: torch.full(s, float("nan"), device="cuda", dtype=torch.float32)
    gr = {"means": z(n, 3), "log_scales": z(n, 3), "quats": z(n, 4), "amps": z(n)}
    if pose:
        gr.update(rot=z(b, 3, 3), shift=z(b, 2))
    return z(b + 1), gr, z(b, D, D)


def _compare(lib, g, v, Y, pose):
    n, b, D = g.n, v.b, v.D
    args = dict(**mixture_args(g), **view_args(v), observed=dev(Y), ctf=ctf_arg(v),
                reduction="mean", want_pose_grads=pose)
    loss_r, gr_r, X_r = lib.loss_and_grad(**args, want_images=True)
    loss_n, gr_n, X_n = _outputs(n, b, D, pose)
    lib.loss_and_grad(**args, grads=gr_n, loss=loss_n, images=X_n, noalloc=True)
    torch.cuda.synchronize()
    img_err = per_image_normwise(host(X_n), host(X_r))
    loss_err = normwise(host(loss_n), host(loss_r))
    assert img_err <= 1e-4, img_err
    assert loss_err <= 1e-4, loss_err
    for k in gr_r:
        e = normwise(host(gr_n[k]), host(gr_r[k]))
        assert e <= 1e-3, (k, e)
    # same kernels, same order, same twiddle table: identical bits
    assert torch.equal(X_n, X_r)
    assert torch.equal(loss_n, loss_r)
    for k in gr_r:
        assert torch.equal(gr_n[k], gr_r[k]), k
    return img_err


def test_noalloc_matches_loss_and_grad_twice_second_smaller(gpu_lib):
    announce("noalloc: N=6000 B=6 D=96 with pose gradients, then N=1500 B=3 D=64")
    g, v, Y = _case(71, 6000, 6, 96, 1.5)
    _compare(gpu_lib, g, v, Y, pose=True)
    g, v, Y = _case(72, 1500, 3, 64, 1.8)
    _compare(gpu_lib, g, v, Y, pose=False)


def test_noalloc_makes_no_device_allocation(gpu_lib):
    announce("noalloc: free device memory unchanged over three calls")
    g, v, Y = _case(73, 4000, 4, 96, 1.5)
    m, vw, c = mixture_args(g), view_args(v), ctf_arg(v)
    obs = dev(Y)
    loss, gr, X = _outputs(g.n, v.b, v.D, False)
    call = lambda: gpu_lib.loss_and_grad(**m, **vw, observed=obs, ctf=c, reduction="mean",
                                         grads=gr, loss=loss, images=X, noalloc=True)
    call()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        call()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    assert torch.isfinite(loss).all()


def test_noalloc_rejects_work_beyond_the_scratch(gpu_lib):
    announce("noalloc: a call too large for the static scratch is refused before launch")
    n, b, D = 200000, 16, 256
    z = lambda *s: torch.zeros(s, device="cuda", dtype=torch.float32)
    rot = torch.eye(3, device="cuda").repeat(b, 1, 1).contiguous()
    quats = z(n, 4)
    quats[:, 0] = 1.0
    with pytest.raises(binding.CryoSplatError) as ei:
        gpu_lib.loss_and_grad(z(n, 3), z(n, 3), quats, z(n), rot, z(b, 2), D, 1.1, z(b, D, D),
                              noalloc=True)
    assert "(-3)" in str(ei.value) and "static scratch" in str(ei.value)
