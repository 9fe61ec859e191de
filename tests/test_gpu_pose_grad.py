"""Pose gradients (dL/dW entry-wise, dL/dt) of the HIP adjoint against the
FP64 oracle: element by element (<= 1e-3 normwise per group, the gradient
bar), against finite differences of the oracle loss, batched vs single
calls (bitwise), through the autograd wrapper, a property at the full
training size, and a few steps of gradient-based pose refinement."""
import numpy as np
import pytest
import torch

from oracle import ctf as o_ctf
from oracle import model as o_model
from oracle import objective as o_obj
from oracle import pose as o_pose
from paper_2508_04929_amd import autograd, binding, inputs

from gpu_util import announce, ctf_arg, dev, host, mixture_args, normwise, view_args

pytestmark = pytest.mark.gpu

Q_MATCHED = 2.0 * np.log(1e6)
GRAD_TOL = 1e-3


def _oracle_Q(g, v, q_cut=Q_MATCHED):
    return o_model.render_pre_ctf(g.means, g.log_scales, g.quats, g.amps, v.rot, v.shift, v.D,
                                  v.pixel, q_cut)


def test_pose_gradients_c2_subset(gpu_lib):
    g, v, gt, rn = inputs.c2(b=256)
    v = v.subset(np.arange(4))
    announce("pose gradients, N=20000 B=4 D=128 with CTF, vs oracle")
    H = o_ctf.ctf_grid_for(v)
    Y = inputs.add_noise(rn, o_ctf.apply_ctf(_oracle_Q(gt, v), H), -20.0)
    ref = o_obj.loss_and_grad(g, v, Y, q_cut=Q_MATCHED)["grads"]
    _, grads, _ = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y),
                                        ctf=ctf_arg(v), want_pose_grads=True)
    for k in ("rot", "shift", "means"):
        err = normwise(host(grads[k]), ref[k])
        announce(f"  {k}: normwise {err:.2e}")
        assert err <= GRAD_TOL, (k, err)
    assert torch.all(grads["rot"][:, 2, :] == 0)


@pytest.mark.parametrize("use_ctf", [False, True])
def test_render_backward_pose_gradients(gpu_lib, use_ctf):
    rng = np.random.default_rng(31 + int(use_ctf))
    g = inputs.mixture_anisotropic(rng, 2000, 22.0)
    v = inputs.views(rng, 3, 96, 1.3, shift_px_sd=2.0)
    dX = rng.standard_normal((3, 96, 96)).astype(np.float32)
    announce(f"render_backward pose gradients, ctf={use_ctf}")
    got = gpu_lib.render_backward(**mixture_args(g), **view_args(v), d_images=dev(dX),
                                  ctf=ctf_arg(v) if use_ctf else None, want_pose_grads=True)
    GQ = o_ctf.apply_ctf(dX, o_ctf.ctf_grid_for(v)) if use_ctf else dX
    ref = o_obj.backward_from_image_grad(g, v, GQ, q_cut=Q_MATCHED)
    for k in ("rot", "shift"):
        err = normwise(host(got[k]), ref[k])
        announce(f"  {k}: normwise {err:.2e}")
        assert err <= GRAD_TOL, (k, err)


def test_pose_gradients_vs_finite_differences(gpu_lib):
    rng = np.random.default_rng(33)
    g = inputs.mixture_anisotropic(rng, 40, 8.0)
    v = inputs.views(rng, 3, 32, 1.0, shift_px_sd=1.0)
    Y = (0.01 * rng.standard_normal((3, 32, 32))).astype(np.float32)
    announce("pose gradients vs FP64 finite differences")
    _, grads, _ = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=dev(Y),
                                        ctf=ctf_arg(v), want_pose_grads=True)
    for field in ("rot", "shift"):
        got = host(grads[field])
        ent = [tuple(e) for e in np.ndindex(got.shape)]
        fd = o_obj.finite_difference_view(g, v, Y, field, ent, q_cut=None)
        gv = np.array([got[e] for e in ent])
        assert np.abs(gv - fd).max() <= GRAD_TOL * np.abs(gv).max(), field


def test_pose_gradients_batched_equal_single(gpu_lib):
    """Two problems in one persistent launch give the same pose gradients as
    two separate calls, bit for bit."""
    rng = np.random.default_rng(34)
    probs, singles = [], []
    for i, (n, D) in enumerate(((1500, 64), (600, 48))):
        g = inputs.mixture_anisotropic(rng, n, 0.3 * D)
        v = inputs.views(rng, 3, D, 1.0, shift_px_sd=1.5)
        Y = dev(rng.standard_normal((3, D, D)).astype(np.float32))
        args = dict(**mixture_args(g), **view_args(v), observed=Y, ctf=ctf_arg(v))
        probs.append(gpu_lib.make_problem(**args, want_pose_grads=True))
        singles.append(gpu_lib.loss_and_grad(**args, want_pose_grads=True)[1])
    gpu_lib.loss_and_grad_multi(probs, use_graph=False)
    torch.cuda.synchronize()
    for pr, s in zip(probs, singles):
        for k in ("rot", "shift", "means", "quats"):
            assert torch.equal(pr.grads[k], s[k]), k


def test_autograd_pose_gradients(gpu_lib):
    rng = np.random.default_rng(35)
    g = inputs.mixture_anisotropic(rng, 800, 15.0)
    v = inputs.views(rng, 2, 64, 1.0, shift_px_sd=1.0)
    Y = dev(rng.standard_normal((2, 64, 64)).astype(np.float32))
    m = mixture_args(g)
    rot, shift = dev(v.rot).requires_grad_(), dev(v.shift).requires_grad_()
    ctf = ctf_arg(v)
    loss = autograd.splat_loss(m["means"], m["log_scales"], m["quats"], m["amps"], rot, shift, Y,
                               64, 1.0, ctf=ctf, reduction="sum")
    (3.0 * loss).backward()
    _, ref, _ = gpu_lib.loss_and_grad(**m, rot=rot.detach(), shift=shift.detach(), D=64,
                                      pixel=1.0, observed=Y, ctf=ctf, want_pose_grads=True)
    assert torch.allclose(rot.grad, 3.0 * ref["rot"], rtol=1e-6, atol=0)
    assert torch.allclose(shift.grad, 3.0 * ref["shift"], rtol=1e-6, atol=0)
    # render + an upstream image gradient: the same pose gradients as the adjoint
    rot.grad = None
    shift.grad = None
    X = autograd.splat_render(m["means"], m["log_scales"], m["quats"], m["amps"], rot, shift, 64,
                              1.0, ctf=ctf)
    dX = torch.randn_like(X)
    (X * dX).sum().backward()
    rb = gpu_lib.render_backward(**m, rot=rot.detach(), shift=shift.detach(), D=64, pixel=1.0,
                                 d_images=dX, ctf=ctf, want_pose_grads=True)
    assert torch.equal(rot.grad, rb["rot"]) and torch.equal(shift.grad, rb["shift"])


def test_pose_gradient_translation_identity_full_size(gpu_lib):
    """N = 200,000, D = 256, one view: dL/dt = P sum_n dL/dmu_n, computed by
    two different reductions (over Gaussians per view, and per Gaussian
    over views), within the FP32 summation error of 200,000 terms."""
    g, v, gt, rn = inputs.c4(b=1)
    announce("pose-gradient translation identity at N=200000, D=256")
    Y = dev(rn.standard_normal((1, v.D, v.D)).astype(np.float32))
    _, grads, _ = gpu_lib.loss_and_grad(**mixture_args(g), **view_args(v), observed=Y,
                                        ctf=ctf_arg(v), want_pose_grads=True)
    P = dev(v.rot)[0, :2].double()
    lhs = grads["shift"][0].double()
    rhs = P @ grads["means"].double().sum(0)
    scale = (grads["means"].double().abs().sum(0)).max()
    err = float((lhs - rhs).abs().max() / scale)
    announce(f"  |dL/dt - P sum dL/dmu| / sum|dL/dmu| = {err:.2e}")
    assert err <= 1e-5


def _so3_step(W, dW, lr):
    """W exp(-lr [w]x) with w_k = <dW, W K_k> (the gradient of the right
    perturbation), by Rodrigues' formula."""
    K = torch.zeros(3, 3, 3, dtype=W.dtype, device=W.device)
    K[0, 1, 2], K[0, 2, 1] = -1, 1
    K[1, 0, 2], K[1, 2, 0] = 1, -1
    K[2, 0, 1], K[2, 1, 0] = -1, 1
    w = torch.stack([(dW * (W @ K[c])).sum((1, 2)) for c in range(3)], 1)
    a = -lr * w
    th = a.norm(dim=1, keepdim=True).clamp_min(1e-12)
    k = a / th
    Kx = torch.einsum("bc,cij->bij", k, K)
    s, c = torch.sin(th)[..., None], torch.cos(th)[..., None]
    Rr = torch.eye(3, dtype=W.dtype, device=W.device) + s * Kx + (1 - c) * (Kx @ Kx)
    return W @ Rr


def test_gradient_pose_refinement_reduces_error(gpu_lib):
    """From poses 4 degrees and 1.5 pixels off, plain gradient steps on
    (rotation, shift) with the library's pose gradients move every particle
    toward its true pose and lower the loss."""
    rng = np.random.default_rng(36)
    D, pixel = 96, 1.5
    g = inputs.mixture_domains(rng, 3000, radius=30.0)
    v = inputs.views(rng, 8, D, pixel, shift_px_sd=0.0)
    announce("gradient-based pose refinement, 8 particles, D=96")
    ctf = ctf_arg(v)
    m = mixture_args(g)
    W_true, t_true = dev(v.rot), dev(v.shift)
    Y = gpu_lib.render(**m, rot=W_true, shift=t_true, D=D, pixel=pixel, ctf=ctf)
    axis = torch.nn.functional.normalize(torch.randn(8, 3, device="cuda", dtype=torch.float64), dim=1)
    ang = np.deg2rad(4.0)
    K = torch.zeros(8, 3, 3, device="cuda", dtype=torch.float64)
    K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -axis[:, 2], axis[:, 1], -axis[:, 0]
    K = K - K.transpose(1, 2)
    R0 = torch.eye(3, device="cuda", dtype=torch.float64) + np.sin(ang) * K + (1 - np.cos(ang)) * (K @ K)
    W = (W_true.double() @ R0)
    t = t_true.double() + 1.5 * pixel * torch.nn.functional.normalize(
        torch.randn(8, 2, device="cuda", dtype=torch.float64), dim=1)
    err0 = o_pose.angular_distance_deg(host(W), host(W_true))
    losses = []
    for it in range(40):
        loss, gr, _ = gpu_lib.loss_and_grad(**m, rot=W.float().contiguous(), shift=t.float().contiguous(),
                                            D=D, pixel=pixel, observed=Y, ctf=ctf,
                                            want_pose_grads=True)
        per = loss[:-1].double()
        losses.append(float(loss[-1]))
        # per-particle step sizes from the gradient scale (a normalised step)
        dW, dt = gr["rot"].double(), gr["shift"].double()
        W = _so3_step(W, dW / dW.flatten(1).norm(dim=1)[:, None, None].clamp_min(1e-30),
                      np.deg2rad(0.25))
        t = t - 0.1 * pixel * dt / dt.norm(dim=1, keepdim=True).clamp_min(1e-30)
    err1 = o_pose.angular_distance_deg(host(W), host(W_true))
    terr = (t - t_true.double()).norm(dim=1)
    announce(f"  angular error {np.median(err0):.2f} -> {np.median(err1):.2f} deg, "
             f"loss {losses[0]:.3e} -> {losses[-1]:.3e}, shift error {float(terr.max()) / pixel:.2f} px")
    assert losses[-1] < 0.2 * losses[0]
    assert np.all(err1 < err0)
    assert float(terr.max()) < 1.5 * pixel
