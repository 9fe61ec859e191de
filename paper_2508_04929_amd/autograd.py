"""torch.autograd.Function wrappers of the HIP renderer.

``SplatRender`` maps Gaussian parameters to images (with or without CTF);
its backward is the library's adjoint (App. A.2, Eq. 15-21) applied to the
upstream image gradient, including the gradients w.r.t. the views'
rotation matrices and shifts when those require grad (joint pose and
Gaussian optimisation).  ``SplatLoss`` fuses render, squared-error loss
(Sec. 3.3.5) and adjoint in one library call: the forward computes the
gradients and the backward only scales them by the upstream scalar.

Only tensors and launch arguments are marshalled here; all arithmetic of
the renderer runs in libcryosplat.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import binding


class SplatRender(torch.autograd.Function):
    """images = render(means, log_scales, quats, amps; poses, CTF)."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, amps, rot, shift, D: int, pixel: float,
                ctf: Optional[binding.Ctf] = None, options: Optional[binding.Options] = None,
                scale_act: str = "exp", amp_act: str = "identity"):
        lib = binding.library()
        args = [t.detach().contiguous() for t in (means, log_scales, quats, amps)]
        rot = rot.detach().contiguous()
        shift = None if shift is None else shift.detach().contiguous()
        images = lib.render(*args, rot, shift, D, pixel, ctf=ctf, options=options,
                            scale_act=scale_act, amp_act=amp_act)
        ctx.save_for_backward(*args, rot, shift if shift is not None else torch.empty(0))
        ctx.meta = (D, pixel, ctf, options, scale_act, amp_act, shift is not None)
        return images

    @staticmethod
    def backward(ctx, d_images):
        means, log_scales, quats, amps, rot, shift = ctx.saved_tensors
        D, pixel, ctf, options, scale_act, amp_act, has_shift = ctx.meta
        pose = ctx.needs_input_grad[4] or (has_shift and ctx.needs_input_grad[5])
        lib = binding.library()
        g = lib.render_backward(means, log_scales, quats, amps, rot,
                                shift if has_shift else None, D, pixel,
                                d_images.contiguous(), ctf=ctf, options=options,
                                scale_act=scale_act, amp_act=amp_act, want_pose_grads=pose)
        return (g["means"], g["log_scales"], g["quats"], g["amps"],
                g["rot"] if pose and ctx.needs_input_grad[4] else None,
                g["shift"] if pose and has_shift and ctx.needs_input_grad[5] else None,
                None, None, None, None, None, None)


class SplatLoss(torch.autograd.Function):
    """loss = scale * sum ||render(...) - observed||^2 (scalar)."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, amps, rot, shift, observed, D: int, pixel: float,
                ctf: Optional[binding.Ctf] = None, options: Optional[binding.Options] = None,
                reduction: str = "mean", scale_act: str = "exp", amp_act: str = "identity"):
        lib = binding.library()
        args = [t.detach().contiguous() for t in (means, log_scales, quats, amps)]
        pose = ctx.needs_input_grad[4] or (shift is not None and ctx.needs_input_grad[5])
        want = any(ctx.needs_input_grad[:4]) or pose
        loss, grads, _ = lib.loss_and_grad(*args, rot.detach().contiguous(),
                                           None if shift is None else shift.detach().contiguous(),
                                           D, pixel, observed.contiguous(),
                                           ctf=ctf, options=options, reduction=reduction,
                                           want_grads=want, scale_act=scale_act,
                                           amp_act=amp_act, want_pose_grads=pose)
        if want:
            z = torch.empty(0, device=rot.device)
            ctx.save_for_backward(grads["means"], grads["log_scales"], grads["quats"],
                                  grads["amps"], grads.get("rot", z), grads.get("shift", z))
        ctx.want, ctx.pose = want, pose
        return loss[-1]

    @staticmethod
    def backward(ctx, g_out):
        if not ctx.want:
            return (None,) * 14
        gm, gl, gq, ga, gr, gs = ctx.saved_tensors
        return (gm * g_out, gl * g_out, gq * g_out, ga * g_out,
                gr * g_out if ctx.pose and ctx.needs_input_grad[4] else None,
                gs * g_out if ctx.pose and ctx.needs_input_grad[5] else None,
                None, None, None, None, None, None, None, None)


def splat_render(means, log_scales, quats, amps, rot, shift, D, pixel, ctf=None, options=None,
                 scale_act="exp", amp_act="identity"):
    return SplatRender.apply(means, log_scales, quats, amps, rot, shift, D, pixel, ctf, options,
                             scale_act, amp_act)


def splat_loss(means, log_scales, quats, amps, rot, shift, observed, D, pixel, ctf=None,
               options=None, reduction="mean", scale_act="exp", amp_act="identity"):
    return SplatLoss.apply(means, log_scales, quats, amps, rot, shift, observed, D, pixel, ctf,
                           options, reduction, scale_act, amp_act)
