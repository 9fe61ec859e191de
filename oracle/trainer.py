"""Paper-faithful training loop pieces (oracle, FP64).

Test infrastructure: used only to check the GPU library.

* FourierShift (Alg. 1, "centre alignment"; Sec. 4.1 applies the published
  particle translations to the observed images by a phase shift in Fourier
  space rather than through the viewing transform).  ``fourier_shift``
  translates images by an in-plane vector t (Angstrom): the content at
  image-plane position r moves to r + t.  On the raster of Eq. 13 (x along
  columns, y up while rows go down) that is a_c = t_x / p columns and
  a_r = -t_y / p rows.  Written as the shift theorem on the DFT with signed
  frequency indices (numpy's fftfreq, the Nyquist index as -D/2) and the
  real part of the complex inverse transform; for even D that real part
  weights the Nyquist lines by cos(pi a) (the mean of the two mirror
  frequencies).  Centring an image observed with translation t is
  ``fourier_shift(Y, -t)``, so that it matches the render at t = 0.

* Initialisation (Sec. 4.1): box-normalised domain [-E, E]^3 with E = 1/2
  (pixel 1/D), means ~ N(0, 0.075^2 I), every scale 0.0075, amplitudes
  1/(2N), softplus activations for scales and amplitudes (Sec. 3.3.1), so
  the stored pre-activations are softplus^-1 of those values; the
  quaternion is the identity (the paper does not give it; all scales are
  equal, so it does not change the initial covariance).  The normal draws
  are an input (``z``).

* Schedule (Sec. 4.1): Adam with batch size 1, one learning rate for all
  parameters, lr_e = lr_0 gamma^e in epoch e (exponential decay per epoch,
  gamma = 0.1 for the main experiments, 0.5 for the large-count study).

* Loop (Alg. 1): for every (Y, W, t, H) of an epoch in the given order:
  centre Y, render at W, apply the CTF, squared-error loss, Adam step.
"""
from __future__ import annotations

import numpy as np

from . import adam, objective

INIT_MEAN_STD = 0.075     # 0.9 * E / 6 with E = 1/2
INIT_SCALE = 0.0075       # 0.1 * 0.075


def softplus_inverse(y):
    y = np.asarray(y, dtype=np.float64)
    return np.log(np.expm1(y))


def fourier_shift(Y, shift, pixel):
    """Translate images Y [B, D, D] by shift [B, 2] (t_x, t_y in the units of
    ``pixel``), band-limited and circular (FP64)."""
    Y = np.asarray(Y, dtype=np.float64)
    shift = np.asarray(shift, dtype=np.float64).reshape(-1, 2)
    D = Y.shape[-1]
    k = np.fft.fftfreq(D) * D
    ac = shift[:, 0] / pixel
    ar = -shift[:, 1] / pixel
    phase = np.exp(-2j * np.pi * (k[None, None, :] * ac[:, None, None]
                                  + k[None, :, None] * ar[:, None, None]) / D)
    return np.real(np.fft.ifft2(np.fft.fft2(Y, axes=(-2, -1)) * phase, axes=(-2, -1)))


def init_attributes(z):
    """Pre-activation parameters (means [N,3], log_scales [N,3], quats [N,4],
    amps [N]) from the normal draws z [N, 3] (FP64)."""
    z = np.asarray(z, dtype=np.float64)
    N = z.shape[0]
    means = INIT_MEAN_STD * z
    log_scales = np.full((N, 3), softplus_inverse(INIT_SCALE))
    quats = np.zeros((N, 4))
    quats[:, 0] = 1.0
    amps = np.full(N, softplus_inverse(1.0 / (2.0 * N)))
    return means, log_scales, quats, amps


def learning_rate(lr0, gamma, epoch):
    return lr0 * gamma ** epoch


class Params:
    """Mixture parameters (pre-activation) as FP64 arrays."""

    def __init__(self, means, log_scales, quats, amps):
        self.means, self.log_scales, self.quats, self.amps = means, log_scales, quats, amps

    @property
    def n(self):
        return int(self.means.shape[0])


class State:
    """Parameters and Adam moments as one flat FP64 vector in the order
    means | log_scales | quats | amps (11 values per Gaussian)."""

    def __init__(self, means, log_scales, quats, amps):
        self.n = int(np.asarray(means).shape[0])
        self.theta = np.concatenate([np.asarray(a, dtype=np.float64).ravel()
                                     for a in (means, log_scales, quats, amps)])
        self.m = np.zeros_like(self.theta)
        self.v = np.zeros_like(self.theta)
        self.step = 0

    def mixture(self):
        n, t = self.n, self.theta
        return Params(t[:3 * n].reshape(n, 3), t[3 * n:6 * n].reshape(n, 3),
                      t[6 * n:10 * n].reshape(n, 4), t[10 * n:])


def train_step(state, view, Y, *, lr, reduction="sum", q_cut=None, use_ctf=True,
               scale_act="softplus", amp_act="softplus"):
    """One batch-1 step of Alg. 1 on a centred image Y [1, D, D]; returns the
    loss before the update."""
    f = objective.loss_and_grad(state.mixture(), view, Y, q_cut=q_cut, reduction=reduction,
                                scale_act=scale_act, amp_act=amp_act, use_ctf=use_ctf)
    g = f["grads"]
    grad = np.concatenate([np.asarray(g[k], dtype=np.float64).ravel()
                           for k in ("means", "log_scales", "quats", "amps")])
    state.step += 1
    state.theta, state.m, state.v = adam.adam_step(state.theta, grad, state.m, state.v,
                                                   state.step, lr=lr)
    return f["loss"]


def train(state, views_of, images, order, *, lr, **kw):
    """Steps over the images in ``order`` (indices); ``views_of(i)`` gives the
    one-image view record of image i, ``images`` the centred images."""
    losses = []
    for i in order:
        losses.append(train_step(state, views_of(int(i)), images[int(i)][None], lr=lr, **kw))
    return np.array(losses)
