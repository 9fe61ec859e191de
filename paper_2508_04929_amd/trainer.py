"""Alg. 1 with the settings of Sec. 4.1: box-normalised units, the paper's
initialisation, FourierShift centring of the observed images, Adam at batch
size 1 with one learning rate, exponential decay per epoch.

Host logic only (epoch loop, per-epoch orders, the decay schedule); every
arithmetic step runs in libcryosplat: ``cs_init_attributes``,
``cs_fourier_shift``, ``cs_train_sequential`` (which stages each image, so
that the loss path can also be replayed as a HIP graph), ``cs_split_gaussians``
for densification, ``cs_voxelize`` / ``cs_fsc`` for the read-out.  Eager
launches are the default: a step's GPU work outlasts its host-side launches,
so a graph replay only adds its own fixed cost.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

from . import binding


@dataclasses.dataclass
class Dataset:
    """Device tensors of a training set in box units (pixel 1/D); ``ctf``
    per image with ``pixel_a`` the Angstrom pixel of its frequency grid."""
    images: torch.Tensor                   # [M, D, D] observed
    rot: torch.Tensor                      # [M, 3, 3]
    shift: Optional[torch.Tensor] = None   # [M, 2] translations (box units), or None
    ctf: Optional[binding.Ctf] = None

    @property
    def m(self):
        return int(self.images.shape[0])

    @property
    def D(self):
        return int(self.images.shape[-1])

    @property
    def pixel(self):
        return 1.0 / self.D


class Trainer:
    """Flat parameters [11 N] (means | log_scales | quats | amps, softplus
    activations) and Adam moments on one device."""

    def __init__(self, lib: binding.Library, z: torch.Tensor, graph: bool = False,
                 options: Optional[binding.Options] = None):
        self.lib = lib
        self.n = int(z.shape[0])
        self.params = lib.init_attributes(z.contiguous())
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        base = options or binding.Options()
        self.options = dataclasses.replace(base, graph=1 if graph else 0)

    def views(self):
        n, p = self.n, self.params
        return {"means": p[:3 * n].view(n, 3), "log_scales": p[3 * n:6 * n].view(n, 3),
                "quats": p[6 * n:10 * n].view(n, 4), "amps": p[10 * n:].view(n)}

    @staticmethod
    def centre(lib, data: Dataset) -> Dataset:
        """FourierShift(Y, t) of Alg. 1 once for the whole set (Sec. 4.1
        applies the translations before reconstruction)."""
        if data.shift is None:
            return data
        images = lib.fourier_shift(data.images, data.shift, data.pixel, direction=-1)
        return Dataset(images=images, rot=data.rot, shift=None, ctf=data.ctf)

    def epoch(self, data: Dataset, order, lr: float, loss: Optional[torch.Tensor] = None):
        """One pass over ``order`` at batch size 1 (images already centred)."""
        self.lib.train_sequential(self.params, self.m, self.v, data.images, data.rot, data.pixel,
                                  order, self.step, lr, ctf=data.ctf, options=self.options,
                                  loss=loss)
        self.step += len(order)
        return loss

    def densify(self):
        """SplitGaussian for every Gaussian (Alg. 1): the count doubles; the
        children inherit their parent's Adam moments."""
        self.params, self.m, self.v = self.lib.split_gaussians(self.params, self.m, self.v)
        self.n *= 2

    def fit(self, data: Dataset, epochs: int = 5, lr: float = 1e-3, gamma: float = 0.1,
            seed: int = 0, record_loss: bool = False, on_epoch=None, densify_after=()):
        """Alg. 1's outer loop: per epoch e a fresh random order of the set
        and learning rate lr gamma^e; after every epoch listed in
        ``densify_after`` (IsDoubleGaussians) all Gaussians are split.
        Returns the per-step losses when asked."""
        data = self.centre(self.lib, data)
        rng = np.random.default_rng(seed)
        losses = []
        for e in range(epochs):
            order = rng.permutation(data.m)
            loss = (torch.empty(data.m, device=self.params.device) if record_loss else None)
            self.epoch(data, order, lr * gamma ** e, loss)
            if record_loss:
                losses.append(loss)
            if e in densify_after:
                self.densify()
            if on_epoch is not None:
                on_epoch(e, self)
        return torch.cat(losses) if record_loss else None

    def voxelize(self, D: int, out=None):
        """The current mixture on a D^3 grid of the box (pixel 1/D)."""
        w = self.views()
        return self.lib.voxelize(w["means"], w["log_scales"], w["quats"], w["amps"], D, 1.0 / D,
                                 scale_act="softplus", amp_act="softplus", out=out)
