"""Host logic of the paper-faithful trainer (paper_2508_04929_amd/trainer.py)
without a GPU: a recording stand-in for the library checks that Alg. 1's
outer loop centres the particles once with direction -1, visits every
particle once per epoch in a fresh order, decays the learning rate as
lr_0 gamma^e (Sec. 4.1), continues the Adam step count across epochs and
splits the mixture after exactly the listed epochs."""
import numpy as np
import torch

from paper_2508_04929_amd import trainer


class Recorder:
    def __init__(self):
        self.calls = []

    def init_attributes(self, z):
        return torch.zeros(11 * z.shape[0])

    def fourier_shift(self, images, shift, pixel, direction=1):
        self.calls.append(("shift", direction, pixel))
        return images + 1.0

    def train_sequential(self, params, m, v, images, rot, pixel, order, step0, lr, **kw):
        self.calls.append(("train", np.asarray(order).copy(), step0, lr, float(images[0, 0, 0]),
                           params.numel(), kw.get("options")))

    def split_gaussians(self, params, m, v, **kw):
        self.calls.append(("split", params.numel()))
        return (torch.zeros(2 * params.numel()), torch.zeros(2 * params.numel()),
                torch.zeros(2 * params.numel()))


def _data(m=7, D=8, shift=True):
    return trainer.Dataset(images=torch.zeros(m, D, D), rot=torch.eye(3).repeat(m, 1, 1),
                           shift=torch.zeros(m, 2) if shift else None)


def test_outer_loop_orders_decay_steps_and_splits():
    lib = Recorder()
    tr = trainer.Trainer(lib, torch.zeros(5, 3))
    assert tr.options.graph == 0
    tr.fit(_data(), epochs=4, lr=2e-3, gamma=0.5, seed=3, densify_after=(1, 2))
    shifts = [c for c in lib.calls if c[0] == "shift"]
    trains = [c for c in lib.calls if c[0] == "train"]
    splits = [c for c in lib.calls if c[0] == "split"]
    assert shifts == [("shift", -1, 1.0 / 8)]
    assert len(trains) == 4
    for e, c in enumerate(trains):
        assert sorted(c[1].tolist()) == list(range(7))         # every particle once
        assert c[2] == 7 * e                                    # Adam steps continue
        assert c[3] == 2e-3 * 0.5 ** e                          # lr_0 gamma^e
        assert c[4] == 1.0                                      # the centred images
    assert not all(np.array_equal(trains[0][1], c[1]) for c in trains[1:])  # fresh orders
    # splits after epochs 1 and 2: 55 -> 110 -> 220 parameters
    assert [c[1] for c in splits] == [55, 110]
    assert [c[5] for c in trains] == [55, 55, 110, 220]
    assert tr.n == 20 and tr.step == 28


def test_centring_is_skipped_without_translations_and_orders_are_seeded():
    a, b = Recorder(), Recorder()
    for lib in (a, b):
        trainer.Trainer(lib, torch.zeros(3, 3), graph=True).fit(_data(shift=False), epochs=2, seed=9)
    assert not [c for c in a.calls if c[0] == "shift"]
    ta = [c[1] for c in a.calls if c[0] == "train"]
    tb = [c[1] for c in b.calls if c[0] == "train"]
    assert all(np.array_equal(x, y) for x, y in zip(ta, tb))
    assert [c for c in a.calls if c[0] == "train"][0][6].graph == 1

