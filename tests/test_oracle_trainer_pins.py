"""Pins of the training-loop oracle (oracle/trainer.py): FourierShift against
whole-pixel rolls, the renderer's own translation and closed forms on the
Nyquist lines; the initialisation against its stated values; the first
Adam step of a training step against its closed form; a short noiseless
training run against the loss it must lower."""
import numpy as np
import pytest

from oracle import model, objective, trainer
from paper_2508_04929_amd import inputs


def test_fourier_shift_whole_pixels_is_a_roll():
    """t = (3 p, -2 p): columns +3, rows +2 (y up, rows down, Eq. 13)."""
    rng = np.random.default_rng(60)
    Y = rng.standard_normal((2, 16, 16))
    p = 1.7
    out = trainer.fourier_shift(Y, [[3 * p, -2 * p], [-5 * p, 4 * p]], p)
    np.testing.assert_allclose(out[0], np.roll(Y[0], (2, 3), axis=(0, 1)), atol=1e-12)
    np.testing.assert_allclose(out[1], np.roll(Y[1], (-4, -5), axis=(0, 1)), atol=1e-12)


def test_fourier_shift_matches_the_rendered_translation():
    """Smooth Gaussians (widths >= 2.5 px, far from the border): shifting the
    t = 0 render by a sub-pixel t equals rendering at t (the image model's
    own mu~ = P mu + t), to the aliasing level of the band limit."""
    rng = np.random.default_rng(61)
    D, p = 64, 1.0
    g = inputs.mixture_anisotropic(rng, 12, 6.0)
    g.log_scales = np.log(rng.uniform(2.5, 3.0, size=(12, 3))).astype(np.float32)
    W = inputs.haar_rotations(rng, 3)
    t = np.array([[0.37, -1.61], [2.25, 0.5], [-0.8, 3.3]])
    args = (g.means, g.log_scales, g.quats, g.amps)
    Q0 = model.render_pre_ctf(*args, W, np.zeros((3, 2)), D, p)
    Qt = model.render_pre_ctf(*args, W, t, D, p)
    out = trainer.fourier_shift(Q0, t, p)
    assert np.abs(out - Qt).max() <= 1e-9 * np.abs(Qt).max()
    # centring undoes the translation
    back = trainer.fourier_shift(Qt, -t, p)
    assert np.abs(back - Q0).max() <= 1e-9 * np.abs(Q0).max()


@pytest.mark.parametrize("a", [0.5, 0.3, 1.25])
def test_fourier_shift_nyquist_lines(a):
    """Pure Nyquist patterns: (-1)^c moved by a columns becomes
    cos(pi a) (-1)^c, (-1)^r by a rows cos(pi a) (-1)^r, and the corner
    pattern (-1)^(r+c) moved by (a, b) becomes cos(pi (a + b)) (-1)^(r+c)."""
    D, p = 8, 1.0
    r, c = np.meshgrid(np.arange(D), np.arange(D), indexing="ij")
    col = (-1.0) ** c
    row = (-1.0) ** r
    cor = (-1.0) ** (r + c)
    np.testing.assert_allclose(trainer.fourier_shift(col[None], [[a, 0.0]], p)[0],
                               np.cos(np.pi * a) * col, atol=1e-12)
    np.testing.assert_allclose(trainer.fourier_shift(row[None], [[0.0, -a]], p)[0],
                               np.cos(np.pi * a) * row, atol=1e-12)
    b = 0.2
    np.testing.assert_allclose(trainer.fourier_shift(cor[None], [[a, -b]], p)[0],
                               np.cos(np.pi * (a + b)) * cor, atol=1e-12)


def test_init_attributes_values():
    z = np.random.default_rng(62).standard_normal((1000, 3))
    means, ls, q, A = trainer.init_attributes(z)
    np.testing.assert_allclose(means, 0.075 * z, rtol=1e-15)
    np.testing.assert_allclose(model.scales_from(ls, "softplus"), 0.0075, rtol=1e-12)
    np.testing.assert_allclose(model.amps_from(A, "softplus"), 1.0 / 2000, rtol=1e-12)
    np.testing.assert_allclose(model.covariance(ls, q, "softplus"),
                               np.broadcast_to(0.0075 ** 2 * np.eye(3), (1000, 3, 3)), rtol=1e-12)
    assert trainer.learning_rate(1e-3, 0.1, 0) == 1e-3
    assert trainer.learning_rate(1e-3, 0.1, 3) == pytest.approx(1e-6, rel=1e-12)


def _problem(seed, n=20, D=24):
    rng = np.random.default_rng(seed)
    g = inputs.mixture_anisotropic(rng, n, 0.15)
    g.log_scales = trainer.softplus_inverse(rng.uniform(0.02, 0.05, size=(n, 3)))
    g.amps = trainer.softplus_inverse(rng.uniform(0.01, 0.05, size=n))
    v = inputs.views(rng, 6, D, 1.0 / D)
    v.pixel_a = 3.0
    v.defocus_u = v.defocus_v = (rng.uniform(1.0, 2.0, 6) * 1e4).astype(np.float32)
    return rng, g, v


def _one(v, i):
    return inputs.Views(rot=v.rot[i:i + 1], shift=v.shift[i:i + 1], defocus_u=v.defocus_u[i:i + 1],
                        defocus_v=v.defocus_v[i:i + 1], astig=v.astig[i:i + 1],
                        phase=v.phase[i:i + 1], D=v.D, pixel=v.pixel, pixel_a=v.pixel_a)


def test_first_training_step_is_a_signed_lr_move():
    """Adam's first step moves each parameter by lr g / (|g| + eps) against
    its gradient; the loss returned is the one before the update."""
    rng, g, v = _problem(63)
    Y = rng.standard_normal((1, v.D, v.D))
    st = trainer.State(g.means, g.log_scales, g.quats, g.amps)
    before = st.theta.copy()
    f = objective.loss_and_grad(st.mixture(), _one(v, 0), Y, scale_act="softplus",
                                amp_act="softplus")
    grad = np.concatenate([f["grads"][k].ravel() for k in ("means", "log_scales", "quats", "amps")])
    loss = trainer.train_step(st, _one(v, 0), Y, lr=1e-3)
    assert loss == pytest.approx(f["loss"], rel=1e-12)
    np.testing.assert_allclose(st.theta - before, -1e-3 * grad / (np.abs(grad) + 1e-8),
                               rtol=1e-9, atol=1e-18)


def test_noiseless_training_lowers_the_loss():
    """Data rendered (with CTF, normalised units) from a mixture; training
    starts from a perturbed copy and two epochs at batch 1 lower the mean
    loss of the data set."""
    rng, g, v = _problem(64, n=15, D=24)
    Y = objective.forward(g, v, scale_act="softplus", amp_act="softplus")["X"]
    pert = trainer.State(g.means + 0.01 * rng.standard_normal(g.means.shape), g.log_scales,
                         g.quats, g.amps)

    def mean_loss(st):
        return float(np.mean([objective.forward(st.mixture(), _one(v, i), Y[i:i + 1],
                                                scale_act="softplus", amp_act="softplus")["loss"]
                              for i in range(6)]))

    l0 = mean_loss(pert)
    for e in range(2):
        trainer.train(pert, lambda i: _one(v, i), Y, rng.permutation(6),
                      lr=trainer.learning_rate(2e-3, 0.5, e))
    assert mean_loss(pert) < 0.5 * l0


def test_normalised_units_scale_the_image_by_the_box_length_squared():
    """The same mixture and CTF in Angstrom (pixel p) and in box units
    (lengths / L, L = D p, pixel 1/D, the CTF on the Angstrom grid): the
    projected density scales as L^2 (Eq. 8's 1 / (2 pi sqrt det)), the CTF
    is unchanged, so X_box = L^2 X_A."""
    rng = np.random.default_rng(65)
    D, p = 32, 2.5
    L = D * p
    g = inputs.mixture_anisotropic(rng, 25, 18.0)
    v = inputs.views(rng, 3, D, p)
    f64 = lambda a: np.asarray(a, dtype=np.float64)
    box = inputs.Mixture(f64(g.means) / L, f64(g.log_scales) - np.log(L), g.quats, g.amps)
    vb = inputs.Views(rot=v.rot, shift=f64(v.shift) / L, defocus_u=v.defocus_u, defocus_v=v.defocus_v,
                      astig=v.astig, phase=v.phase, D=D, pixel=1.0 / D, pixel_a=p)
    XA = objective.forward(g, v)["X"]
    XB = objective.forward(box, vb)["X"]
    np.testing.assert_allclose(XB, L ** 2 * XA, rtol=1e-9, atol=1e-12 * np.abs(L ** 2 * XA).max())
