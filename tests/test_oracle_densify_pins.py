"""Pins of the densification oracle (oracle/densify.py): each pair of
children carries its parent's mass, mean and covariance (closed form,
through the model's own covariance), the isotropic tie rule, mass
conservation of the rendered images, and two splits in a row."""
import numpy as np
import pytest

from oracle import densify, model
from paper_2508_04929_amd import inputs


def _mix(seed, n=40):
    rng = np.random.default_rng(seed)
    g = inputs.mixture_anisotropic(rng, n, 10.0)
    return rng, g


@pytest.mark.parametrize("scale_act,amp_act", [("exp", "identity"), ("softplus", "softplus")])
def test_children_keep_mass_mean_and_covariance(scale_act, amp_act):
    rng, g = _mix(80)
    if scale_act == "softplus":
        g.log_scales = np.log(np.expm1(rng.uniform(0.5, 3.0, size=(g.n, 3)))).astype(np.float32)
        g.amps = np.log(np.expm1(rng.uniform(0.1, 2.0, size=g.n))).astype(np.float32)
    n = g.n
    m, ls, q, a, k = densify.split(g.means, g.log_scales, g.quats, g.amps, scale_act, amp_act)
    S0 = model.covariance(np.asarray(g.log_scales, np.float64), g.quats, scale_act)
    Sc = model.covariance(ls, q, scale_act)
    A0 = model.amps_from(np.asarray(g.amps, np.float64), amp_act)
    Ac = model.amps_from(a, amp_act)
    np.testing.assert_allclose(Ac[:n] + Ac[n:], A0, rtol=1e-12)
    np.testing.assert_allclose(0.5 * (m[:n] + m[n:]), g.means, rtol=0, atol=1e-12)
    d = 0.5 * (m[:n] - m[n:])
    pair_cov = Sc[:n] + np.einsum("ni,nj->nij", d, d)
    np.testing.assert_allclose(pair_cov, S0, rtol=1e-10, atol=1e-12 * np.abs(S0).max())
    np.testing.assert_allclose(Sc[:n], Sc[n:], rtol=0, atol=0)
    # the split axis is the largest scale's
    s = model.scales_from(np.asarray(g.log_scales, np.float64), scale_act)
    assert np.all(s[np.arange(n), k] == s.max(axis=1))


def test_isotropic_gaussians_split_along_their_first_axis():
    n = 5
    rng = np.random.default_rng(81)
    means = rng.standard_normal((n, 3))
    ls = np.full((n, 3), np.log(2.0))
    quats = inputs.haar_quaternions(rng, n)
    m, new_ls, q, a, k = densify.split(means, ls, quats, np.ones(n))
    assert np.all(k == 0)
    R = model.rotation_from_quaternion(quats / np.linalg.norm(quats, axis=1, keepdims=True))
    np.testing.assert_allclose(m[:n] - means, 1.0 * R[:, :, 0], atol=1e-12)
    np.testing.assert_allclose(np.exp(new_ls[:, 0]), np.sqrt(3.0), rtol=1e-12)
    np.testing.assert_allclose(np.exp(new_ls[:, 1:]), 2.0, rtol=1e-12)
    np.testing.assert_allclose(a, 0.5, rtol=0)


def test_split_conserves_the_projected_mass():
    """The images' pixel sums (times p^2) equal the total amplitude before and
    after the split, for Gaussians well inside the raster."""
    rng, g = _mix(82, n=12)
    g.means = (0.3 * g.means).astype(np.float32)
    D, p = 64, 1.0
    W = inputs.haar_rotations(rng, 2)
    before = model.render_pre_ctf(g.means, g.log_scales, g.quats, g.amps, W, None, D, p)
    m, ls, q, a, _ = densify.split(g.means, g.log_scales, g.quats, g.amps)
    after = model.render_pre_ctf(m, ls, q, a, W, None, D, p)
    total = float(np.sum(g.amps))
    np.testing.assert_allclose(before.sum(axis=(1, 2)) * p * p, total, rtol=1e-6)
    np.testing.assert_allclose(after.sum(axis=(1, 2)) * p * p, total, rtol=1e-6)


def test_two_splits_keep_the_moments_of_each_family():
    rng, g = _mix(83, n=10)
    n = g.n
    m1, l1, q1, a1, _ = densify.split(g.means, g.log_scales, g.quats, g.amps)
    m2, l2, q2, a2, _ = densify.split(m1, l1, q1, a1)
    S = model.covariance(l2, q2)
    # family of parent i: indices i, n + i, 2n + i, 3n + i
    fam = np.stack([np.arange(n) + j * n for j in range(4)], axis=1)
    mass = a2[fam].sum(axis=1)
    mean = (a2[fam][..., None] * m2[fam]).sum(axis=1) / mass[:, None]
    dev = m2[fam] - mean[:, None, :]
    cov = (a2[fam][..., None, None] * (S[fam] + np.einsum("nfi,nfj->nfij", dev, dev))).sum(axis=1) / mass[:, None, None]
    np.testing.assert_allclose(mass, g.amps, rtol=1e-12)
    np.testing.assert_allclose(mean, g.means, atol=1e-12)
    np.testing.assert_allclose(cov, model.covariance(np.asarray(g.log_scales, np.float64), g.quats),
                               rtol=1e-9, atol=1e-12)


def test_flat_layout_and_moments():
    rng, g = _mix(84, n=7)
    n = g.n
    theta = np.concatenate([np.asarray(x, np.float32).ravel()
                            for x in (g.means, g.log_scales, g.quats, g.amps)])
    out = densify.split_flat(theta, n)
    m, ls, q, a, _ = densify.split(g.means, g.log_scales, g.quats, g.amps)
    np.testing.assert_array_equal(out, np.concatenate([m.ravel(), ls.ravel(), q.ravel(), a]))
    mom = np.arange(11 * n, dtype=np.float64)
    dup = densify.duplicate_moments(mom, n)
    assert dup.shape == (22 * n,)
    np.testing.assert_array_equal(dup[:3 * n], mom[:3 * n])
    np.testing.assert_array_equal(dup[3 * n:6 * n], mom[:3 * n])
    np.testing.assert_array_equal(dup[-2 * n:], np.concatenate([mom[10 * n:], mom[10 * n:]]))
