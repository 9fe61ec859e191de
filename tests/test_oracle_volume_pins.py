"""Pins of the voxelisation and FSC oracle (oracle/volume.py) against
closed forms, the image oracle and properties of Eq. 10."""
import numpy as np
import pytest

from oracle import model, volume
from paper_2508_04929_amd import inputs


def _mix(rng, n, radius, s_lo=1.2, s_hi=2.5):
    g = inputs.mixture_anisotropic(rng, n, radius)
    g.log_scales = np.log(rng.uniform(s_lo, s_hi, size=(n, 3))).astype(np.float32)
    return g


def test_voxel_mass_equals_total_amplitude():
    """Gaussians well inside the box: sum V p^3 = sum A (closed-form integral)."""
    rng = np.random.default_rng(40)
    g = _mix(rng, 6, 6.0)
    D, p = 40, 1.0
    V = volume.voxelize(g, D, p)
    assert abs(V.sum() * p ** 3 - g.amps.astype(np.float64).sum()) < 1e-6 * g.amps.sum()


def test_voxel_single_gaussian_closed_form():
    """One axis-aligned Gaussian: the value at the voxel nearest its mean."""
    g = inputs.Mixture(means=np.array([[0.3, -0.2, 0.1]], np.float32),
                       log_scales=np.log(np.array([[1.5, 2.0, 2.5]], np.float32)),
                       quats=np.array([[1, 0, 0, 0]], np.float32),
                       amps=np.array([2.0], np.float32))
    V = volume.voxelize(g, 16, 1.0)
    x = np.array([0.0, 0.0, 0.0]) - g.means[0].astype(np.float64)
    s = np.exp(g.log_scales[0].astype(np.float64))
    ref = 2.0 / ((2 * np.pi) ** 1.5 * s.prod()) * np.exp(-0.5 * ((x / s) ** 2).sum())
    assert abs(V[8, 8, 8] - ref) < 1e-12 * ref


def test_voxel_projection_is_the_identity_pose_image():
    """p * sum_z V = the oracle's pre-CTF image at the identity rotation
    (rows flipped: image row i is y = (c0 - i) p)."""
    rng = np.random.default_rng(41)
    g = _mix(rng, 8, 5.0)
    D, p = 32, 1.0
    V = volume.voxelize(g, D, p)
    img = model.render_pre_ctf(g.means, g.log_scales, g.quats, g.amps,
                               np.eye(3)[None], np.zeros((1, 2)), D, p)[0]
    proj = V.sum(axis=0) * p          # [iy][ix], y increasing with iy
    ref = img[::-1, :]                # image rows run downwards in y
    ref = np.roll(ref, 1 if D % 2 == 0 else 0, axis=0)  # row c0 -> y = 0
    assert np.abs(proj - ref).max() < 1e-6 * np.abs(ref).max()


def test_fsc_self_negation_and_scaling():
    rng = np.random.default_rng(42)
    V = rng.standard_normal((24, 24, 24))
    np.testing.assert_allclose(volume.fsc(V, V), 1.0, atol=1e-12)
    np.testing.assert_allclose(volume.fsc(V, -V), -1.0, atol=1e-12)
    np.testing.assert_allclose(volume.fsc(V, 3.5 * V), 1.0, atol=1e-12)
    W = rng.standard_normal((24, 24, 24))
    np.testing.assert_allclose(volume.fsc(V, W), volume.fsc(W, V), atol=1e-12)


def test_fsc_parseval_and_shell_counts():
    """The shell denominators add up to D^3 sum V^2 over shells <= D/2 plus
    the corners, and a constant volume has all its energy in shell 0."""
    rng = np.random.default_rng(43)
    D = 20
    V = rng.standard_normal((D, D, D))
    _, da, _ = volume.fsc_sums(V, V)
    F = np.fft.fftn(V)
    f = np.fft.fftfreq(D) * D
    kz, ky, kx = np.meshgrid(f, f, f, indexing="ij")
    s = np.rint(np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)).astype(int)
    direct = np.bincount(s.ravel(), (np.abs(F) ** 2).ravel())[:D // 2 + 1]
    np.testing.assert_allclose(da, direct, rtol=1e-12)
    C = np.full((D, D, D), 2.0)
    _, dc, _ = volume.fsc_sums(C, C)
    assert dc[0] > 0 and np.all(dc[1:] < 1e-12 * dc[0])


def test_fsc_of_a_circular_shift_is_the_shell_mean_of_the_phase():
    """V_b(x) = V_a(x - s) circularly: the shift theorem gives, shell by
    shell, sum |V^_a|^2 cos(2 pi k.s / D) / sum |V^_a|^2, evaluated here
    by direct enumeration of the full spectrum (no transform of V_b)."""
    rng = np.random.default_rng(44)
    D = 16
    Va = rng.standard_normal((D, D, D))
    s = np.array([1, -2, 3])          # (z, y, x) voxels
    Vb = np.roll(Va, shift=tuple(s), axis=(0, 1, 2))
    F = np.fft.fftn(Va)
    f = np.fft.fftfreq(D) * D
    kz, ky, kx = np.meshgrid(f, f, f, indexing="ij")
    sh = np.rint(np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)).astype(int)
    ph = np.cos(2 * np.pi * (kz * s[0] + ky * s[1] + kx * s[2]) / D)
    P = np.abs(F) ** 2
    num = np.bincount(sh.ravel(), (P * ph).ravel())[:D // 2 + 1]
    den = np.bincount(sh.ravel(), P.ravel())[:D // 2 + 1]
    np.testing.assert_allclose(volume.fsc(Va, Vb), num / den, atol=1e-12)


def test_resolution_threshold():
    curve = np.array([1.0, 0.9, 0.5, 0.2, 0.1, 0.05])
    assert volume.resolution(curve, 10, 2.0) == pytest.approx(10 * 2.0 / 4)
    assert volume.resolution(np.ones(6), 10, 2.0) == pytest.approx(10 * 2.0 / 5)
