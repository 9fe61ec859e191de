"""Pins of the oracle's pair counter and of the listed-pose scorer (CPU).

``oracle.model.pair_count`` counts the (Gaussian, pixel) pairs whose squared
Mahalanobis distance is at most q_cut (the truncation reading of Eq. 8's
splat): it is pinned here by a brute force over every pixel of small images
(no bounding box, the projection written out from scipy's rotation), by the
number of lattice points in a disc for an isotropic Gaussian on a pixel
centre (a textbook count), and by the behaviour at the image border.

``oracle.pose.scores_at`` scores listed (rotation, shift) poses with the
image model and squared error (Eq. 1, 14 and Sec. 3.3.5): pinned by its
equality with the grid scorer at grid poses and shifts, by its zero at the
pose an image was rendered with (a non-zero shift included) and by the
pixel units of its shifts.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import model, objective, pose
from paper_2508_04929_amd import inputs


def _brute_pairs(means, log_scales, quats, rot, shift, D, pixel, q_cut):
    """Every pixel of every image against every Gaussian: q <= q_cut."""
    # scipy takes scalar-last quaternions
    R = Rotation.from_quat(np.asarray(quats, np.float64)[:, [1, 2, 3, 0]]).as_matrix()
    s2 = np.exp(2.0 * np.asarray(log_scales, np.float64))
    c = D // 2
    out = []
    for b in range(len(rot)):
        P = np.asarray(rot[b], np.float64)[:2]
        t = np.zeros(2) if shift is None else np.asarray(shift[b], np.float64)
        n_pairs = 0
        for n in range(len(means)):
            S = R[n] @ np.diag(s2[n]) @ R[n].T
            S2 = P @ S @ P.T
            mu = P @ np.asarray(means[n], np.float64) + t
            Ci = np.linalg.inv(S2)
            for i in range(D):
                for j in range(D):
                    d = np.array([(j - c) * pixel, -(i - c) * pixel]) - mu
                    if d @ Ci @ d <= q_cut:
                        n_pairs += 1
        out.append(n_pairs)
    return np.array(out)


@pytest.mark.parametrize("D,pixel,seed", [(12, 1.0, 0), (15, 1.3, 1), (16, 0.9, 2)])
def test_pair_count_equals_brute_force_over_every_pixel(D, pixel, seed):
    rng = np.random.default_rng(seed)
    n = 6
    means = rng.uniform(-0.45 * D * pixel, 0.45 * D * pixel, size=(n, 3))   # some cross the border
    log_scales = np.log(rng.uniform(0.5, 1.8, size=(n, 3)) * pixel)
    quats = rng.standard_normal((n, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    rot = Rotation.random(3, random_state=seed + 10).as_matrix()
    shift = rng.normal(0.0, 1.5 * pixel, size=(3, 2))
    for q_cut in (2.0 * np.log(1e6), 9.0, 1.0):
        got = model.pair_count(means, log_scales, quats, rot, shift, D, pixel, q_cut)
        ref = _brute_pairs(means, log_scales, quats, rot, shift, D, pixel, q_cut)
        assert got.dtype.kind == "i"
        np.testing.assert_array_equal(got, ref)


def _lattice_points_in_disc(r2):
    m = int(np.floor(np.sqrt(r2)))
    return sum(1 for x in range(-m, m + 1) for y in range(-m, m + 1) if x * x + y * y <= r2)


def test_pair_count_isotropic_on_pixel_centre_is_a_lattice_disc():
    # 81 lattice points lie in the closed disc of radius 5 (Gauss circle
    # problem, N(5) = 81); with sigma = 1 pixel the cut q <= 25.5 is that disc
    # (no integer x^2 + y^2 lies in (25, 25.5], so rounding of the projected
    # covariance cannot move a lattice point across the cut)
    D, pixel = 32, 1.0
    means = np.zeros((1, 3))
    quats = np.array([[0.3, -0.5, 0.1, 0.8]])
    quats /= np.linalg.norm(quats)
    rot = Rotation.random(4, random_state=7).as_matrix()
    got = model.pair_count(means, np.zeros((1, 3)), quats, rot, None, D, pixel, 25.5)
    np.testing.assert_array_equal(got, [81] * 4)
    # sigma = 2 px and the library's cut: r^2 = 4 q_cut
    q_cut = 2.0 * np.log(1e6)
    got = model.pair_count(means, np.full((1, 3), np.log(2.0)), quats, rot[:1], None, D, pixel,
                           q_cut)
    assert got[0] == _lattice_points_in_disc(4.0 * q_cut)
    # centred on pixel (c + 3, c - 2) by an in-plane shift: same count
    got = model.pair_count(means, np.zeros((1, 3)), quats, rot[:1],
                           np.array([[-2.0 * pixel, -3.0 * pixel]]), D, pixel, 25.5)
    assert got[0] == 81


def test_pair_count_clips_to_the_image():
    # a disc centred on the corner pixel (0, 0) keeps only its quadrant with
    # i, j >= 0: points (x, y) with x, y >= 0 and x^2 + y^2 <= 25.5
    D, pixel = 16, 1.0
    c = D // 2
    means = np.array([[-c * pixel, c * pixel, 0.0]])     # x = -c p -> column 0; y = c p -> row 0
    quad = sum(1 for x in range(0, 6) for y in range(0, 6) if x * x + y * y <= 25)
    got = model.pair_count(means, np.zeros((1, 3)), np.array([[1.0, 0, 0, 0]]), np.eye(3)[None],
                           None, D, pixel, 25.5)
    assert got[0] == quad
    # wholly outside: nothing
    far = np.array([[3.0 * D * pixel, 0.0, 0.0]])
    got = model.pair_count(far, np.zeros((1, 3)), np.array([[1.0, 0, 0, 0]]), np.eye(3)[None],
                           None, D, pixel, 25.5)
    assert got[0] == 0


def test_scores_at_equals_grid_scores_and_vanishes_at_the_rendered_pose():
    rng = np.random.default_rng(4)
    g = inputs.mixture_anisotropic(rng, 40, 9.0)
    v = inputs.views(rng, 1, 24, 1.5)
    G = pose.grid(1, 4)
    k_true, dx, dy = 9, -1, 2                  # a non-zero shift in pixels
    v.rot = G[k_true:k_true + 1].astype(np.float32)
    v.shift = np.array([[dx * v.pixel, dy * v.pixel]], dtype=np.float32)
    Y = objective.forward(g, v)["X"][0]
    grid_sc = pose.scores(g, Y, v, G, shift_radius=1)
    ox, oy = pose.shift_offsets(1)
    # listed poses: several grid rotations, every shift of radius 1
    ks = [0, 5, k_true, 30, 47]
    rots = np.repeat(G[ks], len(ox), axis=0)
    shifts = np.tile(np.stack([ox, oy], axis=1), (len(ks), 1))
    sc = pose.scores_at(g, Y, v, rots, shifts)
    np.testing.assert_allclose(sc, grid_sc[ks].reshape(-1), rtol=1e-12, atol=0)
    # the rendered pose, given in pixels, scores zero; its neighbours do not
    W32 = v.rot.astype(np.float64)             # the rotation exactly as rendered
    z = pose.scores_at(g, Y, v, W32, [[dx, dy]])
    ref = np.sum(Y ** 2)
    assert z[0] <= 1e-24 * ref
    off = pose.scores_at(g, Y, v, G[[k_true] * 3], [[dx + 1, dy], [dx, dy - 1], [0, 0]])
    assert np.all(off > 1e-3 * ref)
    # shifts are in pixels: a shift given in Angstrom (p = 1.5) lands elsewhere
    wrong = pose.scores_at(g, Y, v, W32, [[dx * v.pixel, dy * v.pixel]])
    assert wrong[0] > 1e-3 * ref
    # without the CTF the same zero holds for the pre-CTF render
    Q = objective.forward(g, v)["Q"][0]
    zq = pose.scores_at(g, Q, v, W32, [[dx, dy]], use_ctf=False)
    assert zq[0] <= 1e-24 * np.sum(Q ** 2)
