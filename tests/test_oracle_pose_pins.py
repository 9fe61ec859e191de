"""Pins of the pose oracle (CPU): grids, scores and refinement candidates.

The HEALPix enumeration is pinned by the known nside = 1 centres and by
properties every HEALPix tessellation has (pixel count, ring populations,
antipodal symmetry, near-uniform spacing); the view rotation by scipy's
intrinsic ZYZ Euler matrices; the score by its zero at the rendered pose;
the closed-form in-plane angle of the refinement rule by brute force.
"""
import numpy as np
from scipy.spatial.transform import Rotation

from oracle import pose
from paper_2508_04929_amd import inputs


def _unit(th, ph):
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)


def test_healpix_nside1_centres():
    th, ph = pose.healpix_directions(1)
    np.testing.assert_allclose(np.cos(th), [2 / 3] * 4 + [0] * 4 + [-2 / 3] * 4, atol=1e-15)
    q = np.pi / 4
    np.testing.assert_allclose(ph, [q, 3 * q, 5 * q, 7 * q, 0, 2 * q, 4 * q, 6 * q,
                                    q, 3 * q, 5 * q, 7 * q], atol=1e-15)


def test_healpix_tessellation_properties():
    for N in (1, 2, 4, 8):
        th, ph = pose.healpix_directions(N)
        n = _unit(th, ph)
        assert len(n) == 12 * N * N
        np.testing.assert_allclose(n.sum(axis=0), 0.0, atol=1e-9)
        # every centre's antipode is a centre
        d = np.abs(n @ (-n).T - 1.0).min(axis=1)
        assert d.max() < 1e-12
        # rings: 4i pixels in the caps, 4N in the belt
        z, counts = np.unique(np.round(np.cos(th), 12), return_counts=True)
        assert len(z) == 4 * N - 1
        if N > 1:
            assert sorted(counts.tolist())[:2] == [4, 4]
        # near-uniform spacing: nearest-neighbour angles within a factor 2
        g = np.clip(n @ n.T, -1, 1)
        np.fill_diagonal(g, -2)
        nn = np.arccos(g.max(axis=1))
        assert nn.max() / nn.min() < 2.0


def test_view_rotation_matches_scipy_euler_and_direction():
    rng = np.random.default_rng(0)
    for _ in range(20):
        th, ph, ps = rng.uniform(0, np.pi), rng.uniform(0, 2 * np.pi), rng.uniform(0, 2 * np.pi)
        W = pose.view_rotation(th, ph, ps)
        ref = Rotation.from_euler("ZYZ", [ps, -th, -ph]).as_matrix()
        np.testing.assert_allclose(W, ref, atol=1e-14)
        np.testing.assert_allclose(W[2], _unit(np.array([th]), np.array([ph]))[0], atol=1e-14)
    G = pose.grid(2, 6)
    np.testing.assert_allclose(np.einsum("kji,kjl->kil", G, G),
                               np.broadcast_to(np.eye(3), G.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(G), 1.0, atol=1e-14)


def test_angular_distance():
    R = Rotation.random(10, random_state=1).as_matrix()
    a = Rotation.from_rotvec(np.radians(17.0) * np.array([[0.6, 0.0, 0.8]])).as_matrix()[0]
    np.testing.assert_allclose(pose.angular_distance_deg(R, R @ a), 17.0, atol=1e-9)
    np.testing.assert_allclose(pose.angular_distance_deg(R, R), 0.0, atol=1e-5)


def test_score_vanishes_at_the_rendered_pose():
    rng = np.random.default_rng(2)
    g = inputs.mixture_anisotropic(rng, 60, 10.0)
    v = inputs.views(rng, 1, 32, 1.5)
    G = pose.grid(1, 4)
    k_true, dx, dy = 17, 1, -2
    v.rot = G[k_true:k_true + 1].astype(np.float32)
    v.shift = np.array([[dx * v.pixel, dy * v.pixel]], dtype=np.float32)
    from oracle import objective
    Y = objective.forward(g, v)["X"][0]
    sc = pose.scores(g, Y, v, G, shift_radius=2)
    s_true = (dy + 2) * 5 + (dx + 2)
    assert sc[k_true, s_true] < 1e-20 * np.abs(Y).sum() ** 2 + 1e-24
    assert np.all(sc >= 0)
    k, s = np.unravel_index(np.argmin(sc), sc.shape)
    assert (k, s) == (k_true, s_true)
    # shift index convention: (dx, dy) = (s % 5 - 2, s // 5 - 2)
    ox, oy = pose.shift_offsets(2)
    assert (ox[s_true], oy[s_true]) == (dx, dy)


def test_refinement_psi_rule_and_candidates():
    rng = np.random.default_rng(3)
    n_psi = 12
    bank = pose.grid(2, n_psi)
    psis = np.linspace(-np.pi, np.pi, 200001)
    for _ in range(10):
        W = Rotation.random(random_state=rng.integers(1 << 30)).as_matrix()
        A = bank[::n_psi]
        d = int(np.argmax(A[:, 2, :] @ W[2]))
        M = A[d] @ W.T
        closed = np.arctan2(M[0, 1] - M[1, 0], M[0, 0] + M[1, 1])
        tr = [np.trace(W.T @ pose._rz(p) @ A[d]) for p in psis[::50]]
        brute = psis[::50][int(np.argmax(tr))]
        assert abs(np.angle(np.exp(1j * (closed - brute)))) < 2e-3
        c = pose.refine_candidates(W, bank, n_psi, 4, 3)
        assert len(c) == 12 and c[0] // n_psi == d
    # a proposal on the grid recovers its own index first in its direction
    k = 5 * n_psi + 7
    c = pose.refine_candidates(bank[k], bank, n_psi, 3, 3)
    assert k in c[:3]


def _fit_case(seed=31):
    rng = np.random.default_rng(seed)
    g = inputs.mixture_anisotropic(rng, 40, 6.0)
    v = inputs.views(rng, 1, 24, 1.5)
    W = pose.grid(1, 4)[5]
    X = pose.model.render_pre_ctf(g.means, g.log_scales, g.quats, g.amps, W[None],
                                  np.array([[1.0, -1.0]]) * 1.5, v.D, v.pixel)
    X = pose.ctf_mod.apply_ctf(X, pose.ctf_mod.ctf_grid_for(v)[0])[0]
    return g, v, W, X, rng


def test_fit_statistic_closed_forms():
    """z = 2 c - 1 for a particle equal to c times the template at the
    pose (c = 1: exact fit; c = 0: an empty particle gives -1), and
    z = 2 a - 1 with a = <X, Y> / ||X||^2 for any particle."""
    g, v, W, X, rng = _fit_case()
    for c in (1.0, 0.5, 2.0, 0.0):
        z = pose.fit_statistic(g, c * X, v, W, [1.0, -1.0])
        assert abs(z - (2 * c - 1)) <= 1e-12 * max(1.0, abs(2 * c - 1))
    N = rng.standard_normal(X.shape)
    Y = 0.7 * X + 0.1 * np.abs(X).max() * N
    a = np.sum(X * Y) / np.sum(X * X)
    assert abs(pose.fit_statistic(g, Y, v, W, [1.0, -1.0]) - (2 * a - 1)) <= 1e-12
    # a template at another shift fits worse than the particle's own
    assert pose.fit_statistic(g, X, v, W, [0.0, 0.0]) < 1.0 - 1e-3
