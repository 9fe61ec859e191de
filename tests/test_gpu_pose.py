"""Pose scoring on the GPU vs the FP64 pose oracle.

The oracle renders every (rotation, shift) candidate from scratch, applies
the particle's CTF and sums squared differences.  The GPU scores against
bfloat16 template banks with FP32 accumulation, so scores agree to the
bfloat16 operand precision: normwise <= 2e-3 of the particle's largest
score (unit roundoff 2^-9 on both operands of each product).  Where
floating point decides the argmin, the check is that the GPU's choice is
optimal under the oracle's scores within that tolerance.
"""
import numpy as np
import pytest
import torch

from oracle import model, objective
from oracle import pose as o_pose
from paper_2508_04929_amd import binding, inputs

from gpu_util import announce, ctf_arg, dev, host, mixture_args, normwise

pytestmark = pytest.mark.gpu
TOL = 2e-3
U_BF16 = 2.0 ** -9  # unit roundoff of bfloat16 (round to nearest even)


def _bf16_bound(g, Y, particle, rotations, r):
    """Elementwise bound on |GPU score - exact score| from bfloat16 operands.

    The GPU sums w_f |Q^_k(f)|^2 (energy E_k = ||H Q_k||^2) and
    -2 Q_k . S_t Z (Z = H Y) with each factor rounded to bfloat16, so every
    product carries a relative error of at most 2u + u^2; FP32 accumulation
    adds at most n * 2^-24 of the absolute sum.  Bound per (k, s):
        (2u + u^2 + n 2^-24) (E_k + 2 sum |Q_k| |S_t Z|)."""
    D = particle.D
    Q = model.render_pre_ctf(g.means, g.log_scales, g.quats, g.amps, rotations,
                             np.zeros((len(rotations), 2)), D, particle.pixel)
    from oracle import ctf as o_ctf
    H = o_ctf.ctf_grid_for(particle)[0]
    E = np.sum(o_ctf.apply_ctf(Q, H) ** 2, axis=(1, 2))
    Z = o_ctf.apply_ctf(np.asarray(Y, dtype=np.float64), H)
    ox, oy = o_pose.shift_offsets(r)
    absQ = np.abs(Q).reshape(len(Q), -1)
    absC = np.stack([absQ @ np.abs(np.roll(Z, (dy, -dx), axis=(0, 1))).ravel()
                     for dx, dy in zip(ox, oy)], axis=1)
    rel = 2 * U_BF16 + U_BF16 ** 2 + D * D * 2.0 ** -24
    return rel * (E[:, None] + 2.0 * absC)


def _f64(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _particles(g, P, D, pixel, rng, noise_rel=0.3, shift_px=None, q_cut=None):
    v = inputs.views(rng, P, D, pixel)
    if shift_px is not None:
        v.shift = (np.asarray(shift_px, dtype=np.float64) * pixel).astype(np.float32)
    X = objective.forward(g, v, q_cut=q_cut)["X"]
    Y = X + noise_rel * X.std() * rng.standard_normal(X.shape)
    return v, Y.astype(np.float32)


def test_grid_matches_oracle(gpu_lib):
    for nside, n_psi in ((1, 8), (4, 24), (8, 48)):
        np.testing.assert_allclose(gpu_lib.pose_grid(nside, n_psi), o_pose.grid(nside, n_psi),
                                   atol=2e-6)


def test_grid_search_scores_match_oracle(gpu_lib):
    announce("grid search vs oracle scores, D=48, 96 rotations x 25 shifts")
    rng = np.random.default_rng(900)
    g = inputs.mixture_anisotropic(rng, 300, 12.0)
    D, pixel = 48, 1.5
    G = o_pose.grid(1, 8).astype(np.float32)
    v, Y = _particles(g, 3, D, pixel, rng, shift_px=[[0, 0], [1, -2], [-1, 1]])
    bank = gpu_lib.pose_bank(**mixture_args(g), rot=dev(G), n_psi=8, D=D, pixel=pixel)
    out = bank.grid_search(dev(Y), ctf=ctf_arg(v), shift_radius=2, want_scores=True)
    torch.cuda.synchronize()
    scores = host(out["scores"])
    for p in range(3):
        ref = o_pose.scores(g, Y[p], v.subset([p]), _f64(G), 2)
        bound = _bf16_bound(g, Y[p], v.subset([p]), _f64(G), 2)
        err = np.abs(scores[p] - ref)
        announce(f"  particle {p}: max |err| / bound = {np.max(err / bound):.3f}, "
                 f"normwise {normwise(scores[p], ref):.2e}")
        assert np.all(err <= bound), p
        k, s = int(out["rot_idx"][p]), int(out["shift_idx"][p])
        assert ref[k, s] <= ref.min() + bound[k, s] + bound.flat[np.argmin(ref)], p
        # the reported minimum is the minimum of the reported scores
        assert float(out["score"][p]) == scores[p].min()
    bank.close()


@pytest.mark.parametrize("D", [48, 64])
def test_refine_explicit_candidates_match_grid_scores(gpu_lib, D):
    """D = 48: each lane tracks its own image row; D = 64 (a multiple of 32):
    all lanes change row together."""
    announce(f"refine with explicit candidate lists, D={D}")
    rng = np.random.default_rng(901)
    g = inputs.mixture_anisotropic(rng, 400, 12.0)
    pixel = 1.5
    G = o_pose.grid(1, 8).astype(np.float32)
    P, L = 4, 40
    v, Y = _particles(g, P, D, pixel, rng)
    bank = gpu_lib.pose_bank(**mixture_args(g), rot=dev(G), n_psi=8, D=D, pixel=pixel)
    full = bank.grid_search(dev(Y), ctf=ctf_arg(v), shift_radius=2, want_scores=True)
    cand = rng.integers(0, len(G), size=(P, L)).astype(np.int32)
    cand[:, 3] = -1
    cand[:, 7] = len(G) + 5  # skipped entries
    out = bank.refine(dev(Y), ctf=ctf_arg(v), cand=torch.from_numpy(cand).cuda(), shift_radius=2,
                      want_scores=True)
    torch.cuda.synchronize()
    fs, rs = host(full["scores"]), host(out["scores"])
    for p in range(P):
        ok = (cand[p] >= 0) & (cand[p] < len(G))
        assert normwise(rs[p][ok], fs[p][cand[p][ok]]) <= 1e-4
        k = int(out["rot_idx"][p])
        assert k in set(cand[p][ok].tolist())
        best = fs[p][cand[p][ok]].min()
        assert abs(float(out["score"][p]) - best) <= 1e-4 * fs[p].max()
    bank.close()


def test_refine_candidates_from_proposals(gpu_lib):
    announce("refinement candidates from proposals")
    rng = np.random.default_rng(902)
    g = inputs.mixture_anisotropic(rng, 200, 10.0)
    n_psi = 24
    G = o_pose.grid(4, n_psi).astype(np.float32)
    P = 64
    v, Y = _particles(g, P, 32, 2.0, rng)
    props = inputs.haar_rotations(rng, P).astype(np.float32)
    bank = gpu_lib.pose_bank(**mixture_args(g), rot=dev(G), n_psi=n_psi, D=32, pixel=2.0)
    out = bank.refine(dev(Y), ctf=ctf_arg(v), proposal=dev(props), n_dir=6, n_psi_c=3,
                      shift_radius=1)
    torch.cuda.synchronize()
    cand = out["cand"].cpu().numpy()
    mismatches = 0
    for p in range(P):
        ref = o_pose.refine_candidates(_f64(props[p]), _f64(G), n_psi, 6, 3)
        if not np.array_equal(cand[p], ref):
            mismatches += 1
    # FP32 vs FP64 can only differ on near-ties of direction dots or psi rounding
    assert mismatches <= 1, mismatches
    assert int(out["rot_idx"].min()) >= 0
    bank.close()


def test_grid_search_full_size_sampled(gpu_lib):
    """N=20k mixture, D=128, HEALPix nside 4 x 24 psi (4,608 rotations) x 25 shifts."""
    announce("grid search at 20k Gaussians, D=128, 4608 x 25 (sampled oracle checks)")
    rng = np.random.default_rng(903)
    g = inputs.mixture_anisotropic(rng, 20000, 50.0)
    D, pixel = 128, 1.5
    G = o_pose.grid(4, 24).astype(np.float32)
    P = 3
    # truncation at relative 1e-16 (exact in FP64) keeps the oracle renders short
    v, Y = _particles(g, P, D, pixel, rng, noise_rel=3.0,
                      shift_px=[[0, 0], [2, -1], [-2, 2]], q_cut=model.Q_FAITHFUL)
    bank = gpu_lib.pose_bank(**mixture_args(g), rot=dev(G), n_psi=24, D=D, pixel=pixel)
    out = bank.grid_search(dev(Y), ctf=ctf_arg(v), shift_radius=2)
    torch.cuda.synchronize()
    ox, oy = o_pose.shift_offsets(2)
    for p in range(P):
        announce(f"  oracle scores for particle {p}")
        k, s = int(out["rot_idx"][p]), int(out["shift_idx"][p])
        near = int(np.argmin(o_pose.angular_distance_deg(_f64(G), _f64(v.rot[p]))))
        true_s = np.rint(v.shift[p] / pixel).astype(int)
        ks = [k, near] + rng.integers(0, len(G), 3).tolist()
        sh = [(ox[s], oy[s]), tuple(true_s)] + [(ox[j], oy[j]) for j in rng.integers(0, 25, 3)]
        ref = o_pose.scores_at(g, Y[p], v.subset([p]), _f64(G[ks]), np.array(sh, dtype=float),
                               q_cut=model.Q_FAITHFUL)
        assert abs(float(out["score"][p]) - ref[0]) <= TOL * ref.max()
        assert ref[0] <= ref.min() + TOL * ref.max(), (p, ref[0], ref.min())
    bank.close()


def test_batch_api_matches_convenience_calls_and_filter(gpu_lib):
    announce("pose batch API and CTF filter")
    rng = np.random.default_rng(904)
    g = inputs.mixture_anisotropic(rng, 300, 12.0)
    D, pixel = 48, 1.5
    G = o_pose.grid(1, 8).astype(np.float32)
    v, Y = _particles(g, 5, D, pixel, rng)
    bank = gpu_lib.pose_bank(**mixture_args(g), rot=dev(G), n_psi=8, D=D, pixel=pixel)
    ref = bank.grid_search(dev(Y), ctf=ctf_arg(v), shift_radius=2, want_scores=True)
    batch = gpu_lib.pose_batch(D, pixel, 8, shift_radius=2)
    Z = torch.empty(5, D, D, device="cuda")
    batch.load(dev(Y), ctf_arg(v), filtered=Z)
    out = batch.search(bank, want_scores=True)
    props = dev(inputs.haar_rotations(rng, 5).astype(np.float32))
    r1 = bank.refine(dev(Y), ctf=ctf_arg(v), proposal=props, n_dir=3, n_psi_c=3, shift_radius=2,
                     want_scores=True)
    r2 = batch.refine(bank, proposal=props, n_dir=3, n_psi_c=3, want_scores=True)
    torch.cuda.synchronize()
    assert torch.equal(out["scores"], ref["scores"])
    assert torch.equal(out["rot_idx"], ref["rot_idx"])
    # the winning rotation matrices come from the bank's table
    Gd = dev(G)
    assert torch.equal(out["rot"], Gd[out["rot_idx"].long()])
    assert torch.equal(r2["rot"], Gd[r2["rot_idx"].long()])
    assert torch.equal(r1["scores"], r2["scores"]) and torch.equal(r1["rot_idx"], r2["rot_idx"])
    # the batch's filtered images and cs_ctf_filter are H Y (Eq. 14) vs the oracle
    from oracle import ctf as o_ctf
    HY = o_ctf.apply_ctf(Y.astype(np.float64), o_ctf.ctf_grid_for(v))
    assert max(normwise(host(Z)[b], HY[b]) for b in range(5)) <= 1e-5
    F = gpu_lib.ctf_filter(dev(Y), ctf_arg(v), pixel)
    assert max(normwise(host(F)[b], HY[b]) for b in range(5)) <= 1e-5
    bank.close()
    batch.close()


@pytest.mark.parametrize("use_ctf", [True, False])
def test_one_pass_preparation_d128_matches_oracle(gpu_lib, use_ctf):
    """At D = 128 a batch is prepared in one pass per particle (2-D FFT, CTF
    and inverse in LDS): the filtered images, and through the scores the
    energy weights, ||Y||^2 and the padded -2 Z rows, against the oracle."""
    announce(f"one-pass particle preparation at D=128 (ctf={use_ctf})")
    rng = np.random.default_rng(905 + int(use_ctf))
    g = inputs.mixture_anisotropic(rng, 60, 10.0)
    D, pixel = 128, 1.5
    G = o_pose.grid(1, 4).astype(np.float32)
    P = 3
    v, Y = _particles(g, P, D, pixel, rng, shift_px=[[0, 0], [1, -1], [-1, 0]],
                      q_cut=model.Q_FAITHFUL)
    ctf = ctf_arg(v) if use_ctf else None
    bank = gpu_lib.pose_bank(**mixture_args(g), rot=dev(G), n_psi=4, D=D, pixel=pixel)
    batch = gpu_lib.pose_batch(D, pixel, P, shift_radius=1)
    Z = torch.empty(P, D, D, device="cuda")
    batch.load(dev(Y), ctf, filtered=Z)
    out = batch.search(bank, want_scores=True)
    torch.cuda.synchronize()
    from oracle import ctf as o_ctf
    HY = (o_ctf.apply_ctf(Y.astype(np.float64), o_ctf.ctf_grid_for(v)) if use_ctf
          else Y.astype(np.float64))
    zerr = max(normwise(host(Z)[b], HY[b]) for b in range(P))
    announce(f"  filtered images: normwise {zerr:.2e}")
    assert zerr <= 1e-5
    scores = host(out["scores"])
    for p in range(P):
        ref = o_pose.scores(g, Y[p], v.subset([p]), _f64(G), 1, q_cut=model.Q_FAITHFUL,
                            use_ctf=use_ctf)
        bound = (_bf16_bound(g, Y[p], v.subset([p]), _f64(G), 1) if use_ctf else
                 None)
        err = np.abs(scores[p] - ref)
        if bound is not None:
            announce(f"  particle {p}: max |err| / bound = {np.max(err / bound):.3f}")
            assert np.all(err <= bound), p
        else:
            announce(f"  particle {p}: normwise {normwise(scores[p], ref):.2e}")
            assert normwise(scores[p], ref) <= TOL, p
        assert float(out["score"][p]) == scores[p].min()
    bank.close()
    batch.close()


@pytest.mark.parametrize("D", [64, 128])
def test_standardized_network_input(gpu_lib, D):
    """The batch's standardised bfloat16 network input (D = 128: mean and
    variance from the spectrum in the one-pass kernel; other D: the
    network's own standardisation of Z) against the network's
    standardisation of the filtered images and the oracle, and inference
    from it against inference from the FP32 filtered images."""
    announce(f"standardised network input from the pose batch, D={D}")
    rng = np.random.default_rng(906 + D)
    g = inputs.mixture_anisotropic(rng, 200, 10.0)
    pixel, P = 1.5, 6
    v, Y = _particles(g, P, D, pixel, rng)
    batch = gpu_lib.pose_batch(D, pixel, P, shift_radius=2)
    Z = torch.empty(P, D, D, device="cuda")
    S = torch.empty(P, D, D, device="cuda", dtype=torch.bfloat16)
    batch.load(dev(Y), ctf_arg(v), filtered=Z, standardized=S)
    net = gpu_lib.network(D, P, 11)
    _, _, raw_z = net.forward(Z)
    X0 = net.tensor(0, False, (P, D, D))
    _, _, raw_s = net.forward_standardized(X0)
    with pytest.raises(binding.CryoSplatError):
        net.tensor(0, False, (P, D, D))
    torch.cuda.synchronize()
    assert torch.equal(raw_s, raw_z)
    s, x0 = S.float().cpu().numpy(), X0.float().cpu().numpy()
    differ = s != x0
    announce(f"  bfloat16 values that differ from the two-pass standardisation: {differ.mean():.2e}")
    if D == 128:
        assert differ.mean() <= 1e-3
        assert np.all(np.abs(s - x0)[differ] <= 2.0 ** -7 * np.abs(x0)[differ] + 1e-6)
    else:
        assert not differ.any()
    from oracle import cnn as o_cnn
    from oracle import ctf as o_ctf
    HY = o_ctf.apply_ctf(Y.astype(np.float64), o_ctf.ctf_grid_for(v))
    ref = o_cnn.round_bf16(o_cnn.standardize(HY)[..., 0])
    bad = s != ref
    assert bad.mean() <= 1e-3
    assert np.all(np.abs(s - ref)[bad] <= 2.0 ** -7 * np.abs(ref)[bad] + 1e-5)
    batch.close()


@pytest.mark.parametrize("D", [64, 128])
def test_graphed_pose_paths_match_eager(gpu_lib, D):
    """Learned path (batch preparation, network, two refinement stages) and
    grid search captured as HIP graphs: every replay, with eager library
    work and synchronisations in between, equals the eager result."""
    from paper_2508_04929_amd import pose
    announce(f"graph-captured pose paths, D={D}")
    rng = np.random.default_rng(907 + D)
    g = inputs.mixture_anisotropic(rng, 150, 10.0)
    pixel, P = 1.5, 40
    v, Y = _particles(g, P, D, pixel, rng)
    G1, G2 = o_pose.grid(1, 8).astype(np.float32), o_pose.grid(2, 8).astype(np.float32)
    b1 = gpu_lib.pose_bank(**mixture_args(g), rot=dev(G1), n_psi=8, D=D, pixel=pixel)
    b2 = gpu_lib.pose_bank(**mixture_args(g), rot=dev(G2), n_psi=8, D=D, pixel=pixel)
    batch = gpu_lib.pose_batch(D, pixel, P, shift_radius=2)
    net = gpu_lib.network(D, P, 3)
    xbuf = torch.empty(P, D, D, device="cuda", dtype=torch.bfloat16)
    imgs, ctf = dev(Y), ctf_arg(v)
    stages = [pose.Stage(b1, 3, 2), pose.Stage(b2, 3, 2)]
    learned = lambda: pose.learned_poses(gpu_lib, net, batch, imgs, ctf, stages, xbuf)
    grid = lambda: pose.grid_poses(batch, b1, imgs, ctf)
    W_e, s_e, W0_e, z_e, f_e = [t.clone() for t in learned()]
    Wg_e, sg_e = [t.clone() for t in grid()]
    gl, gg = pose.Graphed(learned), pose.Graphed(grid)
    for rep in range(3):
        W, s, W0, z, f = gl()
        Wg, sg = gg()
        torch.cuda.synchronize()
        assert torch.equal(W, W_e) and torch.equal(s, s_e) and torch.equal(W0, W0_e), rep
        assert torch.equal(z, z_e) and torch.equal(f, f_e), rep
        assert torch.equal(Wg, Wg_e) and torch.equal(sg, sg_e), rep
        # eager work between replays: a search with another bank, then a sync
        batch.load(imgs, ctf)
        batch.search(b2)
        torch.cuda.synchronize()
    for h in (b1, b2, batch, net):
        h.close()


def test_fit_statistic_matches_oracle(gpu_lib):
    """cs_pose_batch_confidence at the winning pose of a grid search against
    the oracle's fit statistic at that pose; the error bound carries the
    bfloat16 bound of the score and of the template energy over to z."""
    announce("fit statistic of the winning pose vs oracle, D=48")
    rng = np.random.default_rng(915)
    g = inputs.mixture_anisotropic(rng, 300, 12.0)
    D, pixel, P, r = 48, 1.5, 4, 2
    G = o_pose.grid(1, 8).astype(np.float32)
    v, Y = _particles(g, P, D, pixel, rng, shift_px=[[0, 0], [1, -2], [-1, 1], [2, 2]])
    bank = gpu_lib.pose_bank(**mixture_args(g), rot=dev(G), n_psi=8, D=D, pixel=pixel)
    batch = gpu_lib.pose_batch(D, pixel, P, shift_radius=r)
    batch.load(dev(Y), ctf_arg(v))
    out = batch.search(bank)
    z = host(batch.confidence(bank, out))
    z2, sg = batch.confidence(bank, out, want_sigmas=True)
    torch.cuda.synchronize()
    assert np.array_equal(host(z2), z)
    sg = host(sg)
    dxs, dys = o_pose.shift_offsets(r)
    rel = 2 * U_BF16 + U_BF16 ** 2 + D * D * 2.0 ** -24
    for p in range(P):
        k, s = int(out["rot_idx"][p]), int(out["shift_idx"][p])
        vp = v.subset([p])
        ref = o_pose.fit_statistic(g, Y[p], vp, _f64(G[k]), [dxs[s], dys[s]])
        X = model.render_pre_ctf(g.means, g.log_scales, g.quats, g.amps, _f64(G[k])[None],
                                 np.zeros((1, 2)), D, pixel)
        from oracle import ctf as o_ctf
        E = np.sum(o_ctf.apply_ctf(X, o_ctf.ctf_grid_for(vp)[0]) ** 2)
        bound = _bf16_bound(g, Y[p], vp, _f64(G[k])[None], r)[0, s]
        tol = (bound + rel * E * abs(ref)) / E + 1e-6
        announce(f"  particle {p}: z {z[p]:.5f} vs oracle {ref:.5f} (bound {tol:.1e})")
        assert abs(z[p] - ref) <= tol, p
        # shortfall in noise spreads: (1 - z) ||H Q|| D / (2 ||Y||)
        f = np.sqrt(E) * D / (2.0 * np.sqrt(np.sum(_f64(Y[p]) ** 2)))
        s_ref = (1.0 - ref) * f
        assert abs(sg[p] - s_ref) <= tol * f + rel * abs(s_ref) + 1e-6, p
    bank.close()
    batch.close()
