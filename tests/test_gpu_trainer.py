"""The paper-faithful training loop on the GPU (Alg. 1, Sec. 4.1) against
the FP64 oracle: FourierShift (images within 1e-4 normwise, whole-pixel
shifts as rolls, chunked batches), the initialisation, batch-1 training
steps with Adam (parameters after two epochs, per-step losses), bit
equality of the graph-replayed and eager loops and of the loop with
step-by-step library calls, and a short end-to-end reconstruction from
noisy, translated synthetic particles whose FSC against the ground truth
must improve."""
import numpy as np
import pytest
import torch

from oracle import adam as o_adam, objective, trainer as o_tr, volume as o_vol
from paper_2508_04929_amd import binding, inputs, trainer

from gpu_util import announce, ctf_arg, dev, host, normwise

pytestmark = pytest.mark.gpu

Q_MATCHED = 2.0 * np.log(1e6)


@pytest.mark.parametrize("D,pixel", [(32, 1.0), (48, 2.3), (64, 1.0 / 64)])
def test_fourier_shift_matches_oracle(gpu_lib, D, pixel):
    rng = np.random.default_rng(70 + D)
    Y = rng.standard_normal((5, D, D))
    t = rng.uniform(-4, 4, size=(5, 2)) * pixel
    announce(f"FourierShift D={D} pixel={pixel:.4g}")
    for direction in (1, -1):
        got = host(gpu_lib.fourier_shift(dev(Y), dev(t), pixel, direction=direction))
        ref = o_tr.fourier_shift(Y.astype(np.float32), direction * t.astype(np.float32).astype(np.float64), pixel)
        assert normwise(got, ref) <= 1e-5
    whole = np.array([[3.0, -2.0]] * 5) * pixel
    got = host(gpu_lib.fourier_shift(dev(Y), dev(whole), pixel))
    assert np.abs(got - np.roll(Y, (2, 3), axis=(1, 2))).max() <= 1e-5 * np.abs(Y).max()


def test_fourier_shift_chunks_and_in_place(gpu_lib):
    """More images than one chunk of the staged spectrum (D = 256), in place."""
    rng = np.random.default_rng(73)
    B, D = 1100, 256
    x = torch.randn(B, D, D, device="cuda", generator=torch.Generator(device="cuda").manual_seed(3))
    t = dev(rng.uniform(-3, 3, size=(B, 2)))
    keep = x[[0, 700, 1099]].clone()
    announce("FourierShift of 1100 images at D=256, in place")
    gpu_lib.fourier_shift(x, t, 1.0, out=x)
    torch.cuda.synchronize()
    idx = [0, 700, 1099]
    ref = o_tr.fourier_shift(host(keep), host(t)[idx], 1.0)
    assert normwise(host(x[idx]), ref) <= 1e-5


def test_init_attributes_matches_oracle(gpu_lib):
    z = np.random.default_rng(74).standard_normal((5000, 3)).astype(np.float32)
    got = host(gpu_lib.init_attributes(dev(z)))
    ref = np.concatenate([a.ravel() for a in o_tr.init_attributes(z)])
    np.testing.assert_allclose(got, ref, rtol=2e-7, atol=0)


def _problem(seed, n=20, D=24, M=6):
    rng = np.random.default_rng(seed)
    g = inputs.mixture_anisotropic(rng, n, 0.15)
    g.log_scales = o_tr.softplus_inverse(rng.uniform(0.02, 0.05, size=(n, 3))).astype(np.float32)
    g.amps = o_tr.softplus_inverse(rng.uniform(0.01, 0.05, size=n)).astype(np.float32)
    v = inputs.views(rng, M, D, 1.0 / D)
    v.pixel_a = 3.0
    v.defocus_u = v.defocus_v = (rng.uniform(1.0, 2.0, M) * 1e4).astype(np.float32)
    Y = (objective.forward(g, v, scale_act="softplus", amp_act="softplus")["X"]
         + 0.3 * rng.standard_normal((M, D, D))).astype(np.float32)
    return rng, g, v, Y


def _one(v, i):
    return inputs.Views(rot=v.rot[i:i + 1], shift=v.shift[i:i + 1], defocus_u=v.defocus_u[i:i + 1],
                        defocus_v=v.defocus_v[i:i + 1], astig=v.astig[i:i + 1],
                        phase=v.phase[i:i + 1], D=v.D, pixel=v.pixel, pixel_a=v.pixel_a)


def _flat(g):
    return np.concatenate([np.asarray(a, dtype=np.float32).ravel()
                           for a in (g.means, g.log_scales, g.quats, g.amps)])


def test_training_steps_match_oracle(gpu_lib):
    """Two epochs (12 batch-1 steps) from the same start and orders: every
    parameter within lr * steps * 1e-3 of the oracle's, except where a
    gradient component is so small that its sign is decided by rounding
    (Adam moves such a parameter by up to lr per step either way)."""
    rng, g, v, Y = _problem(75)
    orders = [rng.permutation(6), rng.permutation(6)]
    lr0, gamma = 1e-3, 0.5
    st = o_tr.State(g.means, g.log_scales, g.quats, g.amps)
    ref_losses = []
    for e, order in enumerate(orders):
        ref_losses.append(o_tr.train(st, lambda i: _one(v, i), Y, order,
                                     lr=o_tr.learning_rate(lr0, gamma, e), q_cut=Q_MATCHED))
    p = dev(_flat(g))
    m, vv = torch.zeros_like(p), torch.zeros_like(p)
    ctf = ctf_arg(v)
    losses = []
    announce("12 batch-1 training steps vs the oracle (N=20, D=24, box units, CTF)")
    for e, order in enumerate(orders):
        loss = torch.empty(6, device="cuda")
        gpu_lib.train_sequential(p, m, vv, dev(Y), dev(v.rot), v.pixel, order, 6 * e,
                                 o_tr.learning_rate(lr0, gamma, e), ctf=ctf,
                                 options=binding.Options(graph=1), loss=loss)
        losses.append(host(loss))
    got = host(p)
    np.testing.assert_allclose(np.concatenate(losses), np.concatenate(ref_losses), rtol=1e-4)
    diff = np.abs(got - st.theta)
    steps = 12
    close = diff <= 1e-3 * lr0 * steps
    announce(f"  max |param - oracle| = {diff.max():.2e}; outside 1e-3 lr steps: {np.sum(~close)} of {diff.size}")
    assert np.all(diff <= 2.0 * lr0 * steps)
    assert np.mean(close) >= 0.98


def _adam_dir(g, m, v, t, b1=0.9, b2=0.999, eps=1e-8):
    """m_hat / (sqrt(v_hat) + eps) of one Adam step from moments (m, v) with
    gradient g (broadcast over a trailing axis of candidate gradients)."""
    mm = b1 * m[..., None] + (1 - b1) * g
    vv = b2 * v[..., None] + (1 - b2) * g * g
    return (mm / (1 - b1 ** t)) / (np.sqrt(vv / (1 - b2 ** t)) + eps)


def test_training_steps_teacher_forced(gpu_lib):
    """Every one of 12 batch-1 steps against one oracle step taken from the
    GPU's own state (parameters and Adam moments read back before the step),
    so errors cannot accumulate and every step is bounded.  The bound per
    parameter follows from the gradient bar: with the GPU gradient within
    1e-3 of the oracle's, normwise per parameter group, each component may
    differ by up to delta = 1e-3 ||g_group||, and Adam then moves it by
    lr (u(g') - u(g)) for some g' in [g - delta, g + delta], u(g) =
    m_hat / (sqrt(v_hat) + eps); the test takes the largest such change over
    that interval (densely sampled, plus the stationary point of u), plus
    FP32 rounding of the parameter.  Where the gradient is far above delta
    this is a small fraction of lr; only components with |g| of order delta
    (Adam's sign decided by rounding) get up to ~2 lr."""
    rng, g, v, Y = _problem(75)
    orders = [rng.permutation(6), rng.permutation(6)]
    lr0, gamma = 1e-3, 0.5
    n = g.n
    groups = [slice(0, 3 * n), slice(3 * n, 6 * n), slice(6 * n, 10 * n), slice(10 * n, 11 * n)]
    p = dev(_flat(g))
    m, vv = torch.zeros_like(p), torch.zeros_like(p)
    Yd, rot = dev(Y), dev(v.rot)
    ctf = ctf_arg(v)
    announce("12 batch-1 training steps, each against an oracle step from the GPU state")
    k, worst = 0, 0.0
    for e, order in enumerate(orders):
        lr = o_tr.learning_rate(lr0, gamma, e)
        for i in order:
            th = host(p).astype(np.float64)
            m0, v0 = host(m).astype(np.float64), host(vv).astype(np.float64)
            gpu_lib.train_sequential(p, m, vv, Yd, rot, v.pixel, np.array([i]), k, lr, ctf=ctf,
                                     options=binding.Options(graph=0))
            got = host(p).astype(np.float64)
            st = o_tr.State(th[:3 * n].reshape(n, 3), th[3 * n:6 * n].reshape(n, 3),
                            th[6 * n:10 * n].reshape(n, 4), th[10 * n:])
            f = objective.loss_and_grad(st.mixture(), _one(v, int(i)), Y[int(i)][None],
                                        q_cut=Q_MATCHED, reduction="sum", scale_act="softplus",
                                        amp_act="softplus", use_ctf=True)
            gr = np.concatenate([np.asarray(f["grads"][c], dtype=np.float64).ravel()
                                 for c in ("means", "log_scales", "quats", "amps")])
            t = k + 1
            ref, _, _ = o_adam.adam_step(th, gr, m0, v0, t, lr=lr)
            delta = np.empty_like(gr)
            for sl in groups:
                delta[sl] = 1e-3 * np.linalg.norm(gr[sl])
            cand = gr[:, None] + delta[:, None] * np.linspace(-1.0, 1.0, 65)[None, :]
            b1, b2 = 0.9, 0.999
            with np.errstate(divide="ignore", invalid="ignore"):
                gs = (1 - b1) * b2 * v0 / (b1 * m0 * (1 - b2))  # stationary point of u
            gs = np.where(np.isfinite(gs) & (np.abs(gs - gr) <= delta), gs, gr)
            cand = np.concatenate([cand, gs[:, None]], axis=1)
            u0 = _adam_dir(gr[:, None], m0, v0, t)[:, 0]
            spread = np.abs(_adam_dir(cand, m0, v0, t) - u0[:, None]).max(axis=1)
            bound = lr * spread * 1.01 + 4 * np.finfo(np.float32).eps * (np.abs(ref) + lr)
            err = np.abs(got - ref)
            assert np.all(err <= bound), (k, int(np.argmax(err - bound)), float(err.max()))
            worst = max(worst, float((err / lr).max()))
            k += 1
    announce(f"  largest step deviation {worst:.2e} lr")


def test_graph_eager_and_stepwise_are_bitwise_equal(gpu_lib):
    rng, g, v, Y = _problem(76, n=40, D=32, M=8)
    order = np.concatenate([rng.permutation(8), rng.permutation(8)])
    ctf = ctf_arg(v)
    outs = []
    for graph in (0, 1):
        p = dev(_flat(g))
        m, vv = torch.zeros_like(p), torch.zeros_like(p)
        gpu_lib.train_sequential(p, m, vv, dev(Y), dev(v.rot), v.pixel, order, 0, 1e-3, ctf=ctf,
                                 options=binding.Options(graph=graph))
        outs.append(p)
    # the same steps through the single-call entry points
    p = dev(_flat(g))
    m, vv = torch.zeros_like(p), torch.zeros_like(p)
    n = g.n
    Yd, rot = dev(Y), dev(v.rot)
    for k, i in enumerate(order):
        c = binding.Ctf(defocus_u=ctf.defocus_u[i:i + 1].contiguous(),
                        defocus_v=ctf.defocus_v[i:i + 1].contiguous(),
                        astig=ctf.astig[i:i + 1].contiguous(), phase=ctf.phase[i:i + 1].contiguous(),
                        voltage_kv=ctf.voltage_kv, cs_mm=ctf.cs_mm, amp_contrast=ctf.amp_contrast,
                        bfactor=ctf.bfactor, pixel_a=ctf.pixel_a)
        _, grads, _ = gpu_lib.loss_and_grad(p[:3 * n].view(n, 3), p[3 * n:6 * n].view(n, 3),
                                            p[6 * n:10 * n].view(n, 4), p[10 * n:],
                                            rot[i:i + 1].contiguous(), None, v.D, v.pixel,
                                            Yd[i:i + 1].contiguous(), ctf=c, reduction="sum",
                                            scale_act="softplus", amp_act="softplus")
        flat = torch.cat([grads[k2].reshape(-1) for k2 in ("means", "log_scales", "quats", "amps")])
        gpu_lib.adam_step(p, flat, m, vv, k + 1, lr=1e-3)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
    assert torch.equal(outs[0], p)


def test_train_sequential_rejects_bad_order(gpu_lib):
    p = torch.zeros(11 * 4, device="cuda")
    with pytest.raises(binding.CryoSplatError):
        gpu_lib.train_sequential(p, p.clone(), p.clone(), torch.zeros(2, 16, 16, device="cuda"),
                                 torch.eye(3, device="cuda").repeat(2, 1, 1), 1 / 16, [0, 2], 0, 1e-3)


def _synthetic_set(seed, n_gt, M, D, p_a, snr_db):
    """Ground-truth domain mixture (Angstrom) moved to box units (L = D p_a,
    total amplitude 1/2), particles at Haar-random poses with CTF, whole-set
    translations up to 2 px, white noise at snr_db."""
    rng = np.random.default_rng(seed)
    L = D * p_a
    gt = inputs.mixture_domains(rng, n_gt, radius=0.2 * L, scale_mu=np.log(3.0))
    amps = np.asarray(gt.amps, np.float64)
    box = inputs.Mixture(means=(np.asarray(gt.means, np.float64) / L).astype(np.float32),
                         log_scales=(np.asarray(gt.log_scales, np.float64) - np.log(L)).astype(np.float32),
                         quats=gt.quats, amps=(0.5 * amps / amps.sum()).astype(np.float32))
    v = inputs.views(rng, M, D, 1.0 / D)
    v.pixel_a = p_a
    v.shift = (rng.uniform(-2, 2, size=(M, 2)) / D).astype(np.float32)
    return rng, box, v


def test_end_to_end_reconstruction_improves_fsc(gpu_lib):
    """2,000 Gaussians trained from the paper's initialisation for 5 epochs
    over 3,000 noisy (0 dB), translated particles (D = 64, 3 A pixels):
    the loss falls and the FSC resolution against the ground truth beats
    the initial mixture's by a wide margin."""
    D, p_a, M = 64, 3.0, 3000
    rng, gt, v = _synthetic_set(77, 2000, M, D, p_a, 0.0)
    lib = gpu_lib
    g = {k: dev(getattr(gt, k)) for k in ("means", "log_scales", "quats", "amps")}
    rot, shift, ctf = dev(v.rot), dev(v.shift), ctf_arg(v)
    clean = lib.render(g["means"], g["log_scales"], g["quats"], g["amps"], rot, shift, D, 1.0 / D,
                       ctf=ctf)
    lib.add_noise(clean, 0.0, seed=5)
    data = trainer.Dataset(images=clean, rot=rot, shift=shift, ctf=ctf)
    z = dev(rng.standard_normal((2000, 3)))
    tr = trainer.Trainer(lib, z)
    V0 = tr.voxelize(D)
    Vgt = lib.voxelize(g["means"], g["log_scales"], g["quats"], g["amps"], D, 1.0 / D)
    res0 = lib.resolution(lib.fsc(V0, Vgt), D, p_a)[0]
    announce("end-to-end: 5 epochs x 3000 particles, N=2000, D=64")
    losses = host(tr.fit(data, epochs=5, lr=1e-3, gamma=0.5, seed=1, record_loss=True))
    res = lib.resolution(lib.fsc(tr.voxelize(D), Vgt), D, p_a)[0]
    first, last = losses[:M].mean(), losses[-M:].mean()
    # the noise floor: the ground truth's own loss on the same particles
    floor, _, _ = lib.loss_and_grad(g["means"], g["log_scales"], g["quats"], g["amps"], rot, shift,
                                    D, 1.0 / D, clean, ctf=ctf, want_grads=False)
    floor = float(floor[-1]) / M
    announce(f"  loss per particle {first:.4g} -> {last:.4g} (ground truth {floor:.4g}); "
             f"FSC resolution {res0:.1f} A -> {res:.1f} A")
    assert np.all(np.isfinite(losses))
    assert last < first and last <= 1.1 * floor
    assert res < 0.5 * res0
