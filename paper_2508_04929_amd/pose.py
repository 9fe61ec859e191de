"""Learned pose proposal: data, training and evaluation driven through the library.

Every numerical step runs in libcryosplat: the splatter renders the
training and test particles (with CTF), the library adds the noise, the
network trains with the library's BF16-MFMA forward/backward kernels and
Adam, and poses are scored by the library's grid search and refinement.
This module only sequences those calls, slices batches and times them.

Pipeline of the learned path for a batch of particles:
  1. network forward -> rotation proposal W0 (6-D -> Gram-Schmidt)
  2. refinement stages, each scoring the candidates of one pose bank around
     the current estimate (nearest bank directions x in-plane angles x
     (2r+1)^2 shifts) with the renderer's squared-error score; the best
     candidate seeds the next stage.
  3. fit statistics of the final pose: z = 2 a - 1 (a the least-squares
     amplitude of the winning template in the particle) and its shortfall
     from a perfect fit in units of its noise spread; particles whose
     statistic falls past a threshold go back to the exhaustive grid search.
The exhaustive grid search over the coarse bank is the fallback and the
judge of angular error.  The threshold is calibrated on held-out
validation particles: the smallest fallback fraction whose mean angular
error comes within a margin of the grid search's on the same particles.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import binding, inputs


@dataclasses.dataclass
class PoseSet:
    """Particle poses and CTF parameters resident on the device."""
    rot: torch.Tensor        # [n][3][3] world -> view
    shift: torch.Tensor      # [n][2] Angstrom
    shift_px: torch.Tensor   # [n][2] pixels (network target)
    defocus: torch.Tensor    # [n] Angstrom
    zeros: torch.Tensor      # [n] (astigmatism angle, phase shift)
    D: int
    pixel: float

    @staticmethod
    def from_views(v: inputs.Views, device="cuda") -> "PoseSet":
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        return PoseSet(rot=t(v.rot), shift=t(v.shift), shift_px=t(v.shift / v.pixel),
                       defocus=t(v.defocus_u), zeros=t(np.zeros(len(v.rot))), D=v.D,
                       pixel=v.pixel)

    def __len__(self):
        return self.rot.shape[0]

    def ctf(self, a: int, b: int) -> binding.Ctf:
        return binding.Ctf(defocus_u=self.defocus[a:b], defocus_v=self.defocus[a:b],
                           astig=self.zeros[a:b], phase=self.zeros[a:b])


def mixture_on_device(g: inputs.Mixture, device="cuda"):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
    return dict(means=t(g.means), log_scales=t(g.log_scales), quats=t(g.quats), amps=t(g.amps))


def render_particles(lib, gd, ps: PoseSet, a: int, b: int, snr_db: float, seed: int,
                     out: Optional[torch.Tensor] = None, noise_offset: int = 0):
    """Noisy CTF-modulated particle images a..b-1 (noise counter a + noise_offset)."""
    imgs = lib.render(**gd, rot=ps.rot[a:b], shift=ps.shift[a:b], D=ps.D, pixel=ps.pixel,
                      ctf=ps.ctf(a, b), out=out)
    lib.add_noise(imgs, snr_db, seed, offset=a + noise_offset)
    return imgs


def train(lib, net: binding.Network, gd, ps: PoseSet, *, epochs: int, batch: int, lr: float,
          gamma: float = 0.7, lam: float = 0.1, snr_db: float = -20.0, seed: int = 1,
          matched_filter: bool = True, log=None) -> List[Tuple[int, float]]:
    """Train on ps (re-rendered with fresh noise every epoch); returns (step, loss) samples.

    With matched_filter the network sees Z = H Y, each particle filtered by
    its own CTF (the same Z the pose scores correlate with)."""
    n = len(ps)
    buf = torch.empty(batch, ps.D, ps.D, device=ps.rot.device)
    loss = torch.empty(1, device=ps.rot.device)
    hist, step = [], 0
    for ep in range(epochs):
        lr_ep = lr * gamma ** ep
        for a in range(0, n - batch + 1, batch):
            b = a + batch
            render_particles(lib, gd, ps, a, b, snr_db, seed, out=buf, noise_offset=ep * n)
            if matched_filter:
                lib.ctf_filter(buf, ps.ctf(a, b), ps.pixel, out=buf)
            net.train_step(buf, ps.rot[a:b], ps.shift_px[a:b], lam=lam, lr=lr_ep, loss=loss)
            step += 1
            if step % 50 == 0:
                hist.append((step, float(loss.item())))
                if log:
                    log(f"epoch {ep} step {step} loss {hist[-1][1]:.4f}")
    return hist


def angular_error_deg(R_est: torch.Tensor, R_true: torch.Tensor) -> np.ndarray:
    """Rotation angle between estimated and true world-to-view rotations."""
    tr = torch.einsum("bji,bji->b", R_est.double(), R_true.double())
    return torch.rad2deg(torch.arccos(torch.clamp((tr - 1) / 2, -1, 1))).cpu().numpy()


@dataclasses.dataclass
class Stage:
    bank: binding.PoseBank
    n_dir: int
    n_psi_c: int


def learned_poses(lib, net: binding.Network, batch: binding.PoseBatch, images, ctf: binding.Ctf,
                  stages: Sequence[Stage], xbuf: torch.Tensor,
                  matched_filter: bool = True):
    """Prepare the particles once, network proposal (on Z = H Y with
    matched_filter: the batch writes the standardised bfloat16 network input
    into xbuf [P][D][D] as it prepares the particles), then the refinement
    stages on the prepared batch.
    Returns (rot [P][3][3], shift index [P], proposal [P][3][3])."""
    if matched_filter:
        batch.load(images, ctf, standardized=xbuf)
        W0, _, _ = net.forward_standardized(xbuf)
    else:
        batch.load(images, ctf)
        W0, _, _ = net.forward(images)
    W, out = W0, None
    for st in stages:
        out = batch.refine(st.bank, proposal=W, n_dir=st.n_dir, n_psi_c=st.n_psi_c)
        W = out["rot"]
    z, sig = (batch.confidence(stages[-1].bank, out, want_sigmas=True) if stages
              else (None, None))
    return W, (out["shift_idx"] if out is not None else None), W0, z, sig


def fallback_search(batch: binding.PoseBatch, bank: binding.PoseBank, images, ps: "PoseSet",
                    W: torch.Tensor, z: torch.Tensor, tau: float, chunk: int) -> int:
    """Exhaustive search (in batches of `chunk`) of the particles whose fit
    statistic is below tau (or undefined); their rows of W are replaced by
    the grid-search rotations.  Returns the number of particles searched."""
    idx = torch.nonzero(~(z >= tau)).flatten()
    n = int(idx.numel())
    for a in range(0, n, chunk):
        sel = idx[a:a + chunk]
        ctf = binding.Ctf(defocus_u=ps.defocus.index_select(0, sel),
                          defocus_v=ps.defocus.index_select(0, sel),
                          astig=ps.zeros.index_select(0, sel), phase=ps.zeros.index_select(0, sel))
        batch.load(images.index_select(0, sel).contiguous(), ctf)
        W.index_copy_(0, sel, batch.search(bank)["rot"])
    return n


def calibrate_threshold(z: np.ndarray, err_learned: np.ndarray, err_grid: np.ndarray,
                        margin_deg: float = 0.5) -> Tuple[float, float]:
    """Smallest fallback set (the lowest-z particles) whose mean angular
    error, with those particles taking their grid-search error, is within
    margin_deg of the grid search's mean.  Returns (threshold, fraction):
    particles with z < threshold fall back."""
    z = np.where(np.isfinite(z), z, -np.inf)
    order = np.argsort(z, kind="stable")
    n = len(z)
    target = err_grid.mean() + margin_deg
    total = err_learned.sum()
    for k in range(n + 1):
        if total / n <= target:
            if k == 0:
                return float(z[order[0]]) if n else 0.0, 0.0
            hi = z[order[k]] if k < n else np.inf
            lo = z[order[k - 1]]
            return float(0.5 * (lo + hi)) if np.isfinite(hi) else float("inf"), k / n
        if k < n:
            j = order[k]
            total += err_grid[j] - err_learned[j]
    return float("inf"), 1.0


def grid_poses(batch: binding.PoseBatch, bank: binding.PoseBank, images, ctf: binding.Ctf):
    """Exhaustive search of one bank: (rot [P][3][3], shift index [P])."""
    batch.load(images, ctf)
    out = batch.search(bank)
    return out["rot"], out["shift_idx"]


class Graphed:
    """A fixed sequence of library calls captured once as a HIP graph and
    replayed: one launch instead of one per kernel.  The sequence runs once
    eagerly first, so every library buffer it needs already exists (the
    library must not allocate during capture); its outputs are the tensors
    returned by the captured call, rewritten by every replay."""

    def __init__(self, fn):
        fn()
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.out = fn()
        torch.cuda.synchronize()

    def __call__(self):
        self.graph.replay()
        return self.out


def timed(fn, reps: int = 3):
    """(result, median seconds) of a GPU call sequence."""
    res, ts = None, []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return res, float(np.median(ts))


def literal_grid_search(lib, gd, image, ctf_one: binding.Ctf, grid_rot: torch.Tensor, D: int,
                        pixel: float, shift_radius: int = 2, chunk: int = 4608):
    """Reference: render every (rotation, shift) candidate with the particle's
    CTF and score it by the library's squared-error loss (no shared templates).
    Returns (best rotation index, best shift index, best score)."""
    K = grid_rot.shape[0]
    side = 2 * shift_radius + 1
    best = (None, None, float("inf"))
    obs = image.expand(chunk, D, D).contiguous()
    rep = lambda t: t.expand(chunk).contiguous()
    ctf = binding.Ctf(defocus_u=rep(ctf_one.defocus_u), defocus_v=rep(ctf_one.defocus_v),
                      astig=rep(ctf_one.astig), phase=rep(ctf_one.phase))
    shift = torch.empty(chunk, 2, device=image.device)
    for s in range(side * side):
        dx, dy = s % side - shift_radius, s // side - shift_radius
        shift[:, 0], shift[:, 1] = dx * pixel, dy * pixel
        for k0 in range(0, K, chunk):
            kc = min(chunk, K - k0)
            c = ctf if kc == chunk else binding.Ctf(
                defocus_u=ctf.defocus_u[:kc], defocus_v=ctf.defocus_v[:kc],
                astig=ctf.astig[:kc], phase=ctf.phase[:kc])
            loss, _, _ = lib.loss_and_grad(**gd, rot=grid_rot[k0:k0 + kc].contiguous(),
                                           shift=shift[:kc].contiguous(), D=D, pixel=pixel,
                                           observed=obs[:kc], ctf=c, want_grads=False)
            v, i = torch.min(loss[:kc], dim=0)
            if float(v) < best[2]:
                best = (k0 + int(i), s, float(v))
    return best


def run_c5(lib, *, n_train=200000, n_test=8192, epochs=12, batch=256, lr=1e-3, gamma=0.85,
           lam=0.1, snr_db=-20.0, seed=5, coarse=(4, 24), fine=(8, 48), shift_radius=2,
           stages=((0, 6, 2), (1, 4, 2)), matched_filter=True, chunks=(2048, 4096, 8192),
           literal_particles=2, stage_sweep=(), use_graphs=True, n_val=8192,
           fallback_margin_deg=1.0, log=print):
    """The learned-pose experiment: returns angular errors and throughputs.

    stages: (bank 0 = coarse / 1 = fine, n_dir, n_psi_c) per refinement stage;
    stage_sweep: other stage lists evaluated with the same trained network
    (error and throughput of each, under "stage_sweep").  With use_graphs
    both timed paths are replayed HIP graphs (the eager times are reported
    too).
    Both paths are timed from particle images in device memory to poses,
    particle preparation (CTF filtering, shifted copies) included, in
    batches of each size in ``chunks``; each path's throughput is the one
    at its fastest batch size (the grid search slows with larger batches,
    the learned path speeds up), and every batch size gives the same poses."""
    dev = torch.device("cuda")
    g, tr, te = inputs.c5(seed, n_train, n_test)
    gd = mixture_on_device(g)
    ps_tr, ps_te = PoseSet.from_views(tr), PoseSet.from_views(te)
    D, pixel = ps_te.D, ps_te.pixel
    res = {"n_train": n_train, "n_test": n_test, "D": D, "pixel": pixel, "N": int(len(g.amps)),
           "snr_db": snr_db, "shift_radius": shift_radius, "matched_filter": matched_filter}
    rots = [torch.from_numpy(lib.pose_grid(*coarse)).to(dev),
            torch.from_numpy(lib.pose_grid(*fine)).to(dev)]
    t0 = time.perf_counter()
    banks = [lib.pose_bank(**gd, rot=rots[0], n_psi=coarse[1], D=D, pixel=pixel),
             lib.pose_bank(**gd, rot=rots[1], n_psi=fine[1], D=D, pixel=pixel)]
    torch.cuda.synchronize()
    res["bank_build_s"] = time.perf_counter() - t0
    res["bank_sizes"] = [int(r.shape[0]) for r in rots]
    imgs = render_particles(lib, gd, ps_te, 0, n_test, snr_db, seed + 1000)
    chunks = sorted({min(c, n_test) for c in chunks})
    chunk = chunks[0]
    pbs = {c: lib.pose_batch(D, pixel, c, shift_radius) for c in chunks}
    xbuf = torch.empty(max(chunks), D, D, device=dev, dtype=torch.bfloat16)

    def grid_all(c=chunk):
        return torch.cat([grid_poses(pbs[c], banks[0], imgs[a:min(n_test, a + c)],
                                     ps_te.ctf(a, min(n_test, a + c)))[0]
                          for a in range(0, n_test, c)])

    def per_chunk(make, ref, same):
        """{chunk: (seconds, eager seconds)}; every batch size must give `ref`."""
        out = {}
        for c in chunks:
            fn = make(c)
            r, te_ = timed(fn)
            tg = te_
            if use_graphs:
                r2, tg = timed(Graphed(fn))
                if not same(r2, r):
                    raise RuntimeError("graph replay differs from the eager run")
            if not same(r, ref):
                raise RuntimeError(f"batches of {c} give other poses than batches of {chunk}")
            out[c] = (tg, te_)
        return out

    W_gs = grid_all()
    t_by = per_chunk(lambda c: (lambda: grid_all(c)), W_gs, torch.equal)
    c_gs = min(t_by, key=lambda c: t_by[c][0])
    t_gs, t_gs_eager = t_by[c_gs]
    err_gs = angular_error_deg(W_gs, ps_te.rot)
    res["grid_search"] = {"median_deg": float(np.median(err_gs)), "mean_deg": float(err_gs.mean()),
                          "images_per_s": n_test / t_gs, "seconds": t_gs, "batch": c_gs,
                          "images_per_s_eager": n_test / t_gs_eager,
                          "images_per_s_by_batch": {str(c): n_test / v[0] for c, v in t_by.items()}}
    log(f"grid search: median {np.median(err_gs):.2f} deg, {n_test / t_gs:.0f} img/s "
        f"(batches of {c_gs})")
    st = [Stage(banks[b], nd, npc) for b, nd, npc in stages]
    net = lib.network(D, max_batch=max(batch, max(chunks)), seed=seed)

    def learned(st=st, c=chunk, images=imgs, ps=ps_te, n=n_test):
        Ws, W0s, zs, ss = [], [], [], []
        for a in range(0, n, c):
            b = min(n, a + c)
            W, _, W0, z, sg = learned_poses(lib, net, pbs[c], images[a:b], ps.ctf(a, b), st,
                                            xbuf[:b - a], matched_filter)
            Ws.append(W)
            W0s.append(W0)
            zs.append(z)
            ss.append(sg)
        return torch.cat(Ws), torch.cat(W0s), torch.cat(zs), torch.cat(ss)

    W_u, W0_u, _, _ = learned()
    err_u = angular_error_deg(W_u, ps_te.rot)
    err_pu = angular_error_deg(W0_u, ps_te.rot)
    res["untrained"] = {"median_deg": float(np.median(err_u)),
                        "proposal_median_deg": float(np.median(err_pu))}
    log(f"untrained: proposal {np.median(err_pu):.1f} deg, refined {np.median(err_u):.1f} deg")
    t0 = time.perf_counter()
    hist = train(lib, net, gd, ps_tr, epochs=epochs, batch=batch, lr=lr, gamma=gamma, lam=lam,
                 snr_db=snr_db, seed=seed, matched_filter=matched_filter, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    res["training"] = {"epochs": epochs, "batch": batch,
                       "steps": len(range(0, n_train - batch + 1, batch)) * epochs,
                       "seconds": t_train, "images_per_s": epochs * n_train / t_train,
                       "loss_first": hist[0][1] if hist else None,
                       "loss_last": hist[-1][1] if hist else None}
    W_t, W0_t, _, _ = learned()
    same2 = lambda a, b: torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    t_by = per_chunk(lambda c: (lambda: learned(st, c)), (W_t, W0_t), same2)
    c_l = min(t_by, key=lambda c: t_by[c][0])
    t_l, t_l_eager = t_by[c_l]
    err_t = angular_error_deg(W_t, ps_te.rot)
    err_pt = angular_error_deg(W0_t, ps_te.rot)
    res["learned"] = {"median_deg": float(np.median(err_t)), "mean_deg": float(err_t.mean()),
                      "proposal_median_deg": float(np.median(err_pt)),
                      "images_per_s": n_test / t_l, "seconds": t_l, "batch": c_l,
                      "images_per_s_eager": n_test / t_l_eager,
                      "images_per_s_by_batch": {str(c): n_test / v[0] for c, v in t_by.items()},
                      "stages": [list(s) for s in stages]}
    res["speedup_same_batch"] = {str(c): res["learned"]["images_per_s_by_batch"][str(c)]
                                 / res["grid_search"]["images_per_s_by_batch"][str(c)]
                                 for c in chunks}
    log(f"learned: proposal {np.median(err_pt):.1f} deg, refined {np.median(err_t):.2f} deg, "
        f"{n_test / t_l:.0f} img/s (batches of {c_l})")
    res["speedup_vs_grid_search"] = t_gs / t_l
    res["reaches_grid_search_error"] = bool(np.median(err_t) <= np.median(err_gs))

    # fallback: threshold on the fit statistic, calibrated on validation
    # particles (same distributions, separate stream) against the grid search
    ps_va = PoseSet.from_views(inputs.c5_validation(seed, n_val, D))
    imgs_va = render_particles(lib, gd, ps_va, 0, n_val, snr_db, seed + 2000)
    W_va_g = torch.cat([grid_poses(pbs[chunk], banks[0], imgs_va[a:min(n_val, a + chunk)],
                                   ps_va.ctf(a, min(n_val, a + chunk)))[0]
                        for a in range(0, n_val, chunk)])
    W_va_l, _, z_va, s_va = learned(st, chunk, imgs_va, ps_va, n_val)
    e_va_g = angular_error_deg(W_va_g, ps_va.rot)
    e_va_l = angular_error_deg(W_va_l, ps_va.rot)
    # both statistics as "low = poor fit"; the one that needs the smaller
    # validation fallback at the margin is used, the other reported
    stats_va = {"z": z_va.cpu().numpy(), "neg_sigmas": -s_va.cpu().numpy()}
    tradeoff = {name: {str(m): calibrate_threshold(v, e_va_l, e_va_g, m)[1]
                       for m in (0.5, 1.0, 2.0, 4.0)} for name, v in stats_va.items()}
    cal = {name: calibrate_threshold(v, e_va_l, e_va_g, fallback_margin_deg)
           for name, v in stats_va.items()}
    stat = min(cal, key=lambda k: cal[k][1])
    tau, frac_va = cal[stat]
    log(f"fallback on {stat} < {tau:.4f}: {100 * frac_va:.1f}% of validation particles "
        f"(validation mean error learned {e_va_l.mean():.2f}, grid {e_va_g.mean():.2f} deg; "
        f"fractions by margin {tradeoff})")
    pfb = {c: lib.pose_batch(D, pixel, c, shift_radius) for c in chunks}

    def with_fallback(c, graphed):
        def fn():
            W, W0, z, sg = graphed() if graphed is not None else learned(st, c)
            W = W.clone()
            n_fb = fallback_search(pfb[c], banks[0], imgs, ps_te, W, z if stat == "z" else -sg,
                                   tau, c)
            return W, n_fb
        return fn

    fb_by, W_f, n_f = {}, None, 0
    for c in chunks:
        fn = with_fallback(c, Graphed(lambda c=c: learned(st, c)) if use_graphs else None)
        (W_c, n_c), t_c = timed(fn)
        if W_f is None:
            W_f, n_f = W_c, n_c
        elif not torch.equal(W_c, W_f):
            raise RuntimeError(f"batches of {c} give other fallback poses than batches of {chunk}")
        fb_by[c] = t_c
    err_f = angular_error_deg(W_f, ps_te.rot)
    c_f = min(fb_by, key=fb_by.get)
    res["learned_fallback"] = {
        "statistic": stat, "threshold": tau, "margin_deg": fallback_margin_deg,
        "validation_fallback_fraction_by_margin": tradeoff,
        "fallback_fraction_validation": frac_va, "fallback_fraction": n_f / n_test,
        "validation_mean_deg": {"learned": float(e_va_l.mean()), "grid": float(e_va_g.mean())},
        "median_deg": float(np.median(err_f)), "mean_deg": float(err_f.mean()),
        "images_per_s": n_test / fb_by[c_f], "batch": c_f,
        "images_per_s_by_batch": {str(c): n_test / t for c, t in fb_by.items()},
        "speedup_same_batch": {str(c): (n_test / fb_by[c])
                               / res["grid_search"]["images_per_s_by_batch"][str(c)]
                               for c in chunks}}
    log(f"learned + fallback: {100 * n_f / n_test:.1f}% searched, median {np.median(err_f):.2f} deg, "
        f"mean {err_f.mean():.2f} deg (grid {err_gs.mean():.2f}), {n_test / fb_by[c_f]:.0f} img/s")
    for pb in pfb.values():
        pb.close()
    sweep = []
    for stv in stage_sweep:
        sv = [Stage(banks[b], nd, npc) for b, nd, npc in stv]
        fn_v = (lambda: learned(sv, c_l))
        (W_v, _, _, _), t_v = timed(Graphed(fn_v) if use_graphs else fn_v)
        e_v = angular_error_deg(W_v, ps_te.rot)
        sweep.append({"stages": [list(x) for x in stv], "median_deg": float(np.median(e_v)),
                      "images_per_s": n_test / t_v, "speedup_vs_grid_search": t_gs / t_v})
        log(f"stages {stv}: refined {np.median(e_v):.2f} deg, {n_test / t_v:.0f} img/s, "
            f"{t_gs / t_v:.1f}x grid search")
    if sweep:
        res["stage_sweep"] = sweep
    if literal_particles > 0:
        t0 = time.perf_counter()
        for p in range(literal_particles):
            literal_grid_search(lib, gd, imgs[p], ps_te.ctf(p, p + 1), rots[0], D, pixel,
                                shift_radius)
        torch.cuda.synchronize()
        t_lit = (time.perf_counter() - t0) / literal_particles
        res["literal_grid_search_images_per_s"] = 1.0 / t_lit
        res["speedup_vs_literal_grid_search"] = (n_test / t_l) * t_lit
    for b in banks:
        b.close()
    for pb in pbs.values():
        pb.close()
    net.close()
    return res
