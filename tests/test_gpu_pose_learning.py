"""The trained pose network against the same network untrained (GPU).

A small version of the learned-pose experiment: the network trains for a
few hundred steps on particles the splatter renders (with CTF and noise),
then proposes poses for held-out particles.  Trained proposals must be far
closer to the true poses than untrained ones, and refinement started from
them must beat refinement started from the untrained proposals.
"""
import numpy as np
import pytest
import torch

from paper_2508_04929_amd import inputs
from paper_2508_04929_amd import pose

from gpu_util import announce

pytestmark = pytest.mark.gpu


def test_training_gains_over_untrained_network(gpu_lib):
    announce("pose network training gain, D=64")
    rg, rtr, rte = inputs.streams(77, 3)
    g = inputs.mixture_domains(rg, 3000, n_domains=5, radius=20.0, extent=(4.0, 9.0))
    D, pixel, snr = 64, 2.0, 0.0
    tr = inputs.pose_views(rtr, 16384, D, pixel, shift_px_max=1.0)
    te = inputs.pose_views(rte, 256, D, pixel, shift_px_max=1.0)
    gd = pose.mixture_on_device(g)
    ps_tr, ps_te = pose.PoseSet.from_views(tr), pose.PoseSet.from_views(te)
    imgs = pose.render_particles(gpu_lib, gd, ps_te, 0, 256, snr, seed=99)
    untrained = gpu_lib.network(D, max_batch=256, seed=3)
    net = gpu_lib.network(D, max_batch=256, seed=3)
    pose.train(gpu_lib, net, gd, ps_tr, epochs=3, batch=128, lr=1e-3, gamma=0.7, lam=0.1,
               snr_db=snr, seed=7)
    rot = torch.from_numpy(gpu_lib.pose_grid(2, 12)).cuda()
    bank = gpu_lib.pose_bank(**gd, rot=rot, n_psi=12, D=D, pixel=pixel)
    batch = gpu_lib.pose_batch(D, pixel, 256, shift_radius=1)
    xbuf = torch.empty(256, D, D, device="cuda", dtype=torch.bfloat16)
    st = [pose.Stage(bank, 4, 3)]
    W_t, _, P_t, _, _ = pose.learned_poses(gpu_lib, net, batch, imgs, ps_te.ctf(0, 256), st, xbuf)
    W_u, _, P_u, _, _ = pose.learned_poses(gpu_lib, untrained, batch, imgs, ps_te.ctf(0, 256), st,
                                     xbuf)
    e_u = np.median(pose.angular_error_deg(P_u, ps_te.rot))
    e_t = np.median(pose.angular_error_deg(P_t, ps_te.rot))
    announce(f"median proposal error untrained {e_u:.1f} deg, trained {e_t:.1f} deg")
    assert e_t < 0.5 * e_u
    r_t = np.median(pose.angular_error_deg(W_t, ps_te.rot))
    r_u = np.median(pose.angular_error_deg(W_u, ps_te.rot))
    announce(f"median refined error untrained {r_u:.1f} deg, trained {r_t:.1f} deg")
    assert r_t < 0.5 * r_u
    bank.close()
    batch.close()
    net.close()
    untrained.close()
