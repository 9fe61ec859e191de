"""Densification: SplitGaussian of Alg. 1 (oracle, FP64).

Test infrastructure: used only to check the GPU library.

Alg. 1 optionally splits every Gaussian after selected epochs
(IsDoubleGaussians), doubling the count; App. C.1 gives no split rule.
The rule here preserves each Gaussian's mass, mean and covariance: with
s the activated scales, k the axis of the largest scale (chosen on the
stored pre-activations, lowest index among equals; the activations are
increasing, so this is the largest s) and u = R(q) e_k its direction,

    children  mu +- (s_k / 2) u,   s_k' = s_k sqrt(3) / 2,   A' = A / 2,

the other scales and the quaternion unchanged.  Per pair: total amplitude
A, amplitude-weighted mean mu, and second moment s_k'^2 + s_k^2 / 4 = s_k^2
along u, so the pair's covariance is the parent's.  Layout: child i of the
+ side at index i, of the - side at N + i.  The Adam moments of both
children are the parent's (the caller's optimiser state continues).
"""
from __future__ import annotations

import numpy as np

from . import model

SHRINK = np.sqrt(3.0) / 2.0


def _act_inverse(y, act):
    y = np.asarray(y, dtype=np.float64)
    if act in ("exp",):
        return np.log(y)
    if act == "softplus":
        return np.log(np.expm1(y))
    return y  # identity amplitudes


def split(means, log_scales, quats, amps, scale_act="exp", amp_act="identity"):
    """Children (means [2N,3], log_scales [2N,3], quats [2N,4], amps [2N]),
    FP64, and the split axis per parent."""
    ls32 = np.asarray(log_scales, dtype=np.float32)
    k = np.argmax(ls32, axis=1)                     # first index among equal maxima
    s = model.scales_from(np.asarray(log_scales, dtype=np.float64), scale_act)
    R = model.rotation_from_quaternion(np.asarray(quats, dtype=np.float64))
    n = s.shape[0]
    sk = s[np.arange(n), k]
    u = R[np.arange(n), :, k]                      # column k of R
    mu = np.asarray(means, dtype=np.float64)
    d = 0.5 * sk[:, None] * u
    new_ls = np.asarray(log_scales, dtype=np.float64).copy()
    new_ls[np.arange(n), k] = _act_inverse(SHRINK * sk, scale_act)
    A = model.amps_from(np.asarray(amps, dtype=np.float64), amp_act)
    new_a = _act_inverse(0.5 * A, amp_act)
    q = np.asarray(quats, dtype=np.float64)
    return (np.concatenate([mu + d, mu - d]), np.concatenate([new_ls, new_ls]),
            np.concatenate([q, q]), np.concatenate([new_a, new_a]), k)


def split_flat(theta, n, scale_act="exp", amp_act="identity"):
    """The same on the flat layout means | log_scales | quats | amps."""
    t = np.asarray(theta, dtype=np.float64)
    m, ls, q, a, _ = split(t[:3 * n].reshape(n, 3), np.asarray(theta)[3 * n:6 * n].reshape(n, 3),
                           t[6 * n:10 * n].reshape(n, 4), t[10 * n:], scale_act, amp_act)
    return np.concatenate([m.ravel(), ls.ravel(), q.ravel(), a])


def duplicate_moments(mom, n):
    """Adam moments of the children: each parent's, on both sides."""
    t = np.asarray(mom, dtype=np.float64)
    parts = (t[:3 * n].reshape(n, 3), t[3 * n:6 * n].reshape(n, 3),
             t[6 * n:10 * n].reshape(n, 4), t[10 * n:])
    return np.concatenate([np.concatenate([p, p]).ravel() for p in parts])
