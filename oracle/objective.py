"""Squared-error loss, its analytic gradient and finite differences (oracle).

Test infrastructure: used only to check the GPU library.

Loss (Sec. 3.3.5): L = scale * sum_b ||X_b - Y_b||^2 with scale = 1 for a
sum and 1/(B D^2) for a mean (the paper calls it MSE but writes the squared
norm; both reductions are offered).

Gradient (App. A.2, Eq. 15-21), per image and Gaussian, summed over pixels
r in the image with G_Q = dL/dQ:

    dL/dA              = sum G_Q  G~(r)                                 (Eq. 17)
    dL/dmu~            = sum G_Q  A G~(r) S~^-1 (r - mu~)               (Eq. 18)
    dL/dmu             = P^T dL/dmu~   (the adjoint of mu~ = P mu + t)
    dL/d(S~^-1)        = sum G_Q  1/2 A G~(r) (S~ - d d^T)              (Eq. 20)
    dL/dS~             = -S~^-1 dL/d(S~^-1) S~^-1
    dL/dSigma          = P^T dL/dS~ P  (the 3-D embedding of Eq. 21 pulled
                                        back through Sigma' = W Sigma W^T)

then through Sigma = R diag(s)^2 R^T to s and the quaternion and through the
activations to the stored parameters.

The same per-image terms give the gradient w.r.t. the views themselves
(the joint pose optimisation the paper leaves to future work, Sec. 5):
with P the first two rows of the view rotation W, mu~ = P mu + t and
S~ = P Sigma P^T,

    dL/dt = sum_n dL/dmu~_n,    dL/dP = sum_n dL/dmu~_n mu_n^T + 2 dL/dS~_n P Sigma_n,

and the third row of W does not enter the image.  Eq. 18 prints W where the adjoint of
the viewing transform is W^T; the transpose is used (checked against finite
differences).
"""
from __future__ import annotations

import numpy as np

from . import model, ctf as ctf_mod


def loss_from_images(X, Y, reduction="sum"):
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    scale = 1.0 if reduction == "sum" else 1.0 / X.size
    per = scale * ((X - Y) ** 2).reshape(X.shape[0], -1).sum(axis=1)
    return per, scale


def forward(g, v, Y=None, *, H=None, q_cut=None, reduction="sum",
            scale_act="exp", amp_act="identity", use_ctf=True):
    """Q, X and (when Y is given) per-image losses for mixture g, views v."""
    Q = model.render_pre_ctf(g.means, g.log_scales, g.quats, g.amps, v.rot,
                             v.shift, v.D, v.pixel, q_cut, scale_act, amp_act)
    if use_ctf:
        if H is None:
            H = ctf_mod.ctf_grid_for(v)
        X = ctf_mod.apply_ctf(Q, H)
    else:
        X = Q
    out = {"Q": Q, "X": X, "H": H}
    if Y is not None:
        per, scale = loss_from_images(X, Y, reduction)
        out["loss_per_image"] = per
        out["loss"] = float(per.sum())
        out["scale"] = scale
    return out


def _rotation_jacobian(qhat):
    """dR/dq for R(q) written for unit q (as in model.rotation_from_quaternion).

    Returns J [N,4,3,3] with J[:,k] = dR/dq_k, differentiating the
    expression of R in the components of q directly.
    """
    w, x, y, z = (qhat[:, i] for i in range(4))
    J = np.zeros((qhat.shape[0], 4, 3, 3))
    # R00 = w2+x2-y2-z2, R01 = 2(xy-wz), R02 = 2(xz+wy)
    # R10 = 2(xy+wz), R11 = w2-x2+y2-z2, R12 = 2(yz-wx)
    # R20 = 2(xz-wy), R21 = 2(yz+wx), R22 = w2-x2-y2+z2
    J[:, 0] = 2 * np.stack([np.stack([w, -z, y], -1), np.stack([z, w, -x], -1), np.stack([-y, x, w], -1)], -2)
    J[:, 1] = 2 * np.stack([np.stack([x, y, z], -1), np.stack([y, -x, -w], -1), np.stack([z, w, -x], -1)], -2)
    J[:, 2] = 2 * np.stack([np.stack([-y, x, w], -1), np.stack([x, y, z], -1), np.stack([-w, z, -y], -1)], -2)
    J[:, 3] = 2 * np.stack([np.stack([-z, -w, x], -1), np.stack([w, -z, y], -1), np.stack([x, y, z], -1)], -2)
    return J


def backward_from_image_grad(g, v, GQ, *, q_cut=None, scale_act="exp",
                             amp_act="identity"):
    """Gradients of sum(GQ * Q) w.r.t. the stored Gaussian parameters.

    GQ [B,D,D] is dL/dQ.  Returns a dict with means, log_scales, quats,
    amps (FP64) and the world-frame intermediates dSigma [N,3,3], dA [N].
    """
    N = g.n
    cov = model.covariance(g.log_scales, g.quats, scale_act)
    A = model.amps_from(g.amps, amp_act)
    mu2, cov2 = model.project(g.means, cov, v.rot, v.shift)
    W = np.asarray(v.rot, dtype=np.float64)
    GQ = np.asarray(GQ, dtype=np.float64)
    D, p = v.D, v.pixel

    d_mu = np.zeros((N, 3))
    d_sigma = np.zeros((N, 3, 3))
    d_A = np.zeros(N)
    B = W.shape[0]
    d_rot = np.zeros((B, 3, 3))
    d_shift = np.zeros((B, 2))
    means = np.asarray(g.means, dtype=np.float64)
    for b in range(W.shape[0]):
        P = W[b, :2, :]
        S2 = cov2[b]
        det = S2[:, 0, 0] * S2[:, 1, 1] - S2[:, 0, 1] * S2[:, 1, 0]
        inv = np.stack([np.stack([S2[:, 1, 1], -S2[:, 0, 1]], -1),
                        np.stack([-S2[:, 1, 0], S2[:, 0, 0]], -1)], -2) / det[:, None, None]
        norm = 1.0 / (2.0 * np.pi * np.sqrt(det))
        g_img = GQ[b]
        d_mu2 = np.zeros((N, 2))
        d_inv = np.zeros((N, 2, 2))
        for idx, ii, jj, keep, (dx, dy), q in model.footprints(mu2[b], S2, D, p, q_cut):
            G = norm[idx][:, None, None] * np.exp(-0.5 * q)        # G~(r)
            gq = np.where(keep, g_img[np.minimum(ii, D - 1), np.minimum(jj, D - 1)], 0.0)
            t = gq * G                                              # G_Q G~
            d_A[idx] += t.sum(axis=(1, 2))                          # Eq. 17
            At = A[idx][:, None, None] * t                          # G_Q A G~
            s_x = (At * dx).sum(axis=(1, 2))
            s_y = (At * dy).sum(axis=(1, 2))
            iv = inv[idx]
            d_mu2[idx, 0] += iv[:, 0, 0] * s_x + iv[:, 0, 1] * s_y  # Eq. 18
            d_mu2[idx, 1] += iv[:, 1, 0] * s_x + iv[:, 1, 1] * s_y
            s0 = At.sum(axis=(1, 2))
            sxx = (At * dx * dx).sum(axis=(1, 2))
            sxy = (At * dx * dy).sum(axis=(1, 2))
            syy = (At * dy * dy).sum(axis=(1, 2))
            S = S2[idx]
            d_inv[idx, 0, 0] += 0.5 * (S[:, 0, 0] * s0 - sxx)       # Eq. 20
            d_inv[idx, 0, 1] += 0.5 * (S[:, 0, 1] * s0 - sxy)
            d_inv[idx, 1, 0] += 0.5 * (S[:, 1, 0] * s0 - sxy)
            d_inv[idx, 1, 1] += 0.5 * (S[:, 1, 1] * s0 - syy)
        d_S2 = -inv @ d_inv @ inv                                   # dL/dS~
        d_mu += d_mu2 @ P                                           # P^T dmu~
        d_sigma += np.einsum("ai,nab,bj->nij", P, d_S2, P)         # P^T dS~ P
        d_shift[b] = d_mu2.sum(axis=0)                              # pose: t
        d_rot[b, :2] = (np.einsum("na,nj->aj", d_mu2, means)        # pose: P
                        + 2.0 * np.einsum("nab,bk,nkj->aj", d_S2, P, cov))

    # Sigma = R diag(s^2) R^T  ->  s and R (Eq. 5), then q and activations.
    s = model.scales_from(g.log_scales, scale_act)
    q = np.asarray(g.quats, dtype=np.float64)
    qn = np.linalg.norm(q, axis=1)
    qhat = q / qn[:, None]
    R = model.rotation_from_quaternion(qhat)
    RtGR = np.einsum("nai,nab,nbj->nij", R, d_sigma, R)
    d_s = 2.0 * s * np.stack([RtGR[:, k, k] for k in range(3)], axis=1)
    d_R = 2.0 * d_sigma @ R * (s ** 2)[:, None, :]
    J = _rotation_jacobian(qhat)
    d_qhat = np.einsum("nkab,nab->nk", J, d_R)
    d_q = (d_qhat - qhat * (qhat * d_qhat).sum(1, keepdims=True)) / qn[:, None]
    l = np.asarray(g.log_scales, dtype=np.float64)
    d_l = d_s * (s if scale_act == "exp" else model.sigmoid(l))
    a = np.asarray(g.amps, dtype=np.float64)
    d_a = d_A * (1.0 if amp_act == "identity" else model.sigmoid(a))
    return {"means": d_mu, "log_scales": d_l, "quats": d_q, "amps": d_a,
            "rot": d_rot, "shift": d_shift, "d_sigma": d_sigma, "d_A": d_A}


def loss_and_grad(g, v, Y, *, q_cut=None, reduction="sum", scale_act="exp",
                  amp_act="identity", use_ctf=True):
    """Loss and gradient of the full forward model (Sec. 3.3.5, App. A.2)."""
    H = ctf_mod.ctf_grid_for(v) if use_ctf else None
    f = forward(g, v, Y, H=H, q_cut=q_cut, reduction=reduction,
                scale_act=scale_act, amp_act=amp_act, use_ctf=use_ctf)
    GX = 2.0 * f["scale"] * (f["X"] - np.asarray(Y, dtype=np.float64))
    GQ = ctf_mod.apply_ctf(GX, H) if use_ctf else GX
    grads = backward_from_image_grad(g, v, GQ, q_cut=q_cut, scale_act=scale_act,
                                     amp_act=amp_act)
    f.update(GX=GX, GQ=GQ, grads=grads)
    return f


def finite_difference_view(g, v, Y, field, entries, *, h=1e-6, **kw):
    """Central differences of the loss for entries of the views' "rot"
    [B][3][3] (taken entry-wise, not kept orthonormal) or "shift" [B][2]."""
    import dataclasses
    base = np.asarray(getattr(v, field), dtype=np.float64).copy()
    out = []
    for e in entries:
        vals = []
        for sgn in (+1.0, -1.0):
            a = base.copy()
            a[e] += sgn * h
            vals.append(forward(g, dataclasses.replace(v, **{field: a}), Y, **kw)["loss"])
        out.append((vals[0] - vals[1]) / (2.0 * h))
    return np.array(out)


def finite_difference(g, v, Y, field, entries, *, h_rel=1e-6, **kw):
    """Central differences of the loss for selected entries of one field.

    ``entries`` is a list of index tuples into ``getattr(g, field)``.  The
    parameters are perturbed in FP64 copies of the mixture.
    """
    import dataclasses
    base = {f: np.asarray(getattr(g, f), dtype=np.float64).copy()
            for f in ("means", "log_scales", "quats", "amps")}
    out = []
    for e in entries:
        x0 = base[field][e]
        h = h_rel * max(1.0, abs(x0))
        vals = []
        for sgn in (+1.0, -1.0):
            arrs = {k: a.copy() for k, a in base.items()}
            arrs[field][e] = x0 + sgn * h
            gg = dataclasses.replace(g, **arrs)
            vals.append(forward(gg, v, Y, **kw)["loss"])
        out.append((vals[0] - vals[1]) / (2.0 * h))
    return np.array(out)
