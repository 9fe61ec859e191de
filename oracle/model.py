"""Gaussian mixture geometry and the real-space splat (oracle, FP64).

Test infrastructure: a plain statement of the forward model, used only to
check the GPU library.

Conventions (readings of the paper, listed in the design notes):

* A quaternion is scalar-first (w, x, y, z) and is normalised before use
  (Sec. 3.3.1).
* Scales are ``s = exp(l)`` by default, ``softplus(l)`` when requested; the
  amplitude is used as given, or through softplus when requested (Sec.
  3.3.1 applies softplus to both).
* Covariance ``Sigma = R diag(s)^2 R^T`` (Eq. 5).
* ``W`` maps world to view coordinates.  The projected mean is
  ``P mu + t`` with ``P`` the first two rows of ``W`` and ``t`` an in-plane
  shift in Angstrom; this is the sign the Fourier-space model (Eq. 11)
  fixes through its phase factor.  The projected covariance is
  ``P Sigma P^T`` (Eq. 6, 12).
* The splat keeps the view-dependent normalisation ``1/(2 pi |Sigma~|^1/2)``
  (Eq. 8).
* Pixel (i, j) of a D x D image samples the point
  ``((j - c) p, -(i - c) p)`` with ``c = floor(D/2)``: the origin sits on
  the FFT grid point and rows run against y (Eq. 13).
* Images are point samples at pixel centres, clipped to the D x D grid.
"""
from __future__ import annotations

import numpy as np

#: Truncation that keeps every term above 1e-16 of its Gaussian's peak;
#: the dropped tail is below FP64 resolution ("faithful-truncated" mode).
Q_FAITHFUL = 2.0 * np.log(1e16)


def softplus(x):
    x = np.asarray(x, dtype=np.float64)
    return np.where(x > 30.0, x, np.log1p(np.exp(np.minimum(x, 30.0))))


def sigmoid(x):
    x = np.asarray(x, dtype=np.float64)
    return 1.0 / (1.0 + np.exp(-x))


def scales_from(log_scales, scale_act="exp"):
    """Per-axis standard deviations s from the stored parameters (Sec. 3.3.1)."""
    l = np.asarray(log_scales, dtype=np.float64)
    return np.exp(l) if scale_act == "exp" else softplus(l)


def amps_from(amps, amp_act="identity"):
    a = np.asarray(amps, dtype=np.float64)
    return a if amp_act == "identity" else softplus(a)


def rotation_from_quaternion(quats):
    """Rotation matrices of normalised scalar-first quaternions (Sec. 3.3.1).

    Written as the matrix of the map v -> q v q* for a unit quaternion.
    """
    q = np.asarray(quats, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = w * w + x * x - y * y - z * z
    R[..., 0, 1] = 2.0 * (x * y - w * z)
    R[..., 0, 2] = 2.0 * (x * z + w * y)
    R[..., 1, 0] = 2.0 * (x * y + w * z)
    R[..., 1, 1] = w * w - x * x + y * y - z * z
    R[..., 1, 2] = 2.0 * (y * z - w * x)
    R[..., 2, 0] = 2.0 * (x * z - w * y)
    R[..., 2, 1] = 2.0 * (y * z + w * x)
    R[..., 2, 2] = w * w - x * x - y * y + z * z
    return R


def covariance(log_scales, quats, scale_act="exp"):
    """Eq. 5: Sigma = R S S^T R^T with S = diag(s)."""
    s = scales_from(log_scales, scale_act)
    R = rotation_from_quaternion(quats)
    S = np.zeros(s.shape + (3,))
    S[..., 0, 0], S[..., 1, 1], S[..., 2, 2] = s[..., 0], s[..., 1], s[..., 2]
    RS = R @ S
    return RS @ np.swapaxes(RS, -1, -2)


def project(means, cov, rot, shift=None):
    """Viewing transform and orthogonal projection (Eq. 6, 7, 12).

    Returns the projected means [B,N,2] and covariances [B,N,2,2]: the
    first two rows of W applied to the world-frame mean (plus the in-plane
    shift) and the upper-left 2x2 block of W Sigma W^T.
    """
    mu = np.asarray(means, dtype=np.float64)
    W = np.asarray(rot, dtype=np.float64)
    mu_dot = np.einsum("bij,nj->bni", W, mu)
    cov_dot = np.einsum("bij,njk,blk->bnil", W, cov, W)
    mu2 = mu_dot[..., :2].copy()
    if shift is not None:
        mu2 += np.asarray(shift, dtype=np.float64)[:, None, :]
    return mu2, cov_dot[..., :2, :2].copy()


def pixel_axes(D, pixel):
    """Eq. 13: Angstrom coordinates of columns (x) and rows (y, flipped)."""
    c = D // 2
    idx = np.arange(D, dtype=np.float64)
    return (idx - c) * pixel, -(idx - c) * pixel


def splat_value(mu2, cov2, amp, x, y):
    """Eq. 8 times the amplitude: A / (2 pi |S|^1/2) exp(-d^T S^-1 d / 2)."""
    det = cov2[0, 0] * cov2[1, 1] - cov2[0, 1] * cov2[1, 0]
    inv = np.array([[cov2[1, 1], -cov2[0, 1]], [-cov2[1, 0], cov2[0, 0]]]) / det
    dx, dy = x - mu2[0], y - mu2[1]
    q = inv[0, 0] * dx * dx + (inv[0, 1] + inv[1, 0]) * dx * dy + inv[1, 1] * dy * dy
    return amp / (2.0 * np.pi * np.sqrt(det)) * np.exp(-0.5 * q)


def footprints(mu2, cov2, D, pixel, q_cut=None, chunk_elems=1 << 22):
    """Iterate over (Gaussian, pixel) windows of one image.

    With ``q_cut=None`` every Gaussian is evaluated at every pixel (the
    untruncated sum).  Otherwise each Gaussian is evaluated on the pixel
    box that contains its ellipse ``d^T S^-1 d <= q_cut`` and terms with a
    larger Mahalanobis distance are dropped.

    Yields ``(idx, ii, jj, keep, d, q)`` per chunk of Gaussians where ``ii``
    [n,H,1] and ``jj`` [n,1,W] are pixel indices, ``keep`` masks pixels that
    exist and pass the cut, ``d`` = (dx, dy) in Angstrom and ``q`` is the
    squared Mahalanobis distance.
    """
    mu2 = np.asarray(mu2, dtype=np.float64)
    cov2 = np.asarray(cov2, dtype=np.float64)
    n = mu2.shape[0]
    c = D // 2
    u = mu2[:, 0] / pixel + c          # column coordinate of the centre
    v = c - mu2[:, 1] / pixel          # row coordinate of the centre
    if q_cut is None:
        j0 = np.zeros(n, dtype=np.int64)
        i0 = np.zeros(n, dtype=np.int64)
        j1 = np.full(n, D - 1, dtype=np.int64)
        i1 = np.full(n, D - 1, dtype=np.int64)
    else:
        hx = np.sqrt(q_cut * cov2[:, 0, 0]) / pixel
        hy = np.sqrt(q_cut * cov2[:, 1, 1]) / pixel
        j0 = np.maximum(np.ceil(u - hx), 0).astype(np.int64)
        j1 = np.minimum(np.floor(u + hx), D - 1).astype(np.int64)
        i0 = np.maximum(np.ceil(v - hy), 0).astype(np.int64)
        i1 = np.minimum(np.floor(v + hy), D - 1).astype(np.int64)
    vis = np.nonzero((j0 <= j1) & (i0 <= i1))[0]
    if vis.size == 0:
        return
    area = (j1[vis] - j0[vis] + 1) * (i1[vis] - i0[vis] + 1)
    order = vis[np.argsort(area, kind="stable")]
    det = cov2[:, 0, 0] * cov2[:, 1, 1] - cov2[:, 0, 1] * cov2[:, 1, 0]
    start = 0
    while start < order.size:
        # Grow the chunk while the padded window stays within budget.
        W = int(j1[order[start]] - j0[order[start]] + 1)
        H = int(i1[order[start]] - i0[order[start]] + 1)
        stop = start + 1
        while stop < order.size:
            k = order[stop]
            W2 = max(W, int(j1[k] - j0[k] + 1))
            H2 = max(H, int(i1[k] - i0[k] + 1))
            if (stop - start + 1) * W2 * H2 > chunk_elems:
                break
            W, H, stop = W2, H2, stop + 1
        idx = order[start:stop]
        start = stop
        jj = (j0[idx][:, None] + np.arange(W))[:, None, :]
        ii = (i0[idx][:, None] + np.arange(H))[:, :, None]
        exists = (jj <= j1[idx][:, None, None]) & (ii <= i1[idx][:, None, None])
        x = (jj - c) * pixel
        y = -(ii - c) * pixel
        dx = x - mu2[idx, 0][:, None, None]
        dy = y - mu2[idx, 1][:, None, None]
        s = cov2[idx]
        d_ = det[idx][:, None, None]
        ixx = s[:, 1, 1][:, None, None] / d_
        iyy = s[:, 0, 0][:, None, None] / d_
        ixy = -s[:, 0, 1][:, None, None] / d_
        q = ixx * dx * dx + 2.0 * ixy * dx * dy + iyy * dy * dy
        keep = exists if q_cut is None else (exists & (q <= q_cut))
        yield idx, ii, jj, keep, (dx, dy), q


def splat_image(mu2, cov2, amps, D, pixel, q_cut=None):
    """Eq. 9 without the PSF: Q[i,j] = sum_n A_n G~_n(r_ij) for one image."""
    amps = np.asarray(amps, dtype=np.float64)
    cov2 = np.asarray(cov2, dtype=np.float64)
    det = cov2[:, 0, 0] * cov2[:, 1, 1] - cov2[:, 0, 1] * cov2[:, 1, 0]
    weight = amps / (2.0 * np.pi * np.sqrt(det))
    img = np.zeros(D * D)
    for idx, ii, jj, keep, _d, q in footprints(mu2, cov2, D, pixel, q_cut):
        val = weight[idx][:, None, None] * np.exp(-0.5 * q)
        flat = np.broadcast_to(ii * D + jj, val.shape)
        img += np.bincount(flat[keep], weights=val[keep], minlength=D * D)
    return img.reshape(D, D)


def render_pre_ctf(means, log_scales, quats, amps, rot, shift, D, pixel,
                   q_cut=None, scale_act="exp", amp_act="identity"):
    """Images Q [B,D,D] before the PSF (Eq. 9, 13, 15)."""
    cov = covariance(log_scales, quats, scale_act)
    A = amps_from(amps, amp_act)
    mu2, cov2 = project(means, cov, rot, shift)
    return np.stack([splat_image(mu2[b], cov2[b], A, D, pixel, q_cut)
                     for b in range(mu2.shape[0])])


def pair_count(means, log_scales, quats, rot, shift, D, pixel, q_cut,
               scale_act="exp"):
    """Number of (Gaussian, pixel) pairs with Mahalanobis^2 <= q_cut per image.

    This is the algorithmic work of the splat: the exact footprint of every
    Gaussian inside the image.
    """
    cov = covariance(log_scales, quats, scale_act)
    mu2, cov2 = project(means, cov, rot, shift)
    out = np.zeros(mu2.shape[0], dtype=np.int64)
    for b in range(mu2.shape[0]):
        for _idx, _ii, _jj, keep, _d, _q in footprints(mu2[b], cov2[b], D, pixel, q_cut):
            out[b] += int(keep.sum())
    return out
