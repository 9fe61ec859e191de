"""Voxelisation of the mixture and Fourier shell correlation (oracle).

Test infrastructure: used only to check the GPU library.

The reconstruction is a Gaussian mixture; its 3-D density is read out on a
voxel grid (the overview of Sec. 3: the GMM "can be voxelized to obtain the
final 3D volume"), and two volumes are compared by the Fourier shell
correlation of Eq. 10 with the 0.143 threshold (Sec. 4, evaluation metrics).

Voxel grid: voxel (iz, iy, ix) of a D^3 grid with spacing p sits at
(x, y, z) = ((ix - c0) p, (iy - c0) p, (iz - c0) p), c0 = D // 2 (the
centre convention of the image raster, Eq. 13, without its row flip).  The
value is the mixture's density there,

    V(x) = sum_n A_n (2 pi)^(-3/2) det(Sigma_n)^(-1/2) exp(-q_n(x) / 2),
    q_n(x) = (x - mu_n)^T Sigma_n^-1 (x - mu_n),

whose integral along z is the projected image of the identity pose (Eq. 8),
optionally truncated at q_n <= q_cut like the renderer.

FSC: V^ = DFT of each volume (numpy's rfftn), shells k = round(|k|) with
integer frequency indices (kx, ky, kz) in [-D/2, D/2), shells 0 .. D/2;
per shell sum Re(V^_a conj V^_b), sum |V^_a|^2, sum |V^_b|^2 over the full
spectrum (the half spectrum with weight 2 off the kx = 0 and Nyquist
planes), FSC = num / sqrt(den_a den_b).
"""
from __future__ import annotations

import numpy as np

from . import model


def voxel_axis(D, pixel):
    return (np.arange(D) - D // 2) * float(pixel)


def density_at(g, pts, q_cut=None, scale_act="exp", amp_act="identity", chunk=64):
    """Mixture density at points [P][3] (x, y, z), Angstrom (FP64)."""
    cov = model.covariance(g.log_scales, g.quats, scale_act)
    A = model.amps_from(g.amps, amp_act)
    mu = np.asarray(g.means, dtype=np.float64)
    inv = np.linalg.inv(cov)
    w = A * (2.0 * np.pi) ** -1.5 / np.sqrt(np.linalg.det(cov))
    pts = np.asarray(pts, dtype=np.float64)
    out = np.zeros(len(pts))
    for n0 in range(0, len(mu), chunk):
        d = pts[None, :, :] - mu[n0:n0 + chunk, None, :]
        q = np.einsum("npi,nij,npj->np", d, inv[n0:n0 + chunk], d)
        e = np.exp(-0.5 * q)
        if q_cut is not None:
            e = np.where(q <= q_cut, e, 0.0)
        out += (w[n0:n0 + chunk, None] * e).sum(axis=0)
    return out


def voxel_points(D, pixel, idx=None):
    """Positions (x, y, z) of voxels [iz][iy][ix] (all, or the listed
    (iz, iy, ix) index triples)."""
    ax = voxel_axis(D, pixel)
    if idx is None:
        Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
        return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    idx = np.asarray(idx)
    return np.stack([ax[idx[:, 2]], ax[idx[:, 1]], ax[idx[:, 0]]], axis=1)


def voxelize(g, D, pixel, q_cut=None, scale_act="exp", amp_act="identity", chunk=64):
    """Mixture density on the D^3 grid [iz][iy][ix] (FP64)."""
    return density_at(g, voxel_points(D, pixel), q_cut, scale_act, amp_act,
                      chunk).reshape(D, D, D)


def shell_index(D):
    """Shell of every half-spectrum voxel [kz][ky][kx] (numpy rfftn layout)
    and its weight in the full-spectrum sum (1 on the kx = 0 and Nyquist
    planes, 2 elsewhere)."""
    f = np.fft.fftfreq(D) * D
    fr = np.fft.rfftfreq(D) * D
    kz, ky, kx = np.meshgrid(f, f, fr, indexing="ij")
    s = np.rint(np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)).astype(np.int64)
    w = np.where((kx == 0) | (kx == D // 2), 1.0, 2.0)
    return s, w


def fsc_sums(va, vb):
    """Per-shell sums (num, den_a, den_b) for shells 0 .. D/2 (Eq. 10)."""
    va = np.asarray(va, dtype=np.float64)
    vb = np.asarray(vb, dtype=np.float64)
    D = va.shape[0]
    Fa, Fb = np.fft.rfftn(va), np.fft.rfftn(vb)
    s, w = shell_index(D)
    keep = s <= D // 2
    n_sh = D // 2 + 1
    num = np.bincount(s[keep], (w * (Fa * np.conj(Fb)).real)[keep], minlength=n_sh)
    da = np.bincount(s[keep], (w * np.abs(Fa) ** 2)[keep], minlength=n_sh)
    db = np.bincount(s[keep], (w * np.abs(Fb) ** 2)[keep], minlength=n_sh)
    return num, da, db


def fsc(va, vb):
    """FSC per shell 0 .. D/2 (0 where a shell has no energy)."""
    num, da, db = fsc_sums(va, vb)
    den = np.sqrt(da * db)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def resolution(curve, D, pixel, threshold=0.143):
    """Resolution in Angstrom at the first shell k >= 1 where the curve drops
    below the threshold (D p / k; the last shell if it never does)."""
    curve = np.asarray(curve)
    for k in range(1, len(curve)):
        if curve[k] < threshold:
            return D * float(pixel) / k
    return D * float(pixel) / (len(curve) - 1)
