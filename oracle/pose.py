"""FP64 reference of pose scoring (test infrastructure only).

Nothing in the library imports this module; tests, the smoke check and the
CPU-baseline leg of the benchmark use it.

The paper fixes the image model (Sec. 3.2, Eq. 1: projection of the
mixture, in-plane shift, CTF applied in Fourier space per App. A.2, Eq. 14)
and its squared-error loss (Sec. 3.3.5); it assumes poses are known.  A
pose search scores candidate poses with exactly that model, so the oracle
score of rotation W and shift t for image Y is the plain definition
    score = sum_ij (X(W, t)_ij - Y_ij)^2,   X = CTF-modulated render,
with every candidate rendered from scratch (no shared templates, no
circular-shift shortcut, no Parseval identity).

Pose grids are HEALPix viewing directions (Gorski et al. 2005, ring
scheme, enumerated ring by ring with phi ascending from 0) times uniform
in-plane angles; W = Rz(psi) Ry(-theta) Rz(-phi).
"""
from __future__ import annotations

import numpy as np

from . import ctf as ctf_mod
from . import model


# ---------------------------------------------------------------- grids

def healpix_directions(nside):
    """(theta, phi) of the 12 nside^2 HEALPix pixel centres, ring order."""
    N = int(nside)
    th, ph = [], []
    for i in range(1, 4 * N):
        if i < N:                      # north polar cap
            z = 1.0 - i * i / (3.0 * N * N)
            phis = (np.arange(4 * i) + 0.5) * (np.pi / 2) / i
        elif i <= 3 * N:               # equatorial belt
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * N)
            s = (i - N + 1) % 2
            phis = (np.arange(4 * N) + 0.5 * s) * np.pi / (2 * N)
        else:                          # south polar cap
            k = 4 * N - i
            z = -(1.0 - k * k / (3.0 * N * N))
            phis = (np.arange(4 * k) + 0.5) * (np.pi / 2) / k
        th.extend([np.arccos(z)] * len(phis))
        ph.extend(phis)
    return np.array(th), np.array(ph)


def _rz(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _ry(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def view_rotation(theta, phi, psi):
    """World-to-view W whose third row is the direction (theta, phi)."""
    return _rz(psi) @ _ry(-theta) @ _rz(-phi)


def grid(nside, n_psi):
    """Rotations [12 nside^2 n_psi][3][3], index = direction * n_psi + psi index."""
    th, ph = healpix_directions(nside)
    out = np.empty((len(th) * n_psi, 3, 3))
    for d in range(len(th)):
        for m in range(n_psi):
            out[d * n_psi + m] = view_rotation(th[d], ph[d], 2.0 * np.pi * m / n_psi)
    return out


def angular_distance_deg(R1, R2):
    """Rotation angle of R1^T R2 in degrees (batched)."""
    R1 = np.asarray(R1, dtype=np.float64)
    R2 = np.asarray(R2, dtype=np.float64)
    tr = np.einsum("...ji,...ji->...", R1, R2)
    return np.degrees(np.arccos(np.clip((tr - 1.0) / 2.0, -1.0, 1.0)))


# ---------------------------------------------------------------- shifts

def shift_offsets(r):
    """(dx, dy) in pixels for shift index s = (dy + r)(2r + 1) + (dx + r)."""
    side = 2 * r + 1
    s = np.arange(side * side)
    return s % side - r, s // side - r


# ---------------------------------------------------------------- scores

def scores(g, Y, particle, rotations, shift_radius, q_cut=None, use_ctf=True):
    """score[k][s] of one particle image Y [D][D] for every rotation k and shift s.

    ``particle`` is a one-image Views record of the input generator (its CTF
    parameters, D and pixel size).  Every (rotation, shift) is rendered with
    model.render_pre_ctf, modulated by the particle's CTF on the DFT grid and
    compared with Y."""
    rotations = np.asarray(rotations, dtype=np.float64)
    dx, dy = shift_offsets(shift_radius)
    K, S = len(rotations), len(dx)
    rot = np.repeat(rotations, S, axis=0)
    shift = np.tile(np.stack([dx, dy], axis=1) * float(particle.pixel), (K, 1))
    H = ctf_mod.ctf_grid_for(particle)[0] if use_ctf else None
    Y = np.asarray(Y, dtype=np.float64)
    out = np.empty(K * S)
    chunk = 256
    for c0 in range(0, K * S, chunk):
        sl = slice(c0, min(K * S, c0 + chunk))
        X = model.render_pre_ctf(g.means, g.log_scales, g.quats, g.amps, rot[sl], shift[sl],
                                 particle.D, particle.pixel, q_cut)
        if use_ctf:
            X = ctf_mod.apply_ctf(X, H)
        out[sl] = np.sum((X - Y[None]) ** 2, axis=(1, 2))
    return out.reshape(K, S)


def scores_at(g, Y, particle, rotations, shifts_px, q_cut=None, use_ctf=True):
    """Scores of one particle at listed (rotation [n][3][3], shift [n][2] pixels) poses."""
    rotations = np.asarray(rotations, dtype=np.float64)
    shift = np.asarray(shifts_px, dtype=np.float64) * float(particle.pixel)
    X = model.render_pre_ctf(g.means, g.log_scales, g.quats, g.amps, rotations, shift,
                             particle.D, particle.pixel, q_cut)
    if use_ctf:
        X = ctf_mod.apply_ctf(X, ctf_mod.ctf_grid_for(particle)[0])
    return np.sum((X - np.asarray(Y, dtype=np.float64)[None]) ** 2, axis=(1, 2))


def fit_statistic(g, Y, particle, rotation, shift_px, q_cut=None, use_ctf=True):
    """Fit of one particle Y to the template at one pose (rotation [3][3],
    shift [2] pixels), from the squared error of Sec. 3.3.5:
        z = (||Y||^2 - score) / ||X||^2,  X = the CTF-modulated render,
    which expands to 2 <X, Y> / ||X||^2 - 1 = 2 a - 1 with a the
    least-squares amplitude of X in Y."""
    rot = np.asarray(rotation, dtype=np.float64)[None]
    shift = np.asarray(shift_px, dtype=np.float64)[None] * float(particle.pixel)
    X = model.render_pre_ctf(g.means, g.log_scales, g.quats, g.amps, rot, shift, particle.D,
                             particle.pixel, q_cut)
    if use_ctf:
        X = ctf_mod.apply_ctf(X, ctf_mod.ctf_grid_for(particle)[0])
    Y = np.asarray(Y, dtype=np.float64)
    score = np.sum((X[0] - Y) ** 2)
    return (np.sum(Y ** 2) - score) / np.sum(X[0] ** 2)


# ---------------------------------------------------------------- refinement

def refine_candidates(proposal, bank_rot, n_psi, n_dir, n_psi_c):
    """Candidate bank indices [L] around one proposal rotation W (FP64).

    Directions: the n_dir bank directions with the largest dot product with
    W's viewing direction (third row), ties to the smaller index.  For each,
    psi* maximises trace(W^T Rz(psi) A_d), A_d = bank rotation (d, psi = 0);
    the n_psi_c consecutive grid angles around psi* are taken."""
    W = np.asarray(proposal, dtype=np.float64)
    A = np.asarray(bank_rot, dtype=np.float64)[::n_psi]      # psi = 0 of every direction
    dots = A[:, 2, :] @ W[2]
    order = np.lexsort((np.arange(len(dots)), -dots))[:n_dir]
    step = 2.0 * np.pi / n_psi
    out = []
    for d in order:
        # brute force over psi on a fine circle would also do; the closed form
        # maximiser of c (M00 + M11) + s (M01 - M10) is used and checked in tests
        M = A[d] @ W.T
        psi = np.arctan2(M[0, 1] - M[1, 0], M[0, 0] + M[1, 1])
        base = int(np.floor(psi / step - 0.5 * (n_psi_c - 1) + 0.5))
        out.extend(int(d) * n_psi + ((base + c) % n_psi) for c in range(n_psi_c))
    return np.array(out)
