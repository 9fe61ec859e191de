"""Contrast transfer function and its Fourier-space application (oracle, FP64).

Test infrastructure: used only to check the GPU library.

The paper applies the rasterised CTF in Fourier space after the splat
(App. A.2, Eq. 14) but never writes the CTF itself.  The reading used here
is the standard weak-phase CTF with amplitude contrast ``w``:

    chi(s)  = pi lam df(alpha) s^2 - pi/2 Cs lam^3 s^4 - phi
    df(a)   = (df_u + df_v)/2 + (df_u - df_v)/2 cos 2(a - a_ast)
    CTF(s)  = -(sqrt(1 - w^2) sin chi + w cos chi) exp(-B s^2 / 4)

with lam the relativistic electron wavelength.  Lengths are in Angstrom
(Cs in mm is converted).  The DFT grid is numpy's unshifted grid: index k
has frequency k/(D p) for k < D/2 and (k - D)/(D p) otherwise; rows carry
the y-flip of Eq. 13, so the row frequency is the negative of that value.
The convolution is circular and unpadded (Eq. 14 applies F and F^-1 to the
D x D image as it is).
"""
from __future__ import annotations

import numpy as np

# CODATA 2018 exact / recommended values.
PLANCK = 6.62607015e-34
ELECTRON_MASS = 9.1093837015e-31
ELEMENTARY_CHARGE = 1.602176634e-19
LIGHT_SPEED = 299792458.0


def electron_wavelength(voltage_kv: float) -> float:
    """Relativistic de Broglie wavelength of the beam electrons, in Angstrom."""
    V = voltage_kv * 1e3
    eV = ELEMENTARY_CHARGE * V
    p = np.sqrt(2.0 * ELECTRON_MASS * eV * (1.0 + eV / (2.0 * ELECTRON_MASS * LIGHT_SPEED ** 2)))
    return PLANCK / p * 1e10


def ctf_polar(s, alpha, defocus_u, defocus_v, astig, phase, voltage_kv,
              cs_mm, amp_contrast, bfactor=0.0):
    """CTF at spatial frequency magnitude s (1/A) and azimuth alpha (rad)."""
    lam = electron_wavelength(voltage_kv)
    cs = cs_mm * 1e7
    df = 0.5 * (defocus_u + defocus_v) + 0.5 * (defocus_u - defocus_v) * np.cos(2.0 * (alpha - astig))
    chi = np.pi * lam * df * s ** 2 - 0.5 * np.pi * cs * lam ** 3 * s ** 4 - phase
    w = amp_contrast
    return -(np.sqrt(1.0 - w * w) * np.sin(chi) + w * np.cos(chi)) * np.exp(-0.25 * bfactor * s ** 2)


def frequency_axes(D, pixel):
    """Frequencies (1/A) of DFT columns (s_x) and rows (s_y, y-flipped)."""
    f = np.fft.fftfreq(D, d=pixel)
    return f, -f


def ctf_grid(D, pixel, defocus_u, defocus_v, astig, phase, voltage_kv,
             cs_mm, amp_contrast, bfactor=0.0):
    """The rasterised CTF H^ [B,D,D] on the unshifted DFT grid (Eq. 14).

    For even D the Nyquist row and column are their own mirror images on
    the grid, so an astigmatic CTF sampled there is not exactly even.  The
    grid value there is the mean of the CTF at s and at s with its Nyquist
    component negated, which makes H^ exactly even and X exactly real (a
    no-op without astigmatism).
    """
    sx, sy = frequency_axes(D, pixel)
    col = lambda a: np.asarray(a, dtype=np.float64).reshape(-1, 1, 1)

    def at(SX, SY):
        s = np.sqrt(SX ** 2 + SY ** 2)
        alpha = np.arctan2(SY, SX)
        return ctf_polar(s, alpha, col(defocus_u), col(defocus_v), col(astig),
                         col(phase), voltage_kv, cs_mm, amp_contrast, bfactor)

    SX = sx[None, None, :]
    SY = sy[None, :, None]
    H = at(SX, SY)
    if D % 2 == 0:
        fx = np.where(np.arange(D) == D // 2, -1.0, 1.0)[None, None, :]
        fy = np.where(np.arange(D) == D // 2, -1.0, 1.0)[None, :, None]
        H = 0.5 * (H + at(SX * fx, SY * fy))
    return H


def ctf_grid_for(views):
    """ctf_grid from a ``Views`` record of the input generator (on the Angstrom
    pixel ``pixel_a`` when the geometry is in other units)."""
    pixel = views.pixel_a if getattr(views, "pixel_a", 0.0) > 0 else views.pixel
    return ctf_grid(views.D, pixel, views.defocus_u, views.defocus_v,
                    views.astig, views.phase, views.voltage_kv, views.cs_mm,
                    views.amp_contrast, views.bfactor)


def apply_ctf(Q, H):
    """Eq. 14: X = F^-1(H^ . F(Q)) per image (real part; H^ is real and even)."""
    return np.real(np.fft.ifft2(H * np.fft.fft2(Q, axes=(-2, -1)), axes=(-2, -1)))
