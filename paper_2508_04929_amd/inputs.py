"""Seeded synthetic workloads for the renderer (random draws only).

This module is shared by the tests, the benchmark and the CPU oracle's
callers.  It holds no arithmetic of the rendering method itself: it only
draws the random inputs the method consumes (Gaussian parameters, poses,
CTF parameters, noise) with numpy's PCG64 generator and returns FP32 arrays.
The same FP32 arrays are handed to the GPU path and to the FP64 oracle.

Recipes follow the synthetic stand-ins for the paper's EMPIAR workloads
(Sec. 4.1 uses real particle stacks that are not available):

* ``c1``  N=1,000 isotropic Gaussians in a 40 A cube, 16 images D=64, p=3.0 A.
* ``c2``  N=20,000 anisotropic Gaussians in a ball of radius 60 A,
          256 images D=128, p=1.5 A, shifts N(0, (2 px)^2), SNR -20 dB.
* ``c3``  eight mixtures with uneven N and D in {128, 192, 256}.
* ``c4``  N=200,000 isotropic Gaussians (Sec. 4.1 initialisation scaled to
          A units) in a ball of radius 75 A, 64 images D=256, p=1.1 A.

Noise is white and Gaussian (Eq. 1's epsilon) with variance set from the
requested SNR in dB relative to the clean images' variance.
"""
from __future__ import annotations

import dataclasses
import numpy as np

#: Microscope constants shared by every recipe (300 kV, Cs 2.7 mm, w=0.1).
VOLTAGE_KV = 300.0
CS_MM = 2.7
AMP_CONTRAST = 0.1


@dataclasses.dataclass
class Mixture:
    """Gaussian-mixture parameters, FP32, world frame, Angstrom units."""
    means: np.ndarray       # [N,3]
    log_scales: np.ndarray  # [N,3]  s = exp(log_scales)
    quats: np.ndarray       # [N,4]  (w, x, y, z), not necessarily unit
    amps: np.ndarray        # [N]

    @property
    def n(self) -> int:
        return int(self.means.shape[0])


@dataclasses.dataclass
class Views:
    """Per-image pose and CTF parameters, FP32 arrays of length B."""
    rot: np.ndarray         # [B,3,3] world -> view rotation W (row-major)
    shift: np.ndarray       # [B,2]   in-plane shift t in A
    defocus_u: np.ndarray   # [B] A
    defocus_v: np.ndarray   # [B] A
    astig: np.ndarray       # [B] rad
    phase: np.ndarray       # [B] rad
    D: int
    pixel: float
    voltage_kv: float = VOLTAGE_KV
    cs_mm: float = CS_MM
    amp_contrast: float = AMP_CONTRAST
    bfactor: float = 0.0
    pixel_a: float = 0.0    # A pixel of the CTF grid when `pixel` is in other units (0: pixel)

    @property
    def b(self) -> int:
        return int(self.rot.shape[0])

    def subset(self, idx) -> "Views":
        idx = np.asarray(idx)
        return dataclasses.replace(
            self, rot=self.rot[idx], shift=self.shift[idx],
            defocus_u=self.defocus_u[idx], defocus_v=self.defocus_v[idx],
            astig=self.astig[idx], phase=self.phase[idx])


def streams(seed: int, k: int = 8):
    """Independent PCG64 generators spawned from one seed."""
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(k)]


def haar_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform unit quaternions: normalised 4-D standard normal draws."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def haar_rotations(rng: np.random.Generator, b: int) -> np.ndarray:
    """Haar-uniform rotation matrices by QR of Gaussian matrices.

    The Q factor of a standard-normal matrix with the signs of diag(R)
    absorbed is Haar on O(3); multiplying the det=-1 draws by a fixed
    reflection maps that coset onto SO(3) with Haar measure.
    """
    z = rng.standard_normal((b, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.sign(np.diagonal(r, axis1=1, axis2=2))
    d[d == 0] = 1.0
    q = q * d[:, None, :]
    neg = np.linalg.det(q) < 0
    q[neg, :, 0] *= -1.0
    return q


def uniform_ball(rng: np.random.Generator, n: int, radius: float) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = radius * rng.random(n) ** (1.0 / 3.0)
    return v * r[:, None]


def _f32(x):
    return np.ascontiguousarray(x, dtype=np.float32)


def mixture_anisotropic(rng, n, ball_radius, scale_mu=np.log(1.5), scale_sd=0.3):
    """Anisotropic mixture: means in a ball, log-scales normal, lognormal A."""
    return Mixture(
        means=_f32(uniform_ball(rng, n, ball_radius)),
        log_scales=_f32(scale_mu + scale_sd * rng.standard_normal((n, 3))),
        quats=_f32(haar_quaternions(rng, n)),
        amps=_f32(np.exp(0.5 * rng.standard_normal(n))),
    )


def views(rng, b, D, pixel, defocus_um=(0.8, 2.5), shift_px_sd=0.0):
    rot = haar_rotations(rng, b)
    if shift_px_sd > 0:
        shift = rng.standard_normal((b, 2)) * shift_px_sd * pixel
    else:
        shift = np.zeros((b, 2))
    df = rng.uniform(defocus_um[0], defocus_um[1], size=b) * 1e4
    return Views(rot=_f32(rot), shift=_f32(shift), defocus_u=_f32(df),
                 defocus_v=_f32(df), astig=_f32(np.zeros(b)),
                 phase=_f32(np.zeros(b)), D=int(D), pixel=float(pixel))


def add_noise(rng, clean: np.ndarray, snr_db: float) -> np.ndarray:
    """Clean images plus white Gaussian noise at the requested SNR (dB).

    The SNR is the ratio of the clean batch's variance (all images, all
    pixels) to the noise variance.
    """
    clean = np.asarray(clean, dtype=np.float64)
    sig_var = float(clean.var())
    sd = np.sqrt(sig_var / (10.0 ** (snr_db / 10.0))) if sig_var > 0 else 1.0
    return _f32(clean + sd * rng.standard_normal(clean.shape))


# --------------------------------------------------------------------------
# Workload recipes
# --------------------------------------------------------------------------

def c1(seed: int = 1, b: int = 16):
    """N=1,000, cube of side 40 A, isotropic sd U(1,3) A, D=64, p=3.0 A."""
    rg, rv, rgt = streams(seed, 3)
    n = 1000

    def iso(rng):
        sd = rng.uniform(1.0, 3.0, size=n)
        return Mixture(
            means=_f32(rng.uniform(-20.0, 20.0, size=(n, 3))),
            log_scales=_f32(np.repeat(np.log(sd)[:, None], 3, axis=1)),
            quats=_f32(haar_quaternions(rng, n)),
            amps=_f32(np.exp(0.5 * rng.standard_normal(n))))

    g = iso(rg)
    gt = iso(rgt)
    v = views(rv, b, 64, 3.0, defocus_um=(1.0, 3.0))
    return g, v, gt


def c2(seed: int = 2, b: int = 256, n: int = 20000):
    """N=20,000 anisotropic, ball radius 60 A, D=128, p=1.5 A, SNR -20 dB."""
    rg, rv, rgt, rn = streams(seed, 4)
    g = mixture_anisotropic(rg, n, 60.0)
    gt = mixture_anisotropic(rgt, n, 60.0)
    v = views(rv, b, 128, 1.5, defocus_um=(0.8, 2.5), shift_px_sd=2.0)
    return g, v, gt, rn


def c3(seed: int = 3, b: int = 128):
    """Eight mixtures, uneven N, D_k in (128,192,256), p_k = 1.1+0.1k A."""
    ns = (5000, 10000, 20000, 40000, 60000, 80000, 100000, 150000)
    out = []
    for k, n in enumerate(ns):
        rg, rv, rgt, rn = streams(seed * 1000 + k, 4)
        D = (128, 192, 256)[k % 3]
        p = 1.1 + 0.1 * k
        radius = 0.3125 * D * p
        g = mixture_anisotropic(rg, n, radius)
        gt = mixture_anisotropic(rgt, n, radius)
        v = views(rv, b, D, p, defocus_um=(0.8, 2.5), shift_px_sd=2.0)
        out.append((g, v, gt, rn))
    return out


def c4(seed: int = 4, b: int = 64, n: int = 200000):
    """N=200,000 isotropic s=0.0075*D*p, ball radius 75 A, D=256, p=1.1 A.

    The initial state follows Sec. 4.1 (scale 0.0075 of the box side,
    A = 1/(2N)) with means uniform in the ball.  The ground truth for the
    observed images is an independent anisotropic mixture in the same ball
    with amplitudes rescaled to the same total mass.
    """
    rg, rv, rgt, rn = streams(seed, 4)
    D, p = 256, 1.1
    s0 = 0.0075 * D * p
    g = Mixture(
        means=_f32(uniform_ball(rg, n, 75.0)),
        log_scales=_f32(np.full((n, 3), np.log(s0))),
        quats=_f32(haar_quaternions(rg, n)),
        amps=_f32(np.full(n, 1.0 / (2 * n))))
    gt = mixture_anisotropic(rgt, n, 75.0)
    gt.amps = _f32(gt.amps * (0.5 / float(gt.amps.astype(np.float64).sum())))
    v = views(rv, b, D, p, defocus_um=(0.5, 2.5))
    return g, v, gt, rn


def mixture_domains(rng, n, n_domains=6, radius=40.0, extent=(6.0, 16.0),
                    scale_mu=np.log(1.5), scale_sd=0.3):
    """Random mixture with domain structure (an asymmetric, protein-like mass).

    Domain centres are uniform in a ball of `radius` A; each domain is an
    anisotropic normal cloud of Gaussian means with axis standard deviations
    U(extent) A in a Haar-random frame and a density weight U(0.5, 1.5);
    every Gaussian picks a domain uniformly.  Log-scales, quaternions and
    lognormal amplitudes as in mixture_anisotropic.
    """
    centres = uniform_ball(rng, n_domains, radius)
    frames = haar_rotations(rng, n_domains)
    sds = rng.uniform(extent[0], extent[1], size=(n_domains, 3))
    weight = rng.uniform(0.5, 1.5, size=n_domains)
    dom = rng.integers(0, n_domains, size=n)
    local = rng.standard_normal((n, 3)) * sds[dom]
    means = centres[dom] + np.einsum("nij,nj->ni", frames[dom], local)
    return Mixture(
        means=_f32(means),
        log_scales=_f32(scale_mu + scale_sd * rng.standard_normal((n, 3))),
        quats=_f32(haar_quaternions(rng, n)),
        amps=_f32(np.exp(0.5 * rng.standard_normal(n)) * weight[dom]),
    )


def pose_views(rng, b, D, pixel, defocus_um=(0.8, 2.5), shift_px_max=2.0):
    """Particle poses for pose search: Haar rotations, in-plane shifts
    uniform in [-shift_px_max, shift_px_max]^2 pixels, defocus U(defocus_um)."""
    v = views(rng, b, D, pixel, defocus_um=defocus_um)
    v.shift = _f32(rng.uniform(-shift_px_max, shift_px_max, size=(b, 2)) * pixel)
    return v


def c5(seed: int = 5, n_train: int = 200000, n_test: int = 2048, n: int = 20000, D: int = 128):
    """Learned pose proposal: a fixed N=20,000 random mixture (domain
    structure, radius 40 A domains), D=128, p=1.5 A; training and test
    particles at Haar poses, shifts U(-2, 2) px, defocus U(0.8, 2.5) um,
    white noise at SNR -20 dB added on the device per image."""
    rg, rtr, rte = streams(seed, 3)
    g = mixture_domains(rg, n)
    train = pose_views(rtr, n_train, D, 1.5)
    test = pose_views(rte, n_test, D, 1.5)
    return g, train, test


def c5_validation(seed: int = 5, n_val: int = 2048, D: int = 128):
    """Held-out validation particles of the learned-pose workload (a fourth
    stream of the same seed; the mixture, training and test draws of c5 are
    unchanged): same pose, shift and defocus distributions."""
    rva = streams(seed, 4)[3]
    return pose_views(rva, n_val, D, 1.5)
