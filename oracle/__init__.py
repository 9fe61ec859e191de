"""FP64 CPU oracle of the cryoSplat renderer (test infrastructure only).

This package is a plain, slow, obviously correct statement of what the GPU
hot path computes, written from the paper (Sec. 3.2-3.3, App. A.2) in numpy
FP64.  It exists to check the GPU library: only the tests, the smoke check
and the benchmark's CPU-baseline leg may import it.  It shares no code with
the HIP path and imports nothing from the product package.

Modules
-------
model      3-D Gaussians, viewing transform, orthogonal projection, splat
           sum on the FFT-aligned pixel grid (Eq. 2-9, 12, 13).
ctf        electron wavelength, weak-phase CTF and its Fourier-space
           application (Eq. 14).
objective  squared-error loss and its analytic gradient (Eq. 15-21) plus
           central finite differences.
adam       the Adam update used by the optimisation loop (Alg. 1).

Every function is pinned by tests under ``tests/`` against closed forms,
brute-force line integrals, textbook special cases or finite differences.
"""
from . import model, ctf, objective, adam  # noqa: F401
