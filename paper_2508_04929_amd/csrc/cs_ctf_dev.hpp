// CTF values on the DFT grid, shared by the device code of the Fourier
// passes (App. A.2, Eq. 13-14).
#pragma once

#include "cs_internal.hpp"

namespace cs {

// ---------------------------------------------------------------------------
// CTF on the DFT grid.  Index k has frequency f(k)/(D p) with f(k) = k for
// k < D/2 (k = D/2 maps to -D/2) and k - D above; the row frequency is
// negated (y-flip of Eq. 13).  The Nyquist row/column value is the mean
// over the two mirror frequencies, which keeps H^ exactly even.
// ---------------------------------------------------------------------------
__device__ inline double ctf_at(double sx, double sy, const CtfDev &c, double du, double dv,
                         double c2a, double s2a, double ph, double amp_s) {
  const double s2 = sx * sx + sy * sy;
  double df = 0.5 * (du + dv);
  if (s2 > 0.0 && du != dv) {
    const double cos2 = (sx * sx - sy * sy) / s2, sin2 = 2.0 * sx * sy / s2;
    df += 0.5 * (du - dv) * (cos2 * c2a + sin2 * s2a);
  }
  const double chi = M_PI * c.lam * df * s2 - 0.5 * M_PI * c.cs * c.lam * c.lam * c.lam * s2 * s2 - ph;
  // phase in FP64, reduced to [-pi, pi] in FP64, then one FP32 sincos (about
  // 1e-7 absolute in the CTF)
  const double turns = chi * (0.5 / M_PI);
  const float red = (float)((turns - rint(turns)) * (2.0 * M_PI));
  float sn, cs;
  sincosf(red, &sn, &cs);
  double h = -(amp_s * (double)sn + c.w * (double)cs);
  if (c.bfactor != 0.0) h *= exp(-0.25 * c.bfactor * s2);
  return h;
}

// Per-particle constants of the CTF: defocus, astigmatism angle (as cos 2a,
// sin 2a) and extra phase.
struct CtfParticle {
  double du, dv, c2a, s2a, ph;
};

__device__ inline CtfParticle ctf_particle(const CtfDev &c, int b) {
  CtfParticle q;
  q.du = c.defocus_u[b];
  q.dv = c.defocus_v[b];
  const double a = c.astig ? (double)c.astig[b] : 0.0;
  q.ph = c.phase ? (double)c.phase[b] : 0.0;
  float s2f, c2f;
  sincosf((float)(2.0 * a), &s2f, &c2f);
  q.c2a = c2f;
  q.s2a = s2f;
  return q;
}

// Constants of a CTF grid shared by all its values: the frequency step
// 1 / (L p) and the phase-contrast weight sqrt(1 - w^2).
struct CtfGrid {
  double inv, amp_s;
};

__device__ inline CtfGrid ctf_grid(int L, float pixel, const CtfDev &c) {
  return CtfGrid{1.0 / ((double)L * (double)pixel), sqrt(1.0 - c.w * c.w)};
}

__device__ inline float ctf_value(int ky, int kx, int L, const CtfGrid &g, const CtfDev &c,
                                  const CtfParticle &q) {
  const int half = L / 2;
  const int fkx = (kx < (L + 1) / 2) ? kx : kx - L;
  const int fky = (ky < (L + 1) / 2) ? ky : ky - L;
  const double sx = fkx * g.inv, sy = -fky * g.inv;
  double h = ctf_at(sx, sy, c, q.du, q.dv, q.c2a, q.s2a, q.ph, g.amp_s);
  if ((L % 2 == 0) && (kx == half || ky == half)) {
    const double mx = (kx == half) ? -sx : sx, my = (ky == half) ? -sy : sy;
    h = 0.5 * (h + ctf_at(mx, my, c, q.du, q.dv, q.c2a, q.s2a, q.ph, g.amp_s));
  }
  return (float)h;
}

}  // namespace cs
