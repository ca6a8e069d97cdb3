"""Mie series for plane-wave scattering by a sound-soft sphere (FP64).

The paper checks its solver against the analytical solution for a sphere of
radius a under an incident plane wave, observing the scattered field at r = 4
for scattering angles 0..180 degrees with phi = 0 (Sec. 6.4).  With the
incident field e^{ikz} = sum_n i^n (2n+1) j_n(kr) P_n(cos theta) and
p = 0 on r = a (eq. (7)), the scattered field is

  u_s(r, theta) = - sum_n i^n (2n+1) [j_n(ka) / h_n(ka)] h_n(kr) P_n(cos theta),

and the single-layer density q solving eq. (7) on the sphere follows from the
eigenvalue i k a^2 j_n(ka) h_n(ka) of the single-layer operator on degree-n
harmonics (the addition theorem, eq. (12)):

  q(theta) = - (i / (k a^2)) sum_n i^n (2n+1) P_n(cos theta) / h_n(ka),

with u_s = - (single-layer potential of q) outside the sphere.
"""
from __future__ import annotations

import numpy as np
from scipy import special as sp

from .special import sph_h1, sph_jn


def nmax_for(ka: float) -> int:
    return int(ka + 4.05 * ka ** (1.0 / 3.0) + 10)


def scattered(k: float, a: float, r, theta, nmax=None):
    r = np.asarray(r, np.float64)
    ct = np.cos(np.asarray(theta, np.float64))
    nmax = nmax_for(k * a) if nmax is None else nmax
    out = np.zeros(np.broadcast(r, ct).shape, np.complex128)
    for n in range(nmax + 1):
        cn = (1j ** n) * (2 * n + 1) * sph_jn(n, k * a) / sph_h1(n, k * a)
        out -= cn * sph_h1(n, k * r) * sp.eval_legendre(n, ct)
    return out


def incident(k: float, x, direction=(0.0, 0.0, 1.0)):
    return np.exp(1j * k * (np.asarray(x, np.float64) @ np.asarray(direction, np.float64)))


def density(k: float, a: float, theta, nmax=None):
    ct = np.cos(np.asarray(theta, np.float64))
    nmax = nmax_for(k * a) if nmax is None else nmax
    out = np.zeros(ct.shape, np.complex128)
    for n in range(nmax + 1):
        out += (1j ** n) * (2 * n + 1) * sp.eval_legendre(n, ct) / sph_h1(n, k * a)
    return -1j / (k * a * a) * out


def density_mode(k: float, a: float, n: int):
    """Coefficient of P_n(cos theta) in the Mie density."""
    return -1j / (k * a * a) * (1j ** n) * (2 * n + 1) / sph_h1(n, k * a)
