"""Special functions for the oracle (FP64, scipy).

Convention (the one in which the addition theorem eq. (12) holds as printed):
    Y_n^m(theta, phi) = N_n^|m| P_n^|m|(cos theta) exp(i m phi),
    N_n^m = sqrt((2n+1)/(4 pi) (n-m)!/(n+m)!),
with P_n^m the associated Legendre function WITHOUT the Condon-Shortley phase.
Then Y_n^{-m} = conj(Y_n^m) and the Y_n^m are orthonormal on the unit sphere.

Coefficient index: idx(n, m) = n*n + n + m, for 0 <= n < P, -n <= m <= n.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special as sp


def idx(n: int, m: int) -> int:
    return n * n + n + m


def sph_jn(n, x):
    return sp.spherical_jn(n, x)


def sph_h1(n, x):
    """Spherical Hankel function of the first kind, h_n = j_n + i y_n
    (outgoing for the exp(-i w t) convention of eq. (2))."""
    return sp.spherical_jn(n, x) + 1j * sp.spherical_yn(n, x)


def _norm(n: int, am: int) -> float:
    return math.sqrt((2 * n + 1) / (4.0 * math.pi)
                     * math.factorial(n - am) / math.factorial(n + am))


def cart_to_sph(v):
    """(r, theta, phi) of vectors v (..., 3); direction at r = 0 is +z."""
    v = np.asarray(v, dtype=np.float64)
    r = np.sqrt((v * v).sum(axis=-1))
    safe = np.where(r > 0, r, 1.0)
    ct = np.clip(v[..., 2] / safe, -1.0, 1.0)
    ct = np.where(r > 0, ct, 1.0)
    theta = np.arccos(ct)
    phi = np.arctan2(v[..., 1], v[..., 0])
    return r, theta, phi


def ylm_all(P: int, theta, phi):
    """Y_n^m for all n < P at angles; returns complex array (..., P*P)."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    out = np.zeros(theta.shape + (P * P,), dtype=np.complex128)
    ct = np.cos(theta)
    for n in range(P):
        for m in range(-n, n + 1):
            am = abs(m)
            # scipy's lpmv carries the Condon-Shortley phase (-1)^m; remove it
            p = ((-1) ** am) * sp.lpmv(am, n, ct)
            out[..., idx(n, m)] = _norm(n, am) * p * np.exp(1j * m * phi)
    return out


def regular_all(P: int, k: float, v):
    """R_n^m(v) = j_n(k|v|) Y_n^m(v^) for all n < P; shape (..., P*P)."""
    r, th, ph = cart_to_sph(v)
    Y = ylm_all(P, th, ph)
    for n in range(P):
        jn = sph_jn(n, k * r)
        sl = slice(n * n, (n + 1) * (n + 1))
        Y[..., sl] *= jn[..., None]
    return Y


def singular_all(P: int, k: float, v):
    """S_n^m(v) = h_n(k|v|) Y_n^m(v^) for all n < P (|v| > 0)."""
    r, th, ph = cart_to_sph(v)
    if np.any(r == 0):
        raise ValueError("singular harmonic at the origin")
    Y = ylm_all(P, th, ph)
    for n in range(P):
        hn = sph_h1(n, k * r)
        if not np.all(np.isfinite(hn)):
            raise FloatingPointError("h_n overflow in FP64")
        sl = slice(n * n, (n + 1) * (n + 1))
        Y[..., sl] *= hn[..., None]
    return Y
