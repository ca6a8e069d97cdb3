"""Multipole / local expansions and translation operators (FP64).

Written from Sec. 2.3 (eqs. (12)-(14)) with the convention of
`oracle.special`.  For |x - c| > |y - c| the addition theorem reads

    G(x, y) = e^{ik|x-y|} / (4 pi |x-y|) = ik sum_{n,m} R_n^{-m}(y - c) S_n^m(x - c),

with R_n^m(v) = j_n(k|v|) Y_n^m(v^) (regular) and S_n^m(v) = h_n(k|v|) Y_n^m(v^)
(singular).  Truncation "at P" keeps degrees 0..P-1, i.e. P^2 coefficients
(Sec. 2.3, the text after eq. (14)).

Expansions of a field phi:
  multipole about c:  phi(x) = ik sum M_n^m S_n^m(x - c),  M_n^m = sum_j q_j R_n^{-m}(y_j - c)
  local about c:      phi(x) = ik sum L_n^m R_n^m(x - c),  L_n^m = sum_j q_j S_n^{-m}(y_j - c)

Translations (derived from the plane-wave expansion and the Funk-Hecke
formula; G(...) is `oracle.gaunt.gaunt`):
  R_n^m(r + t) = sum_{n',m'} (R|R)_{n'n}^{m'm}(t) R_{n'}^{m'}(r)                 (all r, t)
  S_n^m(r + t) = sum_{n',m'} (S|R)_{n'n}^{m'm}(t) R_{n'}^{m'}(r)                 (|r| < |t|)
  S_n^m(r + t) = sum_{n',m'} (R|R)_{n'n}^{m'm}(t) S_{n'}^{m'}(r)                 (|r| > |t|)
  (R|R)_{n'n}^{m'm}(t) = 4 pi sum_l i^{n'+l-n} R_l^{m-m'}(t) G(n,m; n',m'; l),
  (S|R) is the same with S_l in place of R_l.
Hence, for matrices with rows (n',m') and columns (n,m):
  M2M  M_parent = RR(c_parent - c_child) @ M_child
  M2L  L_target = SR(c_target - c_source) @ M_source
  L2L  L_child  = RR(c_child - c_parent) @ L_parent
each being the principal block n, n' < P of the exact operator.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np

from .gaunt import gaunt
from .special import (cart_to_sph, idx, regular_all, singular_all,
                      sph_h1, ylm_all, sph_jn)


@lru_cache(maxsize=None)
def _coupling(Pout: int, Pin: int):
    """Sparse list of (row, col, l, mu-index, coeff) with
    coeff = 4 pi i^{n'+l-n} G(n,m; n',m'; l) and mu = m - m'."""
    rows, cols, lidx, vals = [], [], [], []
    for n in range(Pin):
        for m in range(-n, n + 1):
            for n2 in range(Pout):
                for m2 in range(-n2, n2 + 1):
                    mu = m - m2
                    for l in range(abs(n - n2), n + n2 + 1):
                        if abs(mu) > l or (n + n2 + l) % 2:
                            continue
                        g = gaunt(n, m, n2, m2, l)
                        if g == 0.0:
                            continue
                        rows.append(idx(n2, m2))
                        cols.append(idx(n, m))
                        lidx.append(idx(l, mu))
                        vals.append(4.0 * math.pi * (1j ** ((n2 + l - n) % 4)) * g)
    return (np.array(rows), np.array(cols), np.array(lidx),
            np.array(vals, dtype=np.complex128))


def _assemble(harm, Pout: int, Pin: int) -> np.ndarray:
    rows, cols, lidx, vals = _coupling(Pout, Pin)
    T = np.zeros((Pout * Pout, Pin * Pin), dtype=np.complex128)
    np.add.at(T, (rows, cols), vals * harm[lidx])
    return T


def rr_matrix(t, k: float, Pout: int, Pin: int | None = None) -> np.ndarray:
    """(R|R)(t): shape (Pout^2, Pin^2)."""
    Pin = Pout if Pin is None else Pin
    Lmax = Pout + Pin - 1
    harm = regular_all(Lmax, k, np.asarray(t, dtype=np.float64))
    return _assemble(harm, Pout, Pin)


def sr_matrix(t, k: float, Pout: int, Pin: int | None = None) -> np.ndarray:
    """(S|R)(t): shape (Pout^2, Pin^2); requires t != 0."""
    Pin = Pout if Pin is None else Pin
    Lmax = Pout + Pin - 1
    harm = singular_all(Lmax, k, np.asarray(t, dtype=np.float64))
    return _assemble(harm, Pout, Pin)


def p2m(P: int, k, c, y, q) -> np.ndarray:
    """M_n^m = sum_j q_j R_n^{-m}(y_j - c), R_n^{-m}(v) = j_n(k|v|) conj(Y_n^m(v^))
    (for real k this is conj(R_n^m); a complex k stays unconjugated in j_n)."""
    v = np.asarray(y, np.float64) - np.asarray(c, np.float64)
    r, th, ph = cart_to_sph(v)
    Y = ylm_all(P, th, ph)
    qq = np.asarray(q, np.complex128)
    out = np.zeros(P * P, dtype=np.complex128)
    for n in range(P):
        jn = sph_jn(n, k * r)
        sl = slice(n * n, (n + 1) * (n + 1))
        out[sl] = (qq[:, None] * jn[:, None] * np.conj(Y[:, sl])).sum(axis=0)
    return out


def p2l(P: int, k: float, c, y, q) -> np.ndarray:
    """L_n^m = sum_j q_j S_n^{-m}(y_j - c), with S_n^{-m} = h_n conj(Y_n^m)."""
    v = np.asarray(y, np.float64) - np.asarray(c, np.float64)
    r, th, ph = cart_to_sph(v)
    Y = ylm_all(P, th, ph)
    out = np.zeros(P * P, dtype=np.complex128)
    qq = np.asarray(q, np.complex128)
    for n in range(P):
        hn = sph_h1(n, k * r)
        sl = slice(n * n, (n + 1) * (n + 1))
        out[sl] = (qq[:, None] * hn[:, None] * np.conj(Y[:, sl])).sum(axis=0)
    return out


def m2p(P: int, k: float, c, M, x) -> np.ndarray:
    """phi(x) = ik sum M_n^m S_n^m(x - c)."""
    S = singular_all(P, k, np.asarray(x, np.float64) - np.asarray(c, np.float64))
    return 1j * k * (S @ np.asarray(M))


def l2p(P: int, k: float, c, L, x) -> np.ndarray:
    """phi(x) = ik sum L_n^m R_n^m(x - c)   (eq. (13))."""
    R = regular_all(P, k, np.asarray(x, np.float64) - np.asarray(c, np.float64))
    return 1j * k * (R @ np.asarray(L))
