"""Pins for oracle.gaunt against sympy's Wigner 3j and against quadrature."""
import numpy as np
import pytest

from oracle.gaunt import gaunt, wigner3j
from oracle.special import ylm_all, idx


def test_wigner3j_vs_sympy():
    wig = pytest.importorskip("sympy.physics.wigner")
    rng = np.random.default_rng(5)
    for _ in range(200):
        j1, j2 = rng.integers(0, 9, 2)
        j3 = rng.integers(abs(j1 - j2), j1 + j2 + 1)
        m1 = rng.integers(-j1, j1 + 1)
        m2 = rng.integers(-j2, j2 + 1)
        m3 = -m1 - m2
        ref = float(wig.wigner_3j(int(j1), int(j2), int(j3), int(m1), int(m2), int(m3)))
        assert abs(wigner3j(int(j1), int(j2), int(j3), int(m1), int(m2), int(m3)) - ref) < 1e-14


def test_gaunt_vs_quadrature():
    # Gauss-Legendre x trapezoid, exact for the degree-<= 3*8 products used here
    x, w = np.polynomial.legendre.leggauss(20)
    nph = 40
    th = np.arccos(x)
    ph = 2 * np.pi * np.arange(nph) / nph
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(w, np.full(nph, 2 * np.pi / nph)).ravel()
    Y = ylm_all(9, TH.ravel(), PH.ravel())
    rng = np.random.default_rng(9)
    for _ in range(150):
        n, n2 = rng.integers(0, 5, 2)
        l = int(rng.integers(abs(n - n2), n + n2 + 1))
        m = int(rng.integers(-n, n + 1))
        m2 = int(rng.integers(-n2, n2 + 1))
        mu = m - m2
        if abs(mu) > l:
            continue
        q = (W * Y[:, idx(n, m)] * np.conj(Y[:, idx(n2, m2)]) * np.conj(Y[:, idx(l, mu)])).sum()
        assert abs(q - gaunt(int(n), m, int(n2), m2, l)) < 1e-13
