"""Pins for oracle.special: closed forms, symmetry and orthonormality."""
import math

import numpy as np
import pytest
from scipy import special as sp

from oracle.special import idx, sph_h1, sph_jn, ylm_all, cart_to_sph, regular_all


def _sphere_rule(nt=24, nphi=48):
    x, w = np.polynomial.legendre.leggauss(nt)
    th = np.arccos(x)
    ph = 2 * np.pi * np.arange(nphi) / nphi
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(w, np.full(nphi, 2 * np.pi / nphi))
    return TH.ravel(), PH.ravel(), W.ravel()


def test_low_degree_closed_forms():
    th, ph = 0.7, -1.1
    Y = ylm_all(3, np.array([th]), np.array([ph]))[0]
    assert abs(Y[idx(0, 0)] - 1 / math.sqrt(4 * math.pi)) < 1e-15
    assert abs(Y[idx(1, 0)] - math.sqrt(3 / (4 * math.pi)) * math.cos(th)) < 1e-15
    # no Condon-Shortley phase: Y_1^1 = +sqrt(3/8pi) sin(theta) e^{i phi}
    assert abs(Y[idx(1, 1)] - math.sqrt(3 / (8 * math.pi)) * math.sin(th) * np.exp(1j * ph)) < 1e-15
    assert abs(Y[idx(2, 2)] - 0.25 * math.sqrt(15 / (2 * math.pi)) * math.sin(th) ** 2 * np.exp(2j * ph)) < 1e-15


def test_conjugate_symmetry_and_orthonormality():
    P = 8
    th, ph, w = _sphere_rule()
    Y = ylm_all(P, th, ph)
    for n in range(P):
        for m in range(-n, n + 1):
            np.testing.assert_allclose(Y[:, idx(n, -m)], np.conj(Y[:, idx(n, m)]), atol=1e-15)
    G = (Y.conj().T * w) @ Y
    np.testing.assert_allclose(G, np.eye(P * P), atol=1e-12)


def test_addition_theorem_legendre():
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=(2, 3))
    _, ta, pa = cart_to_sph(a)
    _, tb, pb = cart_to_sph(b)
    cg = a @ b / np.linalg.norm(a) / np.linalg.norm(b)
    Ya = ylm_all(10, np.array([ta]), np.array([pa]))[0]
    Yb = ylm_all(10, np.array([tb]), np.array([pb]))[0]
    for n in range(10):
        sl = slice(n * n, (n + 1) ** 2)
        lhs = (Ya[sl] * np.conj(Yb[sl])).sum()
        assert abs(lhs - (2 * n + 1) / (4 * math.pi) * sp.eval_legendre(n, cg)) < 1e-13


def test_bessel_closed_forms():
    x = np.array([0.3, 1.0, 7.5, 40.0])
    np.testing.assert_allclose(sph_jn(0, x), np.sin(x) / x, rtol=1e-14)
    np.testing.assert_allclose(sph_h1(0, x), -1j * np.exp(1j * x) / x, rtol=1e-14)
    np.testing.assert_allclose(sph_h1(1, x), -np.exp(1j * x) * (x + 1j) / x ** 2, rtol=1e-13)


def test_regular_harmonic_at_origin():
    R = regular_all(5, 2.0, np.zeros((1, 3)))[0]
    assert abs(R[0] - 1 / math.sqrt(4 * math.pi)) < 1e-15
    assert np.all(R[1:] == 0)
