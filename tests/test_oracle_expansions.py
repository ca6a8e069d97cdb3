"""Pins for oracle.expansions: the addition theorem (eq. 12) and the
translation identities, checked pointwise against direct evaluation."""
import numpy as np
import pytest

from oracle import expansions as ex
from oracle.fmm import direct_sum, green
from oracle.special import regular_all, singular_all


def test_addition_theorem_eq12():
    k = 2.3
    rng = np.random.default_rng(1)
    y = rng.normal(size=3) * 0.2
    x = np.array([1.1, -0.6, 0.9])
    exact = green(k, x, y)
    P = 24
    R = regular_all(P, k, y[None])[0]
    S = singular_all(P, k, x[None])[0]
    # G = ik sum R_n^{-m}(y) S_n^m(x) with R_n^{-m} = conj(R_n^m) for real k
    approx = 1j * k * (np.conj(R) * S).sum()
    assert abs(approx - exact) / abs(exact) < 1e-13


@pytest.mark.parametrize("kind", ["rr", "sr", "ss"])
def test_translation_pointwise(kind):
    k = 1.7
    rng = np.random.default_rng(2)
    t = np.array([0.9, -0.7, 1.2])
    r = rng.normal(size=3)
    r *= (0.25 if kind == "sr" else 8.0 if kind == "ss" else 0.6) / np.linalg.norm(r)
    Pin, Pout = 6, 26
    if kind == "rr":
        lhs = regular_all(Pin, k, (r + t)[None])[0]
        T = ex.rr_matrix(t, k, Pout, Pin)
        rhs = regular_all(Pout, k, r[None])[0] @ T
    elif kind == "sr":
        lhs = singular_all(Pin, k, (r + t)[None])[0]
        T = ex.sr_matrix(t, k, Pout, Pin)
        rhs = regular_all(Pout, k, r[None])[0] @ T
    else:
        lhs = singular_all(Pin, k, (r + t)[None])[0]
        T = ex.rr_matrix(t, k, Pout, Pin)
        rhs = singular_all(Pout, k, r[None])[0] @ T
    np.testing.assert_allclose(rhs, lhs, rtol=0, atol=1e-9 * np.abs(lhs).max())


def test_p2m_m2l_l2p_error_falls_with_P():
    """Two well-separated boxes: P2M -> M2L -> L2P vs the direct sum."""
    k = 2.0
    rng = np.random.default_rng(4)
    s = 0.25
    cs = np.zeros(3)
    ct = np.array([1.0, 0.0, 0.0])
    ys = cs + rng.uniform(-s / 2, s / 2, (40, 3))
    xt = ct + rng.uniform(-s / 2, s / 2, (30, 3))
    q = rng.normal(size=40) + 1j * rng.normal(size=40)
    ref = direct_sum(k, xt, ys, q)
    errs = []
    for P in (2, 4, 6, 8, 10):
        M = ex.p2m(P, k, cs, ys, q)
        L = ex.sr_matrix(ct - cs, k, P) @ M
        y = ex.l2p(P, k, ct, L, xt)
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-7


def test_p2l_matches_m2l_of_point():
    """A single source: P2L at the target centre equals M2L of its P2M."""
    k, P = 1.3, 6
    ys = np.array([[0.05, -0.02, 0.03]])
    q = np.array([0.7 - 0.2j])
    ct = np.array([0.8, 0.5, -0.4])
    L1 = ex.p2l(P, k, ct, ys, q)
    L2 = ex.sr_matrix(ct, k, P, 30) @ ex.p2m(30, k, np.zeros(3), ys, q)
    np.testing.assert_allclose(L2, L1, atol=1e-10 * np.abs(L1).max())


def test_addition_theorem_complex_wavenumber():
    """Damped waves, k = 2.3 + 0.7i: G = ik sum R_n^{-m}(y) S_n^m(x) with
    R_n^{-m}(y) = j_n(k|y|) conj(Y_n^m) = conj(R_n^m(y) at conj(k))."""
    k = 2.3 + 0.7j
    rng = np.random.default_rng(1)
    y = rng.normal(size=3) * 0.2
    x = np.array([1.1, -0.6, 0.9])
    exact = green(k, x, y)
    assert abs(exact - np.exp(1j * 2.3 * np.linalg.norm(x - y)) * np.exp(-0.7 * np.linalg.norm(x - y))
               / (4 * np.pi * np.linalg.norm(x - y))) < 1e-15
    P = 24
    Rm = np.conj(regular_all(P, np.conj(k), y[None])[0])
    S = singular_all(P, k, x[None])[0]
    approx = 1j * k * (Rm * S).sum()
    assert abs(approx - exact) / abs(exact) < 1e-12


@pytest.mark.parametrize("kind", ["rr", "sr"])
def test_translation_pointwise_complex_wavenumber(kind):
    k = 1.7 + 0.5j
    rng = np.random.default_rng(3)
    t = np.array([0.9, -0.7, 1.2])
    r = rng.normal(size=3)
    r *= (0.25 if kind == "sr" else 0.6) / np.linalg.norm(r)
    Pin, Pout = 6, 26
    f = regular_all if kind == "rr" else singular_all
    lhs = f(Pin, k, (r + t)[None])[0]
    T = (ex.rr_matrix if kind == "rr" else ex.sr_matrix)(t, k, Pout, Pin)
    rhs = regular_all(Pout, k, r[None])[0] @ T
    np.testing.assert_allclose(rhs, lhs, rtol=0, atol=1e-9 * np.abs(lhs).max())


def test_p2m_m2l_l2p_complex_wavenumber():
    k = 2.0 + 0.8j
    rng = np.random.default_rng(5)
    s = 0.25
    cs, ct = np.zeros(3), np.array([1.0, 0.0, 0.0])
    ys = cs + rng.uniform(-s / 2, s / 2, (40, 3))
    xt = ct + rng.uniform(-s / 2, s / 2, (30, 3))
    q = rng.normal(size=40) + 1j * rng.normal(size=40)
    ref = direct_sum(k, xt, ys, q)
    errs = []
    for P in (2, 4, 6, 8, 10):
        L = ex.sr_matrix(ct - cs, k, P) @ ex.p2m(P, k, cs, ys, q)
        errs.append(np.linalg.norm(ex.l2p(P, k, ct, L, xt) - ref) / np.linalg.norm(ref))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-7


def test_m2p_equals_direct_sum_far_from_the_sources():
    """The multipole expansion evaluated at far points (M2P) converges to the
    direct sum as P grows: the other half of the addition theorem, eq. (12),
    with the roles of source and target exchanged (|x - c| > |y - c|)."""
    k = 1.9
    rng = np.random.default_rng(11)
    c = np.array([0.1, -0.2, 0.05])
    ys = c + rng.uniform(-0.15, 0.15, (25, 3))
    q = rng.normal(size=25) + 1j * rng.normal(size=25)
    xt = c + np.array([[1.2, 0.3, -0.4], [-0.9, 0.8, 0.2], [0.1, -0.2, 1.1]])
    ref = direct_sum(k, xt, ys, q)
    errs = []
    for P in (2, 4, 6, 8, 10, 12):
        M = ex.p2m(P, k, c, ys, q)
        errs.append(np.linalg.norm(ex.m2p(P, k, c, M, xt) - ref) / np.linalg.norm(ref))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-9
    # a dropped factor (ik) or a conjugated multipole would be O(1) wrong
    M = ex.p2m(12, k, c, ys, q)
    assert np.linalg.norm(ex.m2p(12, k, c, np.conj(M), xt) - ref) > 0.1 * np.linalg.norm(ref)


def _m_of(P):
    return np.array([m for n in range(P) for m in range(-n, n + 1)])


@pytest.mark.parametrize("t,k,P", [((1.1, 0.6, -0.9), 2.5, 7), ((-0.4, 1.3, 0.8), 6.0, 9),
                                   ((0.0, 0.0, 1.5), 3.0, 6), ((2.0, -2.0, 0.0), 1.0, 8)])
def test_translation_turned_into_the_xz_plane(t, k, P):
    """The M2L translation (S|R)(t) of eq. (14) equals D^-1 (S|R)(t') D with
    t' = t turned about the z axis into the xz-plane and D = diag(e^{i m
    phi}), phi the azimuth of t; (S|R)(t') commutes with the exchange
    m <-> -m, so it splits into a block on M^m + M^-m (m >= 0) and one on
    M^m - M^-m (m > 0) whose sizes are P(P+1)/2 and P(P-1)/2."""
    t = np.asarray(t, np.float64)
    phi = np.arctan2(t[1], t[0])
    tp = np.array([np.hypot(t[0], t[1]), 0.0, t[2]])
    T = ex.sr_matrix(t, k, P)
    Tp = ex.sr_matrix(tp, k, P)
    D = np.diag(np.exp(1j * _m_of(P) * phi))
    assert np.abs(np.linalg.inv(D) @ Tp @ D - T).max() <= 1e-13 * np.abs(T).max()
    # the exchange m <-> -m
    Pi = np.zeros((P * P, P * P))
    for n in range(P):
        for m in range(-n, n + 1):
            Pi[n * n + n - m, n * n + n + m] = 1.0
    assert np.abs(Pi @ Tp - Tp @ Pi).max() <= 1e-14 * np.abs(Tp).max()
    # the symmetric and antisymmetric bases split (S|R)(t') into two blocks
    sym, anti = [], []
    for n in range(P):
        for m in range(0, n + 1):
            u = np.zeros(P * P)
            u[n * n + n + m] += 1.0
            u[n * n + n - m] += 1.0
            sym.append(u / np.linalg.norm(u))
            if m > 0:
                v = np.zeros(P * P)
                v[n * n + n + m] = 1.0
                v[n * n + n - m] = -1.0
                anti.append(v / np.sqrt(2.0))
    B = np.array(sym + anti).T             # orthogonal change of basis
    Tb = B.T @ Tp @ B
    ns = len(sym)
    assert ns == P * (P + 1) // 2 and len(anti) == P * (P - 1) // 2
    off = max(np.abs(Tb[:ns, ns:]).max(), np.abs(Tb[ns:, :ns]).max())
    assert off <= 1e-13 * np.abs(Tb).max()
