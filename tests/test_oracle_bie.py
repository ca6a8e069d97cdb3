"""Pins for oracle.bie, oracle.mie and oracle.gmres."""
import math

import numpy as np
import pytest

import synth
from oracle import bie, gmres, mie


def test_icosphere_closed_and_outward():
    V, T = synth.icosphere(3)
    assert len(T) == 20 * 4 ** 3
    edges = {}
    for t in T:
        for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            edges[(a, b)] = edges.get((a, b), 0) + 1
    # closed, consistently oriented: every directed edge once, its reverse once
    assert all(v == 1 for v in edges.values())
    assert all((b, a) in edges for (a, b) in edges)
    pan = bie.panels(V, T)
    assert np.all((pan["normal"] * pan["centroid"]).sum(axis=1) > 0)
    assert abs(pan["area"].sum() - 4 * math.pi) < 0.02 * 4 * math.pi


def test_gauss_rule_exact_for_quadratics():
    rng = np.random.default_rng(0)
    a, b, c = rng.normal(size=(3, 3))
    pan = bie.panels(np.stack([a, b, c]), np.array([[0, 1, 2]]))
    gp, w = bie.gauss_sources(pan)
    assert abs(w.sum() - pan["area"][0]) < 1e-15
    # exact integral of a quadratic via a high-order Duffy rule (polynomial: exact)
    f = lambda p: 1.0 + p[:, 0] - 2 * p[:, 1] ** 2 + 3 * p[:, 0] * p[:, 2]
    pts, ww = bie.duffy_rule(a, b, c, 6)
    assert abs((w * f(gp)).sum() - (ww * f(pts)).sum()) < 1e-13


def test_self_integral_equilateral_closed_form():
    a = np.array([0.0, 0, 0]); b = np.array([1.0, 0, 0]); c = np.array([0.5, math.sqrt(3) / 2, 0])
    ref = math.sqrt(3) * math.log(2 + math.sqrt(3)) / (4 * math.pi)
    assert abs(bie.self_integral(0.0, a, b, c) - ref) < 1e-12


def test_panel_integrals_vs_laplace_closed_form():
    """Closed form vs Duffy quadrature (self) and vs the subdivided rule (near)."""
    rng = np.random.default_rng(1)
    for _ in range(10):
        # well-shaped panels: perturbed equilateral triangles of random size/pose
        base = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.5, math.sqrt(3) / 2, 0]])
        base += rng.uniform(-0.15, 0.15, (3, 3)) * np.array([1, 1, 0])
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        a, b, c = (base @ Q.T) * rng.uniform(0.01, 2.0) + rng.normal(size=3)
        x = (a + b + c) / 3
        ref = bie.laplace_panel_analytic(x, a, b, c) / (4 * math.pi)
        assert abs(bie.self_integral_duffy(0.0, a, b, c, n=48) - ref) < 1e-10 * abs(ref)
        h = max(np.linalg.norm(b - a), np.linalg.norm(c - b), np.linalg.norm(a - c))
        nrm = np.cross(b - a, c - a); nrm /= np.linalg.norm(nrm)
        xo = x + 0.4 * h * nrm + 0.3 * (b - a)
        ref = bie.laplace_panel_analytic(xo, a, b, c) / (4 * math.pi)
        assert abs(bie.panel_integral(0.0, xo, a, b, c) - ref) < 1e-9 * abs(ref)


def test_self_integral_split_vs_duffy():
    """Closed form + Duffy remainder equals the plain Duffy rule at k > 0."""
    a = np.array([0.0, 0, 0]); b = np.array([0.1, 0, 0]); c = np.array([0.045, 0.09, 0.01])
    for k in (1.0, 20.0):
        assert abs(bie.self_integral(k, a, b, c) - bie.self_integral_duffy(k, a, b, c, n=64)) \
            < 1e-10 * abs(bie.self_integral(k, a, b, c))


def test_self_integral_converged_in_k():
    a = np.array([0.0, 0, 0]); b = np.array([0.1, 0, 0]); c = np.array([0.03, 0.08, 0])
    s1 = bie.self_integral(20.0, a, b, c, n=24)
    s2 = bie.self_integral(20.0, a, b, c, n=40)
    assert abs(s1 - s2) < 1e-13 * abs(s2)


def test_single_layer_of_constant_laplace_limit():
    """sum_j A_ij -> integral of 1/(4 pi |x-y|) over the unit sphere = 1."""
    V, T = synth.icosphere(2)
    A = bie.dense_matrix(1e-8, V, T)
    rs = A.sum(axis=1).real
    assert abs(rs.mean() - 1.0) < 0.03


def test_mie_boundary_condition_and_quadrature():
    k, a = 6.0, 1.0
    th = np.linspace(0, np.pi, 37)
    xs = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    us = mie.scattered(k, a, a, th)
    assert np.max(np.abs(us + mie.incident(k, xs))) < 1e-11
    # -single layer of the Mie density reproduces u_s at r = 4 (quadrature on the exact sphere)
    x, w = np.polynomial.legendre.leggauss(60)
    nph = 120
    tq = np.arccos(x)
    ph = 2 * np.pi * np.arange(nph) / nph
    TQ, PH = np.meshgrid(tq, ph, indexing="ij")
    W = np.outer(w, np.full(nph, 2 * np.pi / nph)).ravel()
    Y = np.stack([np.sin(TQ) * np.cos(PH), np.sin(TQ) * np.sin(PH), np.cos(TQ)], -1).reshape(-1, 3)
    q = mie.density(k, a, TQ.ravel())
    xo = 4.0 * np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    from oracle.fmm import green
    us_q = -(green(k, xo[:, None, :], Y[None]) * (W * q)[None]).sum(axis=1)
    np.testing.assert_allclose(us_q, mie.scattered(k, a, 4.0, th), rtol=0, atol=1e-9)


def test_gmres_matches_dense_solve_and_special_cases():
    rng = np.random.default_rng(2)
    n = 60
    A = np.eye(n) * 4 + rng.normal(size=(n, n)) / math.sqrt(n) + 1j * rng.normal(size=(n, n)) / math.sqrt(n)
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    x, info = gmres.gmres(lambda v: A @ v, b, tol=1e-10, restart=30)
    assert info["converged"]
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-8 * np.abs(x).max())
    x, info = gmres.gmres(lambda v: v, b, tol=1e-12)
    assert info["iters"] == 1
    d = np.repeat([1.0, 2.0, 3.0 + 1j, -4.0], n // 4)
    x, info = gmres.gmres(lambda v: d * v, b, tol=1e-12, restart=30)
    assert info["iters"] <= 4 and info["converged"]


def test_bie_solve_converges_toward_mie():
    """Flat panels: u_s error vs Mie at r = 4 falls with refinement (1 -> 2)."""
    k = 3.0
    th = np.radians(np.arange(0, 181, 5))
    xo = 4.0 * np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    um = mie.scattered(k, 1.0, 4.0, th)
    errs = []
    for s in (1, 2):
        V, T = synth.icosphere(s)
        A = bie.dense_matrix(k, V, T)
        q = np.linalg.solve(A, bie.plane_wave_rhs(k, V, T))
        us = bie.scattered_field(k, V, T, q, xo)
        errs.append(np.linalg.norm(us - um) / np.linalg.norm(um))
    assert errs[1] < 0.6 * errs[0], errs


@pytest.mark.parametrize("height,k", [(0.06, 2 * math.pi), (0.01, 2 * math.pi), (0.01, 20.0)])
def test_self_integral_elongated_panels(height, k):
    """Elongated panels (unit base, apex at the given height; area / longest
    edge^2 = height / 2): the bounded part (e^{ikR} - 1)/(4 pi R) of the self
    integral against a composite rule with no singular treatment at all, 4^7
    uniform sub-triangles with a 7-point rule each (the integrand is bounded
    and continuous, so the composite rule converges)."""
    a = np.array([0.0, 0, 0]); b = np.array([1.0, 0, 0]); c = np.array([0.37, height, 0])
    x = (a + b + c) / 3
    # 7-point degree-5 rule on the reference triangle (barycentric, weights sum 1)
    s15 = math.sqrt(15.0)
    a1, b1 = (6 - s15) / 21, (9 + 2 * s15) / 21
    a2, b2 = (6 + s15) / 21, (9 - 2 * s15) / 21
    lam = np.array([[1 / 3, 1 / 3, 1 / 3], [a1, a1, b1], [a1, b1, a1], [b1, a1, a1],
                    [a2, a2, b2], [a2, b2, a2], [b2, a2, a2]])
    wts = np.array([9 / 40] + [(155 - s15) / 1200] * 3 + [(155 + s15) / 1200] * 3)
    tri = np.array(bie.subdivide(a, b, c, 7))                  # (4^7, 3, 3)
    pts = np.einsum("gv,tvd->tgd", lam, tri)
    R = np.linalg.norm(pts - x, axis=2)
    sub_area = 0.5 * np.linalg.norm(np.cross(b - a, c - a)) / len(tri)
    brute = (np.expm1(1j * k * R) / (4 * np.pi * R) * wts).sum() * sub_area
    smooth = bie.self_integral(k, a, b, c) - bie.laplace_panel_analytic(x, a, b, c) / (4 * math.pi)
    err = abs(smooth - brute) / abs(bie.self_integral(k, a, b, c))
    print(height, k, err)
    assert err < 1e-7


@pytest.mark.parametrize("k", [2.0, 2 * np.pi, 6.0])
def test_mie_density_modes_are_its_legendre_coefficients(k):
    """The n-th Legendre coefficient of the Mie density (density_mode),
    recovered independently by Gauss-Legendre projection of the density
    itself: c_n = (2n+1)/2 * integral of q(theta) P_n(cos theta) over
    cos theta in [-1, 1]."""
    from scipy.special import eval_legendre
    a = 1.0
    x, w = np.polynomial.legendre.leggauss(120)
    q = mie.density(k, a, np.arccos(x))
    for n in range(0, mie.nmax_for(k * a) + 1):
        cn = (2 * n + 1) / 2.0 * np.sum(w * q * eval_legendre(n, x))
        assert abs(cn - mie.density_mode(k, a, n)) <= 1e-12 * max(1.0, abs(cn)), (n, cn)
