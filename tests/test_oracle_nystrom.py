"""Pins of the curved-element Nystrom oracle (oracle/nystrom.py) against what
mathematics fixes: exact polynomial moments of the reference triangle,
interpolation identities, the closed-form integral of 1/R over a flat
triangle, the area of the sphere, the single-layer potential of a constant
density on the unit sphere, and the Mie series."""
import numpy as np
import pytest

import synth
from oracle import bie, mie
from oracle import nystrom as ny


def test_rule_exact_to_degree_4_only():
    """The six-point rule integrates every monomial u^a v^b with a + b <= 4
    exactly (a! b! / (a + b + 2)!) and is not exact at degree 5."""
    worst4, worst5 = 0.0, 0.0
    for a in range(6):
        for b in range(6 - a):
            q = (ny.RULE_W * ny.RULE_UV[:, 0] ** a * ny.RULE_UV[:, 1] ** b).sum()
            e = abs(q - ny.factorial_moment(a, b))
            if a + b <= 4:
                worst4 = max(worst4, e)
            else:
                worst5 = max(worst5, e)
    assert worst4 < 1e-14
    assert worst5 > 1e-6
    # points strictly inside, three near the corners and three near the edges
    bary = np.column_stack([1 - ny.RULE_UV.sum(1), ny.RULE_UV])
    assert bary.min() > 0.05
    assert np.all(bary[:3].max(1) > 0.8) and np.all(np.sort(bary[3:], 1)[:, 1] > 0.4)


def test_lagrange_interpolates_quadratics():
    rng = np.random.default_rng(1)
    L = ny.lagrange(ny.RULE_UV[:, 0], ny.RULE_UV[:, 1])
    np.testing.assert_allclose(L, np.eye(6), atol=1e-13)
    c = rng.normal(size=6)
    u, v = rng.random(50) * 0.5, rng.random(50) * 0.5
    f = lambda u, v: ny.monomials(u, v) @ c
    interp = ny.lagrange(u, v) @ f(ny.RULE_UV[:, 0], ny.RULE_UV[:, 1])
    np.testing.assert_allclose(interp, f(u, v), atol=1e-12)


def test_shape_functions_reproduce_quadratic_maps():
    """Nodes sampled from a quadratic map f(u, v) give back f everywhere;
    the derivatives match f's."""
    rng = np.random.default_rng(2)
    C = rng.normal(size=(6, 3))
    f = lambda u, v: ny.monomials(u, v) @ C
    ref = np.array([[0, 0], [1, 0], [0, 1], [0.5, 0], [0.5, 0.5], [0, 0.5]])
    X = f(ref[:, 0], ref[:, 1])
    u, v = rng.random(20) * 0.5, rng.random(20) * 0.5
    x, jac = ny.map_points(X[None], u, v)
    np.testing.assert_allclose(x[0], f(u, v), atol=1e-12)
    fu = C[1] + 2 * u[:, None] * C[3] + v[:, None] * C[4]
    fv = C[2] + u[:, None] * C[4] + 2 * v[:, None] * C[5]
    np.testing.assert_allclose(jac[0], np.linalg.norm(np.cross(fu, fv), axis=1), rtol=1e-12)


def test_curved_sphere_area_converges_at_fourth_order():
    errs = []
    for s in (1, 2, 3):
        d = ny.discretise(*synth.curved_icosphere(s))
        errs.append(abs((d["w"] * d["jac"]).sum() - 4 * np.pi))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 1e-4 and np.all(orders > 3.5), (errs, orders)


def _flat_element(seed):
    a, b, c = np.random.default_rng(seed).normal(size=(3, 3))
    return a, b, c, np.array([a, b, c, (a + b) / 2, (b + c) / 2, (c + a) / 2])


@pytest.mark.parametrize("seed", [0, 3])
def test_self_rule_equals_flat_closed_form(seed):
    """At k = 0 on a flat element, sum_i of the self integrals is the
    integral of 1/(4 pi R) over the triangle in parameter units: the closed
    form divided by twice the area, at each of the six points."""
    a, b, c, X = _flat_element(seed)
    area2 = np.linalg.norm(np.cross(b - a, c - a))
    for j in range(6):
        p = ny.RULE_UV[j]
        x = ny.map_points(X[None], p[:1], p[1:])[0][0, 0]
        I = ny.element_integrals(0.0, x, X, *ny.duffy_at(p, 8, X)).sum()
        ref = bie.laplace_panel_analytic(x, a, b, c) / (4 * np.pi) / area2
        assert abs(I - ref) < 1e-8 * abs(ref), (j, I, ref)


def test_near_rule_equals_flat_closed_form():
    """Points beside an edge and above the element, k = 0.  The closest
    targets of a sphere mesh (corner points of the neighbour) sit about
    0.08 h from the shared edge."""
    a, b, c, X = _flat_element(1)
    area2 = np.linalg.norm(np.cross(b - a, c - a))
    nrm = np.cross(b - a, c - a)
    nrm /= np.linalg.norm(nrm)
    h = max(np.linalg.norm(b - a), np.linalg.norm(c - b), np.linalg.norm(a - c))
    out = np.cross(b - a, nrm)
    out /= np.linalg.norm(out)
    if out @ ((a + b) / 2 - (a + b + c) / 3) < 0:
        out = -out
    uv, wq = ny.subdivided(3, 8)
    for x in (0.3 * a + 0.7 * b + 0.05 * h * out, (a + b + c) / 3 + 0.1 * h * nrm):
        I = ny.element_integrals(0.0, x, X, uv, wq).sum()
        ref = bie.laplace_panel_analytic(x, a, b, c) / (4 * np.pi) / area2
        assert abs(I - ref) < 1e-6 * abs(ref)


def test_self_rule_converges_on_curved_elements():
    d = ny.discretise(*synth.curved_icosphere(2))
    Xe = d["X"][5]
    for j in range(6):
        vals = [ny.element_integrals(2.0, d["r"][30 + j], Xe, *ny.duffy_at(ny.RULE_UV[j], n, Xe))
                for n in (8, 14)]
        assert np.abs(vals[0] - vals[1]).max() < 1e-8 * np.abs(vals[1]).max()


def test_single_layer_of_constant_density_on_unit_sphere():
    """k -> 0: the single-layer potential of q = 1 on the unit sphere is 1 on
    the surface; with I = q * Jacobian every row of Z I approaches 1."""
    nodes, tri6 = synth.curved_icosphere(1)
    d = ny.discretise(nodes, tri6)
    y = ny.dense_matrix(1e-9, nodes, tri6) @ d["jac"]
    assert np.abs(y - 1).max() < 2e-3


def test_mie_accuracy_beats_flat_panels():
    """Sound-soft sphere, k = 2: u_s at r = 4 against the Mie series, and
    more than 10x better than flat centroid collocation with a comparable
    number of unknowns (subdivision 2: 320 panels vs 480 points)."""
    k = 2.0
    th = np.linspace(0, np.pi, 37)
    xobs = 4 * np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    ref = mie.scattered(k, 1.0, 4.0, th)
    nodes, tri6 = synth.curved_icosphere(1)
    I = np.linalg.solve(ny.dense_matrix(k, nodes, tri6), ny.plane_wave_rhs(k, nodes, tri6))
    e = np.linalg.norm(ny.scattered_field(k, nodes, tri6, I, xobs) - ref) / np.linalg.norm(ref)
    V, F = synth.icosphere(2)
    q = np.linalg.solve(bie.dense_matrix(k, V, F), bie.plane_wave_rhs(k, V, F))
    ef = np.linalg.norm(bie.scattered_field(k, V, F, q, xobs) - ref) / np.linalg.norm(ref)
    print("nystrom s=1", e, "flat s=2", ef)
    assert e < 3e-3 and e * 10 < ef


def test_dense_matrix_rows_subset():
    """The rows= form of the oracle's Nystrom matrix is the full matrix's
    rows, bit for bit (used for sampled rows at sizes the full matrix cannot
    reach)."""
    nodes, tri6 = synth.curved_icosphere(1)
    Z = ny.dense_matrix(3.0, nodes, tri6)
    rows = np.array([0, 5, 77, 400, 479])
    assert np.array_equal(ny.dense_matrix(3.0, nodes, tri6, rows=rows), Z[rows])
