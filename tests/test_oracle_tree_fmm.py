"""Pins for oracle.tree and oracle.fmm: direct-sum closed forms, reciprocity,
the Laplace limit, a Helmholtz finite-difference residual, the covering
invariant of the traversal lists, and FMM error falling with P."""
import math

import numpy as np
import pytest

import synth
from oracle.fmm import FMM, direct_sum, green
from oracle.tree import build_tree, dual_tree_traversal, morton_keys, root_cube


def test_two_point_closed_form():
    k = 3.0
    x = np.array([[0.0, 0.0, 0.0], [0.0, 0.6, 0.8]])
    q = np.array([1.0 + 0.5j, -0.25j])
    y = direct_sum(k, x, x, q)
    g = math.e ** (1j * k * 1.0) / (4 * math.pi)
    assert abs(y[0] - q[1] * g) < 1e-15 and abs(y[1] - q[0] * g) < 1e-15


def test_duplicates_contribute_nothing():
    x = np.array([[0.1, 0.2, 0.3]] * 3 + [[1.0, 0.0, 0.0]])
    q = np.ones(4)
    y = direct_sum(1.0, x, x, q)
    assert abs(y[0] - green(1.0, x[0], x[3])) < 1e-15


def test_reciprocity_complex_symmetric():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(200, 3))
    u = rng.normal(size=200) + 1j * rng.normal(size=200)
    v = rng.normal(size=200) + 1j * rng.normal(size=200)
    Av = direct_sum(2.0, x, x, v)
    Au = direct_sum(2.0, x, x, u)
    assert abs(u @ Av - v @ Au) < 1e-11 * abs(u @ Av)


def test_laplace_limit():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(50, 3))
    q = rng.normal(size=50)
    y = direct_sum(1e-9, x, x, q)
    d = np.linalg.norm(x[:, None] - x[None], axis=-1)
    np.fill_diagonal(d, np.inf)
    ref = (q[None] / (4 * np.pi * d)).sum(axis=1)
    np.testing.assert_allclose(y.real, ref, rtol=1e-12)


def test_helmholtz_fd_residual():
    """The field of the sources satisfies lap u + k^2 u = 0 away from them."""
    k = 4.0
    rng = np.random.default_rng(2)
    src = rng.normal(size=(20, 3)) * 0.3
    q = rng.normal(size=20) + 1j * rng.normal(size=20)
    x0 = np.array([1.5, 0.2, -0.4])
    h = 1e-3
    u = lambda x: direct_sum(k, x[None], src, q)[0]
    lap = sum(u(x0 + h * e) + u(x0 - h * e) - 2 * u(x0) for e in np.eye(3)) / h ** 2
    assert abs(lap + k * k * u(x0)) < 1e-5 * abs(k * k * u(x0))


def test_root_cube_unit_sphere():
    x = synth.sphere_points(5000, 3)
    c, H = root_cube(x)
    assert np.all(c == 0.0) and H == 1.0


def test_keys_and_cells_consistent():
    x = synth.sphere_points(3000, 4)
    t = build_tree(x, None, 32)
    assert np.all(np.diff(t.src_keys) >= 0)
    leaf = t.cb == t.ce
    assert np.all((t.se - t.sb)[leaf] <= 32)
    # every body lies inside its leaf's box
    xs = x[t.src_perm].astype(np.float64)
    for i in np.flatnonzero(leaf):
        cen, h = t.centre(i), t.half(i)
        pts = xs[t.sb[i]:t.se[i]]
        assert np.all(np.abs(pts - cen) <= h)
    # cells are level-ordered and children ranges are contiguous
    assert np.all(np.diff(t.level) >= 0)


@pytest.mark.parametrize("k,kappa", [(1.0, 3.2), (12.0, 4.0)])
def test_every_pair_covered_once(k, kappa):
    """P2P pairs plus M2L pairs of all ancestors cover every (target, source)
    body pair exactly once (brute force on a small cloud)."""
    x = synth.sphere_points(600, 5)
    t = build_tree(x, None, 8)
    m2l, p2p = dual_tree_traversal(t, k, 0.5, kappa)
    n = len(x)
    cover = np.zeros((n, n), np.int64)
    for a, b in p2p + m2l:
        cover[t.tb[a]:t.te[a], t.sb[b]:t.se[b]] += 1
    assert np.all(cover == 1)
    assert len(m2l) > 0


def test_mac_never_accepting_gives_direct_sum():
    x = synth.sphere_points(700, 6)
    q = synth.strengths(700, 6)
    f = FMM(x, k=2.0, P=4, ncrit=16, theta=1e-9)
    assert len(f.m2l) == 0
    ref = direct_sum(2.0, x, x, q)
    np.testing.assert_allclose(f.matvec(q), ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_bie_mode_tree_targets_ride_along():
    V, T = synth.icosphere(2)
    from oracle import bie
    pan = bie.panels(V, T)
    src, _ = bie.gauss_sources(pan)
    t = build_tree(src.astype(np.float32), pan["centroid"].astype(np.float32), 24)
    leaf = t.cb == t.ce
    assert np.all((t.se - t.sb)[leaf] <= 24)
    assert (t.te - t.tb)[0] == len(T) and (t.se - t.sb)[0] == 3 * len(T)


def test_fmm_error_falls_with_P():
    x = synth.sphere_points(1500, 7)
    q = synth.strengths(1500, 7)
    ref = direct_sum(3.0, x, x, q)
    errs = []
    for P in (3, 5, 7, 9):
        f = FMM(x, k=3.0, P=P, ncrit=32)
        errs.append(np.linalg.norm(f.matvec(q) - ref) / np.linalg.norm(ref))
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[-1] < 1e-6


def test_complex_wavenumber_fd_residual_and_fmm():
    """k = 3 + 1i: the direct sum solves lap u + k^2 u = 0 away from the
    sources, and the FMM (tree rules on |k|) converges to it with P."""
    k = 3.0 + 1.0j
    rng = np.random.default_rng(2)
    src = rng.normal(size=(20, 3)) * 0.3
    q0 = rng.normal(size=20) + 1j * rng.normal(size=20)
    x0 = np.array([1.5, 0.2, -0.4])
    h = 1e-3
    u = lambda x: direct_sum(k, x[None], src, q0)[0]
    lap = sum(u(x0 + h * e) + u(x0 - h * e) - 2 * u(x0) for e in np.eye(3)) / h ** 2
    assert abs(lap + k * k * u(x0)) < 1e-5 * abs(k * k * u(x0))
    x = synth.sphere_points(1200, 9)
    q = synth.strengths(1200, 9)
    ref = direct_sum(k, x, x, q)
    errs = []
    for P in (3, 5, 7, 9):
        f = FMM(x, k=3.0, k_imag=1.0, P=P, ncrit=32)
        errs.append(np.linalg.norm(f.matvec(q) - ref) / np.linalg.norm(ref))
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[-1] < 1e-6
