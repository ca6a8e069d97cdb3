"""CPU tests of the native library: symbol exports, argument validation, and
exact equality of the C++ tree and traversal lists with the oracle's."""
import math
import os
import re

import numpy as np
import pytest

import synth
from oracle.tree import build_tree, dual_tree_traversal
from paper_1803_09948_amd import hfmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    L = hfmm.lib()
    hdr = open(os.path.join(ROOT, "include", "hfmm.h")).read()
    names = set(re.findall(r"\b(hfmm_[a-z_0-9]+)\s*\(", hdr))
    assert names, "no declarations parsed"
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(hfmm.EXPORTS) == names


@pytest.mark.parametrize("n,ncrit,seed,axes", [(4096, 64, 11, (1, 1, 1)), (3001, 17, 5, (0.6, 1.7, 1.1)),
                                                 (700, 64, 2, (1, 1, 1)), (1, 64, 3, (1, 1, 1))])
def test_tree_equals_oracle(n, ncrit, seed, axes):
    x = synth.scale_axes(synth.sphere_points(n, seed), axes)
    t = hfmm.Tree.from_points(x, ncrit=ncrit)
    sp, tp, cells = t.export()
    o = build_tree(x, None, ncrit)
    np.testing.assert_array_equal(sp, o.src_perm)
    np.testing.assert_array_equal(tp, o.tgt_perm)
    ref = np.stack([o.level, o.ijk[:, 0], o.ijk[:, 1], o.ijk[:, 2], o.sb, o.se, o.tb, o.te, o.cb, o.ce], 1)
    np.testing.assert_array_equal(cells, ref)
    st = t.stats()
    assert st["centre"] == list(o.c) and st["half"] == o.H


@pytest.mark.parametrize("n,k,P,theta", [(4096, 1.0, 8, 0.5), (2000, 16 * math.pi, 10, 0.5),
                                         (2500, 7.3, 6, 0.7)])
def test_lists_equal_oracle(n, k, P, theta):
    x = synth.sphere_points(n, 7)
    t = hfmm.Tree.from_points(x, ncrit=32, theta=theta)
    m2l, p2p = t.lists(k, P)
    o = build_tree(x, None, 32, split_side=0.4 * P / k)
    _, _, cells = t.export(k, P)
    ref = np.stack([o.level, o.ijk[:, 0], o.ijk[:, 1], o.ijk[:, 2], o.sb, o.se, o.tb, o.te, o.cb, o.ce], 1)
    np.testing.assert_array_equal(cells, ref)
    om2l, op2p = dual_tree_traversal(o, k, theta, 0.4 * P)
    assert sorted(map(tuple, m2l.tolist())) == sorted(om2l)
    assert sorted(map(tuple, p2p.tolist())) == sorted(op2p)
    # same visit order as well
    assert [tuple(v) for v in m2l.tolist()] == om2l


def test_invalid_arguments():
    x = synth.sphere_points(100, 1)
    with pytest.raises(hfmm.HfmmError) as e:
        hfmm.Tree.from_points(np.zeros((0, 3), np.float32))
    assert e.value.code == hfmm.HFMM_EINVAL
    with pytest.raises(hfmm.HfmmError):
        hfmm.Tree.from_points(x, ncrit=0)
    bad = x.copy()
    bad[3, 1] = np.nan
    with pytest.raises(hfmm.HfmmError):
        hfmm.Tree.from_points(bad)
    t = hfmm.Tree.from_points(x)
    for k, P in ((0.0, 8), (-1.0, 8), (float("inf"), 8), (1.0, 0), (1.0, 17)):
        with pytest.raises(hfmm.HfmmError) as e:
            t.prepare(k, P, stream=0)
        assert e.value.code == hfmm.HFMM_EINVAL


def test_bie_tree_equals_oracle():
    from oracle import bie
    V, T = synth.icosphere(3)
    t = hfmm.Tree.from_mesh(V, T, ncrit=32)
    pan = bie.panels(V, T)
    src, _ = bie.gauss_sources(pan)
    o = build_tree(src.astype(np.float32), pan["centroid"].astype(np.float32), 32)
    sp, tp, cells = t.export()
    np.testing.assert_array_equal(sp, o.src_perm)
    np.testing.assert_array_equal(tp, o.tgt_perm)
    ref = np.stack([o.level, o.ijk[:, 0], o.ijk[:, 1], o.ijk[:, 2], o.sb, o.se, o.tb, o.te, o.cb, o.ce], 1)
    np.testing.assert_array_equal(cells, ref)


def test_bie_invalid_mesh():
    V, T = synth.icosphere(1)
    bad = T.copy()
    bad[0, 0] = len(V)
    with pytest.raises(hfmm.HfmmError):
        hfmm.Tree.from_mesh(V, bad)
    deg = T.copy()
    deg[0] = [0, 0, 1]
    with pytest.raises(hfmm.HfmmError):
        hfmm.Tree.from_mesh(V, deg)


def test_nystrom_points_and_tree_equal_oracle():
    """Curved-element handle: the interpolation points, weights and
    Jacobians equal the oracle's discretisation; its tree over the points
    equals the oracle's tree."""
    from oracle import nystrom as ny
    nodes, tri6 = synth.curved_icosphere(2)
    t = hfmm.Tree.from_curved_mesh(nodes, tri6, ncrit=32)
    xyz, w, jac = t.nystrom_points()
    d = ny.discretise(nodes, tri6)
    np.testing.assert_allclose(xyz, d["r"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(w, d["w"], rtol=1e-14)
    np.testing.assert_allclose(jac, d["jac"], rtol=1e-13)
    pts = d["r"].astype(np.float32)
    o = build_tree(pts, pts, 32)
    sp, tp, cells = t.export()
    np.testing.assert_array_equal(sp, o.src_perm)
    np.testing.assert_array_equal(tp, o.tgt_perm)


def test_nystrom_invalid_mesh():
    nodes, tri6 = synth.curved_icosphere(1)
    bad = tri6.copy()
    bad[0, 4] = len(nodes)
    with pytest.raises(hfmm.HfmmError):
        hfmm.Tree.from_curved_mesh(nodes, bad)
    deg = tri6.copy()
    deg[0, :3] = deg[0, 0]
    with pytest.raises(hfmm.HfmmError):
        hfmm.Tree.from_curved_mesh(nodes, deg)
    V, T = synth.icosphere(1)
    with pytest.raises(hfmm.HfmmError):
        hfmm.Tree.from_mesh(V, T).nystrom_points()


def test_complex_wavenumber_lists_and_options():
    """k + i k_imag: cells and lists follow |k + i k_imag| exactly as the
    oracle's; negative or non-finite k_imag is refused on every handle."""
    from oracle.fmm import FMM
    x = synth.sphere_points(2500, 8)
    k, ki, P = 9.0, 4.0, 8
    t = hfmm.Tree.from_points(x, ncrit=32, k_imag=ki)
    m2l, p2p = t.lists(k, P)
    f = FMM(x, k=k, k_imag=ki, P=P, ncrit=32)
    assert sorted(map(tuple, m2l.tolist())) == sorted(f.m2l)
    assert sorted(map(tuple, p2p.tolist())) == sorted(f.p2p)
    # the rules see |k + i k_imag| only: the lists equal those of the real |k|
    m2l_abs, _ = hfmm.Tree.from_points(x, ncrit=32).lists(float(np.hypot(k, ki)), P)
    np.testing.assert_array_equal(m2l, m2l_abs)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(hfmm.HfmmError):
            hfmm.Tree.from_points(x, k_imag=bad)
    V, T = synth.icosphere(1)
    hfmm.Tree.from_mesh(V, T, k_imag=0.5).free()
    with pytest.raises(hfmm.HfmmError):
        hfmm.Tree.from_mesh(V, T, k_imag=-0.5)
    with pytest.raises(hfmm.HfmmError):
        hfmm.Tree.from_curved_mesh(*synth.curved_icosphere(1), k_imag=-0.5)


def test_host_plans_concurrent_equal_serial():
    """Host plans (lists, operators, M2L pair orders) of several handles built
    from a thread pool at once, each itself multi-threaded, have the same
    footprints and statistics as the same plans built one after another."""
    from concurrent.futures import ThreadPoolExecutor
    cases = [(1 << 14, 11, 30.0), (1 << 15, 12, 20.0), (20000, 13, 45.0), (1 << 14, 14, 8.0)]

    def plan(c):
        n, seed, k = c
        t = hfmm.Tree.from_points(synth.sphere_points(n, seed), ncrit=64)
        fp = t.prepare_host(k, 10)
        st = t.stats(k, 10)
        t.free()
        return fp, st["n_m2l"], st["n_tables"], st["p2p_body_pairs"]

    serial = [plan(c) for c in cases]
    with ThreadPoolExecutor(4) as ex:
        concurrent = list(ex.map(plan, cases))
    assert concurrent == serial


def test_tree_plan_counts_and_bytes():
    """hfmm_tree_plan (host only): its counts are those of the oracle's tree
    and traversal at (k, P), its bytes add up, M and L take 2 x cells x P^2
    complex64, the GMRES workspace grows with the restart, and bad arguments
    are refused."""
    x = synth.sphere_points(3000, 21)
    k, P = 9.0, 8
    t = hfmm.Tree.from_points(x, ncrit=32)
    pl = t.plan(k, P)
    o = build_tree(x, None, 32, split_side=0.4 * P / k)
    om2l, op2p = dual_tree_traversal(o, k, 0.5, 0.4 * P)
    assert pl["n_cell"] == len(o.level) and pl["n_leaf"] == int(np.sum(o.cb == o.ce))
    assert pl["n_m2l"] == len(om2l) and pl["n_p2p"] == len(op2p)
    npairs = sum(int((o.te[a] - o.tb[a]) * (o.se[b] - o.sb[b])) for a, b in op2p)
    assert pl["p2p_body_pairs"] == npairs
    assert pl["n_src"] == pl["n_tgt"] == 3000 and pl["resident"] == 0 and pl["bytes_gmres"] == 0
    parts = ("bytes_tree", "bytes_lists", "bytes_expansions", "bytes_corrections", "bytes_gmres")
    assert pl["bytes_total"] == sum(pl[p] for p in parts)
    assert pl["bytes_expansions"] >= 2 * pl["n_cell"] * P * P * 8
    assert pl["bytes_total"] == t.prepare_host(k, P)       # the footprint the device half allocates
    st = t.stats(k, P)
    assert (st["n_m2l"], st["n_tables"], st["p2p_body_pairs"]) == (pl["n_m2l"], pl["n_tables"],
                                                                   pl["p2p_body_pairs"])
    V, T = synth.icosphere(2)
    tb = hfmm.Tree.from_mesh(V, T)
    a, b = tb.plan(3.0, 6, restart=10), tb.plan(3.0, 6, restart=30)
    assert 0 < a["bytes_gmres"] < b["bytes_gmres"] and a["bytes_corrections"] > 0
    assert b["bytes_gmres"] >= 31 * len(T) * 16
    for args in ((0.0, 8, 0), (1.0, 0, 0), (1.0, 17, 0), (1.0, 8, 201)):
        with pytest.raises(hfmm.HfmmError) as e:
            hfmm._check(hfmm.lib().hfmm_tree_plan(t._h, args[0], args[1], args[2], hfmm.C.byref(hfmm.PlanInfo())))
        assert e.value.code == hfmm.HFMM_EINVAL
    with pytest.raises(hfmm.HfmmError):
        hfmm._check(hfmm.lib().hfmm_tree_plan(tb._h, 3.0, 6, 0, hfmm.C.byref(hfmm.PlanInfo())))


def test_binding_checks_device_vectors():
    """The binding refuses vectors of the wrong dtype, length or placement
    before any pointer reaches the library (no device needed)."""
    torch = pytest.importorskip("torch")
    t = hfmm.Tree.from_points(synth.sphere_points(64, 2))
    with pytest.raises((TypeError, ValueError)):
        t.matvec(1.0, 4, torch.zeros(64, dtype=torch.complex64))           # host tensor
    with pytest.raises((TypeError, ValueError)):
        hfmm._dev_vec(torch.zeros(64, dtype=torch.complex128), torch.complex64, 64, "x")
    with pytest.raises((TypeError, ValueError)):
        hfmm.batch_matvec([t], [1.0], [4], [torch.zeros(63, dtype=torch.complex64)],
                          [torch.zeros(64, dtype=torch.complex64)])
    with pytest.raises(hfmm.HfmmError):
        hfmm.debug_fail_alloc(-2)
    hfmm.debug_fail_alloc(-1)
