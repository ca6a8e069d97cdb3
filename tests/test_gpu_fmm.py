"""GPU parity of the point-mode FMM matvec against the FP64 oracle.

Bar (stated for FP32 arithmetic): relative 2-norm difference to the CPU FP64
FMM at the same tree, lists and P <= 1e-5, and every element within 1e-5 of
the largest output (relative infinity norm); the FMM truncation error
against the FP64 direct sum is reported and bounded loosely."""
import math

import numpy as np
import pytest

import synth
from oracle.fmm import FMM, direct_sum

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1803_09948_amd import hfmm  # noqa: E402
from parity import check, rel  # noqa: E402


def _gpu_matvec(x, q, k, P, **opts):
    t = hfmm.Tree.from_points(x, **opts)
    qd = torch.from_numpy(q).to("cuda")
    y = t.matvec(k, P, qd)
    torch.cuda.synchronize()
    return y.cpu().numpy(), t


@pytest.mark.parametrize("n,k,P,ncrit,seed", [
    (4096, 1.0, 8, 64, 11),        # plain matvec workload
    (4097, 1.0, 8, 64, 12),        # ragged
    (3000, 9.0, 10, 32, 13),       # higher frequency, kappa active
    (2000, 2.0, 1, 32, 14),        # P = 1
])
def test_matvec_vs_oracle_fmm(n, k, P, ncrit, seed):
    x = synth.sphere_points(n, seed)
    q = synth.strengths(n, seed)
    print(f"case n={n} k={k} P={P} ncrit={ncrit}", flush=True)
    y, t = _gpu_matvec(x, q, k, P, ncrit=ncrit)
    f = FMM(x, k=k, P=P, ncrit=ncrit)
    yo = f.matvec(q)
    ed = rel(yo, direct_sum(k, x, x, q))
    print(f"  oracle FMM vs direct {ed:.3e}")
    check(y, yo, 1e-5, "gpu vs oracle FMM")


@pytest.mark.parametrize("P", [3, 5, 6, 7, 9])
def test_orders_vs_oracle_fmm(P):
    """Orders whose P^2 leaves 1, 4 or 9 rows past a multiple of 16 (the last
    16-row tile of the matrix-core M2L is partly padding), against the
    oracle FMM."""
    n, k = 1500, 4.0
    x = synth.sphere_points(n, 40 + P)
    q = synth.strengths(n, 40 + P)
    y, t = _gpu_matvec(x, q, k, P, ncrit=32)
    assert t.stats(k, P)["n_m2l"] > 0
    check(y, FMM(x, k=k, P=P, ncrit=32).matvec(q), 1e-5, f"P={P} gpu vs oracle FMM")


@pytest.mark.parametrize("P", [11, 13, 14, 15])
def test_high_orders_vs_direct_sum(P):
    """High orders (remainder rows 9, 9, 4, 1): the truncation error is far
    below FP32 rounding, so the direct sum is the reference."""
    n, k = 1500, 3.0
    x = synth.sphere_points(n, 50 + P)
    q = synth.strengths(n, 50 + P)
    y, t = _gpu_matvec(x, q, k, P, ncrit=32)
    assert t.stats(k, P)["n_m2l"] > 0
    check(y, direct_sum(k, x, x, q), 1e-5, f"P={P} vs direct")


def test_largest_P_vs_direct_sum():
    """P = 16 (the largest order): truncation error is far below FP32 rounding."""
    n, k = 1500, 3.0
    x = synth.sphere_points(n, 15)
    q = synth.strengths(n, 15)
    y, _ = _gpu_matvec(x, q, k, 16, ncrit=32)
    check(y, direct_sum(k, x, x, q), 1e-5, "P=16 vs direct")


def test_p2p_only_equals_direct_sum():
    """theta -> 0: the traversal accepts nothing, so the GPU result is the
    FP32 direct sum of Listing 1 over all pairs."""
    n = 3000
    x = synth.sphere_points(n, 21)
    q = synth.strengths(n, 21)
    y, t = _gpu_matvec(x, q, 5.0, 4, ncrit=40, theta=1e-9)
    assert t.stats(5.0, 4)["n_m2l"] == 0
    check(y, direct_sum(5.0, x, x, q), 2e-6, "p2p only vs direct", barinf=5e-6)


def test_edge_cases():
    # one point: nothing to sum
    y, _ = _gpu_matvec(synth.sphere_points(1, 1), np.array([1 + 1j], np.complex64), 1.0, 4)
    assert y.shape == (1,) and y[0] == 0
    # fewer points than ncrit: a single leaf, direct sum
    x = synth.sphere_points(40, 2)
    q = synth.strengths(40, 2)
    y, _ = _gpu_matvec(x, q, 2.0, 6)
    check(y, direct_sum(2.0, x, x, q), 2e-6, "one leaf vs direct", barinf=5e-6)
    # duplicated points contribute nothing to each other
    x = np.repeat(synth.sphere_points(300, 3), 2, axis=0)
    q = synth.strengths(600, 3)
    y, _ = _gpu_matvec(x, q, 2.0, 6, ncrit=16)
    yo = FMM(x, k=2.0, P=6, ncrit=16).matvec(q)
    check(y, yo, 1e-5, "duplicates vs oracle FMM")
    # ellipsoid, non-unit root cube
    x = synth.scale_axes(synth.sphere_points(2500, 4), (0.5, 2.0, 1.3))
    q = synth.strengths(2500, 4)
    y, _ = _gpu_matvec(x, q, 3.0, 8, ncrit=32)
    check(y, FMM(x, k=3.0, P=8, ncrit=32).matvec(q), 1e-5, "ellipsoid vs oracle FMM")


def test_repeat_and_determinism_of_near_field():
    x = synth.sphere_points(4096, 11)
    q = synth.strengths(4096, 11)
    t = hfmm.Tree.from_points(x)
    qd = torch.from_numpy(q).to("cuda")
    y1 = t.matvec(1.0, 8, qd).cpu().numpy()
    y2 = t.matvec(1.0, 8, qd).cpu().numpy()
    np.testing.assert_array_equal(y1, y2)   # fixed accumulation order: the same bits


@pytest.mark.parametrize("P", [4, 8, 10, 12])
def test_m2l_launch_shapes_bit_identical(P):
    """Every launch shape of the matrix-core M2L gives the same bits, and the
    autotuner reports the shape it chose."""
    n, k = 20000, 12.0
    x = synth.sphere_points(n, 31)
    q = torch.from_numpy(synth.strengths(n, 31)).to("cuda")
    nv = hfmm.variant_count(P)
    assert nv >= 1
    t = hfmm.Tree.from_points(x)
    outs = []
    try:
        for v in range(nv):
            hfmm.set_variant(v)
            outs.append(t.matvec(k, P, q).cpu().numpy())
            assert t.variant(k, P) == v
    finally:
        hfmm.set_variant(-1)
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    t2 = hfmm.Tree.from_points(x)
    y = t2.matvec(k, P, q).cpu().numpy()
    assert 0 <= t2.variant(k, P) < nv
    np.testing.assert_array_equal(y, outs[0])


def test_p2p_launch_shapes_bit_identical():
    """Every variant of the P2P (waves per block, source stages per LDS tile,
    and where it forks off beside the far field) gives the same bits, for a
    point handle with leaves of ragged sizes, a damped one and a BIE handle;
    the autotuner reports the variant used."""
    n, k, P = 20000, 12.0, 8
    x = synth.sphere_points(n, 32)
    q = torch.from_numpy(synth.strengths(n, 32)).to("cuda")
    nv = hfmm.variant_count(P, hfmm.PHASE_P2P)
    assert nv >= 2
    V, T = synth.icosphere(4)
    qb = torch.from_numpy(synth.strengths(len(T), 34)).to("cuda")
    cases = [(hfmm.Tree.from_points(x, ncrit=48), k, q), (hfmm.Tree.from_points(x, k_imag=0.5), k, q),
             (hfmm.Tree.from_mesh(V, T), 6.0, qb)]
    for t, kk, qq in cases:
        outs = []
        try:
            for v in range(nv):
                hfmm.set_variant(v, hfmm.PHASE_P2P)
                outs.append(t.matvec(kk, P, qq).cpu().numpy())
                assert t.variant(kk, P, hfmm.PHASE_P2P) == v
        finally:
            hfmm.set_variant(-1, hfmm.PHASE_P2P)
        for v, o in enumerate(outs[1:], 1):
            np.testing.assert_array_equal(o, outs[0], err_msg=f"P2P variant {v}")
    t2 = hfmm.Tree.from_points(x, ncrit=48)
    y = t2.matvec(k, P, q).cpu().numpy()
    assert 0 <= t2.variant(k, P, hfmm.PHASE_P2P) < nv
    assert np.array_equal(y, hfmm.Tree.from_points(x, ncrit=48).matvec(k, P, q).cpu().numpy())


def test_m2l_staging_segments_bit_identical():
    """A staging budget far below the M2L's needs splits the M2L and its
    reduction into many target segments; results are the same bits."""
    n, k, P = 20000, 12.0, 8
    x = synth.sphere_points(n, 33)
    q = torch.from_numpy(synth.strengths(n, 33)).to("cuda")
    y1 = hfmm.Tree.from_points(x).matvec(k, P, q).cpu().numpy()
    y2 = hfmm.Tree.from_points(x, stage_mb=1).matvec(k, P, q).cpu().numpy()
    np.testing.assert_array_equal(y1, y2)


def test_overlapped_and_serial_sequences_bit_identical():
    """The near field (P2P) runs on a second stream beside the far field, and
    L2P adds the far field after it; with phase timing on, every phase runs
    on one stream in the same order.  Both give the same bits, for a point
    handle and for a BIE handle."""
    n, k, P = 30000, 12.0, 10
    x = synth.sphere_points(n, 41)
    q = torch.from_numpy(synth.strengths(n, 41)).to("cuda")
    t = hfmm.Tree.from_points(x, ncrit=32)
    y0 = t.matvec(k, P, q).cpu().numpy()
    t.set_timing(True)
    y1 = t.matvec(k, P, q).cpu().numpy()
    t.set_timing(False)
    y2 = t.matvec(k, P, q).cpu().numpy()
    assert np.array_equal(y0, y1) and np.array_equal(y0, y2)
    V, T = synth.icosphere(4)
    b = hfmm.Tree.from_mesh(V, T)
    qb = torch.from_numpy(synth.strengths(len(T), 42)).to("cuda")
    z0 = b.matvec(6.0, P, qb).cpu().numpy()
    b.set_timing(True)
    z1 = b.matvec(6.0, P, qb).cpu().numpy()
    assert np.array_equal(z0, z1)


def test_autotune_cache_file(tmp_path):
    """HFMM_TUNE_CACHE: a first process times the M2L and P2P shapes and
    appends its choices to the file (one line per phase); a later process
    takes the shapes from the file without timing (shown by editing the
    file to other valid shapes)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = str(tmp_path / "tune.txt")
    prog = ("import sys; sys.path.insert(0, %r)\n"
            "import torch, synth\n"
            "from paper_1803_09948_amd import hfmm\n"
            "x = synth.sphere_points(20000, 31)\n"
            "q = torch.from_numpy(synth.strengths(20000, 31)).cuda()\n"
            "t = hfmm.Tree.from_points(x)\n"
            "t.matvec(12.0, 10, q)\n"
            "print('variant', t.variant(12.0, 10, 0), t.variant(12.0, 10, 1))\n") % root
    env = dict(os.environ, HFMM_TUNE_CACHE=cache)

    def run():
        r = subprocess.run([sys.executable, "-c", prog], capture_output=True, text=True, env=env, timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        return tuple(int(v) for v in r.stdout.split("variant")[-1].split())

    v1 = run()
    rows = [ln.split() for ln in open(cache).read().splitlines()]
    assert sorted(int(r[0]) for r in rows) == [0, 1]
    byph = {int(r[0]): r for r in rows}
    for ph in (0, 1):
        assert len(byph[ph]) == 4 and int(byph[ph][1]) == 10 and int(byph[ph][3]) == v1[ph]
    other = tuple((v1[ph] + 1) % hfmm.variant_count(10, ph) for ph in (0, 1))
    text = "".join(f"{ph} {byph[ph][1]} {byph[ph][2]} {other[ph]}\n" for ph in (0, 1))
    open(cache, "w").write(text)
    assert run() == other
    assert open(cache).read() == text   # nothing re-timed
