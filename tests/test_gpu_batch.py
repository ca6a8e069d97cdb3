"""Batched (fused, graph-replayed) matvecs over uneven instances: each result
must equal the same instance computed alone bit for bit (every accumulation
has a fixed order), and the smallest ones the FP64 oracle FMM."""
import os

import numpy as np
import pytest

import synth
from oracle.fmm import FMM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1803_09948_amd import hfmm  # noqa: E402
from parity import check  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch64_smallest4.npz")


def test_batch_matches_alone_and_oracle():
    inst = synth.batch_instances(count=10, nmin=1024, nmax=8192, seed=99)
    trees = [hfmm.Tree.from_points(d["points"]) for d in inst]
    ks = [d["k"] for d in inst]
    P = 10
    xs = [torch.from_numpy(d["q"]).to("cuda") for d in inst]
    ys = [torch.empty_like(x) for x in xs]
    alone = [t.matvec(k, P, x).cpu().numpy() for t, k, x in zip(trees, ks, xs)]
    for rep in range(3):
        # different inputs on each replay, with eager work in between
        scale = [complex(1 + rep, -rep) for _ in inst]
        xr = [x * s for x, s in zip(xs, scale)]
        hfmm.batch_matvec(trees, ks, [P] * len(trees), xr, ys)
        torch.cuda.synchronize()
        _ = trees[0].matvec(ks[0], P, xr[0])
        torch.cuda.synchronize()
        for i, (y, x) in enumerate(zip(ys, xr)):
            a = trees[i].matvec(ks[i], P, x).cpu().numpy()
            np.testing.assert_array_equal(y.cpu().numpy(), a, err_msg=f"replay {rep} instance {i}")
    order = np.argsort([d["n"] for d in inst])[:2]
    for i in order:
        d = inst[i]
        yo = FMM(d["points"], k=d["k"], P=P).matvec(d["q"])
        check(ys[i].cpu().numpy() / complex(3, -2), yo, 1e-5, f"instance {i} n {d['n']} k {d['k']:.2f} vs oracle")


def test_batch_forced_shapes_recapture_same_bits():
    """Forcing any M2L or P2P launch shape on a graph-replayed batch
    re-captures its graph with that shape; every shape gives the same bits
    as the autotuned batch."""
    inst = synth.batch_instances(count=6, nmin=2048, nmax=16384, seed=7)
    trees = [hfmm.Tree.from_points(d["points"]) for d in inst]
    ks = [d["k"] for d in inst]
    P = 10
    xs = [torch.from_numpy(d["q"]).to("cuda") for d in inst]
    ys = [torch.empty_like(x) for x in xs]
    hfmm.batch_matvec(trees, ks, [P] * len(trees), xs, ys)
    torch.cuda.synchronize()
    ref = [y.cpu().numpy() for y in ys]
    for phase in (hfmm.PHASE_M2L, hfmm.PHASE_P2P):
        try:
            for v in range(hfmm.variant_count(P, phase)):
                hfmm.set_variant(v, phase)
                for y in ys:
                    y.zero_()
                hfmm.batch_matvec(trees, ks, [P] * len(trees), xs, ys)
                torch.cuda.synchronize()
                for i, y in enumerate(ys):
                    np.testing.assert_array_equal(y.cpu().numpy(), ref[i], err_msg=f"phase {phase} shape {v} "
                                                                                     f"instance {i}")
        finally:
            hfmm.set_variant(-1, phase)


def test_batch64_full_workload():
    """The batched workload at its full size: 64 instances (N log-uniform in
    [2048, 65536], k uniform in [1, 20], spheres and ellipsoids alternating,
    P = 10) in one fused, graph-replayed sequence.  Every result is bitwise
    the instance's product alone, and the four smallest are within 1e-5 of
    the oracle FMM (its products stored by tests/golden/make_batch64_oracle.py)."""
    inst = synth.batch_instances()
    P = 10
    g = np.load(GOLDEN, allow_pickle=False)
    assert int(g["P"]) == P
    trees = [hfmm.Tree.from_points(d["points"]) for d in inst]
    ks = [d["k"] for d in inst]
    xs = [torch.from_numpy(d["q"]).to("cuda") for d in inst]
    ys = [torch.empty_like(x) for x in xs]
    for rep in range(2):
        hfmm.batch_matvec(trees, ks, [P] * 64, xs, ys)
        torch.cuda.synchronize()
    print("total points", sum(d["n"] for d in inst), flush=True)
    for i in range(64):
        a = trees[i].matvec(ks[i], P, xs[i]).cpu().numpy()
        np.testing.assert_array_equal(ys[i].cpu().numpy(), a, err_msg=f"instance {i}")
    for i in g["index"]:
        d = inst[int(i)]
        check(ys[int(i)].cpu().numpy(), g[f"y{int(i)}"], 1e-5,
              f"instance {int(i)} n {d['n']} k {d['k']:.2f} vs oracle FMM")


def test_batch_argument_errors():
    a = hfmm.Tree.from_points(synth.sphere_points(500, 1))
    b = hfmm.Tree.from_points(synth.sphere_points(700, 2))
    xa = torch.ones(500, dtype=torch.complex64, device="cuda")
    xb = torch.ones(700, dtype=torch.complex64, device="cuda")
    with pytest.raises(hfmm.HfmmError):
        hfmm.batch_matvec([a, b], [1.0, 2.0], [8, 10], [xa, xb], [xa.clone(), xb.clone()])
    V, T = synth.icosphere(1)
    m = hfmm.Tree.from_mesh(V, T)
    xm = torch.ones(len(T), dtype=torch.complex64, device="cuda")
    with pytest.raises(hfmm.HfmmError):
        hfmm.batch_matvec([a, m], [1.0, 1.0], [8, 8], [xa, xm], [xa.clone(), xm.clone()])


def test_batch_refuses_segmented_instances():
    """An instance whose M2L staging is split into segments runs alone, not
    inside a fused batch."""
    a = hfmm.Tree.from_points(synth.sphere_points(20000, 5), stage_mb=1)
    b = hfmm.Tree.from_points(synth.sphere_points(3000, 6))
    xa = torch.ones(20000, dtype=torch.complex64, device="cuda")
    xb = torch.ones(3000, dtype=torch.complex64, device="cuda")
    with pytest.raises(hfmm.HfmmError):
        hfmm.batch_matvec([a, b], [12.0, 12.0], [8, 8], [xa, xb], [xa.clone(), xb.clone()])
    ya = a.matvec(12.0, 8, xa)  # alone it runs
    assert torch.isfinite(torch.view_as_real(ya)).all()
