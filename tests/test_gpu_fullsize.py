"""Parity at the full benchmark sizes, in the configuration the benchmark
times (default options, autotuned M2L launch shape), on outputs the FP64
oracle computes one by one: sampled targets of the 1M-point product against
the direct sum, and sampled rows of the flat-panel and curved Nystrom BIE
products against the oracle's matrix rows."""
import math

import numpy as np
import pytest

import synth
from oracle import bie
from oracle import nystrom as ny
from oracle.fmm import direct_sum

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1803_09948_amd import hfmm  # noqa: E402
from parity import check  # noqa: E402


def test_headline_1m_sampled_vs_direct_sum():
    """N = 2^20 on the unit sphere, k = 16 pi, P = 10, ncrit 64 (the
    benchmark's inputs and options): 32 sampled outputs against the FP64
    direct sum over all 1M sources.  The difference is the P = 10 truncation
    (measured 7e-7 over 200 samples); bound 5e-6."""
    n, k, P = 1 << 20, 16 * math.pi, 10
    print(f"case headline n={n} k={k:.4f} P={P}", flush=True)
    x = synth.sphere_points(n, 23)
    q = synth.strengths(n, 23)
    t = hfmm.Tree.from_points(x, ncrit=64)
    y = t.matvec(k, P, torch.from_numpy(q).to("cuda")).cpu().numpy()
    idx = np.sort(np.random.default_rng(3).choice(n, 32, replace=False))
    ref = direct_sum(k, x[idx], x, q, chunk=4)
    print("  stats", t.stats(k, P))
    check(y[idx], ref, 5e-6, "sampled vs direct")


def test_8m_sampled_vs_direct_sum():
    """N = 2^23 on the unit sphere, k = 16 pi, P = 10 (the larger size of
    the precision study): 24 sampled outputs against the FP64 direct sum
    over all 8M sources.  The measured P = 10 error over 1000 targets is
    8.7e-7; bound 5e-6."""
    n, k, P = 1 << 23, 16 * math.pi, 10
    print(f"case n={n} k={k:.4f} P={P}", flush=True)
    x = synth.sphere_points(n, 29)
    q = synth.strengths(n, 29)
    t = hfmm.Tree.from_points(x, ncrit=64)
    y = t.matvec(k, P, torch.from_numpy(q).to("cuda")).cpu().numpy()
    idx = np.sort(np.random.default_rng(6).choice(n, 24, replace=False))
    ref = direct_sum(k, x[idx], x, q, chunk=2)
    print("  stats", t.stats(k, P), flush=True)
    check(y[idx], ref, 5e-6, "8M sampled vs direct")
    t.free()


def test_bie_icosphere5_sampled_rows():
    """Flat-panel BIE at the benchmark size (icosphere s = 5, 20,480 panels,
    k = 2 pi, P = 10): 32 sampled rows of the product against the oracle's
    dense rows."""
    k = 2 * math.pi
    V, T = synth.icosphere(5)
    print(f"case bie s=5 panels={len(T)} k={k:.4f}", flush=True)
    t = hfmm.Tree.from_mesh(V, T)
    q = synth.strengths(len(T), 91)
    y = t.matvec(k, 10, torch.from_numpy(q).to("cuda")).cpu().numpy()
    rows = np.sort(np.random.default_rng(4).choice(len(T), 32, replace=False))
    check(y[rows], bie.dense_matrix(k, V, T, rows=rows) @ q.astype(np.complex128), 1e-5, "sampled rows vs dense")


def test_nystrom_s5_sampled_rows():
    """Curved Nystrom at the benchmark size (s = 5, 122,880 unknowns, k = 2 pi,
    P = 10): 32 sampled rows against the oracle's matrix rows (the oracle at
    its own, finer quadrature orders)."""
    k = 2 * math.pi
    nodes, tri6 = synth.curved_icosphere(5)
    n = 6 * len(tri6)
    print(f"case nystrom s=5 unknowns={n} k={k:.4f}", flush=True)
    t = hfmm.Tree.from_curved_mesh(nodes, tri6)
    rng = np.random.default_rng(8)
    x = (rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)).astype(np.complex64)
    y = t.matvec(k, 10, torch.from_numpy(x).to("cuda")).cpu().numpy()
    rows = np.sort(rng.choice(n, 32, replace=False))
    check(y[rows], ny.dense_matrix(k, nodes, tri6, rows=rows) @ x.astype(np.complex128), 1e-5,
          "sampled rows vs oracle")
