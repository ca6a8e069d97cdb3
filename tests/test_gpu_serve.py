"""Continuous-batching server: every served solution equals the same request
solved alone by the plain GMRES path to within the GMRES tolerance (the
fused M2L adds in a different FP32 order; GMRES carries that rounding
through its iterations, and both solutions meet the residual bound),
admission respects the device-memory budget, and a solve that can never fit
is refused."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1803_09948_amd import hfmm, serve  # noqa: E402


def _trace(n, seed, subdivs=(2, 3), rate=200.0):
    return synth.serve_trace(nreq=n, rate=rate, seed=seed, subdivs=subdivs, kmin=1.0, kmax=8.0)


def test_served_equals_alone():
    tr = _trace(8, 5)
    st, xs = serve.serve(tr, keep_solutions=True, max_active=8)
    sp, xp = serve.serve_plain(tr, keep_solutions=True)
    print("served", st)
    print("plain ", sp)
    assert st["not_converged"] == 0 and sp["not_converged"] == 0
    assert st["peak_active"] >= 2          # solves really overlapped on the device
    for rid in xp:
        a, b = xs[rid], xp[rid]
        e = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        assert e <= 1e-4, (rid, e)


def test_admission_by_memory_budget():
    reqs = [dict(id=i, t_arrival=0.0, subdiv=3, axes=(1.0, 1.0, 1.0), k=4.0) for i in range(4)]
    V, T = synth.icosphere(3)
    t = hfmm.Tree.from_mesh(V, T)
    fp = t.prepare_host(4.0, 10)
    ws = (31 * len(T) + 8 * len(T)) * 16
    budget = int(1.5 * (fp + ws))
    st = serve.serve(reqs, max_active=8, hbm_budget=budget)
    print("budgeted", st)
    assert st["not_converged"] == 0 and st["n"] == 4
    assert st["peak_active"] == 1
    srv = hfmm.Server(hbm_budget_bytes=fp // 2, max_active=4)
    b = t.plane_wave(4.0)
    x = torch.zeros_like(b)
    with pytest.raises(hfmm.HfmmError) as e:
        srv.submit(t, 4.0, 10, b, x)
    assert e.value.code == hfmm.HFMM_ENOMEM
