"""Continuous-batching server: every served solution equals the same request
solved alone by the plain GMRES path bit for bit (the fused product and the
FP64 Arnoldi work run the same operations in the same order), admission
respects the device-memory budget, and a solve that can never fit is
refused."""
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
        np.testing.assert_array_equal(xs[rid], xp[rid], err_msg=f"request {rid}")


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


def test_served_mix_of_flat_and_curved_handles():
    """Flat-panel and curved-element (Nystrom) handles in one served mix:
    every solution is bitwise the handle's own plain GMRES solution."""
    flat = [hfmm.Tree.from_mesh(*synth.icosphere(2)), hfmm.Tree.from_mesh(*synth.icosphere(3))]
    curved = [hfmm.Tree.from_curved_mesh(*synth.curved_icosphere(1)),
              hfmm.Tree.from_curved_mesh(*synth.curved_icosphere(2))]
    trees = flat + curved
    ks = [3.0, 4.5, 2.0, 6.0]
    bs = [t.plane_wave(k) for t, k in zip(trees, ks)]
    alone = [t.gmres(k, 10, b, tol=1e-5)[0].cpu().numpy() for t, k, b in zip(trees, ks, bs)]
    srv = hfmm.Server(max_active=4)
    xs = [torch.zeros_like(b) for b in bs]
    tickets = [srv.submit(t, k, 10, b, x, tol=1e-5)[0] for t, k, b, x in zip(trees, ks, bs, xs)]
    for _ in range(100000):
        na, nq = srv.step()
        if na == 0 and nq == 0:
            break
    torch.cuda.synchronize()
    for i, tk in enumerate(tickets):
        state, info, _ = srv.poll(tk)
        print("request", i, "state", state, "iters", info["iters"])
        assert state == hfmm.Server.CONVERGED
        np.testing.assert_array_equal(xs[i].cpu().numpy(), alone[i], err_msg=f"request {i}")
    srv.free()
