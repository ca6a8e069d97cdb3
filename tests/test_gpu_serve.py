"""Continuous-batching server: every served solution equals the same request
solved alone by the plain GMRES path bit for bit (the fused product and the
FP64 Arnoldi work run the same operations in the same order), served
solutions solve the oracle's dense system, admission respects the
device-memory budget, a solve that can never fit is refused, and the
early-stop policy ends stagnating solves."""
import numpy as np
import pytest

import synth
from oracle import bie

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1803_09948_amd import hfmm, serve  # noqa: E402
from parity import dense_bie_matrix, rel  # noqa: E402


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


def test_served_solutions_vs_dense_oracle():
    """Every served solution of a mixed trace (spheres and ellipsoids,
    subdivisions 2 and 3, k in [1, 8]) against the oracle's dense
    collocation system: its residual against the dense matrix within 2e-4
    (GMRES to 1e-4 on the FP32 product), and its distance to the dense
    solution within 1e-3 or, for an ill-conditioned system, within the
    bound cond(A) x residual that the residual implies."""
    tr = _trace(6, 31)
    st, xs = serve.serve(tr, keep_solutions=True, max_active=6)
    print("served", {k: v for k, v in st.items() if k != "records"})
    assert st["not_converged"] == 0 and st["peak_active"] >= 2
    for req in tr:
        V, T = synth.icosphere(req["subdiv"])
        V = V * np.asarray(req["axes"]).reshape(1, 3)
        A = dense_bie_matrix(req["k"], V, T)
        b = bie.plane_wave_rhs(req["k"], V, T)
        x = xs[req["id"]]
        ex = rel(x, np.linalg.solve(A, b))
        res = float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))
        cond = float(np.linalg.cond(A))
        print(f"  request {req['id']} s={req['subdiv']} k={req['k']:.2f} axes={np.round(req['axes'], 2)}: "
              f"vs dense solve {ex:.2e}, dense residual {res:.2e}, cond {cond:.1f}", flush=True)
        assert res <= 2e-4
        assert ex <= max(1e-3, 1.01 * cond * res)


def test_served_mix_with_a_large_high_frequency_solve():
    """A served mix holding one icosphere-4 solve at k = 21 (5120 panels,
    about 5 panels per wavelength) beside small ones: each result, converged
    or not, is bitwise the plain GMRES result of its own handle."""
    reqs = [(4, 21.0, (1.0, 1.0, 1.0)), (2, 3.0, (1.0, 1.0, 1.0)), (3, 5.5, (0.7, 1.4, 1.1)),
            (2, 7.0, (1.2, 0.8, 1.0))]
    trees, bs = [], []
    for s_, k, ax in reqs:
        V, T = synth.icosphere(s_)
        trees.append(hfmm.Tree.from_mesh(V * np.asarray(ax).reshape(1, 3), T))
        bs.append(trees[-1].plane_wave(k))
    alone = [t.gmres(k, 10, b, tol=1e-4, maxit=600) for t, (_, k, _), b in zip(trees, reqs, bs)]
    srv = hfmm.Server(max_active=4)
    xs = [torch.zeros_like(b) for b in bs]
    tickets = [srv.submit(t, k, 10, b, x, tol=1e-4, maxit=600)[0] for t, (_, k, _), b, x in
               zip(trees, reqs, bs, xs)]
    for _ in range(100000):
        na, nq = srv.step()
        if na == 0 and nq == 0:
            break
    torch.cuda.synchronize()
    for i, tk in enumerate(tickets):
        state, info, _ = srv.poll(tk)
        print("request", reqs[i], "state", state, "iters", info["iters"], "alone", alone[i][1]["iters"])
        assert info["iters"] == alone[i][1]["iters"]
        np.testing.assert_array_equal(xs[i].cpu().numpy(), alone[i][0].cpu().numpy(), err_msg=f"request {i}")
    srv.free()


def test_early_stop_policy():
    """stall_restarts = 1 with stall_factor 1e-6 demands a millionfold drop
    per restart, which no solve makes: every solve stops at its second
    restart boundary in state STOPPED with x its last iterate, which equals
    the plain GMRES iterate after the same number of products.  Bad limits
    are refused."""
    V, T = synth.icosphere(2)
    t = hfmm.Tree.from_mesh(V, T)
    b = t.plane_wave(4.0)
    srv = hfmm.Server(max_active=2)
    with pytest.raises(hfmm.HfmmError):
        srv.set_limits(-1, 0.5, 0.0)
    with pytest.raises(hfmm.HfmmError):
        srv.set_limits(1, 0.0, 0.0)
    srv.set_limits(1, 1e-6, 0.0)
    x = torch.zeros_like(b)
    tk, _ = srv.submit(t, 4.0, 10, b, x, tol=1e-12, restart=5, maxit=1000)
    for _ in range(10000):
        na, nq = srv.step()
        if na == 0 and nq == 0:
            break
    state, info, _ = srv.poll(tk)
    print("stopped", state, info)
    assert state == hfmm.Server.STOPPED and info["iters"] == 5 and info["restarts"] == 1
    xp, ip = t.gmres(4.0, 10, b, tol=1e-12, restart=5, maxit=5)
    assert ip["iters"] == 5 and not ip["converged"]
    np.testing.assert_array_equal(x.cpu().numpy(), xp.cpu().numpy())
    srv.free()
