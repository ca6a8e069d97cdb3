"""The GMRES entry point that allocates nothing (hfmm_gmres_solve_noalloc,
Krylov workspace in the library's static device scratch) against
hfmm_gmres_solve: the same solution bits and iteration counts, on two calls
in a row, the second with fewer unknowns; sizes beyond the scratch and
unprepared (k, P) are refused."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1803_09948_amd import hfmm  # noqa: E402


def _solve_both(s, k, P=10, tol=1e-5, restart=30):
    print(f"case icosphere s={s} k={k} P={P} restart={restart}", flush=True)
    V, T = synth.icosphere(s)
    t = hfmm.Tree.from_mesh(V, T)
    b = t.plane_wave(k)
    x_ref, i_ref = t.gmres(k, P, b, tol=tol, restart=restart)
    torch.cuda.synchronize()
    x = torch.zeros_like(b)
    x, info = t.gmres_noalloc(k, P, b, x, tol=tol, restart=restart)
    torch.cuda.synchronize()
    print("  plain", i_ref, "noalloc", info, flush=True)
    assert info["converged"] and i_ref["converged"]
    assert info["iters"] == i_ref["iters"] and info["restarts"] == i_ref["restarts"]
    np.testing.assert_array_equal(x.cpu().numpy(), x_ref.cpu().numpy())
    return t


def test_noalloc_gmres_equals_gmres_twice_second_smaller():
    big = _solve_both(3, 5.0)          # 1280 unknowns
    small = _solve_both(2, 3.0, restart=12)   # 320 unknowns, after the larger call
    big.free()
    small.free()


def test_noalloc_gmres_refusals():
    V, T = synth.icosphere(2)
    t = hfmm.Tree.from_mesh(V, T)
    b = t.plane_wave(3.0)
    x = torch.zeros_like(b)
    with pytest.raises(hfmm.HfmmError) as e:       # (k, P) not prepared: preparing would allocate
        t.gmres_noalloc(3.0, 10, b, x)
    assert e.value.code == hfmm.HFMM_EINVAL
    t.prepare(3.0, 10)
    with pytest.raises(hfmm.HfmmError) as e:       # restart 200 on 320 unknowns still fits; a huge
        t.gmres_noalloc(3.0, 10, b, x, restart=0)  # restart is refused as an argument error
    assert e.value.code == hfmm.HFMM_EINVAL
    Vb, Tb = synth.icosphere(6)                    # 81920 unknowns x 201 Krylov vectors > 72 MiB
    tb = hfmm.Tree.from_mesh(Vb, Tb)
    bb = torch.zeros(len(Tb), dtype=torch.complex128, device="cuda")
    with pytest.raises(hfmm.HfmmError) as e:
        tb.gmres_noalloc(3.0, 10, bb, torch.zeros_like(bb), restart=200)
    assert e.value.code == hfmm.HFMM_ENOMEM and "static scratch" in str(e.value)
    x, info = t.gmres_noalloc(3.0, 10, b, x, tol=1e-5)
    assert info["converged"]
