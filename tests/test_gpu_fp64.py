"""GPU parity of the FP64 variant of the FMM product and of the FP64 direct
sum (the precision-study references) against the FP64 oracle.

Bars: the FP64 variant matches the oracle FMM at the same tree, lists and P
to 1e-11 (both FP64; they differ in summation order and in how the Gaunt
coefficients are obtained); the FP32 product matches the FP64 variant to
1e-5 (FP32 rounding only); the FP64 direct sum matches the oracle's to
1e-12."""
import numpy as np
import pytest

import synth
from oracle.fmm import FMM, direct_sum

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1803_09948_amd import hfmm  # noqa: E402
from parity import check, rel  # noqa: E402


@pytest.mark.parametrize("n,k,P,ncrit,seed", [
    (4096, 1.0, 8, 64, 11),
    (3000, 9.0, 10, 32, 13),
    (2000, 2.0, 3, 32, 14),
])
def test_fp64_variant_vs_oracle_fmm(n, k, P, ncrit, seed):
    x = synth.sphere_points(n, seed)
    q = synth.strengths(n, seed)
    print(f"case n={n} k={k} P={P}", flush=True)
    t = hfmm.Tree.from_points(x, ncrit=ncrit)
    y64 = t.matvec64(k, P, torch.from_numpy(q.astype(np.complex128)).to("cuda")).cpu().numpy()
    y32 = t.matvec(k, P, torch.from_numpy(q).to("cuda")).cpu().numpy()
    yo = FMM(x, k=k, P=P, ncrit=ncrit).matvec(q)
    check(y64, yo, 1e-11, "fp64 gpu vs oracle")
    check(y32, y64, 1e-5, "fp32 gpu vs fp64 gpu")


def test_direct64_vs_oracle():
    xs = synth.sphere_points(3000, 41)
    q = synth.strengths(3000, 41).astype(np.complex128)
    tg = np.concatenate([synth.sphere_points(200, 42), xs[:50]])  # includes coincident points (R = 0)
    y = hfmm.direct64(torch.from_numpy(xs).to("cuda"), torch.from_numpy(q).to("cuda"),
                      torch.from_numpy(tg).to("cuda"), 7.0).cpu().numpy()
    yo = direct_sum(7.0, tg, xs, q)
    check(y, yo, 1e-12, "direct64 vs oracle")
    # no sources: zeros
    z = hfmm.direct64(torch.zeros((0, 3), dtype=torch.float32, device="cuda"),
                      torch.zeros(0, dtype=torch.complex128, device="cuda"),
                      torch.from_numpy(tg[:5]).to("cuda"), 1.0).cpu().numpy()
    assert np.all(z == 0)


def test_truncation_error_falls_with_P():
    n, k = 6000, 6.0
    x = synth.sphere_points(n, 43)
    q = synth.strengths(n, 43).astype(np.complex128)
    xd, qd = torch.from_numpy(x).to("cuda"), torch.from_numpy(q).to("cuda")
    ref = hfmm.direct64(xd, qd, xd, k).cpu().numpy()
    t = hfmm.Tree.from_points(x, ncrit=32)
    errs = [rel(t.matvec64(k, P, qd).cpu().numpy(), ref) for P in (2, 4, 6, 8, 10)]
    print("FP64 FMM vs direct, P = 2..10:", errs)
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-6


def test_fp64_argument_errors():
    v, tr = synth.icosphere(1)
    b = hfmm.Tree.from_mesh(v, tr)
    x = torch.zeros(b.n_in, dtype=torch.complex128, device="cuda")
    with pytest.raises(hfmm.HfmmError):
        b.matvec64(1.0, 4, x)
    t = hfmm.Tree.from_points(synth.sphere_points(100, 1))
    x = torch.zeros(100, dtype=torch.complex128, device="cuda")
    with pytest.raises(hfmm.HfmmError):
        t.matvec64(1.0, 17, x)
    with pytest.raises(hfmm.HfmmError):
        t.matvec64(-1.0, 4, x)
