"""Coefficient-level parity of the matrix-core M2L: the translation (S|R)
of eqs. (12)-(14) between well-separated cells (Sec. 2.3).  Random
expansion vectors go through one canonical operator under all 16
reflections (hfmm_debug_m2l: the product's own table generator, reflection
codes, matrix-core kernel and reduction), and each column is compared with
the oracle's (S|R) matrix at the reflected offset applied to the same
vector.  Bar: FP32 arithmetic, 1e-5 relative (2-norm and infinity norm)."""
import math

import numpy as np
import pytest

from oracle import expansions as ex

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1803_09948_amd import hfmm  # noqa: E402
from parity import check  # noqa: E402


def sigma(P, rho):
    """The product's per-degree scale s_n = rho^n / (2n+1)!!, one entry per
    coefficient (n, m)."""
    s, df = [], 1.0
    for n in range(P):
        df *= 2 * n + 1
        s += [rho ** n / df] * (2 * n + 1)
    return np.asarray(s)


def reflect(t, g):
    """Offset of a pair with reflection g of the canonical offset t: swap x
    and y (bit 3), then negate x, y, z (bits 0, 1, 2)."""
    x, y, z = t
    if g & 8:
        x, y = y, x
    return np.array([-x if g & 1 else x, -y if g & 2 else y, -z if g & 4 else z])


@pytest.mark.parametrize("P,k,ki,w,side", [
    (10, 16 * math.pi, 0.0, (6, 4, 2), 0.0625),   # the headline: level 6 cells, k side = pi
    (10, 16 * math.pi, 0.0, (8, 0, 0), 0.0625),   # on an axis (m-symmetric operator)
    (10, 16 * math.pi, 0.0, (7, 7, 5), 0.03125),  # x = y (the swap leaves the offset fixed)
    (8, 1.0, 0.0, (10, 6, 4), 0.25),             # low frequency: scaled basis at k side = 0.25
    (12, 9.0, 0.0, (6, 6, 6), 0.125),
    (16, 3.0, 0.0, (8, 2, 0), 0.25),             # the largest order (16-pair chunks)
    (5, 5.0, 0.0, (9, 3, 1), 0.25),              # a partly filled last 16-row tile
    (10, 6.0, 1.5, (6, 2, 2), 0.125),            # complex wavenumber (damped)
])
def test_m2l_coefficients_vs_oracle(P, k, ki, w, side):
    t = np.asarray(w, np.float64) * side / 2.0        # offsets in half-sides, as the plan stores them
    rho = min(1.0, math.hypot(k, ki) * side)
    refl = np.arange(40) % 16                          # every reflection, 40 columns (two chunks)
    rng = np.random.default_rng(P * 1000 + int(k))
    mt = (rng.uniform(-1, 1, (40, P * P)) + 1j * rng.uniform(-1, 1, (40, P * P))).astype(np.complex64)
    s = sigma(P, rho)
    print(f"case P={P} k={k}+{ki}i t={t} rho={rho:.3f}", flush=True)
    out = hfmm.debug_m2l(P, k, t, rho, rho, refl, torch.from_numpy(mt).to("cuda"), k_imag=ki).cpu().numpy()
    L = out.astype(np.complex128) / s[None, :]
    M = mt.astype(np.complex128) * s[None, :]           # the same vectors, unscaled
    kc = complex(k, ki) if ki else k
    Lo = np.stack([ex.sr_matrix(reflect(t, int(g)), kc, P) @ M[c] for c, g in enumerate(refl)])
    # per column in the scaled basis the kernel computes, where all degrees weigh alike
    check((L * s[None, :]).ravel(), (Lo * s[None, :]).ravel(), 1e-5, "scaled L vs oracle (S|R) M")
    for c in range(16):                                  # every reflection on its own
        e = np.linalg.norm((L[c] - Lo[c]) * s) / np.linalg.norm(Lo[c] * s)
        assert e <= 1e-5, (c, e)


def test_m2l_hook_refuses_bad_arguments():
    x = torch.zeros((2, 100), dtype=torch.complex64, device="cuda")
    for t, refl, rho in (((1.0, 2.0, 0.0), [0, 1], 0.5), ((0.0, 0.0, 0.0), [0, 1], 0.5),
                         ((2.0, 1.0, 0.0), [0, 16], 0.5), ((2.0, 1.0, 0.0), [0, 1], 1.5)):
        with pytest.raises(hfmm.HfmmError) as e:
            hfmm.debug_m2l(10, 3.0, t, rho, rho, refl, x)
        assert e.value.code == hfmm.HFMM_EINVAL
