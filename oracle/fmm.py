"""Direct sum and CPU FMM matvec (FP64).

Direct sum (eq. (11) with the kernel of eq. (6)):
    y_i = sum_{j : |x_i - y_j| > 0} q_j e^{ik R_ij} / (4 pi R_ij).
Readings of the P2P listing (Sec. 3.1): the distance is R = |x_i - y_j| (the
listing's 1/sqrt(R) is read as 1/R, since the kernel is 1/R); the 1/(4 pi) of
eq. (6) is included; the target carries no strength factor (eq. (11)); pairs
at zero distance contribute nothing.

FMM (Sec. 2.3): P2M at leaves, M2M upward, M2L over the traversal's accepted
pairs, L2L downward, L2P at leaves, plus the direct sum over the traversal's
leaf pairs.  Operators are the principal blocks of `oracle.expansions`.
"""
from __future__ import annotations

import numpy as np

from . import expansions as ex
from .tree import Tree, build_tree, dual_tree_traversal


def green(k, x, y):
    """G(x, y) = e^{ik|x-y|} / (4 pi |x-y|)  (eq. (6)); zero where x == y.
    k may be complex (k + i k_imag: e^{ikR} = e^{i Re(k) R} e^{-k_imag R})."""
    d = np.asarray(x, np.float64) - np.asarray(y, np.float64)
    R = np.sqrt((d * d).sum(axis=-1))
    with np.errstate(divide="ignore", invalid="ignore"):
        g = np.exp(1j * k * R) / (4.0 * np.pi * R)
    return np.where(R > 0, g, 0.0)


def direct_sum(k: float, targets, sources, q, chunk: int = 256) -> np.ndarray:
    """y_i = sum_j q_j G(x_i, y_j) over all pairs with R > 0."""
    t = np.asarray(targets, np.float64)
    s = np.asarray(sources, np.float64)
    qq = np.asarray(q, np.complex128)
    out = np.zeros(len(t), dtype=np.complex128)
    for i0 in range(0, len(t), chunk):
        g = green(k, t[i0:i0 + chunk, None, :], s[None, :, :])
        out[i0:i0 + chunk] = g @ qq
    return out


class FMM:
    """Tree, lists and cached operators for one geometry and wavenumber."""

    def __init__(self, sources, targets=None, k=1.0, P=8, ncrit=64, theta=0.5,
                 kappa=None, k_imag=0.0):
        """k_imag >= 0: the wavenumber is k + i k_imag (damped waves, the
        imaginary wavenumber of the P2P listing of Sec. 3.1); the tree's
        wavelength rules use |k + i k_imag|."""
        self.src = np.asarray(sources, np.float32)
        self.tgt = self.src if targets is None else np.asarray(targets, np.float32)
        self.k = complex(k, k_imag) if k_imag else float(k)
        self.P, self.theta = int(P), float(theta)
        self.kappa = 0.4 * P if kappa is None else float(kappa)
        kabs = abs(self.k)
        self.tree: Tree = build_tree(self.src, None if targets is None else self.tgt, ncrit,
                                     split_side=self.kappa / kabs)
        self.m2l, self.p2p = dual_tree_traversal(self.tree, kabs, self.theta, self.kappa)
        self._cache: dict = {}

    def _op(self, kind: str, t):
        key = (kind, tuple(np.round(np.asarray(t) * 2.0 ** 40).astype(np.int64)))
        T = self._cache.get(key)
        if T is None:
            f = ex.rr_matrix if kind == "rr" else ex.sr_matrix
            T = f(t, self.k, self.P)
            self._cache[key] = T
        return T

    def matvec(self, q) -> np.ndarray:
        tr, P, k = self.tree, self.P, self.k
        q = np.asarray(q, np.complex128)
        xs = self.src[tr.src_perm].astype(np.float64)
        qs = q[tr.src_perm]
        xt = self.tgt[tr.tgt_perm].astype(np.float64)
        nc = tr.ncell
        cen = np.array([tr.centre(i) for i in range(nc)])
        M = np.zeros((nc, P * P), np.complex128)
        L = np.zeros((nc, P * P), np.complex128)
        leaf = tr.cb == tr.ce
        # P2M
        for i in np.flatnonzero(leaf):
            if tr.se[i] > tr.sb[i]:
                sl = slice(tr.sb[i], tr.se[i])
                M[i] = ex.p2m(P, k, cen[i], xs[sl], qs[sl])
        # M2M, deepest level first
        for lev in range(int(tr.level.max()) - 1, -1, -1):
            for i in np.flatnonzero((tr.level == lev) & ~leaf):
                for ch in range(tr.cb[i], tr.ce[i]):
                    M[i] += self._op("rr", cen[i] - cen[ch]) @ M[ch]
        # M2L
        for a, b in self.m2l:
            L[a] += self._op("sr", cen[a] - cen[b]) @ M[b]
        # L2L, root first
        for lev in range(0, int(tr.level.max())):
            for i in np.flatnonzero((tr.level == lev) & ~leaf):
                for ch in range(tr.cb[i], tr.ce[i]):
                    L[ch] += self._op("rr", cen[ch] - cen[i]) @ L[i]
        y = np.zeros(len(xt), np.complex128)
        # L2P
        for i in np.flatnonzero(leaf):
            if tr.te[i] > tr.tb[i]:
                sl = slice(tr.tb[i], tr.te[i])
                y[sl] += ex.l2p(P, k, cen[i], L[i], xt[sl])
        # P2P
        for a, b in self.p2p:
            ta, sb = slice(tr.tb[a], tr.te[a]), slice(tr.sb[b], tr.se[b])
            y[ta] += green(k, xt[ta, None, :], xs[None, sb, :]) @ qs[sb]
        out = np.zeros_like(y)
        out[tr.tgt_perm] = y
        return out
