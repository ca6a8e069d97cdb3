"""Dense restarted GMRES (FP64) with modified Gram-Schmidt and Givens rotations.

The paper solves the dense system with GMRES (Sec. 1, Sec. 5.1: complex
scalars, exit at 1e-4 relative residual, Sec. 6.4).  Restart length,
orthogonalisation and initial guess are unstated; this oracle takes the
textbook algorithm (Saad and Schultz 1986): x0 = 0, no preconditioner,
modified Gram-Schmidt Arnoldi, complex Givens rotations, stop when the
Arnoldi residual estimate |g_{j+1}| / ||b|| <= tol, then confirm with the
true residual and continue (restart) if it is still above tol.
"""
from __future__ import annotations

import numpy as np


def gmres(matvec, b, tol=1e-4, restart=30, maxit=2000, x0=None):
    b = np.asarray(b, np.complex128)
    n = len(b)
    x = np.zeros(n, np.complex128) if x0 is None else np.array(x0, np.complex128)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros(n, np.complex128), dict(iters=0, restarts=0, resid=0.0, converged=True)
    it = 0
    restarts = 0
    hist = []
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / bn <= tol:
            return x, dict(iters=it, restarts=restarts, resid=beta / bn, converged=True, hist=hist)
        if it >= maxit:
            return x, dict(iters=it, restarts=restarts, resid=beta / bn, converged=False, hist=hist)
        m = restart
        V = np.zeros((m + 1, n), np.complex128)
        H = np.zeros((m + 1, m), np.complex128)
        cs = np.zeros(m, np.complex128)
        sn = np.zeros(m, np.complex128)
        g = np.zeros(m + 1, np.complex128)
        V[0] = r / beta
        g[0] = beta
        j_done = 0
        for j in range(m):
            w = matvec(V[j])
            for i in range(j + 1):                 # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                     # apply previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if den == 0:
                cs[j], sn[j] = 1.0, 0.0
            elif abs(a) == 0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / den
                sn[j] = (a / abs(a)) * np.conj(bb) / den
            H[j, j] = cs[j] * a + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]) / bn)
            if abs(g[j + 1]) / bn <= tol or it >= maxit or H[j, j] == 0:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + V[:j_done].T @ y
        restarts += 1
