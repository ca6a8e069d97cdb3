"""Flat-panel collocation discretisation of the sound-soft equation (FP64).

Written from Sec. 2.1 (eq. (7): the single-layer integral of G q equals the
incident field on S), Sec. 2.2 (Nystrom-type discretisation with point
matching; Duffy treatment of the weak 1/R singularity) and the near/self
branches of the P2P listing (Sec. 3.1) and Sec. 6.4 (self and near
singularity treatment).

Readings (the paper's curvilinear order-p elements are replaced by flat
triangles with one unknown per panel, collocated at the centroid):
* Unknown q_j is constant on panel T_j; row i is collocated at centroid c_i.
* A_ij = (A_j / 3) sum_g G(c_i, y_jg) with the interior 3-point rule
  (barycentric (2/3,1/6,1/6) and permutations, weight A_j/3) for far pairs.
* Near pairs (j != i, |c_i - c_j| < eta h_j, h_j = longest edge of T_j):
  A_ij = integral over T_j of G(c_i, y) dS_y (computed accurately).
* Self term A_ii = integral over T_i of G(c_i, y) dS_y (weakly singular),
  computed here by the Duffy transformation about c_i.
* Right-hand side b_i = exp(i k d . c_i), d the incidence direction (+z).
"""
from __future__ import annotations

import functools

import numpy as np

from .fmm import green

GAUSS3 = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])


def panels(verts, tris):
    """Centroids, areas, longest edges, unit normals, and the 3 Gauss points
    (shape (nt, 3, 3)) of flat triangles."""
    V = np.asarray(verts, np.float64)
    T = np.asarray(tris, np.int64)
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    cen = (a + b + c) / 3.0
    cr = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    nrm = cr / (2.0 * area[:, None])
    h = np.maximum(np.maximum(np.linalg.norm(b - a, axis=1), np.linalg.norm(c - b, axis=1)),
                   np.linalg.norm(a - c, axis=1))
    gp = np.einsum("gv,tvd->tgd", GAUSS3, np.stack([a, b, c], axis=1))
    return dict(centroid=cen, area=area, h=h, normal=nrm, gauss=gp, a=a, b=b, c=c)


@functools.lru_cache(maxsize=None)
def _gl01(n: int):
    """Gauss-Legendre nodes and weights on [0, 1] (computed once per n; the
    arrays are read-only)."""
    x, w = np.polynomial.legendre.leggauss(n)
    u, wu = 0.5 * (x + 1.0), 0.5 * w
    u.flags.writeable = False
    wu.flags.writeable = False
    return u, wu


def duffy_rule(p, q, r, n: int):
    """Points and weights integrating over triangle (p, q, r) with the Duffy
    collapse at vertex p: y = p + u (q - p) + u v (r - q), Jacobian 2A u.
    Exact cancellation of a 1/|y - p| singularity."""
    u, wu = _gl01(n)
    v, wv = _gl01(n)
    U, Vv = np.meshgrid(u, v, indexing="ij")
    W = np.outer(wu, wv)
    p, q, r = (np.asarray(z, np.float64) for z in (p, q, r))
    pts = p + U[..., None] * (q - p) + (U * Vv)[..., None] * (r - q)
    area2 = np.linalg.norm(np.cross(q - p, r - p))
    w = W * U * area2
    return pts.reshape(-1, 3), w.reshape(-1)


def subdivide(a, b, c, L: int):
    tris = [(np.asarray(a, float), np.asarray(b, float), np.asarray(c, float))]
    for _ in range(L):
        nt = []
        for (x, y, z) in tris:
            xy, yz, zx = (x + y) / 2, (y + z) / 2, (z + x) / 2
            nt += [(x, xy, zx), (y, yz, xy), (z, zx, yz), (xy, yz, zx)]
        tris = nt
    return tris


def _ref_rule_subdivided(L: int, n: int):
    """Barycentric points (npts, 3) and weights (sum = 1, i.e. per unit area)
    of 4^L uniform sub-triangles of the reference triangle, each with the
    n x n collapsed Gauss rule."""
    key = (L, n)
    if key not in _RULES:
        E = np.eye(3)
        lam, wt = [], []
        for (p, q, r) in subdivide(E[0], E[1], E[2], L):
            pts, w = duffy_rule(p, q, r, n)   # in barycentric space (area 1/2 plane-wise)
            lam.append(pts)
            wt.append(w)
        lam = np.concatenate(lam)
        wt = np.concatenate(wt)
        _RULES[key] = (lam, wt / wt.sum())
    return _RULES[key]


def _ref_rule_centroid(n: int):
    """Barycentric points and per-unit-area weights of the Duffy rule collapsed
    at the centroid over the three sub-triangles (x, a, b), (x, b, c), (x, c, a)."""
    key = ("c", n)
    if key not in _RULES:
        E = np.eye(3)
        x = np.full(3, 1.0 / 3.0)
        lam, wt = [], []
        for (q, r) in ((E[0], E[1]), (E[1], E[2]), (E[2], E[0])):
            pts, w = duffy_rule(x, q, r, n)
            lam.append(pts)
            wt.append(w)
        lam = np.concatenate(lam)
        wt = np.concatenate(wt)
        _RULES[key] = (lam, wt / wt.sum())
    return _RULES[key]


_RULES: dict = {}


def self_integral(k: float, a, b, c, n: int = 32) -> complex:
    """Integral over triangle (a,b,c) of G(x, y) dS_y with x its centroid.

    G = 1/(4 pi R) + (e^{ikR} - 1)/(4 pi R): the first part by the closed form
    of `laplace_panel_analytic`, the bounded second part by Duffy rules
    collapsed at x.  Each sub-triangle (x, q, r) over an edge qr is cut at
    the foot F of the perpendicular from x onto qr (clamped to the edge) into
    (x, q, F) and (x, F, r): along the edge the distance from x has its
    minimum at F, and on an elongated panel, where x lies close to its long
    edge, that minimum is sharp; with the cut each piece sees a monotone
    distance and the rule converges as it does on a well-shaped panel."""
    a, b, c = (np.asarray(z, np.float64) for z in (a, b, c))
    x = (a + b + c) / 3.0
    smooth = 0.0
    for q, r in ((a, b), (b, c), (c, a)):
        e = r - q
        F = q + min(max(float((x - q) @ e) / float(e @ e), 0.0), 1.0) * e
        for p1, p2 in ((q, F), (F, r)):
            if np.linalg.norm(np.cross(p1 - x, p2 - x)) == 0.0:
                continue
            pts, w = duffy_rule(x, p1, p2, n)
            R = np.linalg.norm(pts - x, axis=1)
            smooth += (w * np.expm1(1j * k * R) / (4 * np.pi * R)).sum()
    return complex(laplace_panel_analytic(x, a, b, c) / (4 * np.pi) + smooth)


def self_integral_duffy(k: float, a, b, c, n: int = 24) -> complex:
    """Same integral by the Duffy rule alone (the paper's treatment, Sec. 2.2)."""
    lam, w = _ref_rule_centroid(n)
    a, b, c = (np.asarray(z, np.float64) for z in (a, b, c))
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a))
    pts = lam @ np.stack([a, b, c])
    x = (a + b + c) / 3.0
    R = np.linalg.norm(pts - x, axis=1)
    return complex((w * area * np.exp(1j * k * R) / (4 * np.pi * R)).sum())


def panel_integral(k: float, x, a, b, c, L: int = 3, n: int = 8) -> complex:
    """Integral over triangle (a,b,c) of G(x, y) dS_y for x off the panel:
    4^L uniform sub-triangles, each with an n x n collapsed Gauss rule."""
    return complex(panel_integrals(k, np.asarray(x)[None, :], np.asarray(a)[None],
                                   np.asarray(b)[None], np.asarray(c)[None], L, n)[0])


def panel_integrals(k: float, x, a, b, c, L: int = 3, n: int = 8):
    """Vectorised panel_integral over pairs: x (m,3) and panels a,b,c (m,3)."""
    lam, w = _ref_rule_subdivided(L, n)
    a, b, c, x = (np.asarray(z, np.float64) for z in (a, b, c, x))
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    pts = (lam[None, :, 0, None] * a[:, None, :] + lam[None, :, 1, None] * b[:, None, :]
           + lam[None, :, 2, None] * c[:, None, :])
    g = green(k, x[:, None, :], pts)
    return (g * w[None, :]).sum(axis=1) * area


def laplace_panel_analytic(x, a, b, c) -> float:
    """Closed form of the integral over a flat triangle of 1/|x - y| dS_y
    (edge-sum formula for a planar polygon; valid for any x)."""
    a, b, c, x = (np.asarray(z, np.float64) for z in (a, b, c, x))
    nrm = np.cross(b - a, c - a)
    nrm /= np.linalg.norm(nrm)
    w0 = float(np.dot(x - a, nrm))
    xp = x - w0 * nrm
    aw = abs(w0)
    tot = 0.0
    for (p, q) in ((a, b), (b, c), (c, a)):
        t = (q - p) / np.linalg.norm(q - p)
        u = np.cross(t, nrm)                        # outward in-plane normal
        P0 = float(np.dot(p - xp, u))
        lm = float(np.dot(p - xp, t))
        lp = float(np.dot(q - xp, t))
        Rm = float(np.linalg.norm(x - p))
        Rp = float(np.linalg.norm(x - q))
        R0sq = P0 * P0 + w0 * w0
        if abs(P0) > 1e-300:
            tot += P0 * np.log((Rp + lp) / (Rm + lm))
            if aw > 0:
                tot -= aw * (np.arctan(P0 * lp / (R0sq + aw * Rp))
                             - np.arctan(P0 * lm / (R0sq + aw * Rm)))
    return tot


def gauss_sources(pan):
    """Flattened 3 Gauss points per panel (panel-major) and their weights A/3."""
    nt = len(pan["area"])
    pts = pan["gauss"].reshape(nt * 3, 3)
    w = np.repeat(pan["area"] / 3.0, 3)
    return pts, w


def dense_matrix(k: float, verts, tris, eta: float = 2.0, rows=None):
    """Collocation matrix A (or the selected rows), complex128."""
    pan = panels(verts, tris)
    nt = len(pan["area"])
    rows = np.arange(nt) if rows is None else np.asarray(rows)
    gp, w = gauss_sources(pan)
    A = np.zeros((len(rows), nt), np.complex128)
    for r0 in range(0, len(rows), 128):
        rr = rows[r0:r0 + 128]
        G = green(k, pan["centroid"][rr][:, None, :], gp[None, :, :]) * w[None, :]
        A[r0:r0 + 128] = G.reshape(len(rr), nt, 3).sum(axis=2)
    cen, h = pan["centroid"], pan["h"]
    for t, i in enumerate(rows):
        d = np.linalg.norm(cen - cen[i], axis=1)
        js = np.flatnonzero(d < eta * h)
        js = js[js != i]
        if len(js):
            A[t, js] = panel_integrals(k, np.repeat(cen[i][None], len(js), 0),
                                       pan["a"][js], pan["b"][js], pan["c"][js])
        A[t, i] = self_integral(k, pan["a"][i], pan["b"][i], pan["c"][i])
    return A


def plane_wave_rhs(k: float, verts, tris, direction=(0.0, 0.0, 1.0)):
    pan = panels(verts, tris)
    d = np.asarray(direction, np.float64)
    return np.exp(1j * k * (pan["centroid"] @ d))


def scattered_field(k: float, verts, tris, q, xobs, L: int = 1):
    """u_s(x) = - integral of G(x, y) q(y) dS_y for x off the surface, with
    q constant per panel (4^L sub-triangles, 3-point rule each)."""
    pan = panels(verts, tris)
    xobs = np.asarray(xobs, np.float64)
    out = np.zeros(len(xobs), np.complex128)
    for (p, qq, r) in subdivide(pan["a"], pan["b"], pan["c"], L):
        ar = 0.5 * np.linalg.norm(np.cross(qq - p, r - p), axis=1)
        for g in GAUSS3:
            y = g[0] * p + g[1] * qq + g[2] * r
            out -= green(k, xobs[:, None, :], y[None, :, :]) @ (np.asarray(q) * ar / 3.0)
    return out
