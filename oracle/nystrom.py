"""Locally corrected Nystrom discretisation on curved six-node triangles (FP64).

Test infrastructure only: the HIP library never imports this module.

Written from Sec. 2.2:
* eq. (8): the unknown at an element's interpolation point is the density
  times the surface Jacobian, interpolated over the element by Lagrange
  polynomials in the element's parameters;
* eqs. (9)-(10): point matching at every interpolation point, so an entry is
  the parametric integral of G times a Lagrange polynomial (the Jacobian
  cancels against the surface measure);
* the Duffy treatment of the weak 1/R singularity (Sec. 2.2), and the
  self/near corrections of Sec. 6.4.
From the dataset description (Sec. 5): six points per curved triangle, three
associated with its corners and three with its edges.

Readings:
* Geometry: the quadratic map of the reference triangle {u, v >= 0,
  u + v <= 1} through the six nodes (v0, v1, v2, m01, m12, m20).
* Points: the symmetric degree-4 six-point rule on the triangle (Strang and
  Fix; Dunavant 1985), one orbit of three points near the corners and one
  near the edge midpoints; its weights w_i (summing to 1/2, the reference
  area) are the far-field quadrature.
* Z_(j,m)(i,n) = w_i G(r_jm, r_in) for far pairs.  The self element (n = m)
  uses the Duffy collapse at the target's parameter point over three
  sub-triangles, with a sinh substitution in the angular variable (Duffy
  alone converges slowly when the point is close to an edge).  Near elements (j's point within eta h_n of the centroid of
  n, h_n the longest corner-to-corner distance) use 4^L uniform
  sub-triangles with an n x n collapsed Gauss rule each.
* Density q = I / Jacobian; scattered field u_s(x) = -sum_in w_i G(x, r_in) I_in.
"""
from __future__ import annotations

import math

import numpy as np

from .fmm import green


def _rule6():
    """Points (6, 2) in (u, v) and weights (6,) of the degree-4 rule on the
    reference triangle (area 1/2)."""
    a1, b1, w1 = 0.816847572980459, 0.091576213509771, 0.109951743655322
    a2, b2, w2 = 0.108103018168070, 0.445948490915965, 0.223381589678011
    bary = []
    wts = []
    for a, b, w in ((a1, b1, w1), (a2, b2, w2)):
        for lam in ((a, b, b), (b, a, b), (b, b, a)):
            bary.append(lam)
            wts.append(0.5 * w)
    bary = np.array(bary)
    return bary[:, 1:3].copy(), np.array(wts)


RULE_UV, RULE_W = _rule6()


def monomials(u, v):
    """[1, u, v, u^2, u v, v^2] along the last axis."""
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    return np.stack([np.ones_like(u), u, v, u * u, u * v, v * v], axis=-1)


# Lagrange polynomials through the six points: L_i(u, v) = monomials(u, v) @ LAGR[:, i]
LAGR = np.linalg.inv(monomials(RULE_UV[:, 0], RULE_UV[:, 1]))


def lagrange(u, v):
    return monomials(u, v) @ LAGR


def shape(u, v):
    """Quadratic shape functions N (..., 6) and their u and v derivatives."""
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    l1, l2, l3 = 1.0 - u - v, u, v
    N = np.stack([l1 * (2 * l1 - 1), l2 * (2 * l2 - 1), l3 * (2 * l3 - 1),
                  4 * l1 * l2, 4 * l2 * l3, 4 * l3 * l1], axis=-1)
    z = np.zeros_like(u)
    Nu = np.stack([-(4 * l1 - 1), 4 * l2 - 1, z, 4 * (l1 - l2), 4 * l3, -4 * l3], axis=-1)
    Nv = np.stack([-(4 * l1 - 1), z, 4 * l3 - 1, -4 * l2, 4 * l2, 4 * (l1 - l3)], axis=-1)
    return N, Nu, Nv


def element_nodes(nodes, tri6):
    """(nt, 6, 3) node coordinates of each element."""
    return np.asarray(nodes, np.float64)[np.asarray(tri6, np.int64)]


def map_points(X, u, v):
    """Positions and Jacobians |x_u x x_v| of parameter points (u, v) on
    elements X (nt, 6, 3): returns (nt, M, 3) and (nt, M)."""
    N, Nu, Nv = shape(u, v)
    x = np.einsum("ma,tad->tmd", N, X)
    xu = np.einsum("ma,tad->tmd", Nu, X)
    xv = np.einsum("ma,tad->tmd", Nv, X)
    return x, np.linalg.norm(np.cross(xu, xv), axis=-1)


def discretise(nodes, tri6):
    """Interpolation points r (nt*6, 3) element-major, their Jacobians,
    their parametric weights, element centroids and sizes."""
    X = element_nodes(nodes, tri6)
    r, jac = map_points(X, RULE_UV[:, 0], RULE_UV[:, 1])
    cen, _ = map_points(X, np.array([1 / 3]), np.array([1 / 3]))
    corners = X[:, :3]
    h = np.max(np.stack([np.linalg.norm(corners[:, 0] - corners[:, 1], axis=1),
                         np.linalg.norm(corners[:, 1] - corners[:, 2], axis=1),
                         np.linalg.norm(corners[:, 2] - corners[:, 0], axis=1)]), axis=0)
    nt = len(X)
    return dict(X=X, r=r.reshape(nt * 6, 3), jac=jac.reshape(nt * 6), w=np.tile(RULE_W, nt),
                centroid=cen[:, 0], h=h)


def _gl01(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def collapsed_rule(p, q, r, n: int):
    """n x n Gauss rule on the parameter-space triangle (p, q, r), collapsed
    at p: y = p + s (q - p) + s t (r - q), weight |det(q - p, r - p)| s.
    Cancels a 1/|y - p| singularity."""
    s, ws = _gl01(n)
    t, wt = _gl01(n)
    S, T = np.meshgrid(s, t, indexing="ij")
    W = np.outer(ws, wt) * S
    p, q, r = (np.asarray(z, np.float64) for z in (p, q, r))
    pts = p + S[..., None] * (q - p) + (S * T)[..., None] * (r - q)
    det = abs((q - p)[0] * (r - p)[1] - (q - p)[1] * (r - p)[0])
    return pts.reshape(-1, 2), (W * det).reshape(-1)


CORNERS = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])


def duffy_at(p, n: int, Xe):
    """Rule over the reference triangle for an integrand with a 1/R
    singularity at the interior parameter point p of element Xe (6, 3).

    Duffy collapse at p over the three sub-triangles (p, corner, next
    corner): y = p + s (e0 + t e), weight |det| s, which removes the 1/R.
    What is left varies sharply in t when p is close to the far edge, so t
    is split at the point of the edge closest to p (in the metric of the
    element's tangent map at p) and each part is mapped by
    t = t0 +/- (H / B) sinh(mu tau), tau in [0, 1] (H: distance from p to
    the edge, B: edge length, sinh(mu) = part length B / H).  For a flat
    element this makes the transformed 1/R integrand constant in tau."""
    p = np.asarray(p, np.float64)
    _, Nu, Nv = shape(np.array([p[0]]), np.array([p[1]]))
    xu, xv = Nu[0] @ Xe, Nv[0] @ Xe
    gm = np.array([[xu @ xu, xu @ xv], [xu @ xv, xv @ xv]])
    s, ws = _gl01(n)
    tau, wtau = _gl01(n)
    pts, wts = [], []
    for a, b in ((0, 1), (1, 2), (2, 0)):
        q, r = CORNERS[a], CORNERS[b]
        e0, e = q - p, r - q
        det = abs(e0[0] * e[1] - e0[1] * e[0])
        t0 = min(max(-(e0 @ gm @ e) / (e @ gm @ e), 0.0), 1.0)
        foot = e0 + t0 * e
        H = math.sqrt(max(foot @ gm @ foot, 1e-300))
        B = math.sqrt(e @ gm @ e)
        ts, wt = [], []
        for length, sign in ((t0, -1.0), (1.0 - t0, 1.0)):
            if length <= 1e-15:
                continue
            mu = math.asinh(length * B / H)
            ts.append(t0 + sign * (H / B) * np.sinh(mu * tau))
            wt.append((H / B) * mu * np.cosh(mu * tau) * wtau)
        t = np.concatenate(ts)
        wt = np.concatenate(wt)
        S, T = np.meshgrid(s, t, indexing="ij")
        W = np.outer(ws, wt) * S * det
        pts.append((p + S[..., None] * e0 + (S * T)[..., None] * e).reshape(-1, 2))
        wts.append(W.reshape(-1))
    return np.concatenate(pts), np.concatenate(wts)


def subdivided(L: int, n: int):
    """Rule over the reference triangle: 4^L uniform sub-triangles, each with
    the n x n collapsed rule."""
    tris = [tuple(CORNERS)]
    for _ in range(L):
        nt = []
        for (x, y, z) in tris:
            xy, yz, zx = (x + y) / 2, (y + z) / 2, (z + x) / 2
            nt += [(x, xy, zx), (y, yz, xy), (z, zx, yz), (xy, yz, zx)]
        tris = nt
    pts, wts = [], []
    for (x, y, z) in tris:
        a, b = collapsed_rule(x, y, z, n)
        pts.append(a)
        wts.append(b)
    return np.concatenate(pts), np.concatenate(wts)


def element_integrals(k: float, x, Xe, uv, wq):
    """Integral over the reference triangle of G(x, x_e(u, v)) L_i(u, v)
    du dv for i = 0..5 with the rule (uv, wq); x (3,), Xe (6, 3)."""
    y, _ = map_points(Xe[None], uv[:, 0], uv[:, 1])
    g = green(k, np.asarray(x, np.float64)[None, :], y[0])
    return (g * wq) @ lagrange(uv[:, 0], uv[:, 1])


def near_elements(d, eta: float, rows=None):
    """For each point (or each of `rows`), the elements other than its own
    whose centroid lies within eta h of it (list of arrays)."""
    r, cen, h = d["r"], d["centroid"], d["h"]
    out = []
    for j in (range(len(r)) if rows is None else rows):
        dist = np.linalg.norm(cen - r[j], axis=1)
        es = np.flatnonzero(dist < eta * h)
        out.append(es[es != j // 6])
    return out


def dense_matrix(k: float, nodes, tri6, eta: float = 2.0, L: int = 3, n_near: int = 8, n_self: int = 12,
                 rows=None):
    """The Nystrom matrix Z (N, N), N = 6 x elements, complex128, or its
    selected rows (len(rows), N)."""
    d = discretise(nodes, tri6)
    r, w, X = d["r"], d["w"], d["X"]
    N = len(r)
    rows = np.arange(N) if rows is None else np.asarray(rows)
    Z = green(k, r[rows][:, None, :], r[None, :, :]) * w[None, :]
    near = near_elements(d, eta, rows)
    uv_near, w_near = subdivided(L, n_near)
    lag_near = lagrange(uv_near[:, 0], uv_near[:, 1])
    for t, j in enumerate(rows):
        m = j // 6
        p = RULE_UV[j % 6]
        uv, wq = duffy_at(p, n_self, X[m])
        Z[t, 6 * m:6 * m + 6] = element_integrals(k, r[j], X[m], uv, wq)
        es = near[t]
        if len(es):
            y_es, _ = map_points(X[es], uv_near[:, 0], uv_near[:, 1])     # (ne, M, 3)
            g = green(k, r[j][None, None, :], y_es)                      # (ne, M)
            vals = (g * w_near[None, :]) @ lag_near                      # (ne, 6)
            for e, v in zip(es, vals):
                Z[t, 6 * e:6 * e + 6] = v
    return Z


def plane_wave_rhs(k: float, nodes, tri6, direction=(0.0, 0.0, 1.0)):
    d = discretise(nodes, tri6)
    return np.exp(1j * k * (d["r"] @ np.asarray(direction, np.float64)))


def scattered_field(k: float, nodes, tri6, I, xobs):
    """u_s(x) = -sum w_i G(x, r_i) I_i at points off the surface."""
    d = discretise(nodes, tri6)
    xobs = np.asarray(xobs, np.float64)
    return -(green(k, xobs[:, None, :], d["r"][None, :, :]) @ (d["w"] * np.asarray(I)))


def factorial_moment(a: int, b: int) -> float:
    """Integral of u^a v^b over the reference triangle: a! b! / (a + b + 2)!."""
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
