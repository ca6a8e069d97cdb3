"""Seeded synthetic inputs shared by the HIP path, the tests and the benchmark.

This module generates *inputs only*: point clouds, strengths, triangle meshes
and request traces.  It contains none of the method's arithmetic (no kernel,
no expansion, no quadrature, no tree), so both the product path and the CPU
oracle may draw from it without sharing any computation.

Every floating-point input that the GPU path consumes in single precision is
produced in FP64 once and rounded to FP32 ("FP32-canonical"), so the oracle
sees exactly the values the kernels see.

The paper's scatterer is a sphere of radius 1 m under plane-wave incidence
(Sec. 5.2); its curvilinear meshes are not available, so unit spheres,
icospheres and affinely scaled ellipsoids stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "sphere_points", "strengths", "icosphere", "scale_axes", "curved_icosphere", "wing_fuselage",
    "WORKLOADS", "batch_instances", "serve_trace",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.PCG64(seed))


def sphere_points(n: int, seed: int, radius: float = 1.0) -> np.ndarray:
    """n points uniform on a sphere (normalised Gaussian triples), FP32-canonical.

    Returns float32 array of shape (n, 3).
    """
    if n == 0:
        return np.zeros((0, 3), np.float32)
    g = _rng(seed).standard_normal((n, 3))
    nrm = np.sqrt((g * g).sum(axis=1, keepdims=True))
    nrm[nrm == 0.0] = 1.0
    return (radius * g / nrm).astype(np.float32)


def strengths(n: int, seed: int) -> np.ndarray:
    """complex64 strengths, real and imaginary parts uniform in [-1, 1]."""
    r = _rng(seed + 0x5151).uniform(-1.0, 1.0, (n, 2))
    return (r[:, 0] + 1j * r[:, 1]).astype(np.complex64)


def scale_axes(points: np.ndarray, axes) -> np.ndarray:
    """Affinely scale points by semi-axes (a, b, c); keeps the input dtype."""
    a = np.asarray(axes, dtype=np.float64).reshape(1, 3)
    return (points.astype(np.float64) * a).astype(points.dtype)


def icosphere(subdiv: int, radius: float = 1.0):
    """Icosphere with 20 * 4**subdiv flat triangles, outward counter-clockwise.

    Vertices are FP64 on the sphere of the given radius; every refinement
    step splits each triangle 1->4 at edge midpoints projected back onto the
    sphere.  Returns (verts float64 (nv,3), tris int32 (nt,3)).
    """
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    verts = [tuple(x) for x in v]
    for _ in range(subdiv):
        cache: dict = {}

        def mid(i: int, j: int) -> int:
            key = (i, j) if i < j else (j, i)
            if key in cache:
                return cache[key]
            a = np.asarray(verts[i]) + np.asarray(verts[j])
            a = a / np.linalg.norm(a)
            verts.append(tuple(a))
            cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for (a, b, c) in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        f = np.array(nf, dtype=np.int64)
    V = np.asarray(verts, dtype=np.float64) * radius
    # orient outward: normal (b-a)x(c-a) must point away from the origin
    a, b, c = V[f[:, 0]], V[f[:, 1]], V[f[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = (nrm * (a + b + c)).sum(axis=1) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return V, f.astype(np.int32)


def curved_icosphere(subdiv: int, radius: float = 1.0):
    """Six-node (quadratic) triangles on the sphere: the icosphere of
    `icosphere(subdiv)` plus one node per edge at the edge midpoint projected
    onto the sphere.  Returns (nodes float64 (nn,3), tri6 int32 (nt,6)) with
    each row (v0, v1, v2, m01, m12, m20), outward counter-clockwise."""
    V, T = icosphere(subdiv, radius)
    nodes = [tuple(x) for x in V]
    cache: dict = {}

    def mid(i: int, j: int) -> int:
        key = (i, j) if i < j else (j, i)
        if key not in cache:
            a = V[i] + V[j]
            nodes.append(tuple(a / np.linalg.norm(a) * radius))
            cache[key] = len(nodes) - 1
        return cache[key]

    tri6 = np.array([[a, b, c, mid(a, b), mid(b, c), mid(c, a)] for (a, b, c) in T.tolist()], dtype=np.int32)
    return np.asarray(nodes, dtype=np.float64), tri6


def _clip_outside(V, T, centre, axes, min_area, snap):
    """Keep the part of each triangle outside the solid ellipsoid
    sum(((x - centre) / axes)^2) <= 1.  An edge that crosses the surface is
    cut at its exact crossing (a quadratic in the edge parameter), moved to
    the nearer end when it lies within `snap` of it (no sliver pieces); the
    kept polygon (3 or 4 corners, same winding) is fanned into triangles, and
    pieces smaller than min_area are dropped.  Returns new (verts, tris),
    vertices not shared between triangles."""
    c = np.asarray(centre, dtype=np.float64)
    ax = np.asarray(axes, dtype=np.float64)

    def f(x):
        u = (x - c) / ax
        return float(u @ u) - 1.0

    def cross(p, q):
        u, w = (p - c) / ax, (q - p) / ax
        A, B, C = float(w @ w), 2.0 * float(u @ w), float(u @ u) - 1.0
        d = math.sqrt(max(B * B - 4.0 * A * C, 0.0))
        for t in ((-B - d) / (2.0 * A), (-B + d) / (2.0 * A)):
            if -1e-12 <= t <= 1.0 + 1e-12:
                t = 0.0 if t < snap else 1.0 if t > 1.0 - snap else t
                return p + t * (q - p)
        raise ValueError("no crossing on a sign-changing edge")

    out_v, out_t = [], []
    for tri in T:
        P = [V[i] for i in tri]
        keep = [f(x) >= 0.0 for x in P]
        if not any(keep):
            continue
        poly = []
        for j in range(3):
            p, q = P[j], P[(j + 1) % 3]
            if keep[j]:
                poly.append(p)
            if keep[j] != keep[(j + 1) % 3]:
                poly.append(cross(p, q))
        for j in range(1, len(poly) - 1):
            a, b, cc = poly[0], poly[j], poly[j + 1]
            if 0.5 * np.linalg.norm(np.cross(b - a, cc - a)) < min_area:
                continue
            base = len(out_v)
            out_v += [a, b, cc]
            out_t.append([base, base + 1, base + 2])
    return np.asarray(out_v, dtype=np.float64).reshape(-1, 3), np.asarray(out_t, dtype=np.int32).reshape(-1, 3)


WING_FUSELAGE = {"fuselage": (2.0, 0.4, 0.4), "wing": (0.6, 1.8, 0.12)}


def wing_fuselage(subdiv: int, fuselage=WING_FUSELAGE["fuselage"], wing=WING_FUSELAGE["wing"],
                  min_frac: float = 0.02, snap: float = 0.3):
    """A wing-fuselage configuration emulated by two intersecting ellipsoids
    centred at the origin (the geometry the paper names as its next target,
    Sec. 7): a fuselage along x and a thin wing along y.  Each body is the
    icosphere(subdiv) scaled to its semi-axes, with the triangles (or parts
    of triangles) inside the other body removed, so the union's surface is
    covered by flat triangles, outward counter-clockwise.  The two clipped
    surfaces meet along the intersection curve without sharing vertices (a
    collocation method needs no conforming mesh); cut pieces smaller than
    min_frac of a body's median triangle are dropped.  Returns (verts
    float64 (nv,3), tris int32 (nt,3))."""
    V0, T0 = icosphere(subdiv)
    parts = []
    for mine, other in ((fuselage, wing), (wing, fuselage)):
        V = V0 * np.asarray(mine, dtype=np.float64).reshape(1, 3)
        a, b, c = V[T0[:, 0]], V[T0[:, 1]], V[T0[:, 2]]
        med = float(np.median(0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)))
        parts.append(_clip_outside(V, T0, (0.0, 0.0, 0.0), other, min_frac * med, snap))
    (Va, Ta), (Vb, Tb) = parts
    return np.concatenate([Va, Vb]), np.concatenate([Ta, Tb + len(Va)]).astype(np.int32)


# --------------------------------------------------------------------------
# Workloads (sizes and parameters of the benchmark and test configurations)
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    n: int = 0
    k: float = 1.0
    P: int = 8
    ncrit: int = 64
    theta: float = 0.5
    kappa: float = -1.0          # <0: use 0.4*P
    seed: int = 1
    subdiv: int = 0
    extra: dict = field(default_factory=dict)

    def kappa_eff(self) -> float:
        return 0.4 * self.P if self.kappa < 0 else self.kappa


WORKLOADS = {
    # plain matvec, small: N=4096 on the unit sphere, k=1, P=8
    "matvec_4k": Workload("matvec_4k", n=4096, k=1.0, P=8, seed=11),
    # BIE solve on an icosphere, subdivision 5 (20480 panels), k = 2*pi
    "bie_ico5": Workload("bie_ico5", k=2.0 * math.pi, P=10, subdiv=5, seed=0),
    # precision study / headline: 1M points, diameter = 16 wavelengths
    "matvec_1m": Workload("matvec_1m", n=1 << 20, k=16.0 * math.pi, P=10, seed=23),
    "matvec_8m": Workload("matvec_8m", n=1 << 23, k=16.0 * math.pi, P=10, seed=29),
}


def batch_instances(count: int = 64, seed: int = 4242, nmin: int = 2048,
                    nmax: int = 65536, kmin: float = 1.0, kmax: float = 20.0):
    """Instances for the batched-matvec workload.

    N log-uniform in [nmin, nmax]; k uniform in [kmin, kmax]; even instances
    are unit spheres, odd ones ellipsoids with semi-axes uniform in [0.5, 2].
    Returns a list of dicts with float32 points and complex64 strengths.
    """
    r = _rng(seed)
    out = []
    for i in range(count):
        n = int(round(math.exp(r.uniform(math.log(nmin), math.log(nmax)))))
        k = float(r.uniform(kmin, kmax))
        axes = (1.0, 1.0, 1.0) if i % 2 == 0 else tuple(r.uniform(0.5, 2.0, 3))
        pts = scale_axes(sphere_points(n, seed * 1000 + i), axes)
        out.append(dict(n=n, k=k, axes=axes, points=pts,
                        q=strengths(n, seed * 1000 + i)))
    return out


def serve_trace(nreq: int = 600, rate: float = 50.0, seed: int = 777,
                subdivs=(3, 4, 5, 6), kmin: float = 1.0, kmax: float = 30.0):
    """Poisson arrival trace of scattering solves.

    Each request: arrival time (s), icosphere subdivision, semi-axes (sphere or
    ellipsoid, 50/50, axes uniform in [0.5, 2]) and wavenumber.
    """
    r = _rng(seed)
    t = np.cumsum(r.exponential(1.0 / rate, nreq))
    reqs = []
    for i in range(nreq):
        s = int(r.choice(subdivs))
        ell = bool(r.uniform() < 0.5)
        axes = tuple(r.uniform(0.5, 2.0, 3)) if ell else (1.0, 1.0, 1.0)
        k = float(r.uniform(kmin, kmax))
        reqs.append(dict(id=i, t_arrival=float(t[i]), subdiv=s, axes=axes, k=k))
    return reqs
