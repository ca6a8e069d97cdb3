"""Checks of the synthetic two-ellipsoid (wing-fuselage) surface mesh, an
input generator: the clipped union surface must enclose the union of the two
solids (divergence-theorem volume against an independent integral of the
union's volume) and no mesh vertex may lie inside both solids."""
import math

import numpy as np

import synth


def _union_volume(fus, wing, n=2000):
    """V_fus + V_wing - V_intersection; the intersection (both bodies centred
    at the origin) is the integral over (x, y) of 2 sqrt(min of the two
    bodies' z^2 extents), midpoint rule on an n x n grid."""
    ax, ay = min(fus[0], wing[0]), min(fus[1], wing[1])
    x = (np.arange(n) + 0.5) / n * 2 * ax - ax
    y = (np.arange(n) + 0.5) / n * 2 * ay - ay
    X, Y = np.meshgrid(x, y, indexing="ij")
    zz = [b[2] ** 2 * (1 - X ** 2 / b[0] ** 2 - Y ** 2 / b[1] ** 2) for b in (fus, wing)]
    m = np.clip(np.minimum(*zz), 0.0, None)
    vi = (2 * np.sqrt(m)).sum() * (2 * ax / n) * (2 * ay / n)
    return 4 / 3 * math.pi * (np.prod(fus) + np.prod(wing)) - vi


def _mesh_volume(V, T):
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    return float((np.cross(b - a, c - a) * (a + b + c)).sum() / 18.0)


def test_wing_fuselage_encloses_the_union():
    fus, wing = synth.WING_FUSELAGE["fuselage"], synth.WING_FUSELAGE["wing"]
    vu = _union_volume(fus, wing)
    # the two solids overlap by about 10% of the union: a mesh that kept the
    # parts inside the other body, or dropped outside parts, misses by that much
    assert 0.08 < (4 / 3 * math.pi * (np.prod(fus) + np.prod(wing)) - vu) / vu < 0.12
    d = []
    for s in (2, 3, 4):
        V, T = synth.wing_fuselage(s)
        d.append((vu - _mesh_volume(V, T)) / vu)
    print("volume deficit by subdivision", d)
    # chords of convex surfaces: the deficit is positive and falls by more
    # than 3x per refinement (cut points snapped to nearby vertices make the
    # seam converge faster than h^2, not slower)
    assert all(x > 0 for x in d) and d[2] < 3e-3
    assert d[0] / d[1] > 3.0 and d[1] / d[2] > 3.0


def test_wing_fuselage_vertices_not_inside_both():
    fus, wing = synth.WING_FUSELAGE["fuselage"], synth.WING_FUSELAGE["wing"]
    V, T = synth.wing_fuselage(3)
    f = [((V / np.asarray(b)) ** 2).sum(axis=1) - 1.0 for b in (fus, wing)]
    # original vertices lie on their own body (f = 0), cut vertices on the other
    assert np.all(np.maximum(f[0], f[1]) >= -1e-9)
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    assert area.min() > 0.0
    # outward orientation: both ellipsoids are centred at the origin and
    # star-shaped about it, so every outward normal points away from it
    assert np.all((np.cross(b - a, c - a) * (a + b + c)).sum(axis=1) > 0)


def test_wing_fuselage_has_no_slivers():
    """Cut points near an edge end are moved to it, so no cut piece is
    thinner (area / longest edge^2; 0.433 for an equilateral triangle) than
    the thinnest triangle of the wing's own scaled icosphere at the same
    subdivision, from subdivision 2 on.  Without the snapping, cut pieces
    reach 0.004.  At subdivision 1 (80 triangles per body) a wing triangle
    cut near the junction leaves a piece of 0.029, 0.7x the wing's own."""
    def quality(V, T):
        a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
        area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
        h = np.max([np.linalg.norm(b - a, axis=1), np.linalg.norm(c - b, axis=1),
                    np.linalg.norm(a - c, axis=1)], axis=0)
        return area / h ** 2
    for s in (2, 3, 4):
        V0, T0 = synth.icosphere(s)
        own = quality(V0 * np.asarray(synth.WING_FUSELAGE["wing"]), T0).min()
        q = quality(*synth.wing_fuselage(s)).min()
        print(s, own, q)
        assert q >= 0.99 * own
