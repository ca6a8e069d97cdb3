"""Adaptive octree, Morton order and dual tree traversal lists (plain Python).

Written from Sec. 2.3 (octree, upward/traverse/downward passes), Sec. 3.1
(bodies sorted by Morton order; a cell is an index and a count into the sorted
bodies) and Sec. 3.2 (keys from cell positions; the dual tree traversal walks
source and target trees together).  The paper leaves the box, the keys' bit
layout, the split rule and the acceptance criterion unspecified; the readings
implemented here are:

* Root cube.  he = max over axes of (max - min)/2 of all points (sources and
  targets); he = 1 if that is 0.  q = largest power of two <= he/64.  Centre
  c_d = floor(mid_d / q + 0.5) * q.  Half-width H = smallest power of two >= q
  with |x_d - c_d| < H for every point and axis.
* Keys.  key_d = floor(((x_d - c_d) + H) / (2H) * 2^21) in FP64 from the FP32
  coordinates, clamped to [0, 2^21 - 1]; interleaved with x in the lowest bit.
* Sort.  Stable by key (ties keep input order), sources and targets apart.
* Split.  A cell splits into its non-empty octants when it holds more than
  ncrit sources (point mode: sources = targets), down to level 20.  With a
  wavenumber-aware acceptance (below), a non-empty cell whose side exceeds
  kappa/k always splits: such a cell can never be accepted, so as a leaf all
  of its targets would interact directly with every source.
* Cells are stored level by level, each level in Morton order.
* Acceptance (M2L) between target A and source B, with half-sides hA, hB:
  3 (sA + sB)^2 < theta^2 D2 and k * 2 max(hA, hB) <= kappa, where sA, sB,
  D2 are the half-sides and the squared centre distance in units of the finer
  cell's half-side (integers).  Radius of a cell = sqrt(3) * half-side.
* Traversal from (root, root): accepted -> M2L; two leaves -> P2P; otherwise
  split the cell with the larger radius (tie: the target); if that one is a
  leaf, split the other.  Pairs with an empty side are dropped.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

KEYBITS = 21
MAXLEVEL = 20


def root_cube(points_f32: np.ndarray):
    x = np.asarray(points_f32, dtype=np.float32).astype(np.float64)
    lo = x.min(axis=0)
    hi = x.max(axis=0)
    he = float(((hi - lo) / 2.0).max())
    if he == 0.0:
        he = 1.0
    q = 2.0 ** math.floor(math.log2(he / 64.0))
    while q * 2.0 <= he / 64.0:
        q *= 2.0
    while q > he / 64.0:
        q /= 2.0
    mid = (lo + hi) / 2.0
    c = np.floor(mid / q + 0.5) * q
    H = q
    while not np.all(np.abs(x - c) < H):
        H *= 2.0
    return c, H


def morton_keys(points_f32: np.ndarray, c, H) -> np.ndarray:
    x = np.asarray(points_f32, dtype=np.float32).astype(np.float64)
    kd = np.floor(((x - c) + H) / (2.0 * H) * float(1 << KEYBITS))
    kd = np.clip(kd, 0, (1 << KEYBITS) - 1).astype(np.int64)
    key = np.zeros(len(x), dtype=np.int64)
    for b in range(KEYBITS):
        for d in range(3):
            key |= ((kd[:, d] >> b) & 1) << (3 * b + d)
    return key


@dataclass
class Tree:
    c: np.ndarray           # root centre (3,)
    H: float                # root half-width
    ncrit: int
    src_perm: np.ndarray    # sorted position -> original source index
    tgt_perm: np.ndarray
    src_keys: np.ndarray    # sorted keys
    tgt_keys: np.ndarray
    level: np.ndarray       # per cell
    ijk: np.ndarray         # integer cell coordinates at its level (ncell, 3)
    sb: np.ndarray          # source range [sb, se)
    se: np.ndarray
    tb: np.ndarray          # target range
    te: np.ndarray
    cb: np.ndarray          # children range [cb, ce) in cell order
    ce: np.ndarray
    parent: np.ndarray

    @property
    def ncell(self) -> int:
        return len(self.level)

    def is_leaf(self, i: int) -> bool:
        return self.cb[i] == self.ce[i]

    def half(self, i: int) -> float:
        return self.H / (1 << int(self.level[i]))

    def centre(self, i: int) -> np.ndarray:
        h = self.half(i)
        return self.c - self.H + (2.0 * self.ijk[i].astype(np.float64) + 1.0) * h


def build_tree(src_f32: np.ndarray, tgt_f32: np.ndarray | None, ncrit: int,
               split_side: float | None = None) -> Tree:
    """Octree over sources and targets (targets None: point mode, same set).
    split_side: non-empty cells with side > split_side always split."""
    src = np.asarray(src_f32, np.float32)
    point_mode = tgt_f32 is None
    tgt = src if point_mode else np.asarray(tgt_f32, np.float32)
    allp = src if point_mode else np.concatenate([src, tgt])
    c, H = root_cube(allp)
    skey = morton_keys(src, c, H)
    sperm = np.argsort(skey, kind="stable")
    skey = skey[sperm]
    if point_mode:
        tperm, tkey = sperm, skey
    else:
        tkey = morton_keys(tgt, c, H)
        tperm = np.argsort(tkey, kind="stable")
        tkey = tkey[tperm]

    level, ijk, sb, se, tb, te, cb, ce, parent = ([] for _ in range(9))
    level.append(0); ijk.append((0, 0, 0))
    sb.append(0); se.append(len(src)); tb.append(0); te.append(len(tgt))
    parent.append(-1)
    cb.append(0); ce.append(0)
    cur = [0]
    lev = 0
    while cur:
        nxt = []
        for ci in cur:
            ns = se[ci] - sb[ci]
            nb = ns if point_mode else ns + (te[ci] - tb[ci])
            force = split_side is not None and 2.0 * H / (1 << lev) > split_side and nb >= 1
            if (ns <= ncrit and not force) or lev >= MAXLEVEL:
                cb[ci] = ce[ci] = len(level)  # leaf: empty child range
                continue
            shift = 3 * (KEYBITS - lev - 1)
            s_oct = (skey[sb[ci]:se[ci]] >> shift) & 7
            t_oct = (tkey[tb[ci]:te[ci]] >> shift) & 7
            first = len(level)
            for o in range(8):
                s_lo = sb[ci] + int(np.searchsorted(s_oct, o, "left"))
                s_hi = sb[ci] + int(np.searchsorted(s_oct, o, "right"))
                t_lo = tb[ci] + int(np.searchsorted(t_oct, o, "left"))
                t_hi = tb[ci] + int(np.searchsorted(t_oct, o, "right"))
                if s_lo == s_hi and t_lo == t_hi:
                    continue
                i, j, kk = ijk[ci]
                level.append(lev + 1)
                ijk.append((2 * i + (o & 1), 2 * j + ((o >> 1) & 1), 2 * kk + ((o >> 2) & 1)))
                sb.append(s_lo); se.append(s_hi); tb.append(t_lo); te.append(t_hi)
                cb.append(0); ce.append(0)
                parent.append(ci)
                nxt.append(len(level) - 1)
            cb[ci] = first
            ce[ci] = len(level)
        cur = nxt
        lev += 1
    A = lambda v: np.asarray(v, dtype=np.int64)
    return Tree(c=c, H=H, ncrit=ncrit, src_perm=sperm, tgt_perm=tperm,
                src_keys=skey, tgt_keys=tkey, level=A(level),
                ijk=np.asarray(ijk, dtype=np.int64).reshape(-1, 3),
                sb=A(sb), se=A(se), tb=A(tb), te=A(te), cb=A(cb), ce=A(ce),
                parent=A(parent))


def mac(tree: Tree, a: int, b: int, k: float, theta: float, kappa: float) -> bool:
    la, lb = int(tree.level[a]), int(tree.level[b])
    L = max(la, lb)
    # centres in units of the finer half-side u = H / 2^L:  -2^L + (2i+1) 2^(L-l)
    ca = -(1 << L) + (2 * tree.ijk[a] + 1) * (1 << (L - la))
    cbv = -(1 << L) + (2 * tree.ijk[b] + 1) * (1 << (L - lb))
    d = ca - cbv
    D2 = int((d * d).sum())
    sA, sB = 1 << (L - la), 1 << (L - lb)
    geo = 3.0 * float((sA + sB) ** 2) < (theta * theta) * float(D2)
    hmax = max(tree.half(a), tree.half(b))
    return geo and (k * (2.0 * hmax) <= kappa)


def dual_tree_traversal(tree: Tree, k: float, theta: float, kappa: float):
    """Returns (m2l, p2p): lists of (target cell, source cell) in visit order."""
    m2l, p2p = [], []
    ntg = tree.te - tree.tb
    nsr = tree.se - tree.sb
    leaf = tree.cb == tree.ce
    rad = np.array([tree.half(i) for i in range(tree.ncell)])  # radius ~ half-side
    stack = [(0, 0)]
    while stack:
        a, b = stack.pop()
        if ntg[a] == 0 or nsr[b] == 0:
            continue
        if mac(tree, a, b, k, theta, kappa):
            m2l.append((a, b))
            continue
        if leaf[a] and leaf[b]:
            p2p.append((a, b))
            continue
        split_a = (not leaf[a]) and (rad[a] >= rad[b] or leaf[b])
        if split_a:
            kids = [(ch, b) for ch in range(tree.cb[a], tree.ce[a])]
        else:
            kids = [(a, ch) for ch in range(tree.cb[b], tree.ce[b])]
        # push in reverse so that children are visited in Morton order
        stack.extend(reversed(kids))
    return m2l, p2p
