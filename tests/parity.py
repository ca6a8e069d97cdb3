"""Parity measures shared by the GPU tests: the relative 2-norm difference
and the relative infinity-norm difference max|y - y_o| / max|y_o| (a bound
on every element at the scale of the largest output), printed and checked
against a stated bar."""
import numpy as np


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def relinf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def check(y, yo, bar, label="", barinf=None):
    """Asserts finite y, rel(y, yo) <= bar and relinf(y, yo) <= barinf
    (default: the same bar); returns both measures."""
    e2, ei = rel(y, yo), relinf(y, yo)
    print(f"  {label} rel2 {e2:.3e} relinf {ei:.3e}", flush=True)
    assert np.all(np.isfinite(y)), label
    assert e2 <= bar, f"{label}: rel2 {e2:.3e} > {bar}"
    assert ei <= (bar if barinf is None else barinf), f"{label}: relinf {ei:.3e}"
    return e2, ei


def _bie_rows(args):
    from oracle import bie
    k, V, T, rows = args
    return bie.dense_matrix(k, V, T, rows=rows)


def dense_bie_matrix(k, V, T, workers=8):
    """The oracle's dense flat-panel collocation matrix, its rows computed in
    spawned worker processes (the oracle's own dense_matrix on each block of
    rows; the same numbers as one call over all rows)."""
    import multiprocessing as mp
    import os
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(workers, os.cpu_count() or 1))
    blocks = [b for b in np.array_split(np.arange(len(T)), 2 * workers) if len(b)]
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_bie_rows, [(k, V, T, b) for b in blocks]))
    return np.concatenate(parts, axis=0)
