"""Writes batch64_smallest4.npz: the oracle FMM products (FP64) of the four
smallest instances of the 64-instance batched-matvec workload (instances
from synth.batch_instances with its defaults: seed 4242, N log-uniform in
[2048, 65536], k uniform in [1, 20], spheres and ellipsoids alternating;
P = 10, ncrit 64), for the fused-batch parity test.  Calls only oracle/ and
the seeded input generators; the oracle takes about three minutes per
instance, so the four run in parallel processes.

Usage: python tests/golden/make_batch64_oracle.py
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle.fmm import FMM  # noqa: E402

P = 10


def smallest4():
    inst = synth.batch_instances()
    return [int(i) for i in np.argsort([d["n"] for d in inst], kind="stable")[:4]], inst


def one(i):
    _, inst = smallest4()
    d = inst[i]
    return FMM(d["points"], k=d["k"], P=P, ncrit=64).matvec(d["q"])


if __name__ == "__main__":
    idx, inst = smallest4()
    with ProcessPoolExecutor(4) as ex:
        ys = list(ex.map(one, idx))
    out = {"index": np.asarray(idx, np.int32), "P": np.int32(P)}
    for i, y in zip(idx, ys):
        out[f"y{i}"] = np.asarray(y, np.complex128)
        print("instance", i, "n", inst[i]["n"], "k", round(inst[i]["k"], 3))
    np.savez_compressed(os.path.join(HERE, "batch64_smallest4.npz"), **out)
