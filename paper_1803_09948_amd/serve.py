"""Serving loop for scattering solves with continuous batching.

Requests (sphere or ellipsoid icosphere meshes, wavenumber k) arrive over
time.  Host-side work of a request (mesh scaling, octree, traversal lists and
operator descriptors) runs in a thread pool as soon as it arrives; the solve
is then queued on an `hfmm.Server`, which admits it when a slot and device
memory are free and advances all running solves together, one GMRES product
per step with a single fused FMM launch sequence.  Latency is measured from
arrival to completion on the host clock.

`serve_plain` runs the same trace one request at a time through
`Tree.gmres` (the plain single-solve path) for comparison.
"""
from __future__ import annotations

import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import synth

from . import hfmm


def _meshes(trace):
    return {s: synth.icosphere(s) for s in sorted({r["subdiv"] for r in trace})}


def _build(req, meshes, P):
    V, T = meshes[req["subdiv"]]
    V = V * np.asarray(req["axes"], dtype=np.float64).reshape(1, 3)
    tree = hfmm.Tree.from_mesh(V, T)
    fp = tree.prepare_host(req["k"], P)
    return tree, fp


def _pct(v, q):
    return float(np.percentile(v, q) * 1e3) if len(v) else None


def _stats(lat, makespan, iters, statuses, records):
    """Throughput and latency over all solves, and latency over the converged
    ones alone (the non-converged count beside them)."""
    lat = np.asarray(lat)
    ok = np.asarray([s == hfmm.Server.CONVERGED for s in statuses], bool)
    return {
        "n": int(len(lat)),
        "solves_per_s": float(len(lat) / makespan) if makespan > 0 else 0.0,
        "p50_ms": _pct(lat, 50),
        "p99_ms": _pct(lat, 99),
        "mean_ms": float(lat.mean() * 1e3) if len(lat) else None,
        "converged": int(ok.sum()),
        "p50_converged_ms": _pct(lat[ok], 50) if len(lat) else None,
        "p99_converged_ms": _pct(lat[ok], 99) if len(lat) else None,
        "makespan_s": float(makespan),
        "iters_p50": float(np.percentile(iters, 50)) if iters else None,
        "iters_max": int(max(iters)) if iters else None,
        "not_converged": int(sum(1 for s in statuses if s != hfmm.Server.CONVERGED)),
        "stopped_early": int(sum(1 for s in statuses if s == hfmm.Server.STOPPED)),
        "records": records,
    }


def _record(req, st, info, latency):
    return dict(id=req["id"], subdiv=req["subdiv"], axes=list(req["axes"]), k=req["k"], state=int(st),
                iters=int(info["iters"]), resid_true=float(info["resid_true"]), latency_ms=latency * 1e3)


def serve(trace, P=10, tol=1e-4, restart=30, maxit=2000, max_active=16, hbm_budget=0, workers=8,
          keep_solutions=False, log=None, stall_restarts=0, stall_factor=0.5, max_seconds=0.0):
    """Runs the trace through the continuous-batching server; returns stats
    (and, with keep_solutions, {request id: x as numpy}).  stall_restarts,
    stall_factor and max_seconds set the server's early-stop policy
    (hfmm_server_set_limits; off by default)."""
    import torch

    meshes = _meshes(trace)
    reqs = sorted(trace, key=lambda r: r["t_arrival"])
    server = hfmm.Server(hbm_budget, max_active)
    server.set_limits(stall_restarts, stall_factor, max_seconds)
    pool = ThreadPoolExecutor(max_workers=workers)
    building = {}
    inflight = {}          # ticket -> (req, tree, b, x)
    lat, iters, statuses, records = [], [], [], []
    sols = {}
    peak_active = 0
    t0 = time.perf_counter()
    i = 0
    steps = 0
    while i < len(reqs) or building or inflight:
        now = time.perf_counter() - t0
        while i < len(reqs) and reqs[i]["t_arrival"] <= now:
            building[pool.submit(_build, reqs[i], meshes, P)] = reqs[i]
            i += 1
        for fut in [f for f in building if f.done()]:
            req = building.pop(fut)
            tree, _ = fut.result()
            b = tree.plane_wave(req["k"])
            x = torch.zeros_like(b)
            ticket, _ = server.submit(tree, req["k"], P, b, x, tol=tol, restart=restart, maxit=maxit)
            inflight[ticket] = (req, tree, b, x)
        if inflight:
            na, nq = server.step()
            steps += 1
            peak_active = max(peak_active, na)
            tnow = time.perf_counter() - t0
            for ticket in list(inflight):
                st, info, _ = server.poll(ticket)
                if st in (hfmm.Server.QUEUED, hfmm.Server.ACTIVE):
                    continue
                req, tree, b, x = inflight.pop(ticket)
                lat.append(tnow - req["t_arrival"])
                iters.append(info["iters"])
                statuses.append(st)
                records.append(_record(req, st, info, lat[-1]))
                if keep_solutions:
                    sols[req["id"]] = x.cpu().numpy()
                server.release(ticket)
                tree.free()
                if log:
                    log(f"done id={req['id']} s={req['subdiv']} k={req['k']:.2f} it={info['iters']} "
                        f"lat={lat[-1]*1e3:.1f} ms active={na} queued={nq}")
        elif building:
            time.sleep(0.0005)
        elif i < len(reqs):
            time.sleep(max(0.0, min(0.01, reqs[i]["t_arrival"] - (time.perf_counter() - t0))))
    torch.cuda.synchronize()
    makespan = time.perf_counter() - t0
    pool.shutdown()
    server.free()
    out = _stats(lat, makespan, iters, statuses, records)
    out.update(steps=steps, peak_active=peak_active)
    return (out, sols) if keep_solutions else out


def serve_plain(trace, P=10, tol=1e-4, restart=30, maxit=2000, keep_solutions=False, log=None):
    """The same trace, one request at a time, through Tree.gmres."""
    import torch

    meshes = _meshes(trace)
    reqs = sorted(trace, key=lambda r: r["t_arrival"])
    lat, iters, statuses, records = [], [], [], []
    sols = {}
    t0 = time.perf_counter()
    for req in reqs:
        wait = req["t_arrival"] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        tree, _ = _build(req, meshes, P)
        b = tree.plane_wave(req["k"])
        x, info = tree.gmres(req["k"], P, b, tol=tol, restart=restart, maxit=maxit)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0 - req["t_arrival"])
        iters.append(info["iters"])
        statuses.append(hfmm.Server.CONVERGED if info["converged"] else hfmm.Server.NOTCONV)
        records.append(_record(req, statuses[-1], info, lat[-1]))
        if keep_solutions:
            sols[req["id"]] = x.cpu().numpy()
        tree.free()
        if log:
            log(f"plain id={req['id']} it={info['iters']} lat={lat[-1]*1e3:.1f} ms")
    makespan = time.perf_counter() - t0
    out = _stats(lat, makespan, iters, statuses, records)
    return (out, sols) if keep_solutions else out
