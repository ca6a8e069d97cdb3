"""Benchmark: FMM matvecs/s for the Helmholtz kernel at 1M points, P=10.

Workload (the headline configuration): N = 1,048,576 points uniform on the
unit sphere (seeded, FP32-canonical), k = 16 pi (diameter = 16 wavelengths),
P = 10, ncrit = 64, theta = 0.5, kappa = 0.4 P, complex64 strengths with
real and imaginary parts uniform in [-1, 1].  Tree, lists and translation
operators are built before the timed region; inputs are resident in HBM.
One step = one full FMM matvec (P2M, M2M, M2L, L2L, L2P, P2P).

Other workloads (`--workload`):
  batch  64 instances (N log-uniform in [2048, 65536], k uniform in [1, 20],
         spheres and ellipsoids alternating, P = 10): aggregate matvecs/s of
         one fused, graph-replayed launch sequence vs 64 sequential matvecs;
  serve  Poisson arrivals at 50/s of sound-soft scattering solves
         (icosphere subdivision 3..6, sphere or ellipsoid, k uniform in
         [1, 30], P = 10, GMRES(30) to 1e-4): solves/s and p50/p99 latency of
         the continuous-batching server vs the one-at-a-time path;
  precision  FP32 product vs its FP64 variant (same tree, lists, P) vs the
         FP64 direct sum on 1000 seeded targets, N = 2^20 and 2^23, P = 8/10/12;
  bie    sound-soft sphere solve (icosphere s=5, k = 2 pi and 6, GMRES(30) to
         1e-4) and the singularity ablation;
  scaling  matvec time against N = 2^16 ... 2^23 (k = 16 pi, P = 10), and the
         error at 1M points with and without the wavenumber rule (kappa);
  nystrom  the sphere solve by the curved-element Nystrom method
         (subdivisions 3..5, k = 2 pi and 6), error against the Mie series.

Prints one JSON line.  `--gpus N` with N > 1 is refused: the library runs on
one GPU (no multi-GPU path).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12      # MI355X FP32 vector / FP32 MFMA, FLOP/s
PEAK_HBM = 8.0e12         # B/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _host_cores():
    """Threads the CPU baseline may use: this process's CPU affinity, capped at
    16 (the host share of one GPU on the boxes)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_job(job):
    """One worker's share of the oracle sample (runs in a forked process with
    one BLAS thread).  Returns (kind, units, seconds)."""
    from threadpoolctl import threadpool_limits
    import oracle.expansions as ex
    from oracle.fmm import direct_sum
    kind, args = job
    with threadpool_limits(1):
        t0 = time.perf_counter()
        if kind == "p2p":
            k, xt, xs, q = args
            direct_sum(k, xt, xs, q, chunk=8)
            units = len(xt) * len(xs)
        elif kind == "m2l":
            k, P, i0, cnt, M = args
            for i in range(i0, i0 + cnt):
                ex.sr_matrix(np.array([0.5, 0.2, 0.1]) + 0.01 * i, k, P) @ M
            units = cnt
        elif kind == "p2m":
            k, P, xb, qb = args
            ex.p2m(P, k, np.zeros(3), xb * 0.01, qb)
            units = len(xb)
        else:  # m2m
            k, P, i0, cnt, M = args
            for i in range(i0, i0 + cnt):
                ex.rr_matrix(np.array([0.01, -0.01, 0.01]) * (i + 1), k, P) @ M
            units = cnt
        return kind, units, time.perf_counter() - t0


def _pool_rates(jobs, cores):
    """Runs the jobs on `cores` forked workers; rate per kind = units / summed
    worker seconds x cores (the throughput of all cores), and the wall time."""
    import multiprocessing as mp
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_job, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    units, secs = {}, {}
    for kind, u, sec in res:
        units[kind] = units.get(kind, 0) + u
        secs[kind] = secs.get(kind, 0.0) + sec
    return {kd: units[kd] / secs[kd] * cores for kd in units}, wall


def cpu_baseline(x, q, k, P, stats):
    """The FP64 oracle, as it stands, timed on a bounded sample of the
    workload on all host cores (forked worker processes, one BLAS thread
    each; run before the GPU is touched) and scaled to one full matvec with
    the traversal's counts: direct-sum pairs for P2P, operator build + apply
    per M2L pair, P2M / L2P per body, M2M / L2L per cell."""
    cores = _host_cores()
    rng = np.random.default_rng(0)
    n = len(x)
    M = rng.normal(size=P * P) + 1j * rng.normal(size=P * P)
    jobs = []
    nt = 12                                   # targets per P2P job
    for j in range(cores):
        ti = rng.choice(n, nt, replace=False)
        jobs.append(("p2p", (k, x[ti], x, q)))
        jobs.append(("m2l", (k, P, 10 * j, 10, M)))
        jobs.append(("p2m", (k, P, x[4096 * j:4096 * (j + 1)], q[4096 * j:4096 * (j + 1)])))
        jobs.append(("m2m", (k, P, j, 1, M)))
    rate, wall = _pool_rates(jobs, cores)
    est = (stats["p2p_body_pairs"] / rate["p2p"] + stats["n_m2l"] / rate["m2l"]
           + 2 * n / rate["p2m"] + 2 * stats["n_cell"] / rate["m2m"])
    return {
        "value": 1.0 / est, "unit": "matvec/s", "cores": cores, "kind": "oracle",
        "nproc": os.cpu_count(),
        "sample": (f"oracle (numpy/scipy FP64) on {cores} forked workers x 1 BLAS thread, {wall:.1f} s wall: "
                   f"{nt * cores} targets x {n} sources of the direct sum, {10 * cores} M2L operator "
                   f"builds+applies, {4096 * cores} P2M bodies and {cores} M2M operators; scaled by this "
                   f"workload's counts: {stats['p2p_body_pairs']} P2P body pairs, {stats['n_m2l']} M2L "
                   f"pairs, {stats['n_cell']} cells"),
        "seconds_per_matvec": est,
        "rates": {"p2p_pairs_per_s": rate["p2p"], "m2l_pairs_per_s": rate["m2l"],
                  "p2m_bodies_per_s": rate["p2m"], "m2m_cells_per_s": rate["m2m"]},
    }


def bench_oracle(a):
    """The oracle measured end to end at the small plain-matvec workload
    (N = 4096 on the unit sphere, k = 1, P = 8, ncrit 64): the direct sum
    over all 4096 x 4096 pairs on all host cores, and the oracle FMM (tree,
    lists, operators, matvec; a single sequential process, minutes)."""
    import synth
    from oracle.fmm import FMM
    n, k, P = 4096, 1.0, 8
    x = synth.sphere_points(n, 11)
    q = synth.strengths(n, 11)
    cores = _host_cores()
    jobs = [("p2p", (k, x[b], x, q)) for b in np.array_split(np.arange(n), 4 * cores)]
    rate, wall = _pool_rates(jobs, cores)
    t0 = time.perf_counter()
    f = FMM(x, k=k, P=P, ncrit=64)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    f.matvec(q)
    t_mv = time.perf_counter() - t0
    out = {
        "metric": "oracle FMM matvec seconds, N=4096, k=1, P=8 (one process)",
        "value": t_build + t_mv, "unit": "s", "n_gpus": 0, "steps": 1, "warmup": 0,
        "ms_per_step": (t_build + t_mv) * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "plain matvec, N=4096 uniform on the unit sphere, k=1, P=8, ncrit=64"},
        "oracle_fmm": {"tree_lists_s": t_build, "matvec_s": t_mv, "cores": 1},
        "direct_sum": {"pairs_per_s": rate["p2p"], "cores": cores, "wall_s": wall, "pairs": n * n},
        "nproc": os.cpu_count(),
    }
    print(json.dumps(out))


def traffic_of(a, kernel):
    """HBM bytes per launch of `kernel` from committed rocprofv3 counter
    summaries (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel of known
    size), if they were taken for this exact kernel build; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
        e = d[kernel]
        if e.get("source_sha") != _kernel_source_sha():
            return None
        return e["bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def _kernel_source_sha():
    import hashlib
    src = os.path.join(ROOT, "paper_1803_09948_amd", "csrc", "fmm_kernels.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def bench_copy(a):
    """A plain device copy of known size (calibrates the traffic counters)."""
    import torch
    n = a.copy_mib << 20
    x = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n, "launches": 3}))


def bench_batch(a):
    import torch

    import synth
    from paper_1803_09948_amd import hfmm

    inst = synth.batch_instances(count=a.count, seed=4242)
    P = 10
    trees = [hfmm.Tree.from_points(d["points"]) for d in inst]
    ks = [d["k"] for d in inst]
    xs = [torch.from_numpy(d["q"]).to("cuda") for d in inst]
    ys = [torch.empty_like(x) for x in xs]
    t0 = time.perf_counter()
    for t, k in zip(trees, ks):
        t.prepare(k, P)
    torch.cuda.synchronize()
    log(f"setup {time.perf_counter() - t0:.2f} s; total points {sum(d['n'] for d in inst)}")
    for _ in range(a.warmup):
        hfmm.batch_matvec(trees, ks, [P] * len(trees), xs, ys)
        for t, k, x, y in zip(trees, ks, xs, ys):
            t.matvec(k, P, x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        hfmm.batch_matvec(trees, ks, [P] * len(trees), xs, ys)
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t0) / a.steps
    t0 = time.perf_counter()
    for _ in range(a.steps):
        for t, k, x, y in zip(trees, ks, xs, ys):
            t.matvec(k, P, x, y)
    torch.cuda.synchronize()
    dt_s = (time.perf_counter() - t0) / a.steps
    # the fused sequence with each M2L launch shape and each P2P variant
    # forced (the graph is re-captured each time), against the autotuned
    # choice timed above
    def forced(phase):
        ms = []
        try:
            for v in range(hfmm.variant_count(P, phase)):
                hfmm.set_variant(v, phase)
                hfmm.batch_matvec(trees, ks, [P] * len(trees), xs, ys)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(max(1, a.steps // 2)):
                    hfmm.batch_matvec(trees, ks, [P] * len(trees), xs, ys)
                torch.cuda.synchronize()
                ms.append(round((time.perf_counter() - t0) / max(1, a.steps // 2) * 1e3, 3))
        finally:
            hfmm.set_variant(-1, phase)
        return ms
    shape_ms = forced(hfmm.PHASE_M2L)
    p2p_shape_ms = forced(hfmm.PHASE_P2P)
    log("batch ms per forced M2L shape:", shape_ms, "per forced P2P variant:", p2p_shape_ms, "autotuned:",
        round(dt_b * 1e3, 3))
    out = {
        "metric": "batched FMM matvecs/s (64 instances, one fused graph launch)",
        "value": len(trees) / dt_b, "unit": "matvec/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt_b * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{len(trees)} instances, N log-uniform [2048, 65536] "
                               f"(total {sum(d['n'] for d in inst)}), k uniform [1, 20], P=10, "
                               "spheres and ellipsoids alternating"},
        "sequential": {"value": len(trees) / dt_s, "ms_per_step": dt_s * 1e3},
        "speedup_vs_sequential": dt_s / dt_b,
        "m2l_shapes_ms": {"autotuned": dt_b * 1e3, "forced": shape_ms},
        "p2p_variants_ms": {"autotuned": dt_b * 1e3, "forced": p2p_shape_ms},
    }
    print(json.dumps(out))


def _spherical_jn_zero_distance(x, nmax):
    """Distance from x to the nearest zero of j_n, n = 0..nmax (interior
    Dirichlet eigenvalues of the unit sphere, where the single-layer
    operator of a sphere is singular)."""
    from scipy.optimize import brentq
    from scipy.special import spherical_jn
    best = np.inf
    grid = np.linspace(max(1e-3, x - 4.0), x + 4.0, 801)
    for n in range(nmax + 1):
        v = spherical_jn(n, grid)
        for i in np.nonzero(np.sign(v[:-1]) * np.sign(v[1:]) < 0)[0]:
            z = brentq(lambda u: spherical_jn(n, u), grid[i], grid[i + 1])
            best = min(best, abs(z - x))
    return float(best)


def serve_diagnostics(records):
    """For each request that did not converge: k h_max, panels per wavelength
    (wavelength over the longest edge) and, for spheres, the distance of k a
    to the nearest zero of j_n."""
    import synth
    out = []
    meshes = {}
    for r in records:
        if r["state"] == 2:
            continue
        if r["subdiv"] not in meshes:
            meshes[r["subdiv"]] = synth.icosphere(r["subdiv"])
        V, T = meshes[r["subdiv"]]
        V = V * np.asarray(r["axes"]).reshape(1, 3)
        e = np.concatenate([np.linalg.norm(V[T[:, i]] - V[T[:, (i + 1) % 3]], axis=1) for i in range(3)])
        hmax = float(e.max())
        d = dict(id=r["id"], subdiv=r["subdiv"], k=r["k"], axes=[round(v, 3) for v in r["axes"]], state=r["state"],
                 iters=r["iters"], resid_true=r["resid_true"], k_hmax=r["k"] * hmax,
                 panels_per_wavelength=2 * math.pi / r["k"] / hmax)
        if all(abs(v - 1.0) < 1e-12 for v in r["axes"]):
            d["ka_to_jn_zero"] = _spherical_jn_zero_distance(r["k"], int(r["k"]) + 10)
        out.append(d)
    return out


def bench_serve(a):
    import synth
    from paper_1803_09948_amd import serve

    trace = synth.serve_trace(nreq=a.nreq, rate=50.0, seed=777)
    log(f"serving {a.nreq} requests")
    st = serve.serve(trace, max_active=a.slots, log=log, stall_restarts=a.stall_restarts, stall_factor=0.5)
    recs = st.pop("records")
    st["diagnostics"] = serve_diagnostics(recs)
    log("served", st)
    sp = None
    if not a.no_plain:
        sp = serve.serve_plain(trace, log=log)
        sp["diagnostics"] = serve_diagnostics(sp.pop("records"))
    log("plain", sp)
    out = {
        "metric": "served BIE solves/s and p99 latency (Poisson 50 req/s)",
        "value": st["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": st["n"], "warmup": 0,
        "ms_per_step": st["mean_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{a.nreq} requests, Poisson 50/s, icosphere subdivision 3..6, sphere or "
                               "ellipsoid, k uniform [1, 30], P=10, GMRES(30) to 1e-4", "slots": a.slots,
                   "stall_restarts": a.stall_restarts},
        "served": st, "plain": sp,
    }
    print(json.dumps(out))


def bench_bie(a):
    """Sound-soft sphere, icosphere subdivision 5 (20480 flat panels), plane
    wave along z, P = 10, GMRES(30) to 1e-4 with FP64 Arnoldi: k = 2 pi (an
    interior resonance) and k = 6; then the singularity ablation at k = 6
    (self + near corrections / self only / neither); then the wing-fuselage
    pair of intersecting ellipsoids (clipped union, subdivision 5) at k = 2 pi."""
    import torch

    import synth
    from paper_1803_09948_amd import hfmm

    sphere = synth.icosphere(5)
    wingfus = synth.wing_fuselage(5)
    rows = []
    for geom, k, mode in (("sphere", 2 * math.pi, 0), ("sphere", 6.0, 0), ("sphere", 6.0, 1), ("sphere", 6.0, 2),
                          ("wing-fuselage", 2 * math.pi, 0)):
        V, T = sphere if geom == "sphere" else wingfus
        t = hfmm.Tree.from_mesh(V, T, bie_treatment=mode)
        t0 = time.perf_counter()
        t.prepare(k, 10)
        torch.cuda.synchronize()
        t_prep = time.perf_counter() - t0
        b = t.plane_wave(k)
        t.gmres(k, 10, b, tol=1e-4, restart=30, maxit=2000)  # warm (tuning, workspace)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = t.gmres(k, 10, b, tol=1e-4, restart=30, maxit=2000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        row = {"geometry": geom, "panels": len(T), "k": k, "treatment": ["self+near", "self", "none"][mode],
               "iters": info["iters"],
               "converged": info["converged"], "resid_true": info["resid_true"], "solve_ms": dt * 1e3,
               "ms_per_iter": dt * 1e3 / max(1, info["iters"]), "setup_s": t_prep}
        rows.append(row)
        log(json.dumps(row))
        t.free()
    out = {
        "metric": "BIE solve time to 1e-4 (icosphere s=5, 20480 panels, k=2 pi, P=10, GMRES(30))",
        "value": rows[0]["solve_ms"], "unit": "ms", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": rows[0]["solve_ms"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 matvec + f64 Arnoldi", "data": "synthetic",
        "config": {"workload": "sound-soft unit sphere, icosphere subdivision 5 (20480 flat triangles), "
                               "plane wave along z, P=10, ncrit=64, GMRES(30) to 1e-4"},
        "results": rows,
    }
    print(json.dumps(out))


def bench_precision(a):
    """FP32 product vs its FP64 variant (same tree, lists and P) vs the FP64
    direct sum on 1000 seeded sampled targets, N in a.prec_n, P in 8/10/12,
    k = 16 pi (16 wavelengths across the unit sphere)."""
    import torch

    import synth
    from paper_1803_09948_amd import hfmm

    k = 16.0 * math.pi
    rows = []
    for n in [int(v) for v in a.prec_n.split(",")]:
        x = synth.sphere_points(n, 23)
        q = synth.strengths(n, 23)
        xd = torch.from_numpy(x).to("cuda")
        q32 = torch.from_numpy(q).to("cuda")
        q64 = q32.to(torch.complex128)
        idx = np.sort(np.random.default_rng(5).choice(n, 1000, replace=False))
        idt = torch.from_numpy(idx).to("cuda")
        t0 = time.perf_counter()
        ref = hfmm.direct64(xd, q64, xd[idt], k)
        torch.cuda.synchronize()
        log(f"n={n}: FP64 direct sum on 1000 targets in {time.perf_counter() - t0:.1f} s")
        for P in [int(v) for v in a.prec_P.split(",")]:
            t0 = time.perf_counter()
            tree = hfmm.Tree.from_points(x, ncrit=a.ncrit)
            tree.prepare(k, P)
            torch.cuda.synchronize()
            t_prep = time.perf_counter() - t0
            y32 = tree.matvec(k, P, q32)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tree.matvec(k, P, q32, y32)
            torch.cuda.synchronize()
            t32 = time.perf_counter() - t0
            t0 = time.perf_counter()
            y64 = tree.matvec64(k, P, q64)
            torch.cuda.synchronize()
            t64 = time.perf_counter() - t0

            def err(u, v):
                return float(torch.linalg.vector_norm(u - v) / torch.linalg.vector_norm(v))

            s32, s64 = y32[idt].to(torch.complex128), y64[idt]
            st = tree.stats(k, P)
            row = {"n": n, "P": P, "err_fp32_vs_direct": err(s32, ref), "err_fp64_vs_direct": err(s64, ref),
                   "err_fp32_vs_fp64_sampled": err(s32, s64),
                   "err_fp32_vs_fp64_all": err(y32.to(torch.complex128), y64),
                   "ms_fp32": t32 * 1e3, "ms_fp64": t64 * 1e3, "setup_s": t_prep,
                   "n_m2l": st["n_m2l"], "p2p_body_pairs": st["p2p_body_pairs"]}
            rows.append(row)
            log(json.dumps(row))
            del y32, y64
            tree.free()
            torch.cuda.empty_cache()
    out = {
        "metric": "relative error vs FP64 direct sum on 1000 sampled targets (FP32 product and FP64 variant)",
        "value": next((r["err_fp32_vs_direct"] for r in rows if r["P"] == 10), rows[0]["err_fp32_vs_direct"]),
        "unit": "relative 2-norm", "n_gpus": 1, "steps": 1, "warmup": 1, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (and f64 reference)", "data": "synthetic",
        "config": {"workload": f"N in {a.prec_n} uniform on the unit sphere, k=16 pi, P in {a.prec_P}, "
                               f"ncrit={a.ncrit}, theta=0.5, kappa=0.4P, 1000 seeded targets"},
        "results": rows,
    }
    print(json.dumps(out))


def bench_nystrom(a):
    """Sound-soft sphere by the curved-element Nystrom method (six-node
    triangles, six unknowns per element), plane wave along z, P = 10,
    GMRES(30) to 1e-4: subdivisions 3, 4, 5 (7680 / 30720 / 122880 unknowns)
    at k = 2 pi and k = 6: setup, iterations and solve time.  (The error of
    u_s against the Mie series is measured by tests/test_gpu_nystrom.py.)"""
    import torch

    import synth
    from paper_1803_09948_amd import hfmm

    rows = []
    for s in [int(v) for v in a.nys_subdiv.split(",")]:
        nodes, tri6 = synth.curved_icosphere(s)
        for k in (2 * math.pi, 6.0):
            t0 = time.perf_counter()
            t = hfmm.Tree.from_curved_mesh(nodes, tri6)
            t.prepare(k, 10)
            torch.cuda.synchronize()
            t_prep = time.perf_counter() - t0
            b = t.plane_wave(k)
            t.gmres(k, 10, b, tol=1e-4, restart=30, maxit=2000)  # warm (tuning, workspace)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = t.gmres(k, 10, b, tol=1e-4, restart=30, maxit=2000)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            row = {"subdiv": s, "unknowns": 6 * len(tri6), "k": k, "iters": info["iters"],
                   "converged": info["converged"], "resid_true": info["resid_true"], "solve_ms": dt * 1e3,
                   "ms_per_iter": dt * 1e3 / max(1, info["iters"]), "setup_s": t_prep}
            rows.append(row)
            log(json.dumps(row))
            t.free()
    main = next(r for r in rows if r["subdiv"] == max(r2["subdiv"] for r2 in rows) and abs(r["k"] - 2 * math.pi) < 1e-9)
    out = {
        "metric": "curved-element Nystrom BIE solve time to 1e-4",
        "value": main["solve_ms"], "unit": "ms", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": main["solve_ms"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 matvec + f64 Arnoldi and self blocks", "data": "synthetic",
        "config": {"workload": f"sound-soft unit sphere, curved six-node icosphere subdivisions {a.nys_subdiv}, "
                               "six unknowns per element, plane wave along z, P=10, ncrit=64, GMRES(30) to 1e-4"},
        "results": rows,
    }
    print(json.dumps(out))


def bench_scaling(a):
    """Matvec time against N (2^16 ... 2^23 points on the unit sphere, k = 16 pi,
    P = 10): the O(N) check.  Then, at 1M points, the error against the FP64
    direct sum (1000 seeded targets) with and without the wavenumber rule of
    the MAC and the split (kappa = 0.4 P vs off)."""
    import torch

    import synth
    from paper_1803_09948_amd import hfmm

    k, P = 16.0 * math.pi, a.P
    rows = []
    for n in [int(v) for v in a.scale_n.split(",")]:
        x = synth.sphere_points(n, 23)
        qd = torch.from_numpy(synth.strengths(n, 23)).to("cuda")
        t0 = time.perf_counter()
        tree = hfmm.Tree.from_points(x, ncrit=a.ncrit)
        tree.prepare(k, P)
        torch.cuda.synchronize()
        t_prep = time.perf_counter() - t0
        yd = tree.matvec(k, P, qd)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            tree.matvec(k, P, qd, yd)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        st = tree.stats(k, P)
        row = {"n": n, "ms": round(ms, 4), "ns_per_point": round(ms * 1e6 / n, 3), "setup_s": round(t_prep, 2),
               "n_m2l": st["n_m2l"], "p2p_body_pairs": st["p2p_body_pairs"], "n_cell": st["n_cell"]}
        rows.append(row)
        log(json.dumps(row))
        tree.free()
        del qd, yd
        torch.cuda.empty_cache()
    # wavenumber rule on / off at 1M points
    n = 1 << 20
    x = synth.sphere_points(n, 23)
    q32 = torch.from_numpy(synth.strengths(n, 23)).to("cuda")
    xd = torch.from_numpy(x).to("cuda")
    idx = torch.from_numpy(np.sort(np.random.default_rng(5).choice(n, 1000, replace=False))).to("cuda")
    ref = hfmm.direct64(xd, q32.to(torch.complex128), xd[idx], k)
    kappa_rows = []
    for label, kappa in (("kappa=0.4P", -1.0), ("kappa off", 1e30)):
        tree = hfmm.Tree.from_points(x, ncrit=a.ncrit, kappa=kappa)
        tree.prepare(k, P)
        yd = tree.matvec(k, P, q32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            tree.matvec(k, P, q32, yd)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / 3 * 1e3
        s = yd[idx].to(torch.complex128)
        err = float(torch.linalg.vector_norm(s - ref) / torch.linalg.vector_norm(ref))
        st = tree.stats(k, P)
        row = {"rule": label, "ms": round(ms, 4), "err_vs_direct": err, "n_m2l": st["n_m2l"],
               "p2p_body_pairs": st["p2p_body_pairs"]}
        kappa_rows.append(row)
        log(json.dumps(row))
        tree.free()
    big = rows[-1]
    out = {
        "metric": "FMM matvec time per point vs N (O(N) check)",
        "value": big["ns_per_point"], "unit": "ns/point", "n_gpus": 1, "steps": 5, "warmup": 1,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"N in {a.scale_n} uniform on the unit sphere, k=16 pi, P={P}, ncrit={a.ncrit}, "
                               "theta=0.5; kappa on/off at N=1048576"},
        "results": rows, "kappa": kappa_rows,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["matvec", "batch", "serve", "precision", "bie", "copy", "scaling", "nystrom",
                                           "oracle"],
                    default="matvec")
    ap.add_argument("--prec-n", default="1048576,8388608", help="sizes of the precision workload")
    ap.add_argument("--prec-P", default="8,10,12", help="orders of the precision workload")
    ap.add_argument("--scale-n", default=",".join(str(1 << e) for e in range(16, 24)),
                    help="sizes of the scaling workload")
    ap.add_argument("--nys-subdiv", default="3,4,5", help="subdivisions of the nystrom workload")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--count", type=int, default=64, help="instances (batch workload)")
    ap.add_argument("--nreq", type=int, default=24, help="requests (serve workload)")
    ap.add_argument("--slots", type=int, default=16, help="concurrent solves (serve workload)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--stall-restarts", type=int, default=10,
                    help="serve workload: stop a solve whose true residual has not halved over this many "
                         "restarts (0: off)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--P", type=int, default=10)
    ap.add_argument("--k", type=float, default=16.0 * math.pi)
    ap.add_argument("--k-imag", type=float, default=0.0, help="imaginary part of the wavenumber (damped waves)")
    ap.add_argument("--ncrit", type=int, default=64)
    ap.add_argument("--stage-mb", type=int, default=0,
                    help="M2L staging budget in MiB (0: the library default); smaller budgets run the "
                         "M2L and its reduction in target segments")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true",
                    help="skip comparing 200 sampled outputs with the FP64 direct sum on the GPU")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if a.workload == "batch":
        return bench_batch(a)
    if a.workload == "serve":
        return bench_serve(a)
    if a.workload == "copy":
        return bench_copy(a)
    if a.workload == "precision":
        return bench_precision(a)
    if a.workload == "bie":
        return bench_bie(a)
    if a.workload == "scaling":
        return bench_scaling(a)
    if a.workload == "nystrom":
        return bench_nystrom(a)
    if a.workload == "oracle":
        return bench_oracle(a)

    import torch

    import synth
    from paper_1803_09948_amd import hfmm

    x = synth.sphere_points(a.n, 23)
    q = synth.strengths(a.n, 23)
    t0 = time.perf_counter()
    tree = hfmm.Tree.from_points(x, ncrit=a.ncrit, k_imag=a.k_imag, stage_mb=a.stage_mb)
    t_tree = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = tree.plan(a.k, a.P)               # host only: tree at (k, P), lists, work lists
    t_plan = time.perf_counter() - t0
    # the oracle on the host cores first, in forked workers, before this
    # process touches the GPU
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(x, q, a.k, a.P, plan)
        log("cpu baseline:", json.dumps(cpu))
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    tree.prepare(a.k, a.P)
    torch.cuda.synchronize()
    t_prep = t_plan + time.perf_counter() - t0
    st = tree.stats(a.k, a.P)
    log(f"setup: tree {t_tree:.2f} s, lists+operators {t_prep:.2f} s; {json.dumps(st)}")
    qd = torch.from_numpy(q).to(dev)
    yd = torch.empty_like(qd)
    for _ in range(a.warmup):
        tree.matvec(a.k, a.P, qd, yd)
    torch.cuda.synchronize()
    log("warmup done")
    # timed region: K full matvecs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        tree.matvec(a.k, a.P, qd, yd)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt / a.steps * 1e3
    log(f"timed {a.steps} steps: {ms:.3f} ms/step")
    # per-phase device times from HIP events on the launch stream (separate pass)
    tree.set_timing(True)
    acc = {}
    nrep = max(3, min(10, a.steps))
    for _ in range(nrep):
        tree.matvec(a.k, a.P, qd, yd)
        for kk, v in tree.phase_times().items():
            acc[kk] = acc.get(kk, 0.0) + v / nrep
    # the M2L time of every launch shape, phases one after another (the
    # autotuner picked one on the first product)
    tuned = tree.variant(a.k, a.P, hfmm.PHASE_M2L)
    shape_ms = []
    try:
        for v in range(hfmm.variant_count(a.P, hfmm.PHASE_M2L)):
            hfmm.set_variant(v, hfmm.PHASE_M2L)
            s = 0.0
            for _ in range(3):
                tree.matvec(a.k, a.P, qd, yd)
                s += tree.phase_times()["m2l"] / 3
            shape_ms.append(round(s, 4))
    finally:
        hfmm.set_variant(-1, hfmm.PHASE_M2L)
    tree.set_timing(False)
    # the overlapped product with every P2P variant (launch shape x fork
    # point) forced: the P2P's cost is how it shares the GPU with the far field
    p2p_tuned = tree.variant(a.k, a.P, hfmm.PHASE_P2P)
    p2p_shape_ms = []
    try:
        for v in range(hfmm.variant_count(a.P, hfmm.PHASE_P2P)):
            hfmm.set_variant(v, hfmm.PHASE_P2P)
            for _ in range(2):
                tree.matvec(a.k, a.P, qd, yd)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                tree.matvec(a.k, a.P, qd, yd)
            torch.cuda.synchronize()
            p2p_shape_ms.append(round((time.perf_counter() - t0) / 5 * 1e3, 3))
    finally:
        hfmm.set_variant(-1, hfmm.PHASE_P2P)
    phases = {n: round(v, 4) for n, v in acc.items()}
    log("phases (ms):", phases, "M2L shapes (ms):", shape_ms, "tuned:", tuned,
        "matvec per P2P variant (ms):", p2p_shape_ms, "tuned:", p2p_tuned)
    # the M2L as the kernel computes it (xz-plane form): the C and S blocks,
    # 8 (C^2 + S^2) = 4 P^4 + 4 P^2 FLOP, plus 16 FLOP per m > 0 entry to turn
    # the input by the azimuth phase and 16 per m' > 0 row to turn the output
    P = a.P
    xs = P * (P - 1) // 2
    xc = xs + P
    m2l_flops = (8.0 * (xc * xc + xs * xs) + 32.0 * xs) * st["n_m2l"]
    # what the matrix cores execute: 3 real products (Gauss) per 16-row tile
    # and k-step, the first KSS k-steps on all RTC + RTS tiles, the rest on the
    # RTC tiles of the C block; 2 * 16 * 16 * 4 FLOP each, per 16 pairs
    kss, ksc, rts, rtc = (xs + 3) // 4, (xc + 3) // 4, (xs + 15) // 16, (xc + 15) // 16
    m2l_issued = 3 * (kss * (rtc + rts) + (ksc - kss) * rtc) * 2048 / 16 * st["n_m2l"]
    p2p_flops = 20.0 * st["p2p_body_pairs"]
    m2l_ach = m2l_flops / (phases["m2l"] * 1e-3)
    p2p_ach = p2p_flops / (phases["p2p"] * 1e-3)
    dominant = "m2l" if phases["m2l"] >= phases["p2p"] else "p2p"
    if dominant == "m2l":
        roof = {"kernel": "k_m2l_mfma", "bound": "mfma", "achieved": m2l_ach / 1e12, "peak": PEAK_FP32 / 1e12,
                "unit": "TFLOP/s", "frac": m2l_ach / PEAK_FP32, "traffic": traffic_of(a, "k_m2l_mfma"),
                "per_unit": "4 P^4 + 20 P^2 - 16 P FLOP per M2L pair (the operator turned into the xz-plane: "
                            "C and S blocks of P(P+1)/2 and P(P-1)/2 complex entries squared, plus the "
                            "azimuth turns; FP32 MFMA)",
                "units_per_launch": st["n_m2l"], "launch_ms": phases["m2l"]}
    else:
        roof = {"kernel": "k_p2p", "bound": "alu", "achieved": p2p_ach / 1e12, "peak": PEAK_FP32 / 1e12,
                "unit": "TFLOP/s", "frac": p2p_ach / PEAK_FP32, "traffic": None,
                "per_unit": "20 FLOP per body pair (plus rsqrt, sin, cos)",
                "units_per_launch": st["p2p_body_pairs"], "launch_ms": phases["p2p"]}
    out = {
        "metric": "FMM matvecs/s at 1M pts P=10 (% FP32 peak)",
        "value": 1e3 / ms,
        "unit": "matvec/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"helmholtz FMM matvec, N={a.n} uniform on the unit sphere, k={a.k:.6g} "
                               f"(16 wavelengths across)" + (f" + {a.k_imag:g}i (damped)" if a.k_imag else "") +
                               f", P={a.P}, ncrit={a.ncrit}, theta=0.5, kappa=0.4P",
                   "n": a.n, "k": a.k, "k_imag": a.k_imag, "P": a.P, "ncrit": a.ncrit,
                   **({"stage_mb": a.stage_mb} if a.stage_mb else {})},
        "roofline": roof,
        "phases_ms": phases,
        "secondary": {"p2p_tflops": p2p_ach / 1e12, "p2p_gpairs_per_s": st["p2p_body_pairs"] / phases["p2p"] / 1e6,
                      "m2l_tflops": m2l_ach / 1e12,
                      "m2l_issued_tflops": m2l_issued / (phases["m2l"] * 1e-3) / 1e12,
                      # the same launch counted as the dense P^2 x P^2 operator (8 P^4 per pair)
                      "m2l_dense_equivalent_tflops": 8.0 * P ** 4 * st["n_m2l"] / (phases["m2l"] * 1e-3) / 1e12,
                      "n_m2l": st["n_m2l"], "p2p_body_pairs": st["p2p_body_pairs"],
                      "n_tables": st["n_tables"], "setup_s": {"tree": t_tree, "prepare": t_prep},
                      "m2l_shapes": {"tuned": tuned, "ms": shape_ms},
                      "p2p_variants": {"tuned": p2p_tuned, "matvec_ms": p2p_shape_ms}},
    }
    if not a.no_check and not a.k_imag:
        # the library's FP64 direct sum on the GPU over all sources, 200 targets
        rng = np.random.default_rng(1)
        idx = torch.from_numpy(np.sort(rng.choice(a.n, 200, replace=False))).to(dev)
        xd = torch.from_numpy(x).to(dev)
        ref = hfmm.direct64(xd, qd.to(torch.complex128), xd[idx], a.k)
        y = yd[idx].to(torch.complex128)
        out["secondary"]["rel_err_vs_direct64_200"] = float(torch.linalg.vector_norm(y - ref) /
                                                            torch.linalg.vector_norm(ref))
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
