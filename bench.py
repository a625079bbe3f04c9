#!/usr/bin/env python3
"""Benchmark of the PMCHWT hot path on one MI355X.

Workload: dielectric sphere of radius 1, icosphere with 5120 triangles (7680
RWG edges, 15360 unknowns), k_e = 5, eps_r = 3.17 + 0.01i, one plane wave
along +z polarised along x.  A is assembled densely with q = (4, 3, 2) and
4^4-point Sauter-Schwab rules; the preconditioner is the reduced S^i on the
barycentric mesh, near field only (cutoff 2 mean edge lengths), q = (1,1,1,1);
GMRES(200) to 1e-5.  One step = assemble A, P and the mass matrices, build
the right-hand side, solve, and evaluate the cross sections.

Prints one JSON line.  value = element-pair quadratures per second over the
whole step (ordered triangle pairs x wavenumbers of A, plus barycentric pairs
of P), for the mixed form (FP32 disjoint pairs and operators, FP64 singular
pairs, Arnoldi and refinement).  The plain FP64 form is timed beside it.
"""

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "element-pair quadratures/s + PMCHWT solves/s (mixed vs FP64); p50/p99 latency"
EPS = 3.17 + 0.01j
# algorithmic FP operations per point pair of the regular kernel: 22 shared
# (d, r^2, x.y, x cross y) + 78 per wavenumber (kernel value and gradient
# factor, 14 complex moment updates); transcendental calls count as one
FLOP_SHARED, FLOP_PER_K = 22, 78
PEAK = {"fp32": 157.3, "fp64": 78.6}  # MI355X vector TFLOP/s (FP32 matrix cores: also 157.3)
HBM_PEAK = 8000.0  # GB/s
# HBM bytes per launch of the dense operator product, by (workload, kernel),
# from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB device copy
# (the summaries under profiles/); valid for that kernel version only
GEMV_TRAFFIC = {("sphere5120", "k_gemv_sym3"): 736.6e6}

WORKLOADS = {
    "sphere5120": "dielectric sphere r=1, 5120 triangles (15360 unknowns), k_e=5, eps_r=3.17+0.01i, 1 plane wave; "
                  "A dense q=(4,3,2,6); P = S^i near field chi=2h, q=(1,1,1,1); GMRES(200) tol 1e-5",
    "prism10368": "hexagonal ice prism d=1 l=2.5, 10368 triangles (31104 unknowns), k_e=8, eps_r=3.17+0.01i, "
                  "128 RHS (64 directions x 2 polarisations); A dense q=(4,3,2,6) on the FP32 matrix cores; "
                  "P = S^i near field chi=2h, q=(1,1,1,1); GMRES(200) tol 1e-5",
    "serve200": "serving: seeded Poisson arrivals of requests mixing spheres, single prisms and 2-8-monomer "
                "aggregates of 500-8000 triangles, k_e ~ U[1,10], eps_r=3.17+0.01i, 1-32 directions x 2 "
                "polarisations; mixed precision with one FP64 refinement step, P = S^i near field chi=2h; "
                "GMRES(200) tol 1e-5, at most 500 iterations; Poisson arrivals at 0.8 x the solo request rate of "
                "the first 24 requests, which are also run all at once (saturation)",
}


def workload(name):
    import synth
    if name == "sphere5120":
        v, t = synth.icosphere(4)
        d, p = synth.single_wave()
        k = 5.0
    else:
        v, t = synth.hex_prism(12, 60)
        d, p = synth.plane_wave_set(64, seed=3)
        k = 8.0
    chi = 2.0 * synth.mean_edge_length(v, t)
    return v, t, chi, d, p, k


def run(P, mesh, chi, dirs, pols, k_ext, precision, steps, warmup):
    v, t = mesh
    lat, stats = [], None
    with P.Context(0) as ctx:
        ctx.add_scatterer(v, t, EPS)
        ctx.set_wavenumber(k_ext)
        oA = P.assembly_opts((4, 3, 2), 4, -1.0, P.MIXED if precision == "mixed" else P.FP64)
        oP = P.assembly_opts((1, 1, 1), 1, chi, P.MIXED if precision == "mixed" else P.FP64)
        so = P.solver_opts(tol=1e-5, restart=200, max_iter=2000, ir_max=2 if precision == "mixed" else 0)
        profs = []
        for s in range(warmup + steps):
            t0 = time.perf_counter()
            ctx.assemble(oA, oP, "S_INT")
            x, st = ctx.solve(dirs, pols, so)
            se, ss = ctx.cross_sections(x, dirs, pols)
            dt = time.perf_counter() - t0
            if s >= warmup:
                lat.append(dt)
                profs.append(ctx.profile())
            stats = st
            pf = ctx.profile()
            print(f"[bench] {precision} step {s} {dt * 1e3:.1f} ms, GMRES iters {st.iterations}; wall setup "
                  f"{pf['wall_setup']:.1f} A {pf['wall_A']:.1f} P {pf['wall_P']:.1f} mass {pf['wall_mass']:.1f} "
                  f"solve {st.ms_solve:.1f} xs {(dt * 1e3 - pf['wall_setup'] - pf['wall_A'] - pf['wall_P'] - pf['wall_mass'] - st.ms_solve):.1f}",
                  file=sys.stderr, flush=True)
    return lat, profs, stats, float(se[0]), float(ss[0])


def run_cold(P, mesh, chi, dirs, pols, k_ext, precision, steps):
    """End-to-end latency of a new problem: every step creates a context,
    passes the host mesh, builds every mesh table, assembles, solves and
    evaluates the cross sections, then destroys the context (nothing reused)."""
    v, t = mesh
    lat, phases = [], []
    for s in range(steps):
        t0 = time.perf_counter()
        with P.Context(0) as ctx:
            ctx.add_scatterer(v, t, EPS)
            ctx.set_wavenumber(k_ext)
            oA = P.assembly_opts((4, 3, 2), 4, -1.0, P.MIXED if precision == "mixed" else P.FP64)
            oP = P.assembly_opts((1, 1, 1), 1, chi, P.MIXED if precision == "mixed" else P.FP64)
            so = P.solver_opts(tol=1e-5, restart=200, max_iter=2000, ir_max=2 if precision == "mixed" else 0)
            ctx.assemble(oA, oP, "S_INT")
            x, st = ctx.solve(dirs, pols, so)
            ctx.cross_sections(x, dirs, pols)
            pf = ctx.profile()
        dt = time.perf_counter() - t0
        lat.append(dt)
        ph = {"setup": pf["wall_setup"], "A": pf["wall_A"], "P": pf["wall_P"], "mass": pf["wall_mass"],
              "solve": st.ms_solve, "tables_A": pf["wall_tables_A"], "tables_P": pf["wall_tables_P"], "dual": pf["wall_dual"]}
        phases.append(ph)
        print(f"[bench] {precision} cold step {s} {dt * 1e3:.1f} ms; wall setup {ph['setup']:.1f} A {ph['A']:.1f} "
              f"P {ph['P']:.1f} mass {ph['mass']:.1f} solve {ph['solve']:.1f}; tables A {ph['tables_A']:.2f} "
              f"P {ph['tables_P']:.2f}; dual cells {ph['dual']:.2f}", file=sys.stderr, flush=True)
    return lat, phases


def _prism_sa(F):
    """Divisions (s per hexagon side, a axially) of a prism with about F triangles (F = 12 s a + 12 s^2)."""
    s = max(2, int(round(np.sqrt(F / 60.0))))
    a = max(2, int(round((F / 12.0 - s * s) / s)))
    return s, a


def serve_requests(n, seed=5):
    """Seeded request mix of the serving workload (meshes built before any timing)."""
    import synth
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        kind = int(rng.integers(0, 3))
        F = float(np.exp(rng.uniform(np.log(500.0), np.log(8000.0))))
        k = float(rng.uniform(1.0, 10.0))
        ndir = int(rng.integers(1, 33))
        if kind == 0:
            meshes = [synth.icosphere(3 if F < 2560 else 4)]
        elif kind == 1:
            meshes = [synth.hex_prism(*_prism_sa(F))]
        else:
            nm = int(rng.integers(2, 9))
            meshes = synth.aggregate(nm, *_prism_sa(F / nm), seed=int(rng.integers(1 << 30)))
        dirs, pols = synth.plane_wave_set(ndir, seed=int(rng.integers(1 << 30)))
        v = np.concatenate([m[0] for m in meshes])
        offs = np.cumsum([0] + [len(m[0]) for m in meshes])
        t = np.concatenate([m[1] + offs[i] for i, m in enumerate(meshes)])
        chi = 2.0 * synth.mean_edge_length(v, t)
        out.append({"meshes": meshes, "k": k, "dirs": dirs, "pols": pols, "chi": chi,
                    "F": int(sum(len(m[1]) for m in meshes))})
    return out


def _serve_summary(results, wall, nrhs_of):
    """Throughput and latency of one serving run; only converged requests count as solves."""
    ok = [r for r in results if r["status"] == 0]
    nc = [r for r in results if r["status"] == -5]
    lat_ok = np.array([r["ms_total"] for r in ok]) if ok else np.array([np.nan])
    lat_nc = np.array([r["ms_total"] for r in nc]) if nc else np.array([np.nan])
    return {
        "wall_s": wall, "requests": len(results), "converged": len(ok), "not_converged": len(nc),
        "failed": len(results) - len(ok) - len(nc),
        "rhs_solves_converged": int(sum(nrhs_of(r) for r in ok)),
        "rhs_solves_per_s": float(sum(nrhs_of(r) for r in ok)) / wall,
        "requests_per_s": len(ok) / wall,
        "latency_ms_p50": float(np.percentile(lat_ok, 50)), "latency_ms_p99": float(np.percentile(lat_ok, 99)),
        "not_converged_latency_ms_p50": float(np.percentile(lat_nc, 50)),
    }


def run_serve(P, n_requests, budget_gb=200, max_live=16, n_sat=24):
    """Three passes over the seeded request mix on one server: (1) the first
    n_sat requests one at a time (solo), (2) the same requests all submitted at
    t = 0 (saturation: the batching gain is solo time / saturated time), (3) all
    n_requests with Poisson arrivals at 0.8 x the solo request rate."""
    import threading
    reqs = serve_requests(n_requests)
    oA = P.assembly_opts((4, 3, 2), 4, -1.0, P.MIXED)
    # at most 500 iterations: meshes under-resolved at high k stop there
    # (status NOT_CONVERGED, reported apart and not counted as solves)
    so = P.solver_opts(tol=1e-5, restart=200, max_iter=500, ir_max=1)

    def submit(srv, r):
        oP = P.assembly_opts((1, 1, 1), 1, r["chi"], P.MIXED)
        return srv.submit(r["meshes"], EPS, r["k"], r["dirs"], r["pols"], oA, oP, "S_INT", so)

    def nrhs_of(res):
        return res["nrhs"]

    n_sat = min(n_sat, n_requests)
    with P.Server(0, budget_gb << 30, max_live) as srv:
        # (1) solo
        solo_res = []
        t0 = time.perf_counter()
        for r in reqs[:n_sat]:
            tk = submit(srv, r)
            solo_res.append(srv.wait(tk))
            srv.fetch(tk)
        solo_wall = time.perf_counter() - t0
        solo = solo_wall / n_sat
        print(f"[bench] serve solo: {n_sat} requests one at a time in {solo_wall:.1f} s", file=sys.stderr, flush=True)
        # (2) saturation
        t0 = time.perf_counter()
        tks = [submit(srv, r) for r in reqs[:n_sat]]
        sat_res = []
        for tk in tks:
            sat_res.append(srv.wait(tk))
            srv.fetch(tk)
        sat_wall = time.perf_counter() - t0
        print(f"[bench] serve saturation: the same {n_sat} requests at once in {sat_wall:.1f} s", file=sys.stderr,
              flush=True)
        # (3) Poisson arrivals
        lam = 0.8 / solo
        s0 = srv.stats()
        rng = np.random.default_rng(5)
        arrivals = np.cumsum(rng.exponential(1.0 / lam, n_requests))
        tickets = [None] * n_requests

        def feeder():
            base = time.perf_counter()
            for i, r in enumerate(reqs):
                dt = arrivals[i] - (time.perf_counter() - base)
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = submit(srv, r)

        t1 = time.perf_counter()
        th = threading.Thread(target=feeder)
        th.start()
        results = []
        for i in range(n_requests):
            while tickets[i] is None:
                time.sleep(0.001)
            res = srv.wait(tickets[i])
            srv.fetch(tickets[i])
            results.append(res)
            if (i + 1) % 20 == 0:
                print(f"[bench] serve: {i + 1}/{n_requests} done", file=sys.stderr, flush=True)
        th.join()
        wall = time.perf_counter() - t1
        s1 = srv.stats()
    out = {
        "poisson": _serve_summary(results, wall, nrhs_of),
        "solo": _serve_summary(solo_res, solo_wall, nrhs_of),
        "saturation": _serve_summary(sat_res, sat_wall, nrhs_of),
        "saturation_speedup_vs_solo": solo_wall / sat_wall,
        "arrival_rate_per_s": lam, "solo_ms_per_request": solo * 1e3,
        "max_live_seen": s1["max_live_seen"], "grouped_launches": s1["grouped_launches"] - s0["grouped_launches"],
        "grouped_jobs": s1["grouped_jobs"] - s0["grouped_jobs"], "rounds": s1["rounds"] - s0["rounds"],
        "triangles_mean": float(np.mean([r["F"] for r in reqs])),
    }
    return out


def _pair_sample_worker(args):
    """One process of the CPU baseline: the oracle's quadrature sums on seeded
    random ordered triangle pairs for budget_s seconds (one thread)."""
    mesh, k_ext, seed, budget_s = args
    from threadpoolctl import threadpool_limits
    from oracle.mesh import Topology
    from oracle import operators as ops
    T = Topology(*mesh)
    rng = np.random.default_rng(seed)
    k_i = k_ext * np.sqrt(EPS)
    done, t_used, n_pairs = 0, 0.0, 0
    with threadpool_limits(1):
        geom = ops._tri_geom(T)
        while t_used < budget_s:
            t1 = rng.integers(0, T.F, 2000)
            t2 = rng.integers(0, T.F, 2000)
            rel = ops.classify(T, t1, t2, geom)
            t0 = time.perf_counter()
            for c in np.unique(rel):
                sel = rel == c
                for k in (k_ext, k_i):
                    ops.local_blocks(T, t1[sel], t2[sel], int(c), k)
            t_used += time.perf_counter() - t0
            done += 2 * len(t1)
            n_pairs += len(t1)
    return done, t_used, n_pairs


def cpu_baseline(mesh, k_ext, budget_s=12.0):
    """The oracle (plain FP64 NumPy, untuned) on the host's cores (at most 16,
    the host share of one GPU): element-pair quadrature rate on a seeded
    sample of the workload's ordered triangle pairs, one process per core;
    and the end-to-end time of the oracle's dense solve of the 320-triangle
    sphere (assembly over all cores, direct solve, cross sections)."""
    import multiprocessing as mp
    import synth
    from oracle import parallel
    from oracle import pmchwt as opm
    from oracle.mesh import Topology
    cores = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_pair_sample_worker, [(mesh, k_ext, 11 + w, budget_s) for w in range(cores)])
    wall = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    n_pairs = sum(r[2] for r in res)
    per_core = sum(r[0] / r[1] for r in res) / cores
    # 320-triangle sphere, k_e = 1: the small workload end to end
    t1 = time.perf_counter()
    m1 = synth.icosphere(2)
    d, p = synth.single_wave()
    pr = opm.Problem([m1], EPS, 1.0)
    pr.assemble_A(parallel.parallel_assembler(cores))
    x = pr.solve_direct(pr.rhs(d, p))
    pr.cross_sections(x, d, p)
    t_c1 = time.perf_counter() - t1
    return {"value": done / wall, "unit": "element-pair quadratures/s", "cores": cores, "kind": "oracle",
            "per_core": per_core, "sphere320_end_to_end_s": t_c1,
            "sample": f"{n_pairs} seeded random ordered triangle pairs of the workload mesh "
                      f"({Topology(*mesh).F} triangles), both wavenumbers, q = (4,3,2) and 4^4 Sauter-Schwab points, "
                      f"{cores} processes x {budget_s:.0f} s; plus the oracle's dense solve of the 320-triangle "
                      f"sphere (assembly on {cores} processes, direct solve, cross sections)"}


def copy_calibration():
    """A plain device-to-device copy of 1 GiB (HIP runtime blit kernel, called
    through ctypes) whose HBM counters calibrate those of the library's
    kernels."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipMemset.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t]
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    n = 1 << 30
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    if hip.hipMalloc(ctypes.byref(a), n) != 0 or hip.hipMalloc(ctypes.byref(b), n) != 0:
        raise RuntimeError("hipMalloc failed")
    try:
        if hip.hipMemset(a, 1, n) != 0:
            raise RuntimeError("hipMemset failed")
        for _ in range(3):
            if hip.hipMemcpy(b, a, n, 3) != 0:  # device to device
                raise RuntimeError("hipMemcpy failed")
        hip.hipDeviceSynchronize()
    finally:
        hip.hipFree(a)
        hip.hipFree(b)
    print(f"[bench] copy calibration: 3 x {n} bytes", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cold-steps", type=int, default=2,
                    help="steps on a fresh context each (end-to-end latency of a new problem), after the timed ones")
    ap.add_argument("--precision", choices=["both", "mixed", "fp64"], default="both")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="sphere5120",
                    help="sphere5120: the benchmark workload; prism10368: the 128-RHS workload")
    ap.add_argument("--requests", type=int, default=200, help="requests of the serving workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="finish with a plain 1 GiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import paper_2008_04772_amd as P
    if args.workload == "serve200":
        sv = run_serve(P, args.requests)
        pz = sv["poisson"]
        out = {"metric": METRIC, "value": pz["rhs_solves_per_s"], "unit": "PMCHWT solves/s (converged RHS)",
               "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": pz["wall_s"] * 1e3, "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "fp32+fp64", "data": "synthetic",
               "config": {"workload": WORKLOADS["serve200"], "requests": args.requests},
               "requests_per_s": pz["requests_per_s"],
               "latency_ms_p50": pz["latency_ms_p50"], "latency_ms_p99": pz["latency_ms_p99"], "serve": sv}
        print(json.dumps(out), flush=True)
        return
    v, t, chi, dirs, pols, k_ext = workload(args.workload)
    results = {}
    for prec in (["mixed", "fp64"] if args.precision == "both" else [args.precision]):
        results[prec] = run(P, (v, t), chi, dirs, pols, k_ext, prec, args.steps, args.warmup)
    head = "mixed" if "mixed" in results else "fp64"
    lat, profs, st, se, ss = results[head]
    pr = profs[-1]
    quads = 2 * (pr["regular_pairs"] + pr["singular_pairs"]) + pr["bary_pairs"]
    ms = 1e3 * statistics.mean(lat)
    value = quads / (ms / 1e3)
    # dominant kernel: the regular-pair assembly kernel, the dense operator
    # GEMV or the matrix-core product, by total time per step
    reg_total = statistics.mean(p["ms_assemble_regular"] for p in profs)
    # one GEMV launch in eight is timed (matvec_timed of matvec_launches)
    gemv_per = [(p["ms_matvec_total"] - p["ms_mfma_total"]) / max(1, p["matvec_timed"]) for p in profs]
    gemv_total = statistics.mean(g * p["matvec_launches"] for g, p in zip(gemv_per, profs))
    mfma_total = statistics.mean(p["ms_mfma_total"] for p in profs)
    dtype_reg = "fp32" if head == "mixed" else "fp64"
    dom = max((reg_total, "reg"), (gemv_total, "gemv"), (mfma_total, "mfma"))[1]
    if dom == "reg":
        flops = (pr["regular_point_pairs"] / 2) * (FLOP_SHARED + 2 * FLOP_PER_K) / pr["regular_launches"]
        ach = flops / (reg_total / pr["regular_launches"] * 1e-3) / 1e12
        roof = {"kernel": "k_regular_rows", "bound": "alu", "achieved": ach, "peak": PEAK[dtype_reg],
                "unit": "TFLOP/s", "frac": ach / PEAK[dtype_reg], "traffic": None}
    elif dom == "gemv":
        per = statistics.mean(gemv_per)
        byt = pr["matvec_bytes"] / max(1, pr["matvec_launches"])
        ach = byt / (per * 1e-3) / 1e9
        # one right-hand side on one scatterer of 4096+ edges: the symmetric
        # tiles (their reduction kernel is timed apart and not counted here)
        kname = "k_gemv_sym3" if pr["ms_matvec_reduce"] > 0 else "k_gemv_pmchwt3"
        traffic = GEMV_TRAFFIC.get((args.workload, kname)) if head == "mixed" else None
        roof = {"kernel": kname, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK, "unit": "GB/s",
                "frac": ach / HBM_PEAK, "traffic": traffic}
    else:
        fl = statistics.mean(p["mfma_flops"] for p in profs)
        ach = fl / (mfma_total * 1e-3) / 1e12
        roof = {"kernel": "k_mfma_pmchwt", "bound": "mfma", "achieved": ach, "peak": PEAK["fp32"], "unit": "TFLOP/s",
                "frac": ach / PEAK["fp32"], "traffic": None}
    out = {
        "metric": METRIC, "value": value, "unit": "element-pair quadratures/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32+fp64" if head == "mixed" else "fp64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "triangles": int(len(t)), "unknowns": int(3 * len(t)),
                   "n_rhs": int(len(dirs))},
        "solves_per_s": len(dirs) * 1e3 / ms,
        "latency_ms_p50": 1e3 * float(np.percentile(lat, 50)),
        "latency_ms_p99": 1e3 * float(np.percentile(lat, 99)),
        "quadratures_per_step": quads,
        "gmres_iterations": st.iterations,
        "assembly_ms": {"A": pr["ms_assemble_A"], "regular": pr["ms_assemble_regular"],
                        "singular": pr["ms_assemble_singular"], "P": pr["ms_assemble_P"], "mass": pr["ms_mass"]},
        "solve_ms": st.ms_solve,
        "fp64_products_ms": {"total": pr["ms_free_apply"], "launches": pr["free_launches"],
                             "note": "matrix-free FP64 A^i c_inc (right-hand side) and A x (refinement residuals)"},
        "sigma_ext_rhs0": se, "sigma_sca_rhs0": ss,
        "roofline": roof,
    }
    if args.cold_steps > 0:
        cl, cph = run_cold(P, (v, t), chi, dirs, pols, k_ext, head, args.cold_steps)
        out["cold"] = {"ms_per_step": 1e3 * statistics.mean(cl), "steps": args.cold_steps,
                       "phases_wall_ms_last": cph[-1],
                       "note": "new context per step: mesh tables (tables_A, tables_P: the classification kernels with their read-backs and the host layout work; dual: barycentric refinement and dual-cell upload), allocations, assembly, solve, cross sections"}
    if "fp64" in results and head == "mixed":
        l64 = results["fp64"][0]
        out["fp64"] = {"ms_per_step": 1e3 * statistics.mean(l64),
                       "quadratures_per_s": quads / statistics.mean(l64),
                       "assembly_regular_ms": results["fp64"][1][-1]["ms_assemble_regular"],
                       "sigma_ext_rhs0": results["fp64"][3]}
        out["mixed_speedup"] = statistics.mean(l64) / statistics.mean(lat)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline((v, t), k_ext)
    if args.copy_calibration:
        copy_calibration()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
