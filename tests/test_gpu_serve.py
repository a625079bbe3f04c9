"""Serving loop (pmchwt_server_*): admission by device-memory budget,
continuous batching of Krylov steps across live requests, and results that
do not depend on the mix.

Tolerances: a request's currents in a mix against the same request served
alone, 1e-9 relative for FP64 operators and 1e-5 for FP32 operators (the
mixed form's bar).  The grouped products compute every request's rows with
the same code and order as a launch of that request alone; what differs
between two assemblies of the same problem is the order of the few atomic
additions per entry in the singular and near-field kernels (last bits of an
entry), which GMRES carries into the solution at up to ~1e-11 (FP64) over
many unpreconditioned iterations; the measured differences are reported.
Served results against pmchwt_solve on a context with the same options: the
same bars.  A served FP64 solve against the oracle's direct solve: 1e-9.
"""

import numpy as np
import pytest

import synth
from gpu_common import note, rel_fro
from oracle import pmchwt as opm

pytestmark = pytest.mark.gpu

EPS = 3.17 + 0.01j


@pytest.fixture(scope="module")
def P():
    import paper_2008_04772_amd as lib
    return lib


def _requests(P):
    """Mixed request set: sizes, precisions, preconditioners and RHS counts
    differ; one uses the matrix-core path (20 RHS)."""
    so = P.solver_opts(tol=1e-8, restart=200, max_iter=1000, ir_max=2)
    nf = P.assembly_opts((1, 1, 1), 1, 0.5, P.MIXED)
    reqs = {
        "sphere2_mixed": ([synth.icosphere(2)], EPS, 2.0, synth.plane_wave_set(2, seed=5),
                          P.assembly_opts((4, 3, 2), 4, -1.0, P.MIXED), nf, "S_INT", so),
        "sphere3_fp64": ([synth.icosphere(3)], EPS, 3.0, synth.single_wave(),
                         P.assembly_opts((4, 3, 2), 4, -1.0, P.FP64), P.assembly_opts((1, 1, 1), 1, 0.3, P.FP64),
                         "S_INT", P.solver_opts(tol=1e-10, restart=200, max_iter=1000)),
        "cubes_mixed": (synth.three_cubes(2.1), 1.311 ** 2 + 0j, 2.1, synth.plane_wave_set(3, seed=6),
                        P.assembly_opts((4, 3, 2), 4, -1.0, P.MIXED), P.assembly_opts((4, 3, 2), 4, -1.0, P.MIXED),
                        "D", so),
        "prism_mfma": ([synth.hex_prism(3, 8)], EPS, 4.0, synth.plane_wave_set(10, seed=7),
                       P.assembly_opts((4, 3, 2), 4, -1.0, P.MIXED), nf, "S_INT", so),
        "sphere1_fp64_I": ([synth.icosphere(1)], EPS, 1.0, synth.single_wave(),
                           P.assembly_opts((4, 3, 2), 4, -1.0, P.FP64), P.assembly_opts((4, 3, 2), 4, -1.0, P.FP64),
                           "I", P.solver_opts(tol=1e-10, restart=100, max_iter=1000)),
    }
    return reqs


def _submit(srv, r):
    meshes, eps, k, (d, p), oA, oP, pc, so = r
    return srv.submit(meshes, eps, k, d, p, oA, oP, pc, so)


def _solve_ctx(P, r):
    meshes, eps, k, (d, p), oA, oP, pc, so = r
    ctx = P.Context(0)
    for v, t in meshes:
        ctx.add_scatterer(v, t, eps)
    ctx.set_wavenumber(k)
    ctx.assemble(oA, oP, pc)
    x, st = ctx.solve(d, p, so)
    se, ss = ctx.cross_sections(x, d, p)
    return x, se, ss


def test_serve_alone_vs_mix_and_vs_context(P):
    reqs = _requests(P)
    alone = {}
    with P.Server(0, 64 << 30, 8) as srv:
        for name, r in reqs.items():
            t = _submit(srv, r)
            res = srv.wait(t)
            assert res["status"] == 0, (name, res)
            alone[name] = srv.fetch(t)
        s0 = srv.stats()
        note(f"alone: rounds {s0['rounds']}, grouped launches {s0['grouped_launches']} jobs {s0['grouped_jobs']}")
        # the same requests all at once, one of them twice
        tickets = [(name, _submit(srv, r)) for name, r in reqs.items()]
        tickets.append(("sphere2_mixed", _submit(srv, reqs["sphere2_mixed"])))
        mix = []
        for name, t in tickets:
            res = srv.wait(t)
            assert res["status"] == 0, (name, res)
            mix.append((name, srv.fetch(t), res))
        s1 = srv.stats()
    note(f"mix: max live {s1['max_live_seen']}, grouped launches {s1['grouped_launches'] - s0['grouped_launches']}, "
         f"jobs {s1['grouped_jobs'] - s0['grouped_jobs']}")
    assert s1["max_live_seen"] >= 3
    assert (s1["grouped_jobs"] - s0["grouped_jobs"]) > (s1["grouped_launches"] - s0["grouped_launches"])
    for name, (x, se, ss), res in mix:
        xa, sea, ssa = alone[name]
        tol = 1e-9 if "fp64" in name else 1e-5
        e = rel_fro(x, xa)
        note(f"  {name}: mix vs alone {e:.2e} (bit-identical: {np.array_equal(x, xa)}), "
             f"queued {res['ms_queued']:.1f} ms, total {res['ms_total']:.1f} ms, iters {res['iterations']}")
        assert e <= tol
        assert np.allclose(se, sea, rtol=tol, atol=0) and np.allclose(ss, ssa, rtol=tol, atol=0)
    for name, r in reqs.items():
        x, se, ss = _solve_ctx(P, r)
        xa, sea, ssa = alone[name]
        tol = 1e-9 if "fp64" in name else 1e-5
        e = rel_fro(xa, x)
        note(f"  {name}: served vs context solve {e:.2e}")
        assert e <= tol


def test_serve_fp64_against_oracle(P):
    mesh = synth.icosphere(1)
    d, p = synth.plane_wave_set(2, seed=8)
    with P.Server(0, 8 << 30, 2) as srv:
        t = srv.submit([mesh], EPS, 1.3, d, p, P.assembly_opts((4, 3, 2), 4, -1.0, P.FP64),
                       P.assembly_opts((4, 3, 2), 4, -1.0, P.FP64), "D",
                       P.solver_opts(tol=1e-12, restart=200, max_iter=500))
        res = srv.wait(t)
        x, se, ss = srv.fetch(t)
    pr = opm.Problem([mesh], EPS, 1.3)
    pr.assemble_A()
    xr = pr.solve_direct(pr.rhs(d, p))
    se_r, ss_r = pr.cross_sections(xr, d, p)
    note(f"served vs oracle: {rel_fro(x, xr):.2e}, iters {res['iterations']}")
    assert res["status"] == 0
    assert rel_fro(x, xr) < 1e-9
    assert np.allclose(se, se_r, rtol=1e-8) and np.allclose(ss, ss_r, rtol=1e-8)


def test_serve_budget_errors_and_cancel(P):
    v, t = synth.icosphere(2)
    oA = P.assembly_opts((4, 3, 2), 4, -1.0, P.MIXED)
    oP = P.assembly_opts((1, 1, 1), 1, 0.5, P.MIXED)
    d, p = synth.single_wave()
    with P.Server(0, 1 << 20, 4) as srv:  # 1 MiB: nothing fits
        with pytest.raises(P.PmchwtError) as e:
            srv.submit([(v, t)], EPS, 2.0, d, p, oA, oP)
        assert e.value.code == P.ERR_OVER_BUDGET
    with P.Server(0, 32 << 30, 1) as srv:
        with pytest.raises(P.PmchwtError) as e:  # odd triangle count: not a closed surface
            srv.submit([(v, t[:-1])], EPS, 2.0, d, p, oA, oP)
        assert e.value.code == P.ERR_INVALID_MESH
        # a mesh that passes the submission checks but not the topology check
        bad = np.concatenate([t, t[:2]])
        tb = srv.submit([(v, bad)], EPS, 2.0, d, p, oA, oP)
        big = srv.submit([synth.icosphere(3)], EPS, 3.0, d, p, oA, oP)
        queued = [srv.submit([(v, t)], EPS, 2.0, d, p, oA, oP) for _ in range(3)]
        srv.cancel(queued[1])
        rb = srv.wait(tb)
        rbig = srv.wait(big)
        rq = [srv.wait(q) for q in queued]
        note(f"bad mesh status {rb['status']}, big {rbig['status']}, queued {[r['status'] for r in rq]}")
        assert rb["status"] == P.ERR_INVALID_MESH
        assert rbig["status"] == 0
        assert rq[1]["status"] == P.ERR_CANCELLED
        assert rq[0]["status"] == 0 and rq[2]["status"] == 0
