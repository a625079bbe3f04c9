"""Run-to-run reproducibility: two contexts built from the same input give
bitwise-equal operators, mass matrices, currents and cross sections.

Every floating-point sum of the path has one writer per output and a fixed
order: the regular pairs' row combine, the singular pairs' scatter over their
entry tables (pair, then local entry), the near-field P's per-entry gather of
its four cell-pair slots, the mass matrix per entry over the children of
T+ then T-, and the solver's reductions in fixed trees.  Sums of at most two
addends onto zero (the right-hand side and the RWG Gram matrix: every edge
has two triangles) do not depend on their order.  So nothing here is compared
with a tolerance."""

import numpy as np
import pytest

import synth
from gpu_common import note

pytestmark = pytest.mark.gpu

EPS = 3.17 + 0.01j


@pytest.fixture(scope="module")
def P():
    import paper_2008_04772_amd as lib
    return lib


def _build(P, meshes, k, precision, precond, chi):
    ctx = P.Context(0)
    for v, t in meshes:
        ctx.add_scatterer(v, t, EPS)
    ctx.set_wavenumber(k)
    ctx.assemble(P.assembly_opts((4, 3, 2), 3, -1.0, precision),
                 P.assembly_opts((2, 1, 1), 2, chi, precision), precond)
    return ctx


def _blocks(P, ctx, nsc):
    out = {}
    for op in (P.OP_S, P.OP_C):
        for m in range(nsc):
            for l in range(nsc):
                out[("ext", op, m, l)] = ctx.get_block(op, P.EXT, P.RWG, m, l)
            out[("int", op, m)] = ctx.get_block(op, P.INT, P.RWG, m, m)
            for med in (P.EXT, P.INT):  # the BC blocks of P that this preconditioner holds
                try:
                    out[("bc", op, med, m)] = ctx.get_block(op, med, P.BC, m, m)
                except P.PmchwtError:
                    pass
        for m in range(nsc):
            out[("mass", m)] = ctx.get_mass(m)
    return out


CASES = [
    ("sphere1280 mixed S_INT", lambda: [synth.icosphere(3)], 3.0, 1, "S_INT", 2.0, 2),
    ("sphere1280 fp64 D", lambda: [synth.icosphere(3)], 3.0, 0, "D", 2.0, 0),
    ("two prisms fp64 A coupled", lambda: synth.aggregate(2, 2, 3, seed=7), 2.0, 0, "A", 2.0, 0),
]


@pytest.mark.parametrize("name,build,k,precision,precond,chi_h,ir", CASES, ids=[c[0] for c in CASES])
def test_two_runs_bitwise_equal(P, name, build, k, precision, precond, chi_h, ir):
    meshes = build()
    h = np.mean([synth.mean_edge_length(v, t) for v, t in meshes])
    d, p = synth.plane_wave_set(2, seed=5)
    note(f"determinism: {name}")
    res = []
    for run in range(2):
        ctx = _build(P, meshes, k, precision, precond, chi_h * h)
        blocks = _blocks(P, ctx, len(meshes))
        x, st = ctx.solve(d, p, P.solver_opts(tol=1e-8, restart=100, max_iter=1000, ir_max=ir))
        assert st.converged
        xs = ctx.cross_sections(x, d, p)
        res.append((blocks, x, xs, st.iterations))
        ctx.close()
    (b0, x0, s0, it0), (b1, x1, s1, it1) = res
    assert b0.keys() == b1.keys()
    assert any(key[0] == "bc" for key in b0), "no BC block of P was returned"
    for key in b0:
        assert np.array_equal(b0[key], b1[key]), key
    assert it0 == it1
    assert np.array_equal(x0, x1)
    for a, b in zip(s0, s1):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    note(f"  {len(b0)} blocks, {it0} iterations: bitwise equal")
