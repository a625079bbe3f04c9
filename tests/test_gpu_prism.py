"""The many-RHS workload: hexagonal ice prism (circumscribed diameter 1,
length 2.5), 12 divisions per hexagon side and 60 axially (10368 triangles,
15552 edges, 31104 unknowns), k_e = 8, eps_r = 3.17 + 0.01i, 128 right-hand
sides (64 seeded directions x 2 polarisations); A in FP32 applied on the
matrix cores, P = S^i near field (chi = 2 mean edge lengths, q = (1,1,1)).

Checks at full size: sampled entries of the four dense operators against the
oracle; the matrix-core product for all 128 right-hand sides against the
GEMV path of the same context; the 128-RHS batched solve against FP64
single-RHS solves on the GPU for two of the incident fields (cross sections
within 1e-5, the bar for the mixed form); both precisions on the first 4
incident fields against the oracle's exact discrete cross sections (1e-8).
"""

import os

import numpy as np
import pytest

import synth
from gpu_common import note, rel_fro, rel_max
from oracle import operators as ops
from oracle.mesh import Topology

pytestmark = pytest.mark.gpu

EPS = 3.17 + 0.01j
K = 8.0


@pytest.fixture(scope="module")
def P():
    import paper_2008_04772_amd as lib
    return lib


@pytest.fixture(scope="module")
def prism():
    v, t = synth.hex_prism(12, 60)
    return v, t, 2.0 * synth.mean_edge_length(v, t)


def _ctx(P, prism, precision):
    v, t, chi = prism
    ctx = P.Context(0)
    ctx.add_scatterer(v, t, EPS)
    ctx.set_wavenumber(K)
    ctx.assemble(P.assembly_opts((4, 3, 2), 4, -1.0, precision), P.assembly_opts((1, 1, 1), 1, chi, precision),
                 "S_INT")
    return ctx


@pytest.fixture(scope="module")
def mixed(P, prism):
    return _ctx(P, prism, P.MIXED)


def test_prism_entries(P, prism, mixed):
    v, t, _ = prism
    note(f"prism entries: {len(t)} triangles")
    T = Topology(v, t)
    rng = np.random.default_rng(31)
    rows = rng.integers(0, T.E, 300)
    # first half random columns, second half an edge sharing a vertex with the row edge
    vert_edges = {}
    for e, (a, b) in enumerate(T.edges):
        vert_edges.setdefault(a, []).append(e)
        vert_edges.setdefault(b, []).append(e)
    near = [vert_edges[T.edges[i][0]][rng.integers(0, len(vert_edges[T.edges[i][0]]))] for i in rows[150:]]
    cols = np.concatenate([rng.integers(0, T.E, 150), near])
    for med, k in ((P.EXT, K), (P.INT, K * np.sqrt(EPS))):
        ref = ops.rwg_entries(T, k, rows, cols, q=(4, 3, 2), n_sing=4)
        for op, name in ((P.OP_S, "S"), (P.OP_C, "C")):
            err = rel_max(mixed.get_entries(op, med, P.RWG, 0, 0, rows, cols), ref[name])
            note(f"  {name}{'ie'[med == P.EXT]}: max rel {err:.2e}")
            assert err < 1e-4


def test_prism_mfma_apply_128(P, mixed):
    N = 2 * mixed.num_edges(0)
    note(f"prism: matrix-core product, 128 RHS, N = {N}")
    rng = np.random.default_rng(32)
    x = rng.normal(size=(128, N)) + 1j * rng.normal(size=(128, N))
    p0 = mixed.profile()
    y = mixed.apply(0, x)
    p1 = mixed.profile()
    y4 = np.concatenate([mixed.apply(0, x[i:i + 4]) for i in range(0, 128, 4)])
    err = rel_fro(y, y4)
    ms = p1["ms_mfma_total"] - p0["ms_mfma_total"]
    fl = p1["mfma_flops"] - p0["mfma_flops"]
    note(f"  vs GEMV path {err:.2e}; {fl / 1e12:.3f} TFLOP in {ms:.2f} ms = {fl / ms / 1e9:.1f} TFLOP/s")
    assert p1["mfma_launches"] > p0["mfma_launches"]
    assert err < 1e-5


def test_prism_batched_solve_vs_fp64(P, prism, mixed):
    dirs, pols = synth.plane_wave_set(64, seed=3)
    note(f"prism: batched mixed solve of {len(dirs)} RHS")
    so = P.solver_opts(tol=1e-5, restart=200, max_iter=2000, ir_max=2)
    x, st = mixed.solve(dirs, pols, so)
    se, ss = mixed.cross_sections(x, dirs, pols)
    note(f"  iterations {st.iterations}, matvecs {st.matvecs}, {st.ms_solve:.0f} ms")
    ctx64 = _ctx(P, prism, P.FP64)
    so64 = P.solver_opts(tol=1e-5, restart=200, max_iter=2000, ir_max=0)
    for i in (0, 77):
        x64, st64 = ctx64.solve(dirs[i:i + 1], pols[i:i + 1], so64)
        e64, s64 = ctx64.cross_sections(x64, dirs[i:i + 1], pols[i:i + 1])
        note(f"  rhs {i}: ext {se[i]:.8f} / {e64[0]:.8f}, sca {ss[i]:.8f} / {s64[0]:.8f}")
        assert abs(se[i] - e64[0]) < 1e-5 * abs(e64[0])
        assert abs(ss[i] - s64[0]) < 1e-5 * abs(s64[0])


def _golden_sigma():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "prism10368_sigma.txt")
    ext, sca = [], []
    with open(path) as f:
        for line in f:
            if line.startswith("rhs"):
                w = line.split()
                ext.append(float(w[3]))
                sca.append(float(w[5]))
    return np.array(ext), np.array(sca)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_prism_cross_sections_vs_oracle_golden(P, prism, mixed, precision):
    """The first 4 incident fields of the workload (2 directions x 2
    polarisations) solved to tol 1e-10 (MIXED: FP32 operators with the FP64
    refinement residual from the FP64 copy of A; FP64: plain) against the
    oracle's exact discrete cross sections (tests/golden/prism10368_sigma.txt,
    written by tests/golden/make_prism10368.py), bar 1e-8."""
    ext_r, sca_r = _golden_sigma()
    dirs, pols = synth.plane_wave_set(64, seed=3)
    dirs, pols = dirs[:len(ext_r)], pols[:len(ext_r)]
    ctx = mixed if precision == "mixed" else _ctx(P, prism, P.FP64)
    so = P.solver_opts(tol=1e-10, restart=200, max_iter=3000, ir_max=4 if precision == "mixed" else 0)
    x, st = ctx.solve(dirs, pols, so)
    se, ss = ctx.cross_sections(x, dirs, pols)
    e_ext = np.max(np.abs(se - ext_r) / np.abs(ext_r))
    e_sca = np.max(np.abs(ss - sca_r) / np.abs(sca_r))
    note(f"  prism golden, {precision}: iterations {st.iterations}, ir {st.ir_steps}; sigma_ext rel {e_ext:.2e}, "
         f"sigma_sca rel {e_sca:.2e}")
    assert st.converged
    assert e_ext < 1e-8 and e_sca < 1e-8
    if precision == "fp64":
        ctx.close()
