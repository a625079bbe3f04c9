"""Classification tables built on the device (Section 3.3: regular pairs by
distance class, singular pairs, the near-field cutoff of P) against counts
the oracle derives from its own classification:

- regular ordered pairs per class and their rule point pairs (oracle
  ``classify`` over every pair of the union of the meshes);
- singular ordered pairs (triangles sharing a vertex) and their Sauter-Schwab
  point pairs;
- the kept entries of P (``nearfield_mask`` on the BC support boxes, per
  scatterer, or over the union when the preconditioner couples scatterers);
- the barycentric pairs of the dual-cell tables: 4 N_v N_w for every pair of
  dual cells (v, w) joined by a kept entry, N_v the number of edges at v.

Integer counts: exact.  The entries themselves are checked against the
oracle's blocks by the P and A parity tests, which read the same tables."""

import numpy as np
import pytest

import synth
from gpu_common import note, make_ctx
from oracle import mesh as om
from oracle import operators as ops
from oracle import quadrature as quad

pytestmark = pytest.mark.gpu

EPS = 3.17 + 0.01j
NPTS = {q: len(quad.triangle_rule(q)[1]) for q in (1, 2, 3, 4)}


@pytest.fixture(scope="module")
def P():
    import paper_2008_04772_amd as lib
    return lib


def _union(meshes):
    vs, ts, off = [], [], 0
    for v, t in meshes:
        vs.append(np.asarray(v, dtype=np.float64))
        ts.append(np.asarray(t, dtype=np.int64) + off)
        off += len(v)
    return om.Topology(np.concatenate(vs), np.concatenate(ts))


def oracle_counts(meshes, qA, nA, chi, cross):
    U = _union(meshes)
    F = U.F
    geom = ops._tri_geom(U)
    t1, t2 = np.meshgrid(np.arange(F), np.arange(F), indexing="ij")
    rel = ops.classify(U, t1.ravel(), t2.ravel(), geom)
    pts_of = {0: NPTS[qA[0]] ** 2, -1: NPTS[qA[1]] ** 2, -2: NPTS[qA[2]] ** 2}
    ss = {k: len(quad.sauter_schwab(k, nA)[2]) for k in (1, 2, 3)}
    out = {"regular_pairs": int((rel <= 0).sum()),
           "regular_point_pairs": int(sum(pts_of[c] * int((rel == c).sum()) for c in (0, -1, -2))),
           "singular_pairs": int((rel > 0).sum()),
           "singular_point_pairs": int(sum(ss[k] * int((rel == k).sum()) for k in (1, 2, 3)))}
    # near-field pattern and dual-cell pairs
    tops = [om.Topology(v, t) for v, t in meshes]
    boxes = [ops.bc_bboxes(om.Barycentric(T)) for T in tops]
    cells, deg, eoff, voff = [], [], 0, 0
    for T in tops:
        cells.append(T.edges + voff)
        deg.append(np.bincount(T.edges.ravel(), minlength=T.nv))
        voff += T.nv
    cells, deg = np.concatenate(cells), np.concatenate(deg)
    E = len(cells)
    keep = np.zeros((E, E), dtype=bool)
    if cross:
        lo = np.concatenate([b[0] for b in boxes])
        hi = np.concatenate([b[1] for b in boxes])
        keep[:] = ops.nearfield_mask(lo, hi, chi)
    else:
        for T, (lo, hi) in zip(tops, boxes):
            keep[eoff:eoff + T.E, eoff:eoff + T.E] = ops.nearfield_mask(lo, hi, chi)
            eoff += T.E
    ii, jj = np.nonzero(keep)
    cp = set()
    for a in (0, 1):
        for b in (0, 1):
            cp.update(zip(cells[ii, a].tolist(), cells[jj, b].tolist()))
    out["nnz_P"] = int(keep.sum())
    out["bary_pairs"] = int(sum(4 * int(deg[v]) * int(deg[w]) for v, w in cp))
    return out


CASES = [
    ("sphere320 chi=2h", lambda: [synth.icosphere(2)], 2.0, "S_INT"),
    ("sphere320 chi=0", lambda: [synth.icosphere(2)], 0.0, "S_INT"),
    ("sphere320 chi=inf", lambda: [synth.icosphere(2)], -1.0, "S_INT"),
    ("prism chi=3h", lambda: [synth.hex_prism(2, 3)], 3.0, "D_INT"),
    ("two prisms chi=2h, blocks", lambda: synth.aggregate(2, 2, 3, seed=7), 2.0, "S_INT"),
    ("two prisms chi=2h, coupled", lambda: synth.aggregate(2, 2, 3, seed=7), 2.0, "A"),
]


@pytest.mark.parametrize("name,build,chi_h,precond", CASES, ids=[c[0] for c in CASES])
def test_device_classification_counts(P, name, build, chi_h, precond):
    meshes = build()
    h = np.mean([synth.mean_edge_length(v, t) for v, t in meshes])
    chi = -1.0 if chi_h < 0 else chi_h * h
    qA, nA = (4, 3, 2), 3
    ctx = make_ctx(P, meshes, EPS, 2.0, qA=qA, nA=nA, qP=(1, 1, 1), nP=1, chi=chi, precond=precond)
    prof = ctx.profile()
    ctx.close()
    cross = precond == "A" and len(meshes) > 1
    want = oracle_counts(meshes, qA, nA, np.inf if chi < 0 else chi, cross)
    got = {k: int(prof[k]) for k in want}
    note(f"  {name}: {got}")
    assert got == want


def test_reassembly_reuses_identical_tables(P):
    """A second assembly on the same context (tables cached) and a fresh
    context (tables rebuilt) give bitwise-equal operators: every entry of A
    and of the near-field P is summed by one thread in a fixed order."""
    meshes = [synth.icosphere(2)]
    chi = 2.0 * synth.mean_edge_length(*meshes[0])
    a = make_ctx(P, meshes, EPS, 2.0, qP=(1, 1, 1), nP=1, chi=chi, precond="S_INT")
    b = make_ctx(P, meshes, EPS, 2.0, qP=(1, 1, 1), nP=1, chi=chi, precond="S_INT")
    b.assemble(P.assembly_opts((4, 3, 2), 4, -1.0, 0), P.assembly_opts((1, 1, 1), 1, chi, 0), "S_INT")
    assert a.profile()["nnz_P"] == b.profile()["nnz_P"]
    # S^i on BC: the one operator of this preconditioner; both RWG operators
    for op, sp, med in ((P.OP_S, P.BC, P.INT), (P.OP_S, P.RWG, P.EXT), (P.OP_C, P.RWG, P.EXT),
                        (P.OP_S, P.RWG, P.INT), (P.OP_C, P.RWG, P.INT)):
        x = a.get_block(op, med, sp, 0, 0)
        y = b.get_block(op, med, sp, 0, 0)
        assert np.array_equal(x, y), (op, med, sp)
    assert np.array_equal(a.get_mass(0), b.get_mass(0))
    a.close()
    b.close()
