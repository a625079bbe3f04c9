"""Host-side checks of the HIP library (no GPU): it loads, exports every entry
point that include/pmchwt.h declares, and its Buffa-Christiansen construction
(explicit ring fluxes) agrees with the oracle's (conservation system)."""

import os
import re

import numpy as np
import pytest

import synth
from oracle.mesh import Topology, Barycentric

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    try:
        import paper_2008_04772_amd as P
    except ImportError as e:
        pytest.fail(f"library not built: {e}")
    return P


def test_library_exports_every_declared_symbol():
    P = _lib()
    hdr = open(os.path.join(ROOT, "include", "pmchwt.h")).read()
    declared = set(re.findall(r"\b(pmchwt_[a-z_]+)\s*\(", hdr))
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(P._lib, name), name
    assert set(P.EXPORTED) <= declared
    assert "gfx950" in P.pmchwt_version()


@pytest.mark.parametrize("mesh", [synth.icosphere(1), synth.hex_prism(3, 4), synth.cube(2)])
def test_bc_fields_match_oracle(mesh):
    P = _lib()
    e_ids, c_ids, alpha, w = P.pmchwt_bc_fields(*mesh)
    T = Topology(*mesh)
    B = Barycentric(T)
    bt = B.topo
    Bd = B.B.tocsr()
    # every (edge, child) pair of the library appears once and covers the support
    assert len(e_ids) == sum(len(B.support_tris(e)) for e in range(T.E))
    for e, c, a, ww in zip(e_ids, c_ids, alpha, w):
        row = dict(zip(Bd.indices[Bd.indptr[e]:Bd.indptr[e + 1]], Bd.data[Bd.indptr[e]:Bd.indptr[e + 1]]))
        coef = [row.get(bt.t2e[c, k], 0.0) * bt.sign[c, k] for k in range(3)]
        P3 = bt.verts[bt.tris[c]]
        A2 = 2 * bt.area[c]
        a_ref = sum(coef) / A2
        w_ref = sum(cf * p for cf, p in zip(coef, P3)) / A2
        assert abs(a - a_ref) < 1e-12 * max(1, abs(a_ref))
        assert np.allclose(ww, w_ref, atol=1e-12)


def test_bc_fields_reject_open_mesh():
    P = _lib()
    v, t = synth.icosphere(1)
    with pytest.raises(P.PmchwtError):
        P.pmchwt_bc_fields(v, t[1:])
