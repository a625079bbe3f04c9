"""Pins of the oracle's mesh topology, RWG and BC functions (no GPU)."""

import numpy as np
import pytest

import synth
from oracle.mesh import Topology, Barycentric
from oracle import operators as ops


@pytest.mark.parametrize("mesh", [synth.icosphere(2), synth.hex_prism(3, 5), synth.cube(3)])
def test_topology_euler_and_counts(mesh):
    T = Topology(*mesh)
    assert 2 * T.E == 3 * T.F
    assert T.nv - T.E + T.F == 2
    # outward normals: divergence theorem, sum n A = 0 and volume > 0
    assert np.linalg.norm((T.normal * T.area[:, None]).sum(axis=0)) < 1e-12
    vol = np.sum(T.area * np.einsum("ij,ij->i", T.normal, T.verts[T.tris[:, 0]])) / 3.0
    assert vol > 0


def test_topology_rejects_bad_meshes():
    v, t = synth.icosphere(1)
    with pytest.raises(ValueError):
        Topology(v, t[1:])                       # open
    bad = t.copy()
    bad[0] = bad[0][[0, 2, 1]]
    with pytest.raises(ValueError):
        Topology(v, bad)                         # inconsistent orientation


def test_rwg_unit_flux_and_normal_continuity():
    T = Topology(*synth.icosphere(1))
    for e in range(0, T.E, 7):
        lo, hi = T.verts[T.edges[e]]
        mid = 0.5 * (lo + hi)
        L = np.linalg.norm(hi - lo)
        flux = []
        for t in (T.tplus[e], T.tminus[e]):
            a = int(np.nonzero(T.t2e[t] == e)[0][0])
            nu = np.cross(hi - lo, T.normal[T.tplus[e]] if t == T.tplus[e] else T.normal[t])
            nu /= np.linalg.norm(nu)
            f = T.rwg_on(t, a, mid[None, :])[0]
            flux.append(f @ nu * L)
        # lo->hi is counter-clockwise in T+, so (hi-lo) x n points out of T+ into T-
        assert abs(flux[0] - 1.0) < 1e-12


def test_barycentric_refinement():
    T = Topology(*synth.icosphere(1))
    B = Barycentric(T)
    assert B.topo.F == 6 * T.F
    assert B.topo.nv == T.nv + T.E + T.F
    parent_area = np.bincount(B.parent, weights=B.topo.area)
    assert np.allclose(parent_area, T.area, rtol=1e-13)
    assert np.allclose(B.topo.normal, T.normal[B.parent], atol=1e-12)


def _valence(T):
    return np.bincount(T.tris.ravel(), minlength=T.nv)


@pytest.mark.parametrize("mesh", [synth.icosphere(2), synth.hex_prism(3, 4)])
def test_bc_structure_matches_closed_form_coefficients(mesh):
    """#BC = #RWG; 2N+ + 2N- - 2 nonzeros per row; the radial coefficients of
    the v+ cell are the Buffa-Christiansen values (k - N)/(2N), k = 1..2N-1
    (up to orientation signs), the two cell-separating edges carry 1/2."""
    T = Topology(*mesh)
    B = Barycentric(T)
    assert B.B.shape[0] == T.E
    val = _valence(T)
    nnz = np.diff(B.B.indptr)
    Np, Nm = val[T.edges[:, 0]], val[T.edges[:, 1]]
    assert np.array_equal(nnz, 2 * Np + 2 * Nm - 2)
    for e in range(0, T.E, 11):
        vp, vm = T.edges[e]
        N = val[vp]
        cols = B.B.indices[B.B.indptr[e]:B.B.indptr[e + 1]]
        vals = B.B.data[B.B.indptr[e]:B.B.indptr[e + 1]]
        radial_p = [abs(c) for b, c in zip(cols, vals) if vp in B.topo.edges[b]]
        expect = sorted(abs(k - N) / (2 * N) for k in range(1, 2 * N) if k != N)
        assert np.allclose(sorted(radial_p), expect, atol=1e-13)
        halves = [abs(c) for b, c in zip(cols, vals)
                  if vp not in B.topo.edges[b] and vm not in B.topo.edges[b]]
        assert np.allclose(sorted(halves), [0.5, 0.5])


def _bary_outflow(B, coeff):
    """Net outflow of a barycentric-RWG coefficient vector from every barycentric triangle."""
    bt = B.topo
    return np.array([sum(coeff[bt.t2e[t, a]] * bt.sign[t, a] for a in range(3)) for t in range(bt.F)])


def test_bc_divergence_and_triangle_loops():
    T = Topology(*synth.icosphere(1))
    B = Barycentric(T)
    val = _valence(T)
    Bd = B.B.toarray()
    for e in range(0, T.E, 9):
        out = _bary_outflow(B, Bd[e])
        vp, vm = T.edges[e]
        expect = np.where(B.cellv == vp, 1.0 / (2 * val[vp]), np.where(B.cellv == vm, -1.0 / (2 * val[vm]), 0.0))
        assert np.allclose(out, expect, atol=1e-14)
    # dual loops around every primal triangle are divergence free
    for t in range(0, T.F, 5):
        x = np.zeros(T.E)
        for a in range(3):
            x[T.t2e[t, a]] += T.sign[t, a]
        assert np.max(np.abs(_bary_outflow(B, Bd.T @ x))) < 1e-14


def test_mixed_gram_stable_under_refinement():
    """RWG and BC are dual (Section 3.2): the mixed Gram M_A stays uniformly
    invertible, unlike the RWG-RWG anti-symmetric pairing matrix."""
    smin = []
    for lv in (1, 2):
        T = Topology(*synth.icosphere(lv))
        M = ops.mixed_mass(Barycentric(T))
        s = np.linalg.svd(M, compute_uv=False)
        smin.append(s[-1] / s[0])
    assert min(smin) > 0.05
    assert smin[1] > 0.5 * smin[0]
