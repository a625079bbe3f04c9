"""Pins of the oracle functions that the full-size GPU parity tests rest on
(no GPU).

* ``rwg_entries`` / ``bc_entries`` (entry-by-entry references at sizes where
  the dense matrices do not fit) equal the dense ``assemble_rwg`` /
  ``assemble_bc`` entry by entry: a wrong local-basis lookup on T+ / T-, a
  dropped triangle pair or a wrong BC coefficient product fails;
* ``bc_bboxes``: the support of BC function e is the union of the dual cells
  of its two end vertices (Section 3.2), i.e. the vertices, the midpoints of
  their edges and the centroids of their triangles; the boxes are compared with
  that closed-form description, built from the primal mesh alone;
* ``nearfield_mask`` (the near-field cutoff chi of Section 3.3, read per basis
  function): hand-built boxes at known separations, just inside and just
  outside chi, and the limits chi = 0 and chi = infinity;
* ``classify``: constructed pairs at relative distances 1.9, 2.1, 3.9, 4.1 of
  the larger diameter land in the near / medium / medium / far classes and are
  integrated with 36 / 16 / 16 / 9 point pairs at the paper's orders
  q = (4, 3, 2); shared vertex / edge / identical pairs are classes 1 / 2 / 3;
* ``tests/mie.py`` against stored Mie efficiencies (tests/golden/mie_sphere.txt)
  and against an independent evaluation of the series by the
  logarithmic-derivative recurrence.
"""

import os

import numpy as np
import pytest

import synth
from mie import mie_efficiencies
from oracle import operators as ops
from oracle import quadrature as quad
from oracle.mesh import Topology, Barycentric

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# entry-by-entry references against the dense assembly
# ---------------------------------------------------------------------------

def _sample_entries(T, n, rng):
    """Random (i, j) plus every entry touched by a vertex-sharing triangle pair
    of a few triangles (all singular classes) and the diagonal."""
    rows = list(rng.integers(0, T.E, n))
    cols = list(rng.integers(0, T.E, n))
    for f in range(0, T.F, max(1, T.F // 6)):
        nb = [g for g in range(T.F) if set(T.tris[f]) & set(T.tris[g])]
        for g in nb:
            for i in T.t2e[f]:
                for j in T.t2e[g]:
                    rows.append(int(i))
                    cols.append(int(j))
    rows += list(range(T.E))
    cols += list(range(T.E))
    return np.array(rows), np.array(cols)


@pytest.mark.parametrize("mesh", ["icosphere1", "prism23"])
def test_rwg_entries_equal_dense_assembly(mesh):
    v, t = synth.icosphere(1) if mesh == "icosphere1" else synth.hex_prism(2, 3)
    T = Topology(v, t)
    rng = np.random.default_rng(11)
    rows, cols = _sample_entries(T, 400, rng)
    for k, q, n in ((1.7 + 0.02j, (4, 3, 2), 4), (5.0, (3, 2, 1), 2)):
        dense = ops.assemble_rwg(T, k, q, n)
        got = ops.rwg_entries(T, k, rows, cols, q, n)
        for op in ("S", "C"):
            ref = dense[op][rows, cols]
            scale = np.abs(dense[op]).max()
            assert np.max(np.abs(got[op] - ref)) <= 1e-14 * scale, (mesh, op, k)


@pytest.mark.parametrize("mesh", ["icosphere0", "prism12"])
def test_bc_entries_equal_dense_assembly(mesh):
    v, t = synth.icosphere(0) if mesh == "icosphere0" else synth.hex_prism(1, 2)
    B = Barycentric(Topology(v, t))
    E = B.primal.E
    rng = np.random.default_rng(12)
    rows = np.concatenate([rng.integers(0, E, 150), np.arange(E)])
    cols = np.concatenate([rng.integers(0, E, 150), np.arange(E)])
    k = 2.3 + 0.01j
    q, n = (2, 1, 1), 2
    dense = ops.assemble_bc(B, k, q, n)
    got = ops.bc_entries(B, k, rows, cols, q, n)
    for op in ("S", "C"):
        scale = np.abs(dense[op]).max()
        assert np.max(np.abs(got[op] - dense[op][rows, cols])) <= 1e-14 * scale, (mesh, op)


# ---------------------------------------------------------------------------
# near-field cutoff
# ---------------------------------------------------------------------------

def _bbox_closed_form(T, e):
    """Box of the two dual cells of edge e's end vertices, from the primal mesh:
    each dual cell is spanned by its vertex, the midpoints of the edges at the
    vertex and the centroids of the triangles at the vertex."""
    pts = []
    for v in T.edges[e]:
        pts.append(T.verts[v])
        for (a, b) in T.edges:
            if v in (a, b):
                pts.append(0.5 * (T.verts[a] + T.verts[b]))
        for tri in T.tris:
            if v in tri:
                pts.append(T.verts[tri].mean(axis=0))
    pts = np.array(pts)
    return pts.min(axis=0), pts.max(axis=0)


@pytest.mark.parametrize("mesh", ["icosphere1", "prism12"])
def test_bc_bboxes_closed_form(mesh):
    v, t = synth.icosphere(1) if mesh == "icosphere1" else synth.hex_prism(1, 2)
    T = Topology(v, t)
    B = Barycentric(T)
    lo, hi = ops.bc_bboxes(B)
    for e in range(T.E):
        l2, h2 = _bbox_closed_form(T, e)
        assert np.allclose(lo[e], l2, atol=1e-15, rtol=0) and np.allclose(hi[e], h2, atol=1e-15, rtol=0), e
    # the support of every BC function holds every barycentric triangle its
    # coefficient row touches (the boxes cover the whole function)
    Bc = B.B.tocsr()
    bt = B.topo
    for e in range(0, T.E, 7):
        for b in Bc.indices[Bc.indptr[e]:Bc.indptr[e + 1]]:
            for tri in (bt.tplus[b], bt.tminus[b]):
                p = B.verts[B.tris[tri]]
                assert np.all(p >= lo[e] - 1e-15) and np.all(p <= hi[e] + 1e-15)


def test_nearfield_mask_hand_cases():
    # unit boxes; box 1 is shifted by (1.3, 1.4, 0): gaps 0.3 and 0.4 -> distance 0.5
    lo = np.array([[0.0, 0.0, 0.0], [1.3, 1.4, 0.0], [0.2, 0.3, 0.4], [-2.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    hi = lo + np.array([[1.0, 1.0, 1.0], [1.0, 1.0, 1.0], [0.1, 0.1, 0.1], [1.0, 1.0, 1.0], [1.0, 1.0, 1.0]])
    # box 2 lies inside box 0; box 3 is 1.0 from box 0 along -x; box 4 touches box 0's face x = 1
    m_in = ops.nearfield_mask(lo, hi, 0.5 + 1e-12)
    m_out = ops.nearfield_mask(lo, hi, 0.5 - 1e-12)
    assert m_in[0, 1] and m_in[1, 0] and not m_out[0, 1] and not m_out[1, 0]
    m0 = ops.nearfield_mask(lo, hi, 0.0)
    assert m0[0, 2] and m0[2, 0] and m0[0, 4] and m0[4, 0]   # nested and touching boxes are kept at chi = 0
    assert not m0[0, 1] and not m0[0, 3] and not m0[3, 4]
    m1 = ops.nearfield_mask(lo, hi, 1.0)
    assert m1[0, 3] and not ops.nearfield_mask(lo, hi, 1.0 - 1e-12)[0, 3]
    # box 3 to box 4: gap 2.0 along x
    assert ops.nearfield_mask(lo, hi, 2.0)[3, 4] and not ops.nearfield_mask(lo, hi, 1.999)[3, 4]
    assert ops.nearfield_mask(lo, hi, np.inf).all()
    for chi in (0.0, 0.5, 1.0, 3.0):
        m = ops.nearfield_mask(lo, hi, chi)
        assert (m == m.T).all() and m.diagonal().all()


def test_nearfield_mask_against_sampled_box_distance():
    """The box distance of the mask equals the smallest distance between
    densely sampled points of the two boxes (up to the sampling step)."""
    rng = np.random.default_rng(5)
    lo = rng.uniform(-1, 1, (6, 3))
    hi = lo + rng.uniform(0.05, 0.6, (6, 3))
    g = np.linspace(0.0, 1.0, 9)
    G = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    for i in range(6):
        for j in range(6):
            pi = lo[i] + G * (hi[i] - lo[i])
            pj = lo[j] + G * (hi[j] - lo[j])
            dmin = np.min(np.linalg.norm(pi[:, None] - pj[None], axis=2))
            step = np.linalg.norm((hi[i] - lo[i]) / 8) + np.linalg.norm((hi[j] - lo[j]) / 8)
            # kept at chi = dmin (distance never above the sampled one) and
            # dropped below dmin - step (never far below it)
            assert ops.nearfield_mask(lo[[i, j]], hi[[i, j]], dmin + 1e-12)[0, 1]
            if dmin > step:
                assert not ops.nearfield_mask(lo[[i, j]], hi[[i, j]], dmin - step - 1e-12)[0, 1]


def test_nearfield_mask_on_mesh_limits():
    T = Topology(*synth.icosphere(1))
    B = Barycentric(T)
    lo, hi = ops.bc_bboxes(B)
    assert ops.nearfield_mask(lo, hi, np.inf).all()
    m0 = ops.nearfield_mask(lo, hi, 0.0)
    # functions whose supports share a point (a common dual-cell vertex: their
    # edges share a primal vertex or lie on one triangle) are always kept
    vert_cells = [set(T.edges[e]) for e in range(T.E)]
    for i in range(T.E):
        for j in range(T.E):
            if vert_cells[i] & vert_cells[j]:
                assert m0[i, j]
    # and far-apart functions are dropped: the cutoff bites
    assert m0.mean() < 0.5


# ---------------------------------------------------------------------------
# relative-distance classes
# ---------------------------------------------------------------------------

def _two_triangle_topo(P1, P2):
    T = Topology.__new__(Topology)
    T.verts = np.concatenate([P1, P2])
    T.tris = np.array([[0, 1, 2], [3, 4, 5]])
    cr = np.cross(T.verts[T.tris][:, 1] - T.verts[T.tris][:, 0], T.verts[T.tris][:, 2] - T.verts[T.tris][:, 0])
    T.area = 0.5 * np.linalg.norm(cr, axis=1)
    T.sign = np.ones((2, 3))
    return T


def _equilateral(side, center, rot=0.0):
    ang = rot + np.array([0.0, 2 * np.pi / 3, 4 * np.pi / 3])
    R = side / np.sqrt(3.0)
    return np.stack([center[0] + R * np.cos(ang), center[1] + R * np.sin(ang), np.full(3, center[2])], axis=1)


@pytest.mark.parametrize("rho,cls,npts", [(1.9, 0, 36), (2.1, -1, 16), (3.9, -1, 16), (4.1, -2, 9)])
def test_classify_thresholds_and_point_counts(rho, cls, npts, monkeypatch):
    # the larger triangle (side 1.5) sets the scale: rho is measured against
    # max(diam T1, diam T2) = 1.5, so a slip to the smaller diameter (1.0) or
    # to the test triangle's own diameter moves every case up a class
    for small_first in (True, False):
        a, b = (1.0, 1.5) if small_first else (1.5, 1.0)
        P1 = _equilateral(a, np.zeros(3))
        P2 = _equilateral(b, rho * 1.5 * np.array([1.0, 0.0, 0.2]) / np.hypot(1.0, 0.2), rot=0.3)
        T = _two_triangle_topo(P1, P2)
        dist = np.linalg.norm(P1.mean(0) - P2.mean(0))
        assert abs(dist / 1.5 - rho) < 1e-12
        assert ops.classify(T, np.array([0]), np.array([1]))[0] == cls
        assert ops.classify(T, np.array([1]), np.array([0]))[0] == cls
        seen = []
        real_rule = quad.triangle_rule

        def spy(order):
            b_, w_ = real_rule(order)
            seen.append(len(w_))
            return b_, w_

        monkeypatch.setattr(quad, "triangle_rule", spy)
        ops.local_blocks(T, np.array([0]), np.array([1]), cls, 1.0, q=(4, 3, 2))
        monkeypatch.setattr(quad, "triangle_rule", real_rule)
        assert seen and seen[0] ** 2 == npts


def test_classify_singular_classes():
    T = Topology(*synth.icosphere(1))
    f = 0
    for g in range(T.F):
        shared = len(set(T.tris[f]) & set(T.tris[g]))
        c = ops.classify(T, np.array([f]), np.array([g]))[0]
        if shared:
            assert c == shared
        else:
            assert c in (0, -1, -2)
    assert ops.classify(T, np.array([f]), np.array([f]))[0] == 3


# ---------------------------------------------------------------------------
# Mie series
# ---------------------------------------------------------------------------

def _mie_log_derivative(x, m):
    """Mie efficiencies by the logarithmic derivative D_n(mx) (downward
    recurrence) and upward Riccati-Bessel recurrences (Bohren & Huffman,
    appendix A), independent of tests/mie.py's spherical Bessel functions."""
    nstop = int(np.floor(x + 4.0 * x ** (1.0 / 3.0) + 2.0))
    mx = m * x
    nmx = int(max(nstop, abs(mx))) + 16
    D = np.zeros(nmx + 1, dtype=np.complex128)
    for n in range(nmx, 0, -1):
        D[n - 1] = n / mx - 1.0 / (D[n] + n / mx)
    psi0, psi1 = np.cos(x), np.sin(x)         # psi_{-1}, psi_0
    chi0, chi1 = -np.sin(x), np.cos(x)        # chi_{-1}, chi_0
    xi1 = psi1 - 1j * chi1
    qext = qsca = 0.0
    for n in range(1, nstop + 1):
        psi = (2 * n - 1) / x * psi1 - psi0
        chi = (2 * n - 1) / x * chi1 - chi0
        xi = psi - 1j * chi
        an = ((D[n] / m + n / x) * psi - psi1) / ((D[n] / m + n / x) * xi - xi1)
        bn = ((m * D[n] + n / x) * psi - psi1) / ((m * D[n] + n / x) * xi - xi1)
        qsca += (2 * n + 1) * (abs(an) ** 2 + abs(bn) ** 2)
        qext += (2 * n + 1) * (an + bn).real
        psi0, psi1, chi0, chi1, xi1 = psi1, psi, chi1, chi, xi
    return 2.0 * qext / x ** 2, 2.0 * qsca / x ** 2


def test_mie_series_against_stored_values():
    rows = np.loadtxt(os.path.join(GOLDEN, "mie_sphere.txt"))
    m = np.sqrt(3.17 + 0.01j)
    for x, qe, qs in rows:
        got = mie_efficiencies(x, m)
        alt = _mie_log_derivative(x, m)
        for v, ref in ((got[0], qe), (got[1], qs), (alt[0], qe), (alt[1], qs)):
            assert abs(v - ref) <= 1e-10 * abs(ref), (x, v, ref)
    # a lossless sphere does not absorb: Q_ext = Q_sca
    qe, qs = mie_efficiencies(3.0, 1.5)
    assert abs(qe - qs) < 1e-12 * qe
