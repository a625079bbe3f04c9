"""Pins of the oracle's Galerkin matrices (no GPU).

* div-div part of S on coincident panels at k -> 0 against the closed-form
  self integral of 1/r (fixes weights and Jacobians of the singular path);
* a regular pair at the paper's orders against a converged composite rule;
* complex symmetry of S and C (same test and trial space), converging with
  the singular order, and exact up to rounding outside the entries that
  vertex-sharing (singular) pairs touch;
* C vanishes on coplanar pairs;
* loop null spaces: vertex loops of RWG and dual loops of BC are divergence
  free, so the div-div part of S annihilates them;
* Calderon projector (Section 2, trace relations): for a field that solves
  Maxwell inside Gamma, A_k u = +u/2; for one radiating outside, A_k u = -u/2;
  the discrete residuals shrink under refinement.
"""

import numpy as np
import pytest

import synth
from oracle.mesh import Topology, Barycentric
from oracle import operators as ops
from oracle import pmchwt
from oracle import quadrature as quad
from test_oracle_quadrature import self_integral_closed_form


def test_divdiv_identical_static_limit():
    v = np.array([[0.0, 0.0, 0.0], [1.0, 0.05, 0.1], [0.35, 0.8, -0.1], [0.6, -0.7, 0.2]])
    t = np.array([[0, 1, 2], [0, 3, 1]])
    # a two-triangle patch is enough for local blocks (no topology needed beyond signs)
    T = Topology.__new__(Topology)
    T.verts, T.tris = v, t
    P = v[t]
    cr = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    T.area = 0.5 * np.linalg.norm(cr, axis=1)
    T.sign = np.ones((2, 3))
    blk = ops.local_blocks(T, np.array([0]), np.array([0]), 3, 1e-9, n_sing=16, want=("Sd",))["Sd"][0]
    ref = self_integral_closed_form(P[0]) / (4 * np.pi) / T.area[0] ** 2
    assert np.allclose(blk, ref, rtol=1e-10)


def test_regular_pair_against_converged_rule():
    T = Topology(*synth.icosphere(2))
    geom = ops._tri_geom(T)
    rel = ops.classify(T, np.zeros(T.F, int), np.arange(T.F), geom)
    k = 2.0 + 0.1j
    for c, tol in ((0, 2e-3), (-1, 2e-3), (-2, 2e-3)):
        t2 = int(np.nonzero(rel == c)[0][0])
        got = ops.local_blocks(T, np.array([0]), np.array([t2]), c, k)
        # converged reference: both triangles split 4^3 times, degree-4 rule each
        P1, P2 = T.verts[T.tris[0]], T.verts[T.tris[t2]]
        X, WX = _composite(P1, 3)
        Y, WY = _composite(P2, 3)
        d = X[:, None, :] - Y[None, :, :]
        r = np.linalg.norm(d, axis=2)
        G = np.exp(1j * k * r) / (4 * np.pi * r)
        W = WX[:, None] * WY[None, :]
        S = np.zeros((3, 3), complex)
        for a in range(3):
            fa = T.rwg_on(0, a, X)
            for b in range(3):
                fb = T.rwg_on(t2, b, Y)
                S[a, b] = np.sum(W * G * (-1j * k * (fa @ fb.T)
                                          - T.sign[0, a] * T.sign[t2, b] / (T.area[0] * T.area[t2]) / (1j * k)))
        assert np.max(np.abs(got["S"][0] - S)) < tol * np.max(np.abs(S))


def _composite(T, levels):
    b, w = quad.triangle_rule(4)
    tris = [np.asarray(T)]
    for _ in range(levels):
        new = []
        for t in tris:
            m01, m12, m20 = (t[0] + t[1]) / 2, (t[1] + t[2]) / 2, (t[2] + t[0]) / 2
            new += [np.array([t[0], m01, m20]), np.array([m01, t[1], m12]),
                    np.array([m20, m12, t[2]]), np.array([m01, m12, m20])]
        tris = new
    X = np.concatenate([b @ t for t in tris])
    W = np.concatenate([w * 0.5 * np.linalg.norm(np.cross(t[1] - t[0], t[2] - t[0])) for t in tris])
    return X, W


def test_symmetry_converges_with_singular_order():
    T = Topology(*synth.icosphere(1))
    asym = []
    for n in (4, 8):
        d = ops.assemble_rwg(T, 1.3 + 0.02j, n_sing=n)
        asym.append([np.abs(M - M.T).max() / np.abs(M).max() for M in (d["S"], d["C"])])
    assert asym[1][0] < 1e-10 and asym[1][1] < 1e-7
    assert asym[1][0] < 1e-3 * asym[0][0] and asym[1][1] < 1e-2 * asym[0][1]


def _vertex_sharing_pattern(T):
    """Entries (i, j) that some pair of triangles sharing a vertex (the
    Sauter-Schwab classes: identical, shared edge, shared vertex) touches."""
    v2t = [[] for _ in range(len(T.verts))]
    for f, tri in enumerate(T.tris):
        for a in tri:
            v2t[a].append(f)
    pat = np.zeros((T.E, T.E), bool)
    for f, tri in enumerate(T.tris):
        for g in {g for a in tri for g in v2t[a]}:
            pat[np.ix_(T.t2e[f], T.t2e[g])] = True
    return pat


@pytest.mark.parametrize("mesh", ["icosphere1", "prism23"])
def test_asymmetry_only_on_vertex_sharing_pairs(mesh):
    """S and C are symmetric forms on one space and every disjoint pair is
    integrated with the same product rule from either side, so the
    assembled matrices are symmetric to rounding except where a singular
    (Sauter-Schwab) rule integrates a vertex-sharing pair, which it does not
    do symmetrically in the two triangles.  A product that stores one
    triangle of the matrix relies on exactly this, with a correction on the
    vertex-sharing pattern."""
    v, t = synth.icosphere(1) if mesh == "icosphere1" else synth.hex_prism(2, 3)
    T = Topology(v, t)
    pat = _vertex_sharing_pattern(T)
    d = ops.assemble_rwg(T, 2.0 * np.sqrt(3.17 + 0.01j), n_sing=4)
    for name in ("S", "C"):
        M = d[name]
        D = np.abs(M - M.T) / np.abs(M).max()
        assert D[~pat].max() < 1e-14, name
        assert D[pat].max() > 1e-8, name  # the correction is needed


def test_C_vanishes_on_coplanar_pairs():
    T = Topology(*synth.cube(2))
    geom = ops._tri_geom(T)
    same_face = [(i, j) for i in range(T.F) for j in range(T.F)
                 if np.allclose(T.normal[i], T.normal[j]) and abs((T.verts[T.tris[i, 0]] - T.verts[T.tris[j, 0]]) @ T.normal[i]) < 1e-14]
    t1 = np.array([p[0] for p in same_face])
    t2 = np.array([p[1] for p in same_face])
    rel = ops.classify(T, t1, t2, geom)
    for c in np.unique(rel):
        s = rel == c
        C = ops.local_blocks(T, t1[s], t2[s], int(c), 3.0, want=("C",))["C"]
        assert np.max(np.abs(C)) < 1e-16


def test_loop_null_spaces():
    T = Topology(*synth.icosphere(1))
    Sd = ops.assemble_rwg(T, 1.0, want=("Sd",))["Sd"]
    for v in range(0, T.nv, 5):
        x = np.zeros(T.E)
        x[T.edges[:, 0] == v] = 1.0
        x[T.edges[:, 1] == v] = -1.0
        assert np.linalg.norm(Sd @ x) < 1e-13 * np.linalg.norm(Sd) * np.linalg.norm(x)
    B = Barycentric(Topology(*synth.icosphere(0)))
    Sdb = ops.assemble_bc(B, 1.0, want=("Sd",))["Sd"]
    Tp = B.primal
    for t in range(Tp.F):
        x = np.zeros(Tp.E)
        for a in range(3):
            x[Tp.t2e[t, a]] += Tp.sign[t, a]
        assert np.linalg.norm(Sdb @ x) < 1e-13 * np.linalg.norm(Sdb) * np.linalg.norm(x)


def _dipole_traces(T, k, x0, p):
    """Traces [E x n ; k gamma_N E] of the radiating field E = grad G x p (source x0 inside)."""
    b, w = quad.triangle_rule(4)
    g = np.zeros(T.E, complex); gN = np.zeros(T.E, complex)
    h = np.zeros(T.E, complex); hN = np.zeros(T.E, complex)
    for t in range(T.F):
        n = T.normal[t]
        x = b @ T.verts[T.tris[t]]
        d = x - x0
        r = np.linalg.norm(d, axis=1)
        rh = d / r[:, None]
        G = np.exp(1j * k * r) / (4 * np.pi * r)
        G1 = G * (1j * k - 1 / r)
        G2 = G * ((1j * k - 1 / r) ** 2 + 1 / r ** 2)
        E = np.cross(G1[:, None] * rh, p[None, :])
        Hs = (G2 - G1 / r)[:, None, None] * rh[:, :, None] * rh[:, None, :] + (G1 / r)[:, None, None] * np.eye(3)[None]
        curlE = np.einsum("qij,j->qi", Hs, p) + (k * k * G)[:, None] * p[None, :]
        uD = np.cross(E, n)
        uN = k * np.cross(curlE / (1j * k), n)
        for a in range(3):
            f = T.rwg_on(t, a, x)
            nf = np.cross(n, f)
            e = T.t2e[t, a]
            wt = w * T.area[t]
            g[e] += np.sum(wt * np.einsum("qd,qd->q", uD, nf)); gN[e] += np.sum(wt * np.einsum("qd,qd->q", uN, nf))
            h[e] += np.sum(wt * np.einsum("qd,qd->q", uD, f)); hN[e] += np.sum(wt * np.einsum("qd,qd->q", uN, f))
    G = ops.rwg_gram(T)
    return np.concatenate([g, gN]), np.concatenate([np.linalg.solve(G, h), np.linalg.solve(G, hN)])


@pytest.mark.slow
def test_calderon_projector_signs():
    k = 1.5
    res_int, res_rad, wrong = [], [], []
    for lv in (1, 2):
        pr = pmchwt.Problem([synth.icosphere(lv)], 1.0, k)
        T = pr.topos[0]
        d = ops.assemble_rwg(T, k)
        Ak = pmchwt.pmchwt_block(d["C"], d["S"], k)
        # interior solution: plane wave at wavenumber k
        pr.Ci, pr.Si, pr.k_i = [np.zeros_like(d["C"])], [np.zeros_like(d["S"])], [k]
        dirs, pols = synth.single_wave((0.3, 0.4, np.sqrt(0.75)), (np.sqrt(0.75), 0.0, -0.3))
        pols = pols - np.outer(np.sum(pols * dirs, axis=1), dirs[0])
        pr.rhs(dirs, pols)
        c = pr.c_inc[0]
        gfull = 2 * pr.rhs(dirs, pols)[0]           # with zero interior operator: b = g/2
        res_int.append(np.linalg.norm(Ak @ c - 0.5 * gfull) / np.linalg.norm(gfull))
        wrong.append(np.linalg.norm(Ak @ c + 0.5 * gfull) / np.linalg.norm(gfull))
        g, c = _dipole_traces(T, k, np.array([0.1, -0.2, 0.15]), np.array([0.3, 1.0, -0.4]))
        res_rad.append(np.linalg.norm(Ak @ c + 0.5 * g) / np.linalg.norm(g))
        wrong.append(np.linalg.norm(Ak @ c - 0.5 * g) / np.linalg.norm(g))
    # the right sign leaves a discretisation-size residual that shrinks under
    # refinement; the opposite sign leaves a residual of order one
    assert res_int[1] < 0.6 * res_int[0] and res_int[1] < 0.1
    assert res_rad[1] < 0.9 * res_rad[0] and res_rad[1] < 0.05
    assert min(wrong) > 0.5
