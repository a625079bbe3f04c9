"""Galerkin matrices of the electric (S) and magnetic (C) boundary integral
operators, mass and Gram matrices (oracle, test infrastructure only).

Weak forms.  With the anti-symmetric pairing <a, b> = int a . (n x b)
(Section 3.2, the pairing that makes RWG and BC dual) and the potentials
and traces of Section 2 (E-potential, H-potential, S = averaged Dirichlet
trace of the E-potential, C = the same of the H-potential), surface
integration by parts and (u x n).(n x v) = -u.v for tangential v give, for
test function psi_i and trial function phi_j,

  S_ij = -ik  int int G(x,y) psi_i(x).phi_j(y)
         -(1/(ik)) int int G(x,y) div psi_i(x) div phi_j(y)
  C_ij = -int int grad_x G(x,y) . (phi_j(y) x psi_i(x))      (principal value)

with G = exp(ik|x-y|)/(4 pi |x-y|) (Section 2) and
grad_x G = (x-y) (ik r - 1) exp(ikr) / (4 pi r^3).  C's integrand vanishes on
coplanar pairs, so the principal value needs no special treatment on flat
panels.

Every Galerkin entry is a sum over triangle pairs of  int_T1 int_T2 F
(Section 3.3).  This module evaluates those integrals by direct quadrature
sums of the integrand at each point pair, basis function by basis function,
with the rules of oracle.quadrature:
  * identical / shared-edge / shared-vertex pairs: Sauter-Schwab, n points
    per coordinate;
  * disjoint pairs: tensor triangle rule of order q_near / q_medium / q_far by
    the relative distance rho = |c1 - c2| / max(diam T1, diam T2):
    near rho < 2, medium 2 <= rho < 4, far rho >= 4.  Reading: the paper
    classifies by distance and size but gives no thresholds (Section 3.3).
"""

import numpy as np
import scipy.sparse as sp

from . import quadrature as quad

FOUR_PI = 4.0 * np.pi
NEAR2, MEDIUM2 = 4.0, 16.0  # squared thresholds of rho


def _tri_geom(topo):
    P = topo.verts[topo.tris]
    cen = (P[:, 0] + P[:, 1] + P[:, 2]) / 3.0
    diam2 = np.zeros(len(P))
    for (u, v) in ((0, 1), (1, 2), (2, 0)):
        e = P[:, u] - P[:, v]
        diam2 = np.maximum(diam2, e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1] + e[:, 2] * e[:, 2])
    return P, cen, diam2


def classify(topo, t1, t2, geom=None):
    """Relation of triangle pairs: 3/2/1 = identical/shared edge/shared vertex,
    0/-1/-2 = regular near/medium/far."""
    P, cen, diam2 = geom if geom is not None else _tri_geom(topo)
    T1, T2 = topo.tris[t1], topo.tris[t2]
    shared = (T1[:, :, None] == T2[:, None, :]).any(axis=2).sum(axis=1)
    d = cen[t1] - cen[t2]
    dist2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
    m2 = np.maximum(diam2[t1], diam2[t2])
    reg = np.where(dist2 < NEAR2 * m2, 0, np.where(dist2 < MEDIUM2 * m2, -1, -2))
    return np.where(shared > 0, shared, reg)


def _regular_points(P1, P2, order):
    b, w = quad.triangle_rule(order)
    x = np.einsum("qk,nkd->nqd", b, P1)
    y = np.einsum("qk,nkd->nqd", b, P2)
    nq = len(w)
    X = np.repeat(x, nq, axis=1)                 # (n, nq*nq, 3), test index slow
    Y = np.tile(y, (1, nq, 1))
    W = np.outer(w, w).ravel()[None, :]
    return X, Y, W


def _singular_points(topo, t1, t2, kind, n):
    xh, yh, ws = quad.sauter_schwab(kind, n)
    X, Y = [], []
    for a, b in zip(t1, t2):
        A, B = [int(v) for v in topo.tris[a]], [int(v) for v in topo.tris[b]]
        common = [v for v in A if v in B]
        oa = common + [v for v in A if v not in common]
        ob = common + [v for v in B if v not in common]
        X.append(quad.ref_to_phys(topo.verts[oa], xh))
        Y.append(quad.ref_to_phys(topo.verts[ob], yh))
    # the Sauter-Schwab weights are on That x That (area 1/2 each); the physical
    # area elements contribute 2 A1 * 2 A2, applied by the caller via the
    # normalised weight convention below
    return np.array(X), np.array(Y), 4.0 * ws[None, :]


def local_blocks(topo, t1, t2, rel, k, q=(4, 3, 2), n_sing=4, want=("S", "C")):
    """3x3 local blocks of S and C for triangle pairs of one relation class.

    Returns dict op -> (n, 3, 3) complex, [a, b] = test basis a of t1 against
    trial basis b of t2 (signs included).  The weights are area-normalised:
    sum over point pairs of w * f, times area(t1) * area(t2).
    """
    P = topo.verts[topo.tris]
    P1, P2 = P[t1], P[t2]
    A1, A2 = topo.area[t1], topo.area[t2]
    if rel > 0:
        X, Y, W = _singular_points(topo, t1, t2, rel, n_sing)
    else:
        order = {0: q[0], -1: q[1], -2: q[2]}[rel]
        X, Y, W = _regular_points(P1, P2, order)
    W = W * (A1 * A2)[:, None]
    d = X - Y
    r = np.sqrt(np.einsum("nqd,nqd->nq", d, d))
    G = np.exp(1j * k * r) / (FOUR_PI * r)
    s1, s2 = topo.sign[t1], topo.sign[t2]
    psi = s1[:, None, :, None] * (X[:, :, None, :] - P1[:, None, :, :]) / (2 * A1)[:, None, None, None]
    phi = s2[:, None, :, None] * (Y[:, :, None, :] - P2[:, None, :, :]) / (2 * A2)[:, None, None, None]
    out = {}
    wG = W * G
    if "S" in want or "Sv" in want or "Sd" in want:
        dot = np.einsum("nqak,nqbk->nqab", psi, phi)
        div = (s1 / A1[:, None])[:, :, None] * (s2 / A2[:, None])[:, None, :]
        Sv = np.einsum("nq,nqab->nab", wG, dot)            # int int G psi . phi
        Sd = wG.sum(axis=1)[:, None, None] * div            # int int G div psi div phi
        if "S" in want:
            out["S"] = -1j * k * Sv - (1.0 / (1j * k)) * Sd
        if "Sv" in want:
            out["Sv"] = Sv
        if "Sd" in want:
            out["Sd"] = Sd
    if "C" in want:
        F = W * G * (1j * k * r - 1.0) / (r * r)
        grad = F[:, :, None] * d                       # w * grad_x G
        cr = np.cross(phi[:, :, None, :, :], psi[:, :, :, None, :])   # (n,q,a,b,3) phi_b x psi_a
        out["C"] = -np.einsum("nqd,nqabd->nab", grad, cr)
    return out


def assemble_rwg(topo, k, q=(4, 3, 2), n_sing=4, want=("S", "C"), chunk=48):
    """Dense Galerkin matrices (E x E) of S and/or C on the RWG space of ``topo``."""
    return assemble_rwg_tests(topo, k, 0, topo.F, q, n_sing, want, chunk)


def assemble_rwg_tests(topo, k, t_begin, t_end, q=(4, 3, 2), n_sing=4, want=("S", "C"), chunk=48):
    """The part of the dense matrices that test triangles t_begin..t_end-1
    contribute (every trial triangle): summed over a partition of the test
    triangles these give assemble_rwg's matrices (up to the order of the
    additions), which lets a caller spread the assembly over processes."""
    E, F = topo.E, topo.F
    out = {op: np.zeros((E, E), dtype=np.complex128) for op in want}
    geom = _tri_geom(topo)
    for s0 in range(t_begin, t_end, chunk):
        s1 = min(t_end, s0 + chunk)
        t1 = np.repeat(np.arange(s0, s1), F)
        t2 = np.tile(np.arange(F), s1 - s0)
        _accumulate(topo, t1, t2, k, q, n_sing, want, out, geom)
    return out


def _accumulate(topo, t1, t2, k, q, n_sing, want, out, geom):
    rel = classify(topo, t1, t2, geom)
    for c in np.unique(rel):
        sel = np.nonzero(rel == c)[0]
        step = 4000 if c <= 0 else 200
        for s0 in range(0, len(sel), step):
            s = sel[s0:s0 + step]
            blocks = local_blocks(topo, t1[s], t2[s], int(c), k, q, n_sing, want)
            rows = topo.t2e[t1[s]]
            cols = topo.t2e[t2[s]]
            for op, L in blocks.items():
                np.add.at(out[op], (rows[:, :, None], cols[:, None, :]), L)


def rwg_entries(topo, k, rows, cols, q=(4, 3, 2), n_sing=4, want=("S", "C")):
    """Individual Galerkin entries (rows[i], cols[i]) by summing the four triangle pairs."""
    rows, cols = np.asarray(rows), np.asarray(cols)
    t1l, a_l, t2l, b_l, idx = [], [], [], [], []
    for n, (i, j) in enumerate(zip(rows, cols)):
        for ti in (topo.tplus[i], topo.tminus[i]):
            a = int(np.nonzero(topo.t2e[ti] == i)[0][0])
            for tj in (topo.tplus[j], topo.tminus[j]):
                b = int(np.nonzero(topo.t2e[tj] == j)[0][0])
                t1l.append(ti); a_l.append(a); t2l.append(tj); b_l.append(b); idx.append(n)
    t1l, t2l = np.array(t1l), np.array(t2l)
    a_l, b_l, idx = np.array(a_l), np.array(b_l), np.array(idx)
    res = {op: np.zeros(len(rows), dtype=np.complex128) for op in want}
    geom = _tri_geom(topo)
    rel = classify(topo, t1l, t2l, geom)
    for c in np.unique(rel):
        s = np.nonzero(rel == c)[0]
        blocks = local_blocks(topo, t1l[s], t2l[s], int(c), k, q, n_sing, want)
        for op, L in blocks.items():
            np.add.at(res[op], idx[s], L[np.arange(len(s)), a_l[s], b_l[s]])
    return res


# --------------------------------------------------------------------------
# Buffa-Christiansen operators: Galerkin matrix on BC = B (matrix on the
# barycentric RWG space) B^T, B the BC coefficient matrix.
# --------------------------------------------------------------------------

def assemble_bc(bary, k, q=(4, 3, 2), n_sing=4, want=("S", "C")):
    bm = assemble_rwg(bary.topo, k, q, n_sing, want)
    B = bary.B
    return {op: np.asarray(B @ (B @ M.T).T) for op, M in bm.items()}


def bc_entries(bary, k, rows, cols, q=(4, 3, 2), n_sing=4, want=("S", "C")):
    B = bary.B.tocsr()
    r1, r2, coef, idx = [], [], [], []
    for n, (i, j) in enumerate(zip(rows, cols)):
        bi = B.indices[B.indptr[i]:B.indptr[i + 1]]
        ci = B.data[B.indptr[i]:B.indptr[i + 1]]
        bj = B.indices[B.indptr[j]:B.indptr[j + 1]]
        cj = B.data[B.indptr[j]:B.indptr[j + 1]]
        for u, cu in zip(bi, ci):
            for v, cv in zip(bj, cj):
                r1.append(u); r2.append(v); coef.append(cu * cv); idx.append(n)
    vals = rwg_entries(bary.topo, k, np.array(r1), np.array(r2), q, n_sing, want)
    idx, coef = np.array(idx), np.array(coef)
    out = {}
    for op, v in vals.items():
        o = np.zeros(len(rows), dtype=np.complex128)
        np.add.at(o, idx, coef * v)
        out[op] = o
    return out


def bc_bboxes(bary):
    """Axis-aligned bounding box of the support of every BC function."""
    E = bary.primal.E
    lo = np.zeros((E, 3))
    hi = np.zeros((E, 3))
    for e in range(E):
        pts = bary.verts[bary.tris[bary.support_tris(e)]].reshape(-1, 3)
        lo[e], hi[e] = pts.min(axis=0), pts.max(axis=0)
    return lo, hi


def nearfield_mask(lo, hi, chi):
    """Entry (i, j) is kept iff the support boxes of functions i and j are at
    distance <= chi (reading of the near-field cutoff of Section 3.3 at the
    level of single basis functions; chi = inf keeps everything)."""
    if np.isinf(chi):
        return np.ones((len(lo), len(lo)), dtype=bool)
    gap = np.maximum(0.0, np.maximum(lo[None, :, :] - hi[:, None, :], lo[:, None, :] - hi[None, :, :]))
    return np.sqrt((gap * gap).sum(axis=2)) <= chi


# --------------------------------------------------------------------------
# Mass and Gram matrices
# --------------------------------------------------------------------------

def mixed_mass(bary):
    """(M_A)_ij = <bc_j, rwg_i> = int bc_j . (n x rwg_i)  (Section 3.2, the mass
    matrix of A: range space BC, dual space RWG).  Rows: RWG i, columns: BC j."""
    pr, bt = bary.primal, bary.topo
    b, w = quad.triangle_rule(4)          # products of linear fields: degree 2, exact
    Mmix = np.zeros((bt.E, pr.E))
    for t in range(bt.F):
        T = bary.parent[t]
        n = pr.normal[T]
        x = b @ bt.verts[bt.tris[t]]
        wt = w * bt.area[t]
        for a in range(3):
            fb = bt.rwg_on(t, a, x)
            for c in range(3):
                fr = pr.rwg_on(T, c, x)
                Mmix[bt.t2e[t, a], pr.t2e[T, c]] += np.sum(wt * np.einsum("qd,qd->q", fb, np.cross(n, fr)))
    return np.asarray((bary.B @ Mmix).T)


def rwg_gram(topo):
    """L2 Gram matrix int rwg_i . rwg_j on the primal mesh."""
    b, w = quad.triangle_rule(4)
    G = np.zeros((topo.E, topo.E))
    for t in range(topo.F):
        x = b @ topo.verts[topo.tris[t]]
        wt = w * topo.area[t]
        for a in range(3):
            fa = topo.rwg_on(t, a, x)
            for c in range(3):
                fc = topo.rwg_on(t, c, x)
                G[topo.t2e[t, a], topo.t2e[t, c]] += np.sum(wt * np.einsum("qd,qd->q", fa, fc))
    return G
