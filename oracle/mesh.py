"""Mesh topology, RWG functions, barycentric refinement and Buffa-Christiansen
functions (oracle, test infrastructure only).

Conventions (the paper fixes the spaces, Section 3.2, not their normalisation):
  * Triangles are counter-clockwise seen from the exterior; n points into the
    exterior medium (Section 2).
  * Edge e = (lo, hi), vertex indices lo < hi.  T+ is the adjacent triangle in
    which the edge is traversed lo -> hi; T- is the other one.
  * Local basis a on triangle t is attached to the edge opposite vertex
    tris[t, a]; its sign is +1 on T+ and -1 on T-.
  * RWG, unit-flux form (reading: the paper gives no normalisation; physical
    outputs do not depend on it):
        f_e(x) = +(x - p+) / (2 A+) on T+,   -(x - p-) / (2 A-) on T-,
    so the flux through e from T+ into T- is 1 and div f_e = +-1/A+-.
  * Barycentric refinement (Section 3.2: six sub-triangles per triangle): for
    a parent (a, b, c) with edge midpoints m_ab, m_bc, m_ca and centroid g the
    children are (a,m_ab,g), (m_ab,b,g), (b,m_bc,g), (m_bc,c,g), (c,m_ca,g),
    (m_ca,a,g), oriented as the parent.  Child j lies in the dual cell of the
    parent vertex (a, b, b, c, c, a)[j].
  * BC functions (Section 3.2; Buffa & Christiansen 2007): one per primal edge
    e = (v+, v-) with v+ = lo, a combination of unit-flux RWG functions on the
    barycentric edges with coefficient = signed flux.  The oracle obtains the
    fluxes by solving the conservation conditions that define the function:
      - flux 1/2 through each of the two barycentric edges m_e-g that separate
        the dual cell of v+ from that of v- (direction v+ -> v-);
      - every barycentric triangle of the v+ cell has net outflow 1/(2 N+),
        every one of the v- cell net inflow 1/(2 N-) (N = number of primal
        triangles at the vertex);
      - no flux through the half edges v+-m_e and v- -m_e (the symmetric
        choice that fixes the circulation), nor through any other edge.
"""

import numpy as np
import scipy.sparse as sp


class Topology:
    """Edge structure of a closed, consistently oriented triangulation."""

    def __init__(self, verts, tris):
        verts = np.asarray(verts, dtype=np.float64)
        tris = np.asarray(tris, dtype=np.int64)
        F = len(tris)
        half = {}
        for t in range(F):
            for a in range(3):
                u, v = int(tris[t, (a + 1) % 3]), int(tris[t, (a + 2) % 3])
                if (u, v) in half:
                    raise ValueError("non-manifold or inconsistently oriented mesh")
                half[(u, v)] = (t, a)
        keys = sorted({(min(u, v), max(u, v)) for (u, v) in half})
        E = len(keys)
        edges = np.array(keys, dtype=np.int64).reshape(E, 2)
        tplus = np.zeros(E, dtype=np.int64)
        tminus = np.zeros(E, dtype=np.int64)
        t2e = np.zeros((F, 3), dtype=np.int64)
        sign = np.zeros((F, 3), dtype=np.float64)
        for e, (lo, hi) in enumerate(keys):
            if (lo, hi) not in half or (hi, lo) not in half:
                raise ValueError("open mesh: edge with a single triangle")
            tp, ap = half[(lo, hi)]
            tm, am = half[(hi, lo)]
            tplus[e], tminus[e] = tp, tm
            t2e[tp, ap], sign[tp, ap] = e, 1.0
            t2e[tm, am], sign[tm, am] = e, -1.0
        P = verts[tris]  # (F, 3, 3)
        cr = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
        area = 0.5 * np.linalg.norm(cr, axis=1)
        if np.any(area <= 0):
            raise ValueError("degenerate triangle")
        self.verts, self.tris = verts, tris
        self.edges, self.tplus, self.tminus = edges, tplus, tminus
        self.t2e, self.sign = t2e, sign
        self.area = area
        self.normal = cr / (2.0 * area[:, None])
        self.E, self.F, self.nv = E, F, len(verts)

    def rwg_on(self, t, a, x):
        """Value of local basis a of triangle t at points x (n, 3)."""
        p = self.verts[self.tris[t, a]]
        return self.sign[t, a] * (x - p) / (2.0 * self.area[t])


class Barycentric:
    """Barycentric refinement of a primal mesh plus the BC coefficient matrix."""

    def __init__(self, primal: Topology):
        self.primal = primal
        E, F, nv = primal.E, primal.F, primal.nv
        mid = {}
        for e, (lo, hi) in enumerate(primal.edges):
            mid[(int(lo), int(hi))] = nv + e
        verts = np.concatenate([primal.verts,
                                0.5 * (primal.verts[primal.edges[:, 0]] + primal.verts[primal.edges[:, 1]]),
                                primal.verts[primal.tris].mean(axis=1)])
        tris, parent, cellv = [], [], []
        for t in range(F):
            a, b, c = (int(x) for x in primal.tris[t])
            m = lambda u, v: mid[(min(u, v), max(u, v))]
            g = nv + E + t
            tris += [(a, m(a, b), g), (m(a, b), b, g), (b, m(b, c), g),
                     (m(b, c), c, g), (c, m(c, a), g), (m(c, a), a, g)]
            parent += [t] * 6
            cellv += [a, b, b, c, c, a]
        self.verts = verts
        self.tris = np.array(tris, dtype=np.int64)
        self.parent = np.array(parent)
        self.cellv = np.array(cellv)
        self.topo = Topology(self.verts, self.tris)
        self.B = self._bc_matrix()

    def _bc_matrix(self):
        pr, bt = self.primal, self.topo
        E, nv = pr.E, pr.nv
        cell = [[] for _ in range(nv)]
        for t, v in enumerate(self.cellv):
            cell[v].append(t)
        rows, cols, vals = [], [], []
        for e, (vp, vm) in enumerate(pr.edges):
            vp, vm = int(vp), int(vm)
            cp, cm = set(cell[vp]), set(cell[vm])
            Np, Nm = len(cp) // 2, len(cm) // 2
            both = cp | cm
            cand = sorted({int(bt.t2e[t, a]) for t in both for a in range(3)})
            unknown = [b for b in cand if bt.tplus[b] in both and bt.tminus[b] in both]
            col = {b: i for i, b in enumerate(unknown)}
            me = nv + e
            A, rhs = [], []
            # one balance equation per cell is implied by the others and the
            # prescribed exchange flux; drop it so the system is square
            skip = {min(cp), min(cm)}
            for t in sorted(both - skip):
                row = np.zeros(len(unknown))
                for a in range(3):
                    b = bt.t2e[t, a]
                    if b in col:
                        row[col[b]] += 1.0 if bt.tplus[b] == t else -1.0
                A.append(row)
                rhs.append(1.0 / (2 * Np) if t in cp else -1.0 / (2 * Nm))
            for b in unknown:
                tp, tm = bt.tplus[b], bt.tminus[b]
                lo, hi = bt.edges[b]
                row = np.zeros(len(unknown))
                row[col[b]] = 1.0
                if (tp in cp) != (tm in cp):
                    # cell-separating edge: flux 1/2 from the v+ cell to the v- cell
                    A.append(row)
                    rhs.append(0.5 if tp in cp else -0.5)
                elif {int(lo), int(hi)} in ({vp, me}, {vm, me}):
                    A.append(row)
                    rhs.append(0.0)
            A, rhs = np.array(A), np.array(rhs)
            if A.shape[0] != A.shape[1]:
                raise RuntimeError("BC conservation system not square")
            c = np.linalg.solve(A, rhs)
            for b, v in zip(unknown, c):
                if abs(v) > 1e-12:
                    rows.append(e)
                    cols.append(b)
                    vals.append(v)
        return sp.csr_matrix((vals, (rows, cols)), shape=(E, bt.E))

    def support_tris(self, e):
        """Barycentric triangles in the support of BC function e (both dual cells)."""
        vp, vm = self.primal.edges[e]
        return np.nonzero((self.cellv == vp) | (self.cellv == vm))[0]
