"""PMCHWT system, Calderon preconditioners, right-hand side, solves, far field
and cross sections (oracle, test infrastructure only).

Notation follows Section 2 and 3 of the paper with mu = 1 everywhere
(reading: permeabilities are not part of the workloads), k_m = k_e sqrt(eps_m)
with the principal square root.

Discretisation (Section 3.2, the choice the paper makes): A is discretised
with RWG as domain and dual space and BC as range; P with BC as domain and
dual and RWG as range.  The matrix of the preconditioned product is
M_P^{-1} P M_A^{-1} A, with M_A = <bc_j, rwg_i> and M_P = -M_A^T.

Reading of the block pairing: the paper pairs the two trace components
crosswise (Section 3.2).  That only permutes block rows of A, M_A, P and M_P
identically, so M^{-1} A, M^{-1} P and the iteration are unchanged; the
oracle uses the plain component-wise pairing.

Unknown layout: scatterer-major, and within scatterer m the Dirichlet block
x_D (E_m RWG coefficients) then the scaled Neumann block x_N (Section 2,
the traces u^s_m).
"""

import numpy as np

from . import operators as ops
from . import quadrature as quad
from .mesh import Topology, Barycentric

PRECONDITIONERS = ("I", "A", "D", "D_INT", "D_EXT", "S_INT", "S_EXT")


def table1_matvecs(kind, M, R, rho):
    """Total matvecs of GMRES for a given preconditioner (Table 1).

    One matvec = one application of one discrete boundary integral operator.
    R iterations, restart rho, M scatterers; includes the one-off
    pre-multiplication of the right-hand side by P.
    """
    cycles = R + R // rho
    per = {"I": (4 * M * M + 4 * M, 0),
           "A": (8 * M * M + 8 * M, 4 * M * M + 4 * M),
           "D": (4 * M * M + 12 * M, 8 * M),
           "D_INT": (4 * M * M + 8 * M, 4 * M), "D_EXT": (4 * M * M + 8 * M, 4 * M),
           "S_INT": (4 * M * M + 6 * M, 2 * M), "S_EXT": (4 * M * M + 6 * M, 2 * M)}[kind]
    return per[0] * cycles + per[1]


def pmchwt_block(C, S, k):
    """[[C, S/k], [-k S, C]]  (the blocks of Section 2 with mu = 1)."""
    return np.block([[C, S / k], [-k * S, C]])


class Problem:
    """Dense FP64 discretisation of the multi-particle PMCHWT problem."""

    def __init__(self, meshes, eps, k_ext, qA=(4, 3, 2), nA=4, qP=(4, 3, 2), nP=4,
                 chiP=np.inf, precond="S_INT"):
        if precond not in PRECONDITIONERS:
            raise ValueError(precond)
        self.k_e = complex(k_ext)
        self.meshes = meshes
        self.M = len(meshes)
        eps = [complex(e) for e in (eps if np.ndim(eps) else [eps] * self.M)]
        self.k_i = [self.k_e * np.sqrt(e) for e in eps]
        self.topos = [Topology(v, t) for (v, t) in meshes]
        self.Es = [T.E for T in self.topos]
        self.offs = np.concatenate([[0], np.cumsum(self.Es)])
        nv = np.concatenate([[0], np.cumsum([len(v) for (v, t) in meshes])])
        uv = np.concatenate([v for (v, t) in meshes])
        ut = np.concatenate([t + nv[m] for m, (v, t) in enumerate(meshes)])
        self.union = Topology(uv, ut)
        # union edges are sorted by (lo, hi); vertex blocks are disjoint and
        # ordered, so the union edge order is the concatenation of the
        # per-scatterer edge orders
        self.qA, self.nA, self.qP, self.nP = qA, nA, qP, nP
        self.chiP, self.precond = chiP, precond
        self.N = 2 * int(self.offs[-1])

    # ---- Galerkin matrices --------------------------------------------------
    def assemble_A(self, assemble=None):
        """A = A^e + A^i (Section 2).  ``assemble`` replaces ops.assemble_rwg
        (same arguments and result), e.g. by one that spreads the same
        quadrature sums over processes."""
        assemble = assemble or ops.assemble_rwg
        ext = assemble(self.union, self.k_e, self.qA, self.nA)
        self.Se, self.Ce = ext["S"], ext["C"]
        self.Si, self.Ci = [], []
        for T, k in zip(self.topos, self.k_i):
            d = assemble(T, k, self.qA, self.nA)
            self.Si.append(d["S"])
            self.Ci.append(d["C"])
        A = np.zeros((self.N, self.N), dtype=np.complex128)
        for m in range(self.M):
            for l in range(self.M):
                rm, rl = self._rng(m), self._rng(l)
                blk = pmchwt_block(self.Ce[rm, rl], self.Se[rm, rl], self.k_e)
                if m == l:
                    blk = blk + pmchwt_block(self.Ci[m], self.Si[m], self.k_i[m])
                A[self._blk(m), self._blk(l)] = blk
        self.A = A
        return A

    def _rng(self, m):
        return slice(int(self.offs[m]), int(self.offs[m + 1]))

    def _blk(self, m):
        return slice(2 * int(self.offs[m]), 2 * int(self.offs[m + 1]))

    def assemble_P(self):
        """Galerkin matrix of the chosen preconditioner on BC x BC."""
        self.barys = [Barycentric(T) for T in self.topos]
        kind = self.precond
        P = np.zeros((self.N, self.N), dtype=np.complex128)
        self.PBC = {}
        if kind == "I":
            self.P = None
            return None
        need_int = kind in ("A", "D", "D_INT", "S_INT")
        need_ext = kind in ("A", "D", "D_EXT", "S_EXT")
        want = ("S",) if kind in ("S_INT", "S_EXT") else ("S", "C")
        if kind == "A" and self.M > 1:
            ub = Barycentric(self.union)
            lo, hi = ops.bc_bboxes(ub)
            mask = ops.nearfield_mask(lo, hi, self.chiP)
            ext = ops.assemble_bc(ub, self.k_e, self.qP, self.nP, want)
            for l in range(self.M):
                for m in range(self.M):
                    rm, rl = self._rng(m), self._rng(l)
                    blk = pmchwt_block(ext["C"][rm, rl] * mask[rm, rl], ext["S"][rm, rl] * mask[rm, rl], self.k_e)
                    P[self._blk(m), self._blk(l)] += blk
            need_ext = False
        for m, bary in enumerate(self.barys):
            lo, hi = ops.bc_bboxes(bary)
            mask = ops.nearfield_mask(lo, hi, self.chiP)
            blk = np.zeros((2 * self.Es[m], 2 * self.Es[m]), dtype=np.complex128)
            for flag, k, tag in ((need_int, self.k_i[m], "int"), (need_ext, self.k_e, "ext")):
                if not flag:
                    continue
                d = ops.assemble_bc(bary, k, self.qP, self.nP, want)
                S = d["S"] * mask
                self.PBC[(tag, m, "S")] = S
                if "C" in d:
                    C = d["C"] * mask
                    self.PBC[(tag, m, "C")] = C
                    blk += pmchwt_block(C, S, k)
                else:
                    E = self.Es[m]
                    blk += np.block([[np.zeros((E, E)), S / k], [-k * S, np.zeros((E, E))]])
            P[self._blk(m), self._blk(m)] += blk
        self.P = P
        return P

    def assemble_mass(self):
        if not hasattr(self, "barys"):
            self.barys = [Barycentric(T) for T in self.topos]
        self.MA = []
        for bary in self.barys:
            self.MA.append(ops.mixed_mass(bary))
        return self.MA

    def precond_matrix(self):
        """Ptilde = M_P^{-1} P M_A^{-1} (identity for P = I)."""
        if self.precond == "I":
            return np.eye(self.N)
        MAinv = np.zeros((self.N, self.N))
        MPinv = np.zeros((self.N, self.N))
        for m in range(self.M):
            E = self.Es[m]
            Mi = np.linalg.inv(self.MA[m])
            Z = np.zeros((E, E))
            MAinv[self._blk(m), self._blk(m)] = np.block([[Mi, Z], [Z, Mi]])
            MPinv[self._blk(m), self._blk(m)] = np.block([[-Mi.T, Z], [Z, -Mi.T]])
        return MPinv @ self.P @ MAinv

    # ---- right-hand side ----------------------------------------------------
    def rhs(self, dirs, pols):
        """b = <(1/2 I - D^i) u^inc, rwg_i>  (Section 3.2) for each incident wave.

        Reading: u^inc is used exactly in the identity term, g_i = int u^inc . (n x rwg_i),
        and through its L2 projection c_inc onto RWG inside D^i (the paper does
        not say how u^inc is discretised).  Incident field E = p exp(i k_e d.x);
        u^inc = [E x n ; k_e ((d x p) exp(i k_e d.x)) x n]  (Section 2, traces
        scaled by k/mu).
        """
        dirs = np.atleast_2d(dirs)
        pols = np.atleast_2d(pols)
        b = np.zeros((len(dirs), self.N), dtype=np.complex128)
        self.c_inc = np.zeros((len(dirs), self.N), dtype=np.complex128)
        bq, wq = quad.triangle_rule(4)
        for m, T in enumerate(self.topos):
            E = T.E
            G = ops.rwg_gram(T)
            for w_i, (d, p) in enumerate(zip(dirs, pols)):
                gD = np.zeros(E, dtype=np.complex128)
                gN = np.zeros(E, dtype=np.complex128)
                hD = np.zeros(E, dtype=np.complex128)
                hN = np.zeros(E, dtype=np.complex128)
                for t in range(T.F):
                    n = T.normal[t]
                    x = bq @ T.verts[T.tris[t]]
                    ph = np.exp(1j * self.k_e * (x @ d))
                    Ei = p[None, :] * ph[:, None]
                    Hi = np.cross(d, p)[None, :] * ph[:, None]
                    uD = np.cross(Ei, n[None, :])
                    uN = self.k_e * np.cross(Hi, n[None, :])
                    wt = wq * T.area[t]
                    for a in range(3):
                        f = T.rwg_on(t, a, x)
                        nf = np.cross(n[None, :], f)
                        e = T.t2e[t, a]
                        gD[e] += np.sum(wt * np.einsum("qd,qd->q", uD, nf))
                        gN[e] += np.sum(wt * np.einsum("qd,qd->q", uN, nf))
                        hD[e] += np.sum(wt * np.einsum("qd,qd->q", uD, f))
                        hN[e] += np.sum(wt * np.einsum("qd,qd->q", uN, f))
                cD = np.linalg.solve(G, hD)
                cN = np.linalg.solve(G, hN)
                k = self.k_i[m]
                Ai = pmchwt_block(self.Ci[m], self.Si[m], k)
                c = np.concatenate([cD, cN])
                b[w_i, self._blk(m)] = 0.5 * np.concatenate([gD, gN]) - Ai @ c
                self.c_inc[w_i, self._blk(m)] = c
        return b

    # ---- solves -------------------------------------------------------------
    def solve_direct(self, b):
        """Exact discrete solution of A x = b (the preconditioner does not change it)."""
        return np.linalg.solve(self.A, np.atleast_2d(b).T).T

    # ---- far field ----------------------------------------------------------
    def far_field(self, x, obs):
        """F(xhat) with E^s ~ exp(i k_e r)/r F(xhat) (Stratton-Chu, Section 2).

        From E^s = -H(gamma_D E^s) - E(gamma_N E^s), gamma_N E^s = x_N / k_e and
        the large-|x| form of G:
          F = -(i/(4 pi)) [k_e xhat x V_D + V_N - xhat (xhat . V_N)],
          V = int u(y) exp(-i k_e xhat . y) ds(y)  (6-point rule per triangle).
        """
        x = np.atleast_2d(x)
        obs = np.atleast_2d(obs)
        bq, wq = quad.triangle_rule(4)
        T = self.union
        E = T.E
        # union coefficients: scatterer-major [D_m, N_m] -> union-edge arrays
        xD = np.zeros((len(x), E), dtype=np.complex128)
        xN = np.zeros((len(x), E), dtype=np.complex128)
        for m in range(self.M):
            o, Em = int(self.offs[m]), self.Es[m]
            xD[:, o:o + Em] = x[:, 2 * o:2 * o + Em]
            xN[:, o:o + Em] = x[:, 2 * o + Em:2 * o + 2 * Em]
        k = self.k_e
        VD = np.zeros((len(x), len(obs), 3), dtype=np.complex128)
        VN = np.zeros_like(VD)
        for t in range(T.F):
            y = bq @ T.verts[T.tris[t]]
            wt = wq * T.area[t]
            ph = np.exp(-1j * k * (obs @ y.T))
            for a in range(3):
                f = T.rwg_on(t, a, y)
                e = T.t2e[t, a]
                base = np.einsum("oq,qd->od", ph * wt[None, :], f)
                VD += xD[:, e][:, None, None] * base[None]
                VN += xN[:, e][:, None, None] * base[None]
        xo = obs[None, :, :]
        return -(1j / (4 * np.pi)) * (k * np.cross(xo, VD) + VN - xo * np.einsum("rod,rod->ro", xo, VN)[..., None])

    def cross_sections(self, x, dirs, pols, n_theta=64, n_phi=128):
        """sigma_ext by the optical theorem, sigma_sca = int |F|^2 over the sphere
        (n_theta Gauss-Legendre nodes in cos(theta) x n_phi uniform in phi)."""
        x = np.atleast_2d(x)
        dirs = np.atleast_2d(dirs)
        pols = np.atleast_2d(pols)
        k = self.k_e.real
        ext = np.array([(4 * np.pi / k) * np.imag(np.vdot(p, self.far_field(xi, d[None, :])[0, 0]))
                        for xi, d, p in zip(x, dirs, pols)])
        ct, wt = np.polynomial.legendre.leggauss(n_theta)
        ph = 2 * np.pi * np.arange(n_phi) / n_phi
        CT, PH = np.meshgrid(ct, ph, indexing="ij")
        st = np.sqrt(1 - CT ** 2)
        obs = np.stack([st * np.cos(PH), st * np.sin(PH), CT], axis=-1).reshape(-1, 3)
        w = (wt[:, None] * np.full(n_phi, 2 * np.pi / n_phi)[None, :]).ravel()
        Fv = self.far_field(x, obs)
        sca = np.einsum("o,rod->r", w, np.abs(Fv) ** 2)
        return ext, sca


def gmres(apply, b, tol=1e-6, restart=200, max_iter=2000):
    """Restarted GMRES with modified Gram-Schmidt and Givens rotations.

    Reading: the paper uses GMRES(rho) with relative tolerance on the system it
    is given (Section 4); the orthogonalisation scheme is not stated.  At the
    end of every full cycle the true residual b - Op x is recomputed (one extra
    operator application, the floor(R/rho) term of Table 1).
    Returns x, iterations, operator applications, relative-residual history.
    """
    b = np.asarray(b, dtype=np.complex128)
    n = len(b)
    x = np.zeros(n, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        return x, 0, 0, [0.0]
    r = b.copy()
    beta = bnorm
    it, napp, hist = 0, 0, [1.0]
    while True:
        V = np.zeros((restart + 1, n), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        done = False
        j_end = 0
        for j in range(restart):
            w = apply(V[j])
            napp += 1
            it += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                H[i, j] = t
            den = np.sqrt(abs(H[j, j]) ** 2 + abs(H[j + 1, j]) ** 2)
            cs[j] = np.conj(H[j, j]) / den if den else 1.0
            sn[j] = np.conj(H[j + 1, j]) / den if den else 0.0
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            res = abs(g[j + 1]) / bnorm
            hist.append(res)
            j_end = j + 1
            if res <= tol or it >= max_iter:
                done = True
                break
        y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
        x = x + V[:j_end].T @ y
        if done:
            return x, it, napp, hist
        r = b - apply(x)
        napp += 1
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            return x, it, napp, hist
