"""Electric field at points near and inside the scatterers from the solved
traces (oracle, test infrastructure only).

The Stratton-Chu representation of Section 2, with the potentials
  E v(x) = ik int v(y) G(x,y) ds(y) - (1/(ik)) grad_x int div v(y) G(x,y) ds(y),
  H v(x) = curl_x int v(y) G(x,y) ds(y) = int grad_x G(x,y) x v(y) ds(y),
  grad_x G = (x - y) (ik r - 1) exp(ikr) / (4 pi r^3),
gives
  outside every scatterer:  E = E^inc + E^s,
      E^s = - sum_m [ H^e(gamma_D E^s) + E^e(gamma_N E^s) ]   (k = k_e, all surfaces);
  inside scatterer m:       E = H^i_m(gamma_D E^i) + E^i_m(gamma_N E^i)   (k = k_m, surface m).
The solved unknowns are the scaled traces u^s = [gamma_D E^s; k_e gamma_N E^s]
(mu = 1), and the transmission conditions give the interior traces
u^i = [gamma_D E^i; k_m gamma_N E^i] = u^s + u^inc.  Reading (as for the
right-hand side, where the paper does not say how u^inc is discretised):
u^inc enters through its L2 projection c_inc onto RWG.  Surface integrals use
the degree-4 symmetric rule (6 points) on every triangle, the rule of the far
field.  A point is inside scatterer m when the solid angle its closed surface
subtends there is 4 pi (winding number 1).
"""

import numpy as np

from . import quadrature as quad

FOUR_PI = 4.0 * np.pi


def inside_mask(topo, pts):
    """Points strictly inside the closed surface of ``topo`` (outward normals):
    the solid angle of every triangle (Van Oosterom and Strackee 1983) summed
    over the surface is 4 pi inside and 0 outside."""
    pts = np.atleast_2d(pts)
    tot = np.zeros(len(pts))
    for t in range(topo.F):
        a, b, c = topo.verts[topo.tris[t]]
        R1, R2, R3 = a[None, :] - pts, b[None, :] - pts, c[None, :] - pts
        n1, n2, n3 = (np.linalg.norm(R, axis=1) for R in (R1, R2, R3))
        num = np.einsum("pd,pd->p", R1, np.cross(R2, R3))
        den = (n1 * n2 * n3 + np.einsum("pd,pd->p", R1, R2) * n3 + np.einsum("pd,pd->p", R1, R3) * n2
               + np.einsum("pd,pd->p", R2, R3) * n1)
        tot += 2.0 * np.arctan2(num, den)
    return np.abs(tot) > 2.0 * np.pi


def quadrature_points(topo):
    """Points y (n, 3), weights w (n,) including the triangle areas, and the
    triangle of every point, for the 6-point rule on every triangle."""
    bq, wq = quad.triangle_rule(4)
    P = topo.verts[topo.tris]                      # (F, 3, 3)
    y = np.einsum("qk,fkd->fqd", bq, P).reshape(-1, 3)
    w = (wq[None, :] * topo.area[:, None]).ravel()
    tri = np.repeat(np.arange(topo.F), len(wq))
    return y, w, tri


def rwg_currents(topo, coef, y, tri):
    """The RWG expansion sum_e coef[e] f_e at points y on triangles tri (the
    unit-flux form (x - p)/(2A) on T+, -(x - p)/(2A) on T-) and its surface
    divergence (constant s/A on each triangle)."""
    J = np.zeros((len(y), 3), dtype=np.complex128)
    div = np.zeros(len(y), dtype=np.complex128)
    for a in range(3):
        e = topo.t2e[tri, a]
        s = topo.sign[tri, a]
        p = topo.verts[topo.tris[tri, a]]
        A = topo.area[tri]
        J += (coef[e] * s / (2.0 * A))[:, None] * (y - p)
        div += coef[e] * s / A
    return J, div


def potentials(k, x, y, w, vH, vE, divE):
    """H vH(x) + E vE(x) for surface fields given at the quadrature points
    (vH, vE (n, 3) complex, divE (n,) the surface divergence of vE)."""
    x = np.atleast_2d(x)
    out = np.zeros((len(x), 3), dtype=np.complex128)
    for i, xi in enumerate(x):
        d = xi[None, :] - y
        r = np.sqrt(np.einsum("nd,nd->n", d, d))
        G = np.exp(1j * k * r) / (FOUR_PI * r)
        gradG = d * (G * (1j * k * r - 1.0) / (r * r))[:, None]
        Hv = np.sum(w[:, None] * np.cross(gradG, vH), axis=0)
        Ev = 1j * k * np.sum((w * G)[:, None] * vE, axis=0) - (1.0 / (1j * k)) * np.sum((w * divE)[:, None] * gradG,
                                                                                          axis=0)
        out[i] = Hv + Ev
    return out


def total_field(pr, x, dirs, pols, pts):
    """Total electric field at pts for the solved traces x of an
    oracle.pmchwt.Problem (rows of x and of dirs, pols: right-hand sides):
    E^inc + E^s outside the scatterers, the interior field inside.  Returns
    (E (nrhs, npts, 3), region (npts,), -1 outside, m inside scatterer m)."""
    x = np.atleast_2d(x)
    dirs, pols = np.atleast_2d(dirs), np.atleast_2d(pols)
    pts = np.atleast_2d(pts)
    if not hasattr(pr, "c_inc") or pr.c_inc.shape[0] != len(dirs):
        pr.rhs(dirs, pols)
    region = np.full(len(pts), -1)
    for m, T in enumerate(pr.topos):
        region[inside_mask(T, pts)] = m
    ke = pr.k_e
    E = np.zeros((len(x), len(pts), 3), dtype=np.complex128)
    out_pts = np.nonzero(region < 0)[0]
    for r in range(len(x)):
        for m, T in enumerate(pr.topos):
            y, w, tri = quadrature_points(T)
            blk = pr._blk(m)
            xm = x[r, blk]
            Em = T.E
            JD, _ = rwg_currents(T, xm[:Em], y, tri)
            JN, divN = rwg_currents(T, xm[Em:], y, tri)
            if len(out_pts):  # E^s = -H(gamma_D E^s) - E(gamma_N E^s), gamma_N E^s = x_N / k_e
                E[r, out_pts] -= potentials(ke, pts[out_pts], y, w, JD, JN / ke, divN / ke)
            ins = np.nonzero(region == m)[0]
            if len(ins):
                ci = pr.c_inc[r, blk]
                ID, _ = rwg_currents(T, xm[:Em] + ci[:Em], y, tri)
                IN, divI = rwg_currents(T, xm[Em:] + ci[Em:], y, tri)
                km = pr.k_i[m]
                E[r, ins] += potentials(km, pts[ins], y, w, ID, IN / km, divI / km)
        if len(out_pts):
            ph = np.exp(1j * ke * (pts[out_pts] @ dirs[r]))
            E[r, out_pts] += pols[r][None, :] * ph[:, None]
    return E, region
