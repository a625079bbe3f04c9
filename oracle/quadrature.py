"""Quadrature rules used by the Galerkin integrals (oracle, test infrastructure only).

Regular pairs (disjoint closures) use tensor products of symmetric triangle
rules; the quadrature orders 4 / 3 / 2 / 1 use 6 / 4 / 3 / 1 points per
triangle, i.e. 36 / 16 / 9 / 1 evaluations per pair (Section 3.3, the
paragraph on default and minimal quadrature orders).  Reading: these are the
symmetric rules of Dunavant (1985) of polynomial degree 4, 3, 2, 1.

Singular pairs (identical, shared edge, shared vertex) use the Sauter-Schwab
transformations (Sauter & Schwab, Boundary Element Methods, 2011, Sec. 5.2.1)
with n Gauss-Legendre points per coordinate on [0,1]^4 and 6 / 5 / 2
sub-regions.  n = 4 reproduces the 1536 / 1280 / 512 evaluations quoted for
q_singular = 6 and n = 1 the 6 / 5 / 2 quoted for q_singular = 1 (Section 3.3).

Pinned by tests/test_oracle_quadrature.py: monomial exactness of every
triangle rule, polynomial exactness of the Sauter-Schwab maps against product
Gauss rules, and the weakly singular 1/r integral against an analytic inner
potential.
"""

import math
import numpy as np

# Reference triangle for the triangle rules: (0,0), (1,0), (0,1); points are
# barycentric (l0, l1, l2) with x = l0*P0 + l1*P1 + l2*P2; weights sum to 1
# (multiply by the physical area).


def _orbit3(beta):
    a = 1.0 - 2.0 * beta
    return [(a, beta, beta), (beta, a, beta), (beta, beta, a)]


def _monomial_ref(i, j):
    """Mean of x^i y^j over the reference triangle (area-normalised)."""
    return 2.0 * math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)


def _degree4_params():
    """Dunavant's 6-point degree-4 rule, refined to double precision by Gauss-Newton.

    Two orbits (1-2b, b, b) with weights w1, w2 and 3 w1 + 3 w2 = 1.  The
    published values (b1 ~ 0.44594849, b2 ~ 0.09157621, w1 ~ 0.22338159) are
    only starting points; the refinement solves the moment equations for all
    monomials of degree <= 4.
    """
    x = np.array([0.445948490915965, 0.091576213509771, 0.223381589678011])
    mons = [(i, j) for i in range(5) for j in range(5 - i)]

    def resid(p):
        b1, b2, w1 = p
        w2 = 1.0 / 3.0 - w1
        pts = _orbit3(b1) + _orbit3(b2)
        ws = [w1] * 3 + [w2] * 3
        r = []
        for (i, j) in mons:
            s = sum(w * (l[1] ** i) * (l[2] ** j) for l, w in zip(pts, ws))
            r.append(s - _monomial_ref(i, j))
        return np.array(r)

    for _ in range(8):
        r = resid(x)
        J = np.zeros((len(r), 3))
        for c in range(3):
            dx = np.zeros(3)
            dx[c] = 1e-7
            J[:, c] = (resid(x + dx) - resid(x - dx)) / 2e-7
        x = x - np.linalg.lstsq(J, r, rcond=None)[0]
    return x


_B1, _B2, _W1 = _degree4_params()


def triangle_rule(order):
    """Symmetric triangle rule of polynomial degree ``order`` (1..4).

    Returns (bary (n,3), weights (n,)) with weights summing to 1.
    """
    if order == 1:
        return np.array([[1 / 3, 1 / 3, 1 / 3]]), np.array([1.0])
    if order == 2:
        return np.array(_orbit3(1.0 / 6.0)), np.full(3, 1.0 / 3.0)
    if order == 3:
        pts = [(1 / 3, 1 / 3, 1 / 3)] + _orbit3(0.2)
        return np.array(pts), np.array([-27.0 / 48.0] + [25.0 / 48.0] * 3)
    if order == 4:
        pts = _orbit3(_B1) + _orbit3(_B2)
        return np.array(pts), np.array([_W1] * 3 + [1.0 / 3.0 - _W1] * 3)
    raise ValueError("triangle rule order must be 1..4")


def gauss_legendre01(n):
    """n-point Gauss-Legendre rule on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


# ---------------------------------------------------------------------------
# Sauter-Schwab.  Reference element That = {(x1, x2): 0 <= x2 <= x1 <= 1},
# mapped to a physical triangle (P0, P1, P2) by  x = P0 + x1 (P1-P0) + x2 (P2-P1),
# |Jacobian| = 2 * area.  For the shared-edge case the common edge is
# {x2 = 0} in both elements with the same parametrisation (P0, P1 shared, in
# the same order); for the shared-vertex case the common vertex is P0.
# Each function returns (xhat (N,2), yhat (N,2), w (N)) with
#     sum w f(xhat, yhat)  ~  int_That int_That f(xhat, yhat) dyhat dxhat.
# ---------------------------------------------------------------------------


def _grid4(n):
    g, w = gauss_legendre01(n)
    X = np.meshgrid(g, g, g, g, indexing="ij")
    W = np.meshgrid(w, w, w, w, indexing="ij")
    xi, e1, e2, e3 = [a.ravel() for a in X]
    wt = W[0].ravel() * W[1].ravel() * W[2].ravel() * W[3].ravel()
    return xi, e1, e2, e3, wt


def ss_identical(n):
    xi, e1, e2, e3, wt = _grid4(n)
    jac = wt * xi ** 3 * e1 ** 2 * e2
    maps = [
        ((xi, xi * (1 - e1 + e1 * e2)), (xi * (1 - e1 * e2 * e3), xi * (1 - e1))),
        ((xi * (1 - e1 * e2 * e3), xi * (1 - e1)), (xi, xi * (1 - e1 + e1 * e2))),
        ((xi, xi * e1 * (1 - e2 + e2 * e3)), (xi * (1 - e1 * e2), xi * e1 * (1 - e2))),
        ((xi * (1 - e1 * e2), xi * e1 * (1 - e2)), (xi, xi * e1 * (1 - e2 + e2 * e3))),
        ((xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3)), (xi, xi * e1 * (1 - e2))),
        ((xi, xi * e1 * (1 - e2)), (xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3))),
    ]
    return _stack(maps, [jac] * 6)


def ss_edge(n):
    xi, e1, e2, e3, wt = _grid4(n)
    j1 = wt * xi ** 3 * e1 ** 2
    j2 = j1 * e2
    maps = [
        ((xi, xi * e1 * e3), (xi * (1 - e1 * e2), xi * e1 * (1 - e2))),
        ((xi, xi * e1), (xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3))),
        ((xi * (1 - e1 * e2), xi * e1 * (1 - e2)), (xi, xi * e1 * e2 * e3)),
        ((xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3)), (xi, xi * e1)),
        ((xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3)), (xi, xi * e1 * e2)),
    ]
    return _stack(maps, [j1, j2, j2, j2, j2])


def ss_vertex(n):
    xi, e1, e2, e3, wt = _grid4(n)
    jac = wt * xi ** 3 * e2
    maps = [
        ((xi, xi * e1), (xi * e2, xi * e2 * e3)),
        ((xi * e2, xi * e2 * e3), (xi, xi * e1)),
    ]
    return _stack(maps, [jac, jac])


def _stack(maps, jacs):
    xs, ys, ws = [], [], []
    for ((x1, x2), (y1, y2)), j in zip(maps, jacs):
        xs.append(np.stack([x1, x2], axis=1))
        ys.append(np.stack([y1, y2], axis=1))
        ws.append(j)
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(ws)


def sauter_schwab(kind, n):
    """kind: 3 = identical, 2 = shared edge, 1 = shared vertex."""
    return {3: ss_identical, 2: ss_edge, 1: ss_vertex}[kind](n)


def ref_to_phys(P, xhat):
    """Map That points to the physical triangle with ordered vertices P (3,3)."""
    return P[0] + xhat[:, :1] * (P[1] - P[0]) + xhat[:, 1:2] * (P[2] - P[1])
