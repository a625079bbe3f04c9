"""Pins of the oracle's quadrature (no GPU).

* Triangle rules: exact for every monomial up to their degree.
* Evaluation counts equal the ones the paper quotes (Section 3.3):
  (q_near, q_medium, q_far) = (4,3,2) -> 36/16/9, (1,1,1) -> 1/1/1;
  q_singular = 6 -> 512/1280/1536 (vertex/edge/identical), q_singular = 1 -> 2/5/6.
* Sauter-Schwab maps: exact on polynomials over That x That (against product
  Gauss-Legendre with a Duffy collapse).
* Weakly singular 1/r: identical panels against the closed-form self
  integral of 1/|x-y| over a triangle; shared edge / shared vertex against an
  analytic inner potential (Wilton et al. 1984) with a composite outer rule.
"""

import math

import numpy as np
import pytest

from oracle import quadrature as q


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_triangle_rule_exactness(order):
    b, w = q.triangle_rule(order)
    assert abs(w.sum() - 1.0) < 1e-15
    for i in range(order + 1):
        for j in range(order + 1 - i):
            exact = 2.0 * math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)
            assert abs(np.sum(w * b[:, 1] ** i * b[:, 2] ** j) - exact) < 2e-16 * 4


def test_triangle_rule_not_exact_beyond_degree():
    # guards against a rule silently replaced by a higher one
    b, w = q.triangle_rule(2)
    exact = 2.0 * math.factorial(3) / math.factorial(5)
    assert abs(np.sum(w * b[:, 1] ** 3) - exact) > 1e-4


def test_paper_evaluation_counts():
    pts = {o: len(q.triangle_rule(o)[1]) for o in (1, 2, 3, 4)}
    assert [pts[4] ** 2, pts[3] ** 2, pts[2] ** 2] == [36, 16, 9]
    assert pts[1] ** 2 == 1
    for n, expect in ((4, (512, 1280, 1536)), (1, (2, 5, 6))):
        got = tuple(len(q.sauter_schwab(kind, n)[2]) for kind in (1, 2, 3))
        assert got == expect


def _product_that(n):
    g, w = q.gauss_legendre01(n)
    U, V = np.meshgrid(g, g, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    return np.stack([U.ravel(), (U * V).ravel()], 1), (WU * WV * U).ravel()


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_sauter_schwab_polynomial_exactness(kind):
    rng = np.random.default_rng(kind)
    C = rng.normal(size=(4, 4, 4, 4))

    def f(x, y):
        s = 0.0
        for a in range(4):
            for b in range(4 - a):
                for c in range(4 - a - b):
                    for d in range(4 - a - b - c):
                        s = s + C[a, b, c, d] * x[:, 0] ** a * x[:, 1] ** b * y[:, 0] ** c * y[:, 1] ** d
        return s

    P, W = _product_that(10)
    X = np.repeat(P, len(P), 0)
    Y = np.tile(P, (len(P), 1))
    WW = np.repeat(W, len(W)) * np.tile(W, len(W))
    ref = np.sum(WW * f(X, Y))
    xh, yh, w = q.sauter_schwab(kind, 6)
    assert abs(np.sum(w) - 0.25) < 1e-15
    assert abs(np.sum(w * f(xh, yh)) - ref) < 1e-13 * max(1.0, abs(ref))


def _area(P):
    return 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))


def self_integral_closed_form(P):
    """int_T int_T 1/|x-y| for a flat triangle with sides a, b, c and area A:
    (4 A^2 / 3) * sum_cyclic (1/a) ln(((a+b)^2 - c^2) / (b^2 - (c-a)^2))."""
    a = np.linalg.norm(P[1] - P[2])
    b = np.linalg.norm(P[2] - P[0])
    c = np.linalg.norm(P[0] - P[1])
    s = 0.0
    for (x, y, z) in ((a, b, c), (b, c, a), (c, a, b)):
        s += np.log(((x + y) ** 2 - z ** 2) / (y ** 2 - (z - x) ** 2)) / x
    return 4.0 * _area(P) ** 2 / 3.0 * s


def inner_potential(T, r):
    """int_T 1/|r - y| dy, analytic (Wilton et al. 1984): sum over edges of
    P0 ln((R+ + l+)/(R- + l-)) - |h| [atan(P0 l+/(R0^2+|h|R+)) - atan(P0 l-/(R0^2+|h|R-))]."""
    n = np.cross(T[1] - T[0], T[2] - T[0])
    n /= np.linalg.norm(n)
    h = (r - T[0]) @ n
    rho = r - np.outer(h, n)
    out = np.zeros(len(r))
    for i in range(3):
        p, qv = T[i], T[(i + 1) % 3]
        lh = (qv - p) / np.linalg.norm(qv - p)
        u = np.cross(lh, n)
        P0 = (p - rho) @ u
        lp = (qv - rho) @ lh
        lm = (p - rho) @ lh
        R02 = P0 ** 2 + h ** 2
        Rp = np.sqrt(lp ** 2 + R02)
        Rm = np.sqrt(lm ** 2 + R02)
        ah = np.abs(h)
        with np.errstate(divide="ignore", invalid="ignore"):
            lg = np.where(np.abs(P0) > 0, P0 * np.log((Rp + lp) / (Rm + lm)), 0.0)
        out += lg - ah * (np.arctan2(P0 * lp, R02 + ah * Rp) - np.arctan2(P0 * lm, R02 + ah * Rm))
    return out


def _composite_rule(T, levels):
    b, w = q.triangle_rule(4)
    tris = [np.asarray(T)]
    for _ in range(levels):
        new = []
        for t in tris:
            m01, m12, m20 = (t[0] + t[1]) / 2, (t[1] + t[2]) / 2, (t[2] + t[0]) / 2
            new += [np.array([t[0], m01, m20]), np.array([m01, t[1], m12]),
                    np.array([m20, m12, t[2]]), np.array([m01, m12, m20])]
        tris = new
    X = np.concatenate([b @ t for t in tris])
    W = np.concatenate([w * _area(t) for t in tris])
    return X, W


def test_inner_potential_against_brute_force():
    T = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1]])
    r = np.array([[0.3, 0.4, 1.5], [2.0, -1.0, 0.3], [0.4, 0.3, 0.02]])
    X, W = _composite_rule(T, 6)
    brute = np.array([np.sum(W / np.linalg.norm(X - ri, axis=1)) for ri in r])
    assert np.allclose(inner_potential(T, r), brute, rtol=1e-5)   # near point: composite rule limits
    assert np.allclose(inner_potential(T, r[:2]), brute[:2], rtol=1e-11)


def _ss_static(P1, P2, kind, n):
    xh, yh, w = q.sauter_schwab(kind, n)
    x = q.ref_to_phys(P1, xh)
    y = q.ref_to_phys(P2, yh)
    return np.sum(w * 4 * _area(P1) * _area(P2) / np.linalg.norm(x - y, axis=1))


def test_sauter_schwab_identical_static():
    P = np.array([[0.0, 0.0, 0.0], [1.0, 0.05, 0.1], [0.35, 0.8, -0.1]])
    ref = self_integral_closed_form(P)
    errs = [abs(_ss_static(P, P, 3, n) - ref) / ref for n in (4, 8, 12, 16)]
    assert errs[-1] < 1e-10
    assert errs[0] < 1e-3  # the paper's default order (n = 4)
    assert errs[3] < errs[1] < errs[0]


@pytest.mark.parametrize("kind", [2, 1])
def test_sauter_schwab_adjacent_static(kind):
    u = np.array([0.0, 0.0, 0.0])
    v = np.array([1.0, 0.0, 0.0])
    P1 = np.array([u, v, [0.4, 0.9, 0.0]])
    if kind == 2:
        P2 = np.array([u, v, [0.6, -0.7, 0.5]])
    else:
        P2 = np.array([u, [-0.8, 0.3, 0.4], [-0.5, -0.6, 0.2]])
    X, W = _composite_rule(P1, 6)
    ref = np.sum(W * inner_potential(P2, X))
    errs = [abs(_ss_static(P1, P2, kind, n) - ref) / ref for n in (2, 4, 8)]
    assert errs[2] < 1e-5
    assert errs[1] < 1e-3
