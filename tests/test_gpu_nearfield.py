"""pmchwt_near_field: the total electric field at points outside and inside
the scatterers (Stratton-Chu representation of Section 2, the field maps of
Section 5) against the oracle's evaluation of the same representation with
the same currents (oracle/nearfield.py, itself pinned by the representation
of a plane wave and the far-field limit).  FP64 throughout: 1e-11 relative
to the largest field value; regions must agree exactly."""

import numpy as np
import pytest

import synth
from gpu_common import note, make_ctx
from oracle import nearfield as nf
from oracle import pmchwt as opm

pytestmark = pytest.mark.gpu

EPS = 3.17 + 0.01j


@pytest.fixture(scope="module")
def P():
    import paper_2008_04772_amd as lib
    return lib


def _dirs(n, seed):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def _check(P, meshes, k, pts, precision):
    d, p = synth.plane_wave_set(2, seed=9)
    ctx = make_ctx(P, meshes, EPS, k, qP=(1, 1, 1), nP=1, chi=0.5, precond="S_INT", precision=precision,
                   precisionP=precision)
    x, st = ctx.solve(d, p, P.solver_opts(tol=1e-10, restart=200, max_iter=2000, ir_max=3 if precision else 0))
    E, reg = ctx.near_field(x, d, p, pts)
    ctx.close()
    pr = opm.Problem(meshes, EPS, k)
    pr.assemble_A()
    Er, regr = nf.total_field(pr, x, d, p, pts)
    err = np.max(np.abs(E - Er)) / np.max(np.abs(Er))
    note(f"  {len(pts)} points ({int((reg >= 0).sum())} inside): max relative difference {err:.2e}")
    assert (reg == regr).all()
    assert err < 1e-11
    return E, reg


@pytest.mark.parametrize("precision", [0, 1])
def test_near_field_sphere(P, precision):
    note(f"near field, 320-triangle sphere, k = 2, precision {precision}")
    u = _dirs(20, 1)
    g = np.linspace(-1.5, 1.5, 5)
    plane = np.array([[a, 1.25, b] for a in g for b in g])  # a plane outside the sphere
    pts = np.concatenate([0.5 * u[:8], 1.6 * u[8:14], 3.0 * u[14:], plane])
    _check(P, [synth.icosphere(2)], 2.0, pts, precision)


def test_near_field_two_prisms(P):
    meshes = synth.aggregate(2, 2, 3, seed=7)
    note("near field, aggregate of two prisms, k = 1.5")
    cents = np.array([v.mean(axis=0) for v, t in meshes])
    allv = np.concatenate([v for v, t in meshes])
    lo, hi = allv.min(axis=0), allv.max(axis=0)
    g = np.linspace(0.0, 1.0, 4)
    box = np.array([lo + (hi - lo) * np.array([a, b, c]) for a in g for b in g for c in g])
    far = cents.mean(axis=0) + 4.0 * _dirs(6, 2)
    pts = np.concatenate([cents, box, far])
    E, reg = _check(P, meshes, 1.5, pts, 0)
    assert reg[0] == 0 and reg[1] == 1
