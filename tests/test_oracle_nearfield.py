"""Pins of the oracle's field evaluation (oracle/nearfield.py) against what
the mathematics fixes, independently of the GPU path:
  * the inside test on meshes whose interior is known;
  * the Stratton-Chu representation (Section 2) of a plane wave, an entire
    solution of Maxwell's equations, from its exact traces on a closed
    icosphere (any closed surface, polyhedral ones included):
    H(gamma_D E) + E(gamma_N E) equals E inside and vanishes outside, up to
    the error of the 6-point rule, which shrinks under refinement (about
    1e-10 at 5120 triangles; a wrong sign of either potential gives an O(1)
    error);
  * the scattered field of a solved problem at large distance against the
    far-field pattern F (itself pinned against the Mie series):
    r exp(-ikr) E^s(r xhat) -> F(xhat), with an O(1/(kr)) difference."""

import numpy as np

import synth
from oracle import nearfield as nf
from oracle import pmchwt as opm
from oracle.mesh import Topology


def _dirs(n, seed):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_inside_mask_sphere_and_cubes():
    T = Topology(*synth.icosphere(2))
    u = _dirs(30, 1)
    assert nf.inside_mask(T, 0.4 * u).all()
    assert not nf.inside_mask(T, 1.6 * u).any()
    assert not nf.inside_mask(T, 5.0 * u).any()
    cubes = synth.three_cubes(2.1)
    centres = np.array([[-0.8, 0.2, 0.2], [0.2, 0.2, 0.2], [1.2, 0.2, 0.2]])
    for m, (v, t) in enumerate(cubes):
        got = nf.inside_mask(Topology(v, t), centres)
        assert got[m] and got.sum() == 1


def _plane_wave_traces(T, k, d, p):
    y, w, tri = nf.quadrature_points(T)
    n = T.normal[tri]
    E = p[None, :] * np.exp(1j * k * (y @ d))[:, None]
    gD = np.cross(E, n)                          # gamma_D E = E x n
    gN = np.cross(np.cross(d[None, :], E), n)    # (1/ik) curl E x n, curl E = ik d x E
    divN = -1j * k * np.einsum("nd,nd->n", n, E)  # n . curl(d x E) = -ik n . E
    return y, w, gD, gN, divN


def test_stratton_chu_plane_wave():
    k = 2.0
    d = np.array([0.3, -0.2, 0.932737905308882])
    d /= np.linalg.norm(d)
    p = np.cross(d, [1.0, 0.0, 0.0])
    p = (p / np.linalg.norm(p)).astype(np.complex128)
    xin = 0.45 * _dirs(12, 2)
    xout = 2.5 * _dirs(12, 3)
    errs_in, errs_out = [], []
    for lvl in (2, 3, 4):
        T = Topology(*synth.icosphere(lvl))
        y, w, gD, gN, divN = _plane_wave_traces(T, k, d, p)
        Ein = nf.potentials(k, xin, y, w, gD, gN, divN)
        ref = p[None, :] * np.exp(1j * k * (xin @ d))[:, None]
        Eout = nf.potentials(k, xout, y, w, gD, gN, divN)
        errs_in.append(np.max(np.abs(Ein - ref)))
        errs_out.append(np.max(np.abs(Eout)))
    assert errs_in[-1] < 1e-9 and errs_out[-1] < 1e-9
    assert errs_in[0] > errs_in[1] > errs_in[2]
    assert errs_out[0] > errs_out[1] > errs_out[2]


def test_scattered_field_tends_to_far_field():
    mesh = synth.icosphere(1)
    k = 2.0
    d, p = synth.single_wave()
    pr = opm.Problem([mesh], 3.17 + 0.01j, k)
    pr.assemble_A()
    x = pr.solve_direct(pr.rhs(d, p))
    obs = _dirs(5, 4)
    F = pr.far_field(x, obs)[0]
    diffs = []
    for R in (100.0, 1000.0):
        E, region = nf.total_field(pr, x, d, p, R * obs)
        assert (region == -1).all()
        Es = E[0] - p[0][None, :] * np.exp(1j * k * (R * obs @ d[0]))[:, None]
        diffs.append(np.max(np.abs(R * np.exp(-1j * k * R) * Es - F)) / np.max(np.abs(F)))
    assert diffs[1] < 2e-3
    assert diffs[1] < 0.2 * diffs[0]
