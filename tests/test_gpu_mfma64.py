"""Many-RHS FP64 products on the matrix cores: the PMCHWT operator (combined
operators of one scatterer, per-medium form for several) and the far-field
sum as a matrix product of plane-wave phases and surface currents (for the
scattering cross section over direction pairs xh, -xh).

Each is checked against the FP64 oracle and against the library's own VALU
path on the same input (the operator in chunks of 4 right-hand sides, below
the matrix-core threshold of 16; the far field in chunks of 4, below its
threshold of 8).  Shapes are ragged: 18, 20 and 40 right-hand sides (36, 40
and 80 real columns per output against 128-wide tiles; 18 also leaves two
right-hand sides after the groups of 4 of the preconditioner's CSR products), 9 and 20 far-field
right-hand sides (108 and 240 real columns), 200 directions, and a
10-triangle bipyramid whose 60 rule points give a K dimension (120) that is
not a multiple of the 16-wide K tile.  Bars: 1e-12 against the oracle, 1e-13
between the two paths (both FP64; they differ in summation order only)."""

import numpy as np
import pytest

import synth
from gpu_common import note, rel_fro, make_ctx
from oracle import pmchwt as opm

pytestmark = pytest.mark.gpu

EPS = 3.17 + 0.01j


@pytest.fixture(scope="module")
def P():
    import paper_2008_04772_amd as lib
    return lib


def _x(n, N, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, N)) + 1j * rng.normal(size=(n, N))


def bipyramid(n=5, h=0.8):
    """Closed n-gonal bipyramid (2n triangles, outward orientation)."""
    ang = 2 * np.pi * np.arange(n) / n
    v = np.concatenate([np.stack([np.cos(ang), np.sin(ang), np.zeros(n)], axis=1), [[0, 0, h], [0, 0, -h]]])
    t = [[i, (i + 1) % n, n] for i in range(n)] + [[(i + 1) % n, i, n + 1] for i in range(n)]
    return v, np.array(t, dtype=np.int64)


@pytest.mark.parametrize("case", ["sphere1", "sphere2", "cubes"])
@pytest.mark.parametrize("nrhs", [18, 20, 40])
def test_mfma64_apply_against_oracle_and_gemv(P, case, nrhs):
    if case == "cubes":
        meshes, eps, k = synth.three_cubes(2.1), 1.311 ** 2 + 0j, 2.1
    else:
        meshes, eps, k = [synth.icosphere(1 if case == "sphere1" else 2)], EPS, 1.7
    note(f"FP64 MFMA apply: {case}, nrhs={nrhs}")
    ctx = make_ctx(P, meshes, eps, k, qP=(1, 1, 1), nP=1, chi=0.5, precond="S_INT", precision=P.FP64,
                   precisionP=P.FP64)
    pr = opm.Problem(meshes, eps, k, qP=(1, 1, 1), nP=1, chiP=0.5, precond="S_INT")
    pr.assemble_A()
    x = _x(nrhs, pr.N, 7)
    y = ctx.apply(0, x)                                                    # matrix cores (nrhs >= 16)
    y4 = np.concatenate([ctx.apply(0, x[i:i + 4]) for i in range(0, nrhs, 4)])  # GEMV path
    e_or, e_gv = rel_fro(y, x @ pr.A.T), rel_fro(y, y4)
    prof = ctx.profile()
    note(f"  A: vs oracle {e_or:.2e}, vs GEMV path {e_gv:.2e}, mfma launches {prof['mfma_launches']}")
    assert prof["mfma_launches"] >= 1
    assert e_or < 1e-12 and e_gv < 1e-13
    # the FP64 preconditioner: the sparse FP32 mass inverse on the matrix cores
    # (block-sparse tiles, inputs rounded to FP32) with its FP64 refinement
    pr.assemble_P()
    pr.assemble_mass()
    yp = ctx.apply(1, x)
    yp4 = np.concatenate([ctx.apply(1, x[i:i + 4]) for i in range(0, nrhs, 4)])
    e_or, e_gv = rel_fro(yp, x @ (pr.precond_matrix() @ pr.A).T), rel_fro(yp, yp4)
    note(f"  Ptilde A: vs oracle {e_or:.2e}, vs CSR path {e_gv:.2e}")
    assert e_or < 1e-10 and e_gv < 1e-10
    ctx.close()


@pytest.mark.parametrize("mesh", ["bipyramid", "sphere2", "two prisms"])
@pytest.mark.parametrize("nrhs", [9, 20])
def test_far_field_mfma_against_oracle_and_valu(P, mesh, nrhs):
    if mesh == "bipyramid":
        meshes = [bipyramid()]
    elif mesh == "sphere2":
        meshes = [synth.icosphere(2)]
    else:
        meshes = synth.aggregate(2, 2, 3, seed=7)
    F = sum(len(t) for _, t in meshes)
    note(f"far field on the matrix cores: {mesh} ({F} triangles, K = {12 * F}), nrhs={nrhs}")
    k = 3.3
    ctx = make_ctx(P, meshes, EPS, k, qP=(1, 1, 1), nP=1, chi=0.5, precond="S_INT")
    pr = opm.Problem(meshes, EPS, k)
    x = _x(nrhs, pr.N, 11)
    rng = np.random.default_rng(4)
    obs = rng.normal(size=(200, 3))
    obs /= np.linalg.norm(obs, axis=1, keepdims=True)
    Fm = ctx.far_field(x, obs)                                                      # nrhs >= 8
    Fv = np.concatenate([ctx.far_field(x[i:i + 4], obs) for i in range(0, nrhs, 4)])  # VALU sum
    Fo = pr.far_field(x, obs)
    e_or, e_v = rel_fro(Fm, Fo), rel_fro(Fm, Fv)
    note(f"  vs oracle {e_or:.2e}, vs VALU path {e_v:.2e}")
    assert e_or < 1e-12 and e_v < 1e-13
    ctx.close()


def test_fp64_batched_solve_cross_sections(P):
    """24 right-hand sides in FP64 (matrix-core products, matrix-core far
    field): currents against the oracle's direct solve, both cross sections
    against the oracle's."""
    mesh = synth.icosphere(2)
    note("FP64 batched solve on the matrix cores: icosphere(2), 24 RHS, k=2")
    ctx = make_ctx(P, [mesh], EPS, 2.0, qP=(1, 1, 1), nP=1, chi=0.6, precond="S_INT", precision=P.FP64,
                   precisionP=P.FP64)
    dirs, pols = synth.plane_wave_set(12, seed=9)
    x, st = ctx.solve(dirs, pols, P.solver_opts(tol=1e-11, restart=200, max_iter=1000))
    pr = opm.Problem([mesh], EPS, 2.0)
    pr.assemble_A()
    xr = pr.solve_direct(pr.rhs(dirs, pols))
    se, ss = ctx.cross_sections(x, dirs, pols)
    se_r, ss_r = pr.cross_sections(xr, dirs, pols)
    err = max(rel_fro(x[i], xr[i]) for i in range(len(dirs)))
    e_ext = np.max(np.abs(se - se_r) / np.abs(se_r))
    e_sca = np.max(np.abs(ss - ss_r) / np.abs(ss_r))
    prof = ctx.profile()
    note(f"  iters={st.iterations} mfma launches={prof['mfma_launches']} current {err:.2e} ext {e_ext:.2e} "
         f"sca {e_sca:.2e}")
    assert st.converged and prof["mfma_launches"] > 0
    assert err < 1e-9 and e_ext < 1e-9 and e_sca < 1e-9
    ctx.close()


def _sphere_grid(n_theta=64, n_phi=128):
    """The cross sections' direction grid: Gauss-Legendre in cos(theta) x
    uniform in phi, with weights."""
    ct, wt = np.polynomial.legendre.leggauss(n_theta)
    ph = 2 * np.pi * np.arange(n_phi) / n_phi
    CT, PH = np.meshgrid(ct, ph, indexing="ij")
    st = np.sqrt(1 - CT ** 2)
    obs = np.stack([st * np.cos(PH), st * np.sin(PH), CT], axis=-1).reshape(-1, 3)
    return obs, (wt[:, None] * np.full(n_phi, 2 * np.pi / n_phi)[None, :]).ravel()


@pytest.mark.parametrize("mesh", ["bipyramid", "sphere2", "two prisms"])
def test_sigma_sca_antipodal_pairs(P, mesh):
    """sigma_sca with 8 or more right-hand sides forms the far field for the
    upper half of the direction grid and takes the antipodes from the same
    cosine and sine sums.  It must equal the grid sum of w |F|^2 over the
    library's own far field at every grid direction (matrix cores, no
    pairing), and sigma_sca of the VALU path (chunks of 4 right-hand sides):
    the same directions and weights up to rounding, other summation orders.
    The bipyramid's 60 rule points leave a ragged K tile."""
    meshes = {"bipyramid": lambda: [bipyramid()], "sphere2": lambda: [synth.icosphere(2)],
              "two prisms": lambda: synth.aggregate(2, 2, 3, seed=7)}[mesh]()
    note(f"sigma_sca from antipodal pairs: {mesh}, 9 RHS")
    ctx = make_ctx(P, meshes, EPS, 2.7, qP=(1, 1, 1), nP=1, chi=0.5, precond="S_INT")
    _, N = ctx.sizes()
    x = _x(9, N, 13)
    d, p = synth.plane_wave_set(5, seed=3)
    d, p = d[:9], p[:9]
    se, ss = ctx.cross_sections(x, d, p)
    obs, w = _sphere_grid()
    Ff = ctx.far_field(x, obs)
    ss_full = np.einsum("o,rod->r", w, np.abs(Ff) ** 2)
    chunks = [ctx.cross_sections(x[i:i + 4], d[i:i + 4], p[i:i + 4]) for i in range(0, 9, 4)]
    se4 = np.concatenate([c[0] for c in chunks])
    ss4 = np.concatenate([c[1] for c in chunks])
    e_full = np.max(np.abs(ss - ss_full) / np.abs(ss_full))
    e_v = np.max(np.abs(ss - ss4) / np.abs(ss4))
    e_ext = np.max(np.abs(se - se4) / np.abs(se4))
    note(f"  sigma_sca vs full grid {e_full:.2e}, vs VALU path {e_v:.2e}; sigma_ext vs VALU path {e_ext:.2e}")
    assert e_full < 1e-12 and e_v < 1e-12 and e_ext < 1e-12
    ctx.close()
