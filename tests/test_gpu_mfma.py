"""Many-RHS operator products on the FP32 matrix cores (the PMCHWT block
product applied to all incident fields at once): parity with the FP64
oracle, agreement with the GEMV path of the same context, and batched solves.

Shapes are ragged on purpose: 120 and 480 edges (leading dimension padded to
128 / 480), 20 and 40 right-hand sides (80 and 160 real GEMM columns
against 128-wide tiles), one and three scatterers.  Tolerance: 1e-4
relative (FP32 operators), the stated bar for FP32 blocks; the measured
errors are reported.
"""

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


@pytest.mark.parametrize("case", ["sphere1", "sphere2", "cubes"])
@pytest.mark.parametrize("nrhs", [20, 40])
def test_mfma_apply_against_oracle_and_gemv(P, case, nrhs):
    if case == "cubes":
        meshes, eps, k = synth.three_cubes(2.1), 1.311 ** 2 + 0j, 2.1
    else:
        meshes, eps, k = [synth.icosphere(1 if case == "sphere1" else 2)], EPS, 1.7
    note(f"MFMA apply: {case}, nrhs={nrhs}")
    ctx = make_ctx(P, meshes, eps, k, qP=(1, 1, 1), nP=1, chi=0.5, precond="S_INT", precision=P.MIXED,
                   precisionP=P.MIXED)
    pr = opm.Problem(meshes, eps, k, qP=(1, 1, 1), nP=1, chiP=0.5, precond="S_INT")
    pr.assemble_A()
    pr.assemble_P()
    pr.assemble_mass()
    x = _x(nrhs, pr.N, 5)
    ops = {0: pr.A, 1: pr.precond_matrix() @ pr.A}
    for which, name in ((0, "A"), (1, "Ptilde A")):
        y = ctx.apply(which, x)                                       # matrix cores (nrhs >= 16)
        y4 = np.concatenate([ctx.apply(which, x[i:i + 4]) for i in range(0, nrhs, 4)])  # GEMV path
        e_or, e_gv = rel_fro(y, x @ ops[which].T), rel_fro(y, y4)
        note(f"  {name}: vs oracle {e_or:.2e}, vs GEMV path {e_gv:.2e}")
        assert e_or < 1e-4 and e_gv < 1e-5
    prof = ctx.profile()
    note(f"  mfma launches {prof['mfma_launches']}")
    assert prof["mfma_launches"] >= 1


def test_mfma_batched_solve(P):
    """32 right-hand sides (16 directions x 2 polarisations) solved as one
    batch through the matrix-core product: every current and cross section
    against the oracle's direct FP64 solve."""
    note("MFMA batched solve: icosphere(2), 32 RHS, k=2")
    mesh = synth.icosphere(2)
    ctx = make_ctx(P, [mesh], EPS, 2.0, qP=(1, 1, 1), nP=1, chi=0.6, precond="S_INT", precision=P.MIXED,
                   precisionP=P.MIXED)
    dirs, pols = synth.plane_wave_set(16, seed=3)
    x, st = ctx.solve(dirs, pols, P.solver_opts(tol=1e-8, restart=200, max_iter=1000, ir_max=3))
    prof = ctx.profile()
    pr = opm.Problem([mesh], EPS, 2.0)
    pr.assemble_A()
    xr = pr.solve_direct(pr.rhs(dirs, pols))
    se, ss = ctx.cross_sections(x, dirs, pols)
    se_r, ss_r = pr.cross_sections(xr, dirs, pols)
    err = max(rel_fro(x[i], xr[i]) for i in range(len(dirs)))
    e_ext = np.max(np.abs(se - se_r) / np.abs(se_r))
    e_sca = np.max(np.abs(ss - ss_r) / np.abs(ss_r))
    note(f"  iters={st.iterations} mfma launches={prof['mfma_launches']} max current err {err:.2e} "
         f"ext {e_ext:.2e} sca {e_sca:.2e}")
    assert prof["mfma_launches"] > 0
    assert err < 1e-5
    assert e_ext < 1e-5 and e_sca < 1e-5
