"""FP64 iterative refinement of MIXED solves (FP32 regular pairs and FP32
operator storage, FP64 singular pairs, Krylov basis and residual).

The refinement residual r = b - A x and the right-hand side's interior
product use the library's matrix-free FP64 product (every entry integrated
again in FP64, the FP64 singular blocks of the assembly), so refinement
converges to the solution of the FP64 Galerkin system, the oracle's.
Checks: that product against the oracle's assembled A and A^i to 1e-12, and
refined MIXED currents against the oracle's direct FP64 solve to 1e-9."""

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


def _cases():
    return {
        "sphere320": ([synth.icosphere(2)], EPS, 2.0),
        "three_cubes": (synth.three_cubes(2.1), 1.311 ** 2 + 0j, 2.1),
        "aggregate2": (synth.aggregate(2, 2, 6, seed=11), EPS, 3.0),
    }


def _interior_matrix(pr):
    Ai = np.zeros_like(pr.A)
    for m in range(pr.M):
        Ai[pr._blk(m), pr._blk(m)] = opm.pmchwt_block(pr.Ci[m], pr.Si[m], pr.k_i[m])
    return Ai


@pytest.mark.parametrize("precision", [1, 0])
def test_free_product_matches_oracle(P, precision):
    """pmchwt_apply(which = 2 / 3): A x and A^i x integrated in FP64 on the
    fly, for an A stored in FP32 (MIXED) or FP64, on two scatterers (one
    exterior operator over both, interior blocks per scatterer)."""
    meshes = synth.aggregate(2, 2, 3, seed=7)
    k = 1.7
    note(f"matrix-free FP64 product, aggregate of 2 prisms, precision={precision}")
    ctx = make_ctx(P, meshes, EPS, k, qP=(1, 1, 1), nP=1, chi=0.3, precond="S_INT", precision=precision,
                   precisionP=precision)
    pr = opm.Problem(meshes, EPS, k)
    pr.assemble_A()
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3, pr.N)) + 1j * rng.standard_normal((3, pr.N))
    for which, M in ((2, pr.A), (3, _interior_matrix(pr))):
        y = ctx.apply(which, x)
        ref = x @ M.T
        err = rel_fro(y, ref)
        note(f"  which={which}: rel. error {err:.2e}")
        assert err < 1e-12
    # one right-hand side more than a multiple of the kernel's chunk of 4
    x5 = rng.standard_normal((5, pr.N)) + 0j
    assert rel_fro(ctx.apply(2, x5), x5 @ pr.A.T) < 1e-12
    ctx.close()


@pytest.mark.parametrize("case", ["sphere320", "three_cubes", "aggregate2"])
def test_mixed_refinement_reaches_fp64_solution(P, case):
    meshes, eps, k = _cases()[case]
    note(f"MIXED solve with FP64 refinement: {case}, k_e={k}")
    d, p = synth.single_wave()
    pr = opm.Problem(meshes, eps, k)
    pr.assemble_A()
    xr = pr.solve_direct(pr.rhs(d, p))
    ctx = make_ctx(P, meshes, eps, k, qP=(1, 1, 1), nP=1, chi=0.6, precond="S_INT", precision=P.MIXED,
                   precisionP=P.MIXED)
    x0, st0 = ctx.solve(d, p, P.solver_opts(tol=1e-11, restart=200, max_iter=2000, ir_max=0))
    x, st = ctx.solve(d, p, P.solver_opts(tol=1e-11, restart=200, max_iter=4000, ir_max=6))
    e0, e1 = rel_fro(x0, xr), rel_fro(x, xr)
    se, ss = ctx.cross_sections(x, d, p)
    se_r, ss_r = pr.cross_sections(xr, d, p)
    note(f"  no refinement: err {e0:.2e} ({st0.iterations} it); refined: err {e1:.2e} "
         f"({st.iterations} it, {st.ir_steps} refinement steps); sigma_ext {se[0]:.12f} / {se_r[0]:.12f}")
    assert st.converged and st.ir_steps >= 1
    assert e1 < 1e-9
    assert abs(se[0] - se_r[0]) < 1e-9 * abs(se_r[0])
    assert abs(ss[0] - ss_r[0]) < 1e-9 * abs(ss_r[0])
    ctx.close()


def test_mixed_refinement_many_rhs_fp64_copy(P):
    """From 4 right-hand sides on, a MIXED solve takes its FP64 residuals from
    an FP64 copy of A (assembled once, in the context's operator slots with
    the FP32 state put back): 6 right-hand sides reach the oracle's direct
    FP64 solve like the matrix-free residual of a 2-RHS solve does, and the
    stored FP32 operator is unchanged afterwards (bit-identical products)."""
    meshes, eps, k = _cases()["sphere320"]
    d, p = synth.plane_wave_set(3, seed=21)
    pr = opm.Problem(meshes, eps, k)
    pr.assemble_A()
    xr = pr.solve_direct(pr.rhs(d, p))
    ctx = make_ctx(P, meshes, eps, k, qP=(1, 1, 1), nP=1, chi=0.6, precond="S_INT", precision=P.MIXED,
                   precisionP=P.MIXED)
    rng = np.random.default_rng(5)
    probe = rng.standard_normal((2, pr.N)) + 1j * rng.standard_normal((2, pr.N))
    before = ctx.apply(0, probe)
    so = P.solver_opts(tol=1e-11, restart=200, max_iter=4000, ir_max=6)
    x, st = ctx.solve(d, p, so)
    prof = ctx.profile()
    after = ctx.apply(0, probe)
    x2, st2 = ctx.solve(d[:2], p[:2], so)
    e6, e2 = rel_fro(x, xr), rel_fro(x2, xr[:2])
    note(f"  6 RHS (FP64 copy, {prof['ms_fp64_copy']:.2f} ms): err {e6:.2e}, {st.ir_steps} refinement steps; "
         f"2 RHS (matrix-free): err {e2:.2e}")
    assert st.converged and st2.converged
    assert prof["ms_fp64_copy"] > 0.0
    assert e6 < 1e-9 and e2 < 1e-9
    assert np.array_equal(before, after)
    ctx.close()
