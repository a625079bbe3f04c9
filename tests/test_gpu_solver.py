"""GPU solver checks: Table 1 matvec accounting on one sphere, the small-sphere
full Calderon case, mixed precision with refinement, error paths (the
three-cube preconditioner family is in test_gpu_precond_family.py)."""

import numpy as np
import pytest

import synth
from mie import mie_efficiencies
from gpu_common import note, rel_fro, make_ctx
from oracle import pmchwt as opm

pytestmark = pytest.mark.gpu

EPS = 3.17 + 0.01j


@pytest.fixture(scope="module")
def P():
    import paper_2008_04772_amd as lib
    return lib


@pytest.mark.parametrize("kind", ["I", "A", "D", "D_INT", "D_EXT", "S_INT", "S_EXT"])
def test_table1_counter_single_sphere(P, kind):
    """The solver's count of boundary-operator applications equals Table 1's
    formula for the iterations it took, with several completed restart cycles
    (rho = 6 preconditioned; rho = 30 unpreconditioned, where short cycles
    stagnate)."""
    rho = 30 if kind == "I" else 6
    note(f"Table 1 counter, icosphere(1), P = {kind}, rho = {rho}")
    ctx = make_ctx(P, [synth.icosphere(1)], EPS, 1.0, qP=(1, 1, 1), nP=1, chi=0.5, precond=kind)
    d, p = synth.single_wave()
    x, st = ctx.solve(d, p, P.solver_opts(tol=1e-8, restart=rho, max_iter=5000))
    note(f"  R={st.iterations} restarts={st.restarts} matvecs={st.matvecs}")
    assert st.converged and st.restarts >= 1
    assert st.restarts == st.iterations // rho
    assert st.matvecs == opm.table1_matvecs(kind, 1, st.iterations, rho)


def test_small_sphere_full_calderon(P):
    """The small sphere case (320 triangles, 960 unknowns, k_e = 1), FP64 dense
    A, full Calderon preconditioner P = A on the barycentric mesh with
    q = (4, 3, 2) and 4^4 singular points, GMRES tol 1e-6: currents and cross
    sections against the oracle's direct FP64 solve, Q_ext near Mie."""
    note("small sphere, full Calderon P = A, k=1")
    mesh = synth.icosphere(2)
    ctx = make_ctx(P, [mesh], EPS, 1.0, qP=(4, 3, 2), nP=4, chi=-1.0, precond="A")
    d, p = synth.single_wave()
    x, st = ctx.solve(d, p, P.solver_opts(tol=1e-6, restart=200, max_iter=400))
    pr = opm.Problem([mesh], EPS, 1.0)
    pr.assemble_A()
    xr = pr.solve_direct(pr.rhs(d, p))
    se, ss = ctx.cross_sections(x, d, p)
    se_r, ss_r = pr.cross_sections(xr, d, p)
    qm = mie_efficiencies(1.0, np.sqrt(EPS))
    note(f"  iters={st.iterations} matvecs={st.matvecs} err={rel_fro(x, xr):.2e} "
         f"Q_ext {se[0] / np.pi:.8f} (oracle {se_r[0] / np.pi:.8f}, Mie {qm[0]:.8f})")
    assert st.converged and st.iterations <= 12
    assert rel_fro(x, xr) < 1e-5
    assert abs(se[0] - se_r[0]) < 1e-5 * abs(se_r[0]) and abs(ss[0] - ss_r[0]) < 1e-5 * abs(ss_r[0])
    assert abs(se[0] / np.pi - qm[0]) < 0.08 * qm[0]


def test_mixed_precision_with_refinement(P):
    """FP32 regular pairs and operators, FP32 copies of the inverted mass
    matrices, FP64 singular pairs / Arnoldi / refinement residual: cross
    sections within 1e-5 of the FP64 oracle."""
    note("mixed precision solve, icosphere(2), k=2")
    mesh = synth.icosphere(2)
    ctx = make_ctx(P, [mesh], EPS, 2.0, qP=(1, 1, 1), nP=1, chi=0.6, precond="S_INT", precision=P.MIXED,
                   precisionP=P.MIXED)
    d, p = synth.single_wave()
    x, st = ctx.solve(d, p, P.solver_opts(tol=1e-8, restart=200, max_iter=1000, ir_max=3))
    se, ss = ctx.cross_sections(x, d, p)
    pr = opm.Problem([mesh], EPS, 2.0)
    pr.assemble_A()
    xr = pr.solve_direct(pr.rhs(d, p))
    se_r, ss_r = pr.cross_sections(xr, d, p)
    note(f"  iters={st.iterations} ir={st.ir_steps} err={rel_fro(x, xr):.2e} "
         f"ext {se[0]:.9f}/{se_r[0]:.9f} sca {ss[0]:.9f}/{ss_r[0]:.9f}")
    assert abs(se[0] - se_r[0]) < 1e-5 * abs(se_r[0])
    assert abs(ss[0] - ss_r[0]) < 1e-5 * abs(ss_r[0])


def test_error_paths(P):
    note("error paths")
    ctx = P.Context(0)
    v, t = synth.icosphere(1)
    with pytest.raises(P.PmchwtError) as e:
        ctx.add_scatterer(v, t[1:], EPS)
    assert e.value.code == P.ERR_INVALID_MESH
    with pytest.raises(P.PmchwtError) as e:
        ctx.solve(*synth.single_wave(), P.solver_opts())
    assert e.value.code == P.ERR_STATE
    ctx.add_scatterer(v, t, EPS)
    with pytest.raises(P.PmchwtError) as e:
        ctx.set_wavenumber(-1.0)
    assert e.value.code == P.ERR_INVALID_ARG
    ctx.set_wavenumber(1.0)
    with pytest.raises(P.PmchwtError) as e:
        ctx.assemble(P.assembly_opts((5, 3, 2), 4), P.assembly_opts(), "D")
    assert e.value.code == P.ERR_INVALID_ARG
    ctx.assemble(P.assembly_opts(), P.assembly_opts((1, 1, 1), 1, 0.5), "S_INT")
    x, st = ctx.solve(*synth.single_wave(), P.solver_opts(tol=1e-14, restart=5, max_iter=3),
                      allow_not_converged=True)
    assert not st.converged and st.iterations == 3
    with pytest.raises(P.PmchwtError) as e:
        ctx.solve(*synth.single_wave(), P.solver_opts(tol=1e-14, restart=5, max_iter=3))
    assert e.value.code == P.ERR_NOT_CONVERGED
    ctx.close()
