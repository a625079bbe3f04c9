"""GPU parity: the HIP library against the FP64 oracle on identical inputs.

Tolerances (stated per operator): FP64 Galerkin blocks 1e-10 relative
(Frobenius and max-entry), FP32-regular / FP64-singular blocks 1e-4, FP64
solves at tol 1e-11 to 1e-8, cross sections 1e-6 (the oracle's
and the library's far-field rules are identical).
"""

import numpy as np
import pytest

import synth
from gpu_common import note, rel_fro, rel_max, make_ctx
from oracle import operators as ops
from oracle import pmchwt as opm
from oracle.mesh import Topology, Barycentric

pytestmark = pytest.mark.gpu

EPS = 3.17 + 0.01j


@pytest.fixture(scope="module")
def P():
    import paper_2008_04772_amd as lib
    return lib


@pytest.fixture(scope="module")
def sphere1():
    return synth.icosphere(1)


@pytest.fixture(scope="module")
def oracle_sphere1(sphere1):
    pr = opm.Problem([sphere1], EPS, 1.3, precond="D", qP=(4, 3, 2), nP=4)
    pr.assemble_A()
    pr.assemble_P()
    pr.assemble_mass()
    return pr


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-4)])
def test_A_blocks(P, sphere1, oracle_sphere1, precision, tol):
    note(f"A blocks: icosphere(1), k=1.3, precision={precision}")
    ctx = make_ctx(P, [sphere1], EPS, 1.3, precond="D", precision=precision)
    pr = oracle_sphere1
    for op, med, ref in ((P.OP_S, P.EXT, pr.Se), (P.OP_C, P.EXT, pr.Ce),
                         (P.OP_S, P.INT, pr.Si[0]), (P.OP_C, P.INT, pr.Ci[0])):
        got = ctx.get_block(op, med, P.RWG, 0, 0)
        note(f"  op={op} med={med} fro={rel_fro(got, ref):.2e} max={rel_max(got, ref):.2e}")
        assert rel_fro(got, ref) < tol and rel_max(got, ref) < tol


def test_P_blocks_full_and_mass(P, sphere1, oracle_sphere1):
    note("P (=D) BC blocks and mixed mass: icosphere(1), q=(4,3,2), n=4")
    ctx = make_ctx(P, [sphere1], EPS, 1.3, precond="D")
    pr = oracle_sphere1
    for op, med, key in ((P.OP_S, P.INT, ("int", 0, "S")), (P.OP_C, P.INT, ("int", 0, "C")),
                         (P.OP_S, P.EXT, ("ext", 0, "S")), (P.OP_C, P.EXT, ("ext", 0, "C"))):
        got = ctx.get_block(op, med, P.BC, 0, 0)
        ref = pr.PBC[key]
        note(f"  {key} fro={rel_fro(got, ref):.2e} max={rel_max(got, ref):.2e}")
        assert rel_fro(got, ref) < 1e-10 and rel_max(got, ref) < 1e-10
    M = ctx.get_mass(0)
    note(f"  mass fro={rel_fro(M, pr.MA[0]):.2e}")
    assert rel_fro(M, pr.MA[0]) < 1e-12


@pytest.mark.parametrize("chi,prec,tol", [(0.3, 0, 1e-10), (0.0, 0, 1e-10), (0.3, 1, 1e-4)])
def test_P_nearfield_cutoff(P, sphere1, chi, prec, tol):
    """FP64 entries to 1e-10; a mixed-precision P integrates them in FP32
    (stored in FP64): the FP32 bar 1e-4."""
    note(f"near-field S^i on BC: icosphere(1), chi={chi}, q=(1,1,1), n=1, precision {prec}")
    ctx = make_ctx(P, [sphere1], EPS, 2.0, qP=(1, 1, 1), nP=1, chi=chi, precond="S_INT", precisionP=prec)
    B = Barycentric(Topology(*sphere1))
    lo, hi = ops.bc_bboxes(B)
    mask = ops.nearfield_mask(lo, hi, chi)
    ref = ops.assemble_bc(B, 2.0 * np.sqrt(EPS), (1, 1, 1), 1, ("S",))["S"] * mask
    got = ctx.get_block(P.OP_S, P.INT, P.BC, 0, 0)
    # entries beyond the cutoff are exactly zero; kept ones match the oracle
    # (some kept entries vanish by symmetry, so they are not tested for != 0)
    assert np.all(got[~mask] == 0)
    note(f"  fro={rel_fro(got, ref):.2e} max={rel_max(got, ref):.2e} nnz={mask.sum()}")
    assert rel_fro(got, ref) < tol and rel_max(got, ref) < tol


def test_rhs_apply_solve_cross_sections(P, sphere1, oracle_sphere1):
    note("rhs / apply / solve / cross sections: icosphere(1), P = D")
    pr = oracle_sphere1
    ctx = make_ctx(P, [sphere1], EPS, 1.3, precond="D")
    dirs, pols = synth.plane_wave_set(2, seed=7)
    b_ref = pr.rhs(dirs, pols)
    b = ctx.rhs(dirs, pols)
    note(f"  rhs fro={rel_fro(b, b_ref):.2e}")
    assert rel_fro(b, b_ref) < 1e-11
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, pr.N)) + 1j * rng.normal(size=(2, pr.N))
    y = ctx.apply(0, x)
    assert rel_fro(y, x @ pr.A.T) < 1e-11
    Pt = pr.precond_matrix()
    y = ctx.apply(1, x)
    note(f"  apply Ptilde A fro={rel_fro(y, x @ (Pt @ pr.A).T):.2e}")
    assert rel_fro(y, x @ (Pt @ pr.A).T) < 1e-10
    xs, st = ctx.solve(dirs, pols, P.solver_opts(tol=1e-12, restart=200, max_iter=500))
    x_ref = pr.solve_direct(b_ref)
    note(f"  solve iters={st.iterations} matvecs={st.matvecs} err={rel_fro(xs, x_ref):.2e}")
    assert rel_fro(xs, x_ref) < 1e-9
    se, ss = ctx.cross_sections(xs, dirs, pols)
    se_ref, ss_ref = pr.cross_sections(x_ref, dirs, pols)
    note(f"  sigma_ext {se} vs {se_ref}; sigma_sca {ss} vs {ss_ref}")
    assert np.allclose(se, se_ref, rtol=1e-8) and np.allclose(ss, ss_ref, rtol=1e-8)
    obs = synth.plane_wave_set(3, seed=9)[0]
    F = ctx.far_field(xs, obs)
    assert rel_fro(F, pr.far_field(x_ref, obs)) < 1e-9


@pytest.mark.parametrize("prec,method,bar", [(0, 0, 1e-10), (0, 1, 1e-10), (1, 0, 1e-4), (1, 1, 1e-4), (1, 2, 1e-4)])
def test_mass_inverse_paths(P, sphere1, prec, method, bar):
    """Every way of applying M_A^-1: the sparse FP32 inverse on the graph
    ball (mass_method 0, the default; radius 8 and 14 Chebyshev steps for an
    FP64 preconditioner, which refines each of its products once against the
    FP64 M_A; radius 6 and 12 steps for MIXED; its last-step residual over
    the ball small), dense Gauss-Jordan (1), the dense
    inverse of mass_method 2 (FP32 by the Chebyshev iteration, its residual
    ||I - X M_A||_F / sqrt(n) below the stopping tolerance 1e-6; FP64 by
    Gauss-Jordan).  The preconditioned operator built from any of them
    matches the oracle's exact one (FP64 1e-10, mixed 1e-4)."""
    note(f"mass inverse, precision {prec}, method {method}")
    ctx = P.Context(0)
    ctx.add_scatterer(*sphere1, EPS)
    ctx.set_wavenumber(2.0)
    ctx.assemble(P.assembly_opts((4, 3, 2), 4, -1.0, prec),
                 P.assembly_opts((1, 1, 1), 1, 0.5, prec, mass_method=method), "S_INT")
    prof = ctx.profile()
    note(f"  Chebyshev steps {prof['mass_iterations']}, residual {prof['mass_residual']:.2e}")
    if method == 0:
        assert prof["mass_iterations"] == (14 if prec == 0 else 12)
        assert prof["mass_residual"] <= (1e-6 if prec == 0 else 1e-5)
    elif method == 2 and prec == 1:
        assert prof["mass_iterations"] > 0 and prof["mass_residual"] <= 1e-6
    else:
        assert prof["mass_iterations"] == 0
    pr = opm.Problem([sphere1], EPS, 2.0, qP=(1, 1, 1), nP=1, chiP=0.5, precond="S_INT")
    pr.assemble_A()
    pr.assemble_P()
    pr.assemble_mass()
    rng = np.random.default_rng(11)
    x = rng.normal(size=(2, pr.N)) + 1j * rng.normal(size=(2, pr.N))
    y = ctx.apply(1, x)
    e = rel_fro(y, x @ (pr.precond_matrix() @ pr.A).T)
    note(f"  Ptilde A vs oracle {e:.2e}")
    assert e < bar


def test_mass_inverse_radius(P, sphere1):
    """The radius of the sparse inverse's column sets (mass_hops) against
    the oracle's exact preconditioned operator: the error of P~ A falls with
    the radius (mixed precision, down to its FP32 floor; the default radius 6
    within the 1e-4 bar of the mixed preconditioner), and one refinement
    step against the FP64 M_A squares it (FP64 at radius 4 against the
    square of the mixed error at radius 4)."""
    pr = opm.Problem([sphere1], EPS, 2.0, qP=(1, 1, 1), nP=1, chiP=0.5, precond="S_INT")
    pr.assemble_A()
    pr.assemble_P()
    pr.assemble_mass()
    ref_op = pr.precond_matrix() @ pr.A
    rng = np.random.default_rng(12)
    x = rng.normal(size=(2, pr.N)) + 1j * rng.normal(size=(2, pr.N))
    ref = x @ ref_op.T
    err = {}
    for prec, hops in ((1, 2), (1, 4), (1, 6), (1, 8), (0, 4)):
        ctx = P.Context(0)
        ctx.add_scatterer(*sphere1, EPS)
        ctx.set_wavenumber(2.0)
        ctx.assemble(P.assembly_opts((4, 3, 2), 4, -1.0, prec),
                     P.assembly_opts((1, 1, 1), 1, 0.5, prec, mass_hops=hops), "S_INT")
        prof = ctx.profile()
        err[(prec, hops)] = rel_fro(ctx.apply(1, x), ref)
        note(f"  precision {prec}, radius {hops}: steps {prof['mass_iterations']}, "
             f"residual {prof['mass_residual']:.2e}, Ptilde A vs oracle {err[(prec, hops)]:.2e}")
        assert prof["mass_iterations"] == hops + 6
        ctx.close()
    assert err[(1, 2)] > err[(1, 4)] > err[(1, 6)] > err[(1, 8)]
    assert err[(1, 6)] < 1e-4 and err[(1, 8)] < 2e-6
    assert err[(0, 4)] < 2.0 * err[(1, 4)] ** 2 + 1e-12


_SYM_MESHES = {"ico1": lambda: synth.icosphere(1), "ico2": lambda: synth.icosphere(2),
               "prism38": lambda: synth.hex_prism(3, 8)}
_sym_oracle = {}


def _oracle_A(name):
    if name not in _sym_oracle:
        pr = opm.Problem([_SYM_MESHES[name]()], EPS, 2.0)
        pr.assemble_A()
        _sym_oracle[name] = pr
    return _sym_oracle[name]


@pytest.mark.parametrize("name,precision,bar_oracle,bar_full", [
    ("ico1", 0, 1e-11, 1e-13), ("ico2", 0, 1e-11, 1e-13), ("prism38", 0, 1e-11, 1e-13),
    ("ico2", 1, 1e-4, 1e-5), ("prism38", 1, 1e-4, 1e-5)])
def test_symmetric_tile_product(P, name, precision, bar_oracle, bar_full):
    """A applied from its upper 128 x 128 tiles plus the singular-pair
    correction (operator_form 2) against the oracle's dense A and against the
    full-row product of the same assembly (operator_form 1).  Meshes: one
    diagonal tile only (120 edges), 4 and 5 tile rows with ragged last tiles
    (480 and 594 edges; the prism's flat faces and sharp edges give the
    largest asymmetry, up to 3e-3 of the largest entry of C).  FP64 bars:
    1e-11 against the oracle, 1e-13 against the full-row product (the
    unsymmetric entries are corrected exactly, the rest differ by rounding);
    mixed: the FP32 block bar 1e-4 against the oracle, 1e-5 against the
    full-row product (X_cr stands in for X_rc, each rounded to FP32)."""
    mesh = _SYM_MESHES[name]()
    pr = _oracle_A(name)
    note(f"symmetric-tile product: {name}, E={pr.N // 2}, precision {precision}")
    cs = make_ctx(P, [mesh], EPS, 2.0, precision=precision, form=2)
    cf = make_ctx(P, [mesh], EPS, 2.0, precision=precision, form=1)
    rng = np.random.default_rng(11)
    for nrhs in (1, 2, 3):  # 3: the full combined matrices, built on demand
        x = rng.normal(size=(nrhs, pr.N)) + 1j * rng.normal(size=(nrhs, pr.N))
        ys, yf = cs.apply(0, x), cf.apply(0, x)
        eo, ef = rel_fro(ys, x @ pr.A.T), rel_fro(ys, yf)
        note(f"  nrhs={nrhs}: vs oracle {eo:.2e}, vs full rows {ef:.2e}")
        assert eo < bar_oracle and ef < bar_full
    if precision == 0 and name != "ico1":
        d, p = synth.plane_wave_set(2, seed=3)
        so = P.solver_opts(tol=1e-11, restart=200, max_iter=600)
        xs, st = cs.solve(d, p, so)
        xf, _ = cf.solve(d, p, so)
        note(f"  solve: iters {st.iterations}, symmetric vs full rows {rel_fro(xs, xf):.2e}")
        assert rel_fro(xs, xf) < 1e-9
