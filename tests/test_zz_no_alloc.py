"""The allocation-free far field (pmchwt_far_field_noalloc) against
pmchwt_far_field on the same context: two calls in a row, the second smaller,
on a two-scatterer problem (scatterer-major currents), FP64 to rounding."""

import numpy as np
import pytest

import synth
from gpu_common import note

pytestmark = pytest.mark.gpu

EPS = 3.17 + 0.01j


def _dirs(n, rng):
    d = rng.standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_far_field_noalloc_matches_far_field():
    import paper_2008_04772_amd as P
    meshes = synth.aggregate(2, 2, 3, seed=7)
    note(f"noalloc far field: aggregate of 2 prisms, {sum(len(m[1]) for m in meshes)} triangles")
    rng = np.random.default_rng(17)
    with P.Context(0) as ctx:
        for v, t in meshes:
            ctx.add_scatterer(v, t, EPS)
        ctx.set_wavenumber(2.0)
        x0 = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        with pytest.raises(P.PmchwtError) as e:
            ctx.far_field_noalloc(x0[None, :1], _dirs(2, rng))
        assert e.value.code == P.ERR_STATE
        ctx.assemble(P.assembly_opts((2, 1, 1), 1), P.assembly_opts((1, 1, 1), 1, chi=0.3), "S_INT")
        _, N = P.pmchwt_sizes(ctx.h)
        for nrhs, nobs in ((3, 700), (1, 40)):
            note(f"noalloc far field: nrhs={nrhs}, nobs={nobs}")
            x = rng.standard_normal((nrhs, N)) + 1j * rng.standard_normal((nrhs, N))
            obs = _dirs(nobs, rng)
            ref = ctx.far_field(x, obs)
            got = ctx.far_field_noalloc(x, obs)
            assert got.shape == ref.shape
            err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
            note(f"  max relative difference {err:.2e}")
            assert err < 1e-12
        # buffers beyond the 64 MiB scratch are refused on the host
        x = rng.standard_normal((200, N)) + 0j
        with pytest.raises(P.PmchwtError) as e:
            ctx.far_field_noalloc(x, _dirs(8192, rng))
        assert e.value.code == P.ERR_INVALID_ARG
        # the context still works after the refusal
        obs = _dirs(16, rng)
        x = rng.standard_normal((1, N)) + 0j
        assert np.allclose(ctx.far_field_noalloc(x, obs), ctx.far_field(x, obs), rtol=1e-12, atol=0)
