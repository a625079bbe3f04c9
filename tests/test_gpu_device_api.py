"""Device-pointer entry points (pmchwt_apply_device, pmchwt_solve_device,
pmchwt_far_field_device) on device memory and a caller stream of the
library's own HIP runtime (reached here through ctypes: hipMalloc,
hipMemcpyAsync, hipStreamCreate).

They run the same kernels in the same order as the host forms; only the
layout change between the API's scatterer-major vectors and the internal
union layout moves to the device.  So their outputs must equal the host
forms' bit for bit, on one scatterer and on three (where the layout change
is a real permutation), below and above the matrix-core thresholds (16
right-hand sides for the products, 8 for the far field)."""

import ctypes

import numpy as np
import pytest

import synth
from gpu_common import note, make_ctx

pytestmark = pytest.mark.gpu

EPS = 3.17 + 0.01j
H2D, D2H = 1, 2  # hipMemcpyHostToDevice, hipMemcpyDeviceToHost


@pytest.fixture(scope="module")
def P():
    import paper_2008_04772_amd as lib
    return lib


@pytest.fixture(scope="module")
def hip(P):
    lib = ctypes.CDLL("libamdhip64.so.7")  # the runtime the library already loaded
    lib.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    lib.hipFree.argtypes = [ctypes.c_void_p]
    lib.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    lib.hipStreamCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    lib.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
    lib.hipStreamDestroy.argtypes = [ctypes.c_void_p]
    return lib


class Dev:
    """A device buffer and the copies to and from it on one stream."""

    def __init__(self, hip, nbytes, stream):
        self.hip, self.n, self.s = hip, nbytes, stream
        self.p = ctypes.c_void_p()
        assert hip.hipMalloc(ctypes.byref(self.p), nbytes) == 0

    def put(self, a):
        a = np.ascontiguousarray(a)
        assert a.nbytes == self.n
        assert self.hip.hipMemcpyAsync(self.p, a.ctypes.data, self.n, H2D, self.s) == 0
        assert self.hip.hipStreamSynchronize(self.s) == 0  # the host array may go away

    def get(self, dtype, shape):
        out = np.empty(shape, dtype=dtype)
        assert out.nbytes == self.n
        assert self.hip.hipMemcpyAsync(out.ctypes.data, self.p, self.n, D2H, self.s) == 0
        assert self.hip.hipStreamSynchronize(self.s) == 0
        return out

    def free(self):
        self.hip.hipFree(self.p)


def _stream(hip):
    s = ctypes.c_void_p()
    assert hip.hipStreamCreate(ctypes.byref(s)) == 0
    return s


CASES = [("sphere320", lambda: [synth.icosphere(2)], EPS, 2.0),
         ("three cubes", lambda: synth.three_cubes(2.1), 1.311 ** 2 + 0j, 2.1)]


@pytest.mark.parametrize("name,build,eps,k", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("nrhs", [3, 20])
def test_apply_device_equals_host(P, hip, name, build, eps, k, nrhs):
    ctx = make_ctx(P, build(), eps, k, qP=(1, 1, 1), nP=1, chi=0.5, precond="S_INT", precision=P.MIXED,
                   precisionP=P.MIXED)
    _, N = ctx.sizes()
    rng = np.random.default_rng(21)
    x = rng.normal(size=(nrhs, N)) + 1j * rng.normal(size=(nrhs, N))
    s = _stream(hip)
    xd, yd = Dev(hip, x.nbytes, s), Dev(hip, x.nbytes, s)
    xd.put(x)
    for which in (0, 1):
        ctx.apply_device(which, xd.p.value, nrhs, yd.p.value, stream=s.value)
        yh = yd.get(np.complex128, x.shape)  # read back on the caller's stream
        ref = ctx.apply(which, x)
        note(f"  {name}, nrhs={nrhs}, which={which}: max |device - host| {np.max(np.abs(yh - ref)):.1e}")
        assert np.array_equal(yh, ref)
    xd.free()
    yd.free()
    hip.hipStreamDestroy(s)
    ctx.close()


@pytest.mark.parametrize("name,build,eps,k", CASES, ids=[c[0] for c in CASES])
def test_solve_and_far_field_device_equal_host(P, hip, name, build, eps, k):
    ctx = make_ctx(P, build(), eps, k, qP=(1, 1, 1), nP=1, chi=0.5, precond="S_INT", precision=P.MIXED,
                   precisionP=P.MIXED)
    _, N = ctx.sizes()
    dirs, pols = synth.plane_wave_set(5, seed=2)  # 10 right-hand sides
    nrhs = len(dirs)
    so = P.solver_opts(tol=1e-8, restart=100, max_iter=1000, ir_max=2)
    xh, sth = ctx.solve(dirs, pols, so)
    s = _stream(hip)
    cur = Dev(hip, 16 * nrhs * N, s)
    std = ctx.solve_device(dirs, pols, so, cur.p.value, stream=s.value)
    xd = cur.get(np.complex128, (nrhs, N))
    note(f"  {name}: solve {std.iterations} / {sth.iterations} iterations, max |device - host| "
         f"{np.max(np.abs(xd - xh)):.1e}")
    assert std.iterations == sth.iterations and np.array_equal(xd, xh)
    rng = np.random.default_rng(3)
    obs = rng.normal(size=(77, 3))
    obs /= np.linalg.norm(obs, axis=1, keepdims=True)
    od = Dev(hip, obs.nbytes, s)
    od.put(obs)
    for nr in (3, 10):  # VALU sum; matrix cores
        Fd = Dev(hip, 16 * 3 * nr * len(obs), s)
        ctx.far_field_device(cur.p.value, nr, od.p.value, len(obs), Fd.p.value, stream=s.value)
        Fh = Fd.get(np.complex128, (nr, len(obs), 3))
        ref = ctx.far_field(xh[:nr], obs)
        note(f"  {name}: far field nrhs={nr}: max |device - host| {np.max(np.abs(Fh - ref)):.1e}")
        assert np.array_equal(Fh, ref)
        Fd.free()
    cur.free()
    od.free()
    hip.hipStreamDestroy(s)
    ctx.close()
