"""Shared helpers of the GPU tests: library context set-up and relative errors."""

import sys

import numpy as np


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_fro(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def make_ctx(P, meshes, eps, k, qA=(4, 3, 2), nA=4, qP=(4, 3, 2), nP=4, chi=-1.0, precond="S_INT", precision=0,
             precisionP=0, form=0):
    ctx = P.Context(0)
    for (v, t) in meshes:
        ctx.add_scatterer(v, t, eps)
    ctx.set_wavenumber(k)
    ctx.assemble(P.assembly_opts(qA, nA, -1.0, precision, operator_form=form),
                 P.assembly_opts(qP, nP, chi, precisionP), precond)
    return ctx
