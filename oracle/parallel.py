"""Process-parallel drivers of the oracle's dense assembly (test
infrastructure: only tests/, the smoke check and the benchmark's CPU
baseline use the oracle).

The quadrature sums are those of oracle.operators; the test triangles are
split into ranges, each process assembles the rows its range contributes
(operators.assemble_rwg_tests) and the parent adds them up.  Only the order
of the additions differs from operators.assemble_rwg.
"""

import multiprocessing as mp

import numpy as np

from . import operators as ops

_JOB = {}


def _part(args):
    t0, t1 = args
    from threadpoolctl import threadpool_limits
    topo, k, q, n = _JOB["topo"], _JOB["k"], _JOB["q"], _JOB["n"]
    with threadpool_limits(1):
        d = ops.assemble_rwg_tests(topo, k, t0, t1, q, n)
    rows = np.unique(topo.t2e[t0:t1])
    return rows, d["S"][rows], d["C"][rows]


def parallel_assembler(procs):
    """A drop-in for operators.assemble_rwg (arguments topo, k, q, n_sing)
    spread over `procs` forked processes."""
    def assemble(topo, k, q, n):
        _JOB.update(topo=topo, k=k, q=q, n=n)
        step = max(1, topo.F // (4 * procs))
        ranges = [(t, min(topo.F, t + step)) for t in range(0, topo.F, step)]
        S = np.zeros((topo.E, topo.E), dtype=np.complex128)
        C = np.zeros((topo.E, topo.E), dtype=np.complex128)
        with mp.get_context("fork").Pool(procs) as pool:
            for rows, s, c in pool.imap_unordered(_part, ranges):
                S[rows] += s
                C[rows] += c
        return {"S": S, "C": C}
    return assemble
