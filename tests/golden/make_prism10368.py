#!/usr/bin/env python3
"""Writes tests/golden/prism10368_sigma.txt: the oracle's cross sections of the
10368-triangle hexagonal ice prism (diameter 1, length 2.5, 12 divisions per
hexagon side, 60 axially; eps_r = 3.17 + 0.01i, k_e = 8) for the first 4
right-hand sides of the 128-RHS workload (plane waves of seed 3: the first
two directions, two polarisations each; A with q = (4, 3, 2) and 4^4
Sauter-Schwab points).  The values are those of the exact discrete solution
of the FP64 Galerkin system A x = b (Sections 2 and 3.2), which any
preconditioner leaves unchanged.

Calls only oracle/ (and synth/ for the mesh and the waves).  The dense
assembly is spread over processes by ranges of test triangles
(oracle.parallel).  To stay within about 35 GB of memory, A (15.5 GB) is
parked in a temporary file while the right-hand side is formed from the
interior blocks, the operator blocks are then released, and the direct solve
holds A and its factorisation only.

    python tests/golden/make_prism10368.py [--procs N]
"""

import argparse
import os
import platform
import shutil
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import parallel  # noqa: E402
from oracle import pmchwt as opm  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "prism10368_sigma.txt")
EPS, K_E, NRHS = 3.17 + 0.01j, 8.0, 4


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count())
    args = ap.parse_args()
    mesh = synth.hex_prism(12, 60)
    d, p = synth.plane_wave_set(64, seed=3)
    d, p = d[:NRHS], p[:NRHS]
    t0 = time.perf_counter()
    pr = opm.Problem([mesh], EPS, K_E)
    pr.assemble_A(parallel.parallel_assembler(args.procs))
    t_asm = time.perf_counter() - t0
    print(f"assembly {t_asm:.1f} s", flush=True)
    tmp = tempfile.mkdtemp(prefix="prism_golden_")
    try:
        np.save(os.path.join(tmp, "A.npy"), pr.A)
        pr.A = None
        pr.Se = pr.Ce = None
        b = pr.rhs(d, p)
        t_rhs = time.perf_counter() - t0 - t_asm
        print(f"right-hand side {t_rhs:.1f} s", flush=True)
        pr.Si, pr.Ci = [], []
        pr.A = np.load(os.path.join(tmp, "A.npy"))
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    x = pr.solve_direct(b)
    t_solve = time.perf_counter() - t0 - t_asm - t_rhs
    print(f"direct solve {t_solve:.1f} s", flush=True)
    pr.A = None
    se, ss = pr.cross_sections(x, d, p)
    t_all = time.perf_counter() - t0
    with open(OUT, "w") as f:
        f.write("# Oracle (FP64, exact discrete solution) cross sections of the 10368-triangle prism:\n")
        f.write("# hex_prism(12, 60) (diameter 1, length 2.5), eps_r = 3.17+0.01i, k_e = 8, the first 4 waves of\n")
        f.write("# plane_wave_set(64, seed=3); A with q = (4,3,2) and 4^4 Sauter-Schwab points;\n")
        f.write("# written by tests/golden/make_prism10368.py\n")
        f.write(f"# oracle time on {args.procs} processes ({platform.processor() or platform.machine()}): "
                f"assembly {t_asm:.1f} s, right-hand side {t_rhs:.1f} s, direct solve {t_solve:.1f} s, "
                f"total {t_all:.1f} s\n")
        for r in range(NRHS):
            f.write(f"rhs {r} sigma_ext {se[r]:.15e} sigma_sca {ss[r]:.15e}\n")
    print(open(OUT).read())


if __name__ == "__main__":
    main()
