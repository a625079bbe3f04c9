#!/usr/bin/env python3
"""Writes tests/golden/sphere5120_sigma.txt: the oracle's cross sections of the
5120-triangle dielectric sphere (radius 1, eps_r = 3.17 + 0.01i, k_e = 5,
plane wave along +z polarised along x; A with q = (4, 3, 2) and 4^4
Sauter-Schwab points).  The values are those of the exact discrete solution
of the FP64 Galerkin system A x = b (Sections 2 and 3.2), which any
preconditioner leaves unchanged.

Calls only oracle/ (and synth/ for the mesh and the wave).  The dense
assembly is spread over processes by ranges of test triangles
(oracle.parallel); the direct solve uses all cores.

    python tests/golden/make_sphere5120.py [--procs N]
"""

import argparse
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import parallel  # noqa: E402
from oracle import pmchwt as opm  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere5120_sigma.txt")
EPS, K_E = 3.17 + 0.01j, 5.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count())
    args = ap.parse_args()
    mesh = synth.icosphere(4)
    d, p = synth.single_wave()
    t0 = time.perf_counter()
    pr = opm.Problem([mesh], EPS, K_E)
    pr.assemble_A(parallel.parallel_assembler(args.procs))
    t_asm = time.perf_counter() - t0
    b = pr.rhs(d, p)
    t_rhs = time.perf_counter() - t0 - t_asm
    x = pr.solve_direct(b)
    t_solve = time.perf_counter() - t0 - t_asm - t_rhs
    se, ss = pr.cross_sections(x, d, p)
    t_all = time.perf_counter() - t0
    with open(OUT, "w") as f:
        f.write("# Oracle (FP64, exact discrete solution) cross sections of the 5120-triangle sphere:\n")
        f.write("# icosphere level 4, radius 1, eps_r = 3.17+0.01i, k_e = 5, d = +z, p = x;\n")
        f.write("# A with q = (4,3,2) and 4^4 Sauter-Schwab points; written by tests/golden/make_sphere5120.py\n")
        f.write(f"# oracle time on {args.procs} processes ({platform.processor() or platform.machine()}): "
                f"assembly {t_asm:.1f} s, right-hand side {t_rhs:.1f} s, direct solve {t_solve:.1f} s, "
                f"total {t_all:.1f} s\n")
        f.write(f"sigma_ext {se[0]:.15e}\n")
        f.write(f"sigma_sca {ss[0]:.15e}\n")
    print(open(OUT).read())


if __name__ == "__main__":
    main()
