"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package builds meshes (icospheres, hexagonal ice prisms, prism aggregates,
the three-cube array) and incident plane-wave sets.  It holds none of the
method's arithmetic: no basis functions, no quadrature, no kernels.  Both the
oracle and the GPU library receive its output as plain vertex/triangle arrays.
"""

from .meshes import (icosphere, hex_prism, aggregate, three_cubes, cube,
                     union_mesh, mean_edge_length)
from .waves import plane_wave_set, single_wave

__all__ = ["icosphere", "hex_prism", "aggregate", "three_cubes", "cube",
           "union_mesh", "mean_edge_length", "plane_wave_set", "single_wave"]
