"""Seeded incident plane-wave sets (direction d, polarisation p, with p orthogonal to d)."""

import numpy as np


def single_wave(direction=(0.0, 0.0, 1.0), polarisation=(1.0, 0.0, 0.0)):
    d = np.asarray(direction, dtype=np.float64)[None, :]
    p = np.asarray(polarisation, dtype=np.complex128)[None, :]
    return d, p


def plane_wave_set(n_dirs, seed=3):
    """``n_dirs`` seeded directions uniform on the sphere, two polarisations each.

    Directions are normalised standard-normal draws from numpy's PCG64 with
    ``seed``.  p1 = normalise(d x z) (x if d is parallel to z), p2 = d x p1.
    Returns (dirs (2n, 3) float64, pols (2n, 3) complex128).
    """
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n_dirs, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    dirs, pols = [], []
    for di in d:
        p1 = np.cross(di, [0.0, 0.0, 1.0])
        if np.linalg.norm(p1) < 1e-12:
            p1 = np.array([1.0, 0.0, 0.0])
        p1 /= np.linalg.norm(p1)
        p2 = np.cross(di, p1)
        dirs += [di, di]
        pols += [p1, p2]
    return np.array(dirs), np.array(pols, dtype=np.complex128)
