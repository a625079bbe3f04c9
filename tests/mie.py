"""Mie series for a homogeneous dielectric sphere (Bohren & Huffman, ch. 4).

Test infrastructure: an exact solution of the continuous scattering problem
that the PMCHWT discretisation must approach under mesh refinement.
"""

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def mie_coefficients(x, m, nmax=None):
    if nmax is None:
        nmax = int(np.ceil(x + 4 * x ** (1 / 3) + 2)) + 5
    n = np.arange(1, nmax + 1)
    mx = m * x
    jx, djx = spherical_jn(n, x), spherical_jn(n, x, derivative=True)
    yx, dyx = spherical_yn(n, x), spherical_yn(n, x, derivative=True)
    jmx, djmx = spherical_jn(n, mx), spherical_jn(n, mx, derivative=True)
    psi_x, dpsi_x = x * jx, jx + x * djx
    xi_x, dxi_x = x * (jx + 1j * yx), (jx + 1j * yx) + x * (djx + 1j * dyx)
    psi_mx, dpsi_mx = mx * jmx, jmx + mx * djmx
    a = (m * psi_mx * dpsi_x - psi_x * dpsi_mx) / (m * psi_mx * dxi_x - xi_x * dpsi_mx)
    b = (psi_mx * dpsi_x - m * psi_x * dpsi_mx) / (psi_mx * dxi_x - m * xi_x * dpsi_mx)
    return n, a, b


def mie_efficiencies(x, m):
    """(Q_ext, Q_sca) for size parameter x = k a and relative index m."""
    n, a, b = mie_coefficients(x, m)
    qext = 2.0 / x ** 2 * np.sum((2 * n + 1) * np.real(a + b))
    qsca = 2.0 / x ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return float(qext), float(qsca)
