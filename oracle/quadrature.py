"""Collapsed Gauss-Jacobi quadrature on the reference triangle and tetrahedron.

The paper evaluates every element and face integral of eq. (11) by Gaussian
quadrature without naming the rule (Sec. II.B).  Reading used here: the
Duffy/collapsed-coordinate product rule with n points per direction, built from
Gauss-Legendre in the first direction and Gauss-Jacobi with weights (1-b)^1 and
(1-c)^2 in the collapsed directions.  It integrates total degree 2n-1 exactly.

Point order: the first collapsed coordinate varies fastest, then the second,
then the third.  SciPy's roots_jacobi is the 1-D building block.
"""
from __future__ import annotations

import numpy as np
from scipy.special import roots_jacobi


def gauss_jacobi(n: int, alpha: float, beta: float):
    """n-point Gauss-Jacobi rule on [-1, 1] for weight (1-x)^alpha (1+x)^beta."""
    x, w = roots_jacobi(n, alpha, beta)
    return np.asarray(x, np.float64), np.asarray(w, np.float64)


def triangle_rule(n: int):
    """Points (N, 2) = (s, t) and weights on {s, t >= 0, s + t <= 1}; weights sum to 1/2."""
    a, wa = gauss_jacobi(n, 0.0, 0.0)
    b, wb = gauss_jacobi(n, 1.0, 0.0)
    pts, wts = [], []
    for jb in range(n):
        for ia in range(n):
            s = (1.0 + a[ia]) * (1.0 - b[jb]) / 4.0
            t = (1.0 + b[jb]) / 2.0
            pts.append((s, t))
            wts.append(wa[ia] * wb[jb] / 8.0)
    return np.array(pts), np.array(wts)


def tet_rule(n: int):
    """Points (N, 3) = (xi, eta, zeta) and weights on the unit tet; weights sum to 1/6."""
    a, wa = gauss_jacobi(n, 0.0, 0.0)
    b, wb = gauss_jacobi(n, 1.0, 0.0)
    c, wc = gauss_jacobi(n, 2.0, 0.0)
    pts, wts = [], []
    for kc in range(n):
        for jb in range(n):
            for ia in range(n):
                xi = (1.0 + a[ia]) * (1.0 - b[jb]) * (1.0 - c[kc]) / 8.0
                eta = (1.0 + b[jb]) * (1.0 - c[kc]) / 4.0
                zeta = (1.0 + c[kc]) / 2.0
                pts.append((xi, eta, zeta))
                wts.append(wa[ia] * wb[jb] * wc[kc] / 64.0)
    return np.array(pts), np.array(wts)
