"""Pins for the oracle's collapsed Gauss-Jacobi rules (element and face integrals, eq. 11).

Against closed forms: int_T xi^a eta^b zeta^c = a! b! c! / (a+b+c+3)! on the unit tet and
int s^a t^b = a! b! / (a+b+2)! on the unit triangle.  An n-point-per-direction rule must be
exact up to total degree 2n-1 (so degree 2p for n = p+1) and must fail at degree 2n.
"""
import itertools
from math import factorial

import numpy as np
import pytest

from oracle.quadrature import tet_rule, triangle_rule


def tet_exact(a, b, c):
    return factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)


def tri_exact(a, b):
    return factorial(a) * factorial(b) / factorial(a + b + 2)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_tet_rule_exactness(n):
    x, w = tet_rule(n)
    assert x.shape == (n ** 3, 3)
    assert np.all(x > 0) and np.all(x.sum(1) < 1)
    assert abs(w.sum() - 1.0 / 6.0) < 1e-15
    for a, b, c in itertools.product(range(2 * n), repeat=3):
        if a + b + c > 2 * n - 1:
            continue
        got = np.sum(w * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c)
        assert abs(got - tet_exact(a, b, c)) <= 3e-15 * tet_exact(a, b, c) + 1e-17, (a, b, c)
    # first failure at degree 2n
    got = np.sum(w * x[:, 2] ** (2 * n))
    assert abs(got - tet_exact(0, 0, 2 * n)) > 1e-10 * tet_exact(0, 0, 2 * n)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_triangle_rule_exactness(n):
    x, w = triangle_rule(n)
    assert x.shape == (n ** 2, 2)
    assert np.all(x > 0) and np.all(x.sum(1) < 1)
    assert abs(w.sum() - 0.5) < 1e-15
    for a, b in itertools.product(range(2 * n), repeat=2):
        if a + b > 2 * n - 1:
            continue
        got = np.sum(w * x[:, 0] ** a * x[:, 1] ** b)
        assert abs(got - tri_exact(a, b)) <= 3e-15 * tri_exact(a, b), (a, b)
    got = np.sum(w * x[:, 1] ** (2 * n))
    assert abs(got - tri_exact(0, 2 * n)) > 1e-10 * tri_exact(0, 2 * n)
