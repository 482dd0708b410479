"""Pins for the oracle's orthonormal PKD basis (the modal expansion of eq. 10).

* exact orthonormality (6 int phi_m phi_n = delta_mn by exact monomial integration);
* the same through the tet rule (exact for degree 2p);
* agreement with an independent evaluation: SciPy Jacobi polynomials in collapsed
  coordinates with the closed-form norm 6 int psi^2 = 6 / ((2i+1)(2i+2j+2)(2i+2j+2k+3));
* gradients against central differences;
* the discrete integration-by-parts identity, which ties volume gradients, face maps,
  face weights and reference normals together.
"""
import numpy as np
import pytest
from scipy.special import eval_jacobi

from oracle import basis
from oracle.quadrature import tet_rule, triangle_rule

REF_AREA_NORMALS = np.array([[0.5, 0.5, 0.5], [-0.5, 0.0, 0.0], [0.0, -0.5, 0.0], [0.0, 0.0, -0.5]])


def random_interior_points(m, seed=0):
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < m:
        x = rng.uniform(0.02, 0.96, 3)
        if x.sum() < 0.97:
            pts.append(x)
    return np.array(pts)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_exact_orthonormality(p):
    M = basis.exact_mass_matrix(p)
    assert np.abs(M - np.eye(basis.n_modes(p))).max() < 1e-15


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_quadrature_mass_matrix(p):
    x, w = tet_rule(p + 1)
    B = basis.eval_basis(p, x)
    M = 6.0 * B.T @ (w[:, None] * B)
    assert np.abs(M - np.eye(basis.n_modes(p))).max() < 2e-13
    assert np.allclose(B[:, 0], 1.0, atol=1e-15, rtol=0)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_matches_collapsed_jacobi_form(p):
    pts = random_interior_points(40, seed=p)
    r, s, t = (2 * pts - 1).T
    a = 2 * (1 + r) / (-s - t) - 1
    b = 2 * (1 + s) / (1 - t) - 1
    c = t
    ref = []
    for (i, j, k) in basis.mode_indices(p):
        psi = (eval_jacobi(i, 0, 0, a) * ((1 - b) / 2) ** i * eval_jacobi(j, 2 * i + 1, 0, b)
               * ((1 - c) / 2) ** (i + j) * eval_jacobi(k, 2 * i + 2 * j + 2, 0, c))
        ref.append(psi * np.sqrt((2 * i + 1) * (2 * i + 2 * j + 2) * (2 * i + 2 * j + 2 * k + 3) / 6.0))
    ref = np.stack(ref, 1)
    got = basis.eval_basis(p, pts)
    assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gradient_central_difference(p):
    pts = random_interior_points(20, seed=10 + p)
    G = basis.eval_basis_grad(p, pts)
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (basis.eval_basis(p, pts + e) - basis.eval_basis(p, pts - e)) / (2 * h)
        assert np.abs(G[d] - fd).max() < 1e-7 * max(1.0, np.abs(G[d]).max())


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_integration_by_parts(p):
    n = p + 1
    x, w = tet_rule(n)
    st, wt = triangle_rule(n)
    B = basis.eval_basis(p, x)
    G = basis.eval_basis_grad(p, x)
    for d in range(3):
        lhs = G[d].T @ (w[:, None] * B) + B.T @ (w[:, None] * G[d])
        rhs = np.zeros_like(lhs)
        for f in range(4):
            Bf = basis.eval_basis(p, basis.face_map(f, st))
            rhs += REF_AREA_NORMALS[f, d] * 2.0 * Bf.T @ (wt[:, None] * Bf)
        assert np.abs(lhs - rhs).max() < 1e-12 * max(1.0, np.abs(lhs).max())


def test_face_map_corners():
    for f in range(4):
        a, b, c = basis.face_vertices(f)
        got = basis.face_map(f, np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]))
        assert np.allclose(got, basis.REF_VERTS[[a, b, c]])
