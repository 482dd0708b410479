"""Orthonormal modal (PKD / Dubiner) basis on the unit tetrahedron.

The paper expands each conserved variable in a modal basis, Q = sum_j c_j(t) b_j(x)
(Sec. II.B, eq. 10), without naming the basis.  Reading used here: the
Proriol-Koornwinder-Dubiner polynomials of total degree <= p,

    psi_ijk = P_i^(0,0)(a) ((1-b)/2)^i P_j^(2i+1,0)(b) ((1-c)/2)^(i+j) P_k^(2i+2j+2,0)(c)

in the collapsed coordinates (a, b, c) of the [-1, 1] tetrahedron (r = 2 xi - 1,
s = 2 eta - 1, t = 2 zeta - 1; a = 2(1+r)/(-s-t) - 1, b = 2(1+s)/(1-t) - 1, c = t),
each scaled so that 6 * integral over the unit tet of phi_m phi_n = delta_mn, which
makes phi_0 = 1 (its coefficient is the cell mean) and the physical mass matrix
|K| I.  Ordering: total degree d = 0..p, then k = 0..d, then j = 0..d-k, i = d-j-k.

The polynomials are expanded exactly with SymPy into monomials xi^a eta^b zeta^c,
so values and gradients are plain monomial sums and integrals over the unit tet
use the closed form a! b! c! / (a+b+c+3)!.
"""
from __future__ import annotations

import functools
import math

import numpy as np
import sympy as sp

XI, ETA, ZETA = sp.symbols("xi eta zeta")

# unit tet vertices; local face f is opposite vertex f
REF_VERTS = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


def n_modes(p: int) -> int:
    return (p + 1) * (p + 2) * (p + 3) // 6


def mode_indices(p: int):
    out = []
    for d in range(p + 1):
        for k in range(d + 1):
            for j in range(d - k + 1):
                out.append((d - j - k, j, k))
    return out


def monomial_integral(a: int, b: int, c: int) -> sp.Rational:
    """Exact integral of xi^a eta^b zeta^c over the unit tetrahedron."""
    return sp.Rational(math.factorial(a) * math.factorial(b) * math.factorial(c),
                       math.factorial(a + b + c + 3))


def _integrate_poly(poly: sp.Poly) -> sp.Expr:
    return sum(coef * monomial_integral(*mon) for mon, coef in poly.terms())


@functools.lru_cache(maxsize=None)
def pkd_polys(p: int):
    """Exact unnormalised PKD polynomials psi_m (sympy Poly, rational coefficients) and
    their squared norms 6 * integral psi_m^2; the basis is phi_m = psi_m / sqrt(norm2_m)."""
    r, s, t = 2 * XI - 1, 2 * ETA - 1, 2 * ZETA - 1
    a = 2 * (1 + r) / (-s - t) - 1
    b = 2 * (1 + s) / (1 - t) - 1
    c = t
    polys = []
    for (i, j, k) in mode_indices(p):
        expr = (sp.jacobi(i, 0, 0, a) * ((-s - t) / 2) ** i
                * sp.jacobi(j, 2 * i + 1, 0, b) * ((1 - t) / 2) ** j
                * sp.jacobi(k, 2 * i + 2 * j + 2, 0, c))
        poly = sp.Poly(sp.expand(sp.cancel(sp.together(expr))), XI, ETA, ZETA)
        norm2 = 6 * _integrate_poly(poly * poly)
        polys.append((poly, norm2))
    return polys


@functools.lru_cache(maxsize=None)
def _monomial_tables(p: int):
    """For each basis function: exponents (M, 3) int and float64 coefficients (M,)."""
    tabs = []
    for poly, norm2 in pkd_polys(p):
        terms = poly.terms()
        scale = 1 / sp.sqrt(norm2)
        exps = np.array([m for m, _ in terms], dtype=np.int64).reshape(-1, 3)
        coefs = np.array([float(sp.N(cf * scale, 40)) for _, cf in terms], dtype=np.float64)
        tabs.append((exps, coefs))
    return tabs


def _powers(x: np.ndarray, deg: int) -> np.ndarray:
    """x (..., ) -> (..., deg+1) with x**0 .. x**deg (0**0 = 1)."""
    out = np.ones(x.shape + (deg + 1,), dtype=np.float64)
    for e in range(1, deg + 1):
        out[..., e] = out[..., e - 1] * x
    return out


def eval_basis(p: int, pts: np.ndarray) -> np.ndarray:
    """Values phi_m(pts): (N, 3) -> (N, Np)."""
    pts = np.asarray(pts, np.float64)
    pw = [_powers(pts[:, d], p) for d in range(3)]
    out = np.zeros((pts.shape[0], n_modes(p)))
    for m, (exps, coefs) in enumerate(_monomial_tables(p)):
        for (a, b, c), cf in zip(exps, coefs):
            out[:, m] += cf * pw[0][:, a] * pw[1][:, b] * pw[2][:, c]
    return out


def eval_basis_grad(p: int, pts: np.ndarray) -> np.ndarray:
    """Reference gradients d phi_m / d xi_d at pts: (N, 3) -> (3, N, Np)."""
    pts = np.asarray(pts, np.float64)
    pw = [_powers(pts[:, d], p) for d in range(3)]
    out = np.zeros((3, pts.shape[0], n_modes(p)))
    for m, (exps, coefs) in enumerate(_monomial_tables(p)):
        for e3, cf in zip(exps, coefs):
            for d in range(3):
                if e3[d] == 0:
                    continue
                de = list(e3)
                de[d] -= 1
                out[d, :, m] += cf * e3[d] * pw[0][:, de[0]] * pw[1][:, de[1]] * pw[2][:, de[2]]
    return out


def face_vertices(f: int):
    """Local vertex indices (ascending) of face f, the face opposite vertex f."""
    return [v for v in range(4) if v != f]


def face_map(f: int, st: np.ndarray) -> np.ndarray:
    """Reference-tet points xi_f(s, t) = V_a + s (V_b - V_a) + t (V_c - V_a) for face f."""
    a, b, c = face_vertices(f)
    st = np.asarray(st, np.float64)
    return (REF_VERTS[a][None, :] + st[:, :1] * (REF_VERTS[b] - REF_VERTS[a])[None, :]
            + st[:, 1:2] * (REF_VERTS[c] - REF_VERTS[a])[None, :])


def exact_mass_matrix(p: int) -> np.ndarray:
    """6 * integral phi_m phi_n over the unit tet, computed exactly (returned as float64)."""
    polys = pkd_polys(p)
    n = len(polys)
    M = np.zeros((n, n))
    for m in range(n):
        for k in range(m, n):
            val = 6 * _integrate_poly(polys[m][0] * polys[k][0]) / sp.sqrt(polys[m][1] * polys[k][1])
            M[m, k] = M[k, m] = float(sp.N(val, 40))
    return M
