"""Pins of the oracle's viscous (BR1) terms, against what the method and the mathematics fix:
the lifted gradient of a uniform state vanishes and that of a continuous polynomial of
degree <= p is its exact gradient away from boundary jumps; the viscous flux of a simple
shear with a temperature gradient has a closed form; the central interface flux conserves;
a small-amplitude shear wave decays at the rate mu k^2 of the viscous momentum equation."""
import math

import numpy as np
import pytest
import torch

from oracle import euler
from oracle.dg import DG
from oracle.viscous import viscous_flux
from synthetic import fields, kuhn_cube


def test_uniform_state_has_zero_gradient_and_viscous_residual():
    m = kuhn_cube(3, jitter=0.2)
    dg = DG(3, m.elem_vid, m.elem_xyz, mu=0.05)
    U = dg.project(lambda x: fields.freestream(x, 1.1, (0.3, -0.2, 0.1), 0.9))
    assert dg.gradient(U).abs().max() < 1e-12
    assert dg.viscous_term(U, dg.gradient(U)).abs().max() < 1e-12


@pytest.mark.parametrize("p", [1, 2])
def test_lifting_exact_for_continuous_polynomials(p):
    """BR1's lifted gradient equals grad U for a continuous U of degree <= p: interior faces
    have no jump.  Elements away from the boundary (whose ghost is the free stream) must
    reproduce the exact gradient of a linear (p = 1) or quadratic (p = 2) field."""
    m = kuhn_cube(4, periodic=(False, False, False), jitter=0.15)
    dg = DG(p, m.elem_vid, m.elem_xyz, m.bface_vid, m.bface_tag)
    a = torch.tensor([0.3, -0.2, 0.5], dtype=torch.float64)

    def prim(x):
        s = (x * a).sum(-1) + (0.4 * x[..., 0] * x[..., 1] if p == 2 else 0.0)
        out = torch.empty(x.shape[:-1] + (5,), dtype=torch.float64)
        out[..., 0] = 1.0 + 0.1 * s
        out[..., 1] = 0.2 * s
        out[..., 2] = -0.1 * s
        out[..., 3] = 0.05
        out[..., 4] = 1.0 + 0.3 * s
        return out

    # the projected primitive field is not polynomial in the conserved variables: project
    # the conserved variables as the polynomial instead
    x = torch.from_numpy(dg.volume_points())
    Uq = prim(x)
    U = 6.0 * torch.einsum("q,qi,eqv->evi", dg.w, dg.B, Uq)
    Z = dg.gradient(U)
    # exact gradient at the volume points, projected: d/dx_k of each variable
    xq = x.clone().requires_grad_(True)
    grads = []
    for v in range(5):
        (g,) = torch.autograd.grad(prim(xq)[..., v].sum(), xq)
        grads.append(g)
    G = torch.stack(grads, -1)                                             # (E, q, k, v)
    Zex = 6.0 * torch.einsum("q,qi,eqkv->ekvi", dg.w, dg.B, G.detach())
    touch = np.zeros(dg.n_elem, bool)
    touch[dg.faces.em[dg.faces.ep < 0]] = True
    inner = torch.from_numpy(~touch)
    assert inner.sum() > 20
    err = (Z[inner] - Zex[inner]).abs().max().item()
    assert err < 1e-11, err


def test_viscous_flux_closed_form():
    """u = (a y, 0, 0), rho = 1, p = 1 + b x: tau_xy = mu a, div u = 0, T = p, q = -kappa (b, 0, 0)."""
    mu, pr, gamma, a, b = 0.03, 0.72, 1.4, 0.7, 0.2
    y, x = 0.4, 0.3
    rho, u, p = 1.0, np.array([a * y, 0.0, 0.0]), 1.0 + b * x
    U = torch.tensor([rho, rho * u[0], 0.0, 0.0, p / (gamma - 1) + 0.5 * rho * u @ u], dtype=torch.float64)
    # gradients of the conserved variables: d(rho u)/dy = a, dE/dx = b/(gamma-1), dE/dy = rho u_x a
    Z = torch.zeros((3, 5), dtype=torch.float64)
    Z[1, 1] = a
    Z[0, 4] = b / (gamma - 1)
    Z[1, 4] = rho * u[0] * a
    F = viscous_flux(U, Z, gamma, mu, pr)
    kappa = mu * gamma / ((gamma - 1) * pr)
    ref = np.zeros((3, 5))
    ref[0] = [0, 0, mu * a, 0, kappa * b]          # x-direction: tau_yx = mu a; u.tau_x = 0; -q_x = kappa b
    ref[1] = [0, mu * a, 0, 0, u[0] * mu * a]      # y-direction: tau_xy = mu a; u_x tau_xy
    assert np.allclose(F.numpy(), ref, rtol=1e-14, atol=1e-15)


def test_viscous_conservation():
    m = kuhn_cube(3, jitter=0.2)
    dg = DG(2, m.elem_vid, m.elem_xyz, mu=0.05)
    U = dg.project(fields.RandomSmooth(5))
    Rv = dg.viscous_term(U, dg.gradient(U))
    total = Rv[:, :, 0].sum(0)
    scale = Rv[:, :, 0].abs().sum(0)
    assert (total.abs() <= 1e-13 * scale + 1e-15).all(), (total, scale)


def test_shear_wave_decay_rate():
    """v = eps sin(2 pi x), rho = p = 1 at rest otherwise: the viscous part of the residual's
    y-momentum is mu d2v/dx2 = -mu (2 pi)^2 eps sin(2 pi x) up to the discretisation error,
    which must fall at least like h^2 (BR1 at P3: the lifted gradient is O(h^p))."""
    mu, eps = 0.05, 1e-3

    def prim(x):
        out = torch.zeros(x.shape[:-1] + (5,), dtype=torch.float64)
        out[..., 0] = 1.0
        out[..., 2] = eps * torch.sin(2 * math.pi * x[..., 0])
        out[..., 4] = 1.0
        return out

    errs = []
    for n in (3, 6):
        m = kuhn_cube(n)
        dg = DG(3, m.elem_vid, m.elem_xyz, mu=mu)
        U = dg.project(prim)
        Rv = -dg.viscous_term(U, dg.gradient(U)) / dg.volume[:, None, None]
        x = torch.from_numpy(dg.volume_points())
        exact = -mu * (2 * math.pi) ** 2 * eps * torch.sin(2 * math.pi * x[..., 0])
        Rq = dg.evaluate(Rv)[..., 2]
        wq = dg.absdet[:, None] * dg.w[None, :]
        errs.append(float(((Rq - exact) ** 2 * wq).sum().sqrt() / ((exact ** 2) * wq).sum().sqrt()))
    assert errs[1] < 0.03 and errs[0] / errs[1] > 4.0, errs


def test_sampled_residual_rows_match_the_full_residual():
    """The sampled viscous residual (Z evaluated only on the sample and its face neighbours)
    reproduces the rows of the full evaluation, on a jittered mesh with boundary faces."""
    far = (1.0, 0.5, 0.1, 0.0, 1.0)
    m = kuhn_cube(3, jitter=0.2, periodic=(False, True, True))
    dg = DG(2, m.elem_vid, m.elem_xyz, m.bface_vid, m.bface_tag, farfield_prim=far, mu=0.03)
    U = dg.project(fields.RandomSmooth(9))
    full = dg.residual(U)
    sample = torch.tensor([0, 5, 17, 40, 77, m.n_elem - 1])
    part = dg.residual(U, sample)
    assert (part - full[sample]).abs().max() <= 1e-13 * full.abs().max()
    Z = dg.gradient(U)
    Zs = dg.gradient(U, sample)
    assert (Zs[sample] - Z[sample]).abs().max() <= 1e-13 * Z.abs().max()
    nb = dg.with_neighbours(sample)
    assert set(sample.tolist()) <= set(nb.tolist()) and nb.shape[0] > sample.shape[0]
