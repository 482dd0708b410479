"""Compressible Euler fluxes (torch, any dtype; used in float64).

Conserved variables U = (rho, rho u, rho v, rho w, E) with E = p/(gamma-1) + rho |u|^2 / 2,
the three-dimensional form of the paper's conserved vector, inviscid fluxes and
energy relation (Sec. II.A, eqs. 1-4 with the viscous switch off).

The paper's inviscid interface flux is Roe's; the hot path studied here uses the
local Lax-Friedrichs (Rusanov) flux instead:
    Fhat(U-, U+, n) = (F(U-).n + F(U+).n)/2 - lambda/2 (U+ - U-),
    lambda = max(|u-.n| + c-, |u+.n| + c+), evaluated per quadrature point.
Boundary faces use the same flux with a ghost state (eq. 11 boundary term):
farfield = the free-stream state, slip wall = density and energy kept, normal
momentum mirrored.
"""
from __future__ import annotations

import torch


def prim_to_cons(prim: torch.Tensor, gamma: float) -> torch.Tensor:
    rho = prim[..., 0]
    vel = prim[..., 1:4]
    p = prim[..., 4]
    out = torch.empty_like(prim)
    out[..., 0] = rho
    out[..., 1:4] = rho[..., None] * vel
    out[..., 4] = p / (gamma - 1.0) + 0.5 * rho * (vel * vel).sum(-1)
    return out


def pressure(U: torch.Tensor, gamma: float) -> torch.Tensor:
    rho = U[..., 0]
    m = U[..., 1:4]
    return (gamma - 1.0) * (U[..., 4] - 0.5 * (m * m).sum(-1) / rho)


def flux(U: torch.Tensor, gamma: float) -> torch.Tensor:
    """Physical flux F_d(U) for d = x, y, z: (..., 5) -> (..., 3, 5)."""
    rho = U[..., 0]
    m = U[..., 1:4]
    E = U[..., 4]
    u = m / rho[..., None]
    p = pressure(U, gamma)
    rows = []
    for d in range(3):
        ud = u[..., d]
        mom = m * ud[..., None]
        mom = mom + torch.nn.functional.one_hot(torch.tensor(d), 3).to(U.dtype) * p[..., None]
        rows.append(torch.cat([m[..., d:d + 1], mom, ((E + p) * ud)[..., None]], dim=-1))
    return torch.stack(rows, dim=-2)


def normal_flux(U: torch.Tensor, n: torch.Tensor, gamma: float) -> torch.Tensor:
    return torch.einsum("...dv,...d->...v", flux(U, gamma), n)


def wave_speed(U: torch.Tensor, n: torch.Tensor, gamma: float) -> torch.Tensor:
    """|u.n| + c."""
    rho = U[..., 0]
    un = (U[..., 1:4] * n).sum(-1) / rho
    c = torch.sqrt(gamma * pressure(U, gamma) / rho)
    return un.abs() + c


def rusanov(Um: torch.Tensor, Up: torch.Tensor, n: torch.Tensor, gamma: float) -> torch.Tensor:
    lam = torch.maximum(wave_speed(Um, n, gamma), wave_speed(Up, n, gamma))
    return 0.5 * (normal_flux(Um, n, gamma) + normal_flux(Up, n, gamma)) - 0.5 * lam[..., None] * (Up - Um)


def slipwall_ghost(Um: torch.Tensor, n: torch.Tensor) -> torch.Tensor:
    mn = (Um[..., 1:4] * n).sum(-1, keepdim=True)
    return torch.cat([Um[..., :1], Um[..., 1:4] - 2.0 * mn * n, Um[..., 4:]], dim=-1)
