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


def roe(Um: torch.Tensor, Up: torch.Tensor, n: torch.Tensor, gamma: float, delta: float = 0.1) -> torch.Tensor:
    """Roe's approximate Riemann flux (the paper's inviscid interface flux, Sec. II.B).

    Fhat = (F(U-).n + F(U+).n)/2 - 1/2 sum_k |lambda_k| alpha_k r_k with Roe averages
    (square-root-density weights) of velocity and total enthalpy, acoustic waves
    u.n -+ c, and the entropy and shear waves at u.n.  Harten's entropy fix on the
    acoustic waves: |lambda| -> (lambda^2 + d^2)/(2 d) when |lambda| < d, d = delta c."""
    rl, rr = Um[..., 0], Up[..., 0]
    ul, ur = Um[..., 1:4] / rl[..., None], Up[..., 1:4] / rr[..., None]
    pl, pr = pressure(Um, gamma), pressure(Up, gamma)
    hl, hr = (Um[..., 4] + pl) / rl, (Up[..., 4] + pr) / rr
    sl, sr = torch.sqrt(rl), torch.sqrt(rr)
    w = sl + sr
    rho = sl * sr
    u = (sl[..., None] * ul + sr[..., None] * ur) / w[..., None]
    h = (sl * hl + sr * hr) / w
    q2 = (u * u).sum(-1)
    c = torch.sqrt((gamma - 1.0) * (h - 0.5 * q2))
    un = (u * n).sum(-1)
    dr = rr - rl
    dp = pr - pl
    du = ur - ul
    dun = (du * n).sum(-1)

    def fix(lam):
        d = delta * c
        a = lam.abs()
        return torch.where(a < d, (lam * lam + d * d) / (2.0 * d), a)

    l1, l2, l4 = fix(un - c), un.abs(), fix(un + c)
    a1 = (dp - rho * c * dun) / (2.0 * c * c)
    a2 = dr - dp / (c * c)
    a4 = (dp + rho * c * dun) / (2.0 * c * c)
    ones = torch.ones_like(rl)
    r1 = torch.cat([ones[..., None], u - c[..., None] * n, (h - un * c)[..., None]], -1)
    r2 = torch.cat([ones[..., None], u, (0.5 * q2)[..., None]], -1)
    r4 = torch.cat([ones[..., None], u + c[..., None] * n, (h + un * c)[..., None]], -1)
    shear_m = du - dun[..., None] * n
    r3 = torch.cat([torch.zeros_like(rl)[..., None], shear_m, ((u * du).sum(-1) - un * dun)[..., None]], -1)
    diss = (l1 * a1)[..., None] * r1 + (l2 * a2)[..., None] * r2 + (l2 * rho)[..., None] * r3 + (l4 * a4)[..., None] * r4
    return 0.5 * (normal_flux(Um, n, gamma) + normal_flux(Up, n, gamma)) - 0.5 * diss


def slipwall_ghost(Um: torch.Tensor, n: torch.Tensor) -> torch.Tensor:
    mn = (Um[..., 1:4] * n).sum(-1, keepdim=True)
    return torch.cat([Um[..., :1], Um[..., 1:4] - 2.0 * mn * n, Um[..., 4:]], dim=-1)
