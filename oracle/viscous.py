"""Viscous (Navier-Stokes) flux of the paper's eq. 1 in 3-D, as a function of the
conserved state U and the auxiliary variable Z = grad U (Sec. II.B: the equation is
rewritten with Z, and the viscous interface flux is taken in BR1 form).

Test infrastructure only (the oracle of the GPU path); plain float64 torch.

With rho, u = m / rho, p = (gamma - 1)(E - rho |u|^2 / 2) and T = p / rho (gas constant 1):
    d_k u_i = (d_k m_i - u_i d_k rho) / rho
    d_k p   = (gamma - 1)(d_k E - |u|^2 / 2 d_k rho - rho u . d_k u)
    d_k T   = (d_k p - T d_k rho) / rho
    tau_ij  = mu (d_j u_i + d_i u_j - 2/3 delta_ij div u)        (Stokes' hypothesis)
    q_j     = -kappa d_j T,  kappa = mu gamma / ((gamma - 1) Pr)  (c_p / Pr with R = 1)
    F_v,j   = (0, tau_1j, tau_2j, tau_3j, u_i tau_ij - q_j)
The paper's 2-D stress tensor and energy row are the restriction of these to (x, y);
the paper leaves the heat-flux law and the viscosity constant unstated (reading:
Fourier's law with a constant Prandtl number, constant mu).
"""
from __future__ import annotations

import torch

from . import euler


def viscous_flux(U: torch.Tensor, Z: torch.Tensor, gamma: float, mu: float, prandtl: float) -> torch.Tensor:
    """F_v for states U (..., 5) and gradients Z (..., 3, 5) [Z[..., k, w] = d_k U_w]:
    returns (..., 3, 5) with [..., j, :] the viscous flux in direction j."""
    rho = U[..., 0]
    u = U[..., 1:4] / rho[..., None]                                  # (..., 3)
    p = euler.pressure(U, gamma)
    T = p / rho
    grho = Z[..., :, 0]                                                # (..., 3) over k
    gu = (Z[..., :, 1:4] - u[..., None, :] * grho[..., :, None]) / rho[..., None, None]   # [k, i] = d_k u_i
    gp = (gamma - 1.0) * (Z[..., :, 4] - 0.5 * (u * u).sum(-1)[..., None] * grho
                          - rho[..., None] * (gu * u[..., None, :]).sum(-1))
    gT = (gp - T[..., None] * grho) / rho[..., None]
    div = gu[..., 0, 0] + gu[..., 1, 1] + gu[..., 2, 2]
    eye = torch.eye(3, dtype=U.dtype)
    # tau[i, j] = mu (d_j u_i + d_i u_j) - 2/3 mu div delta_ij ; gu[j, i] = d_j u_i
    tau = mu * (gu.transpose(-1, -2) + gu) - (2.0 / 3.0) * mu * div[..., None, None] * eye
    kappa = mu * gamma / ((gamma - 1.0) * prandtl)
    energy = (u[..., :, None] * tau).sum(-2) + kappa * gT             # (..., 3) over j
    zero = torch.zeros_like(rho)[..., None].expand(energy.shape)
    return torch.stack([zero, tau[..., 0, :], tau[..., 1, :], tau[..., 2, :], energy], dim=-1)
