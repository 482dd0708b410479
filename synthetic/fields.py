"""Analytic initial/exact fields in primitive variables (rho, u, v, w, p).

Every function takes points x of shape (..., 3) as a torch tensor (any device,
float64) and returns (..., 5) primitive values.  Nothing here knows about the
discretisation; converting to conserved variables and projecting onto a basis
is left to each consumer.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def freestream(x: torch.Tensor, rho=1.0, vel=(0.5, 0.0, 0.0), p=1.0) -> torch.Tensor:
    out = torch.empty(x.shape[:-1] + (5,), dtype=x.dtype, device=x.device)
    out[..., 0] = rho
    out[..., 1] = vel[0]
    out[..., 2] = vel[1]
    out[..., 3] = vel[2]
    out[..., 4] = p
    return out


def sine_wave(x: torch.Tensor, t: float = 0.0, amp: float = 0.2, vel=(1.0, 1.0, 1.0),
              p: float = 1.0) -> torch.Tensor:
    """Density wave rho = 1 + amp sin(2 pi (x + y + z - (u+v+w) t)), constant velocity and pressure."""
    phase = 2.0 * math.pi * (x[..., 0] + x[..., 1] + x[..., 2] - (vel[0] + vel[1] + vel[2]) * t)
    out = freestream(x, 1.0, vel, p)
    out[..., 0] = 1.0 + amp * torch.sin(phase)
    return out


def isentropic_vortex(x: torch.Tensor, t: float = 0.0, length: float = 10.0, beta: float = 5.0,
                      mach: float = 0.5, gamma: float = 1.4) -> torch.Tensor:
    """Shu's isentropic vortex, uniform in z, advected along x by a Mach `mach` mean flow.

    Free stream rho = p = 1, u_inf = mach * sqrt(gamma).  The vortex centre starts at
    (L/2, L/2) and the nearest periodic image (period L in x and y) is used.
    """
    u_inf = mach * math.sqrt(gamma)
    xc = 0.5 * length + u_inf * t
    yc = 0.5 * length
    dx = torch.remainder(x[..., 0] - xc + 0.5 * length, length) - 0.5 * length
    dy = torch.remainder(x[..., 1] - yc + 0.5 * length, length) - 0.5 * length
    r2 = dx * dx + dy * dy
    e = torch.exp(0.5 * (1.0 - r2))
    out = torch.empty(x.shape[:-1] + (5,), dtype=x.dtype, device=x.device)
    temp = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi ** 2) * e * e
    rho = temp ** (1.0 / (gamma - 1.0))
    out[..., 0] = rho
    out[..., 1] = u_inf - beta / (2.0 * math.pi) * e * dy
    out[..., 2] = beta / (2.0 * math.pi) * e * dx
    out[..., 3] = 0.0
    out[..., 4] = rho * temp
    return out


class RandomSmooth:
    """Seeded smooth periodic field on the unit cube.

    Each primitive variable is mean + amp * s(x) with
    s(x) = sum_m a_m sin(2 pi k_m . x + phi_m) / sum_m |a_m|, six modes with integer
    wave vectors k_m in [-2, 2]^3 \\ {0}.  Means/amplitudes: rho 1 +- 0.2,
    velocity components 0 +- 0.28 each, p 1 +- 0.2.
    """

    means = (1.0, 0.0, 0.0, 0.0, 1.0)
    amps = (0.2, 0.28, 0.28, 0.28, 0.2)

    def __init__(self, seed: int = 42, n_modes: int = 6, length: float = 1.0):
        rng = np.random.default_rng(seed)
        self.length = length
        self.k, self.a, self.phi = [], [], []
        for _ in range(5):
            ks = []
            while len(ks) < n_modes:
                k = rng.integers(-2, 3, size=3)
                if np.any(k != 0):
                    ks.append(k)
            self.k.append(np.array(ks, dtype=np.float64))
            self.a.append(rng.uniform(0.0, 1.0, size=n_modes))
            self.phi.append(rng.uniform(0.0, 2.0 * math.pi, size=n_modes))

    def __call__(self, x: torch.Tensor) -> torch.Tensor:
        out = torch.empty(x.shape[:-1] + (5,), dtype=x.dtype, device=x.device)
        for v in range(5):
            k = torch.as_tensor(self.k[v], dtype=x.dtype, device=x.device) * (2.0 * math.pi / self.length)
            a = torch.as_tensor(self.a[v], dtype=x.dtype, device=x.device)
            phi = torch.as_tensor(self.phi[v], dtype=x.dtype, device=x.device)
            s = torch.sin(x @ k.T + phi) @ a / a.abs().sum()
            out[..., v] = self.means[v] + self.amps[v] * s
        return out


def random_coefficients(n_elem: int, n_modes: int, seed: int = 7, scale: float = 0.005) -> np.ndarray:
    """Seeded modal coefficients in user layout [E][5][n_modes] (conserved variables).

    Mode 0 (the cell mean) is drawn in a range with positive density and pressure for
    gamma = 1.4 (rho in [0.9, 1.1], momentum in [-0.3, 0.3]^3, total energy in
    [2.4, 2.8]); higher modes are N(0, scale^2).
    """
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((n_elem, 5, n_modes)) * scale
    c[:, 0, 0] = rng.uniform(0.9, 1.1, n_elem)
    c[:, 1:4, 0] = rng.uniform(-0.3, 0.3, (n_elem, 3))
    c[:, 4, 0] = rng.uniform(2.4, 2.8, n_elem)
    return c


def gaussian(shape, seed: int) -> np.ndarray:
    """Seeded standard normal array (cotangents, directions)."""
    return np.random.default_rng(seed).standard_normal(shape)
