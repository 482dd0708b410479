"""Full configuration: slip wall with a Gaussian bump, farfield sides, periodic in z, Mach 0.5
free stream.  The integrated wall pressure and its gradient against the oracle, the
checkpointed trajectory adjoint of the objective against the oracle, and at the full size
(56^3 x 6 jittered tets, P3) 50 SSP-RK3 steps with the adjoint checked by finite differences."""
import math

import numpy as np
import pytest
import torch

from oracle.adjoint import trajectory_vjp as oracle_traj
from synthetic import fields, kuhn_cube

pytestmark = pytest.mark.gpu

from gpu_common import assert_parity, make_mesh, oracle, random_state, solver, zero_padding  # noqa: E402

FAR = (1.0, 0.5 * math.sqrt(1.4), 0.0, 0.0, 1.0)


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_wall_pressure_and_gradient(p, prec):
    mesh = make_mesh("bump")
    dg = oracle(p, mesh, FAR)
    U = random_state(dg, seed=4)
    Ur = U.clone().requires_grad_(True)
    J_ref = dg.wall_pressure(Ur)
    (g_ref,) = torch.autograd.grad(J_ref, Ur)
    s = solver(p, prec, mesh, farfield=FAR)
    J, g = s.wall_pressure(s.set_state(U.cuda()), grad=True)
    got = s.get_state(g).cpu()
    tol = 1e-13 if prec != "fp32" else 1e-6
    assert abs(J.item() - J_ref.item()) < tol * abs(J_ref.item())
    assert_parity(dg, got, g_ref, 1e-12 if prec != "fp32" else 1e-6, label=f"p={p} {prec} wall-pressure gradient")


def test_objective_trajectory_adjoint_vs_oracle():
    from paper_2209_01877_amd.autograd import rk_trajectory

    mesh = make_mesh("bump")
    p = 2
    dg = oracle(p, mesh, FAR)
    # free stream plus small seeded perturbations of the higher modes
    U0 = dg.project(lambda x: fields.freestream(x, FAR[0], FAR[1:4], FAR[4]))
    U0 = U0 + 0.001 * torch.from_numpy(fields.gaussian(U0.shape, 12)) * (torch.arange(dg.Np) > 0)
    dt = 0.5 * dg.stable_dt(U0)
    n = 4
    Un = U0
    for _ in range(n):
        Un = dg.rk3_step(Un, dt)
    Ur = Un.clone().requires_grad_(True)
    (seed,) = torch.autograd.grad(dg.wall_pressure(Ur), Ur)
    ref = oracle_traj(dg, U0, dt, n, seed, checkpoint_every=3)
    s = solver(p, "fp64", mesh, farfield=FAR)
    Ui = s.set_state(U0.cuda()).requires_grad_(True)
    UN = rk_trajectory(s, Ui, dt, n, checkpoint_every=3)
    _, gN = s.wall_pressure(UN.detach(), grad=True)
    (g0,) = torch.autograd.grad(UN, Ui, gN)
    got = s.get_state(g0.contiguous()).cpu()
    assert_parity(dg, got, ref, 1e-11, label="objective trajectory adjoint")


def test_full_size_fifty_steps():
    """56^3 x 6 jittered tets with the bump, P3: 50 SSP-RK3 steps, checkpoints every 10 steps.
    fp64: adjoint gradient of J(U_50) against a central difference along a random direction.
    bf16 forward with its fp64 adjoint: finite, and close to the fp64 gradient."""
    from paper_2209_01877_amd.autograd import rk_trajectory

    mesh = kuhn_cube(56, periodic=(False, False, True), jitter=0.2, jitter_seed=1877, bump_height=0.05,
                     shuffle_seed=2209, vid_seed=2210)
    p, n = 3, 50
    dt = 0.2 * 0.41 * (1.0 / 56) / ((2 * p + 1) * 1.8)
    grads = {}
    for prec in ["fp64", "bf16"]:
        s = solver(p, prec, mesh, farfield=FAR)
        U0 = s.project_fn(lambda x: fields.freestream(x, FAR[0], FAR[1:4], FAR[4]))
        Ui = U0.clone().requires_grad_(True)
        UN = rk_trajectory(s, Ui, dt, n, checkpoint_every=10)
        J, gN = s.wall_pressure(UN.detach(), grad=True)
        (g0,) = torch.autograd.grad(UN, Ui, gN)
        assert torch.isfinite(g0).all()
        grads[prec] = s.get_state(g0.contiguous())  # caller order: the two contexts number differently
        if prec == "fp64":
            gen = torch.Generator(device="cuda").manual_seed(44)
            V = torch.randn(U0.shape, dtype=torch.float64, device="cuda", generator=gen)
            V *= 0.1
            V[:, 0, :, 0] *= 10.0  # the cell means (mode 0) keep unit size
            zero_padding(s, V)
            eps = 1e-6

            def J_of(U):
                X = U.clone()
                s.rk_step(X, dt, n)
                return s.wall_pressure(X).item()

            fd = (J_of(U0 + eps * V) - J_of(U0 - eps * V)) / (2 * eps)
            ad = (g0 * V).sum().item()
            print(f"full size: J = {J.item():.10f}, FD {fd:.10e}, adjoint {ad:.10e}, rel {abs(fd - ad) / abs(ad):.2e}")
            assert abs(fd - ad) < 1e-5 * abs(ad)
        s.sync()
    diff = (grads["bf16"] - grads["fp64"]).norm() / grads["fp64"].norm()
    print(f"bf16-forward adjoint vs fp64 adjoint: rel {diff.item():.3e}")
    assert diff.item() < 1e-2
