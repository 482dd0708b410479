"""GPU adjoint: the VJP kernel against the oracle's reverse-mode adjoint, against central
finite differences of the GPU residual at the differentiation-form size, and the
checkpointed SSP-RK3 trajectory adjoint against the oracle's trajectory adjoint."""
import math

import numpy as np
import pytest
import torch

from oracle.adjoint import residual_vjp as oracle_vjp
from oracle.adjoint import trajectory_vjp as oracle_traj
from oracle.dg import DG
from synthetic import fields, kuhn_cube

pytestmark = pytest.mark.gpu

from gpu_common import assert_parity, make_mesh, oracle, random_state, solver, zero_padding  # noqa: E402

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 1e-12, "fp16": 1e-12}


def gpu_vjp(s, U, W):
    Ui = s.set_state(U.cuda().contiguous())
    Wi = s.set_state(W.cuda().contiguous())
    out = s.get_state(s.residual_vjp(Ui, Wi)).cpu()
    s.sync()
    return out


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_vjp_vs_oracle(p, prec):
    mesh = make_mesh("ragged")
    dg = oracle(p, mesh)
    U = random_state(dg, seed=5)
    W = torch.from_numpy(fields.gaussian(U.shape, 43))
    ref = oracle_vjp(dg, U, W)
    got = gpu_vjp(solver(p, prec, mesh), U, W)
    assert_parity(dg, got, ref, TOL[prec], label=f"p={p} {prec} vjp")


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_vjp_boundaries(p):
    far = (1.0, 0.5 * math.sqrt(1.4), 0.0, 0.0, 1.0)
    mesh = make_mesh("bump")
    dg = oracle(p, mesh, far)
    U = random_state(dg, seed=8)
    W = torch.from_numpy(fields.gaussian(U.shape, 43))
    ref = oracle_vjp(dg, U, W)
    got = gpu_vjp(solver(p, "fp64", mesh, farfield=far), U, W)
    assert_parity(dg, got, ref, 1e-12, label=f"p={p} boundary vjp")


def sonic_state(n_elem, n_modes, seed):
    """Cell means of a Mach-1 flow along x (rho ~ 1, u_x in [1.0, 1.35] around c = 1.18,
    p = 1): on the mesh's x-normal faces u.n -+ c falls inside Harten's entropy-fix band
    |lambda| < 0.1 c, so both branches of the Roe wave speeds are exercised."""
    U = fields.random_coefficients(n_elem, n_modes, seed=seed, scale=0.01)
    rng = np.random.default_rng(seed + 1)
    rho = rng.uniform(0.95, 1.05, n_elem)
    u = np.stack([rng.uniform(1.0, 1.35, n_elem), rng.uniform(-0.1, 0.1, n_elem), rng.uniform(-0.1, 0.1, n_elem)], 1)
    U[:, 0, 0] = rho
    U[:, 1:4, 0] = rho[:, None] * u
    U[:, 4, 0] = 1.0 / 0.4 + 0.5 * rho * (u * u).sum(1)
    return torch.from_numpy(U)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("state", ["subsonic", "sonic"])
def test_roe_vjp_vs_oracle(p, prec, state):
    """Adjoint of the residual with Roe's flux against the oracle's reverse mode."""
    mesh = make_mesh("ragged")
    dg = DG(p, mesh.elem_vid, mesh.elem_xyz, mesh.bface_vid, mesh.bface_tag, flux="roe")
    U = random_state(dg, seed=5) if state == "subsonic" else sonic_state(dg.n_elem, dg.Np, 9)
    if state == "sonic":
        ux = (U[:, 1, 0] / U[:, 0, 0]).numpy()
        c = np.sqrt(1.4 * 0.4 * (U[:, 4, 0] - 0.5 * (U[:, 1:4, 0] ** 2).sum(1) / U[:, 0, 0]).numpy() / U[:, 0, 0].numpy())
        assert (np.abs(ux - c) < 0.1 * c).mean() > 0.2  # the entropy-fix band is populated
    W = torch.from_numpy(fields.gaussian(U.shape, 43))
    ref = oracle_vjp(dg, U, W)
    s = solver(p, prec, mesh)
    s.set_flux("roe")
    got = gpu_vjp(s, U, W)
    assert_parity(dg, got, ref, TOL[prec], label=f"roe p={p} {prec} {state} vjp")


def test_roe_vjp_boundaries():
    far = (1.0, 0.5 * math.sqrt(1.4), 0.0, 0.0, 1.0)
    mesh = make_mesh("bump")
    dg = DG(2, mesh.elem_vid, mesh.elem_xyz, mesh.bface_vid, mesh.bface_tag, farfield_prim=far, flux="roe")
    U = random_state(dg, seed=8)
    W = torch.from_numpy(fields.gaussian(U.shape, 43))
    ref = oracle_vjp(dg, U, W)
    s = solver(2, "fp64", mesh, farfield=far)
    s.set_flux("roe")
    got = gpu_vjp(s, U, W)
    assert_parity(dg, got, ref, 1e-12, label="roe boundary vjp")


def test_vjp_c4_subset_vs_oracle():
    """P2 on the jittered 4^3 x 6 cube with the differentiation-form seeds (state 42, W 43)."""
    mesh = kuhn_cube(4, jitter=0.2, jitter_seed=1877, shuffle_seed=2209)
    dg = oracle(2, mesh)
    U = dg.project(fields.RandomSmooth(42))
    W = torch.from_numpy(fields.gaussian(U.shape, 43))
    ref = oracle_vjp(dg, U, W)
    got = gpu_vjp(solver(2, "fp64", mesh), U, W)
    assert_parity(dg, got, ref, 1e-12, label="C4 subset vjp")


@pytest.mark.parametrize("p", [1, 2, 3])
def test_vjp_free_stream_ties(p):
    """Adjoint at a uniform state on the unjittered periodic cube (h = 1/4, so the geometry is
    exact in binary): both sides of every face carry the same state, so the two wave-speed
    bounds of max(lambda-, lambda+) are equal at every face point, and the flow along x makes
    u.n = 0 exactly on the faces whose normal has no x component.  The VJP takes half of the
    derivative of the max from each side at a tie and d|x|/dx = 0 at x = 0, as reverse-mode AD
    of the oracle does; the two must agree to the FP64 bar."""
    from oracle import euler

    mesh = kuhn_cube(4, shuffle_seed=2209, vid_seed=2210)
    dg = oracle(p, mesh)
    # cell means only (higher modes exactly zero): every face trace is the mean on both sides
    U = torch.zeros(dg.n_elem, 5, dg.Np, dtype=torch.float64)
    U[:, :, 0] = euler.prim_to_cons(torch.tensor([1.0, 0.6, 0.0, 0.0, 1.0], dtype=torch.float64), 1.4)
    em, ep, Bm, Bp, Um, Up, interior = dg._face_traces(U, torch.arange(dg.f_em.shape[0]))
    n = dg.f_n[:, None, :]
    assert torch.equal(euler.wave_speed(Um, n, 1.4), euler.wave_speed(Up, n, 1.4))  # exact ties
    n_zero = int(((Um[..., 1:4] * n).sum(-1) == 0.0).sum())
    assert n_zero > 0  # face points with u.n = 0 exactly
    W = torch.from_numpy(fields.gaussian(U.shape, 43))
    ref = oracle_vjp(dg, U, W)
    got = gpu_vjp(solver(p, "fp64", mesh), U, W)
    assert_parity(dg, got, ref, 1e-12, label=f"p={p} free-stream vjp ({n_zero} face points with u.n = 0)")


def _c4_fd(V_kind: str):
    """<W, (R(U+eV) - R(U-eV))/2e> and <VJP(W), V> on the jittered 40^3 x 6 cube (384,000 tets,
    P2, FP64, eps = 1e-6), state RandomSmooth(42), W Gaussian (seed 43) in the caller layout;
    V Gaussian (seed 44) or the projection of the smooth field RandomSmooth(44)."""
    mesh = kuhn_cube(40, jitter=0.2, jitter_seed=1877, shuffle_seed=2209)
    s = solver(2, "fp64", mesh)
    U = s.project_fn(fields.RandomSmooth(42))
    shape = (mesh.n_elem, 5, s.n_modes)
    W = zero_padding(s, s.set_state(torch.from_numpy(fields.gaussian(shape, 43)).cuda()))
    if V_kind == "gaussian":
        V = zero_padding(s, s.set_state(torch.from_numpy(fields.gaussian(shape, 44)).cuda()))
    else:
        V = s.project_fn(fields.RandomSmooth(44)) - s.project_fn(lambda x: fields.freestream(x, 1.0, (0, 0, 0), 1.0))

    eps = 1e-6
    Rp = s.residual(U + eps * V)
    Rm = s.residual(U - eps * V)
    lhs = (W * (Rp - Rm)).sum().item() / (2 * eps)
    rhs = (s.residual_vjp(U, W) * V).sum().item()
    s.sync()
    rel = abs(lhs - rhs) / abs(rhs)
    print(f"C4 FD ({V_kind} V): {lhs:.12e} vs {rhs:.12e}, rel {rel:.2e}")
    return rel


def test_vjp_c4_finite_difference():
    """Central differences against the VJP at the differentiation-form size.

    Rusanov's flux has kinks: the max of the two wave-speed bounds, and |u.n| inside them.
    A Gaussian direction (jumps of O(1) between neighbours) moves lambda- - lambda+ by O(eps)
    at every face point, so the central difference straddles the max() kink wherever the
    two bounds are within O(eps) of a tie, and each straddle changes the quotient by O(jump x
    slope change): that limits the agreement to a few 1e-6 (bar 5e-6; measured 2.5e-6).
    A smooth direction (the projection of a smooth field, face jumps O(h^3)) moves the bounds'
    difference only by O(eps h^3), so far fewer points straddle, and it agrees to 1e-6
    (measured 3.5e-7).  Its directional derivative is ~200x smaller than the Gaussian one, so
    what remains at eps = 1e-6 is the round-off of R (about 4e-13 per coefficient, summed over
    19 M coefficients against W and divided by 2 eps: a few 1e-7 relative).  A larger eps does
    not help: for a smooth state the two sides' wave speeds differ by O(h^3) at every face
    point, so ties are dense and the straddled kinks grow with eps (eps = 1e-4 with Richardson
    extrapolation measured 1.6e-6).  A wrong Jacobian term shows up at 1e-3 or more in
    either direction."""
    assert _c4_fd("gaussian") < 5e-6
    assert _c4_fd("smooth") < 1e-6


def test_autograd_residual():
    from paper_2209_01877_amd.autograd import residual

    mesh = make_mesh("jitter4")
    dg = oracle(2, mesh)
    U = random_state(dg, seed=3)
    W = torch.from_numpy(fields.gaussian(U.shape, 7))
    s = solver(2, "fp64", mesh)
    Ui = s.set_state(U.cuda()).requires_grad_(True)
    Wi = s.set_state(W.cuda())
    R = residual(s, Ui)
    (g,) = torch.autograd.grad(R, Ui, Wi)
    got = s.get_state(g.contiguous()).cpu()
    assert_parity(dg, got, oracle_vjp(dg, U, W), 1e-12, label="autograd residual")


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_trajectory_adjoint(prec):
    """d<W, U_n>/dU_0 through 5 SSP-RK3 steps with checkpoints every 2 steps.  In fp64 it
    must match the oracle's trajectory adjoint; the mixed forward's adjoint is taken in fp64
    around the mixed stage states and is compared with a looser bound."""
    from paper_2209_01877_amd.autograd import rk_trajectory

    mesh = make_mesh("jitter4")
    dg = oracle(1, mesh)
    U0 = random_state(dg, seed=5, scale=0.005)
    dt = 0.5 * dg.stable_dt(U0)
    W = torch.from_numpy(fields.gaussian(U0.shape, 43))
    ref = oracle_traj(dg, U0, dt, 5, W, checkpoint_every=2)
    s = solver(1, prec, mesh)
    Ui = s.set_state(U0.cuda()).requires_grad_(True)
    Un = rk_trajectory(s, Ui, dt, 5, checkpoint_every=2)
    (g,) = torch.autograd.grad(Un, Ui, s.set_state(W.cuda()))
    got = s.get_state(g.contiguous()).cpu()
    assert_parity(dg, got, ref, 1e-12 if prec == "fp64" else 1e-3, label=f"{prec} trajectory adjoint")
