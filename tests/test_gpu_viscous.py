"""GPU parity of the viscous (BR1) terms against the oracle: residual for p = 1..4 in
FP64 and FP32 on a ragged periodic jittered mesh and with farfield / slip-wall faces,
SSP-RK3 steps, and a uniform state (zero viscous residual)."""
import math

import pytest
import torch

from synthetic import fields

pytestmark = pytest.mark.gpu

from gpu_common import assert_parity, gpu_residual, make_mesh, oracle, random_state, rel_err, solver  # noqa: E402

TOL = {"fp64": 1e-12, "fp32": 1e-5}
MU = 0.02


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ns_residual(p, prec):
    mesh = make_mesh("ragged")
    dg = oracle(p, mesh, mu=MU)
    U = random_state(dg, seed=41)
    R_ref = dg.residual(U)
    s = solver(p, prec, mesh, mu=MU)
    got = gpu_residual(s, U)
    # the viscous part must matter at this scale for the test to mean anything
    dg0 = oracle(p, mesh)
    assert rel_err(dg, dg0.residual(U), R_ref) > 1e-3
    assert_parity(dg, got, R_ref, TOL[prec], label=f"NS p={p} {prec}")


@pytest.mark.parametrize("p", [2, 3])
def test_ns_residual_boundaries(p):
    far = (1.0, 0.5 * math.sqrt(1.4), 0.0, 0.0, 1.0)
    mesh = make_mesh("bump")
    dg = oracle(p, mesh, far, mu=MU)
    U = random_state(dg, seed=42)
    R_ref = dg.residual(U)
    s = solver(p, "fp64", mesh, farfield=far, mu=MU)
    assert_parity(dg, gpu_residual(s, U), R_ref, 1e-12, label=f"NS boundaries p={p}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ns_rk_steps(prec):
    mesh = make_mesh("jitter4")
    dg = oracle(2, mesh, mu=MU)
    U = random_state(dg, seed=43)
    dt = 0.5 * dg.stable_dt(U, cfl=0.2)
    ref = U.clone()
    for _ in range(3):
        ref = dg.rk3_step(ref, dt)
    s = solver(2, prec, mesh, mu=MU)
    Ui = s.set_state(U.cuda())
    s.rk_step(Ui, dt, 3)
    got = s.get_state(Ui).cpu()
    s.sync()
    assert_parity(dg, got - U, ref - U, TOL[prec], label=f"NS rk {prec}, increment")


def test_ns_uniform_state():
    mesh = make_mesh("jitter4")
    s = solver(3, "fp64", mesh, mu=0.1)
    U = s.project_fn(lambda z: fields.freestream(z, 1.0, (0.3, -0.2, 0.5), 1.0))
    R = s.get_state(s.residual(U)).cpu()
    assert R.abs().max().item() < 1e-11


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ns_residual_with_roe_flux(prec):
    """Viscous terms with Roe's inviscid interface flux (the paper's pairing), p = 2, with
    farfield and slip-wall faces."""
    from oracle.dg import DG

    far = (1.0, 0.5 * math.sqrt(1.4), 0.0, 0.0, 1.0)
    mesh = make_mesh("bump")
    dg = DG(2, mesh.elem_vid, mesh.elem_xyz, mesh.bface_vid, mesh.bface_tag, farfield_prim=far, flux="roe", mu=MU)
    U = random_state(dg, seed=44)
    R_ref = dg.residual(U)
    s = solver(2, prec, mesh, farfield=far, mu=MU)
    s.set_flux("roe")
    assert_parity(dg, gpu_residual(s, U), R_ref, TOL[prec], label=f"NS + Roe {prec}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ns_adaptive_steps(prec):
    """Adaptive steps with the viscous terms: bitwise equal to fixed-step calls with the same
    step sizes, and against the oracle taking the same (inviscid) rule on the host."""
    import numpy as np

    mesh = make_mesh("jitter4")
    dg = oracle(2, mesh, mu=MU)
    U = random_state(dg, seed=45)
    n, cfl = 4, 0.2
    ref, dts_ref = U.clone(), []
    for _ in range(n):
        dts_ref.append(dg.local_dt_min(ref, cfl=cfl))
        ref = dg.rk3_step(ref, dts_ref[-1])
    s = solver(2, prec, mesh, mu=MU)
    Ui = s.set_state(U.cuda())
    dts = s.rk_step_adaptive(Ui, cfl, n)
    Uf = s.set_state(U.cuda())
    for k in range(n):
        s.rk_step(Uf, dts[k].item(), 1)
    assert torch.equal(Ui, Uf)
    got = s.get_state(Ui).cpu()
    s.sync()
    assert np.allclose(dts.cpu().numpy(), dts_ref, rtol={"fp64": 1e-13, "fp32": 1e-5}[prec], atol=0)
    assert_parity(dg, got - U, ref - U, TOL[prec], label=f"NS adaptive {prec}, increment")
