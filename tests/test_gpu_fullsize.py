"""GPU parity at the benchmark sizes: the 48^3 x 6 (663,552 tets, P3) periodic cube with
shuffled element order and vertex ids, renumbered as the benchmark does, checked on sampled
elements against the oracle's per-element residual."""
import numpy as np
import pytest
import torch

from synthetic import fields, kuhn_cube

pytestmark = pytest.mark.gpu

from gpu_common import assert_parity, oracle, solver  # noqa: E402


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_c2_sampled_residual(prec, tol):
    mesh = kuhn_cube(48, length=10.0, shuffle_seed=2209, vid_seed=2210)
    p = 3
    dg = oracle(p, mesh)
    U = torch.from_numpy(fields.random_coefficients(mesh.n_elem, dg.Np, seed=21, scale=0.01))
    s = solver(p, prec, mesh, renumber="hilbert")
    Ui = s.set_state(U.cuda())
    R = s.get_state(s.residual(Ui))
    s.sync()
    rng = np.random.default_rng(0)
    sample = torch.from_numpy(np.sort(rng.choice(mesh.n_elem, 96, replace=False)))
    R_ref = dg.residual(U, sample)
    Rs = R[sample.cuda()].cpu()
    assert_parity(dg, Rs, R_ref, tol, vol=dg.volume[sample], label=f"C2 {prec} sampled residual")
    assert torch.isfinite(R).all()


@pytest.fixture(scope="module")
def c3():
    """The benchmark workload: P3 on the 64^3 x 6 (1,572,864 tets) shuffled periodic cube,
    Hilbert renumbering, with the oracle built once for the sampled checks."""
    mesh = kuhn_cube(64, length=10.0, shuffle_seed=2209, vid_seed=2210)
    dg = oracle(3, mesh)
    rng = np.random.default_rng(1)
    sample = torch.from_numpy(np.sort(rng.choice(mesh.n_elem, 96, replace=False)))
    return mesh, dg, sample


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("bf16", 5e-2), ("fp16", 1e-2)])
def test_c3_sampled_stage(c3, prec, tol):
    """One SSP-RK3 stage (alpha = 3/4, with U0) at the benchmark size and in the launch
    configuration the benchmark times, on a random state: sampled elements against
    alpha U0 + (1 - alpha)(U_in + dt R(U_in)) from the oracle's per-element residual.  The
    error is measured relative to the stage's residual part (dt = 1)."""
    mesh, dg, sample = c3
    U = torch.from_numpy(fields.random_coefficients(mesh.n_elem, dg.Np, seed=21, scale=0.01))
    U0 = torch.from_numpy(fields.random_coefficients(mesh.n_elem, dg.Np, seed=22, scale=0.01))
    s = solver(3, prec, mesh, renumber="hilbert")
    Ui, U0i = s.set_state(U.cuda()), s.set_state(U0.cuda())
    out = s.rk_stage(Ui, U0i, s.new_state(), 0.75, 1.0)
    got = s.get_state(out)[sample.cuda()].cpu()
    s.sync()
    R_ref = dg.residual(U, sample)
    if prec == "fp32":  # the stage inputs are stored in fp32
        U, U0 = U.float().double(), U0.float().double()
    ref = 0.75 * U0[sample] + 0.25 * (U[sample] + R_ref)
    # measured against the stage's residual part 0.25 R (dt = 1), per variable
    vol = dg.volume[sample]
    w = vol[:, None, None]
    l2_scale = torch.sqrt((w * (0.25 * R_ref) ** 2).sum((0, 2)))
    assert_parity(dg, got, ref, tol, vol=vol, l2_scale=l2_scale, elem_scale=(0.25 * R_ref).abs().amax((0, 2)),
                  label=f"C3 {prec} sampled stage")


@pytest.mark.parametrize("prec,tol", [("bf16", 0.1), ("fp16", 0.02)])
def test_c3_sampled_residual_vortex(c3, prec, tol):
    """Mixed precision at the benchmark size on the benchmark's smooth state (the projected
    isentropic vortex): sampled residuals against the oracle (stated error)."""
    mesh, dg, sample = c3
    s64 = solver(3, "fp64", mesh, renumber="hilbert")
    U = s64.get_state(s64.project_fn(lambda x: fields.isentropic_vortex(x, length=10.0))).cpu()
    s = solver(3, prec, mesh, renumber="hilbert")
    R = s.get_state(s.residual(s.set_state(U.cuda())))[sample.cuda()].cpu()
    s.sync()
    R_ref = dg.residual(U, sample)
    # the vortex is uniform in z: the rho w residual is discretisation noise, so every variable
    # is measured against the whole residual (pooled over the five variables)
    vol = dg.volume[sample]
    pooled = torch.sqrt((vol[:, None, None] * R_ref ** 2).sum())
    assert_parity(dg, R, R_ref, tol, 3 * tol, vol=vol, l2_scale=pooled, elem_scale=R_ref.abs().max(),
                  label=f"C3 vortex {prec} sampled residual")


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_c2_sampled_navier_stokes_residual(prec, tol):
    """Viscous (BR1) residual on the Navier-Stokes benchmark mesh (48^3 x 6, shuffled, Hilbert
    order, the launch configuration the benchmark times) on sampled elements: the gradient,
    viscous and neighbour-half kernels at full size against the oracle's sampled residual.
    mu = 0.02 so that the viscous part is a visible share of R."""
    mu = 0.02
    mesh = kuhn_cube(48, length=10.0, shuffle_seed=2209, vid_seed=2210)
    dg = oracle(3, mesh, mu=mu)
    U = torch.from_numpy(fields.random_coefficients(mesh.n_elem, dg.Np, seed=23, scale=0.01))
    s = solver(3, prec, mesh, renumber="hilbert", mu=mu)
    R = s.get_state(s.residual(s.set_state(U.cuda())))
    s.sync()
    rng = np.random.default_rng(2)
    sample = torch.from_numpy(np.sort(rng.choice(mesh.n_elem, 64, replace=False)))
    R_ref = dg.residual(U, sample)
    Rs = R[sample.cuda()].cpu()
    R_inv = oracle(3, mesh).residual(U, sample)
    share = (R_ref - R_inv).norm() / R_ref.norm()
    print(f"C2 Navier-Stokes: viscous share {share:.2e}")
    assert share > 1e-3
    assert_parity(dg, Rs, R_ref, tol, vol=dg.volume[sample], label=f"C2 Navier-Stokes {prec} sampled residual")
    assert torch.isfinite(R).all()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("bf16", 5e-2), ("fp16", 1e-2)])
def test_c3b_sampled_stage_p4(prec, tol):
    """The P4 precision-form workload (40^3 x 6 = 384,000 tets, shuffled, Hilbert order, the
    launch configuration the benchmark's P4 leg times): one SSP-RK3 stage on a random state,
    sampled elements against the oracle (error relative to the stage's residual part)."""
    mesh = kuhn_cube(40, length=10.0, shuffle_seed=2209, vid_seed=2210)
    dg = oracle(4, mesh)
    U = torch.from_numpy(fields.random_coefficients(mesh.n_elem, dg.Np, seed=31, scale=0.01))
    U0 = torch.from_numpy(fields.random_coefficients(mesh.n_elem, dg.Np, seed=32, scale=0.01))
    s = solver(4, prec, mesh, renumber="hilbert")
    out = s.rk_stage(s.set_state(U.cuda()), s.set_state(U0.cuda()), s.new_state(), 0.75, 1.0)
    rng = np.random.default_rng(4)
    sample = torch.from_numpy(np.sort(rng.choice(mesh.n_elem, 64, replace=False)))
    got = s.get_state(out)[sample.cuda()].cpu()
    s.sync()
    R_ref = dg.residual(U, sample)
    if prec == "fp32":  # the stage inputs are stored in fp32
        U, U0 = U.float().double(), U0.float().double()
    ref = 0.75 * U0[sample] + 0.25 * (U[sample] + R_ref)
    vol = dg.volume[sample]
    l2_scale = torch.sqrt((vol[:, None, None] * (0.25 * R_ref) ** 2).sum((0, 2)))
    assert_parity(dg, got, ref, tol, vol=vol, l2_scale=l2_scale, elem_scale=(0.25 * R_ref).abs().amax((0, 2)),
                  label=f"C3b P4 {prec} sampled stage")
