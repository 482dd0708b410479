"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bars: FP64 1e-12 and FP32 1e-5, per conserved variable, both in the normwise relative L2
norm (function-space norm, sum_K |K| sum_i c^2) and element-wise (max |gpu - oracle| over
elements and modes against the variable's largest reference value); mixed bf16/fp16
report their error and are held to a loose sanity bound (their accuracy is a measured
quantity).
"""
import math

import numpy as np
import pytest
import torch

from synthetic import fields

pytestmark = pytest.mark.gpu

from gpu_common import assert_parity, gpu_residual, make_mesh, oracle, random_state, rel_err, solver  # noqa: E402

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 5e-2, "fp16": 1e-2}


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "fp16"])
def test_residual_random_state(p, prec):
    mesh = make_mesh("ragged")
    dg = oracle(p, mesh)
    U = random_state(dg)
    R_ref = dg.residual(U)
    R = gpu_residual(solver(p, prec, mesh), U)
    assert_parity(dg, R, R_ref, TOL[prec], label=f"p={p} {prec} residual")


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "fp16"])
def test_residual_with_boundaries(p, prec):
    far = (1.0, 0.5 * math.sqrt(1.4), 0.0, 0.0, 1.0)
    mesh = make_mesh("bump")
    dg = oracle(p, mesh, far)
    U = random_state(dg, seed=3)
    R_ref = dg.residual(U)
    R = gpu_residual(solver(p, prec, mesh, farfield=far), U)
    assert_parity(dg, R, R_ref, TOL[prec], label=f"p={p} {prec} boundary residual")


@pytest.mark.parametrize("p", [1, 3])
def test_points_and_projection(p):
    mesh = make_mesh("jitter4")
    dg = oracle(p, mesh)
    s = solver(p, "fp64", mesh)
    x = s.volume_points().cpu().numpy()
    assert np.abs(x - dg.volume_points()).max() < 1e-14
    vortex = lambda z: fields.isentropic_vortex(z, length=1.0, beta=0.5)  # noqa: E731
    U_ref = dg.project(vortex)
    U = s.get_state(s.project_fn(vortex)).cpu()
    assert_parity(dg, U, U_ref, 1e-14, label=f"p={p} projection")


def test_c1_ten_rk_steps():
    """P1 density wave on the periodic 4^3 x 6 cube, 10 SSP-RK3 steps at CFL 0.2, FP64."""
    mesh = make_mesh("c1")
    dg = oracle(1, mesh)
    U_ref = dg.project(lambda z: fields.sine_wave(z))
    dt = dg.stable_dt(U_ref, cfl=0.2)
    s = solver(1, "fp64", mesh, renumber="rcm")
    Ui = s.project_fn(lambda z: fields.sine_wave(z))
    U0 = s.get_state(Ui).cpu()
    assert_parity(dg, U0, U_ref, 1e-14, label="C1 projection")
    for _ in range(10):
        U_ref = dg.rk3_step(U_ref, dt)
    s.rk_step(Ui, dt, 10)
    U = s.get_state(Ui).cpu()
    s.sync()
    assert_parity(dg, U - U0, U_ref - U0, 1e-12, label=f"C1: 10 steps dt={dt:.4e}, increment")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rk_step_random_state(prec):
    mesh = make_mesh("ragged")
    p = 2
    dg = oracle(p, mesh)
    U = random_state(dg, seed=5)
    dt = 0.5 * dg.stable_dt(U)
    U_ref = U
    for _ in range(3):
        U_ref = dg.rk3_step(U_ref, dt)
    s = solver(p, prec, mesh)
    Ui = s.set_state(U.cuda())
    s.rk_step(Ui, dt, 3)
    Ug = s.get_state(Ui).cpu()
    s.sync()
    assert_parity(dg, Ug - U, U_ref - U, TOL[prec] * (10 if prec == "fp32" else 1), label=f"{prec} 3 steps, increment")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "fp16"])
def test_renumbering_invariance(prec):
    """Results in the caller's order do not depend on the internal numbering."""
    mesh = make_mesh("jitter4")
    dg = oracle(2, mesh)
    U = random_state(dg, seed=9)
    outs = [gpu_residual(solver(2, prec, mesh, renumber=r), U) for r in ["none", "rcm", "morton", "hilbert"]]
    for o in outs[1:]:
        assert torch.equal(o, outs[0])


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "fp16"])
def test_free_stream_and_conservation(prec, flux):
    """A uniform flow has a zero residual (in the mixed modes to fp64 round-off: a point
    carrying the cell mean reproduces the cell-mean flux exactly), and the volume-weighted
    cell-mean residuals of a random state sum to zero, with either interface flux."""
    mesh = make_mesh("jitter4")
    p = 3
    dg = oracle(p, mesh)
    s = solver(p, prec, mesh)
    s.set_flux(flux)
    U = s.project_fn(lambda z: fields.freestream(z, 1.0, (0.3, -0.2, 0.5), 1.0))
    R = s.get_state(s.residual(U)).cpu()
    bound = {"fp64": 1e-11, "fp32": 1e-4, "bf16": 1e-11, "fp16": 1e-11}[prec]
    assert R.abs().max().item() < bound, R.abs().max().item()
    Ur = random_state(dg, seed=11)
    R = gpu_residual(s, Ur)
    total = (dg.volume[:, None] * R[:, :, 0]).sum(0)
    scale = (dg.volume[:, None] * R[:, :, 0].abs()).sum(0)
    ctol = {"fp64": 1e-13, "fp32": 1e-6, "bf16": 1e-6, "fp16": 1e-6}[prec]
    assert (total.abs() <= ctol * scale).all(), (total, scale)


def test_deterministic():
    mesh = make_mesh("ragged")
    dg = oracle(3, mesh)
    U = random_state(dg)
    s = solver(3, "fp64", mesh)
    a = gpu_residual(s, U)
    b = gpu_residual(s, U)
    assert torch.equal(a, b)


@pytest.mark.parametrize("p", [2, 3, 4])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_padding_elements_of_outputs(p, prec):
    """Elements past the mesh (the arrays are padded to the tile width) carry no result: the
    compute calls leave them unchanged or write zeros there, and never a non-finite value.
    The ragged mesh (360 tets) pads 24 elements."""
    mesh = make_mesh("ragged")
    dg = oracle(p, mesh)
    U = random_state(dg)
    s = solver(p, prec, mesh)
    assert s.n_elem_pad > s.n_elem
    Ui = s.set_state(U.cuda())
    before = Ui[:, :, s.n_elem:].clone()
    R = s.residual(Ui)
    s.rk_step(Ui, 0.5 * dg.stable_dt(U), 2)
    s.sync()
    # R starts as zeros (new_state), so either way its padding is zero
    assert not R[:, :, s.n_elem:].any()
    pad = Ui[:, :, s.n_elem:]
    assert torch.isfinite(pad).all()
    assert torch.equal(pad, before) or not pad.any(), "padding neither unchanged nor zero"


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_stable_dt(prec):
    """GPU minimum of the local time steps against the oracle's."""
    mesh = make_mesh("ragged")
    dg = oracle(2, mesh)
    U = random_state(dg, seed=13)
    s = solver(2, prec, mesh)
    dt = s.stable_dt(s.set_state(U.cuda()), cfl=0.3).item()
    ref = dg.local_dt_min(U, cfl=0.3)
    assert abs(dt - ref) < (1e-14 if prec != "fp32" else 1e-6) * ref


@pytest.mark.parametrize("p", [1, 3])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_single_element(p, prec):
    """Degenerate mesh: one tetrahedron whose four faces are boundary faces (farfield and
    slip wall), i.e. one live column in a padded 16-element tile."""
    far = (1.0, 0.5 * math.sqrt(1.4), 0.0, 0.0, 1.0)
    mesh = make_mesh("single")
    dg = oracle(p, mesh, far)
    U = random_state(dg, seed=31)
    R_ref = dg.residual(U)
    s = solver(p, prec, mesh, farfield=far)
    R = gpu_residual(s, U)
    assert_parity(dg, R, R_ref, {"fp64": 1e-12, "fp32": 1e-5, "bf16": 5e-2}[prec], label=f"single element p={p} {prec}")


def test_zero_steps_leave_state_unchanged():
    mesh = make_mesh("ragged")
    dg = oracle(2, mesh)
    s = solver(2, "bf16", mesh)
    U = s.set_state(random_state(dg, seed=3).cuda())
    V = U.clone()
    s.rk_step(U, 1e-3, 0)
    dts = s.rk_step_adaptive(U, 0.3, 0)
    s.sync()
    assert torch.equal(U, V) and dts.numel() == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_rk_step_adaptive(prec):
    """Steps sized on the device every step (minimum of the local stable steps of the current
    state): bitwise equal to fixed-step calls with the same step sizes, and against the
    oracle taking the same rule on the host (step sizes and end state)."""
    mesh = make_mesh("jitter4")
    dg = oracle(2, mesh)
    U = torch.from_numpy(fields.random_coefficients(dg.n_elem, dg.Np, seed=21, scale=0.01))
    n, cfl = 6, 0.3
    ref, dts_ref = U.clone(), []
    for _ in range(n):
        dts_ref.append(dg.local_dt_min(ref, cfl=cfl))
        ref = dg.rk3_step(ref, dts_ref[-1])
    s = solver(2, prec, mesh)
    Ui = s.set_state(U.cuda())
    dts = s.rk_step_adaptive(Ui, cfl, n)
    Uf = s.set_state(U.cuda())
    for k in range(n):
        s.rk_step(Uf, dts[k].item(), 1)
    assert torch.equal(Ui, Uf)
    got = s.get_state(Ui).cpu()
    s.sync()
    dts = dts.cpu().numpy()
    # the low-precision runs' states (hence their later step sizes) differ from the fp64
    # trajectory at the level of their residual error
    dt_tol = {"fp64": 1e-13, "fp32": 1e-5, "bf16": 1e-4}[prec]
    assert np.allclose(dts, dts_ref, rtol=dt_tol, atol=0), (dts, dts_ref)
    print(f"adaptive {prec}: dt {dts}")
    assert_parity(dg, got - U, ref - U, {"fp64": 1e-12, "fp32": 1e-5, "bf16": 1e-2}[prec], label=f"adaptive {prec}, increment")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("bad", ["negative_pressure", "nan_density"])
def test_inadmissible_state_reports_zero_dt(prec, bad):
    """One element with an inadmissible cell mean: the device minimum of the local steps is
    0 (not the minimum over the remaining elements), the adaptive loop records dt = 0 for
    that step, and the admissibility check counts the element."""
    mesh = make_mesh("jitter4")
    dg = oracle(2, mesh)
    U = torch.from_numpy(fields.random_coefficients(dg.n_elem, dg.Np, seed=21, scale=0.01))
    k = dg.n_elem // 3
    if bad == "negative_pressure":
        U[k, 4, 0] = -1.0  # negative total energy: p < 0
    else:
        U[k, 0, 0] = float("nan")
    s = solver(2, prec, mesh)
    Ui = s.set_state(U.cuda())
    dt = s.stable_dt(Ui, 0.3)
    n_bad = s.check_state(Ui)
    dts = s.rk_step_adaptive(Ui, 0.3, 2)
    s.sync()
    assert dt.item() == 0.0, dt.item()
    assert dts[0].item() == 0.0, dts.cpu()
    assert n_bad.item() >= 1


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_check_state(prec):
    """Elements with a non-finite value or non-positive density or pressure at a volume point,
    counted on the GPU, against the count from the oracle's point values."""
    from oracle import euler

    mesh = make_mesh("ragged")
    dg = oracle(2, mesh)
    U = random_state(dg, seed=23)
    s = solver(2, prec, mesh)
    assert s.check_state(s.set_state(U.cuda())).item() == 0
    U[3, 2, 5] = float("nan")                       # non-finite coefficient
    U[17, 0, 0] = -0.5                              # negative mean density
    U[40, 4, :] = 0.0                               # zero total energy: negative pressure
    U[41, 0, 1] = 3.0                               # density negative at some points only
    Uq = dg.evaluate(U)
    rho, p = Uq[..., 0], euler.pressure(Uq, 1.4)
    bad = ~torch.isfinite(Uq).all(-1) | ~(rho > 0) | ~(p > 0)
    ref = int(bad.any(-1).sum())
    assert ref == 4
    assert s.check_state(s.set_state(U.cuda())).item() == ref


@pytest.mark.parametrize("p", [1, 3])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("kind", ["ragged", "bump"])
def test_roe_flux(p, prec, kind):
    """The paper's Roe interface flux as an option, against the oracle's Roe flux."""
    from oracle.dg import DG

    far = (1.0, 0.5 * math.sqrt(1.4), 0.0, 0.0, 1.0)
    mesh = make_mesh(kind)
    dg = DG(p, mesh.elem_vid, mesh.elem_xyz, mesh.bface_vid, mesh.bface_tag, farfield_prim=far, flux="roe")
    U = random_state(dg, seed=17)
    s = solver(p, prec, mesh, farfield=far)
    s.set_flux("roe")
    assert_parity(dg, gpu_residual(s, U), dg.residual(U), TOL[prec], label=f"roe p={p} {prec} {kind}")


def _pooled(dg, X):
    """Norms of all five variables together: the function-space L2 norm and the largest
    magnitude (scales for variables whose own size is discretisation noise, like rho w of a
    vortex that is uniform in z)."""
    return dg.l2_norm(X).pow(2).sum().sqrt(), X.abs().max()


def test_temporal_mixed_precision():
    """MP-N (the paper's temporal mixed precision, Sec. III.B, Table 2): the first N of 20
    SSP-RK3 steps in FP32, the rest in FP64, against the oracle's FP64 trajectory.

    N = 0 is the FP64 path: its increment U_20 - U_0 matches the oracle's to 1e-12.  For N > 0
    the FP32 steps store the state in fp32 after every stage, 3N roundings of relative size
    2^-24 of a state that is ~700 times the increment here; the error of the increment is
    held to that worst case, 3N 2^-24 |U| / |dU| + 1e-5 (the FP32 residual bar), per
    variable against the pooled increment.  It also equals the plain FP64 run for N = 0 bit
    for bit."""
    from paper_2209_01877_amd.schedule import TemporalMixed

    mesh = make_mesh("jitter4")
    dg = oracle(2, mesh)
    U0 = dg.project(lambda z: fields.isentropic_vortex(z, length=1.0, beta=0.5))
    dt = 0.5 * dg.stable_dt(U0)
    U_ref = U0
    for _ in range(20):
        U_ref = dg.rk3_step(U_ref, dt)
    dU = U_ref - U0
    l2_inc, max_inc = _pooled(dg, dU)
    l2_state, _ = _pooled(dg, U0)
    tm = TemporalMixed(2, mesh)
    plain = solver(2, "fp64", mesh)
    Ui = plain.set_state(U0.cuda())
    plain.rk_step(Ui, dt, 20)
    U_all64 = plain.get_state(Ui).cpu()
    got0 = tm.run(U0.cuda(), dt, 0, 20).cpu()
    assert torch.equal(got0, U_all64)
    assert_parity(dg, got0 - U0, dU, 1e-12, l2_scale=l2_inc, elem_scale=max_inc, label="MP-0 increment vs oracle")
    errs = []
    for n in (5, 10, 20):
        got = tm.run(U0.cuda(), dt, n, 20).cpu()
        bar = 3 * n * 2.0 ** -24 * float(l2_state / l2_inc) + 1e-5
        errs.append(assert_parity(dg, got - U0, dU, bar, l2_scale=l2_inc, elem_scale=max_inc,
                                  label=f"MP-{n} increment vs oracle (bar {bar:.1e})")[0])
    print("MP-N increment errors vs the FP64 oracle:", errs)


@pytest.mark.parametrize("p", [2, 3, 4])
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_rk_step_mixed_multistep(p, prec):
    """Three SSP-RK3 steps in a mixed mode through tdg_rk_step, where each stage kernel writes
    the next stage's low-precision operand companion in its epilogue (at P2 and P4 the records
    have all-padding operand slots, which the epilogue zero-fills).  The work buffer starts
    filled with NaN bytes, so any companion slot left unwritten would poison the result.
    - Equal to the same stages issued one at a time with tdg_rk_stage, which builds each
      companion afresh from the fp64 state, to fp64 round-off: up to P3, rk_step stores the
      second stage as W2 = U0/3 + 2 U2/3 and forms U3 = W2 + (2/3) dt R(U2), the same
      update rounded differently (a companion slot left unwritten or wrong would show at
      the operand precision, ~1e-3); at P4 bit for bit.
    - The increment U_3 - U_0 against the oracle and against the GPU FP64 run (stated error,
      relative to the increment)."""
    mesh = make_mesh("ragged")
    dg = oracle(p, mesh)
    U = random_state(dg, seed=5)
    dt = 0.5 * dg.stable_dt(U)
    s = solver(p, prec, mesh)
    Ua = s.set_state(U.cuda())
    work = s.new_work()
    work.fill_(255)  # NaN as bf16, fp16, fp32 and fp64
    s.rk_step(Ua, dt, 3, work)
    Ub = s.set_state(U.cuda())
    U1, U2 = s.new_state(), s.new_state()
    for _ in range(3):
        s.rk_stage(Ub, None, U1, 0.0, dt)
        s.rk_stage(U1, Ub, U2, 0.75, dt)
        s.rk_stage(U2, Ub, U1, 1.0 / 3.0, dt)
        Ub.copy_(U1)
    s.sync()
    # compared on the mesh's elements (elements past the mesh, which pad the arrays to a
    # multiple of the tile width, are not part of the result)
    A, B = s.get_state(Ua), s.get_state(Ub)
    assert torch.isfinite(A).all()
    assert (A - B).abs().max().item() <= 1e-13 * B.abs().max().item(), (A - B).abs().max().item()
    if p == 4:
        assert torch.equal(A, B)
    got = s.get_state(Ua).cpu()
    ref = U
    for _ in range(3):
        ref = dg.rk3_step(ref, dt)
    s64 = solver(p, "fp64", mesh)
    U64 = s64.set_state(U.cuda())
    s64.rk_step(U64, dt, 3)
    got64 = s64.get_state(U64).cpu()
    s64.sync()
    tol = {"bf16": 1e-2, "fp16": 2e-3}[prec]
    assert_parity(dg, got - U, ref - U, tol, 3 * tol, label=f"p={p} {prec} 3 steps, increment vs oracle")
    assert_parity(dg, got - U, got64 - U, tol, 3 * tol, label=f"p={p} {prec} 3 steps, increment vs GPU FP64")


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_mixed_residual_scales_exactly_with_the_mesh(prec):
    """The deviation fluxes are linear in M = |det J| J^-1, which scales as h^2: on a mesh
    shrunk by 2^-10 they would sit far below fp16's normal range (smallest normal 6.1e-5)
    and be lost in the operand conversion.  The kernel scales M per element by a power of
    two before the fp32 fluxes and undoes it exactly on the fp32 contraction results, so the
    mixed residual of the shrunk mesh is bit for bit 2^10 times that of the unit mesh (the
    geometry scales exactly by powers of two), in bf16 and in fp16; the error against the
    GPU FP64 residual (itself oracle-checked) is the stated one."""
    import dataclasses

    base = make_mesh("jitter4")
    R = {}
    for k in (0, 10):
        mesh = dataclasses.replace(base, elem_xyz=base.elem_xyz * 2.0 ** -k)
        dg = oracle(2, mesh)
        U = random_state(dg, seed=13)
        R[k] = gpu_residual(solver(2, prec, mesh), U)
        if k == 0:
            R64 = gpu_residual(solver(2, "fp64", mesh), U)
            err = float(((R[k] - R64).pow(2).sum() / R64.pow(2).sum()).sqrt())
    print(f"{prec}: residual error vs FP64 {err:.3e}; shrunk mesh max |R - 2^10 R_unit| "
          f"{float((R[10] - R[0] * 2.0 ** 10).abs().max()):.3e}")
    assert err < {"bf16": 5e-2, "fp16": 1e-2}[prec]
    assert torch.equal(R[10], R[0] * 2.0 ** 10)


def test_hundred_rk_steps_p3():
    """Full-length run: P3 isentropic vortex on the shuffled periodic 12^3 x 6 cube (10,368
    tets, Hilbert order), 100 SSP-RK3 steps at CFL 0.2.  FP64 against the oracle to 1e-12;
    FP32 and the mixed modes against that FP64 run (FP32 to 1e-5, the mixed modes at their
    stated error)."""
    from synthetic import kuhn_cube

    mesh = kuhn_cube(12, length=10.0, shuffle_seed=2209, vid_seed=2210)
    dg = oracle(3, mesh)
    vortex = lambda x: fields.isentropic_vortex(x, length=10.0)  # noqa: E731
    U0 = dg.project(vortex)
    dt = 0.2 * 0.41 * (10.0 / 12) / (7 * 3.1)
    U_ref = U0
    for _ in range(100):
        U_ref = dg.rk3_step(U_ref, dt)
    out = {}
    for prec in ["fp64", "fp32", "bf16", "fp16"]:
        s = solver(3, prec, mesh, renumber="hilbert")
        Ui = s.set_state(U0.cuda())
        s.rk_step(Ui, dt, 100)
        out[prec] = s.get_state(Ui).cpu()
        s.sync()
    # per-variable differences relative to the whole state (function-space L2 norm and largest
    # magnitude): the vortex has w = 0 exactly, so the discrete rho w is truncation-error
    # noise (~1e-5 of the state) and its own relative error would measure roundoff against it
    l2_state, max_state = _pooled(dg, U_ref)
    assert_parity(dg, out["fp64"], U_ref, 1e-12, l2_scale=l2_state, elem_scale=max_state,
                  label="100 steps FP64 vs oracle (state-relative)")
    print(f"  (own-norm: {rel_err(dg, out['fp64'], U_ref):.2e})")
    l2_inc, max_inc = _pooled(dg, U_ref - U0)
    stated = {"fp32": 1e-5, "bf16": 1e-3, "fp16": 2e-4}
    for prec, tol in stated.items():
        assert_parity(dg, out[prec], out["fp64"], tol, l2_scale=l2_state, elem_scale=max_state,
                      label=f"100 steps {prec} vs FP64 (state-relative)")
        # the same difference against the pooled increment U_100 - U_0 (reported)
        inc = float(dg.l2_norm(out[prec] - out["fp64"]).pow(2).sum().sqrt() / l2_inc)
        print(f"  {prec}: relative to the increment {inc:.3e}")
