"""Pins for the oracle residual against what the method fixes (Sec. II.B, eq. 11).

* free-stream preservation on jittered, shuffled, relabelled meshes;
* discrete conservation: cell-average residuals weighted by |K| sum to zero on a torus;
* translation and rotation invariance (momentum residual rotates with the mesh);
* p = 0 reduces to the textbook cell-centred finite-volume Rusanov scheme;
* linear-manifold invariant of the density wave (constant u and p);
* order-(p+1) convergence on the density wave and on the isentropic vortex;
* boundary faces: free stream through farfield faces, and a slip wall returns a
  pure-pressure face flux.
"""
import math

import numpy as np
import pytest
import torch

from oracle import euler
from oracle.dg import DG
from synthetic import fields, kuhn_cube

torch.set_num_threads(min(8, torch.get_num_threads()))


def _dg(p, n=4, **kw):
    m = kuhn_cube(n, **kw)
    return DG(p, m.elem_vid, m.elem_xyz, m.bface_vid, m.bface_tag)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_free_stream_jittered(p):
    dg = _dg(p, 4, jitter=0.2, shuffle_seed=2209, vid_seed=2210)
    U = dg.project(lambda x: fields.freestream(x, 1.0, (0.3, -0.2, 0.5), 1.0))
    R = dg.residual(U)
    # flux scale / h_min
    assert R.abs().max().item() < 1e-11 * 4.0 / 0.25 * (1 + p) ** 2


@pytest.mark.parametrize("p", [1, 2, 3])
def test_conservation(p):
    dg = _dg(p, 4, jitter=0.2, shuffle_seed=5)
    U = torch.from_numpy(fields.random_coefficients(dg.n_elem, dg.Np, seed=11, scale=0.01))
    R = dg.residual(U)
    total = (dg.volume[:, None] * R[:, :, 0]).sum(0)
    scale = (dg.volume[:, None] * R[:, :, 0].abs()).sum(0)
    assert (total.abs() <= 1e-13 * scale).all(), (total, scale)


def test_translation_invariance():
    m = kuhn_cube(4, jitter=0.2)
    a = DG(2, m.elem_vid, m.elem_xyz)
    b = DG(2, m.elem_vid, m.elem_xyz + np.array([0.3, -1.7, 2.2]))
    U = torch.from_numpy(fields.random_coefficients(a.n_elem, a.Np, seed=2))
    Ra, Rb = a.residual(U), b.residual(U)
    assert (Ra - Rb).abs().max() < 1e-11 * Ra.abs().max()


def test_rotation_invariance():
    m = kuhn_cube(4, jitter=0.2)
    th = 0.7
    Q = np.array([[math.cos(th), -math.sin(th), 0.0], [math.sin(th), math.cos(th), 0.0], [0.0, 0.0, 1.0]])
    ax = np.array([1.0, 2.0, 3.0]) / math.sqrt(14.0)
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    Q = np.eye(3) + math.sin(1.1) * K + (1 - math.cos(1.1)) * K @ K       # Rodrigues
    a = DG(2, m.elem_vid, m.elem_xyz)
    b = DG(2, m.elem_vid, m.elem_xyz @ Q.T)
    U = torch.from_numpy(fields.random_coefficients(a.n_elem, a.Np, seed=4))
    Qt = torch.from_numpy(Q)
    Ub = U.clone()
    Ub[:, 1:4] = torch.einsum("ab,ebi->eai", Qt, U[:, 1:4])
    Ra, Rb = a.residual(U), b.residual(Ub)
    Ra_rot = Ra.clone()
    Ra_rot[:, 1:4] = torch.einsum("ab,ebi->eai", Qt, Ra[:, 1:4])
    assert (Ra_rot - Rb).abs().max() < 1e-11 * Ra.abs().max()


def _fv_rusanov(elem_vid, elem_xyz, Ubar, gamma=1.4):
    """Textbook cell-centred FV with a Rusanov flux: dU_K/dt = -sum_f A_f Fhat(U_K, U_nb, n_f) / |K|."""
    E = elem_vid.shape[0]
    owners = {}
    for e in range(E):
        for f in range(4):
            key = tuple(sorted(int(v) for i, v in enumerate(elem_vid[e]) if i != f))
            owners.setdefault(key, []).append((e, f))
    out = np.zeros((E, 5))
    for e in range(E):
        X = elem_xyz[e]
        vol = abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1))) / 6.0
        for f in range(4):
            key = tuple(sorted(int(v) for i, v in enumerate(elem_vid[e]) if i != f))
            nb = [o for o in owners[key] if o[0] != e][0][0]
            a, b, c = [X[i] for i in range(4) if i != f]
            av = 0.5 * np.cross(b - a, c - a)
            if np.dot(av, a - X[f]) < 0:
                av = -av
            area = np.linalg.norm(av)
            n = av / area

            def phys(U):
                rho, m, E_ = U[0], U[1:4], U[4]
                u = m / rho
                p = (gamma - 1) * (E_ - 0.5 * rho * u @ u)
                F = np.concatenate([[m @ n], m * (u @ n) + p * n, [(E_ + p) * (u @ n)]])
                return F, abs(u @ n) + math.sqrt(gamma * p / rho)

            FL, sL = phys(Ubar[e])
            FR, sR = phys(Ubar[nb])
            out[e] -= area * (0.5 * (FL + FR) - 0.5 * max(sL, sR) * (Ubar[nb] - Ubar[e])) / vol
    return out


def test_p0_is_finite_volume():
    m = kuhn_cube(3, jitter=0.15, shuffle_seed=1)
    dg = DG(0, m.elem_vid, m.elem_xyz)
    U = torch.from_numpy(fields.random_coefficients(dg.n_elem, 1, seed=9))
    R = dg.residual(U)[:, :, 0].numpy()
    ref = _fv_rusanov(m.elem_vid, m.elem_xyz, U[:, :, 0].numpy())
    assert np.abs(R - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_density_wave_linear_manifold(p):
    dg = _dg(p, 4, jitter=0.2)
    U = dg.project(lambda x: fields.sine_wave(x))
    R = dg.residual(U)
    scale = R[:, 0].abs().max()
    for d in range(3):
        assert (R[:, 1 + d] - 1.0 * R[:, 0]).abs().max() < 1e-11 * scale
    assert (R[:, 4] - 1.5 * R[:, 0]).abs().max() < 1e-11 * scale


def _run(dg, U, T, dt_max):
    steps = int(math.ceil(T / dt_max))
    dt = T / steps
    for _ in range(steps):
        U = dg.rk3_step(U, dt)
    return U


@pytest.mark.parametrize("p,ns,rate", [(1, (8, 12), 1.8), (2, (4, 8), 2.4), (3, (4, 8), 3.5)])
def test_density_wave_convergence(p, ns, rate):
    errs = []
    T = 0.05
    for n in ns:
        dg = _dg(p, n)
        U = _run(dg, dg.project(lambda x: fields.sine_wave(x)), T, 0.1 / n / ((2 * p + 1) * 3.0))
        errs.append(dg.l2_error(U, lambda x: fields.sine_wave(x, t=T))[0].item())
    assert math.log(errs[0] / errs[1]) / math.log(ns[1] / ns[0]) > rate, errs


@pytest.mark.parametrize("p,ns,rate", [(1, (16, 32), 1.8), (2, (8, 16), 2.5), (3, (8, 16), 3.4)])
def test_vortex_convergence(p, ns, rate):
    """Isentropic vortex (uniform in z, so three hexahedra across z suffice)."""
    errs = []
    T = 0.2
    for n in ns:
        m = kuhn_cube((n, n, 3), length=10.0)
        dg = DG(p, m.elem_vid, m.elem_xyz)
        U = _run(dg, dg.project(lambda x: fields.isentropic_vortex(x)), T, 0.2 * (10.0 / n) / ((2 * p + 1) * 2.8))
        errs.append(dg.l2_error(U, lambda x: fields.isentropic_vortex(x, t=T))[0].item())
    assert math.log(errs[0] / errs[1]) / math.log(ns[1] / ns[0]) > rate, errs


def test_boundary_faces():
    """Farfield faces fed the free stream keep R = 0.  With the mirrored-velocity ghost the
    Rusanov wall flux has no mass or energy part and its momentum part is normal to the wall:
    (p + rho u_n (u_n + lambda)) n, lambda = |u_n| + c."""
    m = kuhn_cube(4, periodic=(False, False, True), jitter=0.2, bump_height=0.05)
    prim = (1.0, 0.5 * math.sqrt(1.4), 0.0, 0.0, 1.0)
    dg = DG(2, m.elem_vid, m.elem_xyz, m.bface_vid, m.bface_tag, farfield_prim=prim)
    # all boundaries farfield: free stream is preserved
    dg.f_tag = torch.where(dg.f_tag > 0, torch.ones_like(dg.f_tag), dg.f_tag)
    U = dg.project(lambda x: fields.freestream(x, *([prim[0], prim[1:4], prim[4]])))
    assert dg.residual(U).abs().max() < 1e-11
    rho, vel, p = 1.1, torch.tensor([0.3, -0.4, 0.2], dtype=torch.float64), 0.9
    Um = euler.prim_to_cons(torch.tensor([[rho, *vel.tolist(), p]], dtype=torch.float64), 1.4)
    n = torch.tensor([[0.0, -0.6, 0.8]], dtype=torch.float64)
    F = euler.rusanov(Um, euler.slipwall_ghost(Um, n), n, 1.4)[0]
    un = float(vel @ n[0])
    lam = abs(un) + math.sqrt(1.4 * p / rho)
    assert abs(F[0]) < 1e-14 and abs(F[4]) < 1e-14
    assert torch.allclose(F[1:4], (p + rho * un * (un + lam)) * n[0], atol=1e-14, rtol=0)


def test_wall_pressure_uniform_state():
    """For a uniform state the integrated wall pressure is p times the wall area (sum of the
    wall triangles' areas from their corner coordinates)."""
    m = kuhn_cube(4, periodic=(False, False, True), jitter=0.2, bump_height=0.05)
    dg = DG(2, m.elem_vid, m.elem_xyz, m.bface_vid, m.bface_tag)
    U = dg.project(lambda x: fields.freestream(x, 1.2, (0.3, 0.0, 0.1), 0.8))
    # wall triangles: boundary faces tagged 2, coordinates from the elements that own them
    area = 0.0
    for k in torch.nonzero(dg.f_tag == 2).flatten().tolist():
        e, f = int(dg.f_em[k]), int(dg.f_fm[k])
        X = dg.geo.xyz[e]
        a, b, c = [X[v] for v in range(4) if v != f]
        area += 0.5 * np.linalg.norm(np.cross(b - a, c - a))
    assert abs(dg.wall_pressure(U).item() - 0.8 * area) < 1e-13 * area


def test_local_dt_min_uniform_state():
    """For a uniform state every local step uses the same wave speed, so the minimum of the
    local steps equals the global formula cfl min d_K / ((2p+1) max(|u| + c))."""
    dg = _dg(2, 4, jitter=0.2)
    U = dg.project(lambda x: fields.freestream(x, 1.0, (0.3, -0.2, 0.5), 1.0))
    assert abs(dg.local_dt_min(U, 0.2) - dg.stable_dt(U, 0.2)) < 1e-14 * dg.stable_dt(U, 0.2)


def test_roe_flux_properties():
    """Roe flux: consistency F(U, U) = F(U).n; supersonic flow (all waves moving out of the
    minus side, u.n > c + entropy-fix width) reduces to the upwind flux F(U-).n; Roe's
    property F(U+) - F(U-) = A_roe (U+ - U-) appears as antisymmetry of the jump term."""
    g = 1.4
    rng = np.random.default_rng(0)
    n = torch.from_numpy(rng.standard_normal((50, 3)))
    n = n / n.norm(dim=1, keepdim=True)
    prim_a = torch.from_numpy(np.c_[rng.uniform(0.8, 1.2, 50), rng.uniform(-0.3, 0.3, (50, 3)), rng.uniform(0.8, 1.2, 50)])
    prim_b = torch.from_numpy(np.c_[rng.uniform(0.8, 1.2, 50), rng.uniform(-0.3, 0.3, (50, 3)), rng.uniform(0.8, 1.2, 50)])
    a = euler.prim_to_cons(prim_a, g)
    b = euler.prim_to_cons(prim_b, g)
    assert torch.allclose(euler.roe(a, a, n, g), euler.normal_flux(a, n, g), atol=1e-14, rtol=0)
    # flux from the other side with the opposite normal is the negative
    assert torch.allclose(euler.roe(a, b, n, g), -euler.roe(b, a, -n, g), atol=1e-13, rtol=0)
    # supersonic along n: add 3.0 n to both velocities
    pa, pb = prim_a.clone(), prim_b.clone()
    pa[:, 1:4] += 3.0 * n
    pb[:, 1:4] += 3.0 * n
    a, b = euler.prim_to_cons(pa, g), euler.prim_to_cons(pb, g)
    assert torch.allclose(euler.roe(a, b, n, g), euler.normal_flux(a, n, g), atol=1e-12, rtol=0)


def test_roe_free_stream_and_conservation():
    m = kuhn_cube(4, jitter=0.2, shuffle_seed=2209, vid_seed=2210)
    dg = DG(2, m.elem_vid, m.elem_xyz, flux="roe")
    U = dg.project(lambda x: fields.freestream(x, 1.0, (0.3, -0.2, 0.5), 1.0))
    assert dg.residual(U).abs().max() < 1e-11
    U = torch.from_numpy(fields.random_coefficients(dg.n_elem, dg.Np, seed=11, scale=0.01))
    R = dg.residual(U)
    total = (dg.volume[:, None] * R[:, :, 0]).sum(0)
    scale = (dg.volume[:, None] * R[:, :, 0].abs()).sum(0)
    assert (total.abs() <= 1e-13 * scale).all()
