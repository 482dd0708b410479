"""Pins for two oracle functions by what geometry and linear algebra fix on their own.

* Time-step rule (the paper's global minimum of local explicit steps, Sec. III.C;
  reading: dt_K = cfl d_K / ((2p+1)(|u_K| + c_K)) with d_K the in-sphere diameter and
  cell means of the state).
  - On the Kuhn split every tetrahedron is congruent to the path simplex
    (0,0,0)-(h,0,0)-(h,h,0)-(h,h,h): volume h^3/6, two faces of area h^2/2 and two of
    area h^2/sqrt(2), so its in-sphere diameter is (sqrt 2 - 1) h exactly.
  - On jittered tetrahedra the in-sphere diameter is twice the distance from the
    incentre (the face-area-weighted mean of the vertices) to every face plane; that
    distance is computed here from the corner coordinates alone.
  - A uniform state has one wave speed |u| + c everywhere, so the step is a closed form.
* Roe's flux with Harten's entropy fix (the paper's interface flux, Sec. II.B; fix width
  0.1 c on the acoustic waves, a reading).  Reference: the Roe matrix written as the
  flux Jacobian at the Roe-averaged state, differentiated by complex step and
  diagonalised with numpy.linalg.eig, |A| = R |Lambda|_fix R^-1 -- a route that shares
  no step with the oracle's wave-strength formulas.  The state pairs put u.n - c inside
  the fix band, so the fixed branch decides the value.  Continuity and a continuous
  derivative of the flux where |u.n - c| crosses the band edge pin the fix's form.
"""
import math

import numpy as np
import pytest
import torch

from oracle import euler
from oracle.dg import DG
from synthetic import fields, kuhn_cube

GAMMA = 1.4


# ----------------------------------------------------------------- time step
@pytest.mark.parametrize("p", [1, 2, 3])
def test_kuhn_insphere_and_uniform_state_dt(p):
    """Uniform state rho = 1, u = (0.3, 0, 0.4), p = 1/1.4: |u| = 0.5 and c = 1, so on the
    4^3 x 6 unit cube (h = 1/4) every local step is cfl (sqrt2 - 1)/4 / ((2p+1) 1.5)."""
    m = kuhn_cube(4)
    dg = DG(p, m.elem_vid, m.elem_xyz)
    d = 6.0 * dg.geo.volume / dg.geo.area.sum(1)
    assert np.allclose(d, (math.sqrt(2.0) - 1.0) * 0.25, rtol=1e-14, atol=0)
    U = dg.project(lambda x: fields.freestream(x, 1.0, (0.3, 0.0, 0.4), 1.0 / GAMMA))
    cfl = 0.2
    expect = cfl * (math.sqrt(2.0) - 1.0) * 0.25 / ((2 * p + 1) * 1.5)
    assert abs(dg.local_dt_min(U, cfl) - expect) < 1e-14 * expect
    assert abs(dg.stable_dt(U, cfl) - expect) < 1e-14 * expect


def _insphere_diameter_from_corners(xyz: np.ndarray) -> np.ndarray:
    """2 x distance from the incentre to the face planes, from corner coordinates only."""
    out = np.empty(len(xyz))
    for e, X in enumerate(xyz):
        areas, planes = [], []
        for f in range(4):
            a, b, c = [X[v] for v in range(4) if v != f]
            nvec = np.cross(b - a, c - a)
            areas.append(0.5 * np.linalg.norm(nvec))
            planes.append((nvec / np.linalg.norm(nvec), a))
        w = np.array(areas)
        centre = (w[:, None] * X).sum(0) / w.sum()    # vertex f weighted by the opposite face
        dist = [abs(np.dot(nu, centre - a)) for nu, a in planes]
        assert max(dist) - min(dist) < 1e-12 * max(dist)   # equidistant: it is the incentre
        out[e] = 2.0 * dist[0]
    return out


def test_local_dt_min_jittered_brute_force():
    """min over elements of cfl d_K / ((2p+1)(|u_K| + c_K)) with d_K from the incentre and
    |u_K| + c_K from cell means evaluated on the element's own volume points."""
    m = kuhn_cube(3, jitter=0.2, shuffle_seed=2209, vid_seed=2210)
    p, cfl = 2, 0.3
    dg = DG(p, m.elem_vid, m.elem_xyz)
    U = dg.project(fields.RandomSmooth(seed=42))
    d = _insphere_diameter_from_corners(dg.geo.xyz)
    # cell mean = volume-weighted average of the point values (the rule integrates degree 2p+1)
    Uq = dg.evaluate(U).numpy()
    w = dg.w.numpy() if torch.is_tensor(dg.w) else np.asarray(dg.w)
    mean = (w[None, :, None] * Uq).sum(1) / w.sum()
    rho = mean[:, 0]
    vel = mean[:, 1:4] / rho[:, None]
    pres = (GAMMA - 1.0) * (mean[:, 4] - 0.5 * rho * (vel ** 2).sum(1))
    speed = np.linalg.norm(vel, axis=1) + np.sqrt(GAMMA * pres / rho)
    expect = (cfl * d / ((2 * p + 1) * speed)).min()
    assert abs(dg.local_dt_min(U, cfl) - expect) < 1e-12 * expect


# ----------------------------------------------------------------- Roe / Harten
def _normal_flux_np(U, n):
    rho, m, E = U[0], U[1:4], U[4]
    u = m / rho
    p = (GAMMA - 1.0) * (E - 0.5 * np.dot(m, u))
    un = np.dot(u, n)
    return np.concatenate([[rho * un], m * un + p * n, [(E + p) * un]])


def _jacobian_cs(U, n):
    A = np.zeros((5, 5))
    for k in range(5):
        Uc = U.astype(complex)
        Uc[k] += 1e-30j
        A[:, k] = _normal_flux_np(Uc, n).imag / 1e-30
    return A


def _roe_eig(UL, UR, n, delta=0.1):
    rl, rr = UL[0], UR[0]
    ul, ur = UL[1:4] / rl, UR[1:4] / rr
    pl = (GAMMA - 1.0) * (UL[4] - 0.5 * rl * ul @ ul)
    pr = (GAMMA - 1.0) * (UR[4] - 0.5 * rr * ur @ ur)
    hl, hr = (UL[4] + pl) / rl, (UR[4] + pr) / rr
    sl, sr = math.sqrt(rl), math.sqrt(rr)
    u = (sl * ul + sr * ur) / (sl + sr)
    H = (sl * hl + sr * hr) / (sl + sr)
    c2 = (GAMMA - 1.0) * (H - 0.5 * u @ u)
    # a conserved state with this velocity and enthalpy (the Jacobian depends on u and H only)
    rho_hat = sl * sr
    p_hat = rho_hat * c2 / GAMMA
    Uhat = np.concatenate([[rho_hat], rho_hat * u, [p_hat / (GAMMA - 1.0) + 0.5 * rho_hat * u @ u]])
    A = _jacobian_cs(Uhat, n)
    # complex arithmetic throughout: the triple eigenvalue u.n may come back as a nearly
    # real complex pair whose eigenvectors are complex
    lam, R = np.linalg.eig(A)
    c, un = math.sqrt(c2), u @ n
    d = delta * c
    lr = lam.real
    absl = np.abs(lr)
    for k in range(5):
        acoustic = min(abs(lr[k] - (un - c)), abs(lr[k] - (un + c))) < 1e-8
        if acoustic and abs(lr[k]) < d:
            absl[k] = (lr[k] ** 2 + d * d) / (2.0 * d)
    absA = (R @ np.diag(absl) @ np.linalg.inv(R)).real
    flux = 0.5 * (_normal_flux_np(UL, n) + _normal_flux_np(UR, n)) - 0.5 * absA @ (UR - UL)
    return flux, un - c, d


def _cons(rho, vel, p):
    vel = np.asarray(vel, float)
    return np.concatenate([[rho], rho * vel, [p / (GAMMA - 1.0) + 0.5 * rho * vel @ vel]])


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_roe_sonic_pair_against_eigendecomposition(seed):
    rng = np.random.default_rng(seed)
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    t = np.cross(n, [0.3, 0.5, 0.8])
    t /= np.linalg.norm(t)
    # left state just below, right state just above the sound speed along n
    UL = _cons(1.0, 0.97 * math.sqrt(GAMMA) * n + 0.1 * t, 1.0)
    UR = _cons(1.08, 1.02 * math.sqrt(GAMMA / 1.08 * 1.05) * n - 0.05 * t, 1.05)
    ref, lam_sonic, d = _roe_eig(UL, UR, n)
    assert abs(lam_sonic) < d, "the pair must lie inside the entropy-fix band"
    got = euler.roe(torch.from_numpy(UL), torch.from_numpy(UR), torch.from_numpy(n), GAMMA).numpy()
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max(), (got, ref)


def test_roe_subsonic_pair_against_eigendecomposition():
    """Outside the band the same reference applies with plain |lambda|."""
    n = np.array([0.6, 0.0, 0.8])
    UL = _cons(1.0, [0.2, 0.1, -0.1], 1.0)
    UR = _cons(0.9, [0.1, -0.2, 0.3], 0.8)
    ref, lam_sonic, d = _roe_eig(UL, UR, n)
    assert abs(lam_sonic) > d
    got = euler.roe(torch.from_numpy(UL), torch.from_numpy(UR), torch.from_numpy(n), GAMMA).numpy()
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_entropy_fix_continuous_with_continuous_slope_at_band_edge():
    """Move the right state's normal velocity so that u.n - c of the Roe average sweeps
    through -delta (the band edge): the flux and its slope show no jump there."""
    n = torch.tensor([1.0, 0.0, 0.0], dtype=torch.float64)
    UL = torch.from_numpy(_cons(1.0, [0.7 * math.sqrt(GAMMA), 0.0, 0.0], 1.0))

    def at(s):
        UR = torch.from_numpy(_cons(1.0, [s * math.sqrt(GAMMA), 0.05, 0.0], 1.0))
        return euler.roe(UL, UR, n, GAMMA)

    def sonic(s):
        UR = _cons(1.0, [s * math.sqrt(GAMMA), 0.05, 0.0], 1.0)
        _, lam, d = _roe_eig(UL.numpy(), UR, n.numpy())
        return lam + d      # zero at the band edge lambda = -delta

    # bisect for the edge
    lo, hi = 0.6, 1.2
    assert sonic(lo) < 0 < sonic(hi)
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if sonic(mid) < 0 else (lo, mid)
    s0 = 0.5 * (lo + hi)
    h = 1e-5
    left_slope = (at(s0 - h) - at(s0 - 2 * h)) / h
    right_slope = (at(s0 + 2 * h) - at(s0 + h)) / h
    jump = (at(s0 + 1e-9) - at(s0 - 1e-9)).abs().max()
    assert jump < 1e-8
    # one-sided slopes agree to O(h) (a kinked |lambda| would differ by O(1))
    assert (left_slope - right_slope).abs().max() < 1e-3 * left_slope.abs().max()
