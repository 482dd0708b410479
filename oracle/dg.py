"""Modal DG residual for 3-D Euler on affine tets, and its SSP-RK3 update (FP64, CPU).

Weak form (the inviscid part of the paper's eq. 11, Sec. II.B): for every element
K, conserved variable v and basis function phi_i,

    |K| dc_i/dt = V_i - S_i,
    V_i = integral_K F(U_h) . grad phi_i dx
        = |det J| sum_q w_q sum_d dphi_i/dxi_d(xi_q) (J^-1 F(U_h(xi_q)))_d,
    S_i = sum_f integral_f Fhat(U-, U+, n_f) phi_i dA
        = sum_f 2 A_f sum_q w_q Fhat(U-_q, U+_q, n_f) phi_i(xi_f(s_q, t_q)),

the mass matrix being |K| I for the orthonormal basis.  Element integrals use the
collapsed tet rule with n = p + 1 points per direction, face integrals the
collapsed triangle rule with n = p + 1 (the paper only says Gaussian quadrature).

Assembly is face-centric: every unique face is evaluated once and its flux
integral added to one neighbour and subtracted from the other (the paper's
face-parallel flux mode, Sec. III.A).  Time stepping is the three-stage SSP-RK
scheme in Shu-Osher form (the paper uses an explicit second-order RK; the
explicit RK structure with the residual evaluated once per stage is the same).
"""
from __future__ import annotations

import numpy as np
import torch

from . import basis, euler, quadrature
from .geometry import build_faces, build_geometry

GAMMA = 1.4


class DG:
    def __init__(self, p: int, elem_vid, elem_xyz, bface_vid=None, bface_tag=None,
                 gamma: float = GAMMA, farfield_prim=(1.0, 0.5 * np.sqrt(1.4), 0.0, 0.0, 1.0),
                 chunk: int = 65536, flux: str = "rusanov", mu: float = 0.0, prandtl: float = 0.72):
        self.p = p
        self.mu = mu
        self.prandtl = prandtl
        self.gamma = gamma
        self.chunk = chunk
        self.flux = flux
        self.geo = build_geometry(elem_vid, elem_xyz)
        self.faces = build_faces(self.geo.vid, bface_vid, bface_tag)
        n = p + 1
        self.qpts, self.qw = quadrature.tet_rule(n)
        self.fpts, self.fw = quadrature.triangle_rule(n)
        self.Np = basis.n_modes(p)
        self.B = torch.from_numpy(basis.eval_basis(p, self.qpts))                 # (Nq, Np)
        self.D = torch.from_numpy(basis.eval_basis_grad(p, self.qpts))            # (3, Nq, Np)
        self.Bf = torch.from_numpy(np.stack([basis.eval_basis(p, basis.face_map(f, self.fpts))
                                             for f in range(4)]))                 # (4, Nf, Np)
        self.w = torch.from_numpy(self.qw)
        self.wf = torch.from_numpy(self.fw)
        g = self.geo
        self.jinv = torch.from_numpy(g.jinv)
        self.absdet = torch.from_numpy(g.absdet)
        self.volume = torch.from_numpy(g.volume)
        fc = self.faces
        self.f_em = torch.from_numpy(fc.em).long()
        self.f_fm = torch.from_numpy(fc.fm).long()
        self.f_ep = torch.from_numpy(fc.ep).long()
        self.f_fp = torch.from_numpy(fc.fp).long()
        self.f_tag = torch.from_numpy(fc.tag).long()
        self.f_n = torch.from_numpy(g.normal[fc.em, fc.fm])                      # (F, 3)
        self.f_area = torch.from_numpy(g.area[fc.em, fc.fm])                     # (F,)
        self.farfield = euler.prim_to_cons(torch.tensor(farfield_prim, dtype=torch.float64), gamma)

    @property
    def n_elem(self) -> int:
        return self.geo.vid.shape[0]

    # ---------------------------------------------------------------- inputs
    def volume_points(self) -> np.ndarray:
        """Physical coordinates of the volume quadrature points, (E, Nq, 3)."""
        g = self.geo
        return g.xyz[:, None, 0, :] + np.einsum("kde,qe->kqd", g.jac, self.qpts)

    def project(self, prim_fn) -> torch.Tensor:
        """L2 projection of an analytic primitive field: c_i = (1/|K|) int_K U phi_i = 6 sum_q w_q U_q phi_i."""
        x = torch.from_numpy(self.volume_points())
        Uq = euler.prim_to_cons(prim_fn(x), self.gamma)                          # (E, Nq, 5)
        return 6.0 * torch.einsum("q,qi,eqv->evi", self.w, self.B, Uq)

    def evaluate(self, U: torch.Tensor) -> torch.Tensor:
        """U_h at the volume quadrature points, (E, Nq, 5)."""
        return torch.einsum("qi,evi->eqv", self.B, U)

    # -------------------------------------------------------------- residual
    def volume_term(self, U: torch.Tensor, elems: torch.Tensor | None = None) -> torch.Tensor:
        """V for all elements, or for the listed ones (rows of the result follow `elems`)."""
        idx = torch.arange(self.n_elem) if elems is None else elems
        out = []
        for s in range(0, idx.shape[0], self.chunk):
            ks = idx[s:s + self.chunk]
            Uq = torch.einsum("qi,evi->eqv", self.B, U[ks])
            F = euler.flux(Uq, self.gamma)                                       # (e, q, d, v)
            G = torch.einsum("kde,kqev->kqdv", self.jinv[ks], F)                 # (J^-1 F)_d
            out.append(self.absdet[ks, None, None]
                       * torch.einsum("q,dqi,kqdv->kvi", self.w, self.D, G))
        return torch.cat(out, 0)

    def face_term(self, U: torch.Tensor, elems: torch.Tensor | None = None) -> torch.Tensor:
        """S for all elements, or for the listed ones (rows follow `elems`)."""
        if elems is None:
            row = torch.arange(self.n_elem)
            faces = torch.arange(self.f_em.shape[0])
            nrow = self.n_elem
        else:
            row = torch.full((self.n_elem,), -1, dtype=torch.long)
            row[elems] = torch.arange(elems.shape[0])
            touch = (row[self.f_em] >= 0) | ((self.f_ep >= 0) & (row[self.f_ep.clamp(min=0)] >= 0))
            faces = torch.nonzero(touch).flatten()
            nrow = elems.shape[0]
        S = torch.zeros((nrow,) + tuple(U.shape[1:]), dtype=U.dtype)
        for s in range(0, faces.shape[0], self.chunk):
            fi = faces[s:s + self.chunk]
            em, fm, ep, fp, tag = self.f_em[fi], self.f_fm[fi], self.f_ep[fi], self.f_fp[fi], self.f_tag[fi]
            n = self.f_n[fi][:, None, :]
            Bm = self.Bf[fm]                                                     # (F, Nf, Np)
            Um = torch.einsum("fqi,fvi->fqv", Bm, U[em])
            interior = ep >= 0
            Bp = self.Bf[fp.clamp(min=0)]
            Up = torch.einsum("fqi,fvi->fqv", Bp, U[ep.clamp(min=0)])
            if not bool(interior.all()):
                far = self.farfield.expand_as(Um)
                wall = euler.slipwall_ghost(Um, n.expand(Um.shape[:-1] + (3,)))
                ghost = torch.where((tag == 2)[:, None, None], wall, far)
                Up = torch.where(interior[:, None, None], Up, ghost)
            if self.flux == "roe":
                Fhat = euler.roe(Um, Up, n, self.gamma)
            else:
                Fhat = euler.rusanov(Um, Up, n, self.gamma)                      # (F, Nf, 5)
            scale = 2.0 * self.f_area[fi][:, None, None]
            Sm = scale * torch.einsum("q,fqi,fqv->fvi", self.wf, Bm, Fhat)
            Sp = scale * torch.einsum("q,fqi,fqv->fvi", self.wf, Bp, Fhat)
            rm = row[em]
            rp = torch.where(interior, row[ep.clamp(min=0)], torch.full_like(ep, -1))
            S = S.index_add(0, rm[rm >= 0], Sm[rm >= 0])
            S = S.index_add(0, rp[rp >= 0], -Sp[rp >= 0])
        return S

    def residual(self, U: torch.Tensor, elems: torch.Tensor | None = None) -> torch.Tensor:
        """R(U) = (V - S)/|K|, user layout (E, 5, Np) float64; optionally only for `elems`.
        With mu > 0 the viscous terms of eq. 11 are included: R = (V - S - Vv + Sv)/|K|."""
        vol = self.volume if elems is None else self.volume[elems]
        R = self.volume_term(U, elems) - self.face_term(U, elems)
        if self.mu > 0.0:
            # the viscous face terms of `elems` read Z of the elements and of their neighbours
            R = R - self.viscous_term(U, self.gradient(U, None if elems is None else self.with_neighbours(elems)), elems)
        return R / vol[:, None, None]

    def with_neighbours(self, elems: torch.Tensor) -> torch.Tensor:
        """The elements `elems` and every element sharing a face with one of them (sorted)."""
        inside = torch.zeros(self.n_elem, dtype=torch.bool)
        inside[elems] = True
        interior = self.f_ep >= 0
        ep = self.f_ep.clamp(min=0)
        touch = inside.clone()
        touch[self.f_em[interior & inside[ep]]] = True
        touch[ep[interior & inside[self.f_em]]] = True
        return torch.nonzero(touch).flatten()

    # --------------------------------------------------- viscous terms (BR1)
    def _face_traces(self, U: torch.Tensor, fi: torch.Tensor):
        """Traces of U on faces fi from both sides, with the inviscid ghost on boundary faces."""
        em, fm, ep, fp, tag = self.f_em[fi], self.f_fm[fi], self.f_ep[fi], self.f_fp[fi], self.f_tag[fi]
        n = self.f_n[fi][:, None, :]
        Bm, Bp = self.Bf[fm], self.Bf[fp.clamp(min=0)]
        Um = torch.einsum("fqi,fvi->fqv", Bm, U[em])
        Up = torch.einsum("fqi,fvi->fqv", Bp, U[ep.clamp(min=0)])
        interior = ep >= 0
        if not bool(interior.all()):
            far = self.farfield.expand_as(Um)
            wall = euler.slipwall_ghost(Um, n.expand(Um.shape[:-1] + (3,)))
            ghost = torch.where((tag == 2)[:, None, None], wall, far)
            Up = torch.where(interior[:, None, None], Up, ghost)
        return em, ep, Bm, Bp, Um, Up, interior

    def gradient(self, U: torch.Tensor, elems: torch.Tensor | None = None) -> torch.Tensor:
        """BR1 auxiliary variable Z = grad U, modal, (E, 3, 5, Np):
        |K| Z_i = -integral_K U grad phi_i + sum_f integral_f (U- + U+)/2 n phi_i
        (the first equation of eq. 11 with the central interface value of Bassi and Rebay).
        With `elems`, only those rows are complete (the volume terms of `elems` and the
        faces touching them are evaluated; other rows are partial or zero)."""
        Z = torch.zeros((self.n_elem, 3) + tuple(U.shape[1:]), dtype=U.dtype)
        idx = torch.arange(self.n_elem) if elems is None else elems
        for s in range(0, idx.shape[0], self.chunk):
            ks = idx[s:s + self.chunk]
            Uq = torch.einsum("qi,evi->eqv", self.B, U[ks])
            # d phi_i / d x_e = sum_d D_d jinv[d][e]
            Z[ks] -= self.absdet[ks, None, None, None] * torch.einsum(
                "q,dqi,kde,kqv->kevi", self.w, self.D, self.jinv[ks], Uq)
        if elems is None:
            faces = torch.arange(self.f_em.shape[0])
        else:
            inside = torch.zeros(self.n_elem, dtype=torch.bool)
            inside[elems] = True
            faces = torch.nonzero(inside[self.f_em] | ((self.f_ep >= 0) & inside[self.f_ep.clamp(min=0)])).flatten()
        for s in range(0, faces.shape[0], self.chunk):
            fi = faces[s:s + self.chunk]
            em, ep, Bm, Bp, Um, Up, interior = self._face_traces(U, fi)
            Uh = 0.5 * (Um + Up)
            scale = 2.0 * self.f_area[fi][:, None]
            n = self.f_n[fi]
            Zm = scale[:, :, None, None] * torch.einsum("q,fqi,fqv,fe->fevi", self.wf, Bm, Uh, n)
            Zp = scale[:, :, None, None] * torch.einsum("q,fqi,fqv,fe->fevi", self.wf, Bp, Uh, n)
            Z = Z.index_add(0, em, Zm)
            Z = Z.index_add(0, ep[interior], -Zp[interior])
        return Z / self.volume[:, None, None, None]

    def viscous_term(self, U: torch.Tensor, Z: torch.Tensor, elems: torch.Tensor | None = None) -> torch.Tensor:
        """Vv - Sv with Vv_i = integral_K F_v(U, Z) . grad phi_i and
        Sv_i = sum_f integral_f (F_v(U-, Z-) + F_v(U+, Z+))/2 . n phi_i (BR1; on boundary
        faces U+ is the inviscid ghost and Z+ = Z-); rows follow `elems`."""
        from .viscous import viscous_flux

        idx = torch.arange(self.n_elem) if elems is None else elems
        out = []
        for s in range(0, idx.shape[0], self.chunk):
            ks = idx[s:s + self.chunk]
            Uq = torch.einsum("qi,evi->eqv", self.B, U[ks])
            Zq = torch.einsum("qi,kevi->kqev", self.B, Z[ks])
            Fv = viscous_flux(Uq, Zq, self.gamma, self.mu, self.prandtl)      # (k, q, j, v)
            G = torch.einsum("kde,kqev->kqdv", self.jinv[ks], Fv)
            out.append(self.absdet[ks, None, None] * torch.einsum("q,dqi,kqdv->kvi", self.w, self.D, G))
        Vv = torch.cat(out, 0)
        if elems is None:
            row = torch.arange(self.n_elem)
            faces = torch.arange(self.f_em.shape[0])
        else:
            row = torch.full((self.n_elem,), -1, dtype=torch.long)
            row[elems] = torch.arange(elems.shape[0])
            touch = (row[self.f_em] >= 0) | ((self.f_ep >= 0) & (row[self.f_ep.clamp(min=0)] >= 0))
            faces = torch.nonzero(touch).flatten()
        Sv = torch.zeros_like(Vv)
        for s in range(0, faces.shape[0], self.chunk):
            fi = faces[s:s + self.chunk]
            em, ep, Bm, Bp, Um, Up, interior = self._face_traces(U, fi)
            fm, fp = self.f_fm[fi], self.f_fp[fi]
            Zm = torch.einsum("fqi,fevi->fqev", Bm, Z[em])
            Zp = torch.einsum("fqi,fevi->fqev", Bp, Z[ep.clamp(min=0)])
            Zp = torch.where(interior[:, None, None, None], Zp, Zm)
            n = self.f_n[fi][:, None, :]
            Fm = viscous_flux(Um, Zm, self.gamma, self.mu, self.prandtl)
            Fp = viscous_flux(Up, Zp, self.gamma, self.mu, self.prandtl)
            H = 0.5 * torch.einsum("fqjv,fqj->fqv", Fm + Fp, n.expand(Um.shape[:-1] + (3,)))
            scale = 2.0 * self.f_area[fi][:, None, None]
            Sm = scale * torch.einsum("q,fqi,fqv->fvi", self.wf, Bm, H)
            Sp = scale * torch.einsum("q,fqi,fqv->fvi", self.wf, Bp, H)
            rm = row[em]
            rp = torch.where(interior, row[ep.clamp(min=0)], torch.full_like(ep, -1))
            Sv = Sv.index_add(0, rm[rm >= 0], Sm[rm >= 0])
            Sv = Sv.index_add(0, rp[rp >= 0], -Sp[rp >= 0])
        return Vv - Sv

    def wall_pressure(self, U: torch.Tensor) -> torch.Tensor:
        """Integrated slip-wall pressure, sum over wall faces of 2 A_f sum_q w_q p(U-_q).

        The objective of the full configuration's adjoint (a boundary-face integral of the
        kind in eq. 11); dJ/dU follows by autograd."""
        wall = torch.nonzero(self.f_tag == 2).flatten()
        em, fm = self.f_em[wall], self.f_fm[wall]
        Um = torch.einsum("fqi,fvi->fqv", self.Bf[fm], U[em])
        p = euler.pressure(Um, self.gamma)
        return (2.0 * self.f_area[wall][:, None] * self.wf[None, :] * p).sum()

    # ------------------------------------------------------------------ time
    def rk3_step(self, U: torch.Tensor, dt: float, rhs=None) -> torch.Tensor:
        """One SSP-RK3 (Shu-Osher) step: U_out = a U0 + (1-a)(U_in + dt R(U_in)), a = 0, 3/4, 1/3."""
        rhs = self.residual if rhs is None else rhs
        U1 = U + dt * rhs(U)
        U2 = 0.75 * U + 0.25 * (U1 + dt * rhs(U1))
        return U / 3.0 + (2.0 / 3.0) * (U2 + dt * rhs(U2))

    def stable_dt(self, U: torch.Tensor, cfl: float = 0.2) -> float:
        """dt = cfl * min_K d_K / ((2p+1) max_K (|u_K| + c_K)), d_K = 6|K|/sum_f A_f, cell means of U."""
        d = 6.0 * self.geo.volume / self.geo.area.sum(1)
        mean = U[:, :, 0]
        rho = mean[:, 0]
        speed = torch.linalg.norm(mean[:, 1:4], dim=1) / rho
        c = torch.sqrt(self.gamma * euler.pressure(mean, self.gamma) / rho)
        return float(cfl * d.min() / ((2 * self.p + 1) * (speed + c).max()))

    def local_dt_min(self, U: torch.Tensor, cfl: float = 0.2) -> float:
        """min_K cfl d_K / ((2p+1)(|u_K| + c_K)): the minimum of the local explicit steps over
        all cells (the paper's time-step reduction), cell means of U."""
        d = torch.from_numpy(6.0 * self.geo.volume / self.geo.area.sum(1))
        mean = U[:, :, 0]
        rho = mean[:, 0]
        speed = torch.linalg.norm(mean[:, 1:4], dim=1) / rho
        c = torch.sqrt(self.gamma * euler.pressure(mean, self.gamma) / rho)
        return float((cfl * d / ((2 * self.p + 1) * (speed + c))).min())

    # ---------------------------------------------------------------- norms
    def l2_norm(self, U: torch.Tensor) -> torch.Tensor:
        """Per-variable function-space L2 norm sqrt(sum_K |K| sum_i c_{K,v,i}^2)."""
        return torch.sqrt((self.volume[:, None, None] * U * U).sum((0, 2)))

    def rel_l2(self, a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
        return self.l2_norm(a - b) / self.l2_norm(b)

    def l2_error(self, U: torch.Tensor, prim_fn) -> torch.Tensor:
        """Per-variable L2 error of U_h against an analytic field (volume rule)."""
        x = torch.from_numpy(self.volume_points())
        exact = euler.prim_to_cons(prim_fn(x), self.gamma)
        diff = self.evaluate(U) - exact
        return torch.sqrt((self.absdet[:, None, None] * self.w[None, :, None] * diff * diff).sum((0, 1)))
