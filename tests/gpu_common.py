"""Helpers for the GPU tests (imported only by tests marked gpu)."""
from __future__ import annotations

import numpy as np
import torch

from oracle.dg import DG
from synthetic import fields, kuhn_cube


def make_mesh(kind: str):
    if kind == "ragged":      # 5 x 4 x 3 hexes: 360 tets, not a multiple of 16
        return kuhn_cube((5, 4, 3), length=1.0, jitter=0.2, shuffle_seed=2209, vid_seed=2210)
    if kind == "jitter4":
        return kuhn_cube(4, jitter=0.2, shuffle_seed=2209, vid_seed=2210)
    if kind == "bump":        # farfield x/y sides, slip wall with bump on y = 0, periodic z
        return kuhn_cube(4, periodic=(False, False, True), jitter=0.2, bump_height=0.05,
                         shuffle_seed=2209, vid_seed=2210)
    if kind == "c1":
        return kuhn_cube(4)
    if kind == "single":      # one tetrahedron, every face on the boundary (3 farfield, 1 wall)
        from synthetic.mesh import TetMesh

        xyz = np.array([[[0.0, 0.0, 0.0], [0.9, 0.1, 0.0], [0.2, 1.1, 0.1], [0.1, 0.2, 0.8]]])
        return TetMesh(elem_vid=np.array([[0, 1, 2, 3]], np.int64), elem_xyz=xyz,
                       bface_vid=np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]], np.int64),
                       bface_tag=np.array([1, 2, 1, 1], np.int32), periodic=(False, False, False))
    raise ValueError(kind)


def solver(p, prec, mesh, renumber="hilbert", farfield=None, mu=0.0, prandtl=0.72):
    from paper_2209_01877_amd import Solver

    s = Solver(p, prec)
    if mu > 0.0:
        s.set_viscosity(mu, prandtl)
    s.upload(mesh, renumber=renumber)
    if farfield is not None:
        s.set_farfield(farfield)
    return s


def oracle(p, mesh, farfield=(1.0, 0.5 * np.sqrt(1.4), 0.0, 0.0, 1.0), mu=0.0, prandtl=0.72):
    return DG(p, mesh.elem_vid, mesh.elem_xyz, mesh.bface_vid, mesh.bface_tag, farfield_prim=farfield, mu=mu,
              prandtl=prandtl)


def random_state(dg, seed=7, scale=0.01):
    return torch.from_numpy(fields.random_coefficients(dg.n_elem, dg.Np, seed=seed, scale=scale))


def gpu_residual(s, U_user: torch.Tensor) -> torch.Tensor:
    Ui = s.set_state(U_user.cuda().contiguous())
    R = s.get_state(s.residual(Ui)).cpu()
    s.sync()
    return R


def rel_err(dg, a, b) -> float:
    """Largest per-variable normwise relative L2 error (function-space norm); a variable
    whose reference is identically zero is measured in absolute terms."""
    num = dg.l2_norm(a - b)
    den = dg.l2_norm(b)
    den = torch.where(den > 0, den, torch.ones_like(den))
    return float((num / den).max())


def elem_err(a: torch.Tensor, b: torch.Tensor, scale: torch.Tensor | None = None) -> torch.Tensor:
    """Per variable: the largest element-wise difference max_{K,i} |a - b| divided by the
    largest reference magnitude max_{K,i} |b| of that variable (or by `scale`, one value per
    variable).  A variable whose reference is identically zero is measured in absolute terms.
    Tensors are in the caller layout [elements][5][modes]."""
    d = (a - b).abs().amax(dim=(0, 2))
    s = b.abs().amax(dim=(0, 2)) if scale is None else scale.to(d)
    s = torch.where(s > 0, s, torch.ones_like(s))
    return d / s


def weighted_l2_err(a: torch.Tensor, b: torch.Tensor, vol: torch.Tensor) -> torch.Tensor:
    """Per variable normwise relative L2 error with element weights `vol` (the function-space
    norm restricted to a sample of elements)."""
    w = vol.to(a)[:, None, None]
    num = torch.sqrt((w * (a - b) ** 2).sum((0, 2)))
    den = torch.sqrt((w * b * b).sum((0, 2)))
    den = torch.where(den > 0, den, torch.ones_like(den))
    return num / den


def assert_parity(dg, got: torch.Tensor, ref: torch.Tensor, tol: float, tol_elem: float | None = None,
                  label: str = "", vol: torch.Tensor | None = None, l2_scale: torch.Tensor | None = None,
                  elem_scale: torch.Tensor | None = None):
    """Parity of a GPU result with the oracle's, per conserved variable, by two measures:
    the normwise relative L2 error (function-space norm sum_K |K| sum_i c^2; `vol` restricts
    it to sampled elements) below `tol`, and the element-wise error
    max |got - ref| / max |ref| below `tol_elem` (default `tol`), so that an error confined
    to a few elements cannot hide in the norm.  `l2_scale` / `elem_scale` replace the
    per-variable reference sizes (e.g. by the whole state's) where a variable's own size is
    noise.  Returns (largest L2 error, largest element-wise error)."""
    if vol is None:
        vol = dg.volume
    if l2_scale is None:
        l2 = weighted_l2_err(got, ref, vol)
    else:
        w = vol.to(got)[:, None, None]
        l2 = torch.sqrt((w * (got - ref) ** 2).sum((0, 2))) / l2_scale
    el = elem_err(got, ref, elem_scale)
    te = tol if tol_elem is None else tol_elem
    print(f"{label}: rel L2 {float(l2.max()):.3e} (per variable {' '.join(f'{x:.1e}' for x in l2.tolist())}), "
          f"element-wise {float(el.max()):.3e}")
    assert float(l2.max()) < tol, (label, l2.tolist())
    assert float(el.max()) < te, (label, el.tolist())
    return float(l2.max()), float(el.max())


def zero_padding(s, X: torch.Tensor) -> torch.Tensor:
    """Zero the padding of an internal-layout state [5][ceil(Np/4)][E_pad][4] in place:
    elements past the mesh and the unused modes of the last mode quad."""
    X[:, :, s.n_elem:] = 0
    r = s.n_modes % 4
    if r:
        X[:, -1, :, r:] = 0
    return X

