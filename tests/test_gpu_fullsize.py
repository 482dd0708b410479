"""GPU parity at the benchmark sizes: the 48^3 x 6 (663,552 tets, P3) periodic cube with
shuffled element order and vertex ids, renumbered as the benchmark does, checked on sampled
elements against the oracle's per-element residual."""
import numpy as np
import pytest
import torch

from synthetic import fields, kuhn_cube

pytestmark = pytest.mark.gpu

from gpu_common import oracle, solver  # noqa: E402


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
    err = (Rs - R_ref).norm() / R_ref.norm()
    print(f"C2 {prec}: sampled residual rel error {err:.3e}")
    assert err < tol
    assert torch.isfinite(R).all()
