"""The SSP-RK3 entry point that allocates nothing (tdg_rk_step_noalloc, work buffer in the
library's fixed per-GPU scratch) against tdg_rk_step with a caller work buffer, through the
C ABI: two calls in a row on one GPU, the second on a smaller mesh, bit for bit equal (same
kernels, same inputs); a mesh whose work buffer exceeds the scratch is refused before any
device work."""
import ctypes

import pytest
import torch

from gpu_common import make_mesh, oracle, random_state, solver
from paper_2209_01877_amd._lib import lib
from synthetic import kuhn_cube

pytestmark = pytest.mark.gpu


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _noalloc(s, U, dt, n):
    return lib.tdg_rk_step_noalloc(s.ctx, ctypes.c_void_p(U.data_ptr()), ctypes.c_double(dt), n, _stream())


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_noalloc_equals_rk_step(prec):
    # the second call runs on a smaller mesh, after the first one left its data in the scratch
    for p, kind in ((3, "jitter4"), (2, "ragged")):
        mesh = make_mesh(kind)
        dg = oracle(p, mesh)
        U = random_state(dg, seed=11)
        dt = 0.5 * dg.stable_dt(U)
        s = solver(p, prec, mesh)
        Ua = s.set_state(U.cuda())
        s.rk_step(Ua, dt, 3)
        Ub = s.set_state(U.cuda())
        rc = _noalloc(s, Ub, dt, 3)
        assert rc == 0, lib.tdg_last_error(s.ctx)
        s.sync()
        a, b = s.get_state(Ua), s.get_state(Ub)
        print(f"noalloc {prec} p={p} {kind} ({mesh.n_elem} tets): max |diff| {float((a - b).abs().max()):.1e}")
        assert torch.equal(a, b)


def test_noalloc_refuses_large_mesh():
    mesh = kuhn_cube(32)  # P3 FP64: two 800-byte states per element, 315 MB of work > 64 MiB
    s = solver(3, "fp64", mesh)
    U = s.new_state()
    before = U.clone()
    rc = _noalloc(s, U, 1e-3, 1)
    s.sync()
    assert rc == -6  # TDG_ERR_NOMEM
    assert b"64 MiB" in lib.tdg_last_error(s.ctx)
    assert torch.equal(U, before)
