"""SSP-RK3 steps captured in a HIP graph (torch.cuda.CUDAGraph over the library's launches):
every replay, with the program's own eager work between replays, reproduces the eager
result bit for bit.  The captured calls issue kernel launches only (no memset or copy)."""
import pytest
import torch

from synthetic import fields

pytestmark = pytest.mark.gpu

from gpu_common import make_mesh, solver  # noqa: E402


@pytest.mark.parametrize("prec,mu", [("fp64", 0.0), ("bf16", 0.0), ("fp64", 0.02), ("fp32", 0.02)])
def test_rk_steps_in_a_graph(prec, mu):
    """mu > 0 adds the viscous launches (lifting, viscous part, neighbour halves) per stage."""
    mesh = make_mesh("jitter4")
    s = solver(2, prec, mesh, mu=mu)
    U0 = s.project_fn(lambda z: fields.RandomSmooth(11)(z))
    dt = 1e-3
    work = s.new_work()
    U = U0.clone()
    s.rk_step(U, dt, 2, work)
    torch.cuda.synchronize()
    ref = U.clone()

    Ug = U0.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream
        s.rk_step(Ug, dt, 2, work)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.rk_step(Ug, dt, 2, work)
    for _ in range(3):
        Ug.copy_(U0)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Ug, ref)
        other = U0 * 2.0  # unrelated eager kernel between replays
        torch.cuda.synchronize()
        assert torch.isfinite(other).all()
