"""Write the oracle regression fixtures of tests/golden/ (run from the repository root:
python tests/golden/make_golden.py).  Calls only oracle/ and synthetic/.

c1_density_wave.txt: the P1 density wave on the periodic 4^3 x 6 cube (384 tets),
projected, dt from the CFL 0.2 rule on the initial cell means, 10 SSP-RK3 steps in
fp64: dt, the per-variable L2 norms of the final state, and its L2 error against the
exact travelling wave at the final time (volume rule)."""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.dg import DG  # noqa: E402
from synthetic import fields, kuhn_cube  # noqa: E402


def c1_density_wave():
    mesh = kuhn_cube(4)
    dg = DG(1, mesh.elem_vid, mesh.elem_xyz)
    U = dg.project(lambda z: fields.sine_wave(z))
    dt = dg.stable_dt(U, cfl=0.2)
    for _ in range(10):
        U = dg.rk3_step(U, dt)
    err = dg.l2_error(U, lambda z: fields.sine_wave(z, t=10 * dt))
    return dt, dg.l2_norm(U).tolist(), err.tolist()


if __name__ == "__main__":
    dt, norms, errs = c1_density_wave()
    with open(os.path.join(HERE, "c1_density_wave.txt"), "w") as f:
        f.write("# written by tests/golden/make_golden.py from the oracle (P1 density wave, 384 tets,\n")
        f.write("# CFL 0.2, 10 SSP-RK3 steps, fp64): dt; per-variable L2 norm of U; L2 error vs exact\n")
        f.write(f"dt {dt!r}\n")
        f.write("norm " + " ".join(repr(x) for x in norms) + "\n")
        f.write("error " + " ".join(repr(x) for x in errs) + "\n")
