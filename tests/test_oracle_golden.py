"""Stored fixtures: the paper's Table 1 (renumbering) and the oracle's own regression pin
for the P1 density wave (written by tests/golden/make_golden.py from oracle/ only)."""
import importlib.util
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_rcmk_bandwidth.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, cells, before, after = line.split()
                rows.append((name, int(cells), int(before), int(after)))
    return rows


def smallest_table1_reduction() -> float:
    """Smallest bandwidth reduction factor RCMK achieves in the paper's Table 1 (Sec. III.B)."""
    return min(before / after for _, _, before, after in read_table1())


def test_table1_fixture():
    rows = read_table1()
    assert [r[1] for r in rows] == [2688, 4032, 16128, 64512]
    assert abs(smallest_table1_reduction() - 1427 / 69) < 1e-12


def test_c1_density_wave_regression():
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(GOLDEN, "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    stored = {}
    with open(os.path.join(GOLDEN, "c1_density_wave.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                key, *vals = line.split()
                stored[key] = np.array([float(v) for v in vals])
    dt, norms, errs = mod.c1_density_wave()
    assert abs(dt - stored["dt"][0]) <= 1e-15 * dt
    assert np.allclose(norms, stored["norm"], rtol=1e-12, atol=0)
    assert np.allclose(errs, stored["error"], rtol=1e-9, atol=1e-15)
