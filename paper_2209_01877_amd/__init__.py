"""MI355X-native explicit modal DG (3-D Euler, affine tets): residual, SSP-RK3 stages
and the residual vector-Jacobian product, as HIP kernels behind a C ABI (libtetdg.so).
"""
from .solver import PRECISIONS, RENUMBER, Solver, debug_tables, stream_probe  # noqa: F401
