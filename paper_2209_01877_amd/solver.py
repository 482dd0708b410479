"""Python front end of the HIP DG library: torch tensors supply device memory and
the stream; every computation happens in libtetdg.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import check, lib

PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3}
RENUMBER = {"none": 0, "rcm": 1, "morton": 2, "hilbert": 3}


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Solver:
    """One DG discretisation (order p, precision mode) of one tet mesh on one GPU.

    State tensors returned by this class are in the internal layout
    [5][ceil(N_p/4)][n_elem_pad][4] (renumbered element order, four consecutive modes
    innermost); user-layout tensors are [n_elem][5][N_p] float64 in the caller's order.
    """

    def __init__(self, p: int, precision: str = "fp64", gamma: float = 1.4, device: str = "cuda"):
        self.p = p
        self.precision = precision
        self.gamma = gamma
        self.device = torch.device(device)
        ctx = ctypes.c_void_p()
        check(lib.tdg_create(p, PRECISIONS[precision], gamma, ctypes.byref(ctx)), None, "tdg_create")
        self._ctx = ctx
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib.tdg_sizes(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), ctx)
        self.n_modes, self.n_vol_points, self.n_face_points = a.value, b.value, c.value
        self.state_dtype = torch.float32 if precision == "fp32" else torch.float64
        self._mesh_buf = None
        self.perm = None

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and lib is not None:
            lib.tdg_destroy(ctx)
            self._ctx = None

    @property
    def ctx(self):
        return self._ctx

    # ----------------------------------------------------------------- mesh
    def upload_mesh(self, elem_vid, elem_xyz, bface_vid=None, bface_tag=None, renumber: str = "rcm",
                    stream=None) -> np.ndarray:
        vid = np.ascontiguousarray(elem_vid, dtype=np.int64)
        xyz = np.ascontiguousarray(elem_xyz, dtype=np.float64)
        n = vid.shape[0]
        nb = 0 if bface_vid is None else len(bface_vid)
        bv = np.ascontiguousarray(bface_vid if nb else np.zeros((0, 3)), dtype=np.int64)
        bt = np.ascontiguousarray(bface_tag if nb else np.zeros((0,)), dtype=np.int32)
        perm = np.empty(n, dtype=np.int64)
        check(lib.tdg_mesh_upload(self._ctx, n, vid.ctypes.data, xyz.ctypes.data, nb,
                                  bv.ctypes.data if nb else None, bt.ctypes.data if nb else None,
                                  RENUMBER[renumber], perm.ctypes.data), self._ctx, "tdg_mesh_upload")
        self.perm = perm
        self.n_elem = n
        size = ctypes.c_size_t()
        check(lib.tdg_mesh_device_bytes(self._ctx, ctypes.byref(size)), self._ctx)
        # over-allocate by 256 bytes and bind an aligned view
        raw = torch.empty(size.value + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._mesh_buf = raw
        check(lib.tdg_mesh_bind(self._ctx, ctypes.c_void_p(raw.data_ptr() + off), size.value, _stream(stream)),
              self._ctx, "tdg_mesh_bind")
        epad = ctypes.c_int64()
        check(lib.tdg_state_elems(self._ctx, ctypes.byref(epad)), self._ctx)
        self.n_elem_pad = epad.value
        return perm

    def upload(self, mesh, renumber: str = "rcm", stream=None) -> np.ndarray:
        """Upload a synthetic.TetMesh."""
        return self.upload_mesh(mesh.elem_vid, mesh.elem_xyz, mesh.bface_vid, mesh.bface_tag, renumber, stream)

    def set_flux(self, flux: str) -> None:
        """'rusanov' (default) or 'roe'."""
        check(lib.tdg_set_flux(self._ctx, {"rusanov": 0, "roe": 1}[flux]), self._ctx, "tdg_set_flux")

    def set_viscosity(self, mu: float, prandtl: float = 0.72) -> None:
        """Navier-Stokes terms (BR1) with constant viscosity; call before upload()."""
        check(lib.tdg_set_viscosity(self._ctx, float(mu), float(prandtl)), self._ctx, "tdg_set_viscosity")

    def set_farfield(self, prim) -> None:
        arr = np.ascontiguousarray(prim, dtype=np.float64)
        check(lib.tdg_set_farfield(self._ctx, arr.ctypes.data), self._ctx)

    def mesh_stats(self) -> dict:
        out = np.zeros(7, dtype=np.int64)
        check(lib.tdg_mesh_stats(self._ctx, out.ctypes.data), self._ctx)
        keys = ["n_elem", "n_elem_pad", "interior_faces", "boundary_faces", "bandwidth", "near64", "tile_tables"]
        return dict(zip(keys, out.tolist()))

    # ----------------------------------------------------------------- state
    @property
    def state_shape(self):
        """Internal layout [5][ceil(N_p/4)][n_elem_pad][4]."""
        return (5, (self.n_modes + 3) // 4, self.n_elem_pad, 4)

    def new_state(self) -> torch.Tensor:
        return torch.zeros(self.state_shape, dtype=self.state_dtype, device=self.device)

    def set_state(self, U_user: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        assert U_user.dtype == torch.float64 and U_user.is_contiguous()
        assert tuple(U_user.shape) == (self.n_elem, 5, self.n_modes)
        out = self.new_state() if out is None else out
        check(lib.tdg_set_state(self._ctx, _ptr(U_user), _ptr(out), _stream(stream)), self._ctx, "tdg_set_state")
        return out

    def get_state(self, U_int: torch.Tensor, stream=None) -> torch.Tensor:
        self._check_state(U_int)
        out = torch.empty((self.n_elem, 5, self.n_modes), dtype=torch.float64, device=self.device)
        check(lib.tdg_get_state(self._ctx, _ptr(U_int), _ptr(out), _stream(stream)), self._ctx, "tdg_get_state")
        return out

    def volume_points(self, stream=None) -> torch.Tensor:
        out = torch.empty((self.n_elem, self.n_vol_points, 3), dtype=torch.float64, device=self.device)
        check(lib.tdg_volume_points(self._ctx, _ptr(out), _stream(stream)), self._ctx, "tdg_volume_points")
        return out

    def project(self, prim: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        assert prim.dtype == torch.float64 and prim.is_contiguous()
        assert tuple(prim.shape) == (self.n_elem, self.n_vol_points, 5)
        out = self.new_state() if out is None else out
        check(lib.tdg_project(self._ctx, _ptr(prim), _ptr(out), _stream(stream)), self._ctx, "tdg_project")
        return out

    def project_fn(self, prim_fn, stream=None) -> torch.Tensor:
        """Evaluate an analytic primitive field at the volume points and project it."""
        x = self.volume_points(stream)
        return self.project(prim_fn(x).contiguous(), stream=stream)

    # ----------------------------------------------------------------- hot path
    def _check_state(self, U: torch.Tensor) -> None:
        assert U.device.type == "cuda" and U.dtype == self.state_dtype and U.is_contiguous()
        assert tuple(U.shape) == self.state_shape

    def residual(self, U: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        self._check_state(U)
        out = self.new_state() if out is None else out
        self._check_state(out)
        check(lib.tdg_residual(self._ctx, _ptr(U), _ptr(out), _stream(stream)), self._ctx, "tdg_residual")
        return out

    def new_work(self) -> torch.Tensor:
        size = ctypes.c_size_t()
        check(lib.tdg_work_bytes(self._ctx, ctypes.byref(size)), self._ctx)
        return torch.empty(size.value, dtype=torch.uint8, device=self.device)

    def rk_step(self, U: torch.Tensor, dt: float, n_steps: int = 1, work: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
        """n SSP-RK3 steps in place on U (internal layout)."""
        self._check_state(U)
        work = self.new_work() if work is None else work
        size = ctypes.c_size_t()
        check(lib.tdg_work_bytes(self._ctx, ctypes.byref(size)), self._ctx)
        assert work.is_cuda and work.numel() * work.element_size() >= size.value
        check(lib.tdg_rk_step(self._ctx, _ptr(U), _ptr(work), float(dt), int(n_steps), _stream(stream)),
              self._ctx, "tdg_rk_step")
        return U

    def rk_step_noalloc(self, U: torch.Tensor, dt: float, n_steps: int = 1, stream=None) -> torch.Tensor:
        """As rk_step, with the work buffer in the library's fixed per-GPU scratch (allocates
        nothing; meshes whose work buffer exceeds 64 MiB are refused)."""
        self._check_state(U)
        check(lib.tdg_rk_step_noalloc(self._ctx, _ptr(U), float(dt), int(n_steps), _stream(stream)), self._ctx,
              "tdg_rk_step_noalloc")
        return U

    def rk_step_adaptive(self, U: torch.Tensor, cfl: float, n_steps: int = 1, work: torch.Tensor | None = None,
                         stream=None) -> torch.Tensor:
        """n SSP-RK3 steps in place on U, each with dt = the device minimum of the local stable
        steps of the current U (no host synchronisation).  Returns the steps taken, a device
        tensor of n_steps doubles; an entry 0 marks a step whose state had an inadmissible
        cell mean (the run is invalid from there on)."""
        self._check_state(U)
        work = self.new_work() if work is None else work
        size = ctypes.c_size_t()
        check(lib.tdg_work_bytes(self._ctx, ctypes.byref(size)), self._ctx)
        assert work.is_cuda and work.numel() * work.element_size() >= size.value
        dts = torch.empty(max(1, int(n_steps)), dtype=torch.float64, device=self.device)
        check(lib.tdg_rk_step_adaptive(self._ctx, _ptr(U), _ptr(work), float(cfl), int(n_steps), _ptr(dts),
                                       _stream(stream)), self._ctx, "tdg_rk_step_adaptive")
        return dts[:n_steps]

    def residual_vjp(self, U: torch.Tensor, W: torch.Tensor, out: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
        self._check_state(U)
        self._check_state(W)
        out = self.new_state() if out is None else out
        check(lib.tdg_residual_vjp(self._ctx, _ptr(U), _ptr(W), _ptr(out), _stream(stream)), self._ctx,
              "tdg_residual_vjp")
        return out

    def rk_stage(self, U_in: torch.Tensor, U0: torch.Tensor | None, out: torch.Tensor, alpha: float, dt: float,
                 stream=None) -> torch.Tensor:
        """One SSP-RK3 stage: out = alpha U0 + (1 - alpha)(U_in + dt R(U_in))."""
        self._check_state(U_in)
        self._check_state(out)
        u0 = None if U0 is None else ctypes.c_void_p(_ptr(U0))
        check(lib.tdg_rk_stage(self._ctx, _ptr(U_in), u0, _ptr(out), float(alpha), float(dt), _stream(stream)),
              self._ctx, "tdg_rk_stage")
        return out

    def residual_vjp_axpy(self, U: torch.Tensor, W: torch.Tensor, c: float, terms, out: torch.Tensor,
                          stream=None) -> torch.Tensor:
        """out = c (dR/dU)^T W + sum a_k Y_k for terms = [(a_k, Y_k), ...] (at most three)."""
        self._check_state(U)
        self._check_state(W)
        self._check_state(out)
        n = len(terms)
        ptrs = (ctypes.c_void_p * 3)(*([_ptr(y) for _, y in terms] + [None] * (3 - n)))
        coef = (ctypes.c_double * 3)(*([float(a) for a, _ in terms] + [0.0] * (3 - n)))
        check(lib.tdg_residual_vjp_axpy(self._ctx, _ptr(U), _ptr(W), float(c), n, ptrs, coef, _ptr(out),
                                        _stream(stream)), self._ctx, "tdg_residual_vjp_axpy")
        return out

    def wall_pressure(self, U: torch.Tensor, grad: bool = False, stream=None):
        """Integrated slip-wall pressure J(U) (0-d device tensor) and, if asked, dJ/dU (internal)."""
        self._check_state(U)
        J = torch.empty((), dtype=torch.float64, device=self.device)
        g = self.new_state() if grad else None
        check(lib.tdg_wall_pressure(self._ctx, _ptr(U), _ptr(J), None if g is None else ctypes.c_void_p(_ptr(g)),
                                    _stream(stream)), self._ctx, "tdg_wall_pressure")
        return (J, g) if grad else J

    def stable_dt(self, U: torch.Tensor, cfl: float = 0.2, stream=None) -> torch.Tensor:
        """min_K cfl d_K / ((2p+1)(|u_K| + c_K)) as a 0-d device tensor."""
        self._check_state(U)
        dt = torch.empty((), dtype=torch.float64, device=self.device)
        check(lib.tdg_stable_dt(self._ctx, _ptr(U), float(cfl), _ptr(dt), _stream(stream)), self._ctx,
              "tdg_stable_dt")
        return dt

    def check_state(self, U: torch.Tensor, stream=None) -> torch.Tensor:
        """Number of elements with a non-finite value or non-positive density or pressure at a
        volume quadrature point, as a 0-d device int64 tensor."""
        self._check_state(U)
        n = torch.empty((), dtype=torch.int64, device=self.device)
        check(lib.tdg_check_state(self._ctx, _ptr(U), _ptr(n), _stream(stream)), self._ctx, "tdg_check_state")
        return n

    def sync(self, stream=None) -> None:
        check(lib.tdg_sync_check(self._ctx, _stream(stream)), self._ctx, "tdg_sync_check")


def debug_tables(p: int, which: int) -> np.ndarray:
    """Reference tables computed by the library on the host (see tdg_debug_tables)."""
    need = ctypes.c_size_t()
    check(lib.tdg_debug_tables(p, which, None, 0, ctypes.byref(need)))
    out = np.empty(need.value, dtype=np.float64)
    check(lib.tdg_debug_tables(p, which, out.ctypes.data, need.value, ctypes.byref(need)))
    return out


STREAM_KINDS = {"copy": 0, "read": 1, "write": 2, "read_cached": 3}


def stream_probe(kind: str, src: torch.Tensor | None, dst: torch.Tensor, stream=None) -> None:
    """One streaming pass (see tdg_stream_probe): "copy" src into dst (dst's bytes), "read" or
    "read_cached" all of src (dst: at least 16 bytes, may be overwritten) or "write" zeros
    over dst.  Device tensors; asynchronous on the stream."""
    def nbytes(t):
        return t.numel() * t.element_size()
    if kind == "copy" and (src is None or nbytes(src) < nbytes(dst)):
        raise ValueError("stream_probe: src must hold at least dst's bytes")
    reads = kind in ("read", "read_cached")
    if reads and (src is None or nbytes(dst) < 16):
        raise ValueError("stream_probe: read needs src and a 16-byte dst")
    n = nbytes(src) if reads else nbytes(dst)
    code = lib.tdg_stream_probe(STREAM_KINDS[kind], None if src is None else _ptr(src), _ptr(dst), n,
                                _stream(stream))
    check(code, None, f"tdg_stream_probe({kind})")
