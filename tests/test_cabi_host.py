"""Host-side checks of libtetdg.so (no GPU): the library loads and exports every
symbol of include/tetdg.h; its reference tables agree with the oracle's independent
ones; mesh upload validates input and renumbers; argument errors map to status codes.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import basis, quadrature
from oracle.geometry import build_faces, build_geometry
from synthetic import kuhn_cube
from test_oracle_golden import smallest_table1_reduction

pytest.importorskip("paper_2209_01877_amd._lib", reason="libtetdg.so not built")
from paper_2209_01877_amd import _lib  # noqa: E402
from paper_2209_01877_amd.solver import RENUMBER, debug_tables  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "tetdg.h")).read()
    names = sorted(set(re.findall(r"\b(tdg_[a-z_0-9]+)\s*\(", header)))
    assert len(names) >= 15
    for n in names:
        assert hasattr(_lib.lib, n), n


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_tables_match_oracle(p):
    ox, ow = quadrature.tet_rule(p + 1)
    st, sw = quadrature.triangle_rule(p + 1)
    nq, nf = len(ow), len(sw)
    assert np.abs(debug_tables(p, 0).reshape(nq, 3) - ox).max() < 1e-15
    assert np.abs(debug_tables(p, 1) - ow).max() < 4e-16
    assert np.abs(debug_tables(p, 2).reshape(nf, 2) - st).max() < 1e-15
    assert np.abs(debug_tables(p, 3) - sw).max() < 4e-16
    B = debug_tables(p, 4).reshape(nq, -1)
    G = debug_tables(p, 5).reshape(3, nq, -1)
    Bf = debug_tables(p, 6).reshape(4, nf, -1)
    scale = 10.0 ** p
    assert np.abs(B - basis.eval_basis(p, ox)).max() < 1e-14 * scale
    assert np.abs(G - basis.eval_basis_grad(p, ox)).max() < 1e-13 * scale
    ref_f = np.stack([basis.eval_basis(p, basis.face_map(f, st)) for f in range(4)])
    assert np.abs(Bf - ref_f).max() < 1e-14 * scale


def _ctx(p=2, prec=0):
    ctx = ctypes.c_void_p()
    assert _lib.lib.tdg_create(p, prec, 1.4, ctypes.byref(ctx)) == 0
    return ctx


def _upload(ctx, mesh, renumber=0, perm=None):
    vid = np.ascontiguousarray(mesh.elem_vid, np.int64)
    xyz = np.ascontiguousarray(mesh.elem_xyz, np.float64)
    nb = len(mesh.bface_vid)
    bv = np.ascontiguousarray(mesh.bface_vid, np.int64)
    bt = np.ascontiguousarray(mesh.bface_tag, np.int32)
    return _lib.lib.tdg_mesh_upload(ctx, vid.shape[0], vid.ctypes.data, xyz.ctypes.data, nb,
                                    bv.ctypes.data if nb else None, bt.ctypes.data if nb else None, renumber,
                                    perm.ctypes.data if perm is not None else None)


def _stats(ctx):
    out = np.zeros(7, np.int64)
    assert _lib.lib.tdg_mesh_stats(ctx, out.ctypes.data) == 0
    return out


def test_create_argument_errors():
    ctx = ctypes.c_void_p()
    assert _lib.lib.tdg_create(0, 0, 1.4, ctypes.byref(ctx)) == -1
    assert _lib.lib.tdg_create(5, 0, 1.4, ctypes.byref(ctx)) == -1
    assert _lib.lib.tdg_create(2, 7, 1.4, ctypes.byref(ctx)) == -1
    assert _lib.lib.tdg_create(2, 0, 1.0, ctypes.byref(ctx)) == -1
    assert _lib.lib.tdg_create(2, 0, 1.4, None) == -1


def test_calls_out_of_order():
    ctx = _ctx()
    size = ctypes.c_size_t()
    assert _lib.lib.tdg_mesh_device_bytes(ctx, ctypes.byref(size)) == -3
    assert _lib.lib.tdg_residual(ctx, None, None, None) == -3
    _lib.lib.tdg_destroy(ctx)


def test_mesh_counts_and_faces():
    m = kuhn_cube(4, jitter=0.2, shuffle_seed=3)
    ctx = _ctx()
    assert _upload(ctx, m) == 0
    st = _stats(ctx)
    assert st[0] == 384 and st[1] == 384 and st[2] == 2 * 384 and st[3] == 0
    m = kuhn_cube(4, periodic=(False, False, True), jitter=0.2, bump_height=0.05)
    assert _upload(ctx, m) == 0
    g = build_geometry(m.elem_vid, m.elem_xyz)
    f = build_faces(g.vid, m.bface_vid, m.bface_tag)
    st = _stats(ctx)
    assert st[2] == int((f.ep >= 0).sum()) and st[3] == int((f.ep < 0).sum())
    _lib.lib.tdg_destroy(ctx)


def test_mesh_errors():
    ctx = _ctx()
    m = kuhn_cube(3)
    # zero-volume element
    bad = m.elem_xyz.copy()
    bad[5, 3] = bad[5, 0] + 0.5 * (bad[5, 1] - bad[5, 0]) + 0.5 * (bad[5, 2] - bad[5, 0])
    assert _lib.lib.tdg_mesh_upload(ctx, m.n_elem, np.ascontiguousarray(m.elem_vid).ctypes.data,
                                    np.ascontiguousarray(bad).ctypes.data, 0, None, None, 0, None) == -2
    assert b"volume" in _lib.lib.tdg_last_error(ctx)
    # unmatched faces: drop an element from a periodic mesh
    vid = np.ascontiguousarray(m.elem_vid[1:])
    xyz = np.ascontiguousarray(m.elem_xyz[1:])
    assert _lib.lib.tdg_mesh_upload(ctx, vid.shape[0], vid.ctypes.data, xyz.ctypes.data, 0, None, None, 0, None) == -2
    assert b"unmatched" in _lib.lib.tdg_last_error(ctx)
    # a face shared by three elements: duplicate an element
    vid = np.ascontiguousarray(np.concatenate([m.elem_vid, m.elem_vid[:1]]))
    xyz = np.ascontiguousarray(np.concatenate([m.elem_xyz, m.elem_xyz[:1]]))
    assert _lib.lib.tdg_mesh_upload(ctx, vid.shape[0], vid.ctypes.data, xyz.ctypes.data, 0, None, None, 0, None) == -2
    # bad renumbering mode
    assert _upload(ctx, m, renumber=9) == -1
    _lib.lib.tdg_destroy(ctx)


def test_viscosity_arguments():
    ctx = _ctx()
    assert _lib.lib.tdg_set_viscosity(ctx, -1.0, 0.72) == -1
    assert _lib.lib.tdg_set_viscosity(ctx, 0.01, 0.0) == -1
    assert _lib.lib.tdg_set_viscosity(ctx, 0.01, 0.72) == 0
    assert _upload(ctx, kuhn_cube(3)) == 0
    assert _lib.lib.tdg_set_viscosity(ctx, 0.02, 0.72) == -3  # after the upload
    _lib.lib.tdg_destroy(ctx)
    ctx = _ctx(prec=2)
    assert _lib.lib.tdg_set_viscosity(ctx, 0.01, 0.72) == -5  # mixed modes
    assert _lib.lib.tdg_set_viscosity(ctx, 0.0, 0.72) == 0
    _lib.lib.tdg_destroy(ctx)


def test_mesh_size_limits():
    """An empty mesh and an element count past the kernels' 32-bit element indexing are
    rejected before any array is read."""
    ctx = _ctx()
    one = np.zeros((1, 4), np.int64)
    xyz = np.zeros((1, 4, 3))
    assert _lib.lib.tdg_mesh_upload(ctx, 0, one.ctypes.data, xyz.ctypes.data, 0, None, None, 0, None) == -1
    assert b"n_elem" in _lib.lib.tdg_last_error(ctx)
    assert _lib.lib.tdg_mesh_upload(ctx, 1 << 31, one.ctypes.data, xyz.ctypes.data, 0, None, None, 0, None) == -1
    _lib.lib.tdg_destroy(ctx)


def test_single_element_mesh():
    """One tetrahedron with all four faces on the boundary uploads as a valid mesh (one real
    element in a padded tile, four boundary faces, no interior face)."""
    ctx = _ctx()
    xyz = np.array([[[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]])
    vid = np.array([[0, 1, 2, 3]], np.int64)
    bv = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]], np.int64)
    bt = np.array([1, 2, 1, 1], np.int32)
    assert _lib.lib.tdg_mesh_upload(ctx, 1, vid.ctypes.data, np.ascontiguousarray(xyz).ctypes.data, 4,
                                    bv.ctypes.data, bt.ctypes.data, 1, None) == 0
    st = _stats(ctx)
    assert st[0] == 1 and st[1] % 64 == 0 and st[2] == 0 and st[3] == 4
    _lib.lib.tdg_destroy(ctx)


@pytest.mark.parametrize("mode", ["none", "rcm", "morton", "hilbert"])
def test_permutation_is_valid(mode):
    m = kuhn_cube(6, shuffle_seed=2209, vid_seed=2210)
    ctx = _ctx()
    perm = np.empty(m.n_elem, np.int64)
    assert _upload(ctx, m, RENUMBER[mode], perm) == 0
    assert np.array_equal(np.sort(perm), np.arange(m.n_elem))
    if mode == "none":
        assert np.array_equal(perm, np.arange(m.n_elem))
    _lib.lib.tdg_destroy(ctx)


def test_renumbering_reduces_bandwidth():
    """Table 1 of the paper reports RCM cutting the adjacency bandwidth by one to two orders of
    magnitude (smallest reduction 1427 -> 69, about 20x).  The shuffled 24^3 x 6 mesh must get at
    least that factor from RCM, and the space-filling curves must keep most neighbours close."""
    m = kuhn_cube(24, shuffle_seed=2209, vid_seed=2210)
    ctx = _ctx(1, prec=2)  # mixed mode: plain orders
    out = {}
    for mode in ["none", "rcm", "morton", "hilbert"]:
        assert _upload(ctx, m, RENUMBER[mode]) == 0
        out[mode] = _stats(ctx)
    pairs = 4 * m.n_elem
    table1 = smallest_table1_reduction()  # 1427 -> 69 in the paper's Table 1
    assert out["none"][4] / out["rcm"][4] >= table1
    assert out["morton"][5] > 0.5 * pairs and out["hilbert"][5] > 0.5 * pairs
    assert out["none"][5] < 0.01 * pairs
    _lib.lib.tdg_destroy(ctx)
    # fp64 mode: RCM keeps the bandwidth reduction after the face-code grouping, and the
    # grouping lowers the number of neighbour face tables per tile
    ctx = _ctx(1, prec=0)
    assert _upload(ctx, m, RENUMBER["rcm"]) == 0
    assert out["none"][4] / _stats(ctx)[4] >= table1
    assert _upload(ctx, m, RENUMBER["hilbert"]) == 0
    grouped = _stats(ctx)
    assert grouped[6] < 0.75 * out["hilbert"][6]
    _lib.lib.tdg_destroy(ctx)


def test_stream_probe_argument_errors():
    """The streaming probe rejects bad arguments before any device call (no GPU needed)."""
    f = _lib.lib.tdg_stream_probe
    buf = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation
    odd = ctypes.c_void_p(0x1008)
    assert f(4, buf, buf, 1024, None) == -1  # unknown kind
    assert f(-1, buf, buf, 1024, None) == -1
    assert f(0, buf, buf, 0, None) == -1  # empty
    assert f(0, buf, buf, 1000, None) == -1  # not a multiple of 16 bytes
    assert f(0, None, buf, 1024, None) == -1  # copy without a source
    assert f(1, None, buf, 1024, None) == -1  # read without a source
    assert f(3, None, buf, 1024, None) == -1
    assert f(2, None, None, 1024, None) == -1  # write without a destination
    assert f(0, odd, buf, 1024, None) == -1  # misaligned
    assert f(2, None, odd, 1024, None) == -1
