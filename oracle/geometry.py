"""Element geometry and face-centric topology for affine tetrahedra.

Reading (the paper's code is 2-D and does not describe it): each tet lists its
vertices in ascending global vertex id, x = X0 + J xi with J = [X1-X0 | X2-X0 |
X3-X0].  Two tets sharing a face then list that face's three vertices in the same
order, so the face parameter (s, t) names the same physical point from both sides
(up to a period shift on a torus) and no orientation table is needed.

Face area vectors are taken directly from the physical corners: half the cross
product of two edges of the face, turned to point away from the opposite vertex.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Geometry:
    xyz: np.ndarray        # (E, 4, 3) corners in ascending-id order
    vid: np.ndarray        # (E, 4) sorted vertex ids
    jac: np.ndarray        # (E, 3, 3) J
    jinv: np.ndarray       # (E, 3, 3) J^-1
    absdet: np.ndarray     # (E,) |det J|
    volume: np.ndarray     # (E,) |K| = |det J| / 6
    area_vec: np.ndarray   # (E, 4, 3) outward area vector A_f n_f of local face f
    area: np.ndarray       # (E, 4) A_f
    normal: np.ndarray     # (E, 4, 3) unit outward normal


@dataclass
class Faces:
    """Unique faces.  Side m ("minus") is the element with the lower index."""
    em: np.ndarray         # (F,) element on side m
    fm: np.ndarray         # (F,) its local face
    ep: np.ndarray         # (F,) element on side p, -1 on a boundary face
    fp: np.ndarray         # (F,) its local face, -1 on a boundary face
    tag: np.ndarray        # (F,) boundary tag (0 interior)


def sort_vertices(elem_vid: np.ndarray, elem_xyz: np.ndarray):
    order = np.argsort(elem_vid, axis=1, kind="stable")
    vid = np.take_along_axis(elem_vid, order, axis=1)
    xyz = np.take_along_axis(elem_xyz, order[:, :, None], axis=1)
    return vid, xyz


def build_geometry(elem_vid: np.ndarray, elem_xyz: np.ndarray) -> Geometry:
    vid, xyz = sort_vertices(np.asarray(elem_vid, np.int64), np.asarray(elem_xyz, np.float64))
    jac = np.stack([xyz[:, 1] - xyz[:, 0], xyz[:, 2] - xyz[:, 0], xyz[:, 3] - xyz[:, 0]], axis=2)
    det = np.linalg.det(jac)
    if np.any(np.abs(det) <= 0.0):
        raise ValueError("degenerate element")
    jinv = np.linalg.inv(jac)
    area_vec = np.zeros((xyz.shape[0], 4, 3))
    for f in range(4):
        a, b, c = [v for v in range(4) if v != f]
        vec = 0.5 * np.cross(xyz[:, b] - xyz[:, a], xyz[:, c] - xyz[:, a])
        away = np.einsum("ed,ed->e", vec, xyz[:, a] - xyz[:, f])
        area_vec[:, f] = vec * np.sign(away)[:, None]
    area = np.linalg.norm(area_vec, axis=2)
    return Geometry(xyz=xyz, vid=vid, jac=jac, jinv=jinv, absdet=np.abs(det), volume=np.abs(det) / 6.0,
                    area_vec=area_vec, area=area, normal=area_vec / area[:, :, None])


def build_faces(sorted_vid: np.ndarray, bface_vid=None, bface_tag=None) -> Faces:
    """Match tet faces by their sorted vertex-id triple (face-centric list).

    All 4E (element, local face) slots are sorted by their key; equal neighbouring
    keys are the two sides of an interior face, a key seen once must be a listed
    boundary face, a key seen more than twice is an error.
    """
    E = sorted_vid.shape[0]
    keys = np.concatenate([sorted_vid[:, [v for v in range(4) if v != f]] for f in range(4)])
    slot_e = np.tile(np.arange(E), 4)
    slot_f = np.repeat(np.arange(4), E)
    order = np.lexsort((slot_e, keys[:, 2], keys[:, 1], keys[:, 0]))
    k = keys[order]
    new = np.ones(len(k), bool)
    new[1:] = np.any(k[1:] != k[:-1], axis=1)
    start = np.flatnonzero(new)
    count = np.diff(np.append(start, len(k)))
    if np.any(count > 2):
        bad = k[start[np.argmax(count > 2)]]
        raise ValueError(f"face {tuple(bad)} shared by more than two elements")
    two = start[count == 2]
    one = start[count == 1]
    em = slot_e[order[two]]; fm = slot_f[order[two]]
    ep = slot_e[order[two + 1]]; fp = slot_f[order[two + 1]]
    tags = np.zeros(len(two), np.int64)
    if len(one):
        if bface_vid is None or len(bface_vid) == 0:
            raise ValueError("unmatched face without boundary tag")
        bkey = np.sort(np.asarray(bface_vid, np.int64), axis=1)
        lookup = {tuple(r): int(t) for r, t in zip(bkey.tolist(), np.asarray(bface_tag).tolist())}
        btags = []
        for r in k[one].tolist():
            if tuple(r) not in lookup:
                raise ValueError(f"unmatched face {tuple(r)} without boundary tag")
            btags.append(lookup[tuple(r)])
        em = np.concatenate([em, slot_e[order[one]]]); fm = np.concatenate([fm, slot_f[order[one]]])
        ep = np.concatenate([ep, -np.ones(len(one), np.int64)]); fp = np.concatenate([fp, -np.ones(len(one), np.int64)])
        tags = np.concatenate([tags, np.array(btags, np.int64)])
    return Faces(em=em, fm=fm, ep=ep, fp=fp, tag=tags)
