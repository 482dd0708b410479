"""Kuhn (Freudenthal) cube-split tetrahedral meshes.

An n^3 grid of hexahedra on [0, L]^3 is split into 6 tetrahedra per hexahedron:
for each permutation (a, b, c) of the axes the tet is the monotone lattice
path v, v+e_a, v+e_a+e_b, v+(1,1,1).  The split is conforming and translation
invariant, so the same construction works on a torus.

Vertex ids are "torus" ids: along a periodic axis the lattice index is taken
modulo n, so the two copies of a periodic vertex share one id.  Coordinates are
stored per element *unwrapped* (the true position of that element's corner),
so every element is a plain affine tet and periodic neighbours differ by a
period shift.

Optional perturbations: uniform vertex jitter of +-jitter*h per coordinate
(keyed by vertex id, so shared vertices move together; the component normal to
a non-periodic boundary plane is not jittered), a Gaussian bump mapped into the
y=0 face, a random permutation of the element order and a random relabelling
of the vertex ids.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

# boundary tags understood by the solver
BC_FARFIELD = 1
BC_SLIPWALL = 2


@dataclass
class TetMesh:
    elem_vid: np.ndarray          # (E, 4) int64 vertex ids
    elem_xyz: np.ndarray          # (E, 4, 3) float64 unwrapped coordinates
    bface_vid: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), np.int64))
    bface_tag: np.ndarray = field(default_factory=lambda: np.zeros((0,), np.int32))
    n: tuple = (0, 0, 0)
    length: tuple = (1.0, 1.0, 1.0)
    periodic: tuple = (True, True, True)

    @property
    def n_elem(self) -> int:
        return int(self.elem_vid.shape[0])

    @property
    def h(self) -> float:
        """Smallest hexahedron edge."""
        return min(l / k for l, k in zip(self.length, self.n))


def kuhn_cube(n, length=1.0, periodic=(True, True, True),
              jitter: float = 0.0, jitter_seed: int = 1877,
              shuffle_seed: int | None = None, vid_seed: int | None = None,
              bump_height: float = 0.0, bump_width: float = 0.1,
              wall_tags: dict | None = None) -> TetMesh:
    """Build an n^3 x 6 Kuhn-split tet mesh of the box [0, length]^3.

    n, length    an int/float or a per-axis triple (anisotropic box grid).

    periodic     per-axis periodicity (x, y, z).
    jitter       vertex perturbation amplitude as a fraction of h = length/n.
    bump_height  Gaussian bump y <- y + H exp(-((x-L/2)/(w L))^2) (1 - y/L).
    wall_tags    boundary tag per non-periodic plane, keys ('x',0) ('x',1) ...;
                 default farfield everywhere except a slip wall on y=0.
    """
    periodic = tuple(bool(p) for p in periodic)
    ns = tuple(int(v) for v in (n if np.ndim(n) else (n, n, n)))
    ls = tuple(float(v) for v in (length if np.ndim(length) else (length, length, length)))
    hs = np.array([l / k for l, k in zip(ls, ns)])
    nv = [ns[a] if periodic[a] else ns[a] + 1 for a in range(3)]   # distinct vertex indices per axis

    # lattice corners of each hex
    ii, jj, kk = np.meshgrid(np.arange(ns[0]), np.arange(ns[1]), np.arange(ns[2]), indexing="ij")
    base = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)   # (n^3, 3), x slowest
    unit = np.eye(3, dtype=np.int64)
    tets = []
    for perm in itertools.permutations(range(3)):
        v0 = base
        v1 = v0 + unit[perm[0]]
        v2 = v1 + unit[perm[1]]
        v3 = v2 + unit[perm[2]]
        tets.append(np.stack([v0, v1, v2, v3], axis=1))            # (n^3, 4, 3)
    lat = np.stack(tets, axis=1).reshape(-1, 4, 3)                 # (6 n^3, 4, 3) hex-major

    def vid_of(l):
        idx = [l[..., a] % ns[a] if periodic[a] else l[..., a] for a in range(3)]
        return (idx[0] * nv[1] + idx[1]) * nv[2] + idx[2]

    elem_vid = vid_of(lat).astype(np.int64)
    n_vert = nv[0] * nv[1] * nv[2]
    xyz = lat.astype(np.float64) * hs

    if jitter > 0.0:
        rng = np.random.default_rng(jitter_seed)
        delta = rng.uniform(-1.0, 1.0, size=(n_vert, 3)) * (jitter * hs)
        # keep vertices of non-periodic boundary planes on their plane
        vi = np.arange(n_vert)
        idx = [vi // (nv[1] * nv[2]), (vi // nv[2]) % nv[1], vi % nv[2]]
        for a in range(3):
            if not periodic[a]:
                on_plane = (idx[a] == 0) | (idx[a] == ns[a])
                delta[on_plane, a] = 0.0
        xyz = xyz + delta[elem_vid]

    if bump_height != 0.0:
        x = xyz[..., 0]
        y = xyz[..., 1]
        xyz[..., 1] = y + bump_height * np.exp(-((x - 0.5 * ls[0]) / (bump_width * ls[0])) ** 2) * (1.0 - y / ls[1])

    # boundary faces: tet faces whose three lattice corners lie on one non-periodic plane
    bf_vid, bf_tag = [], []
    if not all(periodic):
        if wall_tags is None:
            wall_tags = {}
        for f in range(4):
            keep = [a for a in range(4) if a != f]
            tri = lat[:, keep, :]                                   # (E, 3, 3)
            for a in range(3):
                if periodic[a]:
                    continue
                for side, val in ((0, 0), (1, ns[a])):
                    on = np.all(tri[:, :, a] == val, axis=1)
                    if not np.any(on):
                        continue
                    tag = wall_tags.get(("xyz"[a], side),
                                        BC_SLIPWALL if (a == 1 and side == 0) else BC_FARFIELD)
                    bf_vid.append(elem_vid[on][:, keep])
                    bf_tag.append(np.full(int(on.sum()), tag, np.int32))
    bface_vid = np.concatenate(bf_vid, 0) if bf_vid else np.zeros((0, 3), np.int64)
    bface_tag = np.concatenate(bf_tag, 0) if bf_tag else np.zeros((0,), np.int32)

    if vid_seed is not None:
        relabel = np.random.default_rng(vid_seed).permutation(n_vert).astype(np.int64)
        elem_vid = relabel[elem_vid]
        bface_vid = relabel[bface_vid]
    if shuffle_seed is not None:
        order = np.random.default_rng(shuffle_seed).permutation(elem_vid.shape[0])
        elem_vid = elem_vid[order]
        xyz = xyz[order]

    return TetMesh(elem_vid=np.ascontiguousarray(elem_vid), elem_xyz=np.ascontiguousarray(xyz),
                   bface_vid=np.ascontiguousarray(bface_vid), bface_tag=bface_tag,
                   n=ns, length=ls, periodic=periodic)
