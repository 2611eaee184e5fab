"""Jittered tetrahedral unit-cube meshes (input generator only).

The paper's test grids are unstructured gmsh tetrahedral meshes that are not
available; a structured-then-jittered tetrahedral cube stands in for them
(same element type, same data model: vertex coordinates, tetrahedra, tagged
boundary triangles).

Recipe (the same on every machine, from ``numpy.random.default_rng(seed)``):

* vertex (i, j, k), 0 <= i, j, k <= n, has id ``i + (n+1)*(j + (n+1)*k)`` and
  position ``(i, j, k) / n``;
* hexahedron (i, j, k), 0 <= i, j, k < n, with id ``i + n*(j + n*k)``, is cut
  into the 6 Kuhn tetrahedra around its main diagonal: for every permutation
  p of the axes (lexicographic order), ``v0`` = the hex corner, ``v1 = v0 +
  e[p0]``, ``v2 = v1 + e[p1]``, ``v3 = v0 + (1, 1, 1)``; the 6 tetrahedra of a
  hex are consecutive, hexes in id order;
* jitter: ``rng.uniform(-a*h, a*h, (Nv, 3))`` in vertex-id order (``h = 1/n``,
  default ``a = 0.2``), with the component normal to every boundary plane a
  vertex lies on set to zero, so the domain stays the unit cube;
* boundary triangles are the tetrahedron faces whose 3 vertices lie on one
  boundary plane, tagged 0..5 = x0, x1, y0, y1, z0, z1.
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import permutations

import numpy as np

BOUNDARY_TAGS = ("x0", "x1", "y0", "y1", "z0", "z1")


@dataclass(frozen=True)
class CubeMesh:
    """Raw mesh as a mesh file would give it (user numbering)."""
    n: int
    seed: int
    xyz: np.ndarray     # float64 [Nv, 3]
    tets: np.ndarray    # int32   [Nc, 4]
    btris: np.ndarray   # int32   [Nb, 3]
    btags: np.ndarray   # int32   [Nb]

    @property
    def nv(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nc(self) -> int:
        return int(self.tets.shape[0])

    @property
    def nb(self) -> int:
        return int(self.btris.shape[0])


def _lattice_tets(n: int) -> np.ndarray:
    """Kuhn split of the n^3 hexes, returned as lattice coords [Nc, 4, 3]."""
    hk, hj, hi = np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                             indexing="ij")
    corner = np.stack([hi.ravel(), hj.ravel(), hk.ravel()], axis=1)  # hex id order
    eye = np.eye(3, dtype=np.int64)
    per_hex = []
    for p in permutations(range(3)):
        v0 = np.zeros(3, np.int64)
        v1 = v0 + eye[p[0]]
        v2 = v1 + eye[p[1]]
        v3 = np.ones(3, np.int64)
        per_hex.append(np.stack([v0, v1, v2, v3]))
    per_hex = np.stack(per_hex)                          # [6, 4, 3]
    return (corner[:, None, None, :] + per_hex[None]).reshape(-1, 4, 3)


def jittered_cube(n: int, seed: int, jitter: float = 0.2) -> CubeMesh:
    if n < 1:
        raise ValueError("n must be >= 1")
    n1 = n + 1
    lat = _lattice_tets(n)                               # [Nc, 4, 3]
    vid = lat[..., 0] + n1 * (lat[..., 1] + n1 * lat[..., 2])
    tets = vid.astype(np.int32)

    kk, jj, ii = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1),
                             indexing="ij")
    ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)  # id order
    h = 1.0 / n
    rng = np.random.default_rng(seed)
    delta = rng.uniform(-jitter * h, jitter * h, (ijk.shape[0], 3))
    on_boundary = (ijk == 0) | (ijk == n)
    delta[on_boundary] = 0.0
    xyz = ijk.astype(np.float64) / n + delta

    # boundary triangles: faces (vertex triples) of each tet lying on a plane
    face_local = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    tris, tags = [], []
    for fl in face_local:
        flat = lat[:, fl, :]                             # [Nc, 3, 3]
        fv = tets[:, fl]
        for axis in range(3):
            for side, val in ((0, 0), (1, n)):
                hit = np.all(flat[:, :, axis] == val, axis=1)
                if hit.any():
                    tris.append(fv[hit])
                    tags.append(np.full(int(hit.sum()), 2 * axis + side,
                                        np.int32))
    btris = np.concatenate(tris).astype(np.int32)
    btags = np.concatenate(tags).astype(np.int32)
    order = np.lexsort((btris[:, 2], btris[:, 1], btris[:, 0], btags))
    return CubeMesh(n=n, seed=seed, xyz=xyz, tets=tets,
                    btris=np.ascontiguousarray(btris[order]),
                    btags=np.ascontiguousarray(btags[order]))
