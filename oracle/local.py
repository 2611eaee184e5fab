"""The oracle's residual and matrix rows for a sample of cells of a large
mesh (test infrastructure only).

The residual of eq. (4) at cell i depends on data within two vertex rings
of i: the face fluxes of i need the gradients and limiters of i and its face
neighbours (Algorithm 1 over their node-neighbour stencils, Barth-Jespersen
over their face neighbours) and the least-squares values (Algorithm 2) at
i's vertices.  Every cell sharing a vertex with a cell that shares a vertex
with i is therefore included in a submesh, which the global oracle functions
evaluate unchanged.  A face of the submesh that is interior in the full mesh
but has only one submesh cell (a cut) cannot contain a vertex of i or of a
face neighbour of i - the cell behind it would then share that vertex and be
in the submesh - so the cut faces (given a tag of their own) influence
nothing that is read.  Cells keep their relative user order, so L/R
orientations are those of the full mesh.
"""
from __future__ import annotations

import numpy as np

from .geometry import build_geometry
from . import fv, poisson

CUT_TAG = 31


class VertexIndex:
    """vertex -> cells incidence of the full mesh (CSR)."""

    def __init__(self, tets, nv):
        tets = np.asarray(tets, np.int64)
        v = tets.ravel()
        c = np.repeat(np.arange(len(tets)), 4)
        order = np.argsort(v, kind="stable")
        self.cells = c[order]
        self.ptr = np.zeros(nv + 1, np.int64)
        self.ptr[1:] = np.cumsum(np.bincount(v, minlength=nv))
        self.tets = tets

    def ring(self, cells):
        """Cells sharing a vertex with any of `cells` (sorted, unique)."""
        verts = np.unique(self.tets[np.asarray(cells)].ravel())
        parts = [self.cells[self.ptr[a]:self.ptr[a + 1]] for a in verts]
        return np.unique(np.concatenate(parts))


def submesh(mesh, vidx: VertexIndex, cell, rings=2):
    """`rings`-vertex-ring submesh around `cell`: (xyz, tets, btris, btags,
    cells) with cells = the original ids in increasing order."""
    cells = [cell]
    for _ in range(rings):
        cells = vidx.ring(cells)
    tets = vidx.tets[cells]
    verts, inv = np.unique(tets.ravel(), return_inverse=True)
    sub_tets = inv.reshape(-1, 4).astype(np.int32)
    xyz = mesh.xyz[verts]
    # true boundary triangles of the submesh cells, plus cut faces
    opp = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    tri = np.sort(sub_tets[:, opp].reshape(-1, 3), axis=1)
    key, cnt = np.unique(tri, axis=0, return_counts=True)
    single = key[cnt == 1]
    glob = np.sort(verts[single], axis=1)
    btri_sorted = np.sort(np.asarray(mesh.btris, np.int64), axis=1)
    m = int(max(glob.max(), btri_sorted.max())) + 1
    gk = (glob[:, 0] * m + glob[:, 1]) * m + glob[:, 2]
    bk = (btri_sorted[:, 0] * m + btri_sorted[:, 1]) * m + btri_sorted[:, 2]
    order = np.argsort(bk)
    pos = np.searchsorted(bk[order], gk)
    pos = np.minimum(pos, len(bk) - 1)
    hit = bk[order][pos] == gk
    tags = np.where(hit, np.asarray(mesh.btags)[order][pos], CUT_TAG).astype(np.int32)
    return xyz, sub_tets, single.astype(np.int32), tags, cells


def residual_at(mesh, vidx, cells, u, vel, D, kinds, values):
    """Res(u)_i of eq. (4) for each i in `cells` (full-mesh user order
    arrays u [Nc], vel [Nc,3]; kinds/values per tag)."""
    kinds = list(kinds) + [0] * (CUT_TAG + 1 - len(kinds))
    values = list(values) + [0.0] * (CUT_TAG + 1 - len(values))
    out = np.empty(len(cells))
    for k, c in enumerate(cells):
        xyz, tets, btris, btags, ids = submesh(mesh, vidx, c)
        geo = build_geometry(xyz, tets, btris, btags)
        phi = fv.face_velocity_flux(geo, vel[ids])
        res = fv.residual(geo, u[ids], phi, D, kinds, values)
        out[k] = res[np.searchsorted(ids, c)]
    return out


def matrix_rows_times(mesh, vidx, cells, x, kinds, values):
    """(K x)_i and c_i for each i in `cells` (eq. (laplace) rows)."""
    kinds = list(kinds) + [0] * (CUT_TAG + 1 - len(kinds))
    values = list(values) + [0.0] * (CUT_TAG + 1 - len(values))
    kx = np.empty(len(cells))
    cc = np.empty(len(cells))
    for k, c in enumerate(cells):
        xyz, tets, btris, btags, ids = submesh(mesh, vidx, c)
        geo = build_geometry(xyz, tets, btris, btags)
        K, cvec = poisson.assemble(geo, kinds, values)
        j = np.searchsorted(ids, c)
        kx[k] = float((K[j] @ x[ids])[0])
        cc[k] = cvec[j]
    return kx, cc


def step_at(mesh, vidx, cells, u, vel, D, kinds, values, dt):
    """u after one step of eq. (6) at each i in `cells`.  The three stages
    each read the residual, which reaches two vertex rings; the stage-k value
    at a cell therefore depends on the data within 2k rings of it, and the
    step at i on the six-ring submesh, whose cut faces lie outside what is
    read (as for the residual above)."""
    kinds = list(kinds) + [0] * (CUT_TAG + 1 - len(kinds))
    values = list(values) + [0.0] * (CUT_TAG + 1 - len(values))
    out = np.empty(len(cells))
    for k, c in enumerate(cells):
        xyz, tets, btris, btags, ids = submesh(mesh, vidx, c, rings=6)
        geo = build_geometry(xyz, tets, btris, btags)
        phi = fv.face_velocity_flux(geo, vel[ids])
        un = fv.rk3_step(geo, u[ids], dt, phi, D, kinds, values)
        out[k] = un[np.searchsorted(ids, c)]
    return out
