"""Mesh geometry for the cell-centred scheme (oracle; test infrastructure only).

Follows Sec. 2.1 of the paper (data at cell centres of gravity, fluxes on
faces with unit normal n_ij and area |sigma_ij|, ghost cells at the boundary,
cell gradients over the cells sharing a vertex - Algorithm 1 - and
least-squares node values - Algorithm 2), plus the diamond cell of
eq. (diamond) with a triangular base (D = C).

Readings where the paper is silent:
* cell centre = mean of the 4 vertices; face "midpoint" = mean of its 3;
* the ghost of a boundary face sits at the mirror image of its owner's centre
  across the face plane;
* the node-neighbour stencil of cell i is every other cell sharing a vertex
  with i, plus the ghost of every boundary face sharing a vertex with i
  (halo/haloghost cells of Algorithm 1 do not exist on one undivided mesh);
* node weights are those of the unweighted least-squares linear fit (with
  intercept) through the cells and ghosts around the node, evaluated at the
  node;
* an interior face's L cell is the owner with the smaller user index, and
  the face vector S_f points from L to R (to the ghost on the boundary).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# boundary-condition kinds (per tag)
ZERO_FLUX, NEUMANN, DIRICHLET = 0, 1, 2


class MeshError(ValueError):
    pass


@dataclass
class Geometry:
    nc: int
    nv: int
    nf: int
    nb: int
    tets: np.ndarray        # [Nc,4] positively oriented
    xyz: np.ndarray         # [Nv,3]
    vol: np.ndarray         # [Nc]
    xc: np.ndarray          # [Nc+Nb,3] cell centres then ghost centres
    # faces
    fL: np.ndarray          # [Nf]
    fR: np.ndarray          # [Nf] cell index, or Nc+g for boundary face of ghost g
    fabc: np.ndarray        # [Nf,3] vertex labels A,B,C with S = 1/2 (B-A)x(C-A)
    fS: np.ndarray          # [Nf,3] face vector (unit normal * area), L -> R
    fx: np.ndarray          # [Nf,3] face centroid
    fghost: np.ndarray      # [Nf] ghost index or -1
    ftag: np.ndarray        # [Nf] boundary tag or -1
    kAC: np.ndarray         # [Nf] diamond coefficients (flux = S . grad)
    kBC: np.ndarray
    kRL: np.ndarray
    # ghosts
    gface: np.ndarray       # [Nb] face of ghost g
    gowner: np.ndarray      # [Nb] owner cell (the face's L)
    gtag: np.ndarray        # [Nb]
    gdist: np.ndarray       # [Nb] |x_g - x_L|
    # cell -> faces
    cfaces: np.ndarray      # [Nc,4] faces of each cell
    csign: np.ndarray       # [Nc,4] +1 if the cell is L of that face, -1 if R
    # node-neighbour stencil (CSR over cells; entries are cells or Nc+g)
    sptr: np.ndarray
    sidx: np.ndarray
    # node -> cells/ghosts with least-squares weights (CSR over vertices)
    nptr: np.ndarray
    nidx: np.ndarray
    nalpha: np.ndarray
    # ghost g -> index of its triangle in the boundary triangles given
    gbtri: np.ndarray = None


def _cross(a, b):
    return np.cross(a, b)


def _dot(a, b):
    return np.einsum("...i,...i->...", a, b)


def _csr_from_pairs(rows, cols, nrows):
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    ptr = np.zeros(nrows + 1, np.int64)
    ptr[1:] = np.cumsum(np.bincount(rows, minlength=nrows))
    return ptr, cols


def build_geometry(xyz, tets, btris, btags) -> Geometry:
    xyz = np.asarray(xyz, np.float64)
    tets = np.array(tets, np.int64)
    btris = np.asarray(btris, np.int64)
    btags = np.asarray(btags, np.int64)
    nc, nv, nb_in = len(tets), len(xyz), len(btris)

    # -- cells: orientation, volume mu_i, centre of gravity ------------------
    p = xyz[tets]
    det = _dot(p[:, 1] - p[:, 0], _cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]))
    neg = det < 0
    tets[neg] = tets[neg][:, [0, 1, 3, 2]]
    vol = np.abs(det) / 6.0
    if np.any(vol <= 1e-14 * vol.mean()):
        raise MeshError("degenerate tetrahedron")
    xcell = xyz[tets].mean(axis=1)

    # -- faces: sorted vertex triples; 2 owners = interior, 1 = boundary -----
    opposite = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    tri = np.sort(tets[:, opposite].reshape(-1, 3), axis=1)   # [4Nc,3]
    owner = np.repeat(np.arange(nc), 4)
    keys, inv, cnt = np.unique(tri, axis=0, return_inverse=True,
                               return_counts=True)
    inv = inv.ravel()
    if np.any(cnt > 2):
        raise MeshError("non-manifold face")
    nf = len(keys)
    # owners per face, sorted by user index -> L = smaller
    order = np.lexsort((owner, inv))
    f_sorted, o_sorted = inv[order], owner[order]
    first = np.searchsorted(f_sorted, np.arange(nf), side="left")
    fL = o_sorted[first]
    fR = np.where(cnt == 2, o_sorted[np.minimum(first + 1, len(o_sorted) - 1)], -1)
    interior = cnt == 2
    nb = int((~interior).sum())

    # boundary tags from the tagged triangles
    bkey = np.sort(btris, axis=1)
    ftag = np.full(nf, -1, np.int64)
    pos = _match_rows(keys, bkey)
    if np.any(pos < 0) or np.any(interior[pos]):
        raise MeshError("tagged triangle is not a boundary face")
    ftag[pos] = btags
    if np.any(ftag[~interior] < 0) or nb != nb_in:
        raise MeshError("untagged boundary face")

    # face centroid and oriented face vector
    fabc = keys.copy()
    xa, xb, xcc = xyz[fabc[:, 0]], xyz[fabc[:, 1]], xyz[fabc[:, 2]]
    fx = (xa + xb + xcc) / 3.0
    S = 0.5 * _cross(xb - xa, xcc - xa)
    flip = _dot(S, fx - xcell[fL]) < 0
    S[flip] = -S[flip]
    fabc[flip] = fabc[flip][:, [0, 2, 1]]

    # ghosts: one per boundary face, numbered in face order
    bfaces = np.nonzero(~interior)[0]
    fghost = np.full(nf, -1, np.int64)
    fghost[bfaces] = np.arange(nb)
    gbtri = np.empty(nb, np.int64)
    gbtri[fghost[pos]] = np.arange(nb_in)
    fR = np.where(interior, fR, nc + fghost)
    n_hat = S[bfaces] / np.linalg.norm(S[bfaces], axis=1)[:, None]
    xL = xcell[fL[bfaces]]
    xg = xL + 2.0 * _dot(fx[bfaces] - xL, n_hat)[:, None] * n_hat
    xc = np.concatenate([xcell, xg])
    gdist = np.linalg.norm(xg - xL, axis=1)

    # diamond coefficients (eq. (diamond), D = C): dual basis of
    # {A-C, B-C, R-L}; the face flux S.grad is kAC(uA-uC)+kBC(uB-uC)+kRL(uR-uL)
    A, B, C = xyz[fabc[:, 0]], xyz[fabc[:, 1]], xyz[fabc[:, 2]]
    c = xc[fR] - xc[fL]
    muD = _dot(S, c) / 3.0
    if np.any(muD <= 0):
        raise MeshError("non-positive diamond volume")
    N1 = 0.5 * _cross(B - C, c)
    N2 = 0.5 * _cross(c, A - C)
    kAC = _dot(N1, S) / (3.0 * muD)
    kBC = _dot(N2, S) / (3.0 * muD)
    kRL = _dot(S, S) / (3.0 * muD)

    # cell -> faces with sign
    cfaces = inv.reshape(nc, 4)
    csign = np.where(fL[cfaces] == np.arange(nc)[:, None], 1, -1)

    # -- incidence: vertex -> cells and ghosts --------------------------------
    v_of = np.concatenate([tets.ravel(), keys[bfaces].ravel()])
    e_of = np.concatenate([np.repeat(np.arange(nc), 4),
                           nc + np.repeat(np.arange(nb), 3)])
    nptr, nidx = _csr_from_pairs(v_of, e_of, nv)

    # node-neighbour stencil: union of the vertex incidences of a cell's 4
    # vertices, minus the cell itself
    cv_cell = np.repeat(np.arange(nc), 4)
    cv_vert = tets.ravel()
    deg = np.diff(nptr)[cv_vert]
    rows = np.repeat(cv_cell, deg)
    base = np.repeat(nptr[cv_vert], deg)
    offs = np.arange(deg.sum()) - np.repeat(np.cumsum(deg) - deg, deg)
    ents = nidx[base + offs]
    keep = ents != rows
    key = np.unique(rows[keep] * (nc + nb) + ents[keep])
    sptr, sidx = _csr_from_pairs(key // (nc + nb), key % (nc + nb), nc)

    # least-squares node weights (Algorithm 2): rows of A are [1, x_e - x_v];
    # alpha = e0^T (A^T A)^{-1} A^T
    vrow = np.repeat(np.arange(nv), np.diff(nptr))
    a = np.concatenate([np.ones((len(nidx), 1)), xc[nidx] - xyz[vrow]], axis=1)
    AtA = np.empty((nv, 4, 4))
    for i in range(4):
        for j in range(4):
            AtA[:, i, j] = np.bincount(vrow, weights=a[:, i] * a[:, j],
                                       minlength=nv)
    w = np.linalg.solve(AtA, np.broadcast_to(np.eye(4)[0], (nv, 4))[..., None])[..., 0]
    nalpha = _dot(a, w[vrow])

    return Geometry(nc=nc, nv=nv, nf=nf, nb=nb, tets=tets, xyz=xyz, vol=vol,
                    xc=xc, fL=fL, fR=fR, fabc=fabc, fS=S, fx=fx,
                    fghost=fghost, ftag=ftag, kAC=kAC, kBC=kBC, kRL=kRL,
                    gface=bfaces, gowner=fL[bfaces], gtag=ftag[bfaces],
                    gdist=gdist, cfaces=cfaces, csign=csign,
                    sptr=sptr, sidx=sidx, nptr=nptr, nidx=nidx, nalpha=nalpha,
                    gbtri=gbtri)


def _match_rows(table, query):
    """Index of each query row in ``table`` (rows sorted lexicographically
    by np.unique), -1 if absent."""
    t = table.astype(np.int64)
    q = query.astype(np.int64)
    m = max(int(t.max()), int(q.max()) if len(q) else 0) + 1
    tk = (t[:, 0] * m + t[:, 1]) * m + t[:, 2]
    qk = (q[:, 0] * m + q[:, 1]) * m + q[:, 2]
    pos = np.searchsorted(tk, qk)
    pos = np.minimum(pos, len(tk) - 1)
    return np.where(tk[pos] == qk, pos, -1)


class PerFace:
    """Boundary values given per boundary triangle, in the order of the
    triangles the mesh was built from, instead of one value per tag (the
    Annexes' per-name values generalised to data that varies along a wall)."""

    def __init__(self, vals):
        self.vals = np.asarray(vals, np.float64)


def ghost_values(geo: Geometry, values):
    """The boundary value at each ghost's face: values[tag], or the ghost's
    triangle's entry of a PerFace."""
    if isinstance(values, PerFace):
        return values.vals[geo.gbtri]
    return np.asarray(values, np.float64)[geo.gtag]


def ghost_coefficients(geo: Geometry, kinds, values):
    """Ghost value u_g = s * u_owner + t for each ghost, from per-tag boundary
    conditions (a1).  Zero-flux and Neumann ghosts mirror the owner (plus the
    prescribed normal derivative times the owner-ghost distance); Dirichlet
    ghosts make the face-midpoint average equal to the prescribed value."""
    kinds = np.asarray(kinds)[geo.gtag]
    values = ghost_values(geo, values)
    s = np.where(kinds == DIRICHLET, -1.0, 1.0)
    t = np.where(kinds == DIRICHLET, 2.0 * values,
                 np.where(kinds == NEUMANN, values * geo.gdist, 0.0))
    return s, t
