"""Translation between the library's internal numbering and the oracle's
user numbering (cells, vertices, faces, ghosts), built from the exported
preprocessed mesh.  Test helper only."""
import numpy as np

from conftest import cube, cube_geometry
from paper_2203_00925_amd import binding as B


def _face_key(tri):
    t = np.sort(np.asarray(tri, np.int64), axis=1)
    return (t[:, 0] * (1 << 21) + t[:, 1]) * (1 << 21) + t[:, 2]


class Mapped:
    """Library arrays translated to user numbering, with oracle face/ghost
    indices for every library face/ghost."""

    def __init__(self, n, seed, renumber=B.RENUMBER_MORTON):
        self.m = cube(n, seed)
        self.geo = cube_geometry(n, seed)
        self.lib = B.Mesh.from_cube(self.m, renumber)
        L = self.lib
        self.cp = L.export("cell_perm")
        self.vp = L.export("vert_perm")
        i = L.info
        abc = L.export("face_abc")
        ukey = _face_key(self.vp[abc.T])
        okey = _face_key(self.geo.fabc)
        order = np.argsort(okey)
        pos = np.searchsorted(okey[order], ukey)
        self.face_map = order[pos]                        # lib face -> oracle face
        assert np.array_equal(okey[self.face_map], ukey)
        # lib ghost g is lib face nfi+g; oracle ghost of that face
        self.ghost_map = self.geo.fghost[self.face_map[i.nf_interior:]]
        assert np.all(self.ghost_map >= 0)

    def ent_to_user(self, e):
        e = np.asarray(e, np.int64)
        nc = self.lib.info.nc
        out = np.empty_like(e)
        cell = e < nc
        out[cell] = self.cp[e[cell]]
        out[~cell] = nc + self.ghost_map[e[~cell] - nc]
        return out

    def cells_to_user(self, a_internal):
        out = np.empty_like(a_internal)
        out[..., self.cp] = a_internal
        return out
