"""The library's host preprocessing (C++, called through the C ABI; no GPU)
against the oracle's independently computed geometry."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from conftest import ROOT, cube, cube_geometry

B = pytest.importorskip("paper_2203_00925_amd.binding")
from mapping import Mapped  # noqa: E402


@pytest.fixture(scope="module", params=[(3, 2), (20, 1)])
def mapped(request):
    return Mapped(*request.param)


def test_counts(mapped):
    i, g = mapped.lib.info, mapped.geo
    assert (i.nc, i.nv, i.nf, i.nb) == (g.nc, g.nv, g.nf, g.nb)
    assert i.nf_interior == g.nf - g.nb
    assert sorted(mapped.cp) == list(range(g.nc))
    assert sorted(mapped.vp) == list(range(g.nv))


def test_cells(mapped):
    g, L = mapped.geo, mapped.lib
    nc = g.nc
    assert np.allclose(L.export("volume"), g.vol[mapped.cp], rtol=1e-14, atol=0)
    cen = L.export("centre")
    ref = g.xc[mapped.ent_to_user(np.arange(nc + g.nb))]
    assert np.abs(cen.T - ref).max() < 1e-15


def test_faces(mapped):
    g, L = mapped.geo, mapped.lib
    fm = mapped.face_map
    lr = L.export("face_lr")
    assert np.array_equal(mapped.ent_to_user(lr[0]), g.fL[fm])
    assert np.array_equal(mapped.ent_to_user(lr[1]), g.fR[fm])
    abc = L.export("face_abc")
    assert np.array_equal(mapped.vp[abc].T, g.fabc[fm])
    S = L.export("face_s")
    assert np.abs(S.T - g.fS[fm]).max() < 1e-16
    k = L.export("face_coef")
    for row, ref in zip(k, (g.kAC, g.kBC, g.kRL)):
        assert np.allclose(row, ref[fm], rtol=1e-12, atol=1e-14)
    # boundary faces come last and carry their tags
    i = L.info
    assert np.all(fm[:i.nf_interior] < g.nf) and np.all(g.fghost[fm[:i.nf_interior]] < 0)
    assert np.array_equal(L.export("ghost_tag"), g.gtag[mapped.ghost_map])
    assert np.array_equal(mapped.cp[L.export("ghost_owner")], g.gowner[mapped.ghost_map])


def test_stencil_and_gradient_matrix(mapped):
    g, L = mapped.geo, mapped.lib
    ptr, idx = L.export("stencil_ptr"), L.export("stencil_idx")
    minv = L.export("minv")
    for i in range(0, g.nc, max(1, g.nc // 400)):
        u = mapped.cp[i]
        got = np.sort(mapped.ent_to_user(idx[ptr[i]:ptr[i + 1]]))
        ref = g.sidx[g.sptr[u]:g.sptr[u + 1]]
        assert np.array_equal(got, ref)
        assert np.all(np.diff(idx[ptr[i]:ptr[i + 1]]) > 0)      # ascending, unique
        d = g.xc[ref] - g.xc[u]
        Mi = np.linalg.inv(d.T @ d)
        mine = np.array([[minv[0, i], minv[1, i], minv[2, i]],
                         [minv[1, i], minv[3, i], minv[4, i]],
                         [minv[2, i], minv[4, i], minv[5, i]]])
        assert np.allclose(mine, Mi, rtol=1e-11, atol=1e-11 * np.abs(Mi).max())


def test_vertex_weights(mapped):
    g, L = mapped.geo, mapped.lib
    ptr, idx, al = L.export("node_ptr"), L.export("node_idx"), L.export("node_alpha")
    for v in range(0, g.nv, max(1, g.nv // 400)):
        uv = mapped.vp[v]
        ents = mapped.ent_to_user(idx[ptr[v]:ptr[v + 1]])
        o = np.argsort(ents)
        ref_e = g.nidx[g.nptr[uv]:g.nptr[uv + 1]]
        ref_a = g.nalpha[g.nptr[uv]:g.nptr[uv + 1]]
        assert np.array_equal(ents[o], ref_e)
        assert np.allclose(al[ptr[v]:ptr[v + 1]][o], ref_a, rtol=1e-11, atol=1e-12)


def test_info_sizes(mapped):
    i = mapped.lib.info
    assert i.stencil_max == 70 and i.row_max <= 70 and i.node_max >= 24
    assert i.stencil_padded >= i.stencil_entries and i.stencil_padded % 64 == 0
    assert i.matrix_nnz <= 71 * i.nc
    assert i.ws_bytes > 0 and i.ws_bytes % 256 == 0


def test_no_renumber_keeps_order():
    m = cube(3, 2)
    L = B.Mesh.from_cube(m, B.RENUMBER_NONE)
    assert np.array_equal(L.export("cell_perm"), np.arange(L.info.nc))


def test_mesh_errors():
    m = cube(2)
    with pytest.raises(B.MifvmError) as e:
        B.Mesh(m.xyz, np.concatenate([m.tets, m.tets[:1]]), m.btris, m.btags)
    assert e.value.code == -2
    with pytest.raises(B.MifvmError) as e:
        B.Mesh(m.xyz, m.tets, m.btris[1:], m.btags[1:])
    assert e.value.code == -2
    xyz = m.xyz.copy()
    xyz[m.tets[0, 3]] = xyz[m.tets[0, :3]].mean(axis=0)
    with pytest.raises(B.MifvmError) as e:
        B.Mesh(xyz, m.tets, m.btris, m.btags)
    assert e.value.code == -2
    bad = m.tets.copy()
    bad[0, 0] = len(m.xyz)
    with pytest.raises(B.MifvmError) as e:
        B.Mesh(m.xyz, bad, m.btris, m.btags)
    assert e.value.code == -1
    with pytest.raises(B.MifvmError) as e:
        B.Mesh(m.xyz, m.tets, m.btris, np.full(len(m.btags), 40, np.int32))
    assert e.value.code == -1


def test_library_exports_every_declared_symbol():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            hdr = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(mifvm_\w+)\s*\(", hdr, re.M)
    assert len(names) >= 35
    assert "mifvm_nn_train" in names and "mifvm_poisson_solve" in names
    lib = C.CDLL(B._LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
