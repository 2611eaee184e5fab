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


def test_star_moment_tables_and_identity(mapped):
    """The tables of the star-moment form of Algorithm 1.  Over the 4 vertex
    lists of a cell (the oracle's, user numbering) every stencil entity
    appears once per vertex it shares with the cell: the library's
    edge-only list is exactly the entities counted twice, the face
    neighbours are counted three times and the cell itself four times.  With
    those sets the stencil sum J_i = sum (x_j - x_i)(u_j - u_i) equals
    sum over the vertex lists of [C_L + n_L (xbar_L - x_i)(ubar_L - u_i)]
    minus the edge-only terms minus twice the face-neighbour terms, for
    random u (brute force against the oracle's stencil)."""
    g, L, m = mapped.geo, mapped.lib, mapped.m
    eptr, eidx = L.export("edge_nbr_ptr"), L.export("edge_nbr_idx")
    assert eptr[-1] == L.info.edge_nbr_entries
    rng = np.random.default_rng(5)
    u = rng.normal(size=g.nc + g.nb) + 3.0      # an offset: the form must not cancel it
    x = g.xc
    # per vertex list: n, mean position, mean value, centred moment
    nl = np.diff(g.nptr)
    own = np.repeat(np.arange(g.nv), nl)
    xb = np.zeros((g.nv, 3)); ub = np.zeros(g.nv)
    np.add.at(xb, own, x[g.nidx]); np.add.at(ub, own, u[g.nidx])
    xb /= nl[:, None]; ub /= nl
    C = np.zeros((g.nv, 3))
    np.add.at(C, own, (x[g.nidx] - xb[own]) * (u[g.nidx] - ub[own])[:, None])
    worst = 0.0
    for i in range(0, g.nc, max(1, g.nc // 300)):
        c = mapped.cp[i]
        count = {}
        for v in g.tets[c]:
            for e in g.nidx[g.nptr[v]:g.nptr[v + 1]]:
                count[int(e)] = count.get(int(e), 0) + 1
        assert count.pop(int(c)) == 4
        sten = g.sidx[g.sptr[c]:g.sptr[c + 1]]
        assert sorted(count) == sorted(sten.tolist())
        two = sorted(e for e, k in count.items() if k == 2)
        three = sorted(e for e, k in count.items() if k == 3)
        assert max(count.values()) == 3
        assert sorted(mapped.ent_to_user(eidx[eptr[i]:eptr[i + 1]]).tolist()) == two
        nbr = sorted(int(np.where(g.fL[f] == c, g.fR[f], g.fL[f])) for f in g.cfaces[c])
        assert three == nbr
        d = x[sten] - x[c]
        direct = (d * (u[sten] - u[c])[:, None]).sum(0)
        mom = np.zeros(3)
        for v in g.tets[c]:
            mom += C[v] + nl[v] * (xb[v] - x[c]) * (ub[v] - u[c])
        for e in two:
            mom -= (x[e] - x[c]) * (u[e] - u[c])
        for e in three:
            mom -= 2.0 * (x[e] - x[c]) * (u[e] - u[c])
        worst = max(worst, np.abs(mom - direct).max() / np.abs(direct).max())
    assert worst < 1e-12, worst


def test_reverse_cuthill_mckee_order():
    """RCM renumbering: a permutation; read backwards it is a breadth-first
    order, so every cell but the last of its component has a face neighbour
    numbered after it; its bandwidth over face pairs is far below the Morton
    order's (whose curve jumps across the domain); and the library built on
    it has the oracle's geometry (the stencils, in user numbering)."""
    n, seed = 8, 2
    m, g = cube(n, seed), cube_geometry(n, seed)
    rcm = Mapped(n, seed, B.RENUMBER_RCM)
    mor = Mapped(n, seed, B.RENUMBER_MORTON)
    assert sorted(rcm.cp) == list(range(g.nc))
    inv = np.empty(g.nc, np.int64)
    inv[rcm.cp] = np.arange(g.nc)                      # user -> internal
    interior = g.fghost < 0
    a, b = inv[g.fL[interior]], inv[g.fR[interior]]
    later = np.zeros(g.nc, bool)
    later[np.minimum(a, b)] = True
    assert later[:-1].all()                            # one component: only the last cell lacks one
    inv_m = np.empty(g.nc, np.int64)
    inv_m[mor.cp] = np.arange(g.nc)
    bw_rcm = np.abs(a - b).max()
    bw_mor = np.abs(inv_m[g.fL[interior]] - inv_m[g.fR[interior]]).max()
    assert bw_rcm < bw_mor / 4
    ptr, idx = rcm.lib.export("stencil_ptr"), rcm.lib.export("stencil_idx")
    for i in range(0, g.nc, 37):
        u = rcm.cp[i]
        assert np.array_equal(np.sort(rcm.ent_to_user(idx[ptr[i]:ptr[i + 1]])), g.sidx[g.sptr[u]:g.sptr[u + 1]])


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
