"""Pins of the oracle's geometry (Sec. 2.1) against closed forms, brute-force
least squares and linear exactness."""
import numpy as np
import pytest

from conftest import cube, cube_geometry
from oracle import fv
from oracle.geometry import build_geometry, MeshError


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_counts_closed_form(n):
    geo = cube_geometry(n)
    assert geo.nc == 6 * n ** 3
    assert geo.nf == 12 * n ** 3 + 6 * n ** 2
    assert geo.nb == 12 * n ** 2
    assert geo.nv == (n + 1) ** 3
    # Euler characteristic of a ball: V - E + F - C = 1
    t = geo.tets
    edges = np.concatenate([np.sort(t[:, [a, b]], axis=1)
                            for a in range(4) for b in range(a + 1, 4)])
    ne = len(np.unique(edges, axis=0))
    assert ne == 3 * n * (n + 1) ** 2 + 3 * n ** 2 * (n + 1) + n ** 3
    assert geo.nv - ne + geo.nf - geo.nc == 1


def test_volumes_and_closed_cells():
    geo = cube_geometry(4)
    assert abs(geo.vol.sum() - 1.0) < 1e-14
    assert np.all(geo.vol > 0)
    # each cell is a closed surface: sum of outward face vectors vanishes
    s = np.einsum("ij,ijk->ik", geo.csign, geo.fS[geo.cfaces])
    assert np.abs(s).max() < 1e-16
    # face vectors point from L to R and have the area of the triangle
    d = geo.xc[geo.fR] - geo.xc[geo.fL]
    assert np.all(np.einsum("ij,ij->i", d, geo.fS) > 0)
    A, B, C = (geo.xyz[geo.fabc[:, k]] for k in range(3))
    area = 0.5 * np.linalg.norm(np.cross(B - A, C - A), axis=1)
    assert np.allclose(np.linalg.norm(geo.fS, axis=1), area, rtol=1e-14)


def test_ghosts_mirror_owner_across_face():
    geo = cube_geometry(3)
    f = geo.gface
    xL = geo.xc[geo.gowner]
    xg = geo.xc[geo.nc:]
    mid = 0.5 * (xL + xg)
    nhat = geo.fS[f] / np.linalg.norm(geo.fS[f], axis=1)[:, None]
    # midpoint on the face plane, offset along the normal
    assert np.abs(np.einsum("ij,ij->i", mid - geo.fx[f], nhat)).max() < 1e-15
    off = xg - xL
    assert np.abs(np.cross(off, nhat)).max() < 1e-15
    # the cube's boundary planes: every ghost lies outside the unit cube
    out = (xg < 0) | (xg > 1)
    assert np.all(out.any(axis=1))


def test_stencil_sizes():
    """Node-neighbour stencil of an interior cell is 70 cells (inclusion-
    exclusion over its 4 vertex stars of 24 cells), no ghosts."""
    n = 4
    geo = cube_geometry(n)
    m = cube(n)
    on_b = np.any((np.abs(m.xyz) < 1e-12) | (np.abs(m.xyz - 1) < 1e-12), axis=1)
    interior_cell = ~np.any(on_b[geo.tets], axis=1)
    cnt = np.diff(geo.sptr)
    assert np.all(cnt[interior_cell] == 70)
    has_ghost = np.array([np.any(geo.sidx[geo.sptr[i]:geo.sptr[i + 1]] >= geo.nc)
                          for i in range(geo.nc)])
    assert not np.any(has_ghost[interior_cell])
    assert np.all(has_ghost[~interior_cell])
    # interior vertex stars hold 24 cells
    nstar = np.diff(geo.nptr)
    assert np.all(nstar[~on_b] == 24)


def test_gradient_equals_lstsq_bruteforce():
    geo = cube_geometry(2, seed=5)
    rng = np.random.default_rng(0)
    u_ext = rng.normal(size=geo.nc + geo.nb)
    g = fv.cell_gradient(geo, u_ext)
    for i in range(geo.nc):
        nb = geo.sidx[geo.sptr[i]:geo.sptr[i + 1]]
        D = geo.xc[nb] - geo.xc[i]
        ref, *_ = np.linalg.lstsq(D, u_ext[nb] - u_ext[i], rcond=None)
        assert np.allclose(g[i], ref, rtol=1e-11, atol=1e-11)


def test_node_weights_equal_lstsq_intercept():
    geo = cube_geometry(2, seed=6)
    rng = np.random.default_rng(1)
    u_ext = rng.normal(size=geo.nc + geo.nb)
    un = fv.node_values(geo, u_ext)
    for v in range(geo.nv):
        ent = geo.nidx[geo.nptr[v]:geo.nptr[v + 1]]
        A = np.concatenate([np.ones((len(ent), 1)), geo.xc[ent] - geo.xyz[v]], axis=1)
        coef, *_ = np.linalg.lstsq(A, u_ext[ent], rcond=None)
        assert abs(un[v] - coef[0]) < 1e-11
        a = geo.nalpha[geo.nptr[v]:geo.nptr[v + 1]]
        assert abs(a.sum() - 1) < 1e-12
        assert np.abs(a @ (geo.xc[ent] - geo.xyz[v])).max() < 1e-13


def test_diamond_equals_3x3_solve():
    geo = cube_geometry(2, seed=7)
    rng = np.random.default_rng(2)
    u_ext = rng.normal(size=geo.nc + geo.nb)
    un = rng.normal(size=geo.nv)
    fl = fv.diamond_flux(geo, u_ext, un)
    for f in range(geo.nf):
        a, b, c = geo.fabc[f]
        M = np.stack([geo.xyz[a] - geo.xyz[c], geo.xyz[b] - geo.xyz[c],
                      geo.xc[geo.fR[f]] - geo.xc[geo.fL[f]]])
        rhs = np.array([un[a] - un[c], un[b] - un[c],
                        u_ext[geo.fR[f]] - u_ext[geo.fL[f]]])
        grad = np.linalg.solve(M, rhs)
        assert abs(grad @ geo.fS[f] - fl[f]) < 1e-12 * (1 + np.abs(grad).max())


def test_linear_exactness():
    geo = cube_geometry(4, seed=3)
    a = np.array([0.3, -1.2, 2.0])
    lin = lambda X: 1.5 + X @ a
    u_ext = lin(geo.xc)
    g = fv.cell_gradient(geo, u_ext)
    assert np.abs(g - a).max() < 1e-13
    un = fv.node_values(geo, u_ext)
    assert np.abs(un - lin(geo.xyz)).max() < 1e-13
    assert np.abs(fv.diamond_flux(geo, u_ext, un) - geo.fS @ a).max() < 1e-14


def test_mesh_errors():
    m = cube(2)
    with pytest.raises(MeshError):       # duplicated cell -> face with 3 owners
        build_geometry(m.xyz, np.concatenate([m.tets, m.tets[:1]]), m.btris, m.btags)
    with pytest.raises(MeshError):       # untagged boundary face
        build_geometry(m.xyz, m.tets, m.btris[1:], m.btags[1:])
    bad = m.tets.copy()
    xyz = m.xyz.copy()
    xyz[bad[0, 3]] = xyz[bad[0, :3]].mean(axis=0)     # flatten one tet
    with pytest.raises(MeshError):
        build_geometry(xyz, bad, m.btris, m.btags)


def test_orientation_is_fixed():
    m = cube(2)
    t = m.tets.copy()
    t[::3] = t[::3][:, [1, 0, 2, 3]]                  # invert some cells
    a = build_geometry(m.xyz, t, m.btris, m.btags)
    b = cube_geometry(2)
    assert np.allclose(a.vol, b.vol, rtol=0, atol=1e-17)
    assert np.all(a.vol > 0)
