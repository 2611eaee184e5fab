"""The oracle's sampled-cell evaluation (two-vertex-ring submeshes) equals
the global oracle on every cell of a small mesh, for mixed boundary
conditions - the pin that lets it stand in for the global oracle on meshes
too large to assemble on the host."""
import numpy as np

import synth
from conftest import cube, cube_geometry
from oracle import fv, poisson, local
from oracle.geometry import ZERO_FLUX, NEUMANN, DIRICHLET


def test_local_residual_equals_global():
    m = cube(5, 21)
    geo = cube_geometry(5, 21)
    rng = np.random.default_rng(3)
    u = synth.gaussian_field(m, (0.4, 0.5, 0.6), 0.2) + 0.05 * rng.normal(size=geo.nc)
    vel = synth.rotating_velocity(m)
    kinds = [DIRICHLET, NEUMANN, ZERO_FLUX, DIRICHLET, NEUMANN, ZERO_FLUX]
    vals = [0.3, -0.2, 0.0, 1.0, 0.5, 0.0]
    ref = fv.residual(geo, u, fv.face_velocity_flux(geo, vel), 2e-2, kinds, vals)
    vidx = local.VertexIndex(m.tets, m.nv)
    cells = np.arange(0, geo.nc, 7)
    got = local.residual_at(m, vidx, cells, u, vel, 2e-2, kinds, vals)
    assert np.abs(got - ref[cells]).max() <= 1e-13 * np.abs(ref).max()


def test_local_matrix_rows_equal_global():
    m = cube(5, 22)
    geo = cube_geometry(5, 22)
    kinds = [DIRICHLET, NEUMANN, DIRICHLET, ZERO_FLUX, NEUMANN, DIRICHLET]
    vals = [1.0, 0.5, -2.0, 0.0, 0.0, 0.25]
    K, c = poisson.assemble(geo, kinds, vals)
    x = np.random.default_rng(4).normal(size=geo.nc)
    vidx = local.VertexIndex(m.tets, m.nv)
    cells = np.arange(3, geo.nc, 11)
    kx, cc = local.matrix_rows_times(m, vidx, cells, x, kinds, vals)
    assert np.abs(kx - (K @ x)[cells]).max() <= 1e-13 * np.abs(K @ x).max()
    assert np.abs(cc - c[cells]).max() <= 1e-13 * max(np.abs(c).max(), 1.0)


def test_local_step_equals_global():
    """One RK3 step of eq. (6) from six-vertex-ring submeshes equals the
    global oracle's step at sampled cells (interior, edge and corner cells;
    on a mesh where the six rings of an interior cell leave cut faces)."""
    m = cube(12, 23)
    geo = cube_geometry(12, 23)
    u = synth.gaussian_field(m, (0.45, 0.5, 0.55), 0.15)
    vel = synth.rotating_velocity(m)
    kinds = [DIRICHLET, NEUMANN, ZERO_FLUX, DIRICHLET, ZERO_FLUX, NEUMANN]
    vals = [0.2, -0.1, 0.0, 0.5, 0.0, 0.3]
    D = 5e-3
    phi = fv.face_velocity_flux(geo, vel)
    dt = fv.cfl_dt(geo, phi, D, 0.4, kinds)
    ref = fv.rk3_step(geo, u, dt, phi, D, kinds, vals)
    vidx = local.VertexIndex(m.tets, m.nv)
    xc = geo.xc[:geo.nc]
    centre = int(np.argmin(np.linalg.norm(xc - 0.5, axis=1)))
    corner = int(np.argmin(np.linalg.norm(xc, axis=1)))
    edge = int(np.argmin(np.linalg.norm(xc - [0.5, 0.0, 1.0], axis=1)))
    cells = np.array([centre, corner, edge, 17, geo.nc - 5])
    _, _, _, _, ids = local.submesh(m, vidx, centre, rings=6)
    assert len(ids) < geo.nc                      # the interior submesh is cut
    got = local.step_at(m, vidx, cells, u, vel, D, kinds, vals, dt)
    assert np.abs(got - ref[cells]).max() <= 1e-13 * np.abs(ref).max()
