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
