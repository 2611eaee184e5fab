"""Pins of the oracle's FV residual and time step (eqs. (4), (6), (15),
(diamond)) against invariants, textbook special cases and the Poisson
operator assembled by a separate code path."""
import numpy as np
import pytest

import synth
from conftest import cube, cube_geometry
from oracle import fv, poisson
from oracle.geometry import ZERO_FLUX, NEUMANN, DIRICHLET


def test_rk3_amplification_polynomial():
    """Mock residual Res(u) = lam*u: eq. (6) with alpha = (1/2, 1/2, 1) has
    amplification 1 + z + z^2/2 + z^3/4."""
    lam = np.array([-3.0, -0.5, 0.7, 2.0])
    dt = 0.13
    out = fv.rk3_step(None, np.ones(4), dt, None, None, None, None,
                      residual_fn=lambda v: lam * v)
    z = lam * dt
    assert np.allclose(out, 1 + z + z ** 2 / 2 + z ** 3 / 4, rtol=1e-15, atol=0)


def test_constant_state_preserved():
    geo = cube_geometry(4, seed=11)
    u = np.full(geo.nc, 2.5)
    vel = np.tile([0.3, -0.2, 0.5], (geo.nc, 1))
    phi = fv.face_velocity_flux(geo, vel)
    r = fv.residual(geo, u, phi, 1e-2, [NEUMANN] * 6, [0.0] * 6)
    assert np.abs(r).max() < 1e-11
    r = fv.residual(geo, u, 0 * phi, 1e-2, [ZERO_FLUX] * 6, [0.0] * 6)
    assert np.abs(r).max() < 1e-11


def test_conservation_config1_10_steps():
    """Zero-flux walls: sum mu_i u_i is conserved through 10 RK3 steps of the
    48,000-cell benchmark problem to round-off."""
    m = cube(20, 1)
    geo = cube_geometry(20, 1)
    pf = synth.problem_fields(m)
    kinds, vals = [ZERO_FLUX] * 6, [0.0] * 6
    phi = fv.face_velocity_flux(geo, pf.vel)
    dt = fv.cfl_dt(geo, phi, pf.diffusivity, pf.cfl, kinds)
    u = pf.u0.copy()
    t0 = fv.conservation_total(geo, u)
    scale = float(np.dot(geo.vol, np.abs(u)))
    for _ in range(10):
        u = fv.rk3_step(geo, u, dt, phi, pf.diffusivity, kinds, vals)
    assert abs(fv.conservation_total(geo, u) - t0) < 10 * 1e-15 * scale * 10
    assert np.isfinite(u).all() and u.max() < pf.u0.max()


def test_first_order_upwind_when_limited_to_zero():
    """psi = 0 reduces eq. (15) to first-order upwind: F = phi * u_upwind."""
    geo = cube_geometry(3, seed=4)
    rng = np.random.default_rng(3)
    u_ext = np.concatenate([rng.normal(size=geo.nc), np.zeros(geo.nb)])
    phi = rng.normal(size=geo.nf)
    grad = rng.normal(size=(geo.nc, 3))
    F = fv.face_fluxes(geo, u_ext, grad, np.zeros(geo.nc), np.zeros(geo.nv),
                       phi, 0.0, [DIRICHLET] * 6, [0.0] * 6)
    interior = geo.fghost < 0
    up = np.where(phi >= 0, u_ext[geo.fL], u_ext[geo.fR])
    assert np.array_equal(F[interior], (phi * up)[interior])


def test_limiter_bounds_reconstruction():
    geo = cube_geometry(4, seed=9)
    rng = np.random.default_rng(4)
    u = rng.normal(size=geo.nc)
    u_ext = fv.extend_with_ghosts(geo, u, np.ones(geo.nb), np.zeros(geo.nb))
    g = fv.cell_gradient(geo, u_ext)
    psi = fv.barth_jespersen(geo, u_ext, g)
    assert np.all((psi >= 0) & (psi <= 1))
    nbv = u_ext[fv.face_neighbours(geo)]
    umax = np.maximum(u, nbv.max(1))
    umin = np.minimum(u, nbv.min(1))
    r = geo.fx[geo.cfaces] - geo.xc[:geo.nc][:, None]
    rec = u[:, None] + psi[:, None] * np.einsum("ij,ikj->ik", g, r)
    assert np.all(rec <= umax[:, None] + 1e-13)
    assert np.all(rec >= umin[:, None] - 1e-13)
    # a strict local maximum with a non-zero gradient is limited to psi = 0
    i = int(np.argmax(u - nbv.max(1)))
    assert u[i] > nbv[i].max() and psi[i] == 0.0


def test_limiter_is_one_for_linear_field():
    """A linear field on interior cells whose reconstructions stay inside the
    neighbour range is not limited."""
    geo = cube_geometry(4, seed=9)
    a = np.array([1.0, 0.5, -0.25])
    u_ext = geo.xc @ a
    g = fv.cell_gradient(geo, u_ext)
    psi = fv.barth_jespersen(geo, u_ext, g)
    nbv = u_ext[fv.face_neighbours(geo)]
    r = geo.fx[geo.cfaces] - geo.xc[:geo.nc][:, None]
    d = np.einsum("ij,ikj->ik", g, r)
    u = u_ext[:geo.nc]
    ok = np.all((u[:, None] + d <= np.maximum(u, nbv.max(1))[:, None])
                & (u[:, None] + d >= np.minimum(u, nbv.min(1))[:, None]), axis=1)
    assert ok.sum() > geo.nc // 2
    assert np.all(psi[ok] == 1.0)


def test_pure_diffusion_matches_assembled_operator():
    """With V = 0 the residual of eq. (4) is D/mu times the discrete Laplacian
    of eq. (7); the Poisson matrix is assembled by a separate code path
    (coefficient expansion), so this pins both."""
    geo = cube_geometry(4, seed=12)
    rng = np.random.default_rng(5)
    u = rng.normal(size=geo.nc)
    kinds = [DIRICHLET, DIRICHLET, NEUMANN, NEUMANN, ZERO_FLUX, DIRICHLET]
    vals = [1.0, -2.0, 0.5, 0.0, 0.0, 0.25]
    D = 0.3
    res = fv.residual(geo, u, np.zeros(geo.nf), D, kinds, vals)
    K, c = poisson.assemble(geo, kinds, vals)
    ref = D * (-(K @ u) + c) / geo.vol
    assert np.abs(res - ref).max() < 1e-11 * np.abs(ref).max()


def test_cfl_dt_definition():
    geo = cube_geometry(3, seed=2)
    m = cube(3, 2)
    phi = fv.face_velocity_flux(geo, synth.rotating_velocity(m))
    dt = fv.cfl_dt(geo, phi, 1e-3, 0.4, [ZERO_FLUX] * 6)
    rate = np.where(geo.fghost < 0, np.abs(phi) + 1e-3 * geo.kRL, 0.0)
    per = rate[geo.cfaces].sum(1)
    assert np.all(dt * per <= 0.4 * geo.vol * (1 + 1e-15))
    assert np.isclose(np.max(dt * per / geo.vol), 0.4, rtol=1e-14)


def _affine_family(geo, rng, nfun=3):
    """Cells carrying one of ``nfun`` global affine functions l_k(x) = c_k + a_k.x
    (assigned at random per cell): u_i = l_k(x_i) and the exact gradient a_k."""
    cs = rng.normal(size=nfun)
    As = rng.normal(size=(nfun, 3))
    k = rng.integers(0, nfun, size=geo.nc)
    xc = geo.xc[:geo.nc]
    u = cs[k] + np.einsum("ij,ij->i", As[k], xc)
    return cs, As, k, u


def test_muscl_reconstruction_of_a_linear_field_is_exact():
    """eq. (15), second-order term: with an exact gradient and psi = 1, the
    reconstruction from either side of a face of a linear field u = b + a.x is
    u(x_f), so every interior face carries phi_f * u(x_f) whatever the sign of
    phi_f (both upwind directions are exercised)."""
    geo = cube_geometry(4, seed=21)
    rng = np.random.default_rng(8)
    a, b = np.array([0.7, -1.3, 0.4]), 2.0
    u_ext = np.concatenate([b + geo.xc[:geo.nc] @ a, np.zeros(geo.nb)])
    grad = np.tile(a, (geo.nc, 1))
    phi = rng.normal(size=geo.nf)
    assert (phi > 0).sum() > geo.nf // 3 and (phi < 0).sum() > geo.nf // 3
    F = fv.face_fluxes(geo, u_ext, grad, np.ones(geo.nc), np.zeros(geo.nv),
                       phi, 0.0, [DIRICHLET] * 6, [0.0] * 6)
    interior = geo.fghost < 0
    exact = phi * (b + geo.fx @ a)
    scale = np.abs(exact[interior]).max()
    assert np.abs(F[interior] - exact[interior]).max() < 1e-13 * scale


def test_muscl_takes_the_upwind_cells_own_limited_reconstruction():
    """eq. (15) with the limiter: a cell carrying the affine function l is
    reconstructed at a face as l evaluated at x_c + psi (x_f - x_c) (the limited
    point on the segment from its centre to the face centroid), and the face
    takes the value of its upwind cell (L when phi_f >= 0, else R).  Neighbours
    carry different affine functions and limiters, so using the wrong side's
    gradient, centre or psi, or dropping psi on one side, changes the flux."""
    geo = cube_geometry(4, seed=22)
    rng = np.random.default_rng(9)
    cs, As, k, u = _affine_family(geo, rng)
    u_ext = np.concatenate([u, np.zeros(geo.nb)])
    grad = As[k]
    psi = rng.choice([0.0, 0.5, 1.0], size=geo.nc)
    phi = rng.normal(size=geo.nf)
    F = fv.face_fluxes(geo, u_ext, grad, psi, np.zeros(geo.nv), phi, 0.0,
                       [DIRICHLET] * 6, [0.0] * 6)
    interior = np.nonzero(geo.fghost < 0)[0]
    up = np.where(phi[interior] >= 0, geo.fL[interior], geo.fR[interior])
    xc = geo.xc[:geo.nc]
    point = xc[up] + psi[up][:, None] * (geo.fx[interior] - xc[up])
    val = cs[k[up]] + np.einsum("ij,ij->i", As[k[up]], point)
    exact = phi[interior] * val
    # the test is only discriminating if the two sides disagree on many faces
    other = np.where(phi[interior] >= 0, geo.fR[interior], geo.fL[interior])
    pt_o = xc[other] + psi[other][:, None] * (geo.fx[interior] - xc[other])
    val_o = cs[k[other]] + np.einsum("ij,ij->i", As[k[other]], pt_o)
    assert (np.abs(val_o - val) > 1e-3).mean() > 0.5
    assert np.abs(F[interior] - exact).max() < 1e-13 * np.abs(exact).max()


def test_neumann_ghosts_give_exact_gradients_of_a_linear_field():
    """Neumann data equal to the normal derivative a.n of a linear field on
    every wall: each ghost value is the field at the ghost centre (the mirror
    of the owner across the face), so the least-squares gradient of
    Algorithm 1 is exact in every cell, boundary cells included."""
    geo = cube_geometry(4, seed=23)
    a = np.array([1.5, -0.75, 2.25])
    u = 0.3 + geo.xc[:geo.nc] @ a
    normals = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0],
                        [0, 0, -1], [0, 0, 1]], np.float64)
    vals = list(normals @ a)
    gs, gt = fv.ghost_coefficients(geo, [NEUMANN] * 6, vals)
    u_ext = fv.extend_with_ghosts(geo, u, gs, gt)
    assert np.abs(u_ext[geo.nc:] - (0.3 + geo.xc[geo.nc:] @ a)).max() < 1e-13
    g = fv.cell_gradient(geo, u_ext)
    assert np.abs(g - a).max() < 1e-11


def test_neumann_flux_balances_a_linear_field():
    """With V = 0, a linear u and Neumann data a.n on every wall, every face
    flux is D a.S_f (the diamond on interior faces, the prescribed D*value*|S|
    on the walls) and each closed cell sums its outward S_f to zero, so the
    residual of eq. (4) vanishes in every cell.  A wrong sign of the Neumann
    flux or of the ghost offset leaves a residual in the boundary cells."""
    geo = cube_geometry(4, seed=24)
    a = np.array([-0.6, 1.1, 0.9])
    u = 1.0 + geo.xc[:geo.nc] @ a
    normals = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0],
                        [0, 0, -1], [0, 0, 1]], np.float64)
    vals = list(normals @ a)
    D = 0.7
    res, p = fv.residual(geo, u, np.zeros(geo.nf), D, [NEUMANN] * 6, vals, parts=True)
    scale = D * np.abs(a).sum() * (np.linalg.norm(geo.fS, axis=1).max() / geo.vol.min())
    assert np.abs(res).max() < 1e-11 * scale
    bnd = geo.fghost >= 0
    assert np.abs(p["F"][bnd] + D * (geo.fS[bnd] @ a)).max() < 1e-13
