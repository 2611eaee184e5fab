"""Pins of the oracle's coupled streamer-type loop (Sec. 4, eq. (10)):
values the mathematics fixes, independent of the oracle's own formulas."""
import numpy as np

import synth
from conftest import cube, cube_geometry
from oracle import fv, poisson, streamer
from oracle.geometry import ZERO_FLUX, NEUMANN, DIRICHLET

# potential: P = 1 on x = 0, P = 0 on x = 1, zero normal derivative elsewhere
POT_KINDS = [DIRICHLET, DIRICHLET, NEUMANN, NEUMANN, NEUMANN, NEUMANN]
POT_VALS = [1.0, 0.0, 0.0, 0.0, 0.0, 0.0]
NE_KINDS = [ZERO_FLUX] * 6
NE_VALS = [0.0] * 6


def setup(n=6, seed=3):
    m, g = cube(n, seed), cube_geometry(n, seed)
    K, c = poisson.assemble(g, POT_KINDS, POT_VALS)
    ne = synth.gaussian_field(m, (0.4, 0.5, 0.5), 0.2) + 0.1
    return m, g, K, c, ne


def test_neutral_plasma_gives_the_linear_potential_and_uniform_field():
    """No charge (n_p = n_e): Delta P = 0 with these conditions has the exact
    solution P = 1 - x, which the scheme reproduces (linear fields are exact
    for the diamond and Algorithm 1), so E = (1, 0, 0) in every cell, v_e =
    -mu E, and S_e = a exp(-b) mu n_e in closed form."""
    m, g, K, c, ne = setup()
    mu, a, b = 2.0, 3.0, 0.5
    out_ne, out_np, P, E, dt, it = streamer.coupled_step(
        g, ne, ne.copy(), np.zeros(g.nc), K, c, 1e-3, NE_KINDS, NE_VALS, POT_KINDS, POT_VALS,
        mu, 7.0, a, b, 0.4, tol=1e-14)
    assert np.abs(P - (1.0 - g.xc[:g.nc, 0])).max() < 1e-11
    assert np.abs(E - np.array([1.0, 0.0, 0.0])).max() < 1e-9
    _, v, S = streamer.fields(g, P, POT_KINDS, POT_VALS, mu, a, b, ne)
    assert np.abs(v - np.array([-mu, 0.0, 0.0])).max() < 1e-9 * mu
    assert np.allclose(S, a * np.exp(-b) * mu * ne, rtol=1e-9, atol=0)
    # the ions gain exactly dt S_e
    assert np.allclose(out_np - ne, dt * S, rtol=1e-12, atol=1e-15)


def test_net_charge_is_conserved_with_zero_flux_walls():
    """With zero-flux walls for n_e the total sum mu_i (n_e - n_p) is conserved
    by the loop (interior fluxes cancel; production adds the same dt S_e to
    both species) even with drift and ionisation."""
    m, g, K, c, ne = setup()
    rng = np.random.default_rng(2)
    n_ion = ne + 0.05 * rng.uniform(size=g.nc)
    P = np.zeros(g.nc)
    q0 = float(np.dot(g.vol, ne - n_ion))
    for _ in range(4):
        ne, n_ion, P, E, dt, it = streamer.coupled_step(
            g, ne, n_ion, P, K, c, 1e-3, NE_KINDS, NE_VALS, POT_KINDS, POT_VALS,
            1.0, 40.0, 2.0, 0.3, 0.4)
        assert dt > 0 and np.abs(E).max() > 0
    q1 = float(np.dot(g.vol, ne - n_ion))
    assert abs(q1 - q0) <= 1e-13 * float(np.dot(g.vol, ne))


def test_no_drift_no_source_reduces_to_diffusion_and_the_poisson_solve():
    """mu = 0 and a = 0: the step is the plain RK3 diffusion step of n_e at
    its CFL bound, n_p is unchanged, and P is the Poisson solution for the
    charge."""
    m, g, K, c, ne = setup()
    n_ion = 0.5 * ne
    D = 2e-2
    out_ne, out_np, P, E, dt, it = streamer.coupled_step(
        g, ne, n_ion, np.zeros(g.nc), K, c, D, NE_KINDS, NE_VALS, POT_KINDS, POT_VALS,
        0.0, 5.0, 0.0, 0.0, 0.4, tol=1e-13)
    phi0 = np.zeros(g.nf)
    dt_ref = fv.cfl_dt(g, phi0, D, 0.4, NE_KINDS)
    assert dt == dt_ref
    ref = fv.rk3_step(g, ne, dt_ref, phi0, D, NE_KINDS, NE_VALS)
    assert np.abs(out_ne - ref).max() <= 1e-15 * np.abs(ref).max()
    assert np.array_equal(out_np, n_ion)
    Pd = poisson.direct_solve(K, poisson.rhs(g, 5.0 * (ne - n_ion), c))
    assert np.abs(P - Pd).max() <= 1e-10 * np.abs(Pd).max()


def test_townsend_law():
    e = np.array([0.0, 1.0, 2.0, 1e3])
    al = streamer.townsend_alpha(e, 2.0, 4.0)
    assert al[0] == 0.0
    assert np.isclose(al[1], 2.0 * np.exp(-4.0)) and np.isclose(al[2], 2.0 * np.exp(-2.0))
    assert np.isclose(al[3], 2.0, rtol=5e-3)
