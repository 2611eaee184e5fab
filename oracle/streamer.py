"""Coupled streamer-type loop (oracle; test infrastructure only).

Sec. 4, eq. (10): the electron density n_e is convected with the electron
velocity, diffused and produced by ionisation, the positive ions n_p only
gain that production, and the potential follows from the charge:

    d n_e/dt + div(n_e v_e) - div(D grad n_e) = S_e,      d n_p/dt = S_e,
    Laplacian(P) = -(e/eps)(n_p - n_e),                   E = -grad P,
    S_e = alpha |v_e| n_e.

Readings where the paper is silent, garbled or gives no values:
* the velocity law eq. (velo) needs C1 and C2, which are not given: the
  electron velocity is v_e = -mu E with a constant mobility mu;
* the ionisation fit eq. (alphaN) is not usable as printed: alpha is the
  Townsend-type law alpha(|E|) = a exp(-b / |E|) (0 where E = 0) with
  caller constants;
* eq. (diff) is garbled (a vector): D is a constant;
* e/eps is a caller constant kappa, so the Poisson right-hand side of the
  library's Delta P = f is f = kappa (n_e - n_p);
* one step: solve for P (Jacobi-CG from the previous P), E = -grad P by
  the least-squares gradient of Algorithm 1 with P's ghost values from the
  potential's boundary conditions, v_e and S_e per cell, the face velocity
  fluxes, dt = CFL bound, one RK3 step of n_e with S_e held over the step
  (the RK3 stages add exactly dt S_e), and n_p += dt S_e.
"""
from __future__ import annotations

import numpy as np

from . import fv, poisson
from .geometry import Geometry, ghost_coefficients


def townsend_alpha(e_norm, a, b):
    """alpha(|E|) = a exp(-b / |E|), 0 where |E| = 0."""
    e_norm = np.asarray(e_norm, np.float64)
    out = np.zeros_like(e_norm)
    pos = e_norm > 0
    out[pos] = a * np.exp(-b / e_norm[pos])
    return out


def fields(geo: Geometry, P, pot_kinds, pot_values, mobility, a, b, ne):
    """E = -grad P (Algorithm 1 with the potential's ghosts), v_e = -mu E,
    S_e = alpha(|E|) |v_e| n_e."""
    gs, gt = ghost_coefficients(geo, pot_kinds, pot_values)
    E = -fv.cell_gradient(geo, fv.extend_with_ghosts(geo, P, gs, gt))
    v = -mobility * E
    en = np.linalg.norm(E, axis=1)
    S = townsend_alpha(en, a, b) * np.linalg.norm(v, axis=1) * ne
    return E, v, S


def coupled_step(geo: Geometry, ne, n_ion, P, K, c, D, kinds, values, pot_kinds, pot_values,
                 mobility, kappa, a, b, cfl, tol=1e-10, restart=500):
    """One step of the loop; returns (n_e, n_p, P, E, dt, CG iterations)."""
    bvec = poisson.rhs(geo, kappa * (ne - n_ion), c)
    P, it, _ = poisson.jacobi_cg(K, bvec, x0=P, tol=tol, restart=restart)
    E, v, S = fields(geo, P, pot_kinds, pot_values, mobility, a, b, ne)
    phi = fv.face_velocity_flux(geo, v)
    dt = fv.cfl_dt(geo, phi, D, cfl, kinds)
    ne_new = fv.rk3_step(geo, ne, dt, phi, D, kinds, values, source=S)
    return ne_new, n_ion + dt * S, P, E, dt, it
