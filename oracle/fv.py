"""Explicit cell-centred FV residual and Runge-Kutta step (oracle; test
infrastructure only).

Residual of eq. (4): for cell i with volume mu_i,
    Res_i = -(1/mu_i) sum_f s_if F_f + S_i,
where the face flux F_f (oriented L -> R) is the upwind convective part of
eq. (15) - a MUSCL reconstruction limited by Barth-Jespersen - minus the
diffusive part D grad(u)_f . S_f with the face gradient of eq. (diamond).
The cell gradient is the least-squares gradient over the node-neighbour
stencil (Algorithm 1) and the vertex values the diamond needs are the
least-squares interpolation of Algorithm 2.  Time integration is eq. (6).

Readings where the paper is silent (listed with the rest of the design):
* Algorithm 1's "f(A_x, A_y, A_z, D)" is the solution of M_i g_i = J_i with
  M_i = sum_j d_ij d_ij^T, d_ij = x_j - x_i, J_i = sum_j d_ij (u_j - u_i);
* Barth-Jespersen (named only): u_max/u_min over the cell and its face
  neighbours (ghosts included); for each face, with Delta = g_i . r_if,
  phi = min(1, (u_max-u_i)/Delta) if Delta > 0, min(1, (u_min-u_i)/Delta) if
  Delta < 0, 1 if Delta = 0; psi_i = the minimum over the 4 faces;
* the face velocity flux is phi_f = 1/2 (V_L + V_R) . S_f (V_L . S_f on the
  boundary); upwind from L when phi_f >= 0, as printed;
* on a boundary face the ghost side is first order (u_g); a zero-flux face
  carries no flux at all, a Neumann face carries D * value * |S_f| as its
  diffusive part, a Dirichlet face uses the diamond with the ghost as R;
* eq. (6) as printed loses Delta t and the final assignment; it is read as
  u^(k) = u^n + alpha_k dt Res(u^(k-1)), alpha = (1/2, 1/2, 1),
  u^{n+1} = u^(3);
* dt = CFL * min_i mu_i / sum_{f of i, not zero-flux} (|phi_f| + D kRL_f).
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry, ZERO_FLUX, NEUMANN, DIRICHLET, ghost_coefficients, ghost_values

RK3_ALPHA = (0.5, 0.5, 1.0)


def extend_with_ghosts(geo: Geometry, u, gs, gt):
    """u_ext = [u_cells, s*u_owner + t for every ghost] (a1)."""
    return np.concatenate([u, gs * u[geo.gowner] + gt])


def cell_gradient(geo: Geometry, u_ext):
    """Least-squares cell gradient over the node-neighbour stencil
    (Algorithm 1); solves the 3x3 normal equations per cell."""
    rows = np.repeat(np.arange(geo.nc), np.diff(geo.sptr))
    d = geo.xc[geo.sidx] - geo.xc[rows]
    du = u_ext[geo.sidx] - u_ext[rows]
    M = np.empty((geo.nc, 3, 3))
    J = np.empty((geo.nc, 3))
    for a in range(3):
        J[:, a] = np.bincount(rows, weights=d[:, a] * du, minlength=geo.nc)
        for b in range(3):
            M[:, a, b] = np.bincount(rows, weights=d[:, a] * d[:, b],
                                     minlength=geo.nc)
    return np.linalg.solve(M, J[..., None])[..., 0]


def face_neighbours(geo: Geometry):
    """[Nc,4] index (cell or Nc+ghost) of the cell across each face."""
    other = np.where(geo.csign > 0, geo.fR[geo.cfaces], geo.fL[geo.cfaces])
    return other


def barth_jespersen(geo: Geometry, u_ext, grad):
    """Barth-Jespersen limiter psi_i in [0, 1] (named in Sec. 2.1)."""
    u = u_ext[:geo.nc]
    nb_vals = u_ext[face_neighbours(geo)]                       # [Nc,4]
    umax = np.maximum(u, nb_vals.max(axis=1))
    umin = np.minimum(u, nb_vals.min(axis=1))
    r = geo.fx[geo.cfaces] - geo.xc[:geo.nc][:, None, :]        # [Nc,4,3]
    delta = np.einsum("ij,ikj->ik", grad, r)
    phi = np.ones_like(delta)
    pos, neg = delta > 0, delta < 0
    up = (umax - u)[:, None] * np.ones((1, 4))
    dn = (umin - u)[:, None] * np.ones((1, 4))
    phi[pos] = np.minimum(1.0, up[pos] / delta[pos])
    phi[neg] = np.minimum(1.0, dn[neg] / delta[neg])
    return phi.min(axis=1)


def node_values(geo: Geometry, u_ext):
    """Least-squares interpolation of cell values to the vertices
    (Algorithm 2): u_v = sum_c alpha_{v,c} u_c."""
    vrow = np.repeat(np.arange(geo.nv), np.diff(geo.nptr))
    return np.bincount(vrow, weights=geo.nalpha * u_ext[geo.nidx],
                       minlength=geo.nv)


def diamond_flux(geo: Geometry, u_ext, u_node):
    """S_f . grad(u)_f with the diamond face gradient (eq. (diamond))."""
    A, B, C = geo.fabc[:, 0], geo.fabc[:, 1], geo.fabc[:, 2]
    return (geo.kAC * (u_node[A] - u_node[C]) + geo.kBC * (u_node[B] - u_node[C])
            + geo.kRL * (u_ext[geo.fR] - u_ext[geo.fL]))


def face_velocity_flux(geo: Geometry, vel):
    """phi_f = V_f . S_f with V_f = 1/2 (V_L + V_R), V_L on the boundary."""
    vel = np.asarray(vel, np.float64)
    interior = geo.fghost < 0
    vR = vel[np.where(interior, geo.fR, geo.fL)]
    vf = 0.5 * (vel[geo.fL] + vR)
    return np.einsum("ij,ij->i", vf, geo.fS)


def face_fluxes(geo: Geometry, u_ext, grad, psi, u_node, phi, D, kinds, values):
    """F_f, oriented L -> R (eq. (4) with eq. (15) and eq. (diamond))."""
    fL, fR = geo.fL, geo.fR
    interior = geo.fghost < 0
    uL = u_ext[fL] + psi[fL] * np.einsum("ij,ij->i", grad[fL], geo.fx - geo.xc[fL])
    Ri = np.where(interior, fR, 0)
    uR_rec = u_ext[Ri] + psi[Ri] * np.einsum("ij,ij->i", grad[Ri], geo.fx - geo.xc[Ri])
    uR = np.where(interior, uR_rec, u_ext[fR])      # ghost side: first order
    u_up = np.where(phi >= 0, uL, uR)
    diff = diamond_flux(geo, u_ext, u_node)
    kind = np.where(interior, DIRICHLET, np.asarray(kinds)[np.maximum(geo.ftag, 0)])
    val = np.where(interior, 0.0, ghost_values(geo, values)[np.maximum(geo.fghost, 0)])
    area = np.linalg.norm(geo.fS, axis=1)
    diff = np.where(kind == NEUMANN, val * area, diff)
    F = u_up * phi - D * diff
    return np.where(kind == ZERO_FLUX, 0.0, F)


def residual(geo: Geometry, u, phi, D, kinds, values, source=None, parts=False):
    """Res(u) of eq. (4)."""
    gs, gt = ghost_coefficients(geo, kinds, values)
    u_ext = extend_with_ghosts(geo, u, gs, gt)
    grad = cell_gradient(geo, u_ext)
    psi = barth_jespersen(geo, u_ext, grad)
    u_node = node_values(geo, u_ext)
    F = face_fluxes(geo, u_ext, grad, psi, u_node, phi, D, kinds, values)
    res = -np.sum(geo.csign * F[geo.cfaces], axis=1) / geo.vol
    if source is not None:
        res = res + source
    if parts:
        return res, dict(u_ext=u_ext, grad=grad, psi=psi, u_node=u_node, F=F)
    return res


def rk3_step(geo: Geometry, u, dt, phi, D, kinds, values, source=None,
             residual_fn=None):
    """One step of the 3-stage Runge-Kutta scheme of eq. (6)."""
    res = residual_fn or (lambda v: residual(geo, v, phi, D, kinds, values, source))
    un = np.array(u, np.float64)
    uk = un
    for a in RK3_ALPHA:
        uk = un + a * dt * res(uk)
    return uk


def cfl_dt(geo: Geometry, phi, D, cfl, kinds):
    """dt = CFL * min_i mu_i / sum_{active faces of i} (|phi_f| + D kRL_f)."""
    interior = geo.fghost < 0
    kind = np.where(interior, DIRICHLET, np.asarray(kinds)[np.maximum(geo.ftag, 0)])
    rate = np.where(kind == ZERO_FLUX, 0.0, np.abs(phi) + D * geo.kRL)
    per_cell = rate[geo.cfaces].sum(axis=1)
    return cfl * float(np.min(geo.vol / per_cell))


def conservation_total(geo: Geometry, u):
    """sum_i mu_i u_i."""
    return float(np.dot(geo.vol, u))
