"""Poisson system of the same discretisation, and its solvers (oracle; test
infrastructure only).

Sec. 2.2 discretises Delta P = f cell by cell (eq. (7)): the Laplacian of
cell i is (1/mu_i) sum_f grad(P)_f . n_f |sigma_f| with the diamond face
gradient (eq. (laplace)); vertex values come from the least-squares
interpolation.  Readings:

* rows are assembled without the 1/mu_i factor and with the sign flipped,
  K = -A_lin, b = -mu * f + (ghost constants moved to the right), so the
  diagonal is positive and the solution is unchanged;
* a Dirichlet face uses the diamond with its ghost (u_g = 2 g - u_L); a
  zero-flux / Neumann face carries its prescribed flux (0 or value*|S_f|);
* convergence is the unpreconditioned true residual
  ||b - K x||_2 <= tol ||b||_2 with tol = 1e-10 (the paper's table caption
  prints the tolerance garbled as "10e^-10").

K is not symmetric on general tetrahedra (diamond cross terms and the
least-squares vertex coupling); ``symmetry_report`` measures how far, and the
CG below is the plain textbook Jacobi-preconditioned CG regardless.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .geometry import Geometry, ZERO_FLUX, NEUMANN, DIRICHLET, ghost_coefficients, ghost_values
from .fv import extend_with_ghosts, node_values, diamond_flux


def _face_kinds(geo: Geometry, kinds, values):
    interior = geo.fghost < 0
    tag = np.maximum(geo.ftag, 0)
    kind = np.where(interior, DIRICHLET, np.asarray(kinds)[tag])
    val = np.where(interior, 0.0, ghost_values(geo, values)[np.maximum(geo.fghost, 0)])
    return kind, val


def apply_laplacian(geo: Geometry, P, kinds, values):
    """Matrix-free (A P)_i = sum_f s_if F_f(P), affine in P (ghost constants
    included): F_f = S_f . grad(P)_f (eq. (laplace)) or the prescribed flux."""
    gs, gt = ghost_coefficients(geo, kinds, values)
    P_ext = extend_with_ghosts(geo, P, gs, gt)
    Pn = node_values(geo, P_ext)
    F = diamond_flux(geo, P_ext, Pn)
    kind, val = _face_kinds(geo, kinds, values)
    area = np.linalg.norm(geo.fS, axis=1)
    F = np.where(kind == NEUMANN, val * area, F)
    F = np.where(kind == ZERO_FLUX, 0.0, F)
    return np.sum(geo.csign * F[geo.cfaces], axis=1)


def assemble(geo: Geometry, kinds, values):
    """K (CSR) and the constant vector c such that K P = -mu*f + c.

    Every face flux is a linear combination of vertex values and of P_R, P_L;
    every vertex value is a combination of cell values and ghost values; every
    ghost value is s*P_owner + t.  The coefficients are expanded and summed
    into (row, column) entries; the t-parts go to c."""
    gs, gt = ghost_coefficients(geo, kinds, values)
    kind, val = _face_kinds(geo, kinds, values)
    nc = geo.nc
    active = kind == DIRICHLET                 # faces whose flux depends on P
    # flux coefficients of each face on its "inputs"
    # vertex part: weight w_v on vertex v, for v in A, B, C
    fv_face, fv_vert, fv_w = [], [], []
    for col, w in ((0, geo.kAC), (1, geo.kBC), (2, -(geo.kAC + geo.kBC))):
        fv_face.append(np.arange(geo.nf))
        fv_vert.append(geo.fabc[:, col])
        fv_w.append(w)
    fv_face = np.concatenate(fv_face)
    fv_vert = np.concatenate(fv_vert)
    fv_w = np.concatenate(fv_w)
    keep = active[fv_face]
    fv_face, fv_vert, fv_w = fv_face[keep], fv_vert[keep], fv_w[keep]
    # expand vertex -> (entity, alpha)
    deg = np.diff(geo.nptr)[fv_vert]
    face_e = np.repeat(fv_face, deg)
    w_e = np.repeat(fv_w, deg)
    base = np.repeat(geo.nptr[fv_vert], deg)
    offs = np.arange(deg.sum()) - np.repeat(np.cumsum(deg) - deg, deg)
    ent = geo.nidx[base + offs]
    coef = w_e * geo.nalpha[base + offs]
    # two-point part: +kRL on R, -kRL on L
    af = np.nonzero(active)[0]
    face_e = np.concatenate([face_e, af, af])
    ent = np.concatenate([ent, geo.fR[af], geo.fL[af]])
    coef = np.concatenate([coef, geo.kRL[af], -geo.kRL[af]])
    # ghost entities -> owner column with factor s, constant t
    is_g = ent >= nc
    g = np.where(is_g, ent - nc, 0)
    col = np.where(is_g, geo.gowner[g], ent)
    lin = np.where(is_g, gs[g], 1.0) * coef
    const = np.where(is_g, gt[g], 0.0) * coef
    # F_f = sum lin * P_col + sum const  (+ prescribed flux on Neumann faces)
    Fc = np.bincount(face_e, weights=const, minlength=geo.nf)
    area = np.linalg.norm(geo.fS, axis=1)
    Fc = Fc + np.where(kind == NEUMANN, val * area, 0.0)
    # scatter face rows into cell rows with sign: row L (+1), row R (-1)
    rows, cols, vals = [geo.fL[face_e]], [col], [lin]
    interior_e = geo.fghost[face_e] < 0
    rows.append(geo.fR[face_e][interior_e])
    cols.append(col[interior_e])
    vals.append(-lin[interior_e])
    rows, cols, vals = map(np.concatenate, (rows, cols, vals))
    A = sp.coo_matrix((vals, (rows, cols)), shape=(nc, nc)).tocsr()
    A.sum_duplicates()
    c_face = np.sum(geo.csign * Fc[geo.cfaces], axis=1)
    K = (-A).tocsr()
    K.sort_indices()
    return K, c_face


def rhs(geo: Geometry, f, c):
    """b = -mu * f + c."""
    return -geo.vol * np.asarray(f, np.float64) + c


def jacobi_cg(K, b, x0=None, tol=1e-10, maxit=20000, restart=0, history=None):
    """Textbook preconditioned CG with the Jacobi preconditioner z = D^{-1} r.

    The loop is opened from the true residual r = b - K x; it is left when the
    recurrence residual satisfies ||r||_2 <= tol ||b||_2, when maxit
    iterations have been done, or - if restart > 0 - after `restart`
    iterations since the last opening.  It is then reopened from the true
    residual (a restart, p = D^{-1} r) unless that already meets the
    tolerance or the limit.  Returns (x, iterations, true relative residual).
    """
    b = np.asarray(b, np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.float64)
    dinv = 1.0 / K.diagonal()
    bnorm = np.linalg.norm(b)
    it = 0
    while True:
        r = b - K @ x
        if np.linalg.norm(r) <= tol * bnorm or it >= maxit:
            return x, it, float(np.linalg.norm(r) / bnorm)
        z = dinv * r
        p = z.copy()
        rz = r @ z
        since = 0
        while True:
            q = K @ p
            alpha = rz / (p @ q)
            x = x + alpha * p
            r = r - alpha * q
            it += 1
            since += 1
            if history is not None:
                history.append(x.copy())
            if (np.linalg.norm(r) <= tol * bnorm or it >= maxit
                    or (restart > 0 and since >= restart)):
                break
            z = dinv * r
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new


def jacobi_fgmres(K, b, x0=None, tol=1e-10, m=30, maxit=20000, precond=None, history=None):
    """Restarted flexible GMRES(m) with right preconditioning, the Krylov
    method of the paper's solver runs (Sec. 3.4.2), here with the Jacobi
    preconditioner z = D^{-1} v unless `precond` (a function v -> z, which may
    vary between calls) is given.

    A cycle opens from the true residual r = b - K x: v_0 = r/|r|,
    g = |r| e_0.  Step j: z_j = M(v_j), w = K z_j; classical Gram-Schmidt
    h_ij = v_i . w (i <= j, all against the same w), w -= sum h_ij v_i;
    h_{j+1,j} = |w|, v_{j+1} = w / h_{j+1,j}; the earlier Givens rotations
    are applied to column j of H, a new rotation zeroes h_{j+1,j}, and
    |g_{j+1}| is the residual norm of the least-squares iterate.  The cycle
    ends when |g_{j+1}| <= tol |b|, after m steps or at maxit; then H y = g
    (upper triangular, j+1 unknowns) and x += Z y.  The loop reopens from the
    true residual until it meets the tolerance or maxit.  `history`, if
    given, receives x after every cycle.  Returns (x, iterations, true
    relative residual)."""
    b = np.asarray(b, np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.float64)
    dinv = 1.0 / K.diagonal()
    M = precond if precond is not None else (lambda v: dinv * v)
    bnorm = np.linalg.norm(b)
    it = 0
    while True:
        r = b - K @ x
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm or it >= maxit:
            return x, it, float(beta / bnorm)
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        for j in range(m):
            z = M(V[j])
            Z.append(z)
            w = K @ z
            h = np.array([vi @ w for vi in V])        # classical: all dots against one w
            w = w - sum(hi * vi for hi, vi in zip(h, V))
            H[:j + 1, j] = h
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j])
            for i in range(j):                          # earlier rotations
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            it += 1
            if abs(g[j + 1]) <= tol * bnorm or it >= maxit:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):                 # back substitution
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + sum(yi * zi for yi, zi in zip(y, Z))
        if history is not None:
            history.append(x.copy())


def direct_solve(K, b):
    """Sparse LU solve (SuperLU), the pin for x* = K^{-1} b."""
    return spla.spsolve(K.tocsc(), b)


def true_relative_residual(K, b, x):
    return float(np.linalg.norm(b - K @ x) / np.linalg.norm(b))


def symmetry_report(K):
    """||K - K^T||_F / ||K + K^T||_F, min diagonal, and the smallest
    eigenvalue of the symmetric part (sparse Lanczos)."""
    Kt = K.T.tocsr()
    asym = spla.norm(K - Kt) / spla.norm(K + Kt)
    Ssym = ((K + Kt) * 0.5).tocsc()
    lam = spla.eigsh(Ssym, k=1, sigma=0, which="LM", return_eigenvectors=False)
    return dict(asym=float(asym), min_diag=float(K.diagonal().min()),
                lambda_min_sym=float(lam[0]))
