"""Aggregation multigrid preconditioner (oracle; test infrastructure only).

Not a method of the paper: the analogue of its fastest solver configuration
(PETSc GAMG, Sec. 3.4.2) for the Poisson system of Sec. 2.2, written as
plain (unsmoothed) aggregation.  Per level, on the matrix A (rows in order):

* strong neighbours of row i: j != i with |a_ij| >= theta max_{k != i} |a_ik|;
* aggregates, three passes over the rows in order:
  1. a row that is free and whose strong neighbours are all free becomes a
     new aggregate together with them;
  2. a row left free joins the pass-1 aggregate of its strong neighbour with
     the largest |a_ij| (the smallest j among equals), if it has one;
  3. a row still free starts a new aggregate with its still-free strong
     neighbours;
* P = the piecewise-constant prolongator (P[i, agg(i)] = 1), A_c = P^T A P;

until a level has at most coarse_max rows; that level is solved with its
exact inverse.  One V(1,1) cycle with damped Jacobi (weight w) from zero:

    x = w D^-1 b;   x += P V(P^T (b - A x));   x += w D^-1 (b - A x).

With gamma = 2 (a W-cycle) the coarse correction of every level whose
coarser level is not the exactly solved one is improved once more before
it is prolonged: with b_c = P^T (b - A x) and x_c = V(b_c),
x_c += V(b_c - A_c x_c).

Parity unpinned in the paper's sense (the paper gives no multigrid): the
pins are the algebra's own facts, checked in the tests.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def strong_neighbours(A: sp.csr_matrix, theta: float):
    out = []
    for i in range(A.shape[0]):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        vals = np.abs(A.data[A.indptr[i]:A.indptr[i + 1]])
        off = cols != i
        mx = vals[off].max() if off.any() else 0.0
        if mx > 0.0:
            keep = off & (vals >= theta * mx)
            order = np.argsort(cols[keep], kind="stable")
            out.append((cols[keep][order], vals[keep][order]))
        else:
            out.append((np.empty(0, np.int64), np.empty(0)))
    return out


def aggregate(A: sp.csr_matrix, theta: float):
    n = A.shape[0]
    S = strong_neighbours(A, theta)
    agg = np.full(n, -1, np.int64)
    na = 0
    for i in range(n):                                   # pass 1
        nb = S[i][0]
        if agg[i] < 0 and np.all(agg[nb] < 0):
            agg[i] = na
            agg[nb] = na
            na += 1
    first = agg.copy()
    for i in range(n):                                   # pass 2
        if first[i] >= 0:
            continue
        nb, w = S[i]
        cand = first[nb] >= 0
        if cand.any():
            best = np.flatnonzero(cand & (w == w[cand].max()))[0]   # smallest j among the strongest
            agg[i] = first[nb[best]]
    for i in range(n):                                   # pass 3
        if agg[i] >= 0:
            continue
        agg[i] = na
        nb = S[i][0]
        agg[nb[agg[nb] < 0]] = na
        na += 1
    return agg, na


def build(A: sp.csr_matrix, theta=0.25, coarse_max=1024, max_levels=10):
    """List of levels (A_l, agg_l) and the coarsest inverse."""
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sort_indices()
    levels = []
    while A.shape[0] > coarse_max:
        if len(levels) + 1 == max_levels:
            raise ValueError("coarsest level above coarse_max")
        agg, na = aggregate(A, theta)
        P = sp.csr_matrix((np.ones(A.shape[0]), (np.arange(A.shape[0]), agg)), shape=(A.shape[0], na))
        levels.append((A, agg))
        A = sp.csr_matrix(P.T @ A @ P)
        A.sort_indices()
    levels.append((A, None))
    return levels, np.linalg.inv(A.toarray())


def v_cycle(levels, cinv, b, omega=2.0 / 3.0, level=0, fine=None, gamma=1):
    """One cycle (V for gamma = 1, W for gamma = 2); fine (optional) is a map
    r -> correction that replaces the Jacobi sweeps on the finest level:
    x = fine(b), coarse correction, x += fine(b - A x) (a learned smoother)."""
    A, agg = levels[level]
    if agg is None:
        return cinv @ b
    dinv = 1.0 / A.diagonal()
    smooth = fine if (fine is not None and level == 0) else (lambda r: omega * dinv * r)
    x = smooth(b)
    r = b - A @ x
    Ac, agg_c = levels[level + 1]
    bc = np.bincount(agg, weights=r, minlength=Ac.shape[0])
    xc = v_cycle(levels, cinv, bc, omega, level + 1, gamma=gamma)
    if agg_c is not None:                    # the coarse level is not solved exactly
        for _ in range(gamma - 1):
            xc = xc + v_cycle(levels, cinv, bc - Ac @ xc, omega, level + 1, gamma=gamma)
    x = x + xc[agg]
    return x + smooth(b - A @ x)


def fcg(K, b, levels, cinv, x0=None, tol=1e-10, maxit=2000, restart=500, omega=2.0 / 3.0, fine=None, gamma=1):
    """Flexible CG (Polak-Ribiere beta) with one cycle as the preconditioner,
    reopened from the true residual when the recurrence meets tol or after
    `restart` iterations; returns (x, iterations).  fine, gamma: as v_cycle."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.float64)
    bb = float(b @ b)
    it = 0
    while True:
        r = b - K @ x
        if r @ r <= tol * tol * bb or it >= maxit:
            return x, it
        z = v_cycle(levels, cinv, r, omega, fine=fine, gamma=gamma)
        p = z.copy()
        rz = float(z @ r)
        since = 0
        while True:
            q = K @ p
            alpha = rz / float(p @ q)
            x = x + alpha * p
            r_old = r
            r = r - alpha * q
            it += 1
            since += 1
            if r @ r <= tol * tol * bb or it >= maxit or since >= restart:
                break
            z = v_cycle(levels, cinv, r, omega, fine=fine, gamma=gamma)
            zr, zro = float(z @ r), float(z @ r_old)
            beta = (zr - zro) / rz
            rz = zr
            p = z + beta * p
