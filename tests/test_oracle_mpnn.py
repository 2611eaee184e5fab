"""Pins of the learned preconditioner's oracle network: the hand-derived
backward against central finite differences (FP64), the neighbour
aggregation against its adjoint, homogeneity in r, and the start as Jacobi."""
import numpy as np

from conftest import cube, cube_geometry
from oracle import mpnn, poisson
from oracle.geometry import DIRICHLET


def setup(n=3, seed=2):
    geo = cube_geometry(n, seed)
    K, _ = poisson.assemble(geo, [DIRICHLET] * 6, [0.0] * 6)
    dinv = 1.0 / K.diagonal()
    nbr = mpnn.face_neighbours(geo)
    r = np.random.default_rng(1).normal(size=geo.nc)
    return geo, K, dinv, nbr, r


import pytest


@pytest.mark.parametrize("kind", ["residual", "energy"])
def test_backward_matches_finite_differences(kind):
    geo, K, dinv, nbr, r = setup()
    p = mpnn.init_params(seed=3, scale=0.3)
    rng = np.random.default_rng(4)
    for k in ("wd", "bd", "be"):
        p[k] = rng.normal(0, 0.3, np.shape(p[k]))
    for l in range(mpnn.LAYERS):
        p[f"b1_{l}"] = rng.normal(0, 0.3, mpnn.H)
        p[f"b2_{l}"] = rng.normal(0, 0.3, mpnn.H)
    L, g = mpnn.loss_and_grad(p, K, r, dinv, nbr, kind=kind)
    v = mpnn.flatten(p)
    gv = mpnn.flatten(g)
    idx = rng.choice(len(v), 60, replace=False)
    eps = 1e-6
    for i in idx:
        vp, vm = v.copy(), v.copy()
        vp[i] += eps
        vm[i] -= eps
        Lp, _ = mpnn.loss_and_grad(mpnn.unflatten(vp, p), K, r, dinv, nbr, kind=kind)
        Lm, _ = mpnn.loss_and_grad(mpnn.unflatten(vm, p), K, r, dinv, nbr, kind=kind)
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - gv[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gv[i])


def test_aggregation_adjoint():
    geo, K, dinv, nbr, r = setup(4, 5)
    rng = np.random.default_rng(6)
    h = rng.normal(size=(geo.nc, 3))
    g = rng.normal(size=(geo.nc, 3))
    lhs = np.sum(mpnn._neigh_mean(h, nbr) * g)
    rhs = np.sum(h * mpnn._neigh_scatter(g, nbr, geo.nc))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # the face-neighbour relation is symmetric
    pairs = {(i, j) for i in range(geo.nc) for j in nbr[i] if j >= 0}
    assert all((j, i) in pairs for i, j in pairs)


def test_homogeneous_and_starts_as_jacobi():
    geo, K, dinv, nbr, r = setup()
    p = mpnn.init_params(seed=7, scale=0.3)
    z0, _ = mpnn.forward(p, r, dinv, nbr)
    assert np.allclose(z0, dinv * r, rtol=0, atol=0)          # decoder starts at 0
    p["wd"] = np.random.default_rng(8).normal(0, 0.3, mpnn.H)
    z1, _ = mpnn.forward(p, r, dinv, nbr)
    z2, _ = mpnn.forward(p, 3.5 * r, dinv, nbr)
    assert np.allclose(z2, 3.5 * z1, rtol=1e-12, atol=0)


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.0e-3])
    b = mpnn.bf16(x)
    assert b[0] == 1.0 and b[1] == 1.0          # tie to even
    assert b[2] == 1.0 + 2 ** -7                # rounds up
    assert b[3] == -2.5
    assert abs(b[4] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_energy_loss_is_the_energy_norm_of_the_error_up_to_a_constant():
    """(z^T K z - 2 z^T r) / r^T D^-1 r = (||z - e||^2_Ks - ||e||^2_Ks) / r^T D^-1 r
    with e = Ks^-1 r, for any z (here: two different networks)."""
    import scipy.sparse.linalg as spla
    geo, K, dinv, nbr, r = setup()
    Ks = ((K + K.T) * 0.5).tocsc()
    e = spla.spsolve(Ks, r)
    rdr = np.dot(r, dinv * r)
    for seed in (1, 2):
        p = mpnn.init_params(seed=seed, scale=0.3)
        p["wd"] = np.random.default_rng(seed).normal(0, 0.3, mpnn.H)
        L, _ = mpnn.loss_and_grad(p, K, r, dinv, nbr, kind="energy")
        z, _ = mpnn.forward(p, r, dinv, nbr)
        d = z - e
        want = (np.dot(d, Ks @ d) - np.dot(e, Ks @ e)) / rdr
        assert abs(L - want) <= 1e-10 * max(1.0, abs(want))
