"""The aggregation multigrid: the oracle pinned by the algebra's own facts,
and the library's host setup (C ABI, no GPU) against the oracle on the same
matrix: aggregates bit-exact, coarse matrices and the coarsest inverse to
rounding."""
import numpy as np
import pytest
import scipy.sparse as sp

from conftest import cube_geometry
from oracle import amg, poisson
from oracle.geometry import DIRICHLET, NEUMANN

B = pytest.importorskip("paper_2203_00925_amd.binding")

KINDS = [DIRICHLET, DIRICHLET, NEUMANN, NEUMANN, NEUMANN, NEUMANN]
VALS = [1.0, 0.0, 0.0, 0.0, 0.0, 0.0]


def poisson_K(n=8, seed=4):
    g = cube_geometry(n, seed)
    K, c = poisson.assemble(g, KINDS, VALS)
    K = sp.csr_matrix(K)
    K.sort_indices()
    return g, K, c


def laplacian_2d(m):
    """The SPD 5-point Laplacian on an m x m grid (Dirichlet)."""
    T = sp.diags([-1.0, 2.0, -1.0], [-1, 0, 1], shape=(m, m))
    I = sp.identity(m)
    return sp.csr_matrix(sp.kron(I, T) + sp.kron(T, I))


def test_aggregates_partition_and_galerkin_by_dense_products():
    _, K, _ = poisson_K()
    levels, cinv = amg.build(K, coarse_max=64)
    assert len(levels) >= 3
    for l, (A, agg) in enumerate(levels[:-1]):
        na = levels[l + 1][0].shape[0]
        assert agg.min() == 0 and agg.max() == na - 1
        assert np.all(np.bincount(agg, minlength=na) > 0)          # no empty aggregate
        assert na < 0.5 * A.shape[0]
        P = np.zeros((A.shape[0], na))
        P[np.arange(A.shape[0]), agg] = 1.0
        Ac = P.T @ A.toarray() @ P
        assert np.abs(levels[l + 1][0].toarray() - Ac).max() <= 1e-13 * np.abs(Ac).max()
    Ac = levels[-1][0].toarray()
    assert np.abs(Ac @ cinv - np.eye(Ac.shape[0])).max() < 1e-9


def test_single_level_is_the_exact_solve_and_the_cycle_is_linear():
    _, K, _ = poisson_K(4, 2)
    rng = np.random.default_rng(0)
    levels, cinv = amg.build(K, coarse_max=10**6)
    b = rng.normal(size=K.shape[0])
    assert np.abs(K @ amg.v_cycle(levels, cinv, b) - b).max() < 1e-10 * np.abs(b).max()
    levels, cinv = amg.build(K, coarse_max=32)
    b1, b2 = rng.normal(size=K.shape[0]), rng.normal(size=K.shape[0])
    lhs = amg.v_cycle(levels, cinv, 3.0 * b1 + b2)
    rhs = 3.0 * amg.v_cycle(levels, cinv, b1) + amg.v_cycle(levels, cinv, b2)
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


def test_cycle_is_symmetric_and_positive_on_an_spd_matrix():
    """With the same Jacobi sweep before and after and Galerkin coarse
    matrices, V is a symmetric positive definite operator for SPD A; a wrong
    transpose, a missing sweep or a sign error breaks it."""
    A = laplacian_2d(30)
    levels, cinv = amg.build(A, coarse_max=40)
    assert len(levels) >= 3
    rng = np.random.default_rng(1)
    x, y = rng.normal(size=A.shape[0]), rng.normal(size=A.shape[0])
    vx, vy = amg.v_cycle(levels, cinv, x), amg.v_cycle(levels, cinv, y)
    assert abs(vx @ y - x @ vy) <= 1e-12 * abs(vx @ y)
    assert vx @ x > 0 and vy @ y > 0


def test_multigrid_flexible_cg_converges_fast():
    g, K, c = poisson_K()
    f = np.sin(3.0 * g.xc[:g.nc, 0]) + g.xc[:g.nc, 1]
    b = poisson.rhs(g, f, c)
    levels, cinv = amg.build(K, coarse_max=64)
    x, it = amg.fcg(K, b, levels, cinv, tol=1e-10)
    assert poisson.true_relative_residual(K, b, x) <= 1e-10
    _, it_j, _ = poisson.jacobi_cg(K, b, tol=1e-10, restart=500)
    print(f"multigrid FCG {it} iterations, Jacobi-CG {it_j}")
    assert it < it_j / 4


def test_a_jacobi_smoother_passed_in_gives_the_plain_cycle():
    """fine = the damped Jacobi map reproduces the default cycle exactly."""
    _, K, _ = poisson_K()
    levels, cinv = amg.build(K, coarse_max=64)
    dinv = 1.0 / K.diagonal()
    b = np.random.default_rng(4).normal(size=K.shape[0])
    z0 = amg.v_cycle(levels, cinv, b)
    z1 = amg.v_cycle(levels, cinv, b, fine=lambda r: (2.0 / 3.0) * dinv * r)
    assert np.array_equal(z0, z1)


@pytest.mark.parametrize("coarse_max", [64, 300])
def test_library_setup_equals_oracle(coarse_max):
    _, K, _ = poisson_K()
    levels, cinv = amg.build(K, coarse_max=coarse_max)
    h = B.AmgHost(K.indptr, K.indices, K.data, coarse_max=coarse_max)
    assert h.info["levels"] == len(levels)
    for l, (A, agg) in enumerate(levels):
        assert h.info["rows"][l] == A.shape[0]
        if agg is not None:
            assert np.array_equal(h.export(l, "agg"), agg)
        if l > 0:
            assert np.array_equal(h.export(l, "ptr"), A.indptr)
            assert np.array_equal(h.export(l, "col"), A.indices)
            assert np.abs(h.export(l, "val") - A.data).max() <= 1e-14 * np.abs(A.data).max()
    n = levels[-1][0].shape[0]
    ci = h.export(len(levels) - 1, "cinv").reshape(n, n)
    assert np.abs(ci - cinv).max() <= 1e-9 * np.abs(cinv).max()


def test_library_setup_rejects_bad_input():
    _, K, _ = poisson_K(4, 2)
    with pytest.raises(B.MifvmError):
        B.AmgHost(K.indptr, K.indices, K.data, theta=2.0)
    with pytest.raises(B.MifvmError):
        B.AmgHost(K.indptr, K.indices, K.data, omega=2.5)          # Jacobi weight outside (0, 2)
    with pytest.raises(B.MifvmError):
        B.AmgHost(K.indptr, K.indices, K.data, coarse_max=5000)    # dense level above 4096 rows
    with pytest.raises(B.MifvmError):
        B.AmgHost(K.indptr, K.indices, K.data, coarse_max=8, max_levels=2)
    bad = K.indices.copy()
    bad[0] = K.shape[0] + 5
    with pytest.raises(B.MifvmError):
        B.AmgHost(K.indptr, bad, K.data)


def test_w_cycle_pins():
    """gamma = 2: on two levels (coarse level exact) the W-cycle is the
    V-cycle; on more levels it is still symmetric positive definite on an
    SPD matrix, equals the V-cycle followed by its defining correction on a
    three-level hierarchy, and needs fewer flexible-CG iterations."""
    A = laplacian_2d(30)
    rng = np.random.default_rng(7)
    b = rng.normal(size=A.shape[0])
    lv2, ci2 = amg.build(A, coarse_max=400)
    assert len(lv2) == 2
    assert np.array_equal(amg.v_cycle(lv2, ci2, b, gamma=2), amg.v_cycle(lv2, ci2, b))
    levels, cinv = amg.build(A, coarse_max=40)
    assert len(levels) >= 3
    x, y = rng.normal(size=A.shape[0]), rng.normal(size=A.shape[0])
    wx, wy = amg.v_cycle(levels, cinv, x, gamma=2), amg.v_cycle(levels, cinv, y, gamma=2)
    assert abs(wx @ y - x @ wy) <= 1e-12 * abs(wx @ y)
    assert wx @ x > 0 and wy @ y > 0
    assert np.abs(wx - amg.v_cycle(levels, cinv, x)).max() > 1e-6 * np.abs(wx).max()
    # three levels written out: level-1 correction = V_1(bc) + V_1(bc - A1 V_1(bc))
    lv3, ci3 = amg.build(A, coarse_max=120)
    assert len(lv3) == 3
    (A0, g0), (A1, g1) = lv3[0], lv3[1]
    d0 = 1.0 / A0.diagonal()
    w = 2.0 / 3.0
    x0 = w * d0 * b
    bc = np.bincount(g0, weights=b - A0 @ x0, minlength=A1.shape[0])
    c1 = amg.v_cycle(lv3, ci3, bc, level=1)
    c1 = c1 + amg.v_cycle(lv3, ci3, bc - A1 @ c1, level=1)
    x0 = x0 + c1[g0]
    x0 = x0 + w * d0 * (b - A0 @ x0)
    assert np.abs(amg.v_cycle(lv3, ci3, b, gamma=2) - x0).max() <= 1e-13 * np.abs(x0).max()
    _, K, c = poisson_K()
    lv, ci = amg.build(K, coarse_max=16)
    bb = rng.normal(size=K.shape[0])
    _, it_v = amg.fcg(K, bb, lv, ci, tol=1e-10)
    xw, it_w = amg.fcg(K, bb, lv, ci, tol=1e-10, gamma=2)
    assert poisson.true_relative_residual(K, bb, xw) <= 1e-10
    print(f"multigrid FCG: V {it_v}, W {it_w} iterations over {len(lv)} levels")
    assert it_w < it_v


def test_library_setup_on_threads_equals_oracle():
    """A matrix of at least 65,536 rows takes the library's threaded setup
    (strength and Galerkin product in row chunks): its aggregates and coarse
    matrices still equal the oracle's."""
    A = laplacian_2d(260)                                   # 67,600 rows
    A.sort_indices()
    levels, cinv = amg.build(A, coarse_max=256)
    h = B.AmgHost(A.indptr, A.indices, A.data, coarse_max=256)
    assert h.info["levels"] == len(levels) >= 3
    for l, (Al, agg) in enumerate(levels):
        assert h.info["rows"][l] == Al.shape[0]
        if agg is not None:
            assert np.array_equal(h.export(l, "agg"), agg)
        if l > 0:
            assert np.array_equal(h.export(l, "ptr"), Al.indptr)
            assert np.array_equal(h.export(l, "col"), Al.indices)
            assert np.abs(h.export(l, "val") - Al.data).max() <= 1e-14 * np.abs(Al.data).max()
