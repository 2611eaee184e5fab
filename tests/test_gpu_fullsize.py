"""Parity at the benchmark's full size (10,368,000-cell jittered cube, the
kernels and launch configuration bench.py times): the oracle evaluates a
sample of cells one by one from their two-vertex-ring neighbourhood
(oracle/local.py, pinned against the global oracle), plus properties that
hold at any size (conservation, the solver's true residual)."""
import os

import numpy as np
import pytest

import synth
from oracle import local
from oracle.geometry import ZERO_FLUX, DIRICHLET

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_2203_00925_amd.binding")

N, SEED = 120, 2


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    print(f"[gpu] full-size parity: building the n={N} mesh", flush=True)
    m = synth.jittered_cube(N, SEED)
    pf = synth.problem_fields(m)
    st = B.State(B.Mesh.from_cube(m), diffusivity=pf.diffusivity)
    st.set_bcs(B.VAR_SCALAR, [ZERO_FLUX] * 6)
    st.set_bcs(B.VAR_POTENTIAL, [DIRICHLET] * 6)
    st.set_field(B.FIELD_VEL, torch.from_numpy(np.ascontiguousarray(pf.vel.T.ravel())))
    st.set_field(B.FIELD_U, torch.from_numpy(pf.u0))
    vidx = local.VertexIndex(m.tets, m.nv)
    yield m, pf, st, vidx
    del st
    torch.cuda.empty_cache()


def sample(m, pf, k=160):
    rng = np.random.default_rng(77)
    nc = m.nc
    # where the pulse is, anywhere, and next to the walls
    hot = np.argsort(-pf.u0)[:200000]
    lat = m.xyz[m.tets].mean(axis=1)
    wall = np.nonzero(np.any((lat < 0.004) | (lat > 0.996), axis=1))[0]
    cells = np.concatenate([rng.choice(hot, k // 2, replace=False),
                            rng.choice(nc, k // 4, replace=False),
                            rng.choice(wall, k // 4, replace=False)])
    return np.unique(cells)


def test_fullsize_residual_sampled(big):
    m, pf, st, vidx = big
    out = st.residual()
    res = out["res"].cpu().numpy()
    cells = sample(m, pf)
    ref = local.residual_at(m, vidx, cells, pf.u0, pf.vel, pf.diffusivity, [ZERO_FLUX] * 6, [0.0] * 6)
    scale = np.abs(res).max()
    err = np.abs(res[cells] - ref).max() / scale
    print(f"[gpu] full-size residual: {len(cells)} sampled cells, max err / max|Res| = {err:.2e}")
    assert err < 1e-12


def test_fullsize_matrix_rows_sampled(big):
    m, pf, st, vidx = big
    st.poisson_assemble()
    x = np.random.default_rng(5).normal(size=m.nc)
    y = st.poisson_apply(torch.from_numpy(x)).cpu().numpy()
    cells = sample(m, pf, 96)
    kx, _ = local.matrix_rows_times(m, vidx, cells, x, [DIRICHLET] * 6, [0.0] * 6)
    err = np.abs(y[cells] - kx).max() / np.abs(y).max()
    print(f"[gpu] full-size K x: {len(cells)} sampled rows, max err / max|Kx| = {err:.2e}")
    assert err < 1e-12


def test_fullsize_step_and_residual_after_it(big):
    """One step as the bench launches it (the captured step graph at the CFL
    time step) from the initial field: u at sampled cells against the
    oracle's step from each cell's six-vertex-ring neighbourhood, then the
    residual of the stepped field against the oracle's on that field."""
    m, pf, st, vidx = big
    st.set_field(B.FIELD_U, torch.from_numpy(pf.u0))
    dt = st.cfl_dt(pf.cfl)
    st.step_graph(1, 0.0)
    u1 = st.get_field(B.FIELD_U).cpu().numpy()
    cells = sample(m, pf, 16)
    ref = local.step_at(m, vidx, cells, pf.u0, pf.vel, pf.diffusivity, [ZERO_FLUX] * 6, [0.0] * 6, dt)
    # the step moves u by about dt |Res| (1e-5 here): compare the increments,
    # allowing the final FP64 rounding of u on each side (an ulp of max|u|)
    du, du_ref = u1[cells] - pf.u0[cells], ref - pf.u0[cells]
    scale = np.abs(u1 - pf.u0).max()
    err = np.abs(du - du_ref).max()
    print(f"[gpu] full-size step: {len(cells)} sampled cells, max |du - du_ref| = {err:.2e} "
          f"(max|du| {scale:.2e})", flush=True)
    assert err <= 1e-12 * scale + 2.0 ** -51 * np.abs(u1).max()
    res = st.residual()["res"].cpu().numpy()
    cells = sample(m, pf, 80)
    ref = local.residual_at(m, vidx, cells, u1, pf.vel, pf.diffusivity, [ZERO_FLUX] * 6, [0.0] * 6)
    err = np.abs(res[cells] - ref).max() / np.abs(res).max()
    print(f"[gpu] full-size residual after the step: {len(cells)} cells, max err / max|Res| = {err:.2e}",
          flush=True)
    assert err < 1e-12


def test_fullsize_step_conserves_and_solve_converges(big):
    m, pf, st, vidx = big
    t0 = st.conservation()
    dt = st.cfl_dt(pf.cfl)
    st.step(2, dt)
    t1 = st.conservation()
    assert abs(t1 - t0) <= 1e-13 * abs(t0)
    st.poisson_assemble()
    info = st.poisson_solve(None, tol=1e-10, restart=500)
    assert info["status"] == B.OK and info["rel_residual"] <= 1e-10
    info2 = st.poisson_solve(None, tol=1e-10, method=B.SOLVE_IR_FP32, inner_tol=1e-2)
    assert info2["status"] == B.OK and info2["rel_residual"] <= 1e-10
