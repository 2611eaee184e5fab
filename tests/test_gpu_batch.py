"""Batched form: several independent meshes of uneven size in one state
(one launch per kernel for all meshes, per-mesh diffusivity, time step and
CG scalars).  Each mesh must match its own single-mesh run and the oracle."""
import numpy as np
import pytest

import synth
from conftest import cube, cube_geometry
from oracle import fv, poisson
from oracle.geometry import ZERO_FLUX, DIRICHLET

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_2203_00925_amd.binding")

TOL = 1e-12
# 384, 750 and 1,296 cells: mesh boundaries fall inside 256-row blocks
SIZES = (4, 5, 6)
SEEDS = (1000, 1001, 1002)
DIFF = (2e-3, 7e-3, 1e-4)
CENTRES = ((0.4, 0.5, 0.6), (0.55, 0.35, 0.5), (0.5, 0.5, 0.45))


def rel(a, b):
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def inputs():
    ms = [cube(n, s) for n, s in zip(SIZES, SEEDS)]
    u0 = [synth.gaussian_field(m, c, 0.15) for m, c in zip(ms, CENTRES)]
    vel = [synth.rotating_velocity(m) for m in ms]
    return ms, u0, vel


def make(mesh, u0, vel, D, precision=B.FP64):
    st = B.State(mesh, precision=precision)
    st.set_bcs(B.VAR_SCALAR, [ZERO_FLUX] * 6)
    st.set_bcs(B.VAR_POTENTIAL, [DIRICHLET] * 6)
    if np.ndim(D) == 0:
        st.set_diffusivity(D)
    else:
        st.set_mesh_diffusivity(D)
    st.set_field(B.FIELD_VEL, dev(np.concatenate([v[:, 0] for v in vel] + [v[:, 1] for v in vel]
                                                 + [v[:, 2] for v in vel])))
    st.set_field(B.FIELD_U, dev(np.concatenate(u0)))
    return st


def test_batch_steps_equal_single_runs_and_oracle():
    ms, u0, vel = inputs()
    batch = make(B.Mesh.from_batch(ms), u0, vel, DIFF)
    batch.cfl_dt(0.4)
    dts = batch.mesh_values("dt")
    batch.step(3, 0.0)                       # each mesh with its own CFL step
    ub = host(batch.get_field(B.FIELD_U))
    off = np.cumsum([0] + [m.nc for m in ms])
    for k, m in enumerate(ms):
        single = make(B.Mesh.from_cube(m), [u0[k]], [vel[k]], DIFF[k])
        dt = single.cfl_dt(0.4)
        assert abs(dt - dts[k]) <= 1e-14 * dt
        single.step(3, dt)
        us = host(single.get_field(B.FIELD_U))
        assert rel(ub[off[k]:off[k + 1]], us) < TOL
        # and the oracle
        g = cube_geometry(SIZES[k], SEEDS[k])
        phi = fv.face_velocity_flux(g, vel[k])
        u = u0[k]
        for _ in range(3):
            u = fv.rk3_step(g, u, dt, phi, DIFF[k], [ZERO_FLUX] * 6, [0.0] * 6)
        assert rel(ub[off[k]:off[k + 1]], u) < TOL
    tot = batch.conservation()
    per = batch.mesh_values("conservation")
    assert abs(tot - per.sum()) <= 1e-15 * abs(tot)


@pytest.mark.parametrize("method", [0, 1])
def test_batch_solves_each_mesh_to_tolerance(method):
    ms, u0, vel = inputs()
    batch = make(B.Mesh.from_batch(ms), u0, vel, DIFF)
    batch.poisson_assemble()
    info = batch.poisson_solve(None, tol=1e-10, method=method)
    assert info["status"] == B.OK
    its = batch.mesh_values("iterations")
    rels = batch.mesh_values("rel_residual")
    assert np.all(rels <= 1e-10)
    x = host(batch.get_field(B.FIELD_P))
    off = np.cumsum([0] + [m.nc for m in ms])
    for k, m in enumerate(ms):
        g = cube_geometry(SIZES[k], SEEDS[k])
        K, c = poisson.assemble(g, [DIRICHLET] * 6, [0.0] * 6)
        b = poisson.rhs(g, u0[k], c)
        assert poisson.true_relative_residual(K, b, x[off[k]:off[k + 1]]) <= 1.01e-10
        single = make(B.Mesh.from_cube(m), [u0[k]], [vel[k]], DIFF[k])
        single.poisson_assemble()
        si = single.poisson_solve(None, tol=1e-10, method=method)
        # the same per-mesh algorithm: iteration counts agree up to rounding
        assert abs(si["iterations"] - its[k]) <= 3
    # uneven meshes need different iteration counts, and each stopped on its own
    assert len(set(its.astype(int))) > 1


def test_graph_replays_equal_direct_launches(tmp_path):
    """A captured step graph and captured CG chunks give the same results as
    direct launches (replayed several times, with other work in between)."""
    ms, u0, vel = inputs()
    a = make(B.Mesh.from_batch(ms), u0, vel, DIFF)
    b = make(B.Mesh.from_batch(ms), u0, vel, DIFF)
    for st in (a, b):
        st.cfl_dt(0.4)
        st.poisson_assemble()
    for rep in range(3):
        a.step(2, 0.0)
        b.step_graph(2, 0.0)
        torch.cuda.synchronize()
        assert np.array_equal(host(a.get_field(B.FIELD_U)), host(b.get_field(B.FIELD_U)))
        ia = a.poisson_solve(None, tol=1e-10, chunk=16, graph=0)
        ib = b.poisson_solve(None, tol=1e-10, chunk=16, graph=1)
        assert ia["iterations"] == ib["iterations"]
        assert np.array_equal(host(a.get_field(B.FIELD_P)), host(b.get_field(B.FIELD_P)))
    # autotune: picks a schedule, restores the state, and caches the choice
    cache = str(tmp_path / "tune.json")
    u_before = host(b.get_field(B.FIELD_U))
    p_before = host(b.get_field(B.FIELD_P))
    t = b.autotune(cache)
    assert t["chunk"] in (8, 16, 32, 64) and t["from_cache"] == 0
    assert np.array_equal(host(b.get_field(B.FIELD_U)), u_before)
    assert np.array_equal(host(b.get_field(B.FIELD_P)), p_before)
    t2 = b.autotune(cache)
    assert t2["from_cache"] == 1 and t2["chunk"] == t["chunk"]
    info = b.poisson_solve(None, tol=1e-10)
    assert info["status"] == B.OK
