"""GPU path (through the C ABI) against the FP64 oracle on the same seeded
inputs.  Deterministic operators and the time step must agree norm-wise to
1e-12 (max |a - b| / max |b|); solves are accepted by the oracle's own
matrix and must follow the oracle's CG iterates."""
import numpy as np
import pytest

import synth
from conftest import cube, cube_geometry
from oracle import fv, poisson
from oracle.geometry import ZERO_FLUX, NEUMANN, DIRICHLET

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_2203_00925_amd.binding")
from mapping import Mapped  # noqa: E402

TOL = 1e-12


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


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


CASES = {
    # name: (n, seed, scalar BC kinds, values, D)
    "ragged_mixed": (5, 3, [DIRICHLET, NEUMANN, ZERO_FLUX, DIRICHLET, NEUMANN, ZERO_FLUX],
                     [0.3, -0.2, 0.0, 1.0, 0.5, 0.0], 2e-2),
    "config1": (20, 1, [ZERO_FLUX] * 6, [0.0] * 6, 1e-3),
}


def make_state(mp, kinds, vals, D, u):
    st = B.State(mp.lib, diffusivity=D)
    st.set_bcs(B.VAR_SCALAR, kinds, vals)
    st.set_field(B.FIELD_VEL, dev(synth.rotating_velocity(mp.m).T.ravel()))
    st.set_field(B.FIELD_U, dev(u))
    return st


@pytest.mark.parametrize("case", list(CASES))
def test_residual_parts(case):
    n, seed, kinds, vals, D = CASES[case]
    print(f"[gpu] residual parts case={case} n={n} seed={seed}", flush=True)
    mp = Mapped(n, seed)
    g = mp.geo
    rng = np.random.default_rng(seed)
    u = synth.gaussian_field(mp.m, (0.45, 0.5, 0.55), 0.2) + 0.05 * rng.normal(size=g.nc)
    st = make_state(mp, kinds, vals, D, u)
    out = st.residual()
    vel = synth.rotating_velocity(mp.m)
    phi = fv.face_velocity_flux(g, vel)
    res, parts = fv.residual(g, u, phi, D, kinds, vals, parts=True)
    assert rel(host(out["grad"]).T, parts["grad"]) < TOL
    assert rel(host(out["u_node"]), parts["u_node"]) < TOL
    F = np.zeros(g.nf)
    F[mp.face_map] = host(out["flux"])
    assert rel(F, parts["F"]) < TOL
    assert rel(host(out["res"]), res) < TOL
    psi = host(out["psi"])
    bad = np.abs(psi - parts["psi"]) > 1e-10
    assert bad.sum() <= max(1, g.nc // 10000), np.nonzero(bad)[0][:10]


@pytest.mark.parametrize("case", list(CASES))
def test_cfl_and_steps(case):
    n, seed, kinds, vals, D = CASES[case]
    print(f"[gpu] steps case={case}", flush=True)
    mp = Mapped(n, seed)
    g = mp.geo
    u0 = synth.gaussian_field(mp.m)
    st = make_state(mp, kinds, vals, D, u0)
    phi = fv.face_velocity_flux(g, synth.rotating_velocity(mp.m))
    dt_ref = fv.cfl_dt(g, phi, D, 0.4, kinds)
    dt = st.cfl_dt(0.4)
    assert abs(dt - dt_ref) <= 1e-14 * dt_ref
    nsteps = 10 if case == "config1" else 4
    st.step(nsteps, dt_ref)
    u_gpu = host(st.get_field(B.FIELD_U))
    u = u0.copy()
    for _ in range(nsteps):
        u = fv.rk3_step(g, u, dt_ref, phi, D, kinds, vals)
    assert rel(u_gpu, u) < TOL
    if all(k == ZERO_FLUX for k in kinds):
        t0 = fv.conservation_total(g, u0)
        tot = st.conservation()
        assert abs(tot - t0) <= 1e-13 * abs(t0)


def test_rcm_order_steps_and_norm():
    """The step under the reverse Cuthill-McKee cell order equals the oracle
    (the order is internal), and mifvm_norm_l2 is the cell-centre L2 norm
    sqrt(sum mu_i (u_i - e_i)^2) of the annex's error report."""
    n, seed, kinds, vals, D = CASES["ragged_mixed"]
    print("[gpu] rcm order steps + L2 norm", flush=True)
    mp = Mapped(n, seed, B.RENUMBER_RCM)
    g = mp.geo
    u0 = synth.gaussian_field(mp.m)
    st = make_state(mp, kinds, vals, D, u0)
    phi = fv.face_velocity_flux(g, synth.rotating_velocity(mp.m))
    dt = fv.cfl_dt(g, phi, D, 0.4, kinds)
    st.step(4, dt)
    u = u0.copy()
    for _ in range(4):
        u = fv.rk3_step(g, u, dt, phi, D, kinds, vals)
    assert rel(host(st.get_field(B.FIELD_U)), u) < TOL
    e = np.sin(g.xc[:g.nc, 0])
    ref = float(np.sqrt(np.sum(g.vol * (u - e) ** 2)))
    got = st.norm_l2(B.FIELD_U, dev(e))
    assert abs(got - ref) <= 1e-12 * ref
    assert abs(st.norm_l2(B.FIELD_U) - float(np.sqrt(np.sum(g.vol * u ** 2)))) <= 1e-12 * ref


def test_zero_steps_and_determinism():
    mp = Mapped(4, 6)
    u0 = synth.gaussian_field(mp.m)
    outs = []
    for _ in range(2):
        st = make_state(mp, [NEUMANN] * 6, [0.0] * 6, 1e-2, u0)
        st.step(0, 1e-3)
        assert np.array_equal(host(st.get_field(B.FIELD_U)), u0)
        st.step(3, 1e-3)
        outs.append(host(st.get_field(B.FIELD_U)))
    assert np.array_equal(outs[0], outs[1])


def test_selected_kernel_timing():
    """Timing a subset of kernels: only the selected ids get launches and
    time, the step's result is unchanged, and an id past the last is
    refused."""
    mp = Mapped(4, 6)
    u0 = synth.gaussian_field(mp.m)
    outs = []
    for only in (None, ["fv_cell"]):
        st = make_state(mp, [NEUMANN] * 6, [0.0] * 6, 1e-2, u0)
        st.kernel_timing(True, only=only)
        st.step(2, 1e-3)
        ks = st.kernel_stats()
        st.kernel_timing(False)
        assert ks["fv_cell"][1] == 6 and ks["fv_cell"][0] > 0.0
        assert ks["grad_limiter"][1] == (6 if only is None else 0)
        outs.append(host(st.get_field(B.FIELD_U)))
    assert np.array_equal(outs[0], outs[1])
    with pytest.raises(B.MifvmError):
        B._check(B._lib.mifvm_kernel_timing_select(st._h, 1 << len(B.KERNELS)))


POISSON = {
    "ragged_mixed": (5, 3, [DIRICHLET, NEUMANN, ZERO_FLUX, DIRICHLET, NEUMANN, DIRICHLET],
                     [1.0, 0.5, 0.0, -2.0, 0.0, 0.25]),
    "config1": (20, 1, [DIRICHLET] * 6, [0.0] * 6),
}


@pytest.mark.parametrize("case", list(POISSON))
def test_poisson_matrix_and_rhs(case):
    n, seed, kinds, vals = POISSON[case]
    print(f"[gpu] poisson matrix case={case}", flush=True)
    mp = Mapped(n, seed)
    g = mp.geo
    st = B.State(mp.lib)
    st.set_bcs(B.VAR_POTENTIAL, kinds, vals)
    st.poisson_assemble()
    K, c = poisson.assemble(g, kinds, vals)
    rng = np.random.default_rng(7)
    for _ in range(3):
        x = rng.normal(size=g.nc)
        assert rel(host(st.poisson_apply(dev(x))), K @ x) < TOL
    f = synth.gaussian_field(mp.m)
    assert rel(host(st.poisson_rhs(dev(f))), poisson.rhs(g, f, c)) < TOL


def test_cg_iterates_follow_oracle():
    n, seed, kinds, vals = POISSON["config1"]
    mp = Mapped(n, seed)
    g = mp.geo
    st = B.State(mp.lib)
    st.set_bcs(B.VAR_POTENTIAL, kinds, vals)
    st.poisson_assemble()
    f = synth.gaussian_field(mp.m)
    info = st.poisson_solve(dev(f), tol=1e-30, maxit=50, allow_not_converged=True)
    assert info["status"] == B.NOT_CONVERGED and info["iterations"] == 50
    K, c = poisson.assemble(g, kinds, vals)
    x50, it, _ = poisson.jacobi_cg(K, poisson.rhs(g, f, c), tol=1e-30, maxit=50)
    assert it == 50
    assert rel(host(st.get_field(B.FIELD_P)), x50) < TOL


def test_solve_config1_accepted_by_oracle():
    n, seed, kinds, vals = POISSON["config1"]
    mp = Mapped(n, seed)
    g = mp.geo
    st = B.State(mp.lib)
    st.set_bcs(B.VAR_POTENTIAL, kinds, vals)
    st.poisson_assemble()
    f = synth.gaussian_field(mp.m)
    info = st.poisson_solve(dev(f), tol=1e-10)
    assert info["status"] == B.OK and info["rel_residual"] <= 1e-10
    x = host(st.get_field(B.FIELD_P))
    K, c = poisson.assemble(g, kinds, vals)
    b = poisson.rhs(g, f, c)
    assert poisson.true_relative_residual(K, b, x) <= 1.01e-10
    xo, it, _ = poisson.jacobi_cg(K, b, tol=1e-10)
    assert abs(info["iterations"] - it) <= 3
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-7
    # warm start from the solution: converged before the first iteration
    again = st.poisson_solve(dev(f), tol=1e-10)
    assert again["iterations"] == 0 and again["rel_residual"] <= 1e-10


def test_annex_example_on_gpu():
    mp = Mapped(6, 3)
    st = B.State(mp.lib)
    st.set_bcs(B.VAR_POTENTIAL, [DIRICHLET, DIRICHLET, NEUMANN, NEUMANN, NEUMANN, NEUMANN],
               [10.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    st.poisson_assemble()
    info = st.poisson_solve(dev(np.zeros(mp.geo.nc)), tol=1e-13)
    assert info["status"] == B.OK
    exact = 10.0 * (1.0 - mp.geo.xc[:mp.geo.nc, 0])
    assert np.abs(host(st.get_field(B.FIELD_P)) - exact).max() < 1e-9


def test_single_hex_mesh():
    """6 cells, every cell on the boundary, one partial 64-row slice."""
    mp = Mapped(1, 9)
    g = mp.geo
    u0 = synth.gaussian_field(mp.m, sigma=0.5)
    kinds, vals = [DIRICHLET, NEUMANN, ZERO_FLUX, DIRICHLET, ZERO_FLUX, NEUMANN], [1, 0.1, 0, 0, 0, 0]
    st = make_state(mp, kinds, vals, 0.1, u0)
    phi = fv.face_velocity_flux(g, synth.rotating_velocity(mp.m))
    st.step(2, 1e-3)
    u = u0
    for _ in range(2):
        u = fv.rk3_step(g, u, 1e-3, phi, 0.1, kinds, vals)
    assert rel(host(st.get_field(B.FIELD_U)), u) < TOL


def test_error_codes():
    mp = Mapped(2, 1)
    st = B.State(mp.lib)
    with pytest.raises(B.MifvmError) as e:
        st.poisson_solve(None)
    assert e.value.code == -5
    with pytest.raises(B.MifvmError) as e:
        st.set_bc(B.VAR_SCALAR, 99, DIRICHLET, 1.0)
    assert e.value.code == -1
    with pytest.raises(B.MifvmError) as e:
        st.step(-1, 1e-3)
    assert e.value.code == -1


@pytest.mark.parametrize("inner_tol", [1e-2, 1e-4])
def test_refined_fp32_solve_accepted_by_oracle(inner_tol):
    """Precision form of the solve: FP32 inner CG inside FP64 iterative
    refinement must reach the same 1e-10 true residual, judged by the
    oracle's FP64 matrix."""
    n, seed, kinds, vals = POISSON["config1"]
    mp = Mapped(n, seed)
    g = mp.geo
    st = B.State(mp.lib)
    st.set_bcs(B.VAR_POTENTIAL, kinds, vals)
    st.poisson_assemble()
    f = synth.gaussian_field(mp.m)
    info = st.poisson_solve(dev(f), tol=1e-10, method=B.SOLVE_IR_FP32, inner_tol=inner_tol)
    assert info["status"] == B.OK and info["rel_residual"] <= 1e-10 and info["outer"] >= 2
    K, c = poisson.assemble(g, kinds, vals)
    b = poisson.rhs(g, f, c)
    x = host(st.get_field(B.FIELD_P))
    assert poisson.true_relative_residual(K, b, x) <= 1.01e-10
    xo, _, _ = poisson.jacobi_cg(K, b, tol=1e-12)
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-7


def test_refined_fp32_solve_mixed_boundaries():
    n, seed, kinds, vals = POISSON["ragged_mixed"]
    mp = Mapped(n, seed)
    st = B.State(mp.lib)
    st.set_bcs(B.VAR_POTENTIAL, kinds, vals)
    st.poisson_assemble()
    f = synth.gaussian_field(mp.m)
    info = st.poisson_solve(dev(f), tol=1e-12, method=B.SOLVE_IR_FP32)
    K, c = poisson.assemble(mp.geo, kinds, vals)
    x = host(st.get_field(B.FIELD_P))
    assert info["status"] == B.OK
    assert poisson.true_relative_residual(K, poisson.rhs(mp.geo, f, c), x) <= 1.01e-12


def test_precision_form_config1_reports_error_per_step():
    """Reduced-precision form on the 48,000-cell benchmark mesh: FP32 fluxes,
    gradients and state, FP64 conservation sum; then the FP32-refined solve
    of the potential.  The per-step error of u against the FP64 oracle is
    printed and bounded: FP32 rounding (6e-8) amplified by the gradient's
    relative coordinates (~1e-6 per step) over 10 steps gives < 1e-5."""
    mp = Mapped(20, 1)
    g = mp.geo
    pf = synth.problem_fields(mp.m)
    kinds, vals = [ZERO_FLUX] * 6, [0.0] * 6
    st = B.State(mp.lib, diffusivity=pf.diffusivity, precision=B.FP32)
    st.set_bcs(B.VAR_SCALAR, kinds, vals)
    st.set_bcs(B.VAR_POTENTIAL, [DIRICHLET] * 6)
    st.set_field(B.FIELD_VEL, dev(pf.vel.T.ravel()))
    st.set_field(B.FIELD_U, dev(pf.u0))
    phi = fv.face_velocity_flux(g, pf.vel)
    dt = fv.cfl_dt(g, phi, pf.diffusivity, 0.4, kinds)
    assert abs(st.cfl_dt(0.4) - dt) <= 1e-14 * dt
    u = pf.u0.copy()
    t0 = fv.conservation_total(g, u)
    errs = []
    for k in range(10):
        st.step(1, dt)
        u = fv.rk3_step(g, u, dt, phi, pf.diffusivity, kinds, vals)
        errs.append(rel(host(st.get_field(B.FIELD_U)), u))
    print("[gpu] fp32 form: per-step rel. error of u:", " ".join(f"{e:.2e}" for e in errs))
    assert max(errs) < 1e-5 and errs[-1] > 0
    # conservation: FP32 rounding of the state, summed in FP64
    assert abs(st.conservation() - t0) <= 1e-6 * abs(t0)
    st.poisson_assemble()
    info = st.poisson_solve(None, tol=1e-10, method=B.SOLVE_IR_FP32)
    assert info["status"] == B.OK
    K, c = poisson.assemble(g, [DIRICHLET] * 6, [0.0] * 6)
    u_gpu = host(st.get_field(B.FIELD_U))
    x = host(st.get_field(B.FIELD_P))
    assert poisson.true_relative_residual(K, poisson.rhs(g, u_gpu, c), x) <= 1.01e-10
    xo, _, _ = poisson.jacobi_cg(K, poisson.rhs(g, u, c), tol=1e-12)
    perr = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    print(f"[gpu] fp32 form: potential rel. error vs FP64 oracle {perr:.2e}")
    assert perr < 1e-4


def shuffled_cube(n=8, seed=3, window=700, rng_seed=17):
    """The cube with its cells shuffled inside consecutive windows of
    `window` cells.  Kept in this order (no renumbering), a 256-cell tile's
    stencil neighbourhood exceeds the 2,048-entity LDS cap, so preprocessing
    falls back to 64-cell tiles whose halos are larger than 8 entities per
    thread: the halo staging runs its remainder passes."""
    import dataclasses
    from oracle.geometry import build_geometry
    m = cube(n, seed)
    rng = np.random.default_rng(rng_seed)
    perm = np.arange(m.nc)
    for s in range(0, m.nc, window):
        perm[s:s + window] = rng.permutation(perm[s:s + window])
    m2 = dataclasses.replace(m, tets=np.ascontiguousarray(m.tets[perm]))
    return m2, build_geometry(m2.xyz, m2.tets, m2.btris, m2.btags)


def test_small_tiles_with_long_halos():
    """FP64 and FP32 steps, the stored-matrix and matrix-free solves on a
    mesh whose tiles hold 64 cells and up to ~1,800 halo entities (halo
    staging beyond its first 8 entities per thread), against the oracle."""
    print("[gpu] 64-cell tiles with long halos", flush=True)
    m, g = shuffled_cube()
    lib = B.Mesh.from_cube(m, B.RENUMBER_NONE)
    assert lib.info.tile_rows == 64 and lib.info.halo_max > 8 * 64
    kinds, vals, D = CASES["ragged_mixed"][2:]
    vel = synth.rotating_velocity(m)
    u0 = synth.gaussian_field(m)
    phi = fv.face_velocity_flux(g, vel)
    dt = fv.cfl_dt(g, phi, D, 0.4, kinds)
    u = u0.copy()
    for _ in range(3):
        u = fv.rk3_step(g, u, dt, phi, D, kinds, vals)
    for prec, tol in ((B.FP64, TOL), (B.FP32, 1e-5)):
        st = B.State(lib, diffusivity=D, precision=prec)
        st.set_bcs(B.VAR_SCALAR, kinds, vals)
        st.set_field(B.FIELD_VEL, dev(vel.T.ravel()))
        st.set_field(B.FIELD_U, dev(u0))
        st.step(3, dt)
        err = rel(host(st.get_field(B.FIELD_U)), u)
        print(f"[gpu] precision {prec}: step error {err:.2e}", flush=True)
        assert err < tol
    pk, pv = POISSON["ragged_mixed"][2:]
    K, c = poisson.assemble(g, pk, pv)
    b = poisson.rhs(g, u0, c)
    st = B.State(lib)
    st.set_bcs(B.VAR_POTENTIAL, pk, pv)
    st.poisson_assemble()
    its = []
    for mf in (False, True):
        st.set_field(B.FIELD_P, dev(np.zeros(m.nc)))
        info = st.poisson_solve(dev(u0), tol=1e-10, matrix_free=mf)
        assert info["status"] == B.OK
        assert poisson.true_relative_residual(K, b, host(st.get_field(B.FIELD_P))) <= 1.01e-10
        its.append(info["iterations"])
    _, it_o, _ = poisson.jacobi_cg(K, b, tol=1e-10)
    print(f"[gpu] stored / matrix-free CG {its} iterations, oracle {it_o}", flush=True)
    assert all(abs(i - it_o) <= 3 for i in its)
