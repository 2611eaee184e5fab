"""Boundary of the library, through the C-ABI: per-face boundary values
(the Annexes' per-name values generalised to data that varies along a wall),
field element types, captured graphs that follow later boundary-condition
and CFL changes, and the matrix-free solve on a mesh without the stored
Poisson matrix (no assembly)."""
import numpy as np
import pytest

import synth
from conftest import cube, cube_geometry
from oracle import fv, poisson
from oracle.geometry import ZERO_FLUX, NEUMANN, DIRICHLET, PerFace

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_2203_00925_amd.binding")

TOL = 1e-12
TOL32 = 1e-5


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _setup_scalar(st, pf):
    st.set_field(B.FIELD_VEL, dev(np.ascontiguousarray(pf.vel.T.ravel())))
    st.set_field(B.FIELD_U, dev(pf.u0))


def _mixed_per_face(m, rng):
    """Kinds per tag; Dirichlet data varying per face on x0 and y1, Neumann
    data per face on x1, per-tag values elsewhere."""
    kinds = [DIRICHLET, NEUMANN, ZERO_FLUX, DIRICHLET, NEUMANN, DIRICHLET]
    tag_vals = [0.0, 0.0, 0.0, 0.0, 0.3, -0.5]
    per_tag = {0: rng.uniform(-1, 1, len(m.btags)), 1: rng.uniform(-0.5, 0.5, len(m.btags)),
               3: rng.uniform(0, 2, len(m.btags))}
    full = np.asarray(tag_vals, np.float64)[m.btags]
    for t, v in per_tag.items():
        full[m.btags == t] = v[m.btags == t]
    return kinds, tag_vals, per_tag, PerFace(full)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_per_face_scalar_values_step_and_residual(precision):
    """Steps and the residual with per-face Dirichlet and Neumann data equal
    the oracle run with the same data (FP64 to 1e-12; the FP32 form states
    its error against it)."""
    print(f"[gpu] per-face scalar values, {precision}", flush=True)
    n, seed = 5, 3
    m = cube(n, seed)
    geo = cube_geometry(n, seed)
    pf = synth.problem_fields(m, diffusivity=1e-2)
    rng = np.random.default_rng(31)
    kinds, tag_vals, per_tag, data = _mixed_per_face(m, rng)
    prec = B.FP32 if precision == "fp32" else B.FP64
    st = B.State(B.Mesh.from_cube(m), diffusivity=pf.diffusivity, precision=prec)
    st.set_bcs(B.VAR_SCALAR, kinds, tag_vals)
    for t, v in per_tag.items():
        st.set_bc_values(B.VAR_SCALAR, t, dev(v))
    _setup_scalar(st, pf)
    phi = fv.face_velocity_flux(geo, pf.vel)
    tol = TOL32 if precision == "fp32" else TOL
    if precision == "fp64":
        got = st.residual()
        ref, parts = fv.residual(geo, pf.u0, phi, pf.diffusivity, kinds, data, parts=True)
        assert rel(host(got["res"]), ref) < tol
    dt = fv.cfl_dt(geo, phi, pf.diffusivity, 0.4, kinds)
    st.step(3, dt)
    u = pf.u0
    for _ in range(3):
        u = fv.rk3_step(geo, u, dt, phi, pf.diffusivity, kinds, data)
    err = rel(host(st.get_field(B.FIELD_U)), u)
    print(f"[gpu] 3 steps, per-face data: error {err:.2e} ({precision})", flush=True)
    assert err < tol
    if precision == "fp64":   # the per-tag values alone give another answer: the data were read
        u_tag = pf.u0
        for _ in range(3):
            u_tag = fv.rk3_step(geo, u_tag, dt, phi, pf.diffusivity, kinds, tag_vals)
        assert rel(u_tag, u) > 1e-8


def _foot_values(geo, a, b0):
    """A linear field's value at each ghost's foot point (the owner centre
    projected on the face plane), per boundary triangle of the mesh."""
    f = geo.gface
    nrm = geo.fS[f] / np.linalg.norm(geo.fS[f], axis=1)[:, None]
    xL = geo.xc[geo.gowner]
    foot = xL - np.einsum("ij,ij->i", xL - geo.fx[f], nrm)[:, None] * nrm
    vals = np.empty(geo.nb)
    vals[geo.gbtri] = b0 + foot @ a
    return vals


@pytest.mark.parametrize("no_matrix", [False, True])
def test_per_face_potential_values_and_assembly_free_solve(no_matrix):
    """Dirichlet data of a linear potential at the foot points, per face: the
    matrix-free solve of Delta P = 0 (on a mesh without the stored matrix: no
    assembly) reproduces the linear field, and the oracle's own K and c with
    the same per-face data accept it."""
    print(f"[gpu] per-face potential data, no_matrix={no_matrix}", flush=True)
    n, seed = 5, 4
    m = cube(n, seed)
    geo = cube_geometry(n, seed)
    a, b0 = np.array([1.2, -0.4, 0.9]), 0.5
    vals = _foot_values(geo, a, b0)
    st = B.State(B.Mesh.from_cube(m, no_matrix=no_matrix))
    st.set_bcs(B.VAR_POTENTIAL, [DIRICHLET] * 6)
    for t in range(6):
        st.set_bc_values(B.VAR_POTENTIAL, t, dev(vals))
    f = np.zeros(geo.nc)
    info = st.poisson_solve(dev(f), tol=1e-12, matrix_free=True)
    assert info["status"] == B.OK
    K, c = poisson.assemble(geo, [DIRICHLET] * 6, PerFace(vals))
    x = host(st.get_field(B.FIELD_P))
    assert poisson.true_relative_residual(K, poisson.rhs(geo, f, c), x) <= 1.01e-12
    assert rel(x, b0 + geo.xc[:geo.nc] @ a) < 1e-9
    # b = -mu f + c on the GPU equals the oracle's c
    assert rel(host(st.poisson_rhs(dev(f))), c) < TOL


def test_assembly_free_solve_equals_assembled_one():
    """A mesh preprocessed without the stored matrix: smaller workspace,
    assembly and stored-matrix solves refused, and the matrix-free plain and
    FP32-refined solves (diagonal, D^-1 and c from the discretisation) accepted
    by the oracle's K, with the same right-hand side (to rounding) and the same
    solution as the matrix-free solve of an assembled state."""
    n, seed = 20, 1
    m = cube(n, seed)
    geo = cube_geometry(n, seed)
    full = B.Mesh.from_cube(m)
    lean = B.Mesh.from_cube(m, no_matrix=True)
    print(f"[gpu] workspace {full.info.ws_bytes} -> {lean.info.ws_bytes} bytes", flush=True)
    assert lean.info.matrix_padded == 0
    assert full.info.ws_bytes - lean.info.ws_bytes >= 10 * full.info.matrix_padded
    kinds, vals = [DIRICHLET, DIRICHLET, NEUMANN, NEUMANN, DIRICHLET, ZERO_FLUX], [1.0, 0.0, 0.2, 0.0, -1.0, 0.0]
    sa, sl = B.State(full), B.State(lean)
    for s in (sa, sl):
        s.set_bcs(B.VAR_POTENTIAL, kinds, vals)
    with pytest.raises(B.MifvmError):
        sl.poisson_assemble()
    f = synth.gaussian_field(m)
    with pytest.raises(B.MifvmError):
        sl.poisson_solve(dev(f))                     # the stored K does not exist
    sa.poisson_assemble()
    # the same sums in the same order (the off-diagonal ones dropped)
    assert rel(host(sl.poisson_rhs(dev(f))), host(sa.poisson_rhs(dev(f)))) < 1e-14
    ia = sa.poisson_solve(dev(f), tol=1e-10, matrix_free=True)
    il = sl.poisson_solve(dev(f), tol=1e-10, matrix_free=True)
    print(f"[gpu] matrix-free solve: assembled {ia['iterations']} it, without matrix {il['iterations']} it",
          flush=True)
    K, c = poisson.assemble(geo, kinds, vals)
    b = poisson.rhs(geo, f, c)
    xl = host(sl.get_field(B.FIELD_P))
    assert poisson.true_relative_residual(K, b, xl) <= 1.01e-10
    assert abs(ia["iterations"] - il["iterations"]) <= 2
    assert rel(xl, host(sa.get_field(B.FIELD_P))) < 1e-8
    sl.set_field(B.FIELD_P, dev(np.zeros(geo.nc)))
    ir = sl.poisson_solve(dev(f), tol=1e-10, matrix_free=True, method=B.SOLVE_IR_FP32)
    assert ir["status"] == B.OK
    assert poisson.true_relative_residual(K, b, host(sl.get_field(B.FIELD_P))) <= 1.01e-10


def test_step_graph_follows_bc_and_cfl_changes():
    """A captured step graph holds boundary kinds and the CFL factor by value:
    after set_bc (kind and value) and a new CFL factor the replay must equal
    direct steps and the oracle; per-face values set between replays are read
    by the replay without a new capture."""
    print("[gpu] step graph across BC and CFL changes", flush=True)
    n, seed = 5, 3
    m = cube(n, seed)
    geo = cube_geometry(n, seed)
    pf = synth.problem_fields(m, diffusivity=1e-2)
    kinds = [DIRICHLET, ZERO_FLUX, NEUMANN, ZERO_FLUX, DIRICHLET, ZERO_FLUX]
    vals = [1.0, 0.0, 0.0, 0.0, 0.5, 0.0]
    sg, sd = (B.State(B.Mesh.from_cube(m), diffusivity=pf.diffusivity) for _ in range(2))
    for s in (sg, sd):
        s.set_bcs(B.VAR_SCALAR, kinds, vals)
        _setup_scalar(s, pf)
    phi = fv.face_velocity_flux(geo, pf.vel)
    u = pf.u0.copy()

    def run(cfl, kinds, data):
        nonlocal u
        dts = [s.cfl_dt(cfl) for s in (sg, sd)]
        sg.step_graph(2, 0.0)
        sd.step(2, 0.0)
        dt = fv.cfl_dt(geo, phi, pf.diffusivity, cfl, kinds)
        assert abs(dts[0] - dt) <= 1e-14 * dt
        for _ in range(2):
            u = fv.rk3_step(geo, u, dt, phi, pf.diffusivity, kinds, data)
        ug, ud = host(sg.get_field(B.FIELD_U)), host(sd.get_field(B.FIELD_U))
        assert np.array_equal(ug, ud)
        assert rel(ug, u) < TOL

    run(0.4, kinds, vals)
    kinds2, vals2 = list(kinds), list(vals)
    kinds2[1], vals2[1] = DIRICHLET, -0.75                 # a kind and a value change
    vals2[0] = 2.0
    for s in (sg, sd):
        s.set_bc(B.VAR_SCALAR, 1, DIRICHLET, -0.75)
        s.set_bc(B.VAR_SCALAR, 0, DIRICHLET, 2.0)
    run(0.2, kinds2, vals2)
    # values only (no new capture needed): per-face data on tag 4
    v4 = np.random.default_rng(5).uniform(0, 1, len(m.btags))
    for s in (sg, sd):
        s.set_bc_values(B.VAR_SCALAR, 4, dev(v4))
    full = np.asarray(vals2, np.float64)[m.btags]
    full[m.btags == 4] = v4[m.btags == 4]
    run(0.2, kinds2, PerFace(full))


def test_graph_solve_follows_potential_bc_change():
    """Matrix-free solves replayed from captured graphs, before and after the
    potential's boundary conditions change (kinds held by value in the graph)
    and the system is assembled again: each equals the direct-launch solve
    bitwise and is accepted by the oracle's K for the conditions of the time."""
    print("[gpu] graph solve across a potential BC change", flush=True)
    n, seed = 5, 3
    m = cube(n, seed)
    geo = cube_geometry(n, seed)
    f = synth.gaussian_field(m)
    sg, sd = B.State(B.Mesh.from_cube(m)), B.State(B.Mesh.from_cube(m))
    for kinds, vals in (([DIRICHLET] * 6, [0.0] * 6),
                        ([DIRICHLET, NEUMANN, DIRICHLET, NEUMANN, ZERO_FLUX, DIRICHLET],
                         [1.0, 0.5, -1.0, 0.0, 0.0, 0.25])):
        for s in (sg, sd):
            s.set_bcs(B.VAR_POTENTIAL, kinds, vals)
            s.poisson_assemble()
            s.set_field(B.FIELD_P, dev(np.zeros(geo.nc)))
        ig = sg.poisson_solve(dev(f), tol=1e-10, matrix_free=True, graph=1, chunk=8)
        idr = sd.poisson_solve(dev(f), tol=1e-10, matrix_free=True, graph=0, chunk=8)
        xg, xd = host(sg.get_field(B.FIELD_P)), host(sd.get_field(B.FIELD_P))
        assert ig["iterations"] == idr["iterations"] and np.array_equal(xg, xd)
        K, c = poisson.assemble(geo, kinds, vals)
        assert poisson.true_relative_residual(K, poisson.rhs(geo, f, c), xg) <= 1.01e-10


def test_field_element_types():
    """float32 fields at the ABI: an FP64 state takes them widened exactly and
    returns float32 by rounding; an FP32 state round-trips float32 bitwise and
    steps from float32 data exactly as from the same values in float64."""
    print("[gpu] field element types", flush=True)
    m = cube(4, 2)
    pf = synth.problem_fields(m, diffusivity=1e-2)
    u32 = pf.u0.astype(np.float32)
    s64 = B.State(B.Mesh.from_cube(m), diffusivity=pf.diffusivity)
    s64.set_field(B.FIELD_U, dev(u32, torch.float32))
    assert np.array_equal(host(s64.get_field(B.FIELD_U)), u32.astype(np.float64))
    s64.set_field(B.FIELD_U, dev(pf.u0))
    assert np.array_equal(host(s64.get_field(B.FIELD_U, dtype=torch.float32)), pf.u0.astype(np.float32))
    sa, sb = (B.State(B.Mesh.from_cube(m), diffusivity=pf.diffusivity, precision=B.FP32) for _ in range(2))
    sa.set_field(B.FIELD_U, dev(u32, torch.float32))
    sb.set_field(B.FIELD_U, dev(u32.astype(np.float64)))
    assert np.array_equal(host(sa.get_field(B.FIELD_U, dtype=torch.float32)), u32)
    for s in (sa, sb):
        s.set_bcs(B.VAR_SCALAR, [ZERO_FLUX] * 6)
        s.set_field(B.FIELD_VEL, dev(np.ascontiguousarray(pf.vel.T.ravel()), torch.float32))
        s.step(2, 1e-4)
    assert np.array_equal(host(sa.get_field(B.FIELD_U, dtype=torch.float32)),
                          host(sb.get_field(B.FIELD_U, dtype=torch.float32)))
    rc = B.lib().mifvm_set_field(sa._h, B.FIELD_U, B._ptr(dev(u32, torch.float32)), 7, None)
    assert rc == -1                                          # E_ARG: unknown dtype
