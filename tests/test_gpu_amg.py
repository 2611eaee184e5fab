"""Aggregation multigrid on the GPU (C ABI) against the oracle: the hierarchy
built from the GPU-assembled K (internal cell order) has the oracle's
aggregates, one V(1,1) cycle equals the oracle's cycle on the same matrix,
and the multigrid-preconditioned flexible CG is accepted by the oracle's K
in about the oracle's iteration count.

Tolerance of the cycle: the GPU's finest-level product is the matrix-free
one and the coarse levels and dense inverse are formed by other routines
than the oracle's (all equal to rounding); 1e-10 relative."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from conftest import cube
from oracle import amg, mpnn, poisson
from oracle.geometry import DIRICHLET, NEUMANN

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_2203_00925_amd.binding")
from mapping import Mapped  # noqa: E402  (after torch: the library loads with torch's HIP runtime)

KINDS = [DIRICHLET, DIRICHLET, NEUMANN, NEUMANN, NEUMANN, NEUMANN]
VALS = [1.0, 0.0, 0.0, 0.0, 0.0, 0.0]
CMAX = 64


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


def setup(n=8, seed=4):
    mp = Mapped(n, seed)
    K, c = poisson.assemble(mp.geo, KINDS, VALS)
    K = sp.csr_matrix(K)
    cp = mp.cp                                              # internal -> user
    K_int = sp.csr_matrix(K[cp][:, cp])
    K_int.sort_indices()
    st = B.State(mp.lib)
    st.set_bcs(B.VAR_POTENTIAL, KINDS, VALS)
    st.poisson_assemble()
    return mp, K, c, K_int, st


def test_cycle_matches_oracle():
    print("[gpu] multigrid cycle n=8", flush=True)
    mp, K, c, K_int, st = setup()
    info = st.amg_build(coarse_max=CMAX)
    levels, cinv = amg.build(K_int, coarse_max=CMAX)
    assert info["levels"] == len(levels) and info["rows"] == [A.shape[0] for A, _ in levels]
    rng = np.random.default_rng(3)
    for _ in range(2):
        r = rng.normal(size=mp.geo.nc)
        z = host(st.amg_apply(dev(r)))
        z_ref = np.empty_like(r)
        z_ref[mp.cp] = amg.v_cycle(levels, cinv, r[mp.cp])
        err = np.abs(z - z_ref).max() / np.abs(z_ref).max()
        print(f"[gpu] cycle error {err:.2e} over {info['levels']} levels", flush=True)
        assert err < 1e-10


@pytest.mark.parametrize("matrix_free", [False, True])
def test_multigrid_solve_accepted_by_oracle(matrix_free):
    print(f"[gpu] multigrid solve matrix_free={matrix_free}", flush=True)
    mp, K, c, K_int, st = setup()
    st.amg_build(coarse_max=CMAX)
    f = synth.gaussian_field(mp.m)
    info = st.poisson_solve(dev(f), tol=1e-10, method=B.SOLVE_AMG, matrix_free=matrix_free)
    assert info["status"] == B.OK and info["rel_residual"] <= 1e-10
    b = poisson.rhs(mp.geo, f, c)
    x = host(st.get_field(B.FIELD_P))
    assert poisson.true_relative_residual(K, b, x) <= 1.01e-10
    levels, cinv = amg.build(K_int, coarse_max=CMAX)
    _, it_ref = amg.fcg(K_int, b[mp.cp], levels, cinv, tol=1e-10)
    _, it_j, _ = poisson.jacobi_cg(K, b, tol=1e-10, restart=500)
    print(f"[gpu] multigrid FCG {info['iterations']} it (oracle {it_ref}), Jacobi-CG {it_j}", flush=True)
    assert abs(info["iterations"] - it_ref) <= 2
    assert info["iterations"] < it_j / 4
    # warm start: converged at once; captured chunks equal direct launches
    again = st.poisson_solve(dev(f), tol=1e-10, method=B.SOLVE_AMG, matrix_free=matrix_free)
    assert again["iterations"] == 0
    st.set_field(B.FIELD_P, dev(np.zeros(mp.geo.nc)))
    g1 = st.poisson_solve(dev(f), tol=1e-10, method=B.SOLVE_AMG, matrix_free=matrix_free, chunk=8, graph=1)
    x1 = host(st.get_field(B.FIELD_P))
    st.set_field(B.FIELD_P, dev(np.zeros(mp.geo.nc)))
    g0 = st.poisson_solve(dev(f), tol=1e-10, method=B.SOLVE_AMG, matrix_free=matrix_free, chunk=8, graph=0)
    assert g1["iterations"] == g0["iterations"]
    assert np.array_equal(x1, host(st.get_field(B.FIELD_P)))


def test_single_level_and_errors():
    m = cube(4, 1)                                           # 384 cells: one dense level
    st = B.State(B.Mesh.from_cube(m))
    st.set_bcs(B.VAR_POTENTIAL, KINDS, VALS)
    with pytest.raises(B.MifvmError):
        st.amg_build()                                       # not assembled
    st.poisson_assemble()
    with pytest.raises(B.MifvmError):
        st.poisson_solve(None, tol=1e-10, method=B.SOLVE_AMG)   # nothing attached
    info = st.amg_build()
    assert info["levels"] == 1
    f = synth.gaussian_field(m)
    s = st.poisson_solve(dev(f), tol=1e-10, method=B.SOLVE_AMG)
    assert s["status"] == B.OK and s["iterations"] <= 2


def random_params(seed=11, scale=0.3):
    """Random network weights with non-zero biases and decoder, rounded to
    FP32 (the GPU's master copy), as the oracle's FP64 dict."""
    rng = np.random.default_rng(seed)
    p = mpnn.init_params(seed, scale)
    for k in p:
        if k.startswith("b") or k == "wd":
            p[k] = rng.normal(0, scale, np.shape(p[k]))
    flat = mpnn.flatten(p).astype(np.float32)
    return flat, mpnn.unflatten(flat.astype(np.float64), p)


def test_learned_smoother_cycle_and_solve():
    """The network as the finest level's smoother.  With the decoder at zero
    the network is exactly z = D^-1 r, so the cycle equals the oracle's cycle
    with that smoother to rounding (1e-10) and the solve takes the oracle's
    iterations.  With random weights the cycle equals the oracle's cycle with
    the oracle network (same bf16 roundings) within the network's own forward
    tolerance (an activation near a bf16 rounding boundary may round the
    other way: about one bf16 ulp locally), and it is exactly 1-homogeneous."""
    print("[gpu] multigrid with the network as smoother", flush=True)
    mp, K, c, K_int, st = setup()
    st.amg_build(coarse_max=CMAX)
    net = B.Network(seed=3)
    flat, p = random_params()
    dinv = 1.0 / K.diagonal()
    dinv_int = 1.0 / K_int.diagonal()
    nbr = mpnn.face_neighbours(mp.geo)
    levels, cinv = amg.build(K_int, coarse_max=CMAX)
    r = np.random.default_rng(8).normal(size=mp.geo.nc)
    z_ref = np.empty_like(r)
    # decoder at zero: the Jacobi map exactly
    flat0 = flat.copy()
    flat0[mpnn.flatten(p).size - 33:] = 0.0
    net.set_params(flat0)
    net.attach(st)
    z = host(st.amg_apply(dev(r), learned_smoother=True))
    z_ref[mp.cp] = amg.v_cycle(levels, cinv, r[mp.cp], fine=lambda r_: dinv_int * r_)
    err = np.abs(z - z_ref).max() / np.abs(z_ref).max()
    print(f"[gpu] Jacobi-decoder cycle error {err:.2e}", flush=True)
    assert err < 1e-10
    f = synth.gaussian_field(mp.m)
    info = st.poisson_solve(dev(f), tol=1e-10, method=B.SOLVE_AMG, matrix_free=True, learned_smoother=True,
                            chunk=4)
    b = poisson.rhs(mp.geo, f, c)
    assert info["status"] == B.OK
    assert poisson.true_relative_residual(K, b, host(st.get_field(B.FIELD_P))) <= 1.01e-10
    _, it_ref = amg.fcg(K_int, b[mp.cp], levels, cinv, tol=1e-10, fine=lambda r_: dinv_int * r_)
    print(f"[gpu] learned-smoother solve (Jacobi decoder) {info['iterations']} it (oracle {it_ref})", flush=True)
    assert abs(info["iterations"] - it_ref) <= 2
    # random weights
    net.set_params(flat)

    def fine_int(r_int):                     # the network is equivariant: apply it in user order
        r_user = np.empty_like(r_int)
        r_user[mp.cp] = r_int
        z_user, _ = mpnn.forward(p, r_user, dinv, nbr, bf16_like_gpu=True)
        return z_user[mp.cp]

    z = host(st.amg_apply(dev(r), learned_smoother=True))
    z_ref[mp.cp] = amg.v_cycle(levels, cinv, r[mp.cp], fine=fine_int)
    err = np.linalg.norm(z - z_ref) / np.linalg.norm(z_ref)
    print(f"[gpu] learned-smoother cycle error {err:.2e} (max {np.abs(z - z_ref).max() / np.abs(z_ref).max():.2e})",
          flush=True)
    assert err < 1e-2
    assert np.array_equal(host(st.amg_apply(dev(2.0 * r), learned_smoother=True)), 2.0 * z)


def test_w_cycle_matches_oracle_and_solves():
    """cycle = W: one cycle equals the oracle's W-cycle (gamma = 2) on the
    same hierarchy to 1e-10; the flexible CG is accepted by the oracle's K in
    the oracle's iteration count; a bad cycle value is refused."""
    print("[gpu] multigrid W-cycle", flush=True)
    mp, K, c, K_int, st = setup()
    with pytest.raises(B.MifvmError):
        st.amg_build(coarse_max=16, cycle=3)
    info = st.amg_build(coarse_max=16, cycle=B.CYCLE_W)
    levels, cinv = amg.build(K_int, coarse_max=16)
    assert info["levels"] == len(levels) >= 4
    r = np.random.default_rng(9).normal(size=mp.geo.nc)
    z = host(st.amg_apply(dev(r)))
    z_ref = np.empty_like(r)
    z_ref[mp.cp] = amg.v_cycle(levels, cinv, r[mp.cp], gamma=2)
    err = np.abs(z - z_ref).max() / np.abs(z_ref).max()
    z_v = np.empty_like(r)
    z_v[mp.cp] = amg.v_cycle(levels, cinv, r[mp.cp])
    print(f"[gpu] W-cycle error {err:.2e} over {info['levels']} levels "
          f"(W - V: {np.abs(z_ref - z_v).max() / np.abs(z_ref).max():.2e})", flush=True)
    assert err < 1e-10
    f = synth.gaussian_field(mp.m)
    s = st.poisson_solve(dev(f), tol=1e-10, method=B.SOLVE_AMG, matrix_free=True)
    b = poisson.rhs(mp.geo, f, c)
    assert s["status"] == B.OK
    assert poisson.true_relative_residual(K, b, host(st.get_field(B.FIELD_P))) <= 1.01e-10
    _, it_w = amg.fcg(K_int, b[mp.cp], levels, cinv, tol=1e-10, gamma=2)
    _, it_v = amg.fcg(K_int, b[mp.cp], levels, cinv, tol=1e-10)
    print(f"[gpu] W-cycle FCG {s['iterations']} it (oracle {it_w}; V-cycle oracle {it_v})", flush=True)
    assert abs(s["iterations"] - it_w) <= 2
    # captured chunks equal direct launches
    out = []
    for graph in (1, 0):
        st.set_field(B.FIELD_P, dev(np.zeros(mp.geo.nc)))
        g = st.poisson_solve(dev(f), tol=1e-10, method=B.SOLVE_AMG, matrix_free=True, chunk=8, graph=graph)
        out.append((g["iterations"], host(st.get_field(B.FIELD_P))))
    assert out[0][0] == out[1][0] and np.array_equal(out[0][1], out[1][1])
    # other strength threshold and Jacobi weight: the oracle's hierarchy and cycle
    info = st.amg_build(coarse_max=16, cycle=B.CYCLE_W, theta=0.4, omega=0.8)
    levels, cinv = amg.build(K_int, theta=0.4, coarse_max=16)
    assert info["rows"] == [A.shape[0] for A, _ in levels]
    z = host(st.amg_apply(dev(r)))
    z_ref[mp.cp] = amg.v_cycle(levels, cinv, r[mp.cp], omega=0.8, gamma=2)
    err = np.abs(z - z_ref).max() / np.abs(z_ref).max()
    print(f"[gpu] W-cycle (theta 0.4, omega 0.8) error {err:.2e} over {info['levels']} levels", flush=True)
    assert err < 1e-10
