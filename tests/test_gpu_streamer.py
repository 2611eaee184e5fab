"""Coupled streamer-type loop (Sec. 4, eq. (10)) through the C ABI against the
oracle's loop on the same seeded inputs: n_e, n_p, the potential and the
field after three coupled steps (drift, diffusion, ionisation, charge).

Tolerance: each Poisson solve stops at a relative residual of 1e-13, so the
library's and the oracle's potentials may differ by up to cond(K) 1e-13
(their CG iterates agree to rounding, but the last iteration can fall on
either side of the test); the field is a gradient of that potential and
the step carries it into n_e and n_p.  The bound is 1e-10 relative; measured
at most 1.4e-14 (E), with equal CG iteration counts."""
import numpy as np
import pytest

import synth
from conftest import cube, cube_geometry
from oracle import poisson, streamer
from oracle.geometry import ZERO_FLUX, NEUMANN, DIRICHLET

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_2203_00925_amd.binding")

POT_KINDS = [DIRICHLET, DIRICHLET, NEUMANN, NEUMANN, NEUMANN, NEUMANN]
POT_VALS = [1.0, 0.0, 0.0, 0.0, 0.0, 0.0]
NE_KINDS = [ZERO_FLUX] * 6
NE_VALS = [0.0] * 6
PARAMS = dict(mobility=1.0, charge_scale=40.0, alpha_a=2.0, alpha_b=0.3, cfl=0.4)
D = 1e-3
TOL = 1e-10


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


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


@pytest.mark.parametrize("matrix_free", [False, True])
def test_coupled_loop_matches_oracle(matrix_free):
    n, seed, steps = 8, 4, 3
    print(f"[gpu] streamer loop n={n} seed={seed} matrix_free={matrix_free}", flush=True)
    m, g = cube(n, seed), cube_geometry(n, seed)
    rng = np.random.default_rng(seed)
    ne = synth.gaussian_field(m, (0.4, 0.5, 0.5), 0.15) + 0.1
    n_ion = ne + 0.05 * rng.uniform(size=g.nc)
    st = B.State(B.Mesh.from_cube(m), diffusivity=D)
    st.set_bcs(B.VAR_SCALAR, NE_KINDS, NE_VALS)
    st.set_bcs(B.VAR_POTENTIAL, POT_KINDS, POT_VALS)
    st.poisson_assemble()
    st.set_field(B.FIELD_U, dev(ne))
    st.set_field(B.FIELD_ION, dev(n_ion))
    st.set_field(B.FIELD_P, dev(np.zeros(g.nc)))
    info = st.streamer_step(steps, tol=1e-13, matrix_free=matrix_free, **PARAMS)
    assert info["steps"] == steps
    K, c = poisson.assemble(g, POT_KINDS, POT_VALS)
    P = np.zeros(g.nc)
    t = 0.0
    its = []
    for _ in range(steps):
        ne, n_ion, P, E, dt, it = streamer.coupled_step(
            g, ne, n_ion, P, K, c, D, NE_KINDS, NE_VALS, POT_KINDS, POT_VALS,
            PARAMS["mobility"], PARAMS["charge_scale"], PARAMS["alpha_a"], PARAMS["alpha_b"],
            PARAMS["cfl"], tol=1e-13)
        t += dt
        its.append(it)
    errs = dict(ne=rel(host(st.get_field(B.FIELD_U)), ne), ni=rel(host(st.get_field(B.FIELD_ION)), n_ion),
                P=rel(host(st.get_field(B.FIELD_P)), P),
                E=rel(host(st.get_field(B.FIELD_EFIELD)).reshape(3, g.nc).T, E))
    print(f"[gpu] streamer errors {errs}, time {info['time']:.6e} vs {t:.6e}, "
          f"CG {info['iterations_sum']} vs {sum(its)}", flush=True)
    assert all(v < TOL for v in errs.values()), errs
    assert abs(info["time"] - t) <= TOL * t
    # the loop did something: ionisation raised both densities, the field is non-uniform
    assert host(st.get_field(B.FIELD_ION)).sum() > 0 and np.abs(E[:, 1]).max() > 1e-3


def test_coupled_loop_rejects_bad_input():
    m = cube(4, 1)
    st = B.State(B.Mesh.from_cube(m), diffusivity=D)
    st.set_bcs(B.VAR_POTENTIAL, POT_KINDS, POT_VALS)
    with pytest.raises(B.MifvmError):
        st.streamer_step(1, **PARAMS)                       # not assembled
    st.poisson_assemble()
    with pytest.raises(B.MifvmError):
        st.streamer_step(1, **dict(PARAMS, cfl=0.0))
    with pytest.raises(B.MifvmError):
        st.streamer_step(1, **dict(PARAMS, mobility=-1.0))
    with pytest.raises(B.MifvmError):
        st.set_field(B.FIELD_EFIELD, dev(np.zeros(3 * m.nc)))
