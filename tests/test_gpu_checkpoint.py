"""Checkpoint and resume: 10 steps of the config-2 loop (an RK3 step, then a
Poisson solve of Delta P = u warm-started from the last P) equal, bitwise, 5
steps, a checkpoint of (u, P, dt, step) written to disk, a new mesh and state
built from scratch and loaded from the checkpoint, and 5 more steps.  The
FP32 form checkpoints its state in float32."""
import json

import numpy as np
import pytest

import synth
from conftest import cube
from oracle.geometry import ZERO_FLUX, DIRICHLET

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_2203_00925_amd.binding")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def new_state(m, pf, precision):
    st = B.State(B.Mesh.from_cube(m, no_matrix=True), diffusivity=pf.diffusivity, precision=precision)
    st.set_bcs(B.VAR_SCALAR, [ZERO_FLUX] * 6)
    st.set_bcs(B.VAR_POTENTIAL, [DIRICHLET] * 6)
    st.set_field(B.FIELD_VEL, torch.as_tensor(np.ascontiguousarray(pf.vel.T.ravel()), device="cuda"))
    return st


def run(st, steps, dt):
    its = []
    for _ in range(steps):
        st.step(1, dt)
        its.append(st.poisson_solve(None, tol=1e-10, matrix_free=True)["iterations"])
    return its


@pytest.mark.parametrize("precision", [B.FP64, B.FP32])
def test_ten_steps_equal_five_checkpoint_five(precision, tmp_path):
    print(f"[gpu] checkpoint/resume, precision {precision}", flush=True)
    m = cube(8, 1)
    pf = synth.problem_fields(m)
    ftype = torch.float32 if precision == B.FP32 else torch.float64
    # straight run
    a = new_state(m, pf, precision)
    a.set_field(B.FIELD_U, torch.as_tensor(pf.u0, device="cuda"))
    dt = a.cfl_dt(pf.cfl)
    its_a = run(a, 10, dt)
    ua, pa = a.get_field(B.FIELD_U, dtype=ftype).cpu().numpy(), a.get_field(B.FIELD_P).cpu().numpy()
    # 5 steps, checkpoint to disk
    b = new_state(m, pf, precision)
    b.set_field(B.FIELD_U, torch.as_tensor(pf.u0, device="cuda"))
    dt_b = b.cfl_dt(pf.cfl)
    its_b = run(b, 5, dt_b)
    np.save(tmp_path / "u.npy", b.get_field(B.FIELD_U, dtype=ftype).cpu().numpy())
    np.save(tmp_path / "p.npy", b.get_field(B.FIELD_P).cpu().numpy())
    (tmp_path / "meta.json").write_text(json.dumps({"step": 5, "dt": dt_b, "t": 5 * dt_b}))
    del b
    # resume in a state built from scratch
    meta = json.loads((tmp_path / "meta.json").read_text())
    c = new_state(m, pf, precision)
    c.set_field(B.FIELD_U, torch.as_tensor(np.load(tmp_path / "u.npy"), device="cuda"))
    c.set_field(B.FIELD_P, torch.as_tensor(np.load(tmp_path / "p.npy"), device="cuda"))
    its_c = run(c, 10 - meta["step"], meta["dt"])
    uc, pc = c.get_field(B.FIELD_U, dtype=ftype).cpu().numpy(), c.get_field(B.FIELD_P).cpu().numpy()
    print(f"[gpu] iterations straight {its_a}, resumed {its_b} + {its_c}", flush=True)
    assert dt_b == dt
    assert its_a == its_b + its_c
    assert np.array_equal(ua, uc) and np.array_equal(pa, pc)


def test_run_log_records_the_library_totals(tmp_path):
    """Per-step and per-solve JSON lines: the logged conservation totals are
    the library's, the drift stays at round-off (zero-flux walls conserve),
    and every solve record carries its residual history."""
    from paper_2203_00925_amd.runlog import RunLog, read
    print("[gpu] run log, 4 steps", flush=True)
    m = cube(6, 2)
    pf = synth.problem_fields(m)
    st = new_state(m, pf, B.FP64)
    st.set_field(B.FIELD_U, torch.as_tensor(pf.u0, device="cuda"))
    dt = st.cfl_dt(pf.cfl)
    total0 = st.conservation()
    path = tmp_path / "run.jsonl"
    totals = []
    with RunLog(str(path), cells=m.nc, conservation0=total0) as rl:
        rl.run(cells=m.nc, dt=dt)
        for k in range(4):
            st.step(1, dt)
            info = st.poisson_solve(None, tol=1e-10, matrix_free=True, history=64)
            totals.append(st.conservation())
            rl.step(k + 1, dt, conservation=totals[-1], ms=1.0)
            rl.solve(k + 1, info, method=B.SOLVE_PLAIN)
    recs = read(str(path))
    steps = [r for r in recs if r["kind"] == "step"]
    solves = [r for r in recs if r["kind"] == "solve"]
    assert [r["conservation"] for r in steps] == totals
    assert max(r["conservation_rel_drift"] for r in steps) < 1e-13
    assert abs(steps[-1]["t"] - 4 * dt) <= 4e-16 * 4 * dt
    for r in solves:
        assert r["rel_residual"] <= 1e-10 and r["iterations"] > 0
        assert 0 < len(r["residual_history"]) <= 64
