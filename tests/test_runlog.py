"""JSON-lines run log: records round-trip, drift and rates follow from the
numbers given, non-finite values stay valid JSON (host only)."""
import io
import json

from paper_2203_00925_amd import runlog


def test_step_and_solve_records_round_trip(tmp_path):
    path = tmp_path / "run.jsonl"
    with runlog.RunLog(str(path), cells=1000) as log:
        log.run(workload="cube", cells=1000)
        log.step(1, 0.5, conservation=2.0, ms=4.0)
        log.step(3, 0.25, conservation=2.0 + 2.0 ** -39, ms=8.0, n_steps=2)
        log.solve(3, dict(status=0, iterations=100, restarts=0, outer=0, rel_residual=9e-11, ms=50.0,
                          history=[1.0, 0.1, 1e-3], fell_back=0, learned_iterations=0),
                  method=0, bytes_per_iteration=1e6)
    recs = runlog.read(str(path))
    assert [r["kind"] for r in recs] == ["run", "step", "step", "solve"]
    s1, s2, sv = recs[1], recs[2], recs[3]
    assert s1["t"] == 0.5 and s2["t"] == 1.0            # 0.5 + 2 x 0.25
    assert s1["conservation_rel_drift"] == 0.0
    assert s2["conservation_rel_drift"] == 2.0 ** -40
    assert s1["cell_updates_per_s"] == 1000 / 4e-3
    assert s2["cell_updates_per_s"] == 2000 / 8e-3
    assert sv["method"] == "jacobi_cg" and sv["iterations"] == 100
    assert sv["residual_history"] == [1.0, 0.1, 1e-3]
    assert abs(sv["GBps"] - 1e6 * 100 / 0.05 / 1e9) < 1e-12


def test_non_finite_values_stay_json():
    buf = io.StringIO()
    log = runlog.RunLog(buf)
    log.solve(0, dict(iterations=5, rel_residual=float("nan"), ms=1.0), method=2)
    line = buf.getvalue().strip()
    rec = json.loads(line)                      # strict JSON: no bare NaN
    assert rec["rel_residual"] == "nan" and rec["method"] == "learned_fcg"
    assert "GBps" not in rec
