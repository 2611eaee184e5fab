"""Per-step and per-solve run records as JSON lines.

One record per line, each a JSON object with a ``kind`` field:

* ``"step"``: an explicit step (eqs. (4), (6)): step number, simulated time,
  the step's dt, the conservation total sum(mu_i u_i) after it and its drift
  from the initial total (given, else the first logged one), the step's GPU milliseconds and the resulting
  cell-updates per second;
* ``"solve"``: a Poisson solve (Sec. 3.4): method, iterations, restarts,
  outer refinement steps, fallbacks, the final relative true residual, the
  residual history when one was recorded, milliseconds, and the achieved
  GB/s when the caller gives the algorithmic bytes of one iteration;
* ``"run"``: free-form run metadata (workload, mesh sizes, options).

The records hold only numbers the library returned; nothing here computes
any part of the method.  ``read`` parses a log back into a list of dicts.
"""
from __future__ import annotations

import json
import math
import time

SOLVE_METHODS = {0: "jacobi_cg", 1: "ir_fp32", 2: "learned_fcg", 3: "fgmres", 4: "multigrid_fcg"}


def _clean(v):
    """JSON-safe copy: non-finite floats become strings (JSON has no NaN)."""
    if isinstance(v, float) and not math.isfinite(v):
        return repr(v)
    if isinstance(v, dict):
        return {str(k): _clean(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [_clean(x) for x in v]
    if hasattr(v, "item") and callable(v.item):           # numpy / torch scalars
        return _clean(v.item())
    return v


class RunLog:
    """Appends JSON-lines records to ``path`` (or to an open text file).

    ``cells`` is the number of cells one step updates (used for the
    cell-updates/s of step records); ``conservation0`` the total the drift
    is measured from (default: the first logged one)."""

    def __init__(self, path_or_file, cells=None, conservation0=None, flush=True):
        if hasattr(path_or_file, "write"):
            self._fh, self._own = path_or_file, False
        else:
            self._fh, self._own = open(path_or_file, "a", encoding="utf-8"), True
        self.cells = cells
        self.flush = flush
        self.t_sim = 0.0
        self.total0 = conservation0
        self.t0 = time.time()

    def _write(self, rec):
        rec = dict(rec)
        rec.setdefault("wall_s", round(time.time() - self.t0, 6))
        self._fh.write(json.dumps(_clean(rec), sort_keys=False) + "\n")
        if self.flush:
            self._fh.flush()

    def run(self, **meta):
        self._write({"kind": "run", **meta})

    def step(self, step, dt, conservation=None, ms=None, n_steps=1, **extra):
        """Record ``n_steps`` RK3 steps ending at step number ``step``."""
        self.t_sim += dt * n_steps
        rec = {"kind": "step", "step": int(step), "n_steps": int(n_steps), "t": self.t_sim, "dt": dt}
        if conservation is not None:
            if self.total0 is None:
                self.total0 = conservation
            rec["conservation"] = conservation
            rec["conservation_rel_drift"] = (abs(conservation - self.total0) / abs(self.total0)
                                             if self.total0 else 0.0)
        if ms is not None:
            rec["ms"] = ms
            if self.cells and ms > 0:
                rec["cell_updates_per_s"] = self.cells * n_steps / (ms * 1e-3)
        rec.update(extra)
        self._write(rec)

    def solve(self, step, info, method=0, bytes_per_iteration=None, ms=None, **extra):
        """Record one solve from the dict ``State.poisson_solve`` returns.
        ``ms`` overrides the library's own timing (e.g. an event pair)."""
        ms = info.get("ms") if ms is None else ms
        its = int(info.get("iterations", 0))
        rec = {"kind": "solve", "step": int(step), "method": SOLVE_METHODS.get(method, str(method)),
               "status": int(info.get("status", 0)), "iterations": its,
               "restarts": int(info.get("restarts", 0)), "outer": int(info.get("outer", 0)),
               "fell_back": int(info.get("fell_back", 0)),
               "learned_iterations": int(info.get("learned_iterations", 0)),
               "rel_residual": info.get("rel_residual"), "ms": ms}
        hist = info.get("history")
        if hist:
            rec["residual_history"] = list(hist)
        if bytes_per_iteration and ms and its > 0:
            rec["GBps"] = bytes_per_iteration * its / (ms * 1e-3) / 1e9
        rec.update(extra)
        self._write(rec)

    def close(self):
        if self._own:
            self._fh.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def read(path):
    """Records of a JSON-lines log, in order."""
    with open(path, encoding="utf-8") as fh:
        return [json.loads(ln) for ln in fh if ln.strip()]
