"""The learned solve's fallback decisions (paper_2203_00925_amd/csrc/
fcg_monitor.h) driven on the host with scripted device-scalar sequences: the
stall window, a 1% drop restarting it, non-finite values at every point
where they are checked, and the three outcomes of a reopening.  No GPU: a
small host program including the header is compiled with g++."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_00925_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <limits>
#include "fcg_monitor.h"
using mifvm::FcgMonitor;
static int fails = 0;
#define EXPECT(a, b) do { int x_ = (a), y_ = (b); if (x_ != y_) { \
    std::printf("line %d: got %d, expected %d\n", __LINE__, x_, y_); ++fails; } } while (0)
int main() {
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double inf = std::numeric_limits<double>::infinity();
    {   // steady 5% drops per chunk of 8: never a stall
        FcgMonitor m; m.window = 16;
        EXPECT(m.open(1.0, 1.0, 1.0), FcgMonitor::CONTINUE);
        double rr = 1.0;
        for (int it = 8; it <= 400; it += 8) { rr *= 0.95; EXPECT(m.after_chunk(rr, 1.0, 0.5, it), FcgMonitor::CONTINUE); }
    }
    {   // a plateau: 1.5% drops (under 2% in rr = 1% in norm) after the best at 8
        FcgMonitor m; m.window = 24;
        m.open(1.0, 1.0, 1.0);
        EXPECT(m.after_chunk(0.5, 1.0, 0.5, 8), FcgMonitor::CONTINUE);      // best at 8
        EXPECT(m.after_chunk(0.5 * 0.985, 1.0, 0.5, 16), FcgMonitor::CONTINUE);
        EXPECT(m.after_chunk(0.5 * 0.98, 1.0, 0.5, 24), FcgMonitor::CONTINUE);   // not below 0.98 best
        EXPECT(m.after_chunk(0.5 * 0.981, 1.0, 0.5, 32), FcgMonitor::FALL_BACK_KEEP);   // 32 - 8 >= 24
    }
    {   // a 2% drop restarts the window
        FcgMonitor m; m.window = 24;
        m.open(1.0, 1.0, 1.0);
        EXPECT(m.after_chunk(0.99, 1.0, 0.5, 8), FcgMonitor::CONTINUE);
        EXPECT(m.after_chunk(0.985, 1.0, 0.5, 16), FcgMonitor::CONTINUE);
        EXPECT(m.after_chunk(0.97, 1.0, 0.5, 20), FcgMonitor::CONTINUE);    // below 0.98: best at 20
        EXPECT(m.after_chunk(0.969, 1.0, 0.5, 40), FcgMonitor::CONTINUE);   // 40 - 20 < 24
        EXPECT(m.after_chunk(0.968, 1.0, 0.5, 44), FcgMonitor::FALL_BACK_KEEP);
    }
    {   // non-finite values: the iterate is restored before the switch
        FcgMonitor m;
        EXPECT(m.open(nan, 1.0, 1.0), FcgMonitor::FALL_BACK_RESTORE);
        EXPECT(m.open(1.0, inf, 1.0), FcgMonitor::FALL_BACK_RESTORE);
        EXPECT(m.open(1.0, 1.0, 1.0), FcgMonitor::CONTINUE);
        EXPECT(m.after_chunk(nan, 1.0, 0.5, 8), FcgMonitor::FALL_BACK_RESTORE);
        EXPECT(m.after_chunk(0.5, -inf, 0.5, 8), FcgMonitor::FALL_BACK_RESTORE);
        EXPECT(m.after_chunk(0.5, 1.0, nan, 8), FcgMonitor::FALL_BACK_RESTORE);
        EXPECT(m.after_reopen(inf, 1.0, 1.0), FcgMonitor::FALL_BACK_RESTORE);
        EXPECT(m.after_reopen(1.0, nan, 0.0), FcgMonitor::FALL_BACK_RESTORE);
    }
    {   // reopening outcomes
        FcgMonitor m;
        EXPECT(m.after_reopen(1e-22, 1.0, 1.0), FcgMonitor::CONVERGED);
        EXPECT(m.after_reopen(1e-3, 1.0, 0.0), FcgMonitor::CONTINUE);       // a restart
        EXPECT(m.after_reopen(1e-3, 1.0, 2.0), FcgMonitor::AT_LIMIT);       // maxit: stop
        m.limit_is_learned = true;
        EXPECT(m.after_reopen(1e-3, 1.0, 2.0), FcgMonitor::FALL_BACK_KEEP); // learned_maxit: switch
    }
    std::printf("%s\n", fails ? "FAILED" : "ok");
    return fails ? 1 : 0;
}
"""


def test_fallback_decisions(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = tmp_path / "monitor_check.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "monitor_check"
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("ok")
