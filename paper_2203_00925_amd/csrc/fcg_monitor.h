// Decisions of the learned solve's flexible-CG phase (host side, no GPU):
// when to fall back to plain Jacobi-CG.  Fed the device scalars the host
// pulls after the opening, after every chunk of iterations and after every
// reopening from the true residual.  Header-only so that a host program can
// drive it with made-up scalar sequences.
#pragma once
#include <cmath>

namespace mifvm {

struct FcgMonitor {
    enum Action {
        CONTINUE = 0,          // run another chunk (or reopen)
        CONVERGED = 1,         // the true residual met the tolerance
        AT_LIMIT = 2,          // maxit reached: stop (not converged)
        FALL_BACK_KEEP = 3,    // switch to Jacobi-CG from the current iterate
        FALL_BACK_RESTORE = 4  // non-finite: restore the last finite iterate, then switch
    };
    int window = 200;          // stall: the best ||r||^2 not 2% (1% in norm) lower for this many iterations
    bool limit_is_learned = false;   // the iteration limit is learned_maxit (< maxit)
    double best = 0.0, best_it = 0.0;

    // after the first opening: true ||r||^2, z.r, recurrence ||r||^2
    Action open(double true_rr, double rz, double rr) {
        if (!std::isfinite(true_rr) || !std::isfinite(rz)) return FALL_BACK_RESTORE;
        best = rr;
        best_it = 0.0;
        return CONTINUE;
    }
    // after a chunk: recurrence ||r||^2, z.r, beta, iterations so far
    Action after_chunk(double rr, double rz, double beta, double it) {
        if (!std::isfinite(rr) || !std::isfinite(rz) || !std::isfinite(beta)) return FALL_BACK_RESTORE;
        if (rr < 0.98 * best) {
            best = rr;
            best_it = it;
        } else if (it - best_it >= window) {
            return FALL_BACK_KEEP;
        }
        return CONTINUE;
    }
    // after a reopening from the true residual: its ||r||^2, z.r and the
    // device's done flag (0 running, 1 converged, 2 at the limit)
    Action after_reopen(double true_rr, double rz, double done) const {
        if (!std::isfinite(true_rr) || !std::isfinite(rz)) return FALL_BACK_RESTORE;
        if (done == 1.0) return CONVERGED;
        if (done == 2.0) return limit_is_learned ? FALL_BACK_KEEP : AT_LIMIT;
        return CONTINUE;
    }
};

}  // namespace mifvm
