"""Oracle: the acceptance rule for computed Ritz pairs (test infrastructure).

Sec. II.C accepts a Ritz value when its residual certifies it.  The reading used here (a
quadratic residual bound, ghost exclusion and a contiguous core) is the one the library states
for its acceptance; this is that rule written out plainly, with a brute-force nearest neighbour.

Candidates are the first len(rnorm) Ritz values in the order of (|theta|, theta).  A candidate
starts accepted when its residual is at most 1e-4 * norm_est.  It is a ghost when its residual
exceeds ten mean level spacings of the window, 10 * 2a / n_w.  In each round, every accepted
candidate gets the estimate min(r, r^2 / eta), where eta is the distance to the window edge
(a - |theta|) or to the nearest Ritz value that is neither accepted nor a ghost at the start of
the round.  A candidate whose estimate exceeds tol is dropped.  Rounds repeat until none is dropped
(at most 8).  The core walks outward from 0 over |theta| <= a: ghosts are skipped, and the first
other rejection ends it.
"""
import math


def accept(theta, rnorm, a, n_w, tol, norm_est):
    """(core positions in the (|theta|, theta) order, estimates per candidate, ghost count)."""
    theta = [float(t) for t in theta]
    rnorm = [float(x) for x in rnorm]
    n_sel = len(rnorm)
    order = sorted(range(len(theta)), key=lambda i: (abs(theta[i]), theta[i]))
    cap = 1e-4 * norm_est
    ghost_thr = 10.0 * (2.0 * a / n_w)
    ok = [False] * len(theta)
    ghost = [False] * len(theta)
    for q in range(n_sel):
        ok[order[q]] = rnorm[q] <= cap
        ghost[order[q]] = rnorm[q] > ghost_thr
    est = [math.inf] * n_sel
    for _ in range(8):
        unresolved = [theta[i] for i in range(len(theta)) if not ok[i] and not ghost[i]]
        dropped = False
        for q in range(n_sel):
            j = order[q]
            if not ok[j]:
                continue
            eta = a - abs(theta[j])
            for u in unresolved:
                eta = min(eta, abs(u - theta[j]))
            est[q] = min(rnorm[q], rnorm[q] * rnorm[q] / eta) if eta > 0.0 else rnorm[q]
            if not est[q] <= tol:
                ok[j] = False
                dropped = True
        if not dropped:
            break
    core = []
    for q in range(n_sel):
        j = order[q]
        if abs(theta[j]) > a:
            break
        if ghost[j]:
            continue
        if not ok[j]:
            break
        core.append(q)
    return core, est, sum(1 for q in range(n_sel) if ghost[order[q]])
