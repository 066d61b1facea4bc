"""Oracle: the acceptance rule for computed Ritz pairs (test infrastructure).

Sec. II.C: the residual r = H phi - theta phi of a Ritz pair bounds the error of theta, and the
paper offers ||r|| as that bound.  At the 1e-10 ||H|| target the plain residual is too coarse
(the residual floor of the overcomplete basis is far above the true error), so the reading used
here is the quadratic form of the same bound, for a cluster of neighbouring Ritz values:

  Block quadratic residual bound.  Let X hold orthonormal Ritz vectors of a set C of Ritz values,
  R = H X - X diag(theta_C) their residual block, and delta the distance from the values of C to
  the spectrum of H restricted to the orthogonal complement of X.  Then the |C| eigenvalues of H
  paired with C lie within ||R||_2^2 / delta of them.  Since ||R||_2^2 <= sum over C of ||r_i||^2,
  sum ||r_i||^2 / delta bounds every error in C.  The rest of the spectrum is represented by the
  Ritz values outside C (each moved towards C by its own residual, by Weyl's bound), and by the
  window edges: levels outside [-a, a] are filtered out of the basis and unresolved.

  Ghosts.  A unit vector built only from eigenvectors outside [-a, a] has a residual of at least
  a - |theta| for any Rayleigh quotient theta inside the window.  A Ritz value whose residual
  reaches that distance may therefore approximate no level at all; it is a ghost and does not
  represent the spectrum.  Below that distance, Weyl's bound puts a level of H within ||r|| of
  theta, inside the window.

The rule, written out plainly (brute force over every cluster):
  * candidates are the first len(rnorm) Ritz values in the order of (|theta|, theta);
  * a candidate is a ghost when rnorm >= a - |theta|;
  * the estimate of a non-ghost candidate is the smallest of its residual and
    sum_C ||r||^2 / delta_C over every run C of at most 8 consecutive non-ghost Ritz values
    (ascending theta) that contains it and holds only candidates, where delta_C is the smallest of
    a - max_C |theta|, and the distances from C to the nearest non-ghost Ritz value below and above
    it, each less that neighbour's residual (zero when the neighbour is not a candidate);
  * accepted: estimate <= tol;
  * the core walks the candidates outward in |theta| while |theta| <= a and stops at the first
    ghost or unaccepted candidate.
"""
import math

MAX_CLUSTER = 8


def accept(theta, rnorm, a, tol):
    """(core positions in the (|theta|, theta) order, estimate per candidate, ghost count)."""
    theta = [float(t) for t in theta]
    rnorm = [float(x) for x in rnorm]
    r = len(theta)
    n_sel = len(rnorm)
    order = sorted(range(r), key=lambda i: (abs(theta[i]), theta[i]))
    res = [None] * r  # residual of each Ritz value, None where it is not a candidate
    pos = [None] * r  # candidate position of each Ritz value
    for q in range(n_sel):
        res[order[q]] = rnorm[q]
        pos[order[q]] = q
    ghost = [res[i] is not None and not (res[i] < a - abs(theta[i])) for i in range(r)]
    kept = [i for i in range(r) if not ghost[i]]  # ascending theta
    est = [math.inf] * n_sel
    for p, j in enumerate(kept):
        if res[j] is None:
            continue
        best = res[j]
        for lo in range(max(0, p - MAX_CLUSTER + 1), p + 1):
            for hi in range(p, min(len(kept), lo + MAX_CLUSTER)):
                cluster = kept[lo:hi + 1]
                if any(res[c] is None for c in cluster):
                    continue
                r2 = sum(res[c] ** 2 for c in cluster)
                delta = a - max(abs(theta[c]) for c in cluster)
                if lo > 0:
                    nb = kept[lo - 1]
                    delta = min(delta, theta[kept[lo]] - theta[nb] - (res[nb] or 0.0))
                if hi < len(kept) - 1:
                    nb = kept[hi + 1]
                    delta = min(delta, theta[nb] - theta[kept[hi]] - (res[nb] or 0.0))
                if delta > 0.0:
                    best = min(best, r2 / delta)
        est[pos[j]] = best
    core = []
    for q in range(n_sel):
        j = order[q]
        if abs(theta[j]) > a:
            break
        if ghost[j] or not est[q] <= tol:
            break
        core.append(q)
    return core, est, sum(1 for q in range(n_sel) if ghost[order[q]])
