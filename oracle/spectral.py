"""Oracle: spectral bound, central density of states and window choice (test infrastructure).

The paper takes E_max = E_0 and E_min = -E_0 from an upper-bound estimator
that "costs little extra computation" (Sec. III, parameter settings) and sets
the window half-width a from an estimate of the density of states so that
[-a, a] holds the wanted number of levels (same paragraph).  The estimator
formula itself is not printed; the reading implemented here is:
  * bound: k-step Lanczos from a given start vector; for the two extreme Ritz
    pairs (theta, y) of the Lanczos tridiagonal the Ritz residual norm is
    |beta_k y_k| (last component of y), and
    E_b = 1.01 * max(|theta_max| + |beta_k y_k(max)|, |theta_min| + |beta_k y_k(min)|),
    clamped to the triangle bound sum_t |c_t| (every Pauli string has norm 1);
  * density: Chebyshev moments mu_k = <R, T_k(G) R> / <R, R> over a random
    block R with G = H / E_b (the kernel polynomial method), damped by the
    Jackson kernel, integrated in closed form over [-a_r, a_r].
"""
import math

import numpy as np

from . import _native


def lanczos(apply, v0, k):
    """Plain k-step Lanczos (no reorthogonalisation) from v0.

    Returns (alpha[0..k-1], beta[0..k-1]) where beta[j] = ||w_j|| after step j."""
    v = np.asarray(v0, dtype=np.float64).copy()
    v /= np.linalg.norm(v)
    v_prev = np.zeros_like(v)
    b_prev = 0.0
    alpha = np.zeros(k)
    beta = np.zeros(k)
    for j in range(k):
        w = apply(v[:, None])[:, 0] - b_prev * v_prev
        alpha[j] = np.dot(w, v)
        w = w - alpha[j] * v
        beta[j] = np.linalg.norm(w)
        if beta[j] == 0.0:
            return alpha[: j + 1], beta[: j + 1]
        v_prev, v = v, w / beta[j]
        b_prev = beta[j]
    return alpha, beta


def lanczos_bound(alpha, beta, sum_abs, safety=1.01):
    """E_b from the Lanczos tridiagonal (reading stated in the module docstring).

    Returns (E_b, Ritz values ascending)."""
    k = len(alpha)
    T = np.diag(np.asarray(alpha, dtype=np.float64))
    if k > 1:
        T += np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    theta, Y = _native.syev(T, vectors=True)
    r_lo = abs(beta[-1] * Y[-1, 0])
    r_hi = abs(beta[-1] * Y[-1, -1])
    eb = safety * max(abs(theta[-1]) + r_hi, abs(theta[0]) + r_lo)
    return min(eb, sum_abs), theta


def kpm_moments(apply, R, e_b, M):
    """mu_k = <R, T_k(H/E_b) R> / <R, R>, k = 0..M-1, by the three-term recurrence."""
    R = np.asarray(R, dtype=np.float64)
    norm = float(np.sum(R * R))
    mu = np.zeros(M)
    t_prev = R.copy()
    mu[0] = 1.0
    if M == 1:
        return mu
    t_cur = apply(R) / e_b
    mu[1] = float(np.sum(R * t_cur)) / norm
    for k in range(2, M):
        t_prev, t_cur = t_cur, 2.0 * apply(t_cur) / e_b - t_prev
        mu[k] = float(np.sum(R * t_cur)) / norm
    return mu


def jackson(M):
    """Jackson damping factors g_k, k = 0..M-1."""
    k = np.arange(M, dtype=np.float64)
    q = math.pi / (M + 1)
    return ((M - k + 1) * np.cos(q * k) + np.sin(q * k) / math.tan(q)) / (M + 1)


def kpm_count(mu, D, a_r):
    """Estimated number of levels of H in [-a_r E_b, a_r E_b]:
    D * integral_{-a_r}^{a_r} [g_0 mu_0 + 2 sum_k g_k mu_k T_k(x)] / (pi sqrt(1-x^2)) dx,
    each term integrated in closed form with x = cos(theta)."""
    M = mu.shape[0]
    g = jackson(M)
    th = math.acos(a_r)
    total = g[0] * mu[0] * (math.pi - 2.0 * th) / math.pi
    for k in range(1, M):
        total += 2.0 * g[k] * mu[k] * (math.sin(k * (math.pi - th)) - math.sin(k * th)) / (k * math.pi)
    return D * total


def window_for_count(mu, D, count, iters=200):
    """Smallest a_r in (0, 1) with kpm_count(a_r) >= count, by bisection."""
    lo, hi = 0.0, 1.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if kpm_count(mu, D, mid) >= count:
            hi = mid
        else:
            lo = mid
    return hi
