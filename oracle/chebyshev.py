"""Oracle: Chebyshev polynomials and the two DACP recurrences (test infrastructure).

Scalar definition (App. A, Eq. cheb): T_k(x) = cos(k arccos x) for |x| <= 1,
cosh(k arccosh x) for x > 1, (-1)^k cosh(k arccosh(-x)) for x < -1; the
three-term recurrence T_{k+1} = 2 x T_k - T_{k-1} with T_0 = 1, T_1 = x
(App. A, Eq. rec) is how both recurrences below are evaluated on vectors.

Filter (Sec. II.A, Eq. F): F = (H^2 - E_c)/E_0 with E_c = (E_max^2 + a^2)/2
and E_0 = (E_max^2 - a^2)/2; psi_E = T_K(F) psi normalised (Eq. target) with
K = 18 E_max / a by default.

Evolution (Sec. II.B, Eq. G2): G = H / E_max, a_r = a / E_max; the basis
(App. C, Eq. set2) collects T_{k_m - 1}(G) psi_E and T_{k_m}(G) psi_E at
k_m = floor(m pi / a_r), m = 1..n, read here as the even number
2 floor(m pi / (2 a_r)) as App. C allows.

Moment mode (App. C, Eq. shift): the basis states are never stored.  With the
product identity T_x T_y = (T_{x+y} + T_{|x-y|})/2 the overlap S and the projected
H follow from the b x b moment matrices mu_k = psi_E^T T_k(G) psi_E alone, recorded
during an evolution to twice the last sampled order.  Sums of sampled orders must
themselves be recorded orders, which fixes the samples on a uniform grid
k_m = m Delta, Delta = 2 floor(pi / (2 a_r)) (even, as App. C assumes).

Every function takes the operator as a callable `apply(X) -> H X` on (D, b)
blocks, so the same code runs on the dense and the matrix-free oracle H.
"""
import math

import numpy as np


def cheb_scalar(k, x):
    """T_k(x) from the piecewise closed form (App. A, Eq. cheb); vectorised in x."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1.0
    out[inside] = np.cos(k * np.arccos(x[inside]))
    hi = x > 1.0
    out[hi] = np.cosh(k * np.arccosh(x[hi]))
    lo = x < -1.0
    out[lo] = (-1.0) ** k * np.cosh(k * np.arccosh(-x[lo]))
    return out


def cheb_scalar_recurrence(k, x):
    """T_k(x) by the three-term recurrence (App. A, Eq. rec)."""
    x = np.asarray(x, dtype=np.float64)
    t0 = np.ones_like(x)
    if k == 0:
        return t0
    t1 = x.copy()
    for _ in range(k - 1):
        t0, t1 = t1, 2.0 * x * t1 - t0
    return t1


def filter_constants(e_max, a):
    """(E_c, E_0) of Eq. F."""
    return 0.5 * (e_max * e_max + a * a), 0.5 * (e_max * e_max - a * a)


def filter_order(e_max, a, kfac=18.0):
    """Cut-off order K = kfac * E_max / a (Sec. II.A uses kfac = 18), rounded up."""
    return int(math.ceil(kfac * e_max / a))


def filter_gain(k, lam, e_max, a):
    """Per-eigencomponent filter factor T_k(F(lambda)) (Sec. II.A)."""
    e_c, e_0 = filter_constants(e_max, a)
    return cheb_scalar(k, (np.asarray(lam) ** 2 - e_c) / e_0)


def exp_semicircle_filter(apply, psi, e_max, a, K, normalise=True):
    """T_K(F) psi by the recurrence on F (Sec. II.A), then per-column 2-norm = 1."""
    e_c, e_0 = filter_constants(e_max, a)

    def f_op(v):
        return (apply(apply(v)) - e_c * v) / e_0

    t_prev = np.array(psi, dtype=np.float64, copy=True)
    if K == 0:
        out = t_prev
    else:
        t_cur = f_op(t_prev)
        for _ in range(K - 1):
            t_prev, t_cur = t_cur, 2.0 * f_op(t_cur) - t_prev
        out = t_cur
    if normalise:
        out = out / np.linalg.norm(out, axis=0, keepdims=True)
    return out


def sample_orders(a_r, n):
    """k_m = 2 floor(m pi / (2 a_r)), m = 1..n (App. B / App. C, even reading)."""
    return [2 * int(math.floor(m * math.pi / (2.0 * a_r))) for m in range(1, n + 1)]


def chebyshev_basis(apply, psi_e, e_max, a, n):
    """Basis panels [psi_E, T_{k_1-1} psi_E, T_{k_1} psi_E, ..., T_{k_n} psi_E]
    (App. C, Eq. set2) from the recurrence T_{k+1} = 2 G T_k - T_{k-1}, G = H/E_max.
    Returns V of shape (D, b (2n+1)), panel p occupying columns p b .. p b + b - 1,
    and the list of sample orders."""
    ks = sample_orders(a / e_max, n)
    want = set()
    for k in ks:
        want.add(k - 1)
        want.add(k)
    psi_e = np.asarray(psi_e, dtype=np.float64)
    panels = {0: psi_e.copy()}
    t_prev = psi_e.copy()
    t_cur = apply(psi_e) / e_max
    k = 1
    if k in want:
        panels[k] = t_cur.copy()
    kmax = ks[-1] if ks else 0
    while k < kmax:
        t_prev, t_cur = t_cur, 2.0 * apply(t_cur) / e_max - t_prev
        k += 1
        if k in want:
            panels[k] = t_cur.copy()
    cols = [panels[0]]
    for km in ks:
        cols.append(panels[km - 1])
        cols.append(panels[km])
    return np.concatenate(cols, axis=1), ks


def uniform_sample_orders(a_r, n):
    """Moment mode: (Delta, [k_1 .. k_n]) with k_m = m Delta, Delta = 2 floor(pi / (2 a_r))."""
    delta = 2 * int(math.floor(math.pi / (2.0 * a_r)))
    return delta, [m * delta for m in range(1, n + 1)]


def panel_orders(ks):
    """Orders of the basis panels (App. C, Eq. set2): [0, k_1 - 1, k_1, ..., k_n - 1, k_n]."""
    return [0] + [k for km in ks for k in (km - 1, km)]


def basis_on_orders(apply, psi_e, e_max, orders):
    """Explicit panels T_x(G) psi_E for the given orders (any order list), G = H / E_max."""
    psi_e = np.asarray(psi_e, dtype=np.float64)
    want = set(orders)
    panels = {}
    t_prev = psi_e.copy()
    if 0 in want:
        panels[0] = t_prev.copy()
    t_cur = apply(psi_e) / e_max
    if 1 in want:
        panels[1] = t_cur.copy()
    for k in range(2, max(orders) + 1):
        t_prev, t_cur = t_cur, 2.0 * apply(t_cur) / e_max - t_prev
        if k in want:
            panels[k] = t_cur.copy()
    return np.concatenate([panels[x] for x in orders], axis=1)


def chebyshev_moments(apply, psi_e, e_max, kmax):
    """mu[k] = psi_E^T T_k(G) psi_E (b x b), k = 0 .. kmax, by the three-term recurrence."""
    psi_e = np.asarray(psi_e, dtype=np.float64)
    b = psi_e.shape[1]
    mu = np.zeros((kmax + 1, b, b))
    t_prev = psi_e.copy()
    mu[0] = psi_e.T @ t_prev
    if kmax == 0:
        return mu
    t_cur = apply(psi_e) / e_max
    mu[1] = psi_e.T @ t_cur
    for k in range(2, kmax + 1):
        t_prev, t_cur = t_cur, 2.0 * apply(t_cur) / e_max - t_prev
        mu[k] = psi_e.T @ t_cur
    return mu


def moment_projection(mu, orders, e_max):
    """S = A^T A and P = A^T H A of the panels T_x(G) psi_E, x in `orders`, from the moments alone
    (App. C, Eq. shift): block (p, q) of S is (mu_{x+y} + mu_{|x-y|}) / 2; with H = E_max T_1(G)
    and T_1 T_y = (T_{y+1} + T_{|y-1|}) / 2, block (p, q) of P is
    E_max (mu_{x+y+1} + mu_{|x-y-1|} + mu_{x+|y-1|} + mu_{|x-|y-1||}) / 4."""
    b = mu.shape[1]
    npan = len(orders)
    S = np.zeros((npan * b, npan * b))
    P = np.zeros_like(S)
    for p, x in enumerate(orders):
        for q, y in enumerate(orders):
            ym = abs(y - 1)
            S[p * b:(p + 1) * b, q * b:(q + 1) * b] = 0.5 * (mu[x + y] + mu[abs(x - y)])
            P[p * b:(p + 1) * b, q * b:(q + 1) * b] = 0.25 * e_max * (
                mu[x + y + 1] + mu[abs(x - y - 1)] + mu[x + ym] + mu[abs(x - ym)])
    return S, P
