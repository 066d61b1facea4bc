"""The moment projection's reading (App. C, Eq. shift, with a stored basis) checked on the CPU.

With the panels T_x(G) psi on the uniform grid of orders {0} u {j Delta - 1, j Delta}, S and P
follow from b x b moments mu_k = psi^T T_k psi and nu_k = psi^T G T_k psi at the orders x + y and
|x - y| of two panel orders, and those moments follow from Gram blocks of seven anchor panels
(orders 0, 1, 2, k_n - 2 .. k_n + 1) and of their H images with the stored panels, through
T_A T_x = (T_{A+x} + T_{|A-x|}) / 2.  These tests fix, independently of the HIP path:
  * that every order S and P read is reachable from the anchors, for every even grid step up to 60
    and up to 30 sample pairs (the library returns an error otherwise);
  * that S and P so derived equal the oracle's explicit V^T V and V^T (H V) of the same panels, on
    the oracle's own basis (grids of step 2, one sample pair, b not a power of two).
"""
import numpy as np
import pytest

from oracle import chebyshev, hamiltonian, subspace
from paper_2011_02107_amd import inputs


def _anchors(kn):
    return sorted({k for k in (0, 1, 2, kn - 2, kn - 1, kn, kn + 1) if k >= 0})


def _needed(orders):
    return {k for x in orders for y in orders for k in (x + y, abs(x - y))}


def _rules(anchors, orders):
    """Derivation rules in the order found: order -> (anchor index, panel index, other order or None)."""
    rules = {}
    changed = True
    while changed:
        changed = False
        for ai, a in enumerate(anchors):
            for q, x in enumerate(orders):
                s, d = a + x, abs(a - x)
                if s == d:
                    if s not in rules:
                        rules[s] = (ai, q, None)
                        changed = True
                elif d in rules and s not in rules:
                    rules[s] = (ai, q, d)
                    changed = True
                elif s in rules and d not in rules:
                    rules[d] = (ai, q, s)
                    changed = True
    return rules


def test_anchor_moments_reach_every_order():
    for delta in range(2, 61, 2):
        for n in range(1, 31):
            orders = [0] + [o for j in range(1, n + 1) for o in (j * delta - 1, j * delta)]
            rules = _rules(_anchors(n * delta), orders)
            missing = _needed(orders) - set(rules)
            assert not missing, (delta, n, sorted(missing)[:5])


def _derive(G, rules, b, na, scale, part):
    """The b x b moments from the Gram blocks, in the order the rules were found (dicts keep it)."""
    mom = {}
    for k, (ai, q, other) in rules.items():
        g = scale * G[(part * na + ai) * b:(part * na + ai + 1) * b, q * b:(q + 1) * b]
        mom[k] = g.copy() if other is None else 2.0 * g - mom[other]
    return mom


@pytest.mark.parametrize("L,b,a_r,n,terms_of", [
    (8, 4, 0.2, 3, lambda L: inputs.ising_chain(L)),
    (9, 3, 0.9, 4, lambda L: inputs.spin_glass(L, 2)),    # grid step 2: anchors and panels overlap
    (10, 5, 0.7, 1, lambda L: inputs.spin_glass(L, 4)),   # one sample pair
    (10, 4, 0.05, 3, lambda L: inputs.ising_chain(L)),    # step 62
])
def test_anchor_moments_reproduce_the_explicit_projection(L, b, a_r, n, terms_of):
    terms = terms_of(L)
    apply = lambda X: hamiltonian.apply_h(L, terms, X)
    e_b = 1.01 * hamiltonian.sum_abs_coeff(terms)
    psi = np.random.default_rng(L + 7).standard_normal((1 << L, b))
    psi /= np.linalg.norm(psi, axis=0, keepdims=True)
    _, ks = chebyshev.uniform_sample_orders(a_r, n)
    orders = chebyshev.panel_orders(ks)
    anchors = _anchors(ks[-1])
    V = chebyshev.basis_on_orders(apply, psi, e_b, orders)
    A = chebyshev.basis_on_orders(apply, psi, e_b, anchors)
    G = np.vstack([A.T @ V, apply(A).T @ V])  # anchors, then their H images
    rules = _rules(anchors, orders)
    na = len(anchors)
    mu = _derive(G, rules, b, na, 1.0, 0)
    nu = _derive(G, rules, b, na, 1.0 / e_b, 1)
    npan = len(orders)
    S = np.zeros((npan * b, npan * b))
    P = np.zeros_like(S)
    for p, x in enumerate(orders):
        for q, y in enumerate(orders):
            S[p * b:(p + 1) * b, q * b:(q + 1) * b] = 0.5 * (mu[x + y] + mu[abs(x - y)])
            P[p * b:(p + 1) * b, q * b:(q + 1) * b] = 0.5 * e_b * (nu[x + y] + nu[abs(x - y)])
    Se, Pe = subspace.project(apply, V)
    D = 1 << L
    assert np.abs(S - Se).max() <= 1e-13 * D * np.abs(Se).max()
    assert np.abs(P - Pe).max() <= 1e-13 * D * np.abs(Pe).max()
    # and the oracle's own moment assembly (mu one order off for P) agrees too
    So, Po = chebyshev.moment_projection(chebyshev.chebyshev_moments(apply, psi, e_b, 2 * ks[-1] + 1), orders, e_b)
    assert np.abs(S - So).max() <= 1e-13 * D * np.abs(So).max()
    assert np.abs(P - Po).max() <= 1e-13 * D * np.abs(Po).max()
