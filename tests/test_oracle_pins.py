"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks an oracle function against something other than itself:
explicit Kronecker products, closed forms, an independent eigen-algorithm,
published known-answer vectors, the Jordan-Wigner reduction, trace
invariants, and eigen-expansions computed with the independent Jacobi solver.
"""
import math
import os

import numpy as np
import pytest

from oracle import _native, acceptance, central, chebyshev, hamiltonian, jordan_wigner, levels, philox, spectral, subspace
from paper_2011_02107_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

PAULI = {
    0: np.eye(2),
    1: np.array([[0.0, 1.0], [1.0, 0.0]]),
    2: np.array([[0.0, -1j], [1j, 0.0]]),
    3: np.array([[1.0, 0.0], [0.0, -1.0]]),
}


def kron_term(L, t):
    """sigma_{L-1} (x) ... (x) sigma_0 for one term (bit i = spin i, little-endian)."""
    ops = [PAULI[0]] * L
    ops[int(t["site_a"])] = PAULI[int(t["op_a"])]
    if int(t["op_b"]):
        ops[int(t["site_b"])] = PAULI[int(t["op_b"])]
    M = np.array([[1.0 + 0j]])
    for site in range(L - 1, -1, -1):
        M = np.kron(M, ops[site])
    return t["coeff"] * M


def random_terms(L, rng, n):
    """Random real one- and two-body terms covering every real op pair."""
    pairs = [(1, 0), (3, 0), (1, 1), (2, 2), (3, 3), (1, 3), (3, 1)]
    rows = []
    for _ in range(n):
        oa, ob = pairs[rng.integers(len(pairs))]
        sa = int(rng.integers(L))
        sb = int(rng.integers(L - 1))
        if sb >= sa:
            sb += 1
        if ob == 0:
            sb = 0
        rows.append((oa, sa, ob, sb, rng.uniform(-1, 1)))
    return inputs.make_terms(rows)


# ---------------------------------------------------------------- Hamiltonian


@pytest.mark.parametrize("L", [1, 2, 3, 5, 6])
def test_dense_h_matches_kronecker(L):
    rng = np.random.default_rng(L)
    terms = random_terms(L, rng, 12) if L > 1 else inputs.make_terms([(1, 0, 0, 0, 0.7), (3, 0, 0, 0, -0.2)])
    H = hamiltonian.dense_h(L, terms)
    K = sum(kron_term(L, t) for t in terms)
    assert np.abs(K.imag).max() < 1e-15
    assert np.abs(H - K.real).max() < 1e-14


@pytest.mark.parametrize("builder", ["chain", "glass", "paper_tfim", "paper_sgs"])
def test_dense_h_kronecker_model_families(builder):
    L = 5
    terms = {
        "chain": inputs.ising_chain(L),
        "glass": inputs.spin_glass(L, 3),
        "paper_tfim": inputs.paper_tfim(L, 4),
        "paper_sgs": inputs.paper_sgs(L, 5),
    }[builder]
    H = hamiltonian.dense_h(L, terms)
    K = sum(kron_term(L, t) for t in terms).real
    assert np.abs(H - K).max() < 1e-13


def test_imaginary_term_rejected():
    with pytest.raises(ValueError):
        hamiltonian.term_masks(2, 0, 0, 0)  # single sigma^y
    with pytest.raises(ValueError):
        hamiltonian.term_masks(1, 0, 2, 1)  # X Y


@pytest.mark.parametrize("L", [4, 7])
def test_matrix_free_apply_matches_dense(L):
    rng = np.random.default_rng(10 + L)
    terms = random_terms(L, rng, 15)
    X = rng.standard_normal((1 << L, 3))
    assert np.abs(hamiltonian.apply_h(L, terms, X) - hamiltonian.dense_h(L, terms) @ X).max() < 1e-12


@pytest.mark.parametrize("L", [4, 6, 8])
def test_trace_invariants(L):
    """tr H = 0 and tr H^2 = D sum c^2 (Pauli strings are traceless and orthogonal);
    for the chain, tr H^3 / D = 6 (L-1) J hz^2 (only Z_i Z_{i+1} * Z_i * Z_{i+1} = I)."""
    D = 1 << L
    for terms in (inputs.ising_chain(L), inputs.spin_glass(L, L)):
        H = hamiltonian.dense_h(L, terms)
        assert abs(np.trace(H)) < 1e-10
        assert abs(np.trace(H @ H) / D - hamiltonian.sum_sq_coeff(terms)) < 1e-10
    H = hamiltonian.dense_h(L, inputs.ising_chain(L, J=1.0, hx=1.05, hz=0.5))
    assert abs(np.trace(H @ H @ H) / D - 6 * (L - 1) * 1.0 * 0.5**2) < 1e-9


# ---------------------------------------------------------------- eigensolvers


def test_syev_vs_jacobi_random():
    rng = np.random.default_rng(0)
    for n in (1, 2, 5, 40, 120):
        A = rng.standard_normal((n, n))
        A = A + A.T
        w, Z = _native.syev(A, vectors=True)
        wj = _native.jacobi(A)
        assert np.abs(w - wj).max() < 1e-11 * max(1.0, np.abs(w).max())
        assert np.abs(A @ Z - Z * w).max() < 1e-12 * max(1.0, np.abs(w).max()) * n
        assert np.abs(Z.T @ Z - np.eye(n)).max() < 1e-13 * n


def test_syev_vs_jacobi_hamiltonian():
    L = 7
    H = hamiltonian.dense_h(L, inputs.ising_chain(L))
    assert np.abs(_native.syev(H) - _native.jacobi(H)).max() < 1e-11


def test_two_spin_closed_form():
    for line in open(os.path.join(GOLDEN, "two_spin_chain.txt")):
        if line.startswith("#") or not line.strip():
            continue
        J, h, *ref = map(float, line.split())
        w = central.full_spectrum_dense(2, inputs.ising_chain(2, J=J, hx=h, hz=0.0))
        assert np.abs(w - np.array(ref)).max() < 1e-14


def test_degenerate_and_diagonal_inputs():
    w = _native.syev(np.diag([3.0, -1.0, 3.0, 0.0]))
    assert np.array_equal(w, np.array([-1.0, 0.0, 3.0, 3.0]))
    w = _native.syev(np.zeros((3, 3)))
    assert np.array_equal(w, np.zeros(3))


@pytest.mark.parametrize("L", [2, 3, 5, 8])
def test_jordan_wigner_vs_dense_uniform(L):
    terms = inputs.ising_chain(L, J=1.0, hx=1.05, hz=0.0)
    w = central.full_spectrum_dense(L, terms)
    j = jordan_wigner.full_spectrum(np.ones(L - 1), 1.05 * np.ones(L))
    assert np.abs(w - j).max() < 1e-12


def test_jordan_wigner_vs_dense_disordered():
    L = 7
    rng = np.random.default_rng(7)
    J = rng.uniform(-1, 1, L - 1)
    h = rng.uniform(-1, 1, L)
    rows = [(3, i, 3, i + 1, J[i]) for i in range(L - 1)] + [(1, i, 0, 0, h[i]) for i in range(L)]
    w = central.full_spectrum_dense(L, inputs.make_terms(rows))
    assert np.abs(w - jordan_wigner.full_spectrum(J, h)).max() < 1e-12


def test_jordan_wigner_paper_tfim_mapping():
    """The paper's (1/4) J X X + (1/2) Gamma Z chain equals the Z Z + X form with
    J -> J/4, h -> Gamma/2 after exchanging x and z."""
    L = 6
    terms = inputs.paper_tfim(L, 11)
    Jb = np.array([t["coeff"] for t in terms if t["op_b"] == 1])
    g = np.array([t["coeff"] for t in terms if t["op_b"] == 0])
    w = central.full_spectrum_dense(L, terms)
    assert np.abs(w - jordan_wigner.full_spectrum(Jb, g)).max() < 1e-12


@pytest.mark.parametrize("L", [6, 9])
def test_spectral_sums(L):
    terms = inputs.spin_glass(L, 1)
    w = central.full_spectrum_dense(L, terms)
    assert abs(w.sum()) < 1e-9
    assert abs(np.sum(w * w) - (1 << L) * hamiltonian.sum_sq_coeff(terms)) < 1e-8


def test_central_selection_ties_and_order():
    w = np.array([-2.0, -1.0, -0.5, 0.5, 1.0, 3.0])
    assert np.array_equal(central.select_central(w, 3), np.array([-1.0, -0.5, 0.5]))
    # odd N: tie |-1| = |1| broken towards the smaller value
    assert np.array_equal(central.select_central(w, 3)[0], -1.0)
    assert np.array_equal(central.select_central(np.array([1.0, -1.0, 0.2]), 2), np.array([-1.0, 0.2]))


# ---------------------------------------------------------------- Chebyshev


def test_cheb_closed_form_vs_recurrence():
    x = np.concatenate([np.linspace(-1.3, 1.3, 101), [-1.0, 1.0, 0.0]])
    for k in (0, 1, 2, 5, 17, 40):
        assert np.abs(chebyshev.cheb_scalar(k, x) - chebyshev.cheb_scalar_recurrence(k, x)).max() < 1e-9 * max(
            1.0, np.abs(chebyshev.cheb_scalar(k, x)).max()
        )


def test_cheb_bounded_and_product_identity():
    """|T_k| <= 1 on [-1, 1] (App. A) and T_i T_j = (T_{i+j} + T_{|i-j|}) / 2 (App. C, Eq. shift)."""
    x = np.linspace(-1, 1, 2001)
    for k in (3, 4, 5, 100):
        assert np.abs(chebyshev.cheb_scalar_recurrence(k, x)).max() <= 1.0 + 1e-12
    for i, j in ((3, 5), (7, 7), (10, 2), (0, 4)):
        lhs = chebyshev.cheb_scalar(i, x) * chebyshev.cheb_scalar(j, x)
        rhs = 0.5 * (chebyshev.cheb_scalar(i + j, x) + chebyshev.cheb_scalar(abs(i - j), x))
        assert np.abs(lhs - rhs).max() < 1e-12


def test_filter_gain_matches_exp_semicircle_shape():
    """Fig. 1 setting (E_max = 1, k a = 24): inside [-a, a] the filter equals
    (-1)^k cosh(k theta) and ln|T_k(F(x))| stays within ln 2 + k a^3 of
    2 k sqrt(a^2 - x^2) (Eq. filter); outside the window |T_k(F)| <= 1."""
    for a in (0.1, 0.05, 0.025):
        k = int(round(24 / a))
        x_in = np.linspace(-a, a, 401)[1:-1]
        g = chebyshev.filter_gain(k, x_in, 1.0, a)
        theta = np.arccosh(1 + 2 * (a * a - x_in**2) / (1 - a * a))
        assert np.allclose(g, (-1.0) ** k * np.cosh(k * theta), rtol=1e-9)
        dev = np.abs(np.log(np.abs(g)) - 2 * k * np.sqrt(a * a - x_in**2))
        assert dev.max() <= math.log(2) + k * a**3 + 1e-9
        x_out = np.concatenate([np.linspace(a, 1, 500), -np.linspace(a, 1, 500)])
        assert np.abs(chebyshev.filter_gain(k, x_out, 1.0, a)).max() <= 1.0 + 1e-9


def _jacobi_eigenpairs(L, terms):
    return _native.jacobi(hamiltonian.dense_h(L, terms), vectors=True)


def test_filter_recurrence_matches_eigen_expansion():
    """T_K(F) psi = sum_j T_K(F(lambda_j)) <phi_j|psi> phi_j (Sec. II.A, Eq. chevo),
    eigenpairs from the independent Jacobi solver."""
    L = 6
    terms = inputs.ising_chain(L)
    lam, Phi = _jacobi_eigenpairs(L, terms)
    e_max = 1.01 * np.abs(lam).max()
    a = 0.8
    K = 40
    psi = np.random.default_rng(1).standard_normal((1 << L, 2))
    got = chebyshev.exp_semicircle_filter(lambda X: hamiltonian.apply_h(L, terms, X), psi, e_max, a, K, normalise=False)
    ref = Phi @ (chebyshev.filter_gain(K, lam, e_max, a)[:, None] * (Phi.T @ psi))
    assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max()
    normed = chebyshev.exp_semicircle_filter(lambda X: hamiltonian.apply_h(L, terms, X), psi, e_max, a, K)
    assert np.allclose(np.linalg.norm(normed, axis=0), 1.0)
    assert np.abs(normed - ref / np.linalg.norm(ref, axis=0)).max() < 1e-10


def test_sample_orders_even_and_spaced():
    for a_r in (0.3, 0.05, 0.0071):
        ks = chebyshev.sample_orders(a_r, 12)
        assert all(k % 2 == 0 for k in ks)
        assert all(abs(k - m * math.pi / a_r) <= 2.0 for m, k in enumerate(ks, 1))
        assert all(k2 > k1 for k1, k2 in zip(ks, ks[1:]))


def test_basis_matches_eigen_expansion():
    """Columns T_k(G) psi_E = sum_j cos(k arccos(lambda_j / E_max)) <phi_j|psi_E> phi_j (Sec. II.B, Eq. chevo2)."""
    L = 6
    terms = inputs.ising_chain(L)
    lam, Phi = _jacobi_eigenpairs(L, terms)
    e_max = 1.01 * np.abs(lam).max()
    a = 1.5
    psi = np.random.default_rng(2).standard_normal((1 << L, 2))
    V, ks = chebyshev.chebyshev_basis(lambda X: hamiltonian.apply_h(L, terms, X), psi, e_max, a, 3)
    b = 2
    assert V.shape == (1 << L, b * 7)
    coef = Phi.T @ psi
    orders = [0] + [k for km in ks for k in (km - 1, km)]
    for p, k in enumerate(orders):
        ref = Phi @ (np.cos(k * np.arccos(lam / e_max))[:, None] * coef)
        assert np.abs(V[:, p * b : (p + 1) * b] - ref).max() < 1e-10 * np.abs(psi).max() * max(1, k)


def test_overlap_from_moments_product_identity():
    """App. C: S_ij = <psi|T_x T_y|psi> = (<psi|T_{x+y}|psi> + <psi|T_{|x-y|}|psi>)/2 and
    P_ij = (<psi|H T_{x+y}|psi> + <psi|H T_{|x-y|}|psi>)/2, from moments alone."""
    L = 7
    terms = inputs.spin_glass(L, 2)
    apply = lambda X: hamiltonian.apply_h(L, terms, X)
    lam = central.full_spectrum_dense(L, terms)
    e_max = 1.01 * np.abs(lam).max()
    psi = np.random.default_rng(3).standard_normal((1 << L, 1))
    psi /= np.linalg.norm(psi)
    V, ks = chebyshev.chebyshev_basis(apply, psi, e_max, 2.0, 4)
    S, P = subspace.project(apply, V)
    orders = [0] + [k for km in ks for k in (km - 1, km)]
    kmax = 2 * max(orders)
    t_prev, t_cur = psi.copy(), apply(psi) / e_max
    mom_s = [float(psi[:, 0] @ psi[:, 0]), float(psi[:, 0] @ t_cur[:, 0])]
    hpsi = apply(psi)
    mom_h = [float(hpsi[:, 0] @ psi[:, 0]), float(hpsi[:, 0] @ t_cur[:, 0])]
    for _ in range(2, kmax + 1):
        t_prev, t_cur = t_cur, 2.0 * apply(t_cur) / e_max - t_prev
        mom_s.append(float(psi[:, 0] @ t_cur[:, 0]))
        mom_h.append(float(hpsi[:, 0] @ t_cur[:, 0]))
    for i, x in enumerate(orders):
        for j, y in enumerate(orders):
            assert abs(S[i, j] - 0.5 * (mom_s[x + y] + mom_s[abs(x - y)])) < 1e-9
            assert abs(P[i, j] - 0.5 * (mom_h[x + y] + mom_h[abs(x - y)])) < 1e-8


def test_moment_projection_matches_explicit_basis_on_the_uniform_grid():
    """Moment mode (App. C): S and P assembled from the b x b moments mu_k = psi^T T_k(G) psi by
    the product identity equal the explicit A^T A and A^T H A of the panels on the same uniform
    grid k_m = m Delta, within the recurrence's rounding; the recorded orders reach 2 k_n + 1."""
    L = 7
    terms = inputs.spin_glass(L, 5)
    apply = lambda X: hamiltonian.apply_h(L, terms, X)
    lam = central.full_spectrum_dense(L, terms)
    e_max = 1.01 * np.abs(lam).max()
    psi = np.random.default_rng(4).standard_normal((1 << L, 3))
    psi /= np.linalg.norm(psi, axis=0, keepdims=True)
    delta, ks = chebyshev.uniform_sample_orders(0.3, 4)
    assert delta % 2 == 0 and ks == [delta * m for m in range(1, 5)]
    orders = chebyshev.panel_orders(ks)
    V = chebyshev.basis_on_orders(apply, psi, e_max, orders)
    S_ex, P_ex = subspace.project(apply, V)
    mu = chebyshev.chebyshev_moments(apply, psi, e_max, 2 * ks[-1] + 1)
    S, P = chebyshev.moment_projection(mu, orders, e_max)
    assert np.abs(S - S_ex).max() < 1e-11 * np.abs(S_ex).max()
    assert np.abs(P - P_ex).max() < 1e-11 * np.abs(P_ex).max() * 10
    # moments of exact eigenvectors are diagonal with entries T_k(lambda / E_max)
    w, Z = _native.jacobi(hamiltonian.dense_h(L, terms), vectors=True)
    mu_e = chebyshev.chebyshev_moments(apply, Z[:, :2], e_max, 9)
    for k in (0, 3, 9):
        assert np.allclose(mu_e[k], np.diag(chebyshev.cheb_scalar(k, w[:2] / e_max)), atol=1e-10)


# ---------------------------------------------------------------- subspace diagonalisation


def test_rayleigh_ritz_exact_eigenvectors():
    """With V = a set of exact eigenvectors, S = I and the Ritz values are the eigenvalues."""
    L = 6
    terms = inputs.ising_chain(L)
    lam, Phi = _jacobi_eigenpairs(L, terms)
    sel = np.arange(20, 31)
    V = Phi[:, sel]
    S, P = subspace.project(lambda X: hamiltonian.apply_h(L, terms, X), V)
    assert np.abs(S - np.eye(len(sel))).max() < 1e-12
    theta, B, r = subspace.rayleigh_ritz(S, P)
    assert r == len(sel)
    assert np.abs(theta - lam[sel]).max() < 1e-12


def test_rayleigh_ritz_overcomplete_invariant_subspace():
    """A redundant basis of an invariant subspace (singular S) still gives the exact
    eigenvalues once the S eigenvalues below epsilon are dropped (App. C)."""
    L = 6
    terms = inputs.spin_glass(L, 9)
    lam, Phi = _jacobi_eigenpairs(L, terms)
    rng = np.random.default_rng(4)
    sel = np.arange(25, 37)
    core = Phi[:, sel] @ rng.standard_normal((len(sel), len(sel)))
    V = np.concatenate([core, core[:, :5] @ rng.standard_normal((5, 4))], axis=1)
    S, P = subspace.project(lambda X: hamiltonian.apply_h(L, terms, X), V)
    theta, B, r = subspace.rayleigh_ritz(S, P)
    assert r == len(sel)
    assert np.abs(np.sort(theta) - lam[sel]).max() < 1e-10
    rn, _ = subspace.residual_norms(lambda X: hamiltonian.apply_h(L, terms, X), V, B, theta)
    assert rn.max() < 1e-9


def test_neighbour_gaps():
    g = subspace.neighbour_gaps(np.array([0.0, 1.0, 3.0, 3.5]))
    assert np.array_equal(g, np.array([1.0, 1.0, 0.5, 0.5]))


# ---------------------------------------------------------------- random numbers


def test_philox_known_answers():
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        out = philox.philox4x32_10(*v[:6])
        assert [int(o) for o in out] == v[6:]


def test_gaussian_block_statistics():
    z = philox.gaussian_block(1 << 14, 4, seed=12345)
    assert z.shape == (1 << 14, 4)
    assert abs(z.mean()) < 0.03 and abs(z.std() - 1.0) < 0.03
    # distinct columns and rows are distinct streams
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 0.05


# ---------------------------------------------------------------- bounds and density


def test_lanczos_bound_is_upper_bound():
    for L, terms in ((8, inputs.ising_chain(8)), (8, inputs.spin_glass(8, 5)), (9, inputs.paper_sgs(9, 1))):
        D = 1 << L
        w = central.full_spectrum_dense(L, terms)
        norm = max(-w[0], w[-1])
        al, be = spectral.lanczos(lambda X: hamiltonian.apply_h(L, terms, X), np.random.default_rng(0).standard_normal(D), 60)
        eb, theta = spectral.lanczos_bound(al, be, hamiltonian.sum_abs_coeff(terms))
        assert eb >= norm
        assert eb <= 1.05 * norm
        assert theta[0] >= w[0] - 1e-9 and theta[-1] <= w[-1] + 1e-9


def test_kpm_exact_trace_and_count():
    """With R = identity the moments are exactly tr T_k(G)/D; the Jackson-damped
    count over a wide window tracks the exact count (kernel polynomial method)."""
    L = 8
    terms = inputs.ising_chain(L)
    D = 1 << L
    w = central.full_spectrum_dense(L, terms)
    e_b = 1.01 * np.abs(w).max()
    mu = spectral.kpm_moments(lambda X: hamiltonian.apply_h(L, terms, X), np.eye(D), e_b, 64)
    for k in (0, 1, 7, 30):
        assert abs(mu[k] - np.mean(chebyshev.cheb_scalar(k, w / e_b))) < 1e-12
    mu = spectral.kpm_moments(lambda X: hamiltonian.apply_h(L, terms, X), np.eye(D), e_b, 256)
    for a_r in (0.1, 0.2, 0.4):
        exact = np.sum(np.abs(w) <= a_r * e_b)
        assert abs(spectral.kpm_count(mu, D, a_r) - exact) <= 0.08 * exact + 3
    a_r = spectral.window_for_count(mu, D, 60)
    assert abs(spectral.kpm_count(mu, D, a_r) - 60) < 1e-6


def test_jackson_kernel_limits():
    g = spectral.jackson(50)
    assert abs(g[0] - 1.0) < 1e-12
    assert np.all(np.diff(g) < 0) and g[-1] > 0


# ---------------------------------------------------------------- plain definition


@pytest.mark.slow
def test_central_eigenvalues_jw_twin_l12():
    L, N = 12, 150
    terms = inputs.ising_chain(L, hz=0.0)
    got, norm = central.central_eigenvalues(L, terms, N)
    ref, norm_jw = central.central_eigenvalues_jw(np.ones(L - 1), 1.05 * np.ones(L), N)
    assert abs(norm - norm_jw) < 1e-10
    assert np.abs(got - ref).max() <= 1e-10 * norm


# ------------------------------------------------------------------ learned window network


def test_mlp_gradient_matches_central_differences():
    from oracle import mlp

    n_in, hidden, layers, n_out = 3, 5, 2, 2
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(mlp.n_params(n_in, hidden, layers, n_out)) * 0.7
    X = rng.standard_normal((7, n_in))
    T = rng.standard_normal((7, n_out))
    loss, g = mlp.loss_and_grad(theta, X, T, n_in, hidden, layers, n_out)
    h = 1e-6
    num = np.zeros_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        num[i] = (mlp.loss_and_grad(theta + e, X, T, n_in, hidden, layers, n_out)[0]
                  - mlp.loss_and_grad(theta - e, X, T, n_in, hidden, layers, n_out)[0]) / (2 * h)
    assert np.abs(g - num).max() <= 1e-7 * max(1.0, np.abs(num).max())


def test_mlp_linear_special_cases():
    """No hidden layer: least squares, gradient X^T (X W^T + b - T) / n in closed form; a zero
    input layer makes every hidden tanh output 0, so only the output bias matters."""
    from oracle import mlp

    rng = np.random.default_rng(1)
    X = rng.standard_normal((9, 4))
    T = rng.standard_normal((9, 2))
    W = rng.standard_normal((2, 4))
    b = rng.standard_normal(2)
    theta = np.concatenate([W.ravel(), b])
    loss, g = mlp.loss_and_grad(theta, X, T, 4, 0, 0, 2)
    R = X @ W.T + b - T
    assert np.isclose(loss, 0.5 * np.sum(R * R) / 9)
    assert np.allclose(g, np.concatenate([(R.T @ X / 9).ravel(), R.sum(0) / 9]), atol=1e-14)
    # zero first layer: the first hidden activations vanish for every input, so every sample
    # gives the same output, and dL/db_out is the mean residual
    n = mlp.n_params(4, 6, 2, 2)
    theta = rng.standard_normal(n)
    theta[: 6 * 4 + 6] = 0.0
    y, _ = mlp.forward(theta, X, 4, 6, 2, 2)
    assert np.allclose(y, y[0][None, :], atol=1e-15)
    _, g = mlp.loss_and_grad(theta, X, T, 4, 6, 2, 2)
    assert np.allclose(g[-2:], (y - T).mean(0), atol=1e-14)


def test_mlp_adam_first_step_is_signed_lr():
    """With m = v = 0 the first Adam step moves every parameter by lr * sign(g) (eps aside)."""
    from oracle import mlp

    g = np.array([0.3, -2.0, 1e-3, -5e-4])
    th, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01, eps=0.0)
    assert np.allclose(th, -0.01 * np.sign(g), rtol=1e-12)


# ------------------------------------------------------------------ level statistics


def test_spacing_ratios_worked_example():
    """Levels 0, 1, 3, 4, 4, 4: spacings 1, 2, 1, 0, 0 give ratios 1/2, 1/2, 0 and no ratio for
    the two zero spacings."""
    r, mean = levels.spacing_ratios([0.0, 1.0, 3.0, 4.0, 4.0, 4.0])
    assert np.array_equal(r[:3], [0.5, 0.5, 0.0]) and np.isnan(r[3])
    assert mean == pytest.approx(1.0 / 3.0, abs=1e-15)
    with pytest.raises(ValueError):
        levels.spacing_ratios([0.0, 2.0, 1.0])


def test_spacing_ratios_poisson_closed_form():
    """Uncorrelated levels (i.i.d. uniform): the ratio has density 2 / (1 + r)^2 on [0, 1], so its
    mean is 2 ln 2 - 1 and P(r < 0.1) = 2 (1 - 1/1.1).  2e5 levels: standard error ~7e-4."""
    E = np.sort(np.random.default_rng(0).uniform(0.0, 1.0, 200_000))
    r, mean = levels.spacing_ratios(E)
    assert abs(mean - (2 * np.log(2) - 1)) < 4e-3
    assert abs(np.mean(r < 0.1) - 2 * (1 - 1 / 1.1)) < 5e-3


def test_spacing_ratios_goe_level_repulsion():
    """Bulk levels of a GOE matrix (eigenvalues from numpy's LAPACK driver) repel: the mean ratio is
    about 0.53 (Atas et al. 2013), far above the Poisson 0.386, and small ratios are rare."""
    rng = np.random.default_rng(1)
    n = 1200
    A = rng.standard_normal((n, n))
    w = np.linalg.eigvalsh((A + A.T) / 2)
    r, mean = levels.spacing_ratios(w[n // 4: 3 * n // 4])
    assert abs(mean - 0.5307) < 0.03
    assert np.mean(r < 0.1) < 0.05


# ------------------------------------------------------------------ acceptance rule


def test_acceptance_worked_cases():
    """Hand-checked cases of the acceptance rule (block quadratic residual bound, ghosts, core)."""
    theta = [-0.3, -0.1, 0.05, 0.2, 0.6]  # (|theta|, theta) order: 0.05, -0.1, 0.2, -0.3, 0.6
    a, tol = 0.5, 1e-10
    # all converged: the core is the four values inside a; 0.6 lies beyond the window (a ghost,
    # since a - |theta| < 0); the best cluster of 0.05 is itself, 0.15 - 1e-12 from its neighbours
    core, est, ng = acceptance.accept(theta, [1e-12] * 5, a, tol)
    assert core == [0, 1, 2, 3] and ng == 1 and math.isinf(est[4])
    assert est[0] == pytest.approx(1e-24 / (0.15 - 1e-12), rel=1e-15)
    # -0.1 unconverged: it ends the core, and its residual moves it towards its neighbour 0.05
    core, est, ng = acceptance.accept(theta, [1e-12, 1e-3, 1e-12, 1e-12, 1e-12], a, tol)
    assert core == [0] and est[0] == pytest.approx(1e-24 / (0.15 - 1e-3), rel=1e-14)
    # its best cluster is all four values: their distance to the window edge, 0.2
    assert est[1] == pytest.approx(1e-6 / 0.2, rel=1e-10)
    # -0.1 a ghost (residual 3 >= a - 0.1): it represents no level and ends the core
    core, est, ng = acceptance.accept(theta, [1e-12, 3.0, 1e-12, 1e-12, 1e-12], a, tol)
    assert core == [0] and ng == 2 and math.isinf(est[1])
    assert est[0] == pytest.approx(1e-24 / (0.15 - 1e-12), rel=1e-15)
    # a near-degenerate pair 1e-9 apart with residuals 1e-8: alone, each is closer to its twin than
    # the twin's residual (no bound); the cluster {-0.2, 0, 1e-9} is 0.3 - 1e-9 - 1e-12 from 0.3
    theta = [-0.2, 0.0, 1e-9, 0.3]
    core, est, ng = acceptance.accept(theta, [1e-8, 1e-8, 1e-12, 1e-12], a, tol)
    assert core == [0, 1, 2, 3] and ng == 0
    assert est[0] == pytest.approx((1e-24 + 2e-16) / (0.3 - 1e-9 - 1e-12), rel=1e-12)
    # the same pair with residuals 1e-5: the cluster bound 2e-10 / 0.3 exceeds tol
    core, est, ng = acceptance.accept(theta, [1e-5, 1e-5, 1e-12, 1e-12], a, tol)
    assert core == [] and est[0] > tol
