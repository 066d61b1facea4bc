"""Parity of the HIP path (through the C ABI) with the CPU oracle, on MI355X.

Tolerances (derived in the module docstring of each group):
  * apply (FP64): each output element is a sum of <= L + 2 products of
    O(1) magnitudes, evaluated in a different order than the oracle, so the
    difference is a few ulp of sum |c| * max|x|: 1e-14 relative to that scale.
  * apply (FP32): the same sum in FP32 (unit roundoff 6e-8): 1e-6 relative.
  * recurrences: T_k(G) is bounded by 1, rounding accumulates at most
    linearly in k (Chebyshev recurrence stability), so 1e-15 * k relative to
    max|psi| (1e-12 floor); the filter output is normalised and dominated by
    its amplified window components: 1e-10 absolute on unit columns.
  * Gram / projection: 2 D terms of magnitude <= 1 summed in FP64 with a
    different blocking: 1e-13 * D relative to max |S|.
  * central eigenvalues: the target |delta lambda| <= 1e-10 ||H||, with
    counts matching exactly.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import central, chebyshev, hamiltonian, jordan_wigner, levels, philox, spectral, subspace  # noqa: E402
from oracle import _native  # noqa: E402
from paper_2011_02107_amd import binding as B  # noqa: E402
from paper_2011_02107_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def random_real_terms(L, seed, n):
    rng = np.random.default_rng(seed)
    pairs = [(1, 0), (3, 0), (1, 1), (2, 2), (3, 3), (1, 3), (3, 1), (2, 2)]
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


# ------------------------------------------------------------------ GEMM


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (37, 129, 70), (128, 128, 16), (300, 257, 513), (1100, 1030, 40)])
def test_dgemm_mfma_parity(ctx, ta, tb, M, N, K):
    rng = np.random.default_rng(M * 7 + N + K)
    A = rng.standard_normal((K, M) if ta else (M, K))
    Bm = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    ref = 0.5 * (A.T if ta else A) @ (Bm.T if tb else Bm) - 2.0 * C0
    dC = to_dev(C0)
    B.dacp_gemm(ctx, ta, tb, to_dev(A), to_dev(Bm), dC, alpha=0.5, beta=-2.0)
    assert np.abs(host(dC) - ref).max() < 1e-13 * max(1.0, np.abs(ref).max()) * math.sqrt(K)


def test_mfma_output_layout_single_tile(ctx):
    """One 16x16x4 product with distinct entries pins the accumulator lane layout."""
    A = np.arange(16 * 4, dtype=np.float64).reshape(16, 4) / 7.0
    Bm = np.arange(4 * 16, dtype=np.float64).reshape(4, 16) / 11.0 - 2.0
    dC = to_dev(np.zeros((16, 16)))
    B.dacp_gemm(ctx, 0, 0, to_dev(A), to_dev(Bm), dC)
    assert np.abs(host(dC) - A @ Bm).max() < 1e-13


# ------------------------------------------------------------------ apply


@pytest.mark.parametrize(
    "L,b,which",
    [(1, 1, "chain"), (3, 2, "chain"), (8, 4, "chain"), (10, 64, "chain"), (12, 8, "glass"), (9, 5, "random"),
     (11, 3, "paper_sgs"), (13, 1, "glass"), (14, 16, "chain")],
)
def test_apply_f64_parity(ctx, L, b, which):
    terms = {
        "chain": lambda: inputs.ising_chain(L),
        "glass": lambda: inputs.spin_glass(L, L),
        "random": lambda: random_real_terms(L, L, 25),
        "paper_sgs": lambda: inputs.paper_sgs(L, 3),
    }[which]()
    X = np.random.default_rng(L + b).standard_normal((1 << L, b))
    ref = hamiltonian.apply_h(L, terms, X)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    dy = torch.empty((1 << L, b), dtype=torch.float64, device=DEV)
    B.dacp_apply(ctx, ham, to_dev(X), dy)
    scale = hamiltonian.sum_abs_coeff(terms) * np.abs(X).max()
    assert np.abs(host(dy) - ref).max() <= 1e-14 * scale


@pytest.mark.parametrize(
    "L,b,which",
    [(15, 8, "chain"), (16, 8, "glass"), (15, 4, "random"), (16, 16, "paper_sgs"), (15, 1, "chain"), (16, 2, "paper_sgs")],
)
def test_apply_two_pass_parity(ctx, L, b, which):
    """L >= 15 with a power-of-two width runs the two-pass apply (low-bit tiles, then high-bit
    cosets, mixed masks gathered); same tolerance as the single-pass kernel."""
    terms = {
        "chain": lambda: inputs.ising_chain(L),
        "glass": lambda: inputs.spin_glass(L, L),
        "random": lambda: random_real_terms(L, L, 25),
        "paper_sgs": lambda: inputs.paper_sgs(L, 3),
    }[which]()
    X = np.random.default_rng(L * b).standard_normal((1 << L, b))
    ref = hamiltonian.apply_h(L, terms, X)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    dy = torch.empty((1 << L, b), dtype=torch.float64, device=DEV)
    B.dacp_apply(ctx, ham, to_dev(X), dy)
    scale = hamiltonian.sum_abs_coeff(terms) * np.abs(X).max()
    assert np.abs(host(dy) - ref).max() <= 1e-14 * scale
    dy32 = torch.empty((1 << L, b), dtype=torch.float32, device=DEV)
    B.dacp_apply(ctx, ham, to_dev(X, torch.float32), dy32)
    assert np.abs(host(dy32).astype(np.float64) - ref).max() <= 1e-6 * scale


def test_apply_f32_parity(ctx):
    L, b = 12, 32
    terms = inputs.ising_chain(L)
    X = np.random.default_rng(5).standard_normal((1 << L, b)).astype(np.float32)
    ref = hamiltonian.apply_h(L, terms, X.astype(np.float64))
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    dy = torch.empty((1 << L, b), dtype=torch.float32, device=DEV)
    B.dacp_apply(ctx, ham, to_dev(X, torch.float32), dy)
    scale = hamiltonian.sum_abs_coeff(terms) * np.abs(X).max()
    assert np.abs(host(dy).astype(np.float64) - ref).max() <= 1e-6 * scale


def test_hamiltonian_info_and_validation(ctx):
    L = 6
    terms = inputs.spin_glass(L, 1)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    info = ham.info()
    assert info["L"] == L and info["n_flip_groups"] == L
    assert abs(info["sum_abs"] - hamiltonian.sum_abs_coeff(terms)) < 1e-12
    assert abs(info["sum_sq"] - hamiltonian.sum_sq_coeff(terms)) < 1e-12
    for bad in (
        inputs.make_terms([(2, 0, 0, 0, 1.0)]),  # single Y: imaginary
        inputs.make_terms([(1, 7, 0, 0, 1.0)]),  # site >= L
        inputs.make_terms([(3, 2, 3, 2, 1.0)]),  # two-body on one site
    ):
        with pytest.raises(B.DacpError) as ei:
            B.dacp_build_hamiltonian(ctx, L, bad)
        assert ei.value.status == -1


# ------------------------------------------------------------------ random start states


def test_philox_block_matches_oracle(ctx):
    D, b, seed = 4096, 8, 0x1234_5678_9ABC
    out = torch.empty((D, b), dtype=torch.float64, device=DEV)
    B.dacp_random_block(ctx, D, b, seed, out)
    ref = philox.gaussian_block(D, b, seed)
    assert np.abs(host(out) - ref).max() < 1e-13


# ------------------------------------------------------------------ bound and density


def test_spectral_bound_parity_and_validity(ctx):
    L = 10
    terms = inputs.ising_chain(L)
    v0 = np.random.default_rng(3).standard_normal(1 << L)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    eb, tlo, thi = B.dacp_spectral_bound(ctx, ham, 60, v0=to_dev(v0))
    al, be = spectral.lanczos(lambda X: hamiltonian.apply_h(L, terms, X), v0, 60)
    eb_ref, theta = spectral.lanczos_bound(al, be, hamiltonian.sum_abs_coeff(terms))
    assert abs(tlo - theta[0]) < 1e-9 and abs(thi - theta[-1]) < 1e-9
    assert abs(eb - eb_ref) < 1e-6 * eb_ref
    w = central.full_spectrum_dense(L, terms)
    assert eb >= max(-w[0], w[-1])


def test_dos_moments_parity(ctx):
    L, nvec, M = 11, 4, 64
    terms = inputs.spin_glass(L, 2)
    R = np.random.default_rng(4).standard_normal((1 << L, nvec))
    eb = 1.02 * np.abs(central.full_spectrum_dense(L, terms)).max()
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    mu = B.dacp_dos_moments(ctx, ham, eb, M, nvec, R=to_dev(R))
    ref = spectral.kpm_moments(lambda X: hamiltonian.apply_h(L, terms, X), R, eb, M)
    assert np.abs(mu - ref).max() < 1e-11


# ------------------------------------------------------------------ filter and basis


@pytest.mark.parametrize("L,b,kfac", [(8, 2, 12.0), (10, 4, 18.0)])
def test_filter_f64_parity(ctx, L, b, kfac):
    terms = inputs.ising_chain(L)
    w = central.full_spectrum_dense(L, terms)
    eb = 1.01 * np.abs(w).max()
    a = 0.08 * eb
    K = chebyshev.filter_order(eb, a, kfac)
    psi = np.random.default_rng(L).standard_normal((1 << L, b))
    ref = chebyshev.exp_semicircle_filter(lambda X: hamiltonian.apply_h(L, terms, X), psi, eb, a, K)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    out = torch.empty((1 << L, b), dtype=torch.float64, device=DEV)
    B.dacp_filter(ctx, ham, out, eb, a, K, start=to_dev(psi))
    assert np.abs(host(out) - ref).max() < 1e-10


def test_filter_grouped_two_pass_parity(ctx):
    """L = 15, b = 16: the filter runs per column group of 8 with the two-pass apply."""
    L, b = 15, 16
    terms = inputs.spin_glass(L, 11)
    eb = 1.01 * hamiltonian.sum_abs_coeff(terms)
    a = 0.3 * eb
    K = chebyshev.filter_order(eb, a, 12.0)
    psi = np.random.default_rng(6).standard_normal((1 << L, b))
    ref = chebyshev.exp_semicircle_filter(lambda X: hamiltonian.apply_h(L, terms, X), psi, eb, a, K)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    out = torch.empty((1 << L, b), dtype=torch.float64, device=DEV)
    B.dacp_filter(ctx, ham, out, eb, a, K, start=to_dev(psi))
    assert np.abs(host(out) - ref).max() < 1e-10


def test_filter_f32_with_fp64_tail(ctx):
    """FP32 recurrence then an FP64 tail: the output stays within FP32-rounding
    distance of the FP64 oracle filter (window components dominate)."""
    L, b = 10, 4
    terms = inputs.ising_chain(L)
    eb = 1.01 * np.abs(central.full_spectrum_dense(L, terms)).max()
    a = 0.08 * eb
    K = chebyshev.filter_order(eb, a, 12.0)
    psi = np.random.default_rng(1).standard_normal((1 << L, b))
    ref = chebyshev.exp_semicircle_filter(lambda X: hamiltonian.apply_h(L, terms, X), psi, eb, a, K)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    out = torch.empty((1 << L, b), dtype=torch.float64, device=DEV)
    B.dacp_filter(ctx, ham, out, eb, a, K, start=to_dev(psi), precision=B.DACP_F32, fp64_tail=K // 5)
    err = np.abs(host(out) - ref).max()
    assert err < 1e-5


@pytest.mark.parametrize("which", ["chain", "signed"])
def test_filter_fused_chain_f64_parity(ctx, which):
    """L = 16, b = 16: the FP64 filter orders run as the fused split chain (groups of 8), including
    the old-term read of the low kernel; signed flips exercise the z-mask path."""
    L, b = 16, 16
    terms = inputs.ising_chain(L) if which == "chain" else _signed_flip_terms(L, 5)
    eb = 1.02 * hamiltonian.sum_abs_coeff(terms)
    a = 0.3 * eb
    K = chebyshev.filter_order(eb, a, 12.0)
    psi = np.random.default_rng(17).standard_normal((1 << L, b))
    ref = chebyshev.exp_semicircle_filter(lambda X: hamiltonian.apply_h(L, terms, X), psi, eb, a, K)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    out = torch.empty((1 << L, b), dtype=torch.float64, device=DEV)
    B.dacp_filter(ctx, ham, out, eb, a, K, start=to_dev(psi))
    assert np.abs(host(out) - ref).max() < 1e-10
    # same orders through the unfused applies
    out2 = torch.empty_like(out)
    try:
        ctx.tune("fused", 0)
        B.dacp_filter(ctx, ham, out2, eb, a, K, start=to_dev(psi))
    finally:
        ctx.tune("fused", 1)
    assert np.abs(host(out2) - host(out)).max() < 1e-12


@pytest.mark.parametrize("g32", [8, 16])
def test_filter_fused_chain_f32_tail(ctx, g32):
    """L = 16, b = 16: FP32 orders as the fused chain (float kernels) on groups of 8 or one group of
    16, then the FP64 tail on the same groups (fused at 8 columns, the single-pass apply at 16)."""
    L, b = 16, 16
    terms = _signed_flip_terms(L, 6)
    eb = 1.02 * hamiltonian.sum_abs_coeff(terms)
    a = 0.3 * eb
    K = chebyshev.filter_order(eb, a, 12.0)
    psi = np.random.default_rng(18).standard_normal((1 << L, b))
    ref = chebyshev.exp_semicircle_filter(lambda X: hamiltonian.apply_h(L, terms, X), psi, eb, a, K)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    out = torch.empty((1 << L, b), dtype=torch.float64, device=DEV)
    try:
        ctx.tune("filter_group_f32", g32)
        B.dacp_filter(ctx, ham, out, eb, a, K, start=to_dev(psi), precision=B.DACP_F32, fp64_tail=K // 3)
    finally:
        ctx.tune("filter_group_f32", 8)
    assert np.abs(host(out) - ref).max() < 1e-5 * np.abs(ref).max()


def test_basis_parity(ctx):
    L, b, n = 9, 3, 5
    terms = inputs.spin_glass(L, 7)
    eb = 1.01 * np.abs(central.full_spectrum_dense(L, terms)).max()
    a = 0.1 * eb
    psi = np.random.default_rng(2).standard_normal((1 << L, b))
    psi /= np.linalg.norm(psi, axis=0)
    ref, ks = chebyshev.chebyshev_basis(lambda X: hamiltonian.apply_h(L, terms, X), psi, eb, a, n)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    m = b * (2 * n + 1)
    V = torch.zeros((1 << L, m), dtype=torch.float64, device=DEV)
    got_m = B.dacp_basis(ctx, ham, to_dev(psi), V, eb, a, n)
    assert got_m == m
    assert np.abs(host(V) - ref).max() < 1e-15 * max(ks) + 1e-12


def test_basis_column_groups_match_full_block(ctx):
    L, b, n = 10, 8, 3
    terms = inputs.ising_chain(L)
    eb = 1.01 * np.abs(central.full_spectrum_dense(L, terms)).max()
    psi = np.random.default_rng(9).standard_normal((1 << L, b))
    psi /= np.linalg.norm(psi, axis=0)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    m = b * (2 * n + 1)
    V1 = torch.zeros((1 << L, m), dtype=torch.float64, device=DEV)
    V2 = torch.zeros_like(V1)
    B.dacp_basis(ctx, ham, to_dev(psi), V1, eb, 0.2 * eb, n, group=0)
    B.dacp_basis(ctx, ham, to_dev(psi), V2, eb, 0.2 * eb, n, group=3)
    assert np.array_equal(host(V1), host(V2))


def test_basis_two_pass_groups_match_oracle(ctx):
    """L = 15 runs the evolution in column groups of 8 with the two-pass apply."""
    L, b, n = 15, 16, 2
    terms = inputs.ising_chain(L)
    eb = 1.01 * (1.723 * L)  # above ||H|| for this chain (checked by the norm guard of dacp_basis)
    a = 0.3 * eb
    psi = np.random.default_rng(5).standard_normal((1 << L, b))
    psi /= np.linalg.norm(psi, axis=0)
    ref, ks = chebyshev.chebyshev_basis(lambda X: hamiltonian.apply_h(L, terms, X), psi, eb, a, n)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    V = torch.zeros((1 << L, b * (2 * n + 1)), dtype=torch.float64, device=DEV)
    B.dacp_basis(ctx, ham, to_dev(psi), V, eb, a, n)
    assert np.abs(host(V) - ref).max() < 1e-15 * max(ks) + 1e-12


def _signed_flip_terms(L, seed):
    """Chain plus X Z and Y Y terms whose x-masks never straddle the middle bits (sign paths of the
    fused kernels), with a single-spin-flip part that keeps every fused split admissible."""
    rng = np.random.default_rng(seed)
    X, Y, Z = inputs.X, inputs.Y, inputs.Z
    rows = [(Y, i, Y, i + 1, rng.uniform(-0.5, 0.5)) for i in (0, 1, L - 3, L - 2)]
    for _ in range(4):
        i, j = rng.choice(L, 2, replace=False)
        rows.append((X, int(i), Z, int(j), rng.uniform(-0.5, 0.5)))
    return np.concatenate([inputs.ising_chain(L), inputs.make_terms(rows)])


@pytest.mark.parametrize("g", [2, 4, 8])
@pytest.mark.parametrize("threads,hi_w,rec_tile,persist", [(1024, 0, 8192, 0), (512, 0, 8192, 0), (1024, 1, 4096, 0),
                                                           (512, 2, 4096, 0), (1024, 8, 8192, 0), (1024, 1, 4096, 1),
                                                           (512, 0, 8192, 2), (1024, 0, 2048, 3)])
def test_basis_fused_layouts_match_oracle(ctx, g, threads, hi_w, rec_tile, persist):
    L, b, n = 16, 8, 1
    terms = _signed_flip_terms(L, 3)
    eb = 1.05 * hamiltonian.sum_abs_coeff(terms)
    a = 0.45 * eb
    psi = np.random.default_rng(11).standard_normal((1 << L, b))
    psi /= np.linalg.norm(psi, axis=0)
    ref, ks = chebyshev.chebyshev_basis(lambda X: hamiltonian.apply_h(L, terms, X), psi, eb, a, n)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    V = torch.zeros((1 << L, b * (2 * n + 1)), dtype=torch.float64, device=DEV)
    try:
        ctx.tune("rec_threads", threads)
        ctx.tune("rec_hi_w", hi_w)
        ctx.tune("rec_tile", rec_tile)
        ctx.tune("rec_persist", persist)
        B.dacp_basis(ctx, ham, to_dev(psi), V, eb, a, n, group=g)
    finally:
        ctx.tune("rec_persist", 0)
        ctx.tune("rec_threads", 1024)
        ctx.tune("rec_hi_w", 0)
        ctx.tune("rec_tile", 8192)
    assert np.abs(host(V) - ref).max() < 1e-15 * max(ks) + 1e-12


def test_basis_graph_replay_matches_step_launches(ctx):
    """Below 2^19 rows, runs of sample-free evolution steps replay a captured hipGraph (rec_graph
    steps each): the basis equals, bit for bit, the one launched step by step, and the oracle."""
    L, b, n = 16, 8, 2
    terms = _signed_flip_terms(L, 5)
    eb = 1.05 * hamiltonian.sum_abs_coeff(terms)
    a = 0.02 * eb
    psi = np.random.default_rng(13).standard_normal((1 << L, b))
    psi /= np.linalg.norm(psi, axis=0)
    ref, ks = chebyshev.chebyshev_basis(lambda X: hamiltonian.apply_h(L, terms, X), psi, eb, a, n)
    assert max(ks) > 4 * 32  # long enough for graph runs between the samples
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    V0 = torch.zeros((1 << L, b * (2 * n + 1)), dtype=torch.float64, device=DEV)
    V1 = torch.zeros_like(V0)
    B.dacp_basis(ctx, ham, to_dev(psi), V0, eb, a, n, group=8)
    try:
        ctx.tune("rec_graph", 32)
        B.dacp_basis(ctx, ham, to_dev(psi), V1, eb, a, n, group=8)
    finally:
        ctx.tune("rec_graph", 0)
    assert torch.equal(V0, V1)
    assert np.abs(host(V1) - ref).max() < 1e-15 * max(ks) + 1e-12


def test_basis_detects_bound_below_norm(ctx):
    L = 8
    terms = inputs.ising_chain(L)
    norm = np.abs(central.full_spectrum_dense(L, terms)).max()
    psi = np.random.default_rng(0).standard_normal((1 << L, 2))
    psi /= np.linalg.norm(psi, axis=0)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    V = torch.zeros((1 << L, 2 * 9), dtype=torch.float64, device=DEV)
    with pytest.raises(B.DacpError) as ei:
        B.dacp_basis(ctx, ham, to_dev(psi), V, 0.9 * norm, 0.05 * norm, 4)
    assert ei.value.status == -4


# ------------------------------------------------------------------ projection and GEP


def test_project_parity(ctx):
    L, m = 11, 150
    terms = inputs.spin_glass(L, 4)
    V = np.random.default_rng(6).standard_normal((1 << L, m)) / math.sqrt(1 << L)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    S = torch.zeros((m, m), dtype=torch.float64, device=DEV)
    P = torch.zeros((m, m), dtype=torch.float64, device=DEV)
    B.dacp_project(ctx, ham, to_dev(V), S, P)
    S_ref, P_ref = subspace.project(lambda X: hamiltonian.apply_h(L, terms, X), V)
    assert np.abs(host(S) - S_ref).max() < 1e-13
    assert np.abs(host(P) - P_ref).max() < 1e-12
    assert np.array_equal(host(S), host(S).T) and np.array_equal(host(P), host(P).T)


def test_project_parity_many_tile_blocks(ctx):
    """m = 1100: 9 x 9 output tiles, so the Gram's upper-triangle walk spans several 8 x 8 tile
    blocks, including the ragged last block row and column."""
    L, m = 10, 1100
    terms = inputs.spin_glass(L, 9)
    V = np.random.default_rng(9).standard_normal((1 << L, m)) / math.sqrt(1 << L)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    S = torch.zeros((m, m), dtype=torch.float64, device=DEV)
    P = torch.zeros((m, m), dtype=torch.float64, device=DEV)
    B.dacp_project(ctx, ham, to_dev(V), S, P)
    S_ref, P_ref = subspace.project(lambda X: hamiltonian.apply_h(L, terms, X), V)
    assert np.abs(host(S) - S_ref).max() < 1e-13
    assert np.abs(host(P) - P_ref).max() < 1e-12 * max(1.0, np.abs(P_ref).max())
    assert np.array_equal(host(S), host(S).T) and np.array_equal(host(P), host(P).T)


def test_project_parity_split_k(ctx):
    """Column-chunked P at D = 2^16 splits K over several workgroup layers (narrow P chunks);
    two chunks of 512 and 128 columns.  Then the one-GEMM form of P on the same input."""
    L, m = 16, 640
    terms = inputs.ising_chain(L)
    V = np.random.default_rng(8).standard_normal((1 << L, m)) / math.sqrt(1 << L)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    S = torch.zeros((m, m), dtype=torch.float64, device=DEV)
    P = torch.zeros((m, m), dtype=torch.float64, device=DEV)
    try:
        ctx.tune("project_splitk", 0)
        ctx.tune("project_whole", 0)
        B.dacp_project(ctx, ham, to_dev(V), S, P)
        ctx.tune("project_whole", 1)
        # the one-GEMM form on the same input
        P1 = torch.zeros_like(P)
        B.dacp_project(ctx, ham, to_dev(V), S, P1)
    finally:
        ctx.tune("project_whole", 1)
        ctx.tune("project_splitk", 1)
    S_ref, P_ref = subspace.project(lambda X: hamiltonian.apply_h(L, terms, X), V)
    assert np.abs(host(S) - S_ref).max() < 1e-13
    assert np.abs(host(P) - P_ref).max() < 1e-12 * np.abs(P_ref).max()
    assert np.abs(host(P1) - P_ref).max() < 1e-12 * np.abs(P_ref).max()
    # upper-triangle tiles with K split 35 ways (15 tiles), mirrored
    S2, P2 = torch.zeros_like(S), torch.zeros_like(P)
    B.dacp_project(ctx, ham, to_dev(V), S2, P2)
    assert np.abs(host(S2) - S_ref).max() < 1e-13
    assert np.abs(host(P2) - P_ref).max() < 1e-12 * np.abs(P_ref).max()
    assert np.array_equal(host(S2), host(S2).T) and np.array_equal(host(P2), host(P2).T)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 130, 400])
def test_syev_parity(ctx, n):
    A = np.random.default_rng(n).standard_normal((n, n))
    A = A + A.T
    w_ref = _native.syev(A)
    dA = to_dev(A)
    Z = torch.zeros((n, n), dtype=torch.float64, device=DEV)
    w = B.dacp_syev(ctx, dA, Z)
    assert np.abs(w - w_ref).max() < 1e-12 * max(1.0, np.abs(w_ref).max()) * max(1, n) ** 0.5
    Zr = host(Z)  # rows are eigenvectors
    assert np.abs(Zr @ A @ Zr.T - np.diag(w)).max() < 1e-12 * max(1.0, np.abs(w).max()) * n
    assert np.abs(Zr @ Zr.T - np.eye(n)).max() < 1e-13 * n


def _check_eig(ctx, A, tol_scale=1.0):
    n = A.shape[0]
    w_ref = _native.syev(A)
    Z = torch.zeros((n, n), dtype=torch.float64, device=DEV)
    w = B.dacp_syev(ctx, to_dev(A), Z)
    scale = max(1.0, np.abs(w_ref).max())
    assert np.abs(w - w_ref).max() < 1e-12 * scale * max(1, n) ** 0.5 * tol_scale
    Zr = host(Z)
    assert np.abs(Zr @ A @ Zr.T - np.diag(w)).max() < 1e-12 * scale * n * tol_scale
    assert np.abs(Zr @ Zr.T - np.eye(n)).max() < 1e-13 * n


@pytest.mark.parametrize("n", [97, 1000, 2047])
def test_syev_divide_and_conquer_random(ctx, n):
    A = np.random.default_rng(n).standard_normal((n, n))
    _check_eig(ctx, A + A.T)


@pytest.mark.parametrize("n", [300, 1000, 2047])
def test_syev_blocked_tridiagonalisation(ctx, n):
    """The panel tridiagonalisation and compact-WY Q formation (the default from n = 3500 on)
    forced at smaller sizes, including a ragged last panel."""
    A = np.random.default_rng(n + 5).standard_normal((n, n))
    try:
        ctx.tune("blocked", 256)
        _check_eig(ctx, A + A.T)
    finally:
        ctx.tune("blocked", 3500)


def test_syev_batched_matches_oracle(ctx):
    """One launch, one workgroup per matrix, mixed sizes (1, 2, 3 and odd sizes up to 700), including a
    diagonal and a repeated-eigenvalue matrix; eigenvalues against the oracle's eigensolver,
    eigenvectors through A Z^T = Z^T diag(w) and orthonormality."""
    rng = np.random.default_rng(21)
    mats = []
    for n in (1, 2, 3, 17, 130, 257, 700):
        X = rng.standard_normal((n, n))
        mats.append(X + X.T)
    mats.append(np.diag(rng.standard_normal(40)))
    u = rng.standard_normal((60, 2))
    mats.append(np.eye(60) + u @ u.T)
    As = [to_dev(A) for A in mats]
    Zs = [torch.zeros(A.shape, dtype=torch.float64, device=DEV) for A in mats]
    ws = B.dacp_syev_batched(ctx, As, Zs)
    for A, w, Z in zip(mats, ws, Zs):
        n = A.shape[0]
        w_ref = _native.syev(A)
        scale = max(1.0, np.abs(w_ref).max())
        assert np.abs(w - w_ref).max() < 1e-12 * scale * max(1, n) ** 0.5
        Zr = host(Z)
        assert np.abs(Zr @ A @ Zr.T - np.diag(w)).max() < 1e-12 * scale * n
        assert np.abs(Zr @ Zr.T - np.eye(n)).max() < 1e-13 * n


@pytest.mark.parametrize("sizes", [(1100, 40), (2048,)], ids=["two_sweeps_per_batch", "one_sweep_per_batch"])
def test_syev_batched_large_sizes(ctx, sizes):
    """The largest matrix of a launch sets how many QR sweeps share one pass over Zr (fewer at
    large n, where their Givens buffers fill the LDS); a Gram-like PSD matrix (rank 2/3 n, wide
    spread of eigenvalues) rides along with the largest."""
    rng = np.random.default_rng(22)
    mats = []
    for n in sizes:
        X = rng.standard_normal((n, n))
        mats.append(X + X.T)
    n0, r = 300, 200
    X = rng.standard_normal((r, n0)) * np.logspace(0, -7, n0)[None, :]
    mats.append(X.T @ X)
    As = [to_dev(A) for A in mats]
    Zs = [torch.zeros(A.shape, dtype=torch.float64, device=DEV) for A in mats]
    ws = B.dacp_syev_batched(ctx, As, Zs)
    for A, w, Z in zip(mats, ws, Zs):
        n = A.shape[0]
        w_ref = _native.syev(A)
        scale = max(1.0, np.abs(w_ref).max())
        assert np.abs(w - w_ref).max() < 1e-12 * scale * max(1, n) ** 0.5
        Zr = host(Z)
        assert np.abs(Zr @ A @ Zr.T - np.diag(w)).max() < 1e-12 * scale * n
        assert np.abs(Zr @ Zr.T - np.eye(n)).max() < 1e-13 * n


def test_syev_batched_rejects_large(ctx):
    A = torch.zeros((2049, 2049), dtype=torch.float64, device=DEV)
    with pytest.raises(B.DacpError) as ei:
        B.dacp_syev_batched(ctx, [A])
    assert ei.value.status == -1


def test_syev_divide_and_conquer_deflation_cases(ctx):
    n = 300
    rng = np.random.default_rng(1)
    # diagonal: every z component deflates
    _check_eig(ctx, np.diag(rng.standard_normal(n)))
    # repeated eigenvalues: identity plus a rank-two update
    u = rng.standard_normal((n, 2))
    _check_eig(ctx, np.eye(n) + u @ u.T)
    # clustered spectrum from a random orthogonal similarity
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat([-1.0, 0.0, 2.0], n // 3) + 1e-10 * rng.standard_normal(n)
    _check_eig(ctx, (q * lam) @ q.T)


def test_syev_gram_like_psd(ctx):
    """Overlap-matrix-like input: PSD of rank ~ 2/3 n with a wide spread of eigenvalues."""
    n, r = 600, 400
    rng = np.random.default_rng(2)
    X = rng.standard_normal((r, n)) * np.logspace(0, -7, n)[None, :]
    _check_eig(ctx, X.T @ X)


def test_rayleigh_ritz_parity(ctx):
    """Same S, P on both sides: the App. C solve gives the same Ritz values."""
    L = 9
    terms = inputs.ising_chain(L)
    lam, Phi = np.linalg.eigh(hamiltonian.dense_h(L, terms))
    rng = np.random.default_rng(8)
    sel = np.arange(200, 240)
    core = Phi[:, sel] @ rng.standard_normal((len(sel), len(sel)))
    V = np.concatenate([core, core[:, :10] @ rng.standard_normal((10, 6))], axis=1)
    S, P = subspace.project(lambda X: hamiltonian.apply_h(L, terms, X), V)
    theta_ref, _, r_ref = subspace.rayleigh_ritz(S, P)
    theta, r = B.dacp_rayleigh_ritz(ctx, to_dev(S), to_dev(P))
    assert r == r_ref == len(sel)
    assert np.abs(theta - theta_ref).max() < 1e-10
    assert np.abs(theta - lam[sel]).max() < 1e-10


# ------------------------------------------------------------------ end to end


def _check_central(got, ref, norm, N, errs=None):
    """Counts, order and values against the oracle; with `errs`, every returned error estimate must
    bound the true error (up to the rounding of the value itself, 64 eps ||H||)."""
    assert len(got) == N
    assert np.all(np.diff(got) >= 0)
    err = np.abs(np.sort(got) - ref)
    assert err.max() <= 1e-10 * norm
    if errs is not None:
        below = err > np.asarray(errs) + 64 * 2.220446049250313e-16 * norm
        assert not below.any(), f"{int(below.sum())} estimates below the true error (max {err.max():.2e})"


def test_central_eigs_chain_L10(ctx):
    """Chaotic Ising chain L = 10, N = 100, block of 4 start states."""
    L, N = 10, 100
    terms = inputs.ising_chain(L)
    ref, norm = central.central_eigenvalues(L, terms, N)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    for seed in (0, 1, 2):
        opts = B.default_opts(b=4, seed=seed)
        eigs, errs, rep, st = B.dacp_central_eigs(ctx, ham, N, opts)
        _check_central(eigs, ref, norm, N, errs=errs)
        assert np.all(errs <= 1e-10 * norm)


def test_central_eigs_spin_glass_L12(ctx):
    L, N = 12, 200
    terms = inputs.spin_glass(L, 0)
    ref, norm = central.central_eigenvalues(L, terms, N)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    eigs, errs, rep, st = B.dacp_central_eigs(ctx, ham, N, B.default_opts(b=8))
    _check_central(eigs, ref, norm, N, errs=errs)


def test_central_eigs_jw_twin_L14(ctx):
    """Integrable twin (hz = 0) against the Jordan-Wigner closed form."""
    L, N = 14, 300
    terms = inputs.ising_chain(L, hz=0.0)
    ref, norm = central.central_eigenvalues_jw(np.ones(L - 1), 1.05 * np.ones(L), N)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    eigs, errs, rep, st = B.dacp_central_eigs(ctx, ham, N, B.default_opts(b=16))
    _check_central(eigs, ref, norm, N, errs=errs)


def _check_eigvecs(X, eigs, errs, Hd, norm, a):
    """Unit vectors whose Rayleigh quotient is the returned value, whose residual r = H x - theta x
    obeys the acceptance rule (estimate min(||r||, ||r||^2 / eta) <= 1e-10 ||H|| with eta <= a, so
    ||r|| <= sqrt(1e-10 ||H|| a)), and whose angle to the dense eigenvector of the nearest level is
    at most ||r|| / delta, delta = distance from theta to every other level (the sin-theta bound of
    a Ritz pair).

    Rounding: x = V b with b = U y, U = S's eigenvectors over sqrt(eigenvalues) >= sqrt(1e-12), so
    the FP64 product cancels by up to ~1e6 and x carries relative errors up to ~1e-10: the norm and
    angle checks allow 1e-9 absolute; the Rayleigh quotient is second order in them."""
    lam, Phi = np.linalg.eigh(Hd)
    N = len(eigs)
    nrm2 = np.einsum("si,si->i", X, X)
    assert np.abs(np.sqrt(nrm2) - 1.0).max() < 1e-9
    assert np.abs(np.einsum("si,si->i", X, Hd @ X) / nrm2 - eigs).max() <= 1e-12 * norm
    rn = np.linalg.norm(Hd @ X - X * eigs[None, :], axis=0)
    assert np.all(errs <= rn * (1 + 1e-6) + 1e-13 * norm)  # the estimate never exceeds ||r||
    assert rn.max() <= 1.01 * math.sqrt(1.01e-10 * norm * a) + 1e-13 * norm
    sin_max = 0.0
    for i in range(N):
        k = int(np.argmin(np.abs(lam - eigs[i])))
        others = np.delete(lam, k)
        delta = np.abs(others - eigs[i]).min()
        perp = X[:, i] - Phi[:, k] * (Phi[:, k] @ X[:, i])
        sin_t = np.linalg.norm(perp)
        assert sin_t <= rn[i] / delta * 1.01 + 1e-9, (i, sin_t, rn[i], delta)
        sin_max = max(sin_max, sin_t)
    # orthogonality follows from the angles: |x_i . x_j| <= sin_i + sin_j for distinct levels
    G = X.T @ X
    np.fill_diagonal(G, 0.0)
    assert np.abs(G).max() <= 2 * sin_max + 1e-9
    return sin_max


def test_central_eigpairs_vectors_against_dense_eigenvectors(ctx):
    """Eigenvector output (Sec. II.C Ritz vectors) of the L = 10 spin glass and the L = 11 chain:
    the values equal dacp_central_eigs', the vectors land in the requested columns of a padded
    block and satisfy the Ritz-pair angle bound against the dense eigenvectors."""
    for L, N, terms, ld in ((10, 100, inputs.spin_glass(10, 3), 103), (11, 64, inputs.ising_chain(11), 64)):
        Hd = hamiltonian.dense_h(L, terms)
        ref, norm = central.central_eigenvalues(L, terms, N)
        ham = B.dacp_build_hamiltonian(ctx, L, terms)
        opts = B.default_opts(b=4)
        e0, r0, _, _ = B.dacp_central_eigs(ctx, ham, N, opts)
        vecs = torch.full((1 << L, ld), float("nan"), dtype=torch.float64, device=DEV)
        eigs, errs, rep, st = B.dacp_central_eigpairs(ctx, ham, N, vecs, opts)
        _check_central(eigs, ref, norm, N, errs=errs)
        assert np.array_equal(eigs, e0) and np.array_equal(errs, r0)
        Xp = host(vecs)
        assert np.isnan(Xp[:, N:]).all()  # the padding columns are left alone
        _check_eigvecs(Xp[:, :N], eigs, errs, Hd, norm, rep["a"])


def test_central_eigpairs_chain_L16_properties(ctx):
    """At L = 16, N = 1000 (no dense oracle), in the benchmark's tuned options: the returned vectors,
    checked with the oracle's CPU matrix-free apply, are unit and mutually orthogonal up to the
    S cut-off's rounding, their Rayleigh quotients are the returned values and their residuals obey
    the acceptance rule's bound ||r|| <= sqrt(1e-10 ||H|| a) (||H|| <= sum |c|)."""
    L, N = 16, 1000
    terms = inputs.ising_chain(L)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    opts = B.default_opts(b=64, kfac=12.0, window_ratio=2.2, basis_ratio=1.2, precision=B.DACP_F32,
                          fp64_tail_frac=0.3)
    vecs = torch.empty((1 << L, N), dtype=torch.float64, device=DEV)
    eigs, errs, rep, st = B.dacp_central_eigpairs(ctx, ham, N, vecs, opts)
    assert len(eigs) == N and np.all(np.diff(eigs) >= 0)
    X = host(vecs)
    del vecs
    bound = hamiltonian.sum_abs_coeff(terms)
    HX = hamiltonian.apply_h(L, terms, X)
    nrm2 = np.einsum("si,si->i", X, X)
    assert np.abs(np.sqrt(nrm2) - 1.0).max() < 1e-9
    G = X.T @ X
    np.fill_diagonal(G, 0.0)
    assert np.abs(G).max() < 1e-8
    assert np.abs(np.einsum("si,si->i", X, HX) / nrm2 - eigs).max() <= 1e-12 * bound
    rn = np.linalg.norm(HX - X * eigs[None, :], axis=0)
    assert rn.max() <= 1.01 * math.sqrt(1.01e-10 * bound * rep["a"]) + 1e-13 * bound
    assert np.all(errs <= rn * (1 + 1e-6) + 1e-13 * bound)


def test_central_eigpairs_rejects_bad_stride(ctx):
    L, N = 10, 20
    ham = B.dacp_build_hamiltonian(ctx, L, inputs.ising_chain(L))
    vecs = torch.zeros((1 << L, N), dtype=torch.float64, device=DEV)
    opts = B.default_opts(b=4)
    eigs = np.zeros(N)
    n_out = B.ctypes.c_int()
    st = ctx.lib.dacp_central_eigpairs(ctx.handle, ham.handle, N, B.ctypes.byref(opts), B._f64(eigs), None,
                                       B._ptr(vecs), N - 1, B.ctypes.byref(n_out), None)
    assert st == -1
    st = ctx.lib.dacp_central_eigpairs(ctx.handle, ham.handle, N, B.ctypes.byref(opts), B._f64(eigs), None, None,
                                       N, B.ctypes.byref(n_out), None)
    assert st == -1


def test_central_eigs_paper_tfim_L14_against_jordan_wigner(ctx):
    """The paper's random transverse-field chain, (1/4) sum J X X + (1/2) sum Gamma Z with
    J ~ U[-10/sqrt(L), 10/sqrt(L)] and Gamma ~ U[0, 1] (Sec. III), against its Jordan-Wigner
    spectrum (x and z exchanged: couplings J/4, fields Gamma/2)."""
    L, N = 14, 300
    terms = inputs.paper_tfim(L, 2)
    Jb = np.array([t["coeff"] for t in terms if t["op_b"] == 1])
    g = np.array([t["coeff"] for t in terms if t["op_b"] == 0])
    ref, norm = central.central_eigenvalues_jw(Jb, g, N)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    eigs, errs, rep, st = B.dacp_central_eigs(ctx, ham, N, B.default_opts(b=16))
    _check_central(eigs, ref, norm, N, errs=errs)
    # gap ratios of the computed levels: each level is within 1e-10 ||H||, so each spacing within
    # 2e-10 ||H|| and each ratio within (1 + r) 2e-10 ||H|| / max(s_i, s_i+1) of the exact one
    r, _ = B.dacp_spacing_ratios(eigs)
    r_ref, _ = levels.spacing_ratios(ref)
    s = np.diff(ref)
    assert np.all(np.abs(r - r_ref) <= 4.4e-10 * norm / np.maximum(s[:-1], s[1:]) + 1e-12)


def test_central_eigs_paper_spin_glass_shard_L12(ctx):
    """The paper's spin-glass shard, sum_{i<j} J_ij X_i X_j + sum Gamma_i Z_i with the same
    distributions (Sec. III), against the dense oracle."""
    L, N = 12, 200
    terms = inputs.paper_sgs(L, 5)
    ref, norm = central.central_eigenvalues(L, terms, N)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    eigs, errs, rep, st = B.dacp_central_eigs(ctx, ham, N, B.default_opts(b=8))
    _check_central(eigs, ref, norm, N, errs=errs)


@pytest.mark.parametrize("moment_mode", [0, 2])
def test_central_eigs_jw_twin_L20_full_size(ctx, moment_mode):
    """Full size, in the benchmark's tuned configuration (D = 2^20, N = 5000, b = 64, FP32 filter with
    an FP64 tail, window 2.4 N, basis ratio 1.2), with S and P as explicit products (0) and from the
    anchor panels' moments (2, the benchmark's): the integrable twin (hz = 0) of the benchmark chain
    against the exact Jordan-Wigner spectrum, every one of the N values."""
    L, N = 20, 5000
    terms = inputs.ising_chain(L, hz=0.0)
    ref, norm = central.central_eigenvalues_jw(np.ones(L - 1), 1.05 * np.ones(L), N)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    opts = B.default_opts(b=64, kfac=12.0, window_ratio=2.4, basis_ratio=1.2, precision=B.DACP_F32,
                          fp64_tail_frac=0.3, moment_mode=moment_mode)
    import time

    t0 = time.perf_counter()
    eigs, errs, rep, st = B.dacp_central_eigs(ctx, ham, N, opts)
    dt = time.perf_counter() - t0
    _check_central(eigs, ref, norm, N, errs=errs)
    assert np.all(errs <= 1e-10 * norm)
    err = np.abs(np.sort(eigs) - ref) / norm
    print(f"JW twin L=20 N=5000 moment_mode {moment_mode}: {dt:.1f} s, max error {err.max():.1e} (median "
          f"{np.median(err):.1e}) of ||H||, m {rep['m']}, rank {rep['rank']}, core {rep['n_accepted']}, "
          f"retries {rep['retries']}")


def test_central_eigs_paper_tfim_L19_full_size(ctx):
    """The paper's error experiment on its Ising model (Sec. III, the L = 19 panel of its relative-
    error figure) with our own disorder seed: 5000 central levels of the random transverse-field
    chain at L = 19 in the benchmark's tuned configuration, against the exact Jordan-Wigner
    spectrum.  Its levels cluster (integrable model): the closest pair among the 5000 is 2.7e-9
    apart, 3.5x the 1e-10 ||H|| tolerance.  Prints the paper's measure, the count of values with
    relative error eta = |E - E_exact| / |E_exact| below 1e-6."""
    import time

    L, N = 19, 5000
    terms = inputs.paper_tfim(L, 0)
    Jb = np.array([t["coeff"] for t in terms if t["op_b"] == 1])
    g = np.array([t["coeff"] for t in terms if t["op_b"] == 0])
    ref, norm = central.central_eigenvalues_jw(Jb, g, N)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    opts = B.default_opts(b=64, kfac=12.0, window_ratio=2.2, basis_ratio=1.2, precision=B.DACP_F32,
                          fp64_tail_frac=0.3)
    t0 = time.perf_counter()
    eigs, errs, rep, st = B.dacp_central_eigs(ctx, ham, N, opts)
    dt = time.perf_counter() - t0
    _check_central(eigs, ref, norm, N, errs=errs)
    assert np.all(errs <= 1e-10 * norm)
    err = np.abs(eigs - ref)
    eta = err / np.abs(ref)
    print(f"paper TFIM L=19 N=5000: {dt:.1f} s, max |dE|/||H|| {err.max() / norm:.2e}, "
          f"eta < 1e-6 for {int(np.sum(eta < 1e-6))} of {N}, max eta {eta.max():.2e}, m {rep['m']}, "
          f"rank {rep['rank']}, K {rep['K']}, evolution steps {rep['evol_steps']}, retries {rep['retries']}")


def test_fp32_tail_error_table(ctx):
    """Error of the FP32 filter with an FP64 tail against the dense FP64 oracle, per tail fraction
    (spin glass L = 12, N = 200, b = 8, kfac 12, no retries).  FP64 and tails of 0.2 and 0.3 must
    reach N with the full accuracy; shorter tails may fall short (printed, not asserted)."""
    L, N = 12, 200
    terms = inputs.spin_glass(L, 0)
    ref, norm = central.central_eigenvalues(L, terms, N)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    for prec, frac in ((B.DACP_F64, 1.0), (B.DACP_F32, 0.0), (B.DACP_F32, 0.05), (B.DACP_F32, 0.1),
                       (B.DACP_F32, 0.2), (B.DACP_F32, 0.3)):
        o = B.default_opts(b=8, kfac=12.0, precision=prec, fp64_tail_frac=frac, max_retries=0)
        eigs, errs, rep, st = B.dacp_central_eigs(ctx, ham, N, o, raise_on_window=False)
        line = (f"{'f64' if prec == B.DACP_F64 else 'f32'} tail {frac}: status {st}, core {rep['n_accepted']} "
                f"of {rep['n_candidates']}")
        if st == 0:
            d = np.abs(np.sort(eigs) - ref) / norm
            line += f", max {d.max():.1e}, median {np.median(d):.1e} (of ||H|| = {norm:.2f})"
        print(line)
        if prec == B.DACP_F64 or frac >= 0.2:
            assert st == 0
            _check_central(eigs, ref, norm, N, errs=errs)


# ------------------------------------------------------------------ batched realisations


@pytest.mark.parametrize("moment_mode", [0, 2], ids=["explicit_products", "moment_projection"])
@pytest.mark.parametrize("batch_eig", [1, 2], ids=["eigensolver_auto", "batched_eigensolver"])
def test_central_eigs_batched_mixed_L_matches_dense_oracle(ctx, batch_eig, moment_mode):
    """Realisations of different L in one persistent launch, each against its dense oracle; with
    the default eigensolver choice (five realisations: the per-problem solver) and with the
    batched eigensolver forced; S and P as explicit products and from the anchor panels' moments
    (the kernel then samples the uniform grid and stores the anchors)."""
    N = 40
    specs = [(8, 1), (10, 2), (9, 3), (10, 4), (8, 5)]
    hams, refs = [], []
    for L, seed in specs:
        terms = inputs.spin_glass(L, seed)
        refs.append(central.central_eigenvalues(L, terms, N))
        hams.append(B.dacp_build_hamiltonian(ctx, L, terms))
    for precision in (B.DACP_F64, B.DACP_F32):
        opts = B.default_opts(b=8, precision=precision, fp64_tail_frac=0.3, moment_mode=moment_mode)
        try:
            ctx.tune("batch_eig", batch_eig)
            eigs, errs, n_out, reps, st = B.dacp_central_eigs_batched(ctx, hams, N, opts)
        finally:
            ctx.tune("batch_eig", 1)
        assert st == 0 and np.all(n_out == N)
        for r, (ref, norm) in enumerate(refs):
            _check_central(eigs[r], ref, norm, N, errs=errs[r])
            assert np.all(errs[r] <= 1e-10 * norm)
            # the batched Lanczos bound equals the single-realisation one up to reduction order
            eb, _, _ = B.dacp_spectral_bound(ctx, hams[r], steps=80, seed=0x5BD1E995)
            assert abs(reps[r]["e_bound"] - eb) <= 1e-9 * eb


@pytest.mark.parametrize("batch_eig", [0, 2], ids=["per_problem_eigensolver", "batched_eigensolver"])
def test_central_eigs_batched_moment_projection_explicit_switch(ctx, batch_eig):
    """Batched calls with the moment projection and the explicit products of each stored basis
    forced after the moment solve (moment_explicit = 2: the path a realisation takes when its
    moment-solve core falls short of N), against the dense oracle."""
    N = 40
    specs = [(8, 21), (10, 22), (9, 23)]
    hams, refs = [], []
    for L, seed in specs:
        terms = inputs.spin_glass(L, seed)
        refs.append(central.central_eigenvalues(L, terms, N))
        hams.append(B.dacp_build_hamiltonian(ctx, L, terms))
    opts = B.default_opts(b=8, moment_mode=2)
    try:
        ctx.tune("batch_eig", batch_eig)
        ctx.tune("moment_explicit", 2)
        eigs, errs, n_out, reps, st = B.dacp_central_eigs_batched(ctx, hams, N, opts)
    finally:
        ctx.tune("batch_eig", 1)
        ctx.tune("moment_explicit", 1)
    assert st == 0 and np.all(n_out == N)
    for r, (ref, norm) in enumerate(refs):
        _check_central(eigs[r], ref, norm, N, errs=errs[r])


def test_central_eigs_batched_per_problem_eigensolver(ctx):
    """The batched path with the finishing threads' eigen-decompositions solved one by one (knob
    batch_eig = 0) gives the same eigenvalues as with the batched eigensolver forced
    (batch_eig = 2), both at the oracle."""
    N = 40
    specs = [(8, 11), (10, 12), (9, 13)]
    hams, refs = [], []
    for L, seed in specs:
        terms = inputs.spin_glass(L, seed)
        refs.append(central.central_eigenvalues(L, terms, N))
        hams.append(B.dacp_build_hamiltonian(ctx, L, terms))
    opts = B.default_opts(b=8)
    try:
        ctx.tune("batch_eig", 2)
        e1, _, n1, _, st1 = B.dacp_central_eigs_batched(ctx, hams, N, opts)
        ctx.tune("batch_eig", 0)
        e0, _, n0, _, st0 = B.dacp_central_eigs_batched(ctx, hams, N, opts)
    finally:
        ctx.tune("batch_eig", 1)
    assert st0 == 0 and st1 == 0 and np.all(n0 == N) and np.all(n1 == N)
    for r, (ref, norm) in enumerate(refs):
        _check_central(e0[r], ref, norm, N)
        _check_central(e1[r], ref, norm, N)


def test_central_eigs_batched_repeat_reuses_cached_blocks(ctx):
    """Device buffers of a batched call come from a block cache whose reuse is ordered by stream
    events: a second identical call (served from the cache, its blocks handed between the worker
    threads' streams) returns the same values bit for bit, also after a larger call in between
    (whose first realisations, with the same indices and start blocks, match bit for bit too)."""
    N = 40
    specs = [(9, 21), (10, 22), (8, 23), (10, 24)]
    hams = [B.dacp_build_hamiltonian(ctx, L, inputs.spin_glass(L, seed)) for L, seed in specs]
    opts = B.default_opts(b=8)
    e1, r1, n1, _, st1 = B.dacp_central_eigs_batched(ctx, hams[:3], N, opts)
    e2, r2, n2, _, st2 = B.dacp_central_eigs_batched(ctx, hams[:3], N, opts)
    big = B.dacp_central_eigs_batched(ctx, hams + hams, N, opts)
    e3, r3, n3, _, st3 = B.dacp_central_eigs_batched(ctx, hams[:3], N, opts)
    assert st1 == st2 == st3 == big[4] == 0
    assert np.all(n1 == N) and np.all(n2 == N) and np.all(n3 == N) and np.all(big[2] == N)
    assert np.array_equal(e1, e2) and np.array_equal(e1, e3)
    assert np.array_equal(r1, r2) and np.array_equal(r1, r3)
    assert np.array_equal(big[0][:3], e1)
    # realisations 4..6 repeat the Hamiltonians of 0..2 with start blocks of their own index
    ref, norm = central.central_eigenvalues(10, inputs.spin_glass(10, 22), N)
    _check_central(e1[1], ref, norm, N)
    _check_central(big[0][5], ref, norm, N)


def test_central_eigs_batched_L14_and_L12(ctx):
    """L = 14 keeps the older recurrence term in global scratch; checked against the Jordan-Wigner
    closed form, next to an L = 12 spin glass against the dense oracle."""
    N = 120
    L1 = 14
    ham1 = B.dacp_build_hamiltonian(ctx, L1, inputs.ising_chain(L1, hz=0.0))
    ref1, norm1 = central.central_eigenvalues_jw(np.ones(L1 - 1), 1.05 * np.ones(L1), N)
    L2 = 12
    terms2 = inputs.spin_glass(L2, 7)
    ref2, norm2 = central.central_eigenvalues(L2, terms2, N)
    ham2 = B.dacp_build_hamiltonian(ctx, L2, terms2)
    eigs, errs, n_out, reps, st = B.dacp_central_eigs_batched(ctx, [ham1, ham2, ham1], N, B.default_opts(b=8))
    assert st == 0 and np.all(n_out == N)
    _check_central(eigs[0], ref1, norm1, N, errs=errs[0])
    _check_central(eigs[2], ref1, norm1, N, errs=errs[2])
    _check_central(eigs[1], ref2, norm2, N, errs=errs[1])


def test_central_eigs_batched_rejects_large_L(ctx):
    ham = B.dacp_build_hamiltonian(ctx, 15, inputs.ising_chain(15))
    with pytest.raises(B.DacpError) as ei:
        B.dacp_central_eigs_batched(ctx, [ham], 10, B.default_opts(b=4))
    assert ei.value.status == -1


# ------------------------------------------------------------------ learned window


def _mlp_dims():
    return B.WINDOW_FEATURES, 64, 3, 2


def test_mlp_gradient_matches_oracle(ctx):
    """FP32 forward/backward kernels against the FP64 oracle network on the same parameters."""
    from oracle import mlp as omlp

    n_in, hidden, layers, n_out = _mlp_dims()
    net = B.Mlp(ctx, n_in, hidden, layers, n_out, seed=3)
    theta = B.dacp_mlp_params(ctx, net).astype(np.float64)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((100, n_in))
    T = rng.standard_normal((100, n_out))
    loss, g = B.dacp_mlp_loss_grad(ctx, net, X, T)
    loss_ref, g_ref = omlp.loss_and_grad(theta, X, T, n_in, hidden, layers, n_out)
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    assert np.abs(g - g_ref).max() <= 1e-3 * np.abs(g_ref).max()
    # the same on a deeper-than-wide case with a ragged last mini-batch-like size
    net2 = B.Mlp(ctx, 3, 5, 2, 2, seed=9)
    th2 = B.dacp_mlp_params(ctx, net2).astype(np.float64)
    X2, T2 = rng.standard_normal((7, 3)), rng.standard_normal((7, 2))
    l2, g2 = B.dacp_mlp_loss_grad(ctx, net2, X2, T2)
    l2r, g2r = omlp.loss_and_grad(th2, X2, T2, 3, 5, 2, 2)
    assert abs(l2 - l2r) <= 1e-5 * l2r and np.abs(g2 - g2r).max() <= 1e-4 * np.abs(g2r).max()


def test_mlp_adam_step_matches_oracle(ctx):
    """One full-batch epoch = one Adam step on the standardised data."""
    from oracle import mlp as omlp

    n_in, hidden, layers, n_out = 4, 16, 2, 2
    net = B.Mlp(ctx, n_in, hidden, layers, n_out, seed=1)
    theta = B.dacp_mlp_params(ctx, net).astype(np.float64)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((40, n_in)) * 3 + 1
    Y = rng.standard_normal((40, n_out)) * 2 - 5
    Xs = (X - X.mean(0)) / X.std(0)
    Ys = (Y - Y.mean(0)) / Y.std(0)
    _, g = omlp.loss_and_grad(theta, Xs, Ys, n_in, hidden, layers, n_out)
    ref, _, _ = omlp.adam_step(theta, g, np.zeros_like(g), np.zeros_like(g), 1, 1e-2)
    B.dacp_mlp_train(ctx, net, X, Y, epochs=1, batch=40, lr=1e-2)
    got = B.dacp_mlp_params(ctx, net).astype(np.float64)
    assert np.abs(got - ref).max() <= 2e-5


def test_mlp_learns_a_smooth_map(ctx):
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (600, 8))
    Y = np.stack([np.sin(2 * X[:, 0]) + 0.5 * X[:, 1] ** 2, X[:, 2] * X[:, 3] - 0.3 * X[:, 4]], axis=1)
    net = B.Mlp(ctx, seed=0)
    loss = B.dacp_mlp_train(ctx, net, X[:500], Y[:500], epochs=300, batch=64, lr=3e-3, seed=1)
    assert loss < 0.02
    pred = B.dacp_mlp_predict(ctx, net, X[500:])
    assert np.sqrt(np.mean((pred - Y[500:]) ** 2)) < 0.1


def test_window_labels_match_the_estimators(ctx):
    """Labels equal log(E_b / sigma) of the Lanczos bound and the KPM density near 0, and the
    density is close to the exact central level density of the dense spectrum."""
    hams, terms_l = [], []
    for L, seed in ((9, 1), (10, 2), (11, 3)):
        t = inputs.spin_glass(L, seed)
        terms_l.append((L, t))
        hams.append(B.dacp_build_hamiltonian(ctx, L, t))
    lab = B.dacp_window_labels(ctx, hams)
    for (L, t), h, (y0, y1) in zip(terms_l, hams, lab):
        sig = np.sqrt(hamiltonian.sum_sq_coeff(t))
        eb, _, _ = B.dacp_spectral_bound(ctx, h, steps=80, seed=0x5BD1E995)
        assert abs(y0 - np.log(eb / (sig * np.sqrt(2 * L * np.log(2))))) <= 1e-9
        ev = central.full_spectrum_dense(L, t)
        assert eb >= np.abs(ev).max()
        D = 1 << L
        half = 0.02 * eb
        exact = np.sum(np.abs(ev) <= half) / (2 * half)
        rho = D * np.exp(y1) / (np.sqrt(2 * np.pi) * sig)
        assert abs(rho - exact) <= 0.25 * exact


def _trained_window_model(ctx, seed=0):
    hams, feats = [], []
    for L in (8, 9, 10, 11, 12):
        for s in range(40):
            h = B.dacp_build_hamiltonian(ctx, L, inputs.spin_glass(L, 1000 + 97 * L + s))
            hams.append(h)
            feats.append(B.dacp_window_features(ctx, h))
    lab = B.dacp_window_labels(ctx, hams)
    net = B.Mlp(ctx, seed=seed)
    B.dacp_mlp_train(ctx, net, np.array(feats), lab, epochs=400, batch=64, lr=2e-3, seed=seed)
    return net


def test_central_eigs_learned_matches_dense_oracle(ctx):
    net = _trained_window_model(ctx)
    L, N = 12, 150
    terms = inputs.spin_glass(L, 11)
    ref, norm = central.central_eigenvalues(L, terms, N)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    eigs, errs, rep, st = B.dacp_central_eigs_learned(ctx, ham, net, N, bound_margin=0.05, opts=B.default_opts(b=8))
    assert rep["model_used"] == 1
    _check_central(eigs, ref, norm, N, errs=errs)


def test_central_eigs_learned_falls_back_on_a_bad_model(ctx):
    """A network that predicts a bound far below ||H||: the evolution's norm guard trips and the
    Lanczos / KPM path redoes the call, with the same answer."""
    rng = np.random.default_rng(0)
    X = rng.standard_normal((64, B.WINDOW_FEATURES))
    Y = np.stack([np.full(64, -4.0), np.zeros(64)], axis=1) + 1e-3 * rng.standard_normal((64, 2))
    net = B.Mlp(ctx, seed=2)
    B.dacp_mlp_train(ctx, net, X, Y, epochs=50, batch=64, lr=1e-2)
    L, N = 10, 60
    terms = inputs.spin_glass(L, 21)
    ref, norm = central.central_eigenvalues(L, terms, N)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    eigs, errs, rep, st = B.dacp_central_eigs_learned(ctx, ham, net, N, bound_margin=0.0, opts=B.default_opts(b=8))
    assert rep["model_used"] == 1 and rep["model_fallback"] == 1
    _check_central(eigs, ref, norm, N, errs=errs)


def test_autotune_keeps_a_working_configuration(ctx):
    """The autotuner times every evolution configuration at the real shape and keeps the fastest;
    the basis built with the kept configuration still matches the oracle."""
    L, b, n = 16, 16, 1
    terms = inputs.ising_chain(L)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    try:
        g, us = B.dacp_autotune(ctx, ham, b=b, steps=32)
        assert g in (1, 2, 4, 8, 16) and us > 0
        eb = 1.01 * (1.723 * L)
        a = 0.45 * eb
        psi = np.random.default_rng(3).standard_normal((1 << L, b))
        psi /= np.linalg.norm(psi, axis=0)
        ref, ks = chebyshev.chebyshev_basis(lambda X: hamiltonian.apply_h(L, terms, X), psi, eb, a, n)
        V = torch.zeros((1 << L, b * (2 * n + 1)), dtype=torch.float64, device=DEV)
        B.dacp_basis(ctx, ham, to_dev(psi), V, eb, a, n)
        assert np.abs(host(V) - ref).max() < 1e-15 * max(ks) + 1e-12
    finally:
        for k, v in (("group", 8), ("rec_threads", 1024), ("rec_tile", 8192), ("rec_hi_w", 0)):
            ctx.tune(k, v)
