"""Seeded synthetic inputs shared by tests, the benchmark and the smoke check.

Holds no arithmetic of the method: only coupling lists of the benchmark
Hamiltonians and seeded random blocks.  Terms use the C-ABI record layout
(`TERM_DTYPE`, 16 bytes): op_a, op_b in {0=I, 1=X, 2=Y, 3=Z}; site_a, site_b;
coeff.  Bit i of a basis index is spin i.

Workloads (the paper's models are in Sec. III; the benchmark configurations
use the stated variants with unpublished realisations replaced by seeds):
  * `ising_chain`: H = J sum Z_i Z_{i+1} + hx sum X_i + hz sum Z_i, open chain
    (J=1, hx=1.05, hz=0.5 chaotic; hz=0 is the Jordan-Wigner-solvable twin).
  * `spin_glass`: H = sum Gamma_i X_i + sum_{i<j} J_ij Z_i Z_j with
    Gamma, J ~ U[-1, 1] i.i.d. (all-to-all "spin glass shard" form).
  * `paper_tfim`, `paper_sgs`: the paper's own disordered models with its
    parameters (J = 10, Gamma = 1).
"""
import numpy as np

TERM_DTYPE = np.dtype(
    [("op_a", "u1"), ("op_b", "u1"), ("site_a", "<u2"), ("site_b", "<u2"), ("reserved", "<u2"), ("coeff", "<f8")]
)
I, X, Y, Z = 0, 1, 2, 3


def make_terms(rows):
    """rows: iterable of (op_a, site_a, op_b, site_b, coeff)."""
    rows = list(rows)
    t = np.zeros(len(rows), dtype=TERM_DTYPE)
    for n, (oa, sa, ob, sb, c) in enumerate(rows):
        t[n] = (oa, ob, sa, sb, 0, c)
    return t


def ising_chain(L, J=1.0, hx=1.05, hz=0.5):
    rows = [(Z, i, Z, i + 1, J) for i in range(L - 1)]
    rows += [(X, i, I, 0, hx) for i in range(L)]
    if hz != 0.0:
        rows += [(Z, i, I, 0, hz) for i in range(L)]
    return make_terms(rows)


def spin_glass(L, seed):
    rng = np.random.default_rng(seed)
    gamma = rng.uniform(-1.0, 1.0, size=L)
    jmat = rng.uniform(-1.0, 1.0, size=(L, L))
    rows = [(X, i, I, 0, gamma[i]) for i in range(L)]
    rows += [(Z, i, Z, j, jmat[i, j]) for i in range(L) for j in range(i + 1, L)]
    return make_terms(rows)


def paper_tfim(L, seed, J=10.0, Gamma=1.0):
    """(1/4) sum J_{i,i+1} X_i X_{i+1} + (1/2) sum Gamma_i Z_i, J ~ U[-J/sqrt(L), J/sqrt(L)], Gamma_i ~ U[0, Gamma]."""
    rng = np.random.default_rng(seed)
    jb = rng.uniform(-J / np.sqrt(L), J / np.sqrt(L), size=L - 1)
    g = rng.uniform(0.0, Gamma, size=L)
    rows = [(X, i, X, i + 1, 0.25 * jb[i]) for i in range(L - 1)]
    rows += [(Z, i, I, 0, 0.5 * g[i]) for i in range(L)]
    return make_terms(rows)


def paper_sgs(L, seed, J=10.0, Gamma=1.0):
    """sum_{i<j} J_ij X_i X_j + sum Gamma_i Z_i with the paper's distributions."""
    rng = np.random.default_rng(seed)
    jm = rng.uniform(-J / np.sqrt(L), J / np.sqrt(L), size=(L, L))
    g = rng.uniform(0.0, Gamma, size=L)
    rows = [(X, i, X, j, jm[i, j]) for i in range(L) for j in range(i + 1, L)]
    rows += [(Z, i, I, 0, g[i]) for i in range(L)]
    return make_terms(rows)


def gaussian_block(D, b, seed):
    """[D][b] FP64 block of i.i.d. N(0,1) values (numpy PCG64 stream)."""
    return np.random.default_rng(seed).standard_normal((D, b))


def batched_spin_glass_set(count_per_L=32, Ls=(12, 13, 14), seed0=0):
    """Interleaved realisations L = 12, 13, 14, 12, ... with disorder seeds seed0, seed0+1, ..."""
    out = []
    seed = seed0
    for _ in range(count_per_L):
        for L in Ls:
            out.append((L, seed, spin_glass(L, seed)))
            seed += 1
    return out
