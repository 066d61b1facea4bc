"""Oracle: spin-1/2 Hamiltonians from one- and two-body Pauli terms (test infrastructure).

The paper (Sec. III, model definitions) writes each Hamiltonian as a sum of
single Pauli operators and products of two Pauli operators on distinct spins,
each acting on a state as a simple function.  Here a term is (op_a, site_a,
op_b, site_b, coeff) with op codes 0=I, 1=X, 2=Y, 3=Z (op_b = 0 for a one-body
term).  Basis convention: bit i of the index s is spin i, and
sigma^z |b> = (1 - 2b) |b>.

Element formula used throughout the oracle.  With x = mask of sites carrying X
or Y, z = mask of sites carrying Z or Y and ny = number of Y factors,
    P |s> = i^ny (-1)^popcount(s & z) |s ^ x>,
because sigma^y = i sigma^x sigma^z.  A real Hamiltonian needs ny even, so
i^ny = (-1)^(ny/2).
"""
import numpy as np

OP_I, OP_X, OP_Y, OP_Z = 0, 1, 2, 3


def term_masks(op_a, site_a, op_b, site_b):
    """(x_mask, z_mask, real phase) of one Pauli string (element formula above)."""
    x = z = 0
    ny = 0
    for op, site in ((int(op_a), int(site_a)), (int(op_b), int(site_b))):
        if op == OP_I:
            continue
        bit = 1 << site
        if op in (OP_X, OP_Y):
            x |= bit
        if op in (OP_Z, OP_Y):
            z |= bit
        if op == OP_Y:
            ny += 1
    if ny % 2:
        raise ValueError("term with an odd number of Y factors is imaginary")
    phase = -1.0 if (ny // 2) % 2 else 1.0
    return x, z, phase


def _popcount_parity(v):
    return (np.bitwise_count(v) & 1).astype(np.int64)


def dense_h(L, terms):
    """Dense D x D Hamiltonian (FP64) from the element formula."""
    D = 1 << L
    H = np.zeros((D, D))
    s = np.arange(D, dtype=np.int64)
    for t in terms:
        x, z, phase = term_masks(t["op_a"], t["site_a"], t["op_b"], t["site_b"])
        sign = 1.0 - 2.0 * _popcount_parity(s & z)
        np.add.at(H, (s ^ x, s), float(t["coeff"]) * phase * sign)
    return H


def apply_h(L, terms, X):
    """Matrix-free y = H x on a block X of shape (D, b) (FP64), element formula:
    y[s] = sum_t c_t phase_t (-1)^popcount((s ^ x_t) & z_t) X[s ^ x_t]."""
    D = 1 << L
    X = np.asarray(X, dtype=np.float64)
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None]
    assert X.shape[0] == D
    s = np.arange(D, dtype=np.int64)
    Y = np.zeros_like(X)
    for t in terms:
        x, z, phase = term_masks(t["op_a"], t["site_a"], t["op_b"], t["site_b"])
        src = s ^ x
        sign = 1.0 - 2.0 * _popcount_parity(src & z)
        Y += (float(t["coeff"]) * phase * sign)[:, None] * X[src]
    return Y[:, 0] if squeeze else Y


def sum_abs_coeff(terms):
    """Triangle-inequality bound sum_t |c_t| >= ||H|| (each Pauli string has norm 1)."""
    return float(np.sum(np.abs(np.asarray([t["coeff"] for t in terms], dtype=np.float64))))


def sum_sq_coeff(terms):
    """tr(H^2)/D = sum_t c_t^2 when all Pauli strings are distinct (orthogonality)."""
    return float(np.sum(np.asarray([t["coeff"] for t in terms], dtype=np.float64) ** 2))
