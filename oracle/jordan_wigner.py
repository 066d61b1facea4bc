"""Oracle: Jordan-Wigner closed-form spectrum of the open transverse-field Ising chain.

The paper checks its Ising results against the Jordan-Wigner reduction of the
2^N x 2^N problem to a 2N x 2N one from which the full spectrum is restored
(Sec. III, discussion of Fig. 2).  For
    H = sum_{i<L-1} J_i Z_i Z_{i+1} + sum_i h_i X_i          (open chain)
the many-body levels are { sum_k s_k eps_k : s in {+1,-1}^L }, where eps_k are
the singular values of the L x L upper-bidiagonal M (M_ii = h_i,
M_{i,i+1} = J_i).  They are the positive eigenvalues of the 2L x 2L
Golub-Kahan tridiagonal with zero diagonal and off-diagonal
(h_0, J_0, h_1, J_1, ..., J_{L-2}, h_{L-1}) -- the paper's 2N x 2N matrix.
The paper's disordered model maps onto this form by exchanging x and z and
rescaling J -> J/4, Gamma -> Gamma/2.
"""
import numpy as np

from . import _native


def single_particle_energies(J, h):
    """eps_k >= 0 (ascending) from the Golub-Kahan tridiagonal, own QL."""
    h = np.asarray(h, dtype=np.float64)
    J = np.asarray(J, dtype=np.float64)
    L = h.shape[0]
    assert J.shape[0] == L - 1
    off = np.empty(2 * L - 1)
    off[0::2] = h
    off[1::2] = J
    w = _native.tridiag_eigvals(np.zeros(2 * L), off)
    eps = w[L:]  # spectrum is symmetric: +/- eps_k
    return np.sort(np.abs(eps))


def full_spectrum(J, h):
    """All 2^L levels (ascending), each sum formed directly by pairwise summation."""
    eps = single_particle_energies(J, h)
    L = eps.shape[0]
    s = np.arange(1 << L, dtype=np.int64)
    signs = 1.0 - 2.0 * ((s[:, None] >> np.arange(L)[None, :]) & 1)  # (D, L)
    vals = signs * eps[None, :]
    # pairwise summation along the spin axis
    while vals.shape[1] > 1:
        if vals.shape[1] % 2:
            vals = np.concatenate([vals, np.zeros((vals.shape[0], 1))], axis=1)
        vals = vals[:, 0::2] + vals[:, 1::2]
    return np.sort(vals[:, 0])
