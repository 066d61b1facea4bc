"""Oracle: the central eigenvalues by their plain definition (test infrastructure).

The method is presented as exact (Sec. I, Sec. IV): it must return the N
eigenvalues of H closest to the band centre E = 0 (Sec. III, discussion of
Fig. 2).  The definition, written out: build the dense H from the element
formula, diagonalise it fully with the oracle's own Householder + QL, order by
the key (|lambda|, lambda) and return the first N in ascending order.
"""
import numpy as np

from . import _native, hamiltonian, jordan_wigner


def select_central(eigs, N, centre=0.0):
    """First N of `eigs` under the key (|lambda - centre|, lambda), ascending."""
    eigs = np.asarray(eigs, dtype=np.float64)
    key = np.lexsort((eigs, np.abs(eigs - centre)))
    return np.sort(eigs[key[:N]])


def full_spectrum_dense(L, terms):
    return _native.syev(hamiltonian.dense_h(L, terms))


def central_eigenvalues(L, terms, N):
    """(N central eigenvalues ascending, ||H||) from dense full diagonalisation."""
    w = full_spectrum_dense(L, terms)
    return select_central(w, N), float(max(abs(w[0]), abs(w[-1])))


def central_eigenvalues_jw(J, h, N):
    """Same selection on the Jordan-Wigner closed-form spectrum of the open
    chain sum J_i Z_i Z_{i+1} + sum h_i X_i."""
    w = jordan_wigner.full_spectrum(J, h)
    return select_central(w, N), float(max(abs(w[0]), abs(w[-1])))
