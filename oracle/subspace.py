"""Oracle: projection and subspace diagonalisation (test infrastructure).

Sec. II.C and App. C: with the basis A (columns Psi_i), form S = A^T A and
H = A^T (H A) (Eq. gep), diagonalise S = V Lambda_s V^T, discard eigenvalues
whose absolute value is below epsilon = 1e-12, U = V~ Lambda~_s^(-1/2),
H~ = U^T H U, diagonalise H~ = Y Lambda Y^T; B = U Y and Phi = A B.  The
residual norm ||H phi - theta phi|| bounds the eigenvalue error (Sec. II.C).
Dense eigen-decompositions use the oracle's own Householder + QL.
"""
import numpy as np

from . import _native


def project(apply, V):
    """(S, P) = (V^T V, V^T H V) with H V formed by `apply` (Sec. II.C, Eq. gep)."""
    V = np.asarray(V, dtype=np.float64)
    W = apply(V)
    return V.T @ V, V.T @ W


def rayleigh_ritz(S, P, eps=1e-12):
    """Generalised eigenproblem P B = S B Lambda by the App. C procedure.

    Returns (theta ascending, B = U Y, rank of S kept)."""
    S = 0.5 * (S + S.T)
    P = 0.5 * (P + P.T)
    lam, Vs = _native.syev(S, vectors=True)
    keep = np.abs(lam) >= eps
    keep &= lam > 0.0
    U = Vs[:, keep] / np.sqrt(lam[keep])[None, :]
    Ht = U.T @ P @ U
    Ht = 0.5 * (Ht + Ht.T)
    theta, Y = _native.syev(Ht, vectors=True)
    return theta, U @ Y, int(np.count_nonzero(keep))


def residual_norms(apply, V, B, theta):
    """||H phi_j - theta_j phi_j|| for phi = V B (Sec. II.C residual check)."""
    Phi = V @ B
    R = apply(Phi) - Phi * theta[None, :]
    return np.linalg.norm(R, axis=0), np.linalg.norm(Phi, axis=0)


def rayleigh_quotients(apply, V, B, theta):
    """For the computed Ritz vectors phi = V b_j: their Rayleigh quotients phi^T H phi / phi^T phi
    and the residual norms ||H phi - theta phi|| / ||phi|| about the projected problem's values
    (Sec. II.C).  The Rayleigh quotient of phi is the Ritz value in exact arithmetic; computed
    directly from phi it does not carry the rounding of the ill-conditioned projected problem, and
    its own residual is at most the one returned."""
    Phi = V @ B
    HPhi = apply(Phi)
    nx = np.einsum("ij,ij->j", Phi, Phi)
    rq = np.einsum("ij,ij->j", Phi, HPhi) / nx
    rn = np.linalg.norm(HPhi - Phi * theta[None, :], axis=0) / np.sqrt(nx)
    return rq, rn


def neighbour_gaps(theta):
    """Distance of each Ritz value to its nearest other Ritz value."""
    theta = np.asarray(theta)
    n = theta.shape[0]
    gaps = np.full(n, np.inf)
    if n > 1:
        order = np.argsort(theta)
        t = theta[order]
        d = np.diff(t)
        g = np.full(n, np.inf)
        g[:-1] = d
        g[1:] = np.minimum(g[1:], d)
        gaps[order] = g
    return gaps
