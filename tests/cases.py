"""Small test problems shared by the CPU pins and the GPU parity tests (inputs
only: no arithmetic of the method)."""
import numpy as np

from oracle import recycle as rc
from oracle.krylov import as_csr
from paper_1010_0762_amd import workloads as wl


def eig_case(cplx, n=60, m=6, seed=11):
    """A = S diag(lam) S^{-1} (n x n, dense) with six small eigenvalues; b in
    the span of the first m right eigenvectors (columns of S), b~ in the span
    of the matching left eigenvectors (columns of Y = S^{-H}).  Returns
    (A, b, b~, S, Y)."""
    lam = np.concatenate([[0.3, 0.5, 0.7, 2.5, 3.1, 4.4], np.linspace(6.0, 12.0, n - 6)])
    rng = np.random.default_rng(seed)
    S = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    if cplx:
        S = S + 0.3j * rng.standard_normal((n, n)) / np.sqrt(n)
    A = S @ np.diag(lam) @ np.linalg.inv(S)
    Y = np.linalg.inv(S).conj().T
    c = np.random.default_rng(5)
    b = S[:, :m] @ (c.standard_normal(m) + 1.0)
    bt = Y[:, :m] @ (c.standard_normal(m) + 1.0)
    return A, b, bt, S, Y


def stall_case():
    """A recycle space whose C = A U and C~ = A^H U~ are nearly orthogonal
    (cosines near 1e-6, kept by a cut of 1e-7) on a non-normal 2D conv-diff
    operator (16 x 16 grid, beta = (40, 20)): the oblique projector
    I - C C~^H has a norm near 1e7 and amplifies rounding, so that Algorithm 2
    does not converge.  Returns (A, b, b~, U, U~, C, C~) with C~^H C = I."""
    A = as_csr(wl.convdiff(16, 2, [40.0, 20.0]))
    AH = A.conj().T.tocsr()
    n = A.shape[0]
    rng = np.random.default_rng(1)
    U = rng.standard_normal((n, 6))
    Ut = rng.standard_normal((n, 6))
    U, Ut, C, Ct = rc.biorthogonalize(A, AH, U, Ut, 0.0)
    Q, _ = np.linalg.qr(C)
    # remove all but 1e-6 of the part of A^H U~ inside range(C)
    Ut = Ut - np.linalg.solve(AH.toarray(), Q @ (Q.T @ (AH @ Ut))) * (1 - 1e-6)
    U, Ut, C, Ct = rc.biorthogonalize(A, AH, U, Ut, 1e-7)
    b = rng.standard_normal(n)
    bt = rng.standard_normal(n)
    return A, b, bt, U, Ut, C, Ct
